// Device-side helpers shared by the kernel files (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "gsf_internal.h"

namespace gsf {

// Raw buffer addressing: a descriptor over [base, base + bytes).  A load
// whose 32-bit byte offset falls outside returns 0 and a store there is
// dropped, so rows and columns past a cube face need no branch.  Offsets
// are unsigned: a "negative" offset wraps above the range and is dropped too.
constexpr uint32_t kOOB = 0x80000000u;   // offset that is always outside a range < 2^31

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             0x00020000);
}

// The b32 buffer builtins move raw 32-bit words: reinterpret, never convert.
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}

__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, float v, uint32_t off)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)off, 0, 0);
}

// Two consecutive floats (8-byte aligned offset) in one access.
typedef unsigned int gsf_u2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float2 buf_ld2(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    const gsf_u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
    return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
}

__device__ __forceinline__ void buf_st2(__amdgpu_buffer_rsrc_t r, float a, float b, uint32_t off)
{
    gsf_u2 v;
    v.x = __float_as_uint(a);
    v.y = __float_as_uint(b);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)off, 0, 0);
}

// Four consecutive floats (16-byte aligned offset) in one store.
typedef unsigned int gsf_u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void buf_st4(__amdgpu_buffer_rsrc_t r, float a, float b, float c,
                                        float d, uint32_t off)
{
    gsf_u4 v;
    v.x = __float_as_uint(a);
    v.y = __float_as_uint(b);
    v.z = __float_as_uint(c);
    v.w = __float_as_uint(d);
    __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)off, 0, 0);
}

// ---- storage types ----
// Cubes are stored as float (FP32), _Float16 (IEEE binary16) or __bf16
// (bfloat16); kernels compute in FP32, widen on load (exact) and round to
// nearest even on store.
template <typename S>
__device__ __forceinline__ float widen(S v)
{
    return (float)v;
}

template <typename S>
__device__ __forceinline__ S narrow(float v)
{
    return (S)v;
}

// One element of storage type S through a buffer descriptor; off in bytes.
template <typename S>
__device__ __forceinline__ float sbuf_ld(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    if constexpr (sizeof(S) == 4) {
        return buf_ld(r, off);
    } else {
        const unsigned short u = __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0);
        return (float)__builtin_bit_cast(S, u);
    }
}

// Raw form of a loaded element: the float itself for FP32, the 16 bits for
// 16-bit types.  Prefetched values stay raw until the step that uses them, so
// the widening does not wait on the load in the step that issues it.
template <typename S>
using raw_t = std::conditional_t<sizeof(S) == 4, float, unsigned short>;

template <typename S>
__device__ __forceinline__ raw_t<S> sbuf_ld_raw(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    if constexpr (sizeof(S) == 4)
        return buf_ld(r, off);
    else
        return __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0);
}

template <typename S>
__device__ __forceinline__ float from_raw(raw_t<S> v)
{
    if constexpr (sizeof(S) == 4)
        return v;
    else
        return (float)__builtin_bit_cast(S, v);
}

template <typename S>
__device__ __forceinline__ void sbuf_st(__amdgpu_buffer_rsrc_t r, float v, uint32_t off)
{
    if constexpr (sizeof(S) == 4) {
        buf_st(r, v, off);
    } else {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (S)v), r,
                                              (int)off, 0, 0);
    }
}

// Host-side dispatch on a storage type: fn receives a null St pointer whose
// type selects the instantiation.
template <typename Fn>
hipError_t with_store(Store st, Fn &&fn)
{
    switch (st) {
    case Store::F16: return fn((_Float16 *)nullptr);
    case Store::BF16: return fn((__bf16 *)nullptr);
    default: return fn((float *)nullptr);
    }
}

#define GSF_STORE_T(tag) std::remove_pointer_t<decltype(tag)>

}  // namespace gsf
