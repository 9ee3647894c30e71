// Device-side helpers shared by the kernel files (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

}  // namespace gsf
