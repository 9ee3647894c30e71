// gsf_stats.hip -- local statistics and selection (§3.3) for gfx950.
//
// The window sums of a = F - s and a^2 over the box around each voxel are
// computed as directional sums in two kernels:
//   k_box_yz<BY>: for one x-plane and a 64-wide z strip per wave, walk y with
//     a running window sum per column (the value leaving the window comes
//     from a register ring of the last BY rows, so F is read once), then take
//     the z window across lanes with wave-wide DPP prefix sums.  Writes the
//     yz-window sums G1 = sum a, G2 = sum a^2 for every voxel.
//   k_box_x_select<BX>: one lane per (y, z) walks x with a running window sum
//     of G1, G2 (leaving plane from a register ring of the last BX planes),
//     then forms mean = s + S1/n and std = sqrt(max(0, S2/n - (S1/n)^2)),
//     and the selection bit F > mean + k*std, packed along z by wave ballot.
// Running sums and the lane prefix sums of the z window are FP64, so every
// window sum is exact to well below FP32 rounding before it is stored.
#include <hip/hip_runtime.h>

#include "gsf_internal.h"

namespace gsf {
namespace {

constexpr int kThreads = 256;

// ---- wave64 inclusive prefix sum with DPP (row shifts, then row broadcasts) ----
template <int CTRL, int ROW_MASK, int BANK_MASK, bool BOUND_ZERO>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, BANK_MASK, BOUND_ZERO));
}

__device__ __forceinline__ float wave_incl_scan(float v)
{
    v += dpp_f<0x111, 0xf, 0xf, true>(v);   // row_shr:1
    v += dpp_f<0x112, 0xf, 0xf, true>(v);   // row_shr:2
    v += dpp_f<0x114, 0xf, 0xf, true>(v);   // row_shr:4
    v += dpp_f<0x118, 0xf, 0xf, true>(v);   // row_shr:8
    v += dpp_f<0x142, 0xa, 0xf, false>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_f<0x143, 0xc, 0xf, false>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

__device__ __forceinline__ int64_t win_len(int64_t i, int64_t n, int B)
{
    int64_t lo = i - (B / 2);
    int64_t hi = lo + B;
    if (lo < 0) lo = 0;
    if (hi > n) hi = n;
    return hi - lo;
}

// FP64 lane shift through DPP, one 32-bit half at a time.
template <int CTRL, int ROW_MASK, int BANK_MASK, bool BOUND_ZERO>
__device__ __forceinline__ double dpp_d(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, BANK_MASK,
                                               BOUND_ZERO);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, BANK_MASK,
                                               BOUND_ZERO);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_incl_scan_d(double v)
{
    v += dpp_d<0x111, 0xf, 0xf, true>(v);
    v += dpp_d<0x112, 0xf, 0xf, true>(v);
    v += dpp_d<0x114, 0xf, 0xf, true>(v);
    v += dpp_d<0x118, 0xf, 0xf, true>(v);
    v += dpp_d<0x142, 0xa, 0xf, false>(v);
    v += dpp_d<0x143, 0xc, 0xf, false>(v);
    return v;
}

__device__ __forceinline__ double readlane_d(double v, int lane)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// z window of one row for the 64 outputs of a wave.  Lane i carries the
// column sums c(i) and c(i + 64) of the strip plus its window; output i is
// H(i) = P(i + bz - 1) - P(i - 1) with P the inclusive prefix over the 128
// columns.  P is FP64, so the difference keeps FP64 accuracy relative to the
// strip's largest prefix and H is exact to well below FP32 rounding.
__device__ __forceinline__ float zwin(double lo, double hi, double *q, int lane, int bz)
{
    const double plo = wave_incl_scan_d(lo);
    const double phi = wave_incl_scan_d(hi) + readlane_d(plo, 63);
    q[lane] = plo;
    q[lane + 64] = phi;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const double h = q[lane + bz - 1] - (lane > 0 ? q[lane - 1] : 0.0);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return (float)h;
}

__device__ __forceinline__ void emit_row(double a1, double a2, double b1, double b2, double *q1,
                                         double *q2, int lane, int bz, bool live, float *g1,
                                         float *g2)
{
    const float h1 = zwin(a1, b1, q1, lane, bz);
    const float h2 = zwin(a2, b2, q2, lane, bz);
    if (live) {
        *g1 = h1;
        *g2 = h2;
    }
}

// One wave per (x, 64-wide z strip); 4 independent waves per block.
// Requires bz <= 65 so the strip plus its window spans at most 128 columns.
template <int BY>
__global__ __launch_bounds__(kThreads) void k_box_yz(const float *__restrict__ F, int64_t nx,
                                                     int64_t ny, int64_t nz, int bz,
                                                     const double *__restrict__ shift,
                                                     float *__restrict__ G1,
                                                     float *__restrict__ G2)
{
    __shared__ double qs[4][2][128];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t nstrips = (nz + 63) / 64;
    const int64_t job = (int64_t)blockIdx.x * 4 + wave;
    if (job >= nx * nstrips) return;                 // whole wave exits together
    const int64_t x = job / nstrips;
    const int64_t z0 = (job % nstrips) * 64;
    const int loz = -(bz / 2);
    const int loy = -(BY / 2);
    const int hiy = loy + BY - 1;
    const float s = (float)shift[0];
    // the two columns this lane carries: c = lane and c = lane + 64
    const int64_t zc0 = z0 + loz + lane;
    const int64_t zc1 = zc0 + 64;
    const bool v0 = zc0 >= 0 && zc0 < nz;
    const bool v1 = (lane + 64 < 64 + bz - 1) && zc1 >= 0 && zc1 < nz;
    const float *pl = F + x * ny * nz;
    const int64_t zo = z0 + lane;
    float ring0[BY], ring1[BY];
#pragma unroll
    for (int j = 0; j < BY; ++j) ring0[j] = ring1[j] = 0.0f;
    double a1 = 0.0, a2 = 0.0, b1 = 0.0, b2 = 0.0;   // running y sums, columns 0 and 1
    double *q1 = qs[wave][0];
    double *q2 = qs[wave][1];
    const int64_t nsteps = ny + hiy;                  // entering rows 0 .. ny-1+hiy
    for (int64_t y0 = 0; y0 < nsteps; y0 += BY) {
#pragma clang loop unroll(full)
        for (int j = 0; j < BY; ++j) {
            const int64_t yin = y0 + j;                   // yin mod BY == j
            if (yin < nsteps) {
                float e0 = 0.0f, e1 = 0.0f;
                if (yin < ny) {
                    if (v0) e0 = pl[yin * nz + zc0] - s;
                    if (v1) e1 = pl[yin * nz + zc1] - s;
                }
                const float l0 = ring0[j], l1 = ring1[j];
                ring0[j] = e0;
                ring1[j] = e1;
                a1 += (double)e0 - (double)l0;
                a2 += (double)(e0 * e0) - (double)(l0 * l0);
                b1 += (double)e1 - (double)l1;
                b2 += (double)(e1 * e1) - (double)(l1 * l1);
                const int64_t y = yin - hiy;
                if (y >= 0) emit_row(a1, a2, b1, b2, q1, q2, lane, bz, zo < nz,
                                     G1 + (x * ny + y) * nz + zo, G2 + (x * ny + y) * nz + zo);
            }
        }
    }
}

// One lane per (y, z), 256 consecutive z per block; walks x.
template <int BX>
__global__ __launch_bounds__(kThreads) void k_box_x_select(
    const float *__restrict__ G1, const float *__restrict__ G2, const float *__restrict__ F,
    int64_t nx, int64_t ny, int64_t nz, int by, int bz, const double *__restrict__ shift,
    float *__restrict__ mean, float *__restrict__ stdev, uint64_t *__restrict__ mask, double k)
{
#pragma clang fp contract(off)
    const int64_t y = blockIdx.y;
    const int64_t zb = (int64_t)blockIdx.x * kThreads;
    const int64_t z = zb + threadIdx.x;
    const bool live = z < nz;
    const int64_t plane = ny * nz;
    const int64_t off = y * nz + (live ? z : 0);
    const int64_t W = (nz + 63) / 64;
    const int lox = -(BX / 2);
    const int hix = lox + BX - 1;
    const double s = (double)(float)shift[0];   // the same FP32 shift the sums used
    const double inv_yz = live ? 1.0 / (double)(win_len(y, ny, by) * win_len(z, nz, bz)) : 1.0;
    const double inv_bx = 1.0 / (double)BX;
    float r1[BX], r2[BX];
#pragma unroll
    for (int j = 0; j < BX; ++j) r1[j] = r2[j] = 0.0f;
    double s1 = 0.0, s2 = 0.0;
    const int64_t nsteps = nx + hix;
    for (int64_t p0 = 0; p0 < nsteps; p0 += BX) {
#pragma clang loop unroll(full)
        for (int j = 0; j < BX; ++j) {
            const int64_t p = p0 + j;                         // entering plane, p mod BX == j
            if (p < nsteps) {
                float g1 = 0.0f, g2 = 0.0f;
                if (p < nx && live) {
                    g1 = G1[p * plane + off];
                    g2 = G2[p * plane + off];
                }
                s1 += (double)g1 - (double)r1[j];
                s2 += (double)g2 - (double)r2[j];
                r1[j] = g1;
                r2[j] = g2;
                const int64_t x = p - hix;
                if (x >= 0) {
                    bool bit = false;
                    if (live) {
                        const int64_t cx = win_len(x, nx, BX);
                        const double inv_n = inv_yz * (cx == BX ? inv_bx : 1.0 / (double)cx);
                        const double m1 = s1 * inv_n;
                        double var = s2 * inv_n - m1 * m1;
                        if (var < 0.0) var = 0.0;
                        const float mf = (float)(s + m1);
                        const float sf = (float)sqrt(var);
                        const int64_t i = x * plane + off;
                        if (mean) mean[i] = mf;
                        if (stdev) stdev[i] = sf;
                        if (mask) bit = (double)F[i] > (double)mf + k * (double)sf;
                    }
                    if (mask) {
                        const uint64_t word = __ballot(bit);
                        if ((threadIdx.x & 63) == 0 && live)
                            mask[(x * ny + y) * W + z / 64] = word;
                    }
                }
            }
        }
    }
}

template <int BY>
hipError_t box_yz(const float *F, Dims d, int bz, const double *shift, float *G1, float *G2,
                  hipStream_t s)
{
    const int64_t jobs = d.nx * ((d.nz + 63) / 64);
    prof::Scope scope("k_box_yz", s);
    hipLaunchKernelGGL(k_box_yz<BY>, dim3((unsigned)((jobs + 3) / 4)), dim3(kThreads), 0, s, F,
                       d.nx, d.ny, d.nz, bz, shift, G1, G2);
    return hipGetLastError();
}

template <int BX>
hipError_t box_x_select(const float *G1, const float *G2, const float *F, Dims d, Box b,
                        const double *shift, float *mean, float *stdev, uint64_t *mask, double k,
                        hipStream_t s)
{
    const dim3 grid((unsigned)((d.nz + kThreads - 1) / kThreads), (unsigned)d.ny);
    prof::Scope scope("k_box_x_select", s);
    hipLaunchKernelGGL(k_box_x_select<BX>, grid, dim3(kThreads), 0, s, G1, G2, F, d.nx, d.ny, d.nz,
                       b.by, b.bz, shift, mean, stdev, mask, k);
    return hipGetLastError();
}

using YZFn = hipError_t (*)(const float *, Dims, int, const double *, float *, float *,
                            hipStream_t);
using XFn = hipError_t (*)(const float *, const float *, const float *, Dims, Box, const double *,
                           float *, float *, uint64_t *, double, hipStream_t);

YZFn yz_fn(int by)
{
    switch (by) {
    case 8: return &box_yz<8>;
    case 16: return &box_yz<16>;
    case 32: return &box_yz<32>;
    case 64: return &box_yz<64>;
    default: return nullptr;
    }
}

XFn x_fn(int bx)
{
    switch (bx) {
    case 8: return &box_x_select<8>;
    case 16: return &box_x_select<16>;
    case 32: return &box_x_select<32>;
    case 64: return &box_x_select<64>;
    default: return nullptr;
    }
}

}  // namespace

bool stats_fast_path(Box b) { return yz_fn(b.by) && x_fn(b.bx) && b.bz >= 1 && b.bz <= 65; }

hipError_t launch_stats_fast(const float *F, Dims d, Box b, const double *shift, float *G1,
                             float *G2, float *mean, float *stdev, uint64_t *mask, double k,
                             hipStream_t s)
{
    if (!stats_fast_path(b)) return hipErrorInvalidValue;
    hipError_t e = yz_fn(b.by)(F, d, b.bz, shift, G1, G2, s);
    if (e != hipSuccess) return e;
    return x_fn(b.bx)(G1, G2, F, d, b, shift, mean, stdev, mask, k, s);
}

}  // namespace gsf
