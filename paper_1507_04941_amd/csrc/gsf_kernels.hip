// gsf_kernels.hip -- HIP kernels for gfx950 (wave64).
//
// Filter: Eq. 2 of §2.1 as three 1-D passes (the 3-D Gaussian is the outer
// product of its axis kernels).  Statistics: §3.3's per-voxel mean and
// standard deviation over a box window, computed as three directional window
// sums of F - s and (F - s)^2.  Selection: F > mean + k*std.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gsf_device.h"
#include "gsf_internal.h"

namespace gsf {
namespace {

constexpr int kBlock = 256;   // four wave64s along z

// ---------------------------------------------------------------------------
// Filter passes.  Each output sums its taps in order -r..r with FMA.
// ---------------------------------------------------------------------------

// Spectral (z) pass: a block stages one row segment plus its +-r halo in LDS
// with coalesced loads, then every lane reads its 2r+1 neighbours from LDS.
template <typename St>
__global__ __launch_bounds__(kBlock) void k_zpass(const St *__restrict__ in,
                                                  float *__restrict__ out, int64_t nz, int64_t NZ,
                                                  int64_t zoff, Taps t)
{
    extern __shared__ float tile[];
    const int r = t.r;
    const int64_t row = blockIdx.x;
    const int64_t z0 = (int64_t)blockIdx.y * kBlock;
    // output z (core, nz per row) reads input z + zoff (NZ per row)
    const St *src = in + row * NZ + zoff;
    for (int i = threadIdx.x; i < kBlock + 2 * r; i += kBlock) {
        const int64_t z = z0 - r + i;
        tile[i] = (z + zoff >= 0 && z + zoff < NZ) ? widen(src[z]) : 0.0f;
    }
    __syncthreads();
    const int64_t z = z0 + threadIdx.x;
    if (z < nz) {
        float acc = 0.0f;
        for (int o = 0; o <= 2 * r; ++o) acc = fmaf(t.g[o], tile[threadIdx.x + o], acc);
        out[row * nz + z] = acc;
    }
}

// Pass along a strided axis.  Output row (X, y) of NYo rows per plane reads
// input rows of NYi rows per plane: along y, input row y + off + o of plane X
// (inside [0, NYi)); along x, row y of plane X + off + o (inside [0, NXi)).
// Lanes run along z so every tap load is a coalesced row read.
template <typename Si, typename So>
__global__ __launch_bounds__(kBlock) void k_strided_pass(const Si *__restrict__ in,
                                                         So *__restrict__ out, int64_t NXi,
                                                         int64_t NYi, int64_t NYo, int64_t nz,
                                                         int axis_x, int64_t off, Taps t)
{
    const int r = t.r;
    const int64_t row = blockIdx.x;          // X*NYo + y
    const int64_t z = (int64_t)blockIdx.y * kBlock + threadIdx.x;
    if (z >= nz) return;
    const int64_t y = row % NYo, X = row / NYo;
    float acc = 0.0f;
    for (int o = -r; o <= r; ++o) {
        const int64_t xi = axis_x ? X + off + o : X;
        const int64_t yi = axis_x ? y : y + off + o;
        if (xi >= 0 && xi < NXi && yi >= 0 && yi < NYi)
            acc = fmaf(t.g[o + r], widen(in[(xi * NYi + yi) * nz + z]), acc);
    }
    out[row * nz + z] = narrow<So>(acc);
}

// ---------------------------------------------------------------------------
// Global shift: mean of F with a fixed reduction tree (deterministic).
// ---------------------------------------------------------------------------

__device__ double block_sum(double v, double *lds)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
        __syncthreads();
    }
    return lds[0];
}

template <typename St>
__global__ __launch_bounds__(kBlock) void k_partial_sums(const St *__restrict__ F, int64_t V,
                                                         double *__restrict__ partials)
{
    __shared__ double lds[kBlock];
    const int64_t chunk = (V + gridDim.x - 1) / gridDim.x;
    const int64_t a = (int64_t)blockIdx.x * chunk;
    const int64_t b = a + chunk < V ? a + chunk : V;
    double s = 0.0;
    for (int64_t i = a + threadIdx.x; i < b; i += kBlock) s += (double)widen(F[i]);
    const double tot = block_sum(s, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_final_mean(const double *__restrict__ partials,
                                                       int n, int64_t V, double *__restrict__ out)
{
    __shared__ double lds[kBlock];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kBlock) s += partials[i];
    const double tot = block_sum(s, lds);
    if (threadIdx.x == 0) out[0] = tot / (double)V;
}

// ---------------------------------------------------------------------------
// Statistics: directional window sums.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int64_t win_count(int64_t i, int64_t n, int B)
{
    int64_t lo = i - (B / 2);
    int64_t hi = lo + B;
    if (lo < 0) lo = 0;
    if (hi > n) hi = n;
    return hi - lo;
}

// z window sums of a = F - s and a^2, one row segment per block staged in LDS.
template <typename St>
__global__ __launch_bounds__(kBlock) void k_zbox(const St *__restrict__ F, int64_t nz, int B,
                                                 const double *__restrict__ shift,
                                                 float *__restrict__ Z1, float *__restrict__ Z2)
{
    extern __shared__ float lds[];
    float *a1 = lds;
    float *a2 = lds + kBlock + B - 1;
    const double s = shift[0];
    const int lo = -(B / 2);
    const int64_t row = blockIdx.x;
    const int64_t z0 = (int64_t)blockIdx.y * kBlock;
    const St *src = F + row * nz;
    for (int i = threadIdx.x; i < kBlock + B - 1; i += kBlock) {
        const int64_t z = z0 + lo + i;
        double a = 0.0;
        if (z >= 0 && z < nz) a = (double)widen(src[z]) - s;
        a1[i] = (float)a;
        a2[i] = (float)(a * a);
    }
    __syncthreads();
    const int64_t z = z0 + threadIdx.x;
    if (z < nz) {
        double s1 = 0.0, s2 = 0.0;
        for (int j = 0; j < B; ++j) {
            s1 += (double)a1[threadIdx.x + j];
            s2 += (double)a2[threadIdx.x + j];
        }
        Z1[row * nz + z] = (float)s1;
        Z2[row * nz + z] = (float)s2;
    }
}

// Running window sums along a strided axis (y or x), FP64 accumulators.
// in/out indexed as base + p*stride for p = 0..n-1.
__device__ __forceinline__ void running_axis(const float *__restrict__ in1,
                                             const float *__restrict__ in2,
                                             float *__restrict__ out1, float *__restrict__ out2,
                                             int64_t n, int64_t stride, int B)
{
    const int64_t lo = -(B / 2);
    double s1 = 0.0, s2 = 0.0;
    for (int64_t p = 0; p < lo + B && p < n; ++p) {
        s1 += (double)in1[p * stride];
        s2 += (double)in2[p * stride];
    }
    for (int64_t i = 0; i < n; ++i) {
        if (i > 0) {
            const int64_t add = i + lo + B - 1;
            const int64_t sub = i + lo - 1;
            if (add < n) { s1 += (double)in1[add * stride]; s2 += (double)in2[add * stride]; }
            if (sub >= 0) { s1 -= (double)in1[sub * stride]; s2 -= (double)in2[sub * stride]; }
        }
        out1[i * stride] = (float)s1;
        out2[i * stride] = (float)s2;
    }
}

__global__ __launch_bounds__(kBlock) void k_ybox(const float *__restrict__ Z1,
                                                 const float *__restrict__ Z2,
                                                 float *__restrict__ Y1, float *__restrict__ Y2,
                                                 int64_t ny, int64_t nz, int B)
{
    const int64_t x = blockIdx.x;
    const int64_t z = (int64_t)blockIdx.y * kBlock + threadIdx.x;
    if (z >= nz) return;
    const int64_t base = x * ny * nz + z;
    running_axis(Z1 + base, Z2 + base, Y1 + base, Y2 + base, ny, nz, B);
}

// x window sums, then mean/std and the selection bit, packed by wave ballot.
template <typename St>
__global__ __launch_bounds__(kBlock) void k_xbox_final(
    const float *__restrict__ Y1, const float *__restrict__ Y2, const St *__restrict__ F,
    int64_t nx, int64_t ny, int64_t nz, Box b, const double *__restrict__ shift,
    float *__restrict__ mean, float *__restrict__ stdev, uint64_t *__restrict__ mask, double k)
{
#pragma clang fp contract(off)
    const int64_t y = blockIdx.x;
    const int64_t z = (int64_t)blockIdx.y * kBlock + threadIdx.x;
    const bool live = z < nz;
    const int64_t plane = ny * nz;
    const int64_t base = y * nz + (live ? z : 0);
    const int64_t W = (nz + 63) / 64;
    const double s = shift[0];
    const int lo = -(b.bx / 2);
    const double cyz = live ? (double)(win_count(y, ny, b.by) * win_count(z, nz, b.bz)) : 1.0;
    double s1 = 0.0, s2 = 0.0;
    if (live)
        for (int64_t p = 0; p < lo + b.bx && p < nx; ++p) {
            s1 += (double)Y1[base + p * plane];
            s2 += (double)Y2[base + p * plane];
        }
    for (int64_t x = 0; x < nx; ++x) {
        bool bit = false;
        if (live) {
            if (x > 0) {
                const int64_t add = x + lo + b.bx - 1;
                const int64_t sub = x + lo - 1;
                if (add < nx) { s1 += (double)Y1[base + add * plane]; s2 += (double)Y2[base + add * plane]; }
                if (sub >= 0) { s1 -= (double)Y1[base + sub * plane]; s2 -= (double)Y2[base + sub * plane]; }
            }
            const double n = cyz * (double)win_count(x, nx, b.bx);
            const double m1 = s1 / n;
            double var = s2 / n - m1 * m1;
            if (var < 0.0) var = 0.0;
            const float mf = (float)(s + m1);
            const float sf = sqrtf((float)var);
            const int64_t i = x * plane + base;
            if (mean) mean[i] = mf;
            if (stdev) stdev[i] = sf;
            if (mask) {
                const double thr = (double)mf + k * (double)sf;
                bit = (double)widen(F[i]) > thr;
            }
        }
        if (mask) {
            const uint64_t word = __ballot(bit);
            if ((threadIdx.x & 63) == 0 && (int64_t)blockIdx.y * kBlock + threadIdx.x < nz)
                mask[(x * ny + y) * W + ((int64_t)blockIdx.y * kBlock + threadIdx.x) / 64] = word;
        }
    }
}

template <typename St>
__global__ __launch_bounds__(kBlock) void k_threshold(const St *__restrict__ F,
                                                      const float *__restrict__ mean,
                                                      const float *__restrict__ stdev,
                                                      int64_t nz, double k,
                                                      uint64_t *__restrict__ mask)
{
#pragma clang fp contract(off)
    const int64_t row = blockIdx.x;
    const int64_t z = (int64_t)blockIdx.y * kBlock + threadIdx.x;
    const int64_t W = (nz + 63) / 64;
    bool bit = false;
    if (z < nz) {
        const int64_t i = row * nz + z;
        const double thr = (double)mean[i] + k * (double)stdev[i];
        bit = (double)widen(F[i]) > thr;
    }
    const uint64_t word = __ballot(bit);
    if ((threadIdx.x & 63) == 0 && z < nz) mask[row * W + z / 64] = word;
}

// ---------------------------------------------------------------------------
// Weighted convolution (Eq. 1): elementwise product and quotient.
// ---------------------------------------------------------------------------

// P = d * w, grid-stride over the cube.
__global__ __launch_bounds__(kBlock) void k_mul(const float *__restrict__ d,
                                                const float *__restrict__ w,
                                                float *__restrict__ P, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        P[i] = d[i] * w[i];
}

// F = N / D where D != 0, else 0 (no weighted support).  F may be N (in
// place: each element is read, then written, by the same lane).
__global__ __launch_bounds__(kBlock) void k_div(const float *N, const float *__restrict__ D,
                                                float *F, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const float den = D[i];
        F[i] = den != 0.0f ? N[i] / den : 0.0f;
    }
}

inline unsigned ztiles(int64_t nz) { return (unsigned)((nz + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_zpass(const void *in, void *T1, Store st, Dims d, const Halo &h,
                        const Taps &tz, hipStream_t s)
{
    if (zpass_fast(tz.r)) return launch_zpass_fast(in, T1, st, d, h, tz, s);
    const dim3 grid((unsigned)(h.NX * h.NY), ztiles(d.nz));
    prof::Scope scope_("k_zpass", s);
    return with_store(st, [&](auto *tag) {
        using St = GSF_STORE_T(tag);
        hipLaunchKernelGGL(k_zpass<St>, grid, dim3(kBlock), (kBlock + 2 * tz.r) * sizeof(float), s,
                           (const St *)in, (float *)T1, d.nz, h.NZ, (int64_t)h.hz, tz);
        return hipGetLastError();
    });
}

hipError_t launch_yx(const void *T1, void *F, void *tmp, Store st, Dims d, const Halo &h,
                     const Taps &txy, double *partials, int *nparts, hipStream_t s)
{
    if (yx_fast(txy.r, d) && yx_fast(txy.r, Dims{h.NX, h.NY, d.nz}))
        return launch_yx_fast(T1, F, st, d, h, txy, partials, nparts, s);
    if (nparts) *nparts = 0;
    return with_store(st, [&](auto *tag) {
        using St = GSF_STORE_T(tag);
        {
            // y pass: T1 (NX x NY rows, FP32) -> tmp (NX x ny rows, FP32)
            prof::Scope scope_("k_strided_pass", s);
            hipLaunchKernelGGL((k_strided_pass<float, float>),
                               dim3((unsigned)(h.NX * d.ny), ztiles(d.nz)), dim3(kBlock), 0, s,
                               (const float *)T1, (float *)tmp, h.NX, h.NY, d.ny, d.nz, 0,
                               (int64_t)h.hy, txy);
        }
        {
            // x pass: tmp (NX x ny rows) -> F (nx x ny rows, storage type)
            prof::Scope scope_("k_strided_pass", s);
            hipLaunchKernelGGL((k_strided_pass<float, St>),
                               dim3((unsigned)(d.nx * d.ny), ztiles(d.nz)), dim3(kBlock), 0, s,
                               (const float *)tmp, (St *)F, h.NX, d.ny, d.ny, d.nz, 1,
                               (int64_t)h.hx, txy);
        }
        return hipGetLastError();
    });
}

hipError_t launch_mean_partials(const double *partials, int n, int64_t V, double *shift,
                                hipStream_t s)
{
    {
        prof::Scope scope_("k_final_mean", s);
        hipLaunchKernelGGL(k_final_mean, dim3(1), dim3(kBlock), 0, s, partials, n, V, shift);
    }
    return hipGetLastError();
}

hipError_t launch_mean(const void *F, Store st, Dims d, double *partials, double *shift,
                       hipStream_t s)
{
    const hipError_t e = with_store(st, [&](auto *tag) {
        using St = GSF_STORE_T(tag);
        prof::Scope scope_("k_partial_sums", s);
        hipLaunchKernelGGL(k_partial_sums<St>, dim3(kShiftBlocks), dim3(kBlock), 0, s,
                           (const St *)F, d.voxels(), partials);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    {
        prof::Scope scope_("k_final_mean", s);
        hipLaunchKernelGGL(k_final_mean, dim3(1), dim3(kBlock), 0, s, (const double *)partials,
                           kShiftBlocks, d.voxels(), shift);
    }
    return hipGetLastError();
}

hipError_t launch_stats(const void *F, Store st, Dims d, Box b, const double *shift, float *ws1,
                        float *ws2, float *ws3, float *ws4, float *mean, float *stdev,
                        uint64_t *mask, double k, hipStream_t s)
{
    // ws1 .. ws4 are consecutive pieces of one workspace, each at least a
    // cube: the fast path's pairs take ws1 and ws2 as one two-cube block
    if (stats_fast_path(b, d))
        return launch_stats_fast(F, st, d, b, shift, ws1, mean, stdev, mask, k, s);
    return with_store(st, [&](auto *tag) {
        using St = GSF_STORE_T(tag);
        const size_t zlds = 2 * (size_t)(kBlock + b.bz - 1) * sizeof(float);
        {
            prof::Scope scope_("k_zbox", s);
            hipLaunchKernelGGL(k_zbox<St>, dim3((unsigned)(d.nx * d.ny), ztiles(d.nz)), dim3(kBlock),
                               zlds, s, (const St *)F, d.nz, b.bz, shift, ws1, ws2);
        }
        {
            prof::Scope scope_("k_ybox", s);
            hipLaunchKernelGGL(k_ybox, dim3((unsigned)d.nx, ztiles(d.nz)), dim3(kBlock), 0, s,
                               (const float *)ws1, (const float *)ws2, ws3, ws4, d.ny, d.nz, b.by);
        }
        {
            prof::Scope scope_("k_xbox_final", s);
            hipLaunchKernelGGL(k_xbox_final<St>, dim3((unsigned)d.ny, ztiles(d.nz)), dim3(kBlock), 0,
                               s, (const float *)ws3, (const float *)ws4, (const St *)F, d.nx, d.ny,
                               d.nz, b, shift, mean, stdev, mask, k);
        }
        return hipGetLastError();
    });
}

hipError_t launch_mul(const float *d, const float *w, float *P, int64_t n, hipStream_t s)
{
    prof::Scope scope_("k_mul", s);
    const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, 65536);
    hipLaunchKernelGGL(k_mul, dim3((unsigned)blocks), dim3(kBlock), 0, s, d, w, P, n);
    return hipGetLastError();
}

hipError_t launch_div(const float *N, const float *D, float *F, int64_t n, hipStream_t s)
{
    prof::Scope scope_("k_div", s);
    const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, 65536);
    hipLaunchKernelGGL(k_div, dim3((unsigned)blocks), dim3(kBlock), 0, s, N, D, F, n);
    return hipGetLastError();
}

hipError_t launch_threshold(const void *F, Store st, const float *mean, const float *stdev,
                            Dims d, double k, uint64_t *mask, hipStream_t s)
{
    prof::Scope scope_("k_threshold", s);
    return with_store(st, [&](auto *tag) {
        using St = GSF_STORE_T(tag);
        hipLaunchKernelGGL(k_threshold<St>, dim3((unsigned)(d.nx * d.ny), ztiles(d.nz)), dim3(kBlock),
                           0, s, (const St *)F, mean, stdev, d.nz, k, mask);
        return hipGetLastError();
    });
}

}  // namespace gsf
