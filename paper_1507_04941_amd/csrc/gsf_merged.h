// gsf_merged.h -- the merged spatial sweep: one kernel applies the spatial
// passes of two or three filters that share one spectral pass (equal
// sigma_z), so T1 is read once for all of them.  Included by the per-type
// instantiation files gsf_merged_<type>.hip and, for the form table, by
// gsf_filter.hip.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <string>

#include "gsf_device.h"
#include "gsf_internal.h"

namespace gsf {

using MergedFn = hipError_t (*)(const void *, void *const *, Dims, const Halo &, const Taps *,
                                double *, int *, hipStream_t);

// Compiled radius sets (ascending) and block shapes (rows per lane P, waves
// per block NW).  Measured register use (FP32, radii 3, 6, 12): P2 NW8 164
// VGPRs (3 waves per SIMD, one block per CU), P1 NW8 103 VGPRs (two blocks
// per CU), P1 NW16 103 VGPRs (one block of 16 waves), P2 NW4 (three blocks
// of 4 waves per CU: half the LDS reads per output of P1, the same T1 rows
// per plane as P1 NW8).
struct MergedRadii {
    int nf;
    int r[3];
};
constexpr int kMergedForms = 4;
constexpr MergedRadii kMergedRadii[kMergedForms] = {
    {3, {3, 6, 12}}, {2, {3, 6, 0}}, {2, {3, 12, 0}}, {2, {6, 12, 0}}};
constexpr int kMergedShapes = 4;
constexpr int kMergedShape[kMergedShapes][2] = {{1, 8}, {2, 8}, {1, 16}, {2, 4}};

// Launcher of compiled form `form` with block shape `shape` for each storage
// type (defined in gsf_merged_f32.hip, _f16.hip, _bf16.hip).
MergedFn merged_fn_f32(int form, int shape);
MergedFn merged_fn_f16(int form, int shape);
MergedFn merged_fn_bf16(int form, int shape);

namespace merged {

// The spatial sweep of every filter of a group that shares one spectral
// pass (equal sigma_z), from one read of T1.  Filters i = 0..NF-1 of radii
// R0, R1, R2 (R2 = 0: two filters): the block's LDS tile holds the rows of the
// widest one (TY + 2 RM); the y pass of row q (centre tile row RM + q) adds
// the two rows at each distance d first, once for all filters, and filter i
// sums its taps over d = R_i .. 1 and the centre in the order k_yx_r uses.
// Each filter keeps its own register ring of partial x sums.  One unrolled turn
// is L = 2 RM + 1 planes for all rings: the partial sum of output plane xo
// lives in slot (xo - p_start) mod L, which a filter of radius R_i fills
// from plane xo - R_i to xo + R_i, writes, and clears; it is next filled from
// plane xo + L - R_i > xo + R_i, so slots never mix outputs, and a filter
// with R_i < RM holds at most 2 R_i + 1 live sums per row (the others are
// constant zeros, which take no register).  Every output is summed in the
// order of k_yx_r, so F is bit for bit what the single-filter sweep gives.
// Shift partials: one block sum per filter, at partials + i * kMaxPartials.
struct TapsM {
    float g[3][2 * kMaxMergedR + 1];
};

template <int A, int B>
constexpr int cmax() { return A > B ? A : B; }

// Tap index o of a radius-R kernel folded onto 0..R: the sampled Gaussian is
// symmetric bit for bit (g[o] and g[2R-o] come from the same exp(-o^2/2s^2)
// and the same sum), so only R+1 taps need registers.
__host__ __device__ constexpr int sym(int o, int R) { return o <= R ? o : 2 * R - o; }

template <int P, int NW, typename St, int R0, int R1, int R2>
__global__ __launch_bounds__(64 * NW) void k_yxm(const float *__restrict__ T, St *F0, St *F1,
                                                 St *F2, int64_t nx64, int64_t ny64,
                                                 int64_t nz64, int64_t xchunk, TapsM t,
                                                 double *__restrict__ partials, int64_t NX64,
                                                 int64_t NY64, int64_t hx64, int64_t hy64)
{
    constexpr int NF = R2 > 0 ? 3 : 2;
    constexpr int RM = cmax<cmax<R0, R1>(), R2>();
    constexpr int L = 2 * RM + 1;
    constexpr int Rs[3] = {R0, R1, R2};
    constexpr int TY = NW * P;
    constexpr int TR = TY + 2 * RM;
    constexpr int LW = (TR + NW - 1) / NW;
    constexpr int S = 2;
    constexpr int D = RM <= 3 ? 2 : 3;
    static_assert(RM <= kMaxMergedR, "merged radius");
    __shared__ float stage[S][TR][64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __builtin_assume(wave >= 0 && wave < NW);
    // Plane indices are 32-bit (planes, rows and in-plane offsets all fit):
    // the x loop's bounds and tests then stay in scalar registers and scalar
    // compares, and leave room for the taps, which are also uniform.
    const int z = (int)blockIdx.x * 64 + lane;
    const int yb = (int)blockIdx.y * TY;
    const int y0 = yb + wave * P;
    const int nx = (int)nx64, ny = (int)ny64, nz = (int)nz64, NX = (int)NX64;
    const int xa = (int)blockIdx.z * (int)xchunk;
    const int xb = xa + (int)xchunk < nx ? xa + (int)xchunk : nx;
    const int hx = (int)hx64;
    const bool zl = z < nz;
    constexpr uint32_t SZ = sizeof(St);
    constexpr uint32_t TSZ = sizeof(float);
    const uint32_t tplane = (uint32_t)NY64 * (uint32_t)nz;         // < 2^28 voxels
    const uint32_t tplane_b = tplane * TSZ;
    const uint32_t plane = (uint32_t)ny * (uint32_t)nz;
    const uint32_t plane_b = plane * SZ;
    const uint32_t row_b = (uint32_t)nz * SZ;
    St *const Fs[3] = {F0, F1, F2};
    uint32_t ldo[LW];
#pragma unroll
    for (int i = 0; i < LW; ++i) {
        const int tr = wave + i * NW;
        ldo[i] = tr < TR ? (uint32_t)((yb + (int)hy64 - RM + tr) * nz + z) * TSZ : kOOB;
    }
    const uint32_t st0 = zl ? (uint32_t)(y0 * nz + z) * SZ : kOOB;

    float acc[3][P][L];
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int q = 0; q < P; ++q)
#pragma unroll
            for (int m = 0; m < L; ++m) acc[f][q][m] = 0.0f;
    double fsum[3] = {0.0, 0.0, 0.0};
    const int p_start = xa - RM;
    const int p_end = xb - 1 + RM;

    auto load_plane = [&](int xq, float (&r)[LW]) {
        const int xt = xq + hx;
        const bool in = (unsigned)xt < (unsigned)NX;
        const __amdgpu_buffer_rsrc_t rt =
            buf(T + (size_t)(in ? xt : 0) * tplane, in ? tplane_b : 0u);
#pragma unroll
        for (int i = 0; i < LW; ++i) r[i] = buf_ld(rt, ldo[i]);
    };
    auto store_stage = [&](int st, const float (&r)[LW]) {
#pragma unroll
        for (int i = 0; i < LW; ++i) {
            const int tr = wave + i * NW;
            if (tr < TR) stage[st][tr][lane] = r[i];
        }
    };
    float rq[D][LW];
    load_plane(p_start, rq[0]);
    store_stage(p_start & (S - 1), rq[0]);
#pragma unroll
    for (int k = 0; k < D; ++k) load_plane(p_start + 1 + k, rq[k]);

#pragma nounroll
    for (int p0 = p_start; p0 <= p_end; p0 += L) {
#pragma unroll
        for (int j = 0; j < L; ++j) {
            const int xp = p0 + j;
            __syncthreads();
            store_stage((xp + 1) & (S - 1), rq[0]);
#pragma unroll
            for (int k = 0; k + 1 < D; ++k)
#pragma unroll
                for (int i = 0; i < LW; ++i) rq[k][i] = rq[k + 1][i];
            load_plane(xp + D + 1, rq[D - 1]);
            const int sx = xp & (S - 1);
            // y passes in pair form: the sums of the two rows at distance d
            // from each output row's centre are formed once and shared by
            // every filter of the group (radius R_i uses d <= R_i), outermost
            // pair first, the centre last, as the single-filter sweep sums
            float pd[P][RM + 1];
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const int c = wave * P + q + RM;
                pd[q][0] = stage[sx][c][lane];
#pragma unroll
                for (int d = 1; d <= RM; ++d)
                    pd[q][d] = stage[sx][c - d][lane] + stage[sx][c + d][lane];
            }
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const int R = Rs[f];
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    float t2 = 0.0f;
#pragma unroll
                    for (int d = R; d >= 1; --d) t2 = fmaf(t.g[f][R - d], pd[q][d], t2);
                    t2 = fmaf(t.g[f][R], pd[q][0], t2);
#pragma unroll
                    for (int k = 0; k <= 2 * R; ++k) {
                        const int slot = (j - R + k + L) % L;
                        acc[f][q][slot] = fmaf(t.g[f][sym(2 * R - k, R)], t2, acc[f][q][slot]);
                    }
                }
                const int slot_o = (j - R + L) % L;
                const int xo = xp - R;
                if (xo >= xa && xo < xb) {
                    const __amdgpu_buffer_rsrc_t rf = buf(Fs[f] + (size_t)xo * plane, plane_b);
#pragma unroll
                    for (int q = 0; q < P; ++q) {
                        const float v = widen(narrow<St>(acc[f][q][slot_o]));
                        sbuf_st<St>(rf, v, st0 + (uint32_t)q * row_b);
                        if (zl && y0 + q < ny) fsum[f] += (double)v;
                    }
                }
#pragma unroll
                for (int q = 0; q < P; ++q) acc[f][q][slot_o] = 0.0f;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    if (partials) {
        __shared__ double red[64 * NW];
        const int64_t bid = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            __syncthreads();
            red[threadIdx.x] = fsum[f];
            __syncthreads();
            for (int w = 32 * NW; w > 0; w >>= 1) {
                if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
                __syncthreads();
            }
            if (threadIdx.x == 0) partials[(int64_t)f * kMaxPartials + bid] = red[0];
        }
    }
}

// Launch of a merged sweep; F[i] and txy[i] belong to the filter of radius
// Rs[i] (R0, R1[, R2] as compiled).  The grid is k_yx_r's for the widest
// radius, with its rows per lane P.
template <int P, int NW, typename St, int R0, int R1, int R2>
hipError_t yxm(const void *T, void *const *F, Dims d, const Halo &h, const Taps *txy,
               double *partials, int *nparts, hipStream_t s)
{
    constexpr int RM = cmax<cmax<R0, R1>(), R2>();
    constexpr int NF = R2 > 0 ? 3 : 2;
    const int64_t tz = (d.nz + 63) / 64;
    const int64_t ty = (d.ny + NW * P - 1) / (NW * P);
    const int64_t target = active_tune().sweep_blocks;
    int64_t nxc = (target + tz * ty - 1) / (tz * ty);
    const int64_t max_chunks = d.nx / (4 * (2 * RM + 1)) > 0 ? d.nx / (4 * (2 * RM + 1)) : 1;
    if (nxc > max_chunks) nxc = max_chunks;
    if (nxc < 1) nxc = 1;
    const int64_t xchunk = (d.nx + nxc - 1) / nxc;
    nxc = (d.nx + xchunk - 1) / xchunk;
    const dim3 grid((unsigned)tz, (unsigned)ty, (unsigned)nxc);
    const int64_t blocks = tz * ty * nxc;
    if (!partials || blocks > kMaxPartials) partials = nullptr;
    if (nparts) *nparts = partials ? (int)blocks : 0;
    TapsM tm{};
    for (int f = 0; f < NF; ++f)
        for (int o = 0; o <= 2 * txy[f].r; ++o) tm.g[f][o] = txy[f].g[o];
    static const std::string name = "k_yx" + std::to_string(NF) + "_r<" + std::to_string(R0) +
                                    "," + std::to_string(R1) +
                                    (R2 > 0 ? "," + std::to_string(R2) : std::string()) +
                                    store_suffix<St>() + ",p" + std::to_string(P) + "w" +
                                    std::to_string(NW) + ">";
    prof::Scope scope(name.c_str(), s);
    hipLaunchKernelGGL((k_yxm<P, NW, St, R0, R1, R2>), grid, dim3(64 * NW), 0, s,
                       (const float *)T, (St *)F[0], (St *)F[1], (St *)(NF > 2 ? F[2] : nullptr),
                       d.nx, d.ny, d.nz, xchunk, tm, partials, h.NX, h.NY, (int64_t)h.hx,
                       (int64_t)h.hy);
    return hipGetLastError();
}



// The launchers of every compiled form and shape for storage type St.
template <typename St, int R0, int R1, int R2>
constexpr std::array<MergedFn, kMergedShapes> shapes_of()
{
    return {&yxm<kMergedShape[0][0], kMergedShape[0][1], St, R0, R1, R2>,
            &yxm<kMergedShape[1][0], kMergedShape[1][1], St, R0, R1, R2>,
            &yxm<kMergedShape[2][0], kMergedShape[2][1], St, R0, R1, R2>,
            &yxm<kMergedShape[3][0], kMergedShape[3][1], St, R0, R1, R2>};
}

template <typename St>
MergedFn lookup(int form, int shape)
{
    static const std::array<MergedFn, kMergedShapes> tab[kMergedForms] = {
        shapes_of<St, 3, 6, 12>(), shapes_of<St, 3, 6, 0>(), shapes_of<St, 3, 12, 0>(),
        shapes_of<St, 6, 12, 0>()};
    return tab[form][shape];
}

}  // namespace merged
}  // namespace gsf
