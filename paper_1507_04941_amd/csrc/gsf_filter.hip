// gsf_filter.hip -- the separable Gaussian filter (Eq. 2, §2.1) for gfx950.
//
// The 3-D filter is the outer product gxy (x) gxy (x) gz, so Eq. 2 is applied
// as a spectral pass followed by a fused spatial pass:
//   k_zpass_rows<R>: T1 = gz * d along z (contiguous).  A block walks 16
//     rows of a 1024-wide z chunk (256 wide for short rows), staging each
//     row with its +-R halo in a double-buffered LDS tile one row ahead of
//     use (coalesced loads); every
//     lane then holds a (4 + 2R)-wide window in registers (ds_read_b128) and
//     produces 4 consecutive outputs, so each staged value feeds up to
//     4(2R+1) FMAs.
//   k_yx_r<R, P, NW>: F = gxy * (gxy * T1 along y) along x.  A block owns a
//     64-wide z strip (one lane per z, coalesced rows) and NW waves x P rows of
//     y, and sweeps an x range plane by plane.  The block's waves load each
//     plane's NW*P + 2R rows once, cooperatively, two or three planes ahead,
//     into a two-stage LDS ring (one barrier per plane); each lane then forms the
//     y pass of its P points from LDS and scatters it into a register ring of
//     2R+1 partial x sums per point; the oldest sum is complete and written
//     after every plane.  T1 is read once (plus the 2R halo rows per block)
//     and F written once.
// Taps are compile-time indexed kernel arguments (scalar registers).  Every
// output sums its taps in ascending offset order, as in the definition.
#include <hip/hip_runtime.h>

#include <array>
#include <string>
#include <utility>

#include "gsf_device.h"
#include "gsf_internal.h"
#include "gsf_merged.h"

namespace gsf {
namespace {

constexpr int kThreads = 256;

// Four consecutive elements (16-byte aligned for FP32, 8-byte for 16-bit).
template <typename St>
__device__ __forceinline__ float4 load4(const St *p)
{
    if constexpr (sizeof(St) == 4) {
        return *reinterpret_cast<const float4 *>(p);
    } else {
        const uint2 u = *reinterpret_cast<const uint2 *>(p);
        return make_float4(widen(__builtin_bit_cast(St, (unsigned short)(u.x & 0xffffu))),
                           widen(__builtin_bit_cast(St, (unsigned short)(u.x >> 16))),
                           widen(__builtin_bit_cast(St, (unsigned short)(u.y & 0xffffu))),
                           widen(__builtin_bit_cast(St, (unsigned short)(u.y >> 16))));
    }
}

template <typename St>
__device__ __forceinline__ void store4(St *p, const float (&v)[4])
{
    if constexpr (sizeof(St) == 4) {
        *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
        const unsigned b0 = __builtin_bit_cast(unsigned short, narrow<St>(v[0]));
        const unsigned b1 = __builtin_bit_cast(unsigned short, narrow<St>(v[1]));
        const unsigned b2 = __builtin_bit_cast(unsigned short, narrow<St>(v[2]));
        const unsigned b3 = __builtin_bit_cast(unsigned short, narrow<St>(v[3]));
        *reinterpret_cast<uint2 *>(p) = make_uint2(b0 | (b1 << 16), b2 | (b3 << 16));
    }
}

// The spectral pass: a block of T threads walks kZRows consecutive rows of
// one z chunk of 4T outputs (T = 256, or 64 for short rows; four outputs per
// lane), loading each row one row ahead of its use
// into a double-buffered FP32 LDS tile (one barrier per row).  When the row
// lengths and the z halo are multiples of 4 (A), every row starts aligned
// and a lane loads and stores its four values with single 4-element
// accesses; otherwise it uses element accesses through range-checked buffer
// descriptors (values past the row read 0, stores past it are dropped).
// With MUL the pass filters the voxel-wise product in * wv (FP32 products,
// as a separate multiply would store them): the weighted numerator of Eq. 1.
constexpr int kZRows = 16;

template <int R, typename St, bool A, bool MUL = false, int T = kThreads>
__global__ __launch_bounds__(T) void k_zpass_rows(const St *__restrict__ in,
                                                         float *__restrict__ out, int64_t nrows,
                                                         int64_t nz, int64_t NZ, int64_t zoff,
                                                         Taps t, const St *__restrict__ wv = nullptr)
{
    static_assert(2 * R <= T, "halo lanes");
    constexpr int NW = (4 + 2 * R + 3) / 4;          // float4 window per lane
    constexpr int ZO = 4 * T;                        // z outputs per block
    constexpr int TL = ZO + 4 * NW + 4;           // tile length, float4 multiple
    constexpr uint32_t SZ = sizeof(St);
    __shared__ float4 tile4[2][TL / 4];
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * kZRows;
    const int64_t r1 = r0 + kZRows < nrows ? r0 + kZRows : nrows;
    const int64_t z0 = (int64_t)blockIdx.y * ZO;
    // core z of the output maps to input z + zoff in rows of NZ values
    const int64_t zm = z0 + 4 * tid;                 // this lane's four values and outputs
    const bool mine = zm < nz;                       // outputs inside the core (A)
    const bool load = zm + zoff < NZ;                // inputs inside the array (A)
    // halo: lanes 0 .. 2R-1 fetch z0 - R + lane (left) and z0 + ZO + lane - R (right)
    const int64_t zh = tid < R ? z0 - R + tid : z0 + ZO + (tid - R);
    const bool halo = tid < 2 * R && zh + zoff >= 0 && zh + zoff < NZ;
    const int th = tid < R ? tid : ZO + tid;      // its tile index
    // element form: byte offsets inside a row (zm + zoff >= 0; a row is
    // below 2^31 bytes)
    const uint32_t om = (uint32_t)((zm + zoff) * SZ);
    const uint32_t oh = halo ? (uint32_t)((zh + zoff) * SZ) : kOOB;
    const uint32_t os = (uint32_t)(zm * sizeof(float));
    auto fetch_one = [&](const St *src, int64_t r, float4 &m, float &h) {
        if constexpr (A) {
            const St *row = src + r * NZ + zoff;
            m = load ? load4(row + zm) : make_float4(0.f, 0.f, 0.f, 0.f);
            h = halo ? widen(row[zh]) : 0.0f;
        } else {
            const __amdgpu_buffer_rsrc_t rr = buf(src + r * NZ, (uint32_t)(NZ * SZ));
            m.x = sbuf_ld<St>(rr, om);
            m.y = sbuf_ld<St>(rr, om + SZ);
            m.z = sbuf_ld<St>(rr, om + 2 * SZ);
            m.w = sbuf_ld<St>(rr, om + 3 * SZ);
            h = sbuf_ld<St>(rr, oh);
        }
    };
    auto fetch = [&](int64_t r, float4 &m, float &h) {
        fetch_one(in, r, m, h);
        if constexpr (MUL) {
            float4 mw;
            float hw;
            fetch_one(wv, r, mw, hw);
            m.x *= mw.x;
            m.y *= mw.y;
            m.z *= mw.z;
            m.w *= mw.w;
            h *= hw;
        }
    };
    float4 m;
    float h;
    fetch(r0, m, h);
    for (int64_t r = r0; r < r1; ++r) {
        const int b = (int)((r - r0) & 1);
        float *tile = reinterpret_cast<float *>(tile4[b]);
        tile[R + 4 * tid] = m.x;
        tile[R + 4 * tid + 1] = m.y;
        tile[R + 4 * tid + 2] = m.z;
        tile[R + 4 * tid + 3] = m.w;
        if (tid < 2 * R) tile[th] = h;
        __syncthreads();
        if (r + 1 < r1) fetch(r + 1, m, h);
        float w[4 * NW];
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            const float4 q = tile4[b][tid + j];
            w[4 * j] = q.x;
            w[4 * j + 1] = q.y;
            w[4 * j + 2] = q.z;
            w[4 * j + 3] = q.w;
        }
        // pair form (taps symmetric bit for bit): outermost pair first, the
        // centre last, as every spectral and spatial pass here sums
        float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int d = R; d >= 1; --d) {
            const float g = t.g[R - d];
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[k] = fmaf(g, w[k + R - d] + w[k + R + d], acc[k]);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = fmaf(t.g[R], w[k + R], acc[k]);
        if constexpr (A) {
            if (mine) store4(out + r * nz + zm, acc);
        } else {
            const __amdgpu_buffer_rsrc_t ro = buf(out + r * nz, (uint32_t)(nz * sizeof(float)));
#pragma unroll
            for (int k = 0; k < 4; ++k) buf_st(ro, acc[k], os + (uint32_t)k * sizeof(float));
        }
    }
}

// Two spectral passes of radii R1 < R2 from one read of the input: the
// block stages each row with the +-R2 halo, every lane holds the
// (4 + 2 R2)-wide window, and output k of the radius-R1 pass takes the
// window's entries R2 - R1 + k .. R2 + R1 + k, the same values in the same
// tap order as k_zpass_rows<R1>, so both outputs are bit for bit those of
// the single passes.  Used when two filter groups of one call have
// different sigma_z (the cube is then read once instead of twice).
template <int R1, int R2, typename St, bool A, int T = kThreads>
__global__ __launch_bounds__(T) void k_zpass2_rows(const St *__restrict__ in,
                                                          float *__restrict__ out1,
                                                          float *__restrict__ out2,
                                                          int64_t nrows, int64_t nz, int64_t NZ,
                                                          int64_t zoff, Taps t1, Taps t2)
{
    static_assert(R1 < R2, "radii ascending");
    static_assert(2 * R2 <= T, "halo lanes");
    constexpr int R = R2;
    constexpr int NW = (4 + 2 * R + 3) / 4;          // float4 window per lane
    constexpr int ZO = 4 * T;                        // z outputs per block
    constexpr int TL = ZO + 4 * NW + 4;           // tile length, float4 multiple
    constexpr int DR = R2 - R1;
    constexpr uint32_t SZ = sizeof(St);
    __shared__ float4 tile4[2][TL / 4];
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * kZRows;
    const int64_t r1 = r0 + kZRows < nrows ? r0 + kZRows : nrows;
    const int64_t z0 = (int64_t)blockIdx.y * ZO;
    const int64_t zm = z0 + 4 * tid;
    const bool mine = zm < nz;
    const bool load = zm + zoff < NZ;
    const int64_t zh = tid < R ? z0 - R + tid : z0 + ZO + (tid - R);
    const bool halo = tid < 2 * R && zh + zoff >= 0 && zh + zoff < NZ;
    const int th = tid < R ? tid : ZO + tid;
    const uint32_t om = (uint32_t)((zm + zoff) * SZ);
    const uint32_t oh = halo ? (uint32_t)((zh + zoff) * SZ) : kOOB;
    const uint32_t os = (uint32_t)(zm * sizeof(float));
    auto fetch = [&](int64_t r, float4 &m, float &h) {
        if constexpr (A) {
            const St *row = in + r * NZ + zoff;
            m = load ? load4(row + zm) : make_float4(0.f, 0.f, 0.f, 0.f);
            h = halo ? widen(row[zh]) : 0.0f;
        } else {
            const __amdgpu_buffer_rsrc_t rr = buf(in + r * NZ, (uint32_t)(NZ * SZ));
            m.x = sbuf_ld<St>(rr, om);
            m.y = sbuf_ld<St>(rr, om + SZ);
            m.z = sbuf_ld<St>(rr, om + 2 * SZ);
            m.w = sbuf_ld<St>(rr, om + 3 * SZ);
            h = sbuf_ld<St>(rr, oh);
        }
    };
    auto put = [&](float *out, int64_t r, const float (&acc)[4]) {
        if constexpr (A) {
            if (mine) store4(out + r * nz + zm, acc);
        } else {
            const __amdgpu_buffer_rsrc_t ro = buf(out + r * nz, (uint32_t)(nz * sizeof(float)));
#pragma unroll
            for (int k = 0; k < 4; ++k) buf_st(ro, acc[k], os + (uint32_t)k * sizeof(float));
        }
    };
    float4 m;
    float h;
    fetch(r0, m, h);
    for (int64_t r = r0; r < r1; ++r) {
        const int b = (int)((r - r0) & 1);
        float *tile = reinterpret_cast<float *>(tile4[b]);
        tile[R + 4 * tid] = m.x;
        tile[R + 4 * tid + 1] = m.y;
        tile[R + 4 * tid + 2] = m.z;
        tile[R + 4 * tid + 3] = m.w;
        if (tid < 2 * R) tile[th] = h;
        __syncthreads();
        if (r + 1 < r1) fetch(r + 1, m, h);
        float w[4 * NW];
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            const float4 q = tile4[b][tid + j];
            w[4 * j] = q.x;
            w[4 * j + 1] = q.y;
            w[4 * j + 2] = q.z;
            w[4 * j + 3] = q.w;
        }
        // both radii share the centre (window entry R2 + k) and the pair sums
        // of the inner R1 distances; each pass sums in pair form (outermost
        // pair first, centre last), as the single passes do
        float pr[4][R1 + 1];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int d = 1; d <= R1; ++d) pr[k][d] = w[k + R2 - d] + w[k + R2 + d];
        float a1[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int d = R1; d >= 1; --d) {
            const float g = t1.g[R1 - d];
#pragma unroll
            for (int k = 0; k < 4; ++k) a1[k] = fmaf(g, pr[k][d], a1[k]);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) a1[k] = fmaf(t1.g[R1], w[k + R2], a1[k]);
        put(out1, r, a1);
        float a2[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int d = R2; d >= 1; --d) {
            const float g = t2.g[R2 - d];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                a2[k] = fmaf(g, d <= R1 ? pr[k][d <= R1 ? d : 0] : w[k + R2 - d] + w[k + R2 + d],
                             a2[k]);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) a2[k] = fmaf(t2.g[R2], w[k + R2], a2[k]);
        put(out2, r, a2);
    }
}

// With DIV, F holds the numerator N of Eq. 1 on entry and the sweep's
// result D is not stored: each output becomes N / D (0 where D = 0), read
// and written in place by the same lane.
template <int R, int P, int NW, typename St, bool DIV = false>
__global__ __launch_bounds__(64 * NW) void k_yx_r(const float *__restrict__ T,
                                                  St *F, int64_t nx64, int64_t ny64,
                                                  int64_t nz64, int64_t xchunk, Taps t,
                                                  double *__restrict__ partials, int64_t NX64,
                                                  int64_t NY64, int64_t hx64, int64_t hy64)
{
    constexpr int L = 2 * R + 1;
    constexpr int TY = NW * P;            // output rows of the block
    constexpr int TR = TY + 2 * R;        // rows of T1 one plane of the block needs
    constexpr int LW = (TR + NW - 1) / NW;   // rows each wave loads per plane
    // Two LDS stages, one barrier per plane: plane xp is read from one stage
    // while plane xp+1 is stored into the other, after the barrier that
    // retired plane xp-1.  Measured with R = 12: 0.665 ms; one barrier per two
    // planes with four stages 0.668 ms; storing the next plane before the
    // barrier (three stages) 0.695 ms.
    constexpr int S = 2;
    // Planes held in registers ahead of their store.  Measured: R = 12, 6, 3
    // with two planes 0.666, 0.477, 0.436 ms; three 0.645, 0.464, 0.441 ms;
    // four 0.795 ms for R = 12 (its registers then allow one block per CU).
    constexpr int D = R <= 3 ? 2 : 3;
    __shared__ float stage[S][TR][64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    __builtin_assume(wave >= 0 && wave < NW);
    // 32-bit plane, row and in-plane indices (a plane holds < 2^28 voxels):
    // the x loop's bounds and tests stay scalar, which keeps the uniform
    // state (taps included) in scalar registers without spills.
    const int z = (int)blockIdx.x * 64 + lane;
    const int yb = (int)blockIdx.y * TY;                    // first output row of the block
    const int y0 = yb + wave * P;                           // this wave's first row
    const int nx = (int)nx64, ny = (int)ny64, nz = (int)nz64, NX = (int)NX64;
    const int xa = (int)blockIdx.z * (int)xchunk;
    const int xb = xa + (int)xchunk < nx ? xa + (int)xchunk : nx;
    const int hx = (int)hx64;
    const bool zl = z < nz;
    // T1 is NX x NY rows of nz (core z); F is the nx x ny x nz core, whose
    // (x, y) reads T1 at (x + hx, y + hy)
    constexpr uint32_t SZ = sizeof(St);
    constexpr uint32_t TSZ = sizeof(float);                 // T1 is FP32
    const uint32_t tplane = (uint32_t)NY64 * (uint32_t)nz;
    const uint32_t tplane_b = tplane * TSZ;
    const uint32_t plane = (uint32_t)ny * (uint32_t)nz;
    const uint32_t plane_b = plane * SZ;
    const uint32_t row_b = (uint32_t)nz * SZ;
    // rows w, w + NW, ... of the block's TR-row window are this wave's to load;
    // offsets wrap for rows above the array and read 0 through the range check
    uint32_t ldo[LW];
#pragma unroll
    for (int i = 0; i < LW; ++i) {
        const int tr = wave + i * NW;
        ldo[i] = tr < TR ? (uint32_t)((yb + (int)hy64 - R + tr) * nz + z) * TSZ : kOOB;
    }
    const uint32_t st0 = zl ? (uint32_t)(y0 * nz + z) * SZ : kOOB;

    float acc[P][L];
#pragma unroll
    for (int q = 0; q < P; ++q)
#pragma unroll
        for (int m = 0; m < L; ++m) acc[q][m] = 0.0f;

    double fsum = 0.0;                                       // this lane's share of sum(F)
    const int p_start = xa - R;
    const int p_end = xb - 1 + R;                            // inclusive

    // a plane outside [0, nx) gets an empty range, so its rows read 0
    auto load_plane = [&](int xq, float (&r)[LW]) {
        const int xt = xq + hx;                              // T1 plane of core plane xq
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
    // prologue: plane p_start in LDS, planes p_start+1 .. p_start+D in
    // registers.  Step xp meets the barrier (plane xp visible, plane xp-1
    // retired), stores plane xp+1 into the retired stage and issues the loads
    // of plane xp+D+1, so a load has D planes of compute to arrive.  Ring
    // turns start at p_start (the ring slot of plane xp is (xp - p_start)
    // mod L) and the last turn runs to its end: the surplus planes read 0 or
    // feed only outputs past xb, which are never written.  (Branching around
    // them defeats the load pipelining.)
    float rq[D][LW];
    load_plane(p_start, rq[0]);
    store_stage(p_start & (S - 1), rq[0]);
#pragma unroll
    for (int k = 0; k < D; ++k) load_plane(p_start + 1 + k, rq[k]);

#pragma nounroll
    for (int p0 = p_start; p0 <= p_end; p0 += L) {
#pragma unroll
        for (int j = 0; j < L; ++j) {
            // Planes outside [0, nx) read 0.
            const int xp = p0 + j;                           // (xp - p_start) mod L == j
            __syncthreads();
            store_stage((xp + 1) & (S - 1), rq[0]);          // plane xp+1
#pragma unroll
            for (int k = 0; k + 1 < D; ++k)
#pragma unroll
                for (int i = 0; i < LW; ++i) rq[k][i] = rq[k + 1][i];
            load_plane(xp + D + 1, rq[D - 1]);               // plane xp+D+1
            const int sx = xp & (S - 1);                     // stage of plane xp
#pragma unroll
            for (int q = 0; q < P; ++q) {
                // y pass in pair form: rows at equal distance from the centre
                // row are added first (taps symmetric bit for bit), outermost
                // pair first, the centre last
                const int c = wave * P + q + R;
                float t2 = 0.0f;
#pragma unroll
                for (int d = R; d >= 1; --d)
                    t2 = fmaf(t.g[R - d], stage[sx][c - d][lane] + stage[sx][c + d][lane], t2);
                t2 = fmaf(t.g[R], stage[sx][c][lane], t2);
#pragma unroll
                for (int k = 0; k < L; ++k) {
                    const int slot = (j + R + 1 + k) % L;
                    acc[q][slot] = fmaf(t.g[2 * R - k], t2, acc[q][slot]);
                }
            }
            const int slot_o = (j + R + 1) % L;
            const int xo = xp - R;
            if (xo >= xa && xo < xb) {
                const __amdgpu_buffer_rsrc_t rf = buf(F + (size_t)xo * plane, plane_b);
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    if constexpr (DIV) {
                        const uint32_t o = st0 + (uint32_t)q * row_b;
                        const float den = acc[q][slot_o];
                        const float num = sbuf_ld<St>(rf, o);
                        sbuf_st<St>(rf, den != 0.0f ? num / den : 0.0f, o);
                    } else {
                        // the shift sums the stored (rounded) values
                        const float v = widen(narrow<St>(acc[q][slot_o]));
                        sbuf_st<St>(rf, v, st0 + (uint32_t)q * row_b);
                        if (zl && y0 + q < ny) fsum += (double)v;
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < P; ++q) acc[q][slot_o] = 0.0f;
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    if (partials) {
        // fixed-order block reduction of the lane sums (for the statistics' shift)
        __shared__ double red[64 * NW];
        red[threadIdx.x] = fsum;
        __syncthreads();
        for (int w = 32 * NW; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0)
            partials[((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = red[0];
    }
}

// Timing names per radius and storage type (the profile aggregates launches
// by name), built once.
template <typename St>
const char *kernel_name(const char *base, int r)
{
    static const std::array<std::array<std::string, kMaxFastRz + 1>, 2> tab = [] {
        std::array<std::array<std::string, kMaxFastRz + 1>, 2> t;
        const char *bases[2] = {"k_zpass_r", "k_yx_r"};
        for (int k = 0; k < 2; ++k)
            for (int i = 0; i <= kMaxFastRz; ++i)
                t[k][i] = std::string(bases[k]) + "<" + std::to_string(i) + store_suffix<St>() + ">";
        return t;
    }();
    return tab[base[2] == 'z' ? 0 : 1][r].c_str();
}

// Block width of a spectral pass over rows of nz outputs with halo r: 256
// threads (1024 outputs per block) or 64 (256 outputs), whichever stages the
// fewest values per row, ceil(nz / outputs) (outputs + 2r); ties to the wide
// block.  A 1024-wide block over a short row leaves most lanes idle (rows of
// 112 values, the smallest halo sub-cubes, use 11% of them).
inline bool zpass_narrow(int64_t nz, int r)
{
    const int64_t wide = (nz + 4 * kThreads - 1) / (4 * kThreads) * (4 * kThreads + 2 * r);
    const int64_t narrow = (nz + 4 * 64 - 1) / (4 * 64) * (4 * 64 + 2 * r);
    return narrow < wide;
}

template <int R, typename St, bool MUL>
hipError_t zpass_impl(const void *in_, void *out_, Dims d, const Halo &h, const Taps &tz,
                      hipStream_t s, const void *w_)
{
    const St *in = (const St *)in_;
    const St *w = (const St *)w_;
    float *out = (float *)out_;
    const int64_t rows = h.NX * h.NY;
    prof::Scope scope(MUL ? "k_zpass_r_mul" : kernel_name<St>("k_zpass_r", R), s);
    const bool A = d.nz % 4 == 0 && h.NZ % 4 == 0 && h.hz % 4 == 0;
    auto go = [&](auto tc, auto ac) {
        constexpr int T = decltype(tc)::value;
        constexpr bool AL = decltype(ac)::value;
        const dim3 grid((unsigned)((rows + kZRows - 1) / kZRows),
                        (unsigned)((d.nz + 4 * T - 1) / (4 * T)));
        hipLaunchKernelGGL((k_zpass_rows<R, St, AL, MUL, T>), grid, dim3(T), 0, s, in, out, rows,
                           d.nz, h.NZ, (int64_t)h.hz, tz, w);
    };
    using W = std::integral_constant<int, kThreads>;
    using N = std::integral_constant<int, 64>;
    using Y = std::true_type;
    using F = std::false_type;
    if (zpass_narrow(d.nz, R)) {
        if (A) go(N{}, Y{}); else go(N{}, F{});
    } else {
        if (A) go(W{}, Y{}); else go(W{}, F{});
    }
    return hipGetLastError();
}

template <int R, typename St>
hipError_t zpass_r(const void *in, void *out, Dims d, const Halo &h, const Taps &tz,
                   hipStream_t s)
{
    return zpass_impl<R, St, false>(in, out, d, h, tz, s, nullptr);
}

// Radius pairs with a compiled two-pass spectral kernel (ascending).
constexpr int kZPairs = 6;
constexpr int kZPair[kZPairs][2] = {{3, 6}, {3, 12}, {6, 12}, {6, 24}, {12, 24}, {3, 24}};

template <int R1, int R2, typename St>
hipError_t zpass2_impl(const void *in_, void *o1, void *o2, Dims d, const Halo &h,
                       const Taps &t1, const Taps &t2, hipStream_t s)
{
    const St *in = (const St *)in_;
    const int64_t rows = h.NX * h.NY;
    static const std::string name = "k_zpass2_r<" + std::to_string(R1) + "," +
                                    std::to_string(R2) + store_suffix<St>() + ">";
    prof::Scope scope(name.c_str(), s);
    const bool A = d.nz % 4 == 0 && h.NZ % 4 == 0 && h.hz % 4 == 0;
    auto go = [&](auto tc, auto ac) {
        constexpr int T = decltype(tc)::value;
        constexpr bool AL = decltype(ac)::value;
        const dim3 grid((unsigned)((rows + kZRows - 1) / kZRows),
                        (unsigned)((d.nz + 4 * T - 1) / (4 * T)));
        hipLaunchKernelGGL((k_zpass2_rows<R1, R2, St, AL, T>), grid, dim3(T), 0, s, in,
                           (float *)o1, (float *)o2, rows, d.nz, h.NZ, (int64_t)h.hz, t1, t2);
    };
    using W = std::integral_constant<int, kThreads>;
    using N = std::integral_constant<int, 64>;
    using Y = std::true_type;
    using F = std::false_type;
    if (zpass_narrow(d.nz, R2)) {
        if (A) go(N{}, Y{}); else go(N{}, F{});
    } else {
        if (A) go(W{}, Y{}); else go(W{}, F{});
    }
    return hipGetLastError();
}

using Z2Fn = hipError_t (*)(const void *, void *, void *, Dims, const Halo &, const Taps &,
                            const Taps &, hipStream_t);

template <typename St>
const Z2Fn *z2tab()
{
    static const Z2Fn tab[kZPairs] = {&zpass2_impl<3, 6, St>,   &zpass2_impl<3, 12, St>,
                                      &zpass2_impl<6, 12, St>,  &zpass2_impl<6, 24, St>,
                                      &zpass2_impl<12, 24, St>, &zpass2_impl<3, 24, St>};
    return tab;
}

template <int R, int P, int NW, typename St, bool DIV = false>
hipError_t yx_r(const void *T, void *F, Dims d, const Halo &h, const Taps &txy, double *partials,
                int *nparts, hipStream_t s)
{
    const int64_t tz = (d.nz + 63) / 64;
    const int64_t ty = (d.ny + NW * P - 1) / (NW * P);
    // Split x so the grid has enough blocks to fill the chip; each chunk
    // re-reads 2R planes of halo.
    const int64_t target = active_tune().sweep_blocks;
    int64_t nxc = (target + tz * ty - 1) / (tz * ty);
    const int64_t max_chunks = d.nx / (4 * (2 * R + 1)) > 0 ? d.nx / (4 * (2 * R + 1)) : 1;
    if (nxc > max_chunks) nxc = max_chunks;
    if (nxc < 1) nxc = 1;
    const int64_t xchunk = (d.nx + nxc - 1) / nxc;
    nxc = (d.nx + xchunk - 1) / xchunk;
    const dim3 grid((unsigned)tz, (unsigned)ty, (unsigned)nxc);
    const int64_t blocks = tz * ty * nxc;
    if (!partials || blocks > kMaxPartials) partials = nullptr;
    if (nparts) *nparts = partials ? (int)blocks : 0;
    if (DIV) partials = nullptr;
    if (nparts && DIV) *nparts = 0;
    prof::Scope scope(DIV ? "k_yx_r_div" : kernel_name<St>("k_yx_r", R), s);
    hipLaunchKernelGGL((k_yx_r<R, P, NW, St, DIV>), grid, dim3(64 * NW), 0, s, (const float *)T, (St *)F,
                       d.nx, d.ny, d.nz, xchunk, txy, partials, h.NX, h.NY, (int64_t)h.hx,
                       (int64_t)h.hy);
    return hipGetLastError();
}

using ZFn = hipError_t (*)(const void *, void *, Dims, const Halo &, const Taps &, hipStream_t);
using YXFn = hipError_t (*)(const void *, void *, Dims, const Halo &, const Taps &, double *,
                            int *, hipStream_t);

template <typename St, int... R>
const ZFn *ztab_of(std::integer_sequence<int, R...>)
{
    static const ZFn tab[] = {nullptr, &zpass_r<R + 1, St>...};
    return tab;
}

// 8 waves per block so a block's y tile (8 waves x P rows) is tall enough to
// amortise the 2R halo rows it re-reads: blocks sweeping x drift apart, so
// halo rows are not shared through L2 across blocks.  P shrinks as the ring
// of 2R+1 partial sums per row grows.
// Rows per lane, measured on the 512x512x1024 cube.  R = 12: two rows (115
// VGPRs, two 8-wave blocks per CU) 0.70 ms, three rows (one block per CU)
// 0.89 ms, one row (3.5x halo rows per output row) 0.87 ms.  R = 6: two rows
// 0.49 ms, three 0.52 ms, four 0.51 ms.  R = 3: four rows 0.44 ms, two
// 0.45 ms, three 0.49 ms.
template <int R>
constexpr int yx_rows() { return R <= 3 ? 4 : R <= 12 ? 2 : 1; }

template <typename St, int... R>
const YXFn *yxtab_of(std::integer_sequence<int, R...>)
{
    static const YXFn tab[] = {nullptr, &yx_r<R + 1, yx_rows<R + 1>(), 8, St>...};
    return tab;
}

// FP32 forms for the weighted convolution (Eq. 1): the spectral pass of the
// product d * w and the spatial sweep that ends in the quotient.
using ZMulFn = hipError_t (*)(const void *, void *, Dims, const Halo &, const Taps &, hipStream_t,
                              const void *);

template <int... R>
const ZMulFn *zmultab_of(std::integer_sequence<int, R...>)
{
    static const ZMulFn tab[] = {nullptr, &zpass_impl<R + 1, float, true>...};
    return tab;
}

template <int... R>
const YXFn *yxdivtab_of(std::integer_sequence<int, R...>)
{
    static const YXFn tab[] = {nullptr, &yx_r<R + 1, yx_rows<R + 1>(), 8, float, true>...};
    return tab;
}


}  // namespace

bool zpass_fast(int rz) { return rz >= 1 && rz <= kMaxFastRz; }
bool plane_fits(Dims d) { return d.ny * d.nz <= ((int64_t)1 << 28); }
bool yx_fast(int rxy, Dims d) { return rxy >= 1 && rxy <= kMaxFastRxy && plane_fits(d); }

hipError_t launch_zpass_fast(const void *in, void *T1, Store st, Dims d, const Halo &h,
                             const Taps &tz, hipStream_t s)
{
    if (!zpass_fast(tz.r)) return hipErrorInvalidValue;
    const auto seq = std::make_integer_sequence<int, kMaxFastRz>{};
    switch (st) {
    case Store::F16: return ztab_of<_Float16>(seq)[tz.r](in, T1, d, h, tz, s);
    case Store::BF16: return ztab_of<__bf16>(seq)[tz.r](in, T1, d, h, tz, s);
    default: return ztab_of<float>(seq)[tz.r](in, T1, d, h, tz, s);
    }
}

hipError_t launch_zpass_mul_fast(const float *in, const float *w, float *T1, Dims d,
                                 const Taps &tz, hipStream_t s)
{
    if (!zpass_fast(tz.r)) return hipErrorInvalidValue;
    return zmultab_of(std::make_integer_sequence<int, kMaxFastRz>{})[tz.r](
        in, T1, d, no_halo(d), tz, s, w);
}

hipError_t launch_yx_div_fast(const float *T1, float *F, Dims d, const Taps &txy, hipStream_t s)
{
    if (!yx_fast(txy.r, d)) return hipErrorInvalidValue;
    return yxdivtab_of(std::make_integer_sequence<int, kMaxFastRxy>{})[txy.r](
        T1, F, d, no_halo(d), txy, nullptr, nullptr, s);
}

int zpass_pair(int ra, int rb)
{
    const int lo = ra < rb ? ra : rb, hi = ra < rb ? rb : ra;
    for (int i = 0; i < kZPairs; ++i)
        if (kZPair[i][0] == lo && kZPair[i][1] == hi) return i;
    return -1;
}

hipError_t launch_zpass_pair(const void *in, void *Ta, void *Tb, Store st, Dims d, const Halo &h,
                             const Taps &ta, const Taps &tb, hipStream_t s)
{
    const int i = zpass_pair(ta.r, tb.r);
    if (i < 0) return hipErrorInvalidValue;
    // the kernel takes the smaller radius first
    const bool sw = ta.r > tb.r;
    void *o1 = sw ? Tb : Ta, *o2 = sw ? Ta : Tb;
    const Taps &t1 = sw ? tb : ta, &t2 = sw ? ta : tb;
    switch (st) {
    case Store::F16: return z2tab<_Float16>()[i](in, o1, o2, d, h, t1, t2, s);
    case Store::BF16: return z2tab<__bf16>()[i](in, o1, o2, d, h, t1, t2, s);
    default: return z2tab<float>()[i](in, o1, o2, d, h, t1, t2, s);
    }
}

int merged_form(const int *r, int nf)
{
    if (nf < 2 || nf > 3) return -1;
    for (int i = 0; i < kMergedForms; ++i) {
        const MergedRadii &m = kMergedRadii[i];
        if (m.nf != nf) continue;
        bool same = true;
        for (int f = 0; f < nf; ++f) same = same && m.r[f] == r[f];
        if (same) return i;
    }
    return -1;
}

hipError_t launch_yx_merged(int form, int shape, const void *T1, void *const *F, Store st,
                            Dims d, const Halo &h, const Taps *txy, double *partials,
                            int *nparts, hipStream_t s)
{
    if (form < 0 || form >= kMergedForms || shape < 0 || shape >= kMergedShapes)
        return hipErrorInvalidValue;
    const MergedRadii &m = kMergedRadii[form];
    for (int f = 0; f < m.nf; ++f)
        if (txy[f].r != m.r[f] || !F[f]) return hipErrorInvalidValue;
    if (!yx_fast(m.r[m.nf - 1], d) || !yx_fast(m.r[m.nf - 1], Dims{h.NX, h.NY, d.nz}))
        return hipErrorInvalidValue;
    MergedFn fn = nullptr;
    switch (st) {
    case Store::F16: fn = merged_fn_f16(form, shape); break;
    case Store::BF16: fn = merged_fn_bf16(form, shape); break;
    default: fn = merged_fn_f32(form, shape); break;
    }
    return fn(T1, F, d, h, txy, partials, nparts, s);
}

hipError_t launch_yx_fast(const void *T1, void *F, Store st, Dims d, const Halo &h,
                          const Taps &txy, double *partials, int *nparts, hipStream_t s)
{
    if (!yx_fast(txy.r, d) || !yx_fast(txy.r, Dims{h.NX, h.NY, d.nz})) return hipErrorInvalidValue;
    const auto seq = std::make_integer_sequence<int, kMaxFastRxy>{};
    switch (st) {
    case Store::F16: return yxtab_of<_Float16>(seq)[txy.r](T1, F, d, h, txy, partials, nparts, s);
    case Store::BF16: return yxtab_of<__bf16>(seq)[txy.r](T1, F, d, h, txy, partials, nparts, s);
    default: return yxtab_of<float>(seq)[txy.r](T1, F, d, h, txy, partials, nparts, s);
    }
}

}  // namespace gsf
