// gsf_stats.hip -- local statistics and selection (§3.3) for gfx950.
//
// The window sums of a = F - s and a^2 over the box around each voxel are
// computed as directional sums in two kernels:
//   k_box_yz_seg<BY,BZ,NW> (z window BZ = 16, 32, 64) and k_box_yz<BY> (any
//     z window up to 65): for one x-plane, walk y with a running window sum
//     per column (the value leaving the window comes from a register ring of
//     the last BY rows, so F is read once), then take the z window across the
//     lanes of a 64-wide strip with DPP lane scans (k_box_yz_seg: the column
//     sums pass through an LDS tile shared by the block's NW waves).
//     Writes the yz-window sums G1 = sum a, G2 = sum a^2 for every voxel,
//     interleaved (G[v] = {G1, G2}, one 8-byte access per voxel).
//   k_box_x_select<BX>: one lane per (y, z) walks x with a running window sum
//     of G1, G2 (leaving plane from a register ring of the last BX planes),
//     then forms mean = s + S1/n and std = sqrt(max(0, S2/n - (S1/n)^2)),
//     and the selection bit F > mean + k*std, packed along z by wave ballot.
// Running sums are FP64.  The z window is either an FP32 sum of a segment
// tail and the next segment's head (power-of-two windows: no subtraction, so
// it is accurate relative to itself) or a difference of FP64 lane prefix
// sums (any window).
#include <hip/hip_runtime.h>

#include <array>
#include <utility>
#include <string>

#include "gsf_device.h"
#include "gsf_internal.h"

namespace gsf {
namespace {

constexpr int kThreads = 256;

// ---- lane shifts through DPP ----
template <int CTRL, int ROW_MASK, int BANK_MASK, bool BOUND_ZERO>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, BANK_MASK, BOUND_ZERO));
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

// z window of one row for the 64 outputs of a wave.  Lane i carries the
// column sums u = c(2i) and v = c(2i + 1) of the strip plus its window; the
// output of lane i is H(i) = P(i + bz - 1) - P(i - 1), P the inclusive prefix
// over the 128 columns.  P is FP64 (one wave scan of the lane pair sums), so
// the difference keeps FP64 accuracy relative to the strip's largest prefix
// and H is exact to well below FP32 rounding.
__device__ __forceinline__ float zwin(double u, double v, double *q, int lane, int bz)
{
    const double pair = u + v;
    const double incl = wave_incl_scan_d(pair);
    const double excl = incl - pair;
    q[2 * lane] = excl + u;
    q[2 * lane + 1] = incl;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const double h = q[lane + bz - 1] - (lane > 0 ? q[lane - 1] : 0.0);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return (float)h;
}

// Loads issued ahead of use.  The y walk is latency-bound: 16 rows ahead
// (2 waves per SIMD) beat 4 rows (3 waves) and 32 (register-starved).  The
// x walk's time does not move between 4 and 16 planes ahead, and 4 keeps it
// at 3 waves per SIMD.
constexpr int kAhead = 16;    // rows the y walk loads before use
constexpr int kAheadX = 4;    // planes the x walk loads before use
constexpr int kXChunk = 16;   // steps between the x walk's exit tests (EXITS)

// One wave per (x, 64-wide z strip); 4 independent waves per block.
// Requires bz <= 65 so the strip plus its window spans at most 128 columns.
template <int BY, typename St>
__global__ __launch_bounds__(kThreads) void k_box_yz(const St *__restrict__ F, int64_t nx,
                                                     int64_t ny, int64_t nz, int bz,
                                                     const double *__restrict__ shift,
                                                     float *__restrict__ G)
{
    constexpr int AH = BY < kAhead ? BY : kAhead;   // prefetch depth, at most the ring length
    static_assert(BY % AH == 0, "ring length must be a multiple of the prefetch depth");
    __shared__ double qs[4][2][128];
    const int lane = threadIdx.x & 63;
    // wave-uniform by construction; readfirstlane lets the compiler keep the
    // plane's buffer descriptors in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nstrips = (nz + 63) / 64;
    const int64_t job = (int64_t)blockIdx.x * 4 + wave;
    if (job >= nx * nstrips) return;                 // whole wave exits together
    const int64_t x = job / nstrips;
    const int64_t z0 = (job % nstrips) * 64;
    const int loz = -(bz / 2);
    const int loy = -(BY / 2);
    const int hiy = loy + BY - 1;
    const float s = (float)shift[0];
    constexpr int64_t SZ = sizeof(St);
    const int64_t plane = ny * nz;
    const uint32_t plane_b = (uint32_t)(plane * 8);     // G planes and rows (FP32 pairs)
    const uint32_t row_b = (uint32_t)(nz * 8);
    const uint32_t fplane_b = (uint32_t)(plane * SZ);   // F planes and rows (storage type)
    const uint32_t frow_b = (uint32_t)(nz * SZ);
    // the two adjacent columns this lane carries: t = 2*lane and 2*lane + 1
    const int64_t zc0 = z0 + loz + 2 * lane;
    const int64_t zc1 = zc0 + 1;
    const bool v0 = (2 * lane < 64 + bz - 1) && zc0 >= 0 && zc0 < nz;
    const bool v1 = (2 * lane + 1 < 64 + bz - 1) && zc1 >= 0 && zc1 < nz;
    const uint32_t o0 = v0 ? (uint32_t)(zc0 * SZ) : kOOB;
    const uint32_t o1 = v1 ? (uint32_t)(zc1 * SZ) : kOOB;
    const __amdgpu_buffer_rsrc_t rf = buf(F + x * plane, fplane_b);
    const int64_t zo = z0 + lane;
    const uint32_t og = zo < nz ? (uint32_t)(zo * 8) : kOOB;
    const __amdgpu_buffer_rsrc_t rg = buf(G + 2 * x * plane, plane_b);
    float ring0[BY], ring1[BY];
#pragma unroll
    for (int j = 0; j < BY; ++j) ring0[j] = ring1[j] = 0.0f;
    // rows AH steps ahead; rows past the cube and dead columns load 0
    raw_t<St> pf0[AH], pf1[AH];
#pragma unroll
    for (int j = 0; j < AH; ++j) {
        pf0[j] = sbuf_ld_raw<St>(rf, o0 + (uint32_t)j * frow_b);
        pf1[j] = sbuf_ld_raw<St>(rf, o1 + (uint32_t)j * frow_b);
    }
    double a1 = 0.0, a2 = 0.0, b1 = 0.0, b2 = 0.0;   // running y sums of the two columns
    double *q1 = qs[wave][0];
    double *q2 = qs[wave][1];
    // entering rows 0 .. ny-1+hiy, rounded up to whole rings: surplus steps
    // read rows past the cube (0) and emit nothing.  No branch encloses the
    // loads or the ring, so prefetched values are never copied before use.
    const int64_t nsteps = ny + hiy;
#pragma nounroll
    for (int64_t y0 = 0; y0 < nsteps; y0 += BY) {
#pragma clang loop unroll(full)
        for (int j = 0; j < BY; ++j) {
            const int64_t yin = y0 + j;                   // yin mod BY == j
            const bool row = yin < ny;
            const float e0 = (row && v0) ? from_raw<St>(pf0[j % AH]) - s : 0.0f;
            const float e1 = (row && v1) ? from_raw<St>(pf1[j % AH]) - s : 0.0f;
            const uint32_t ra = (uint32_t)(yin + AH) * frow_b;   // past ny: outside the plane
            pf0[j % AH] = sbuf_ld_raw<St>(rf, o0 + ra);
            pf1[j % AH] = sbuf_ld_raw<St>(rf, o1 + ra);
            const float l0 = ring0[j], l1 = ring1[j];
            ring0[j] = e0;
            ring1[j] = e1;
            a1 += (double)e0 - (double)l0;
            a2 += (double)(e0 * e0) - (double)(l0 * l0);
            b1 += (double)e1 - (double)l1;
            b2 += (double)(e1 * e1) - (double)(l1 * l1);
            const int64_t y = yin - hiy;
            if (y >= 0 && y < ny) {
                const float h1 = zwin(a1, b1, q1, lane, bz);
                const float h2 = zwin(a2, b2, q2, lane, bz);
                buf_st2(rg, h1, h2, og + (uint32_t)y * row_b);
            }
            // look-ahead comes from the explicit prefetch, not from hoisting
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Inclusive prefix sums inside each group of BZ consecutive lanes (BZ = 16,
// 32 or 64) of four independent values, level by level so that no DPP read
// waits on the add just before it.  Row shifts stop at 16-lane rows; the row
// broadcasts join rows (lane 15 into rows 1 and 3, then lane 31 into rows 2
// and 3).  A broadcast add leaves the rows outside its row mask unchanged,
// which the compiler's DPP builtins can only express with an extra zeroed
// register and a separate add, so those two levels are written as one DPP
// add each; the leading s_nop provides the wait states a DPP read needs
// after the VALU write of its source.
template <int CTRL>
__device__ __forceinline__ void shr_level(float (&v)[4])
{
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] += dpp_f<CTRL, 0xf, 0xf, true>(v[i]);
}

__device__ __forceinline__ void bcast15_level(float (&v)[4])
{
    asm volatile(
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "v_add_f32_dpp %2, %2, %2 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "v_add_f32_dpp %3, %3, %3 row_bcast:15 row_mask:0xa bank_mask:0xf"
        : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]));
}

__device__ __forceinline__ void bcast31_level(float (&v)[4])
{
    asm volatile(
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
        "v_add_f32_dpp %2, %2, %2 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
        "v_add_f32_dpp %3, %3, %3 row_bcast:31 row_mask:0xc bank_mask:0xf"
        : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]));
}

template <int BZ>
__device__ __forceinline__ void seg_scan4(float (&v)[4])
{
    shr_level<0x111>(v);   // row_shr:1
    shr_level<0x112>(v);   // row_shr:2
    shr_level<0x114>(v);   // row_shr:4
    shr_level<0x118>(v);   // row_shr:8
    if constexpr (BZ >= 32) bcast15_level(v);
    if constexpr (BZ >= 64) bcast31_level(v);
}

// Workgroups go to the 8 XCDs round robin (workgroup i to XCD i mod 8).
// Renumbered, each XCD runs a contiguous range of logical blocks, so
// neighbouring blocks share that XCD's L2.
__device__ __forceinline__ int64_t xcd_block(int64_t i, int64_t n)
{
    const int64_t q = n / 8, r = n % 8, xcd = i % 8, k = i / 8;
    return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + k;
}

// Rows per LDS exchange of the segmented kernel.
constexpr int kYzRows = 8;

// The same job as k_box_yz for a power-of-two z window BZ, with the z window
// built from sums that never subtract.  Columns are cut into segments of BZ,
// and the window of output z is the tail of one segment plus the head of the
// next.
//
// A block owns one x-plane and NO = 64 (NW - 1) consecutive output columns.
// Its NW waves walk y over the NO + 64 columns starting 32 before the first
// output, one column per lane: FP64 running sums of the FP32 increments
// (F - s) and (F - s)^2, the leaving row's value from a register ring of the
// last BY rows.  Every kYzRows rows each lane writes its column's sums,
// rounded once to FP32, to a double-buffered LDS tile and the block meets
// at a barrier.  Then each of the first NW - 1 waves finishes the rows for
// its 64-column strip: lane i (segment j = i / BZ, position q = i % BZ)
// takes column A = start of segment j + BZ-1-q and column B = start of
// segment j+1 + q from the tile; an inclusive scan of the A values inside
// each BZ-lane group gives at lane i the tail of segment j from BZ-1-q, a
// scan of the B values gives heads of segment j+1, and lane i finishes output
// column j*BZ + BZ-1-q by adding the head of length BZ-1-q fetched from lane
// j*BZ + BZ-2-q (for BZ = 32 and 64 the pair form below does the same with
// two adjacent columns per lane).  A scan only adds same-window partial
// sums, so each window sum is accurate relative to itself.  Every column is
// walked once, plus one strip of halo per block.  The sums are written as
// interleaved {G1, G2} pairs.
//
// Measured on the 512x512x1024 cube (64^3 box): 9 waves (one block per CU)
// 0.63 ms; 5 waves (a quarter of the walk is halo) 0.70 ms; 16 rows per
// exchange (the tile halves occupancy) 0.92 ms; 8 or 4 rows loaded ahead
// instead of 16, 0.68 and 0.87 ms.  The earlier form, in which each lane
// walked both its A and its B column (two rings, no LDS), took 0.65 ms.
template <int BY, int BZ, int NW, typename St>
__global__ __launch_bounds__(64 * NW) void k_box_yz_seg(const St *__restrict__ F, int64_t nx,
                                                        int64_t ny64, int64_t nz64,
                                                        const double *__restrict__ shift,
                                                        float *__restrict__ G)
{
#pragma clang fp contract(off)
    constexpr int AH = BY < kAhead ? BY : kAhead;   // prefetch depth, at most the ring length
    constexpr int YB = kYzRows < BY ? kYzRows : BY;
    constexpr int NC = 64 * NW;                     // columns the block walks
    constexpr int NO = NC - 64;                     // output columns of the block
    static_assert(BY % AH == 0 && BY % YB == 0, "ring length");
    static_assert(BZ == 16 || BZ == 32 || BZ == 64, "segment length");
    __shared__ __attribute__((aligned(16))) float2 hs[2][YB][NC];
    // a plane holds at most 2^28 voxels, so in-plane indices fit 32 bits
    const int ny = (int)ny64, nz = (int)nz64;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int zblocks = (nz + NO - 1) / NO;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t x = blk / zblocks;
    const int Z0 = (int)(blk % zblocks) * NO;
    const int hiy = BY / 2 - 1;
    const float s = (float)shift[0];
    constexpr uint32_t SZ = sizeof(St);
    const int64_t plane = (int64_t)ny * nz;
    const uint32_t plane_b = (uint32_t)(plane * 8);     // G planes and rows (FP32 pairs)
    const uint32_t row_b = (uint32_t)nz * 8u;
    const uint32_t frow_b = (uint32_t)nz * SZ;          // F rows (storage type)
    // the column this lane walks: tile column threadIdx.x
    const int zc = Z0 - 32 + (int)threadIdx.x;
    const uint32_t oc = zc >= 0 && zc < nz ? (uint32_t)zc * SZ : kOOB;
    const __amdgpu_buffer_rsrc_t rf = buf(F + x * plane, (uint32_t)(plane * SZ));
    // output strip of wave w < NW - 1: columns Z0 + 64 w + 0..63; tile
    // columns of its A and B values
    const bool out_wave = wave < NW - 1;
    const int seg = lane / BZ, q = lane % BZ;
    const int ia = 64 * wave + 32 - BZ / 2 + seg * BZ + (BZ - 1 - q);
    const int ib = ia + 2 * q + 1;
    const int zo = Z0 + 64 * wave + seg * BZ + (BZ - 1 - q);
    const uint32_t og = out_wave && zo < nz ? (uint32_t)zo * 8u : kOOB;
    const bool has_head = q < BZ - 1;
    const int src = has_head ? seg * BZ + (BZ - 2 - q) : lane;
    // Pair form (BZ = 32, 64): waves 2k and 2k+1 share the 128-column strip
    // pair k (even and odd rows); lane i holds two adjacent columns of a
    // segment's A side and of the next segment's B side, so a segment is
    // HG = BZ/2 lanes and one scan finishes two outputs (zp, zp + 1): the
    // scans lose a level and serve twice the outputs (10 instead of 24 DPP
    // adds per output; measured 0.622 -> 0.610 ms).  The lane before's
    // inclusive sums give the exclusive ones (no subtraction), so every
    // window sum still only adds partial sums of its own window.
    constexpr bool PAIR = BZ >= 32 && (NW - 1) % 2 == 0;
    constexpr int HG = BZ / 2;
    const int pg = lane / HG, pq = lane % HG;
    const int pk = wave >> 1, par = wave & 1;
    const int a_lo = 128 * pk + 32 - BZ / 2 + pg * BZ + BZ - 2 - 2 * pq;   // positions BZ-2-2q, BZ-1-2q
    const int b_lo = 128 * pk + 32 - BZ / 2 + (pg + 1) * BZ + 2 * pq;     // positions 2q, 2q+1
    const int zp = Z0 + 128 * pk + pg * BZ + BZ - 2 - 2 * pq;
    const int srcP = pq > 0 ? lane - 1 : lane;            // the lane before, in the segment
    const int srcE = pg * HG + (HG - 1 - pq);             // head through BZ-2-2q (even)
    const bool hasO = pq <= HG - 2;
    const int srcO = hasO ? pg * HG + (HG - 2 - pq) : lane;   // head through BZ-3-2q (odd)
    const __amdgpu_buffer_rsrc_t rg = buf(G + 2 * x * plane, plane_b);
    float ring[BY];
#pragma unroll
    for (int j = 0; j < BY; ++j) ring[j] = 0.0f;
    raw_t<St> pf[AH];
#pragma unroll
    for (int j = 0; j < AH; ++j) pf[j] = sbuf_ld_raw<St>(rf, oc + (uint32_t)j * frow_b);
    double c1 = 0.0, c2 = 0.0;                      // running y sums of the column
    const int nsteps = ny + hiy;
    int bsel = 0;                                   // tile buffer of the current rows
    // A ring turn is unrolled as NQ chunks of YQ steps (whole exchange
    // groups); the walk leaves after the first chunk that reaches nsteps, so
    // at most YQ - 1 surplus steps run.  The exits leave the loop (uniform
    // over the block), so the steps carry no branch around their loads.
    constexpr int YQ = BY / 4 > YB ? BY / 4 : YB;
    constexpr int NQ = BY / YQ;
    static_assert(NQ == 1 || NQ == 2 || NQ == 4, "chunks per turn");
#pragma nounroll
    for (int y0 = 0;; y0 += BY) {
        auto chunk = [&](auto cc) __attribute__((always_inline)) {
            constexpr int c = decltype(cc)::value;
#pragma clang loop unroll(full)
            for (int jj = 0; jj < YQ; ++jj) {
                const int j = c * YQ + jj;
                    const int yin = y0 + j;                       // yin mod BY == j
                    // rows past ny and columns outside [0, nz) count as 0 (their
                    // loads read 0 through the range check)
                    const float e = from_raw<St>(pf[j % AH]) - s;
                    const float ev = yin < ny && oc != kOOB ? e : 0.0f;
                    pf[j % AH] = sbuf_ld_raw<St>(rf, oc + (uint32_t)(yin + AH) * frow_b);
                    const float l = ring[j];
                    ring[j] = ev;
                    c1 += (double)(ev - l);
                    c2 += (double)(ev * ev - l * l);
                    hs[bsel][j % YB][threadIdx.x] = make_float2((float)c1, (float)c2);
                    if (j % YB == YB - 1) {
                        // rows yin-YB+1 .. yin are in the tile; the other buffer was
                        // last read before this barrier's predecessor
                        __syncthreads();
                        if constexpr (PAIR) {
                            if (out_wave) {
        #pragma unroll
                                for (int i = 0; i < YB / 2; ++i) {
                                    const int r = 2 * i + par;
                                    const int y = yin - (YB - 1) + r - hiy;
                                    if (y >= 0 && y < ny) {
                                        const float4 *row4 =
                                            reinterpret_cast<const float4 *>(&hs[bsel][r][0]);
                                        // av: {G1, G2} at positions BZ-2-2q (x, y) and BZ-1-2q
                                        // (z, w); bv: at 2q (x, y) and 2q+1 (z, w)
                                        const float4 av = row4[a_lo / 2], bv = row4[b_lo / 2];
                                        float t[4] = {av.x + av.z, av.y + av.w, bv.x + bv.z,
                                                      bv.y + bv.w};
                                        seg_scan4<HG>(t);   // tails from BZ-2-2q, heads to 2q+1
                                        float e[4];
        #pragma unroll
                                        for (int m = 0; m < 4; ++m) {
                                            const float v = __int_as_float(__builtin_amdgcn_ds_bpermute(
                                                srcP * 4, __float_as_int(t[m])));
                                            e[m] = pq > 0 ? v : 0.0f;
                                        }
                                        const float hE1 = e[2] + bv.x, hE2 = e[3] + bv.y;   // heads to 2q
                                        const float gE1 = __int_as_float(
                                            __builtin_amdgcn_ds_bpermute(srcE * 4, __float_as_int(hE1)));
                                        const float gE2 = __int_as_float(
                                            __builtin_amdgcn_ds_bpermute(srcE * 4, __float_as_int(hE2)));
                                        const float gO1 = __int_as_float(
                                            __builtin_amdgcn_ds_bpermute(srcO * 4, __float_as_int(t[2])));
                                        const float gO2 = __int_as_float(
                                            __builtin_amdgcn_ds_bpermute(srcO * 4, __float_as_int(t[3])));
                                        // window at zp: tail from BZ-2-2q + head to BZ-3-2q;
                                        // at zp + 1: tail from BZ-1-2q + head to BZ-2-2q
                                        const float o1 = hasO ? t[0] + gO1 : t[0];
                                        const float o2 = hasO ? t[1] + gO2 : t[1];
                                        const float p1 = (e[0] + av.z) + gE1;
                                        const float p2 = (e[1] + av.w) + gE2;
                                        const uint32_t oy = (uint32_t)zp * 8u + (uint32_t)y * row_b;
                                        if (zp + 1 < nz)
                                            buf_st4(rg, o1, o2, p1, p2, oy);
                                        else if (zp < nz)
                                            buf_st2(rg, o1, o2, oy);
                                    }
                                }
                            }
                        } else if (out_wave) {
        #pragma unroll
                            for (int r = 0; r < YB; ++r) {
                                const int y = yin - (YB - 1) + r - hiy;
                                if (y >= 0 && y < ny) {
                                    const float2 a = hs[bsel][r][ia], b = hs[bsel][r][ib];
                                    float t[4] = {a.x, a.y, b.x, b.y};
                                    seg_scan4<BZ>(t);
                                    const float h1 = __int_as_float(
                                        __builtin_amdgcn_ds_bpermute(src * 4, __float_as_int(t[2])));
                                    const float h2 = __int_as_float(
                                        __builtin_amdgcn_ds_bpermute(src * 4, __float_as_int(t[3])));
                                    buf_st2(rg, has_head ? t[0] + h1 : t[0], has_head ? t[1] + h2 : t[1],
                                            og + (uint32_t)y * row_b);
                                }
                            }
                        }
                        bsel ^= 1;
                    }
                __builtin_amdgcn_sched_barrier(0);
            }
        };
        chunk(std::integral_constant<int, 0>{});
        if (y0 + YQ >= nsteps) break;
        if constexpr (NQ > 1) {
            chunk(std::integral_constant<int, 1>{});
            if (y0 + 2 * YQ >= nsteps) break;
        }
        if constexpr (NQ > 2) {
            chunk(std::integral_constant<int, 2>{});
            if (y0 + 3 * YQ >= nsteps) break;
            chunk(std::integral_constant<int, 3>{});
            if (y0 + 4 * YQ >= nsteps) break;
        }
    }
}

__device__ __forceinline__ int win_len32(int i, int n, int B)
{
    int lo = i - (B / 2);
    int hi = lo + B;
    if (lo < 0) lo = 0;
    if (hi > n) hi = n;
    return hi - lo;
}

// A copy of a uniform value the compiler cannot see through: offsets built
// from it each ring turn are recomputed per step instead of being hoisted
// out of the loop into dozens of live registers.
__device__ __forceinline__ uint32_t opaque(uint32_t v)
{
    uint32_t r;
    asm volatile("s_mov_b32 %0, %1" : "=s"(r) : "s"(v));
    return r;
}

// Buffer descriptor over planes [p, p + span) of a cube with nx planes,
// clipped to the cube (empty when p >= nx).  Loads and stores address a
// plane inside it with (plane - p) * plane bytes added to the lane's 32-bit
// offset (the range-checked one); a plane past the clip lies outside the
// range and reads 0 / drops the store.
template <typename E>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_span(const E *c, int p, int span, int nx,
                                                             uint32_t plane)
{
    const int n = p < nx ? (nx - p < span ? nx - p : span) : 0;
    const int pc = p < nx ? p : nx;
    return buf(c + (int64_t)pc * plane, (uint32_t)n * plane * (uint32_t)sizeof(E));
}

// One lane per (y, z), 256 consecutive z per block; walks x.  Per step the
// lane loads the entering plane's {G1, G2} pair and the output plane's F (issued
// kAheadX steps early), updates the FP64 window sums with the ring of the
// last BX planes, and finishes the output plane.  Plane addressing is
// 32-bit: every BX steps the kernel sets up descriptors over the next BX
// planes of each stream and steps through them with scalar offsets, which
// needs BX + 1 planes to span less than 2^31 bytes.
//
// The walk runs whole ring turns: after the last entering plane the rest of
// the last turn reads empty ranges and emits nothing.  With EXITS the last
// turn stops at the first 16-step boundary past the end instead (a uniform
// exit between unrolled chunks), which saves up to 48 steps on small cubes
// and costs registers (fewer waves per SIMD); the tuning table chooses.
template <int BX, typename St, bool STATS, bool EXITS = false>
__global__ __launch_bounds__(kThreads) void k_box_x_select(
    const float2 *__restrict__ G, const St *__restrict__ F,
    int64_t nx64, int64_t ny64, int64_t nz64, int by, int bz, const double *__restrict__ shift,
    float *__restrict__ mean, float *__restrict__ stdev, uint64_t *__restrict__ mask, double k)
{
#pragma clang fp contract(off)
    constexpr int AX = BX < kAheadX ? BX : kAheadX;   // prefetch depth, at most the ring length
    static_assert(BX % AX == 0 && BX <= 64, "ring length");
    constexpr int XQ = BX < kXChunk ? BX : kXChunk;   // steps per unrolled chunk
    constexpr int NQ = BX / XQ;
    static_assert(NQ == 1 || NQ == 2 || NQ == 4, "chunks per turn");
    const int nx = (int)nx64, ny = (int)ny64, nz = (int)nz64;
    const int y = blockIdx.y;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int z = blockIdx.x * kThreads + threadIdx.x;
    const bool live = z < nz;
    constexpr uint32_t SZ = sizeof(St);
    const uint32_t plane = (uint32_t)ny * (uint32_t)nz;
    const uint32_t plane_b = plane * 4u;                 // mean, std (FP32)
    const uint32_t gplane_b = plane * 8u;                // G (FP32 pairs)
    const uint32_t fplane_b = plane * SZ;                // F (storage type)
    // offset of (y, z) inside a plane; dead lanes address outside every range
    const uint32_t off = live ? ((uint32_t)y * (uint32_t)nz + (uint32_t)z) * 4u : kOOB;
    const uint32_t offg = live ? ((uint32_t)y * (uint32_t)nz + (uint32_t)z) * 8u : kOOB;
    const uint32_t offf = live ? ((uint32_t)y * (uint32_t)nz + (uint32_t)z) * SZ : kOOB;
    const int W = (nz + 63) / 64;
    const int hix = -(BX / 2) + BX - 1;
    const double s = (double)(float)shift[0];   // the same FP32 shift the sums used
    const double inv_yz =
        live ? 1.0 / (double)(win_len(y, ny, by) * win_len(z, nz, bz)) : 1.0;
    // this wave's mask word of plane 0 (wave-uniform, bytes); plane x adds
    // x * mplane_b.  The mask array is below 2^31 bytes (checked on the host).
    const uint32_t mplane_b = (uint32_t)ny * (uint32_t)W * 8u;
    const uint32_t mword_b =
        ((uint32_t)y * (uint32_t)W + blockIdx.x * (kThreads / 64) + (uint32_t)wave) * 8u;
    const __amdgpu_buffer_rsrc_t rmask =
        buf(mask, mask ? (uint32_t)nx * mplane_b : 0u);
    float r1[BX], r2[BX];
#pragma unroll
    for (int j = 0; j < BX; ++j) r1[j] = r2[j] = 0.0f;
    // loads issued AX steps early: plane pa of G (entering) and plane
    // pa - hix of F (output)
    float2 pg[AX];
    raw_t<St> pfv[AX];
    {
        const __amdgpu_buffer_rsrc_t qg = plane_span(G, 0, AX, nx, plane);
        const __amdgpu_buffer_rsrc_t qf = plane_span(F, 0, AX, nx, plane);
#pragma unroll
        for (int j = 0; j < AX; ++j) {
            const int xf = j - hix;
            pg[j] = buf_ld2(qg, offg + (uint32_t)j * gplane_b);
            pfv[j] = sbuf_ld_raw<St>(qf, offf + (uint32_t)(xf >= 0 ? xf : BX) * fplane_b);
        }
    }
    double s1 = 0.0, s2 = 0.0;
    // entering planes 0 .. nx-1+hix, rounded up to whole rings: surplus steps
    // load empty ranges and emit nothing; only the output part is branched.
    // (Branching around the surplus steps costs more than it saves: the
    // kernel rises from 166 to 178 registers, below three waves per SIMD.)
    const int nsteps = nx + hix;
#pragma nounroll
    for (int p0 = 0; p0 < nsteps; p0 += BX) {
        // planes loaded in this ring turn: G planes ga + j, F planes fa + j;
        // output planes xo + j (j < BX).  A plane offset of BX planes is
        // outside every span.
        const int ga = p0 + AX;
        const int fa = ga - hix;
        const int fb = fa > 0 ? fa : 0;
        const int xo = p0 - hix;
        const int xb = xo > 0 ? xo : 0;
        const uint32_t pb = opaque(plane_b);
        const uint32_t pbg = opaque(gplane_b);
        const uint32_t pbf = opaque(fplane_b);
        const __amdgpu_buffer_rsrc_t rg = plane_span(G, ga, BX, nx, plane);
        const __amdgpu_buffer_rsrc_t rfv = plane_span(F, fb, BX, nx, plane);
        // the turn as NQ unrolled chunks of XQ steps; with EXITS the walk
        // leaves after the chunk that passes the last entering plane (a
        // uniform test between chunks, so every ring index stays static)
        auto chunk = [&](auto cc) __attribute__((always_inline)) {
            constexpr int c = decltype(cc)::value;
#pragma clang loop unroll(full)
            for (int jj = 0; jj < XQ; ++jj) {
                const int j = c * XQ + jj;
                const float g1 = pg[j % AX].x, g2 = pg[j % AX].y;
                const raw_t<St> fraw = pfv[j % AX];
                const int xf = fa + j;
                pg[j % AX] = buf_ld2(rg, offg + (uint32_t)j * pbg);
                pfv[j % AX] = sbuf_ld_raw<St>(rfv, offf + (uint32_t)(xf >= 0 ? xf - fb : BX) * pbf);
                s1 += (double)g1 - (double)r1[j];
                s2 += (double)g2 - (double)r2[j];
                r1[j] = g1;
                r2[j] = g2;
                const int x = xo + j;
                if (x >= 0 && x < nx) {
                    // n = cx * cy * cz, cx the clipped window length along x; away
                    // from the x faces cx = BX and 1/BX is exact
                    const int cx = win_len32(x, nx, BX);
                    double icx = 1.0 / BX;
                    if (cx != BX) icx = 1.0 / (double)cx;   // IEEE division: correctly rounded
                    const double inv_n = inv_yz * icx;
                    const double m1 = s1 * inv_n;
                    double var = s2 * inv_n - m1 * m1;
                    var = var < 0.0 ? 0.0 : var;
                    const float mf = (float)(s + m1);
                    const float sf = __builtin_amdgcn_sqrtf((float)var);   // std is stored in FP32
                    const uint32_t so = off + (uint32_t)(x - xb) * pb;
                    if (STATS) {   // compiled out when only masks are wanted
                        if (mean) buf_st(plane_span(mean, xb, BX, nx, plane), mf, so);
                        if (stdev) buf_st(plane_span(stdev, xb, BX, nx, plane), sf, so);
                    }
                    if (mask) {
                        const float fv = from_raw<St>(fraw);
                        const bool bit = live && (double)fv > (double)mf + k * (double)sf;
                        const uint64_t word = __ballot(bit);
                        if ((threadIdx.x & 63) == 0 && live)
                            buf_st2(rmask, __uint_as_float((uint32_t)word),
                                    __uint_as_float((uint32_t)(word >> 32)),
                                    mword_b + (uint32_t)x * mplane_b);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        };
        chunk(std::integral_constant<int, 0>{});
        if constexpr (EXITS) {
            if (p0 + XQ >= nsteps) break;
        }
        if constexpr (NQ > 1) {
            chunk(std::integral_constant<int, 1>{});
            if constexpr (EXITS) {
                if (p0 + 2 * XQ >= nsteps) break;
            }
        }
        if constexpr (NQ > 2) {
            chunk(std::integral_constant<int, 2>{});
            if constexpr (EXITS) {
                if (p0 + 3 * XQ >= nsteps) break;
            }
            chunk(std::integral_constant<int, 3>{});
        }
    }
}

// Timing names by window lengths and storage type, built once.
template <typename St>
const char *yz_name(int by, int bz)
{
    static const std::array<std::array<std::string, 4>, 4> tab = [] {
        std::array<std::array<std::string, 4>, 4> t;
        const int bys[4] = {8, 16, 32, 64}, bzs[4] = {0, 16, 32, 64};
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c)
                t[r][c] = c == 0 ? "k_box_yz<" + std::to_string(bys[r]) + store_suffix<St>() + ">"
                                 : "k_box_yz_seg<" + std::to_string(bys[r]) + "," +
                                       std::to_string(bzs[c]) + store_suffix<St>() + ">";
        return t;
    }();
    const int r = by == 8 ? 0 : by == 16 ? 1 : by == 32 ? 2 : 3;
    const int c = bz == 16 ? 1 : bz == 32 ? 2 : bz == 64 ? 3 : 0;
    return tab[r][c].c_str();
}

template <typename St>
const char *x_name(int bx)
{
    static const std::array<std::string, 4> tab = [] {
        std::array<std::string, 4> t;
        const int bxs[4] = {8, 16, 32, 64};
        for (int i = 0; i < 4; ++i)
            t[i] = "k_box_x_select<" + std::to_string(bxs[i]) + store_suffix<St>() + ">";
        return t;
    }();
    return tab[bx == 8 ? 0 : bx == 16 ? 1 : bx == 32 ? 2 : 3].c_str();
}

template <int BY, int NW, typename St>
hipError_t yz_seg(const St *F, Dims d, int bz, const double *shift, float *G,
                  hipStream_t s)
{
    constexpr int NO = 64 * (NW - 1);
    const dim3 grid((unsigned)(d.nx * ((d.nz + NO - 1) / NO)));
    const dim3 block(64 * NW);
    if (bz == 16)
        hipLaunchKernelGGL((k_box_yz_seg<BY, 16, NW, St>), grid, block, 0, s, F, d.nx, d.ny, d.nz,
                           shift, G);
    else if (bz == 32)
        hipLaunchKernelGGL((k_box_yz_seg<BY, 32, NW, St>), grid, block, 0, s, F, d.nx, d.ny, d.nz,
                           shift, G);
    else
        hipLaunchKernelGGL((k_box_yz_seg<BY, 64, NW, St>), grid, block, 0, s, F, d.nx, d.ny, d.nz,
                           shift, G);
    return hipGetLastError();
}

template <int BY, typename St>
hipError_t box_yz(const void *F_, Dims d, int bz, const double *shift, float *G,
                  hipStream_t s)
{
    const St *F = (const St *)F_;
    prof::Scope scope(yz_name<St>(BY, bz), s);
    if (bz == 16 || bz == 32 || bz == 64) {
        // 3, 5 or 9 waves per block (2, 4 or 8 output strips), whichever
        // walks the fewest columns for this depth (ties to the larger block)
        int best = 9;
        int64_t cost = 0;
        for (int nw : {9, 5, 3}) {
            const int64_t c = (d.nz + 64 * (nw - 1) - 1) / (64 * (nw - 1)) * nw;
            if (nw == 9 || c < cost) best = nw, cost = c;
        }
        const int tuned = active_tune().yz_waves;
        if (tuned == 3 || tuned == 5 || tuned == 9) best = tuned;
        if (best == 3) return yz_seg<BY, 3, St>(F, d, bz, shift, G, s);
        if (best == 5) return yz_seg<BY, 5, St>(F, d, bz, shift, G, s);
        return yz_seg<BY, 9, St>(F, d, bz, shift, G, s);
    }
    const int64_t jobs = d.nx * ((d.nz + 63) / 64);
    hipLaunchKernelGGL((k_box_yz<BY, St>), dim3((unsigned)((jobs + 3) / 4)), dim3(kThreads), 0, s,
                       F, d.nx, d.ny, d.nz, bz, shift, G);
    return hipGetLastError();
}

template <int BX, typename St>
hipError_t box_x_select(const float *G, const void *F, Dims d, Box b,
                        const double *shift, float *mean, float *stdev, uint64_t *mask, double k,
                        hipStream_t s)
{
    const dim3 grid((unsigned)((d.nz + kThreads - 1) / kThreads), (unsigned)d.ny);
    prof::Scope scope(x_name<St>(BX), s);
    const bool exits = active_tune().x_exits != 0;
    auto go = [&](auto stc, auto exc) {
        constexpr bool ST = decltype(stc)::value;
        constexpr bool EX = decltype(exc)::value;
        hipLaunchKernelGGL((k_box_x_select<BX, St, ST, EX>), grid, dim3(kThreads), 0, s,
                           (const float2 *)G, (const St *)F, d.nx, d.ny, d.nz, b.by, b.bz, shift,
                           mean, stdev, mask, k);
    };
    using T = std::true_type;
    using N = std::false_type;
    if (mean || stdev) {
        if (exits) go(T{}, T{}); else go(T{}, N{});
    } else {
        if (exits) go(N{}, T{}); else go(N{}, N{});
    }
    return hipGetLastError();
}

using YZFn = hipError_t (*)(const void *, Dims, int, const double *, float *, hipStream_t);
using XFn = hipError_t (*)(const float *, const void *, Dims, Box, const double *, float *,
                           float *, uint64_t *, double, hipStream_t);

template <typename St>
YZFn yz_fn(int by)
{
    switch (by) {
    case 8: return &box_yz<8, St>;
    case 16: return &box_yz<16, St>;
    case 32: return &box_yz<32, St>;
    case 64: return &box_yz<64, St>;
    default: return nullptr;
    }
}

template <typename St>
XFn x_fn(int bx)
{
    switch (bx) {
    case 8: return &box_x_select<8, St>;
    case 16: return &box_x_select<16, St>;
    case 32: return &box_x_select<32, St>;
    case 64: return &box_x_select<64, St>;
    default: return nullptr;
    }
}

}  // namespace

bool stats_fast_path(Box b, Dims d)
{
    // the x walk addresses BX + 1 planes of 8-byte pairs with 32-bit offsets;
    // a plane of pairs stays below 2^30 bytes so that a dead lane's offset
    // (2^31) plus a row or plane offset never wraps into range
    const int64_t plane = d.ny * d.nz;
    const bool x_fits = (int64_t)(b.bx + 1) * plane * 8 < ((int64_t)1 << 31);
    // the mask words are stored with 32-bit byte offsets
    const bool mask_fits = d.nx * d.ny * ((d.nz + 63) / 64) * 8 < ((int64_t)1 << 31);
    return yz_fn<float>(b.by) && x_fn<float>(b.bx) && b.bz >= 1 && b.bz <= 65 &&
           plane <= ((int64_t)1 << 27) && x_fits && mask_fits;
}

hipError_t launch_stats_fast(const void *F, Store st, Dims d, Box b, const double *shift,
                             float *G, float *mean, float *stdev, uint64_t *mask,
                             double k, hipStream_t s)
{
    if (!stats_fast_path(b, d)) return hipErrorInvalidValue;
    return with_store(st, [&](auto *tag) {
        using St = GSF_STORE_T(tag);
        hipError_t e = yz_fn<St>(b.by)(F, d, b.bz, shift, G, s);
        if (e != hipSuccess) return e;
        return x_fn<St>(b.bx)(G, F, d, b, shift, mean, stdev, mask, k, s);
    });
}

}  // namespace gsf
