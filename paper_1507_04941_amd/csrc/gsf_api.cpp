// gsf_api.cpp -- the C ABI declared in include/gsf.h: argument validation,
// host-side filter taps, workspace sizing and the launch schedule.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gsf_internal.h"
#include "gsf_merged.h"

namespace {

thread_local std::string g_err;

gsf_status fail(gsf_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

gsf_status ok()
{
    g_err.clear();
    return GSF_OK;
}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

bool overlaps(const void *a, size_t na, const void *b, size_t nb)
{
    if (!a || !b || na == 0 || nb == 0) return false;
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

// Limits keep every grid dimension and index product in range: a dispatch's
// grid size is a 32-bit count of work-items per dimension, and the widest
// grids launch nx*ny blocks of 256 work-items.
constexpr int64_t kMaxRows = (int64_t)1 << 24;      // nx*ny, exclusive
constexpr int64_t kMaxNz = (int64_t)1 << 23;        // ceil(nz/256) blocks along grid y
constexpr int64_t kMaxVoxels = (int64_t)1 << 40;

gsf_status check_dims(gsf_dims d)
{
    if (d.nx < 1 || d.ny < 1 || d.nz < 1)
        return fail(GSF_ERR_INVALID_ARG, "dims must be >= 1 (got %lld x %lld x %lld)",
                    (long long)d.nx, (long long)d.ny, (long long)d.nz);
    if (d.nx >= kMaxRows || d.ny >= kMaxRows || d.nx * d.ny >= kMaxRows || d.nz > kMaxNz ||
        d.nx * d.ny > kMaxVoxels / d.nz)
        return fail(GSF_ERR_INVALID_ARG, "dims too large (%lld x %lld x %lld)", (long long)d.nx,
                    (long long)d.ny, (long long)d.nz);
    return GSF_OK;
}

// Radius r = ceil(truncate * sigma), FP64, as the filter definition states.
gsf_status check_filter(const gsf_filter *f)
{
    if (!f) return fail(GSF_ERR_INVALID_ARG, "filter pointer is NULL");
    if (!(std::isfinite(f->sigma_xy) && f->sigma_xy > 0.0) ||
        !(std::isfinite(f->sigma_z) && f->sigma_z > 0.0))
        return fail(GSF_ERR_INVALID_ARG, "sigma must be finite and > 0 (got %g, %g)",
                    f->sigma_xy, f->sigma_z);
    if (!(std::isfinite(f->truncate) && f->truncate > 0.0))
        return fail(GSF_ERR_INVALID_ARG, "truncate must be finite and > 0 (got %g)", f->truncate);
    const double rxy = std::ceil(f->truncate * f->sigma_xy);
    const double rz = std::ceil(f->truncate * f->sigma_z);
    if (rxy > GSF_MAX_RADIUS || rz > GSF_MAX_RADIUS)
        return fail(GSF_ERR_INVALID_ARG, "filter radius exceeds %d (r_xy=%g, r_z=%g)",
                    GSF_MAX_RADIUS, rxy, rz);
    return GSF_OK;
}

gsf_status check_box(gsf_box b)
{
    if (b.bx < 1 || b.by < 1 || b.bz < 1 || b.bx > GSF_MAX_BOX || b.by > GSF_MAX_BOX ||
        b.bz > GSF_MAX_BOX)
        return fail(GSF_ERR_INVALID_ARG, "box lengths must be in [1, %d] (got %d, %d, %d)",
                    GSF_MAX_BOX, b.bx, b.by, b.bz);
    return GSF_OK;
}

gsf_status check_dtype(gsf_dtype t, const char *what)
{
    if (t == GSF_F32 || t == GSF_F16 || t == GSF_BF16) return GSF_OK;
    return fail(GSF_ERR_INVALID_ARG, "%s: unknown dtype %d", what, (int)t);
}

gsf::Store to_store(gsf_dtype t) { return (gsf::Store)(int)t; }
size_t elem_bytes(gsf_dtype t) { return gsf::store_bytes(to_store(t)); }

gsf_status check_ptr(const void *p, size_t align, const char *what)
{
    if (!p) return fail(GSF_ERR_INVALID_ARG, "%s is NULL", what);
    if (!aligned(p, align))
        return fail(GSF_ERR_INVALID_ARG, "%s is not %zu-byte aligned", what, align);
    return GSF_OK;
}

// Sampled unit-sum Gaussian, offsets -r..r, computed in FP64 and rounded to FP32.
gsf::Taps make_taps(double sigma, double truncate)
{
    gsf::Taps t{};
    const int r = (int)std::ceil(truncate * sigma);
    double w[gsf::kMaxTaps];
    double sum = 0.0;
    for (int o = -r; o <= r; ++o) {
        w[o + r] = std::exp(-(double)(o * o) / (2.0 * sigma * sigma));
        sum += w[o + r];
    }
    for (int i = 0; i <= 2 * r; ++i) t.g[i] = (float)(w[i] / sum);
    t.r = r;
    return t;
}

gsf::Dims to_dims(gsf_dims d) { return gsf::Dims{d.nx, d.ny, d.nz}; }
gsf::Box to_box(gsf_box b) { return gsf::Box{b.bx, b.by, b.bz}; }

size_t cube_bytes(gsf_dims d) { return align_up((size_t)(d.nx * d.ny * d.nz) * sizeof(float)); }

// Scratch cubes the statistics need: the interleaved window-sum pairs (two
// cubes of floats) where the fast kernels apply, four cubes on the generic
// path.
int stats_cubes(gsf_box b, gsf_dims d)
{
    return gsf::stats_fast_path(to_box(b), to_dims(d)) ? 2 : 4;
}

// The per-block partial sums of n shifts and the n shifts themselves.
size_t shift_bytes(int n)
{
    return (size_t)n * align_up(gsf::kMaxPartials * sizeof(double)) +
           align_up((size_t)n * sizeof(double));
}

// gsf_local_stats: [statistics cubes][partials][shift].
size_t stats_ws(gsf_dims d, gsf_box b)
{
    return (size_t)stats_cubes(b, d) * cube_bytes(d) + shift_bytes(1);
}

// Statistics workspace: w1..w4 (w3, w4 null with two cubes); partials of
// shift i at partials + i * kMaxPartials, shift i at shift[i].
struct StatsWs {
    float *w1, *w2, *w3, *w4;
    double *partials, *shift;
};

StatsWs carve_stats(char *p, gsf_dims d, int ncubes, int nshift)
{
    StatsWs w{};
    const size_t c = cube_bytes(d);
    float **cubes[4] = {&w.w1, &w.w2, &w.w3, &w.w4};
    for (int i = 0; i < ncubes; ++i, p += c) *cubes[i] = (float *)p;
    w.partials = (double *)p;
    p += (size_t)nshift * align_up(gsf::kMaxPartials * sizeof(double));
    w.shift = (double *)p;
    return w;
}

// gsf_filter3d needs T1, plus a second scratch cube on the generic spatial path.
size_t filter_ws(gsf_dims d, const gsf_filter *f)
{
    const int rxy = (int)std::ceil(f->truncate * f->sigma_xy);
    return cube_bytes(d) * (gsf::yx_fast(rxy, to_dims(d)) ? 1 : 2);
}

// gsf_filter3d_weighted: P = d*w, T1, D, plus the generic path's scratch cube.
size_t weighted_ws(gsf_dims d, const gsf_filter *f)
{
    const int rxy = (int)std::ceil(f->truncate * f->sigma_xy);
    return cube_bytes(d) * (gsf::yx_fast(rxy, to_dims(d)) ? 3 : 4);
}

gsf_status device_status(hipError_t e, const char *what)
{
    if (e != hipSuccess)
        return fail(GSF_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return ok();
}

// ---- tuning table: one entry per (size class, storage type) ----
constexpr int kSizeClasses = 41;   // floor(log2(voxels)) of a core, 0 .. 40

thread_local gsf::Tune t_active;
std::mutex g_tune_mu;

// Default entry of a storage type and size class: the measured best on the
// 512x512x1024 cube with the six-filter bank for cores of 2^26 voxels and
// more (the merged sweep's block: FP32 1 row x 16 waves, 1.16 against 1.21 ms
// for 2 x 8; 16-bit 2 rows x 4 waves, 1.06 against 1.09 ms for 1 x 8), 1 x 8
// below; the x walk stops its last ring turn at the first 16-step boundary
// past the cube everywhere (measured cube: 0.768 -> 0.726 ms, no class of
// the 96-cube batch slower).
gsf::Tune default_tune(int t, int cls)
{
    gsf::Tune v;
    v.x_exits = 1;
    if (cls >= 26) v.merged_shape = t == (int)GSF_F32 ? 2 : 3;
    return v;
}

struct TuneTable {
    gsf::Tune e[3][kSizeClasses];
    TuneTable() { reset(); }
    void reset()
    {
        for (int t = 0; t < 3; ++t)
            for (int c = 0; c < kSizeClasses; ++c) e[t][c] = default_tune(t, c);
    }
};
TuneTable g_table;
gsf::Tune (&g_tune)[3][kSizeClasses] = g_table.e;

int size_class(gsf_dims d)
{
    const int64_t v = d.nx * d.ny * d.nz;
    int c = 0;
    while (c + 1 < kSizeClasses && ((int64_t)1 << (c + 1)) <= v) ++c;
    return c;
}

gsf::Tune tune_for(gsf_dims core, gsf_dtype t)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_tune[(int)t][size_class(core)];
}

gsf_status check_tuning(const gsf_tuning *c)
{
    if (!c) return fail(GSF_ERR_INVALID_ARG, "tuning pointer is NULL");
    if (c->merge_sweeps != 0 && c->merge_sweeps != 1)
        return fail(GSF_ERR_INVALID_ARG, "merge_sweeps must be 0 or 1");
    if (c->merged_shape < 0 || c->merged_shape >= gsf::kMergedShapes)
        return fail(GSF_ERR_INVALID_ARG, "merged_shape must be in [0, %d)", gsf::kMergedShapes);
    if (c->sweep_blocks < 64 || c->sweep_blocks > 65536)
        return fail(GSF_ERR_INVALID_ARG, "sweep_blocks must be in [64, 65536]");
    if (c->yz_waves != 0 && c->yz_waves != 3 && c->yz_waves != 5 && c->yz_waves != 9)
        return fail(GSF_ERR_INVALID_ARG, "yz_waves must be 0, 3, 5 or 9");
    if (c->pair_spectral != 0 && c->pair_spectral != 1)
        return fail(GSF_ERR_INVALID_ARG, "pair_spectral must be 0 or 1");
    if (c->x_exits != 0 && c->x_exits != 1)
        return fail(GSF_ERR_INVALID_ARG, "x_exits must be 0 or 1");
    return GSF_OK;
}

}  // namespace

namespace gsf {
const Tune &active_tune() { return t_active; }
void set_active_tune(const Tune &t) { t_active = t; }
}  // namespace gsf

extern "C" {

const char *gsf_version(void) { return "gsf 0.1.0 (gfx950)"; }

const char *gsf_status_string(gsf_status s)
{
    switch (s) {
    case GSF_OK: return "ok";
    case GSF_ERR_INVALID_ARG: return "invalid argument";
    case GSF_ERR_UNSUPPORTED: return "unsupported";
    case GSF_ERR_WORKSPACE: return "workspace too small";
    case GSF_ERR_DEVICE: return "device error";
    case GSF_ERR_BUDGET: return "over memory budget";
    }
    return "unknown status";
}

const char *gsf_last_error(void) { return g_err.c_str(); }

int64_t gsf_mask_words(gsf_dims d)
{
    if (check_dims(d) != GSF_OK) return -1;
    return to_dims(d).words();
}

gsf_status gsf_filter3d_workspace_size(gsf_dims d, const gsf_filter *f, size_t *bytes)
{
    gsf_status st;
    if (!bytes) return fail(GSF_ERR_INVALID_ARG, "bytes is NULL");
    if ((st = check_dims(d)) || (st = check_filter(f))) return st;
    *bytes = filter_ws(d, f);
    return ok();
}

gsf_status gsf_filter3d(const void *in, gsf_dtype in_t, gsf_dims d, const gsf_filter *f, void *out,
                        gsf_dtype out_t, void *ws, size_t ws_bytes, void *stream)
{
    gsf_status st;
    if ((st = check_dims(d)) || (st = check_filter(f)) || (st = check_ptr(in, 16, "in")) ||
        (st = check_ptr(out, 16, "out")) || (st = check_dtype(in_t, "in_t")) ||
        (st = check_dtype(out_t, "out_t")))
        return st;
    if (in_t != out_t)
        return fail(GSF_ERR_UNSUPPORTED, "in_t and out_t must be the same storage type");
    const size_t nb = (size_t)(d.nx * d.ny * d.nz) * elem_bytes(in_t);
    const size_t need = filter_ws(d, f);
    if (ws_bytes < need) return fail(GSF_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    if ((st = check_ptr(ws, 16, "ws"))) return st;
    if (overlaps(in, nb, out, nb) || overlaps(in, nb, ws, need) || overlaps(out, nb, ws, need))
        return fail(GSF_ERR_INVALID_ARG, "in, out and ws must not overlap");
    const gsf::Taps txy = make_taps(f->sigma_xy, f->truncate);
    const gsf::Taps tz = make_taps(f->sigma_z, f->truncate);
    const gsf::Dims dd = to_dims(d);
    const hipStream_t s = (hipStream_t)stream;
    // T1 (and the generic path's second scratch cube) are FP32 for every in_t
    void *T1 = ws;
    void *tmp = (char *)ws + cube_bytes(d);
    const gsf::Store sto = to_store(in_t);
    const gsf::Halo h = gsf::no_halo(dd);
    gsf::set_active_tune(tune_for(d, in_t));
    hipError_t e = gsf::launch_zpass(in, T1, sto, dd, h, tz, s);
    if (e == hipSuccess) e = gsf::launch_yx(T1, out, tmp, sto, dd, h, txy, nullptr, nullptr, s);
    return device_status(e, "gsf_filter3d launch");
}

gsf_status gsf_filter3d_weighted_workspace_size(gsf_dims d, const gsf_filter *f, size_t *bytes)
{
    gsf_status st;
    if (!bytes) return fail(GSF_ERR_INVALID_ARG, "bytes is NULL");
    if ((st = check_dims(d)) || (st = check_filter(f))) return st;
    *bytes = weighted_ws(d, f);
    return ok();
}

gsf_status gsf_filter3d_weighted(const void *in, const void *w, gsf_dtype t, gsf_dims d,
                                 const gsf_filter *f, void *out, void *ws, size_t ws_bytes,
                                 void *stream)
{
    gsf_status st;
    if ((st = check_dims(d)) || (st = check_filter(f)) || (st = check_ptr(in, 16, "in")) ||
        (st = check_ptr(w, 16, "w")) || (st = check_ptr(out, 16, "out")) ||
        (st = check_dtype(t, "t")))
        return st;
    if (t != GSF_F32)
        return fail(GSF_ERR_UNSUPPORTED, "the weighted convolution is implemented for GSF_F32");
    const size_t nb = (size_t)(d.nx * d.ny * d.nz) * sizeof(float);
    const size_t need = weighted_ws(d, f);
    if (ws_bytes < need) return fail(GSF_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    if ((st = check_ptr(ws, 16, "ws"))) return st;
    if (overlaps(in, nb, out, nb) || overlaps(w, nb, out, nb) || overlaps(in, nb, ws, need) ||
        overlaps(w, nb, ws, need) || overlaps(out, nb, ws, need))
        return fail(GSF_ERR_INVALID_ARG, "in, w, out and ws must not overlap");
    const gsf::Taps txy = make_taps(f->sigma_xy, f->truncate);
    const gsf::Taps tz = make_taps(f->sigma_z, f->truncate);
    const gsf::Dims dd = to_dims(d);
    const gsf::Halo h = gsf::no_halo(dd);
    const hipStream_t s = (hipStream_t)stream;
    // [P = d*w][T1][D][generic-path scratch]; N goes to out.  Where the radii
    // have compiled forms the product is formed inside the first spectral
    // pass and the quotient inside the last sweep (P and D stay unused).
    const size_t c = cube_bytes(d);
    float *P = (float *)ws;
    float *T1 = (float *)((char *)ws + c);
    float *D = (float *)((char *)ws + 2 * c);
    void *tmp = (char *)ws + 3 * c;
    const bool fused = gsf::zpass_fast(tz.r) && gsf::yx_fast(txy.r, dd);
    gsf::set_active_tune(tune_for(d, t));
    hipError_t e;
    if (fused) {
        e = gsf::launch_zpass_mul_fast((const float *)in, (const float *)w, T1, dd, tz, s);
    } else {
        e = gsf::launch_mul((const float *)in, (const float *)w, P, dd.voxels(), s);
        if (e == hipSuccess) e = gsf::launch_zpass(P, T1, gsf::Store::F32, dd, h, tz, s);
    }
    if (e == hipSuccess)
        e = gsf::launch_yx(T1, out, tmp, gsf::Store::F32, dd, h, txy, nullptr, nullptr, s);
    if (e == hipSuccess) e = gsf::launch_zpass(w, T1, gsf::Store::F32, dd, h, tz, s);
    if (fused) {
        if (e == hipSuccess) e = gsf::launch_yx_div_fast(T1, (float *)out, dd, txy, s);
    } else {
        if (e == hipSuccess)
            e = gsf::launch_yx(T1, D, tmp, gsf::Store::F32, dd, h, txy, nullptr, nullptr, s);
        if (e == hipSuccess)
            e = gsf::launch_div((const float *)out, D, (float *)out, dd.voxels(), s);
    }
    return device_status(e, "gsf_filter3d_weighted launch");
}

gsf_status gsf_local_stats_workspace_size(gsf_dims d, gsf_box b, size_t *bytes)
{
    gsf_status st;
    if (!bytes) return fail(GSF_ERR_INVALID_ARG, "bytes is NULL");
    if ((st = check_dims(d)) || (st = check_box(b))) return st;
    *bytes = stats_ws(d, b);
    return ok();
}

gsf_status gsf_local_stats(const void *F, gsf_dtype t, gsf_dims d, gsf_box b, float *mean,
                           float *stdev, void *ws, size_t ws_bytes, void *stream)
{
    gsf_status st;
    if ((st = check_dims(d)) || (st = check_box(b)) || (st = check_ptr(F, 16, "F")) ||
        (st = check_dtype(t, "t")))
        return st;
    if (!mean && !stdev) return fail(GSF_ERR_INVALID_ARG, "mean and stdev are both NULL");
    if (mean && (st = check_ptr(mean, 16, "mean"))) return st;
    if (stdev && (st = check_ptr(stdev, 16, "stdev"))) return st;
    const size_t nb = (size_t)(d.nx * d.ny * d.nz) * sizeof(float);
    const size_t fb = (size_t)(d.nx * d.ny * d.nz) * elem_bytes(t);
    const size_t need = stats_ws(d, b);
    if (ws_bytes < need) return fail(GSF_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    if ((st = check_ptr(ws, 16, "ws"))) return st;
    if (overlaps(F, fb, mean, nb) || overlaps(F, fb, stdev, nb) || overlaps(mean, nb, stdev, nb) ||
        overlaps(ws, need, F, fb) || overlaps(ws, need, mean, nb) || overlaps(ws, need, stdev, nb))
        return fail(GSF_ERR_INVALID_ARG, "F, mean, stdev and ws must not overlap");
    const gsf::Dims dd = to_dims(d);
    const StatsWs w = carve_stats((char *)ws, d, stats_cubes(b, d), 1);
    const hipStream_t s = (hipStream_t)stream;
    const gsf::Store sto = to_store(t);
    gsf::set_active_tune(tune_for(d, t));
    hipError_t e = gsf::launch_mean(F, sto, dd, w.partials, w.shift, s);
    if (e == hipSuccess)
        e = gsf::launch_stats(F, sto, dd, to_box(b), w.shift, w.w1, w.w2, w.w3, w.w4, mean, stdev,
                              nullptr, 0.0, s);
    return device_status(e, "gsf_local_stats launch");
}

gsf_status gsf_threshold(const void *F, gsf_dtype t, const float *mean, const float *stdev,
                         gsf_dims d, double k, uint64_t *mask, void *stream)
{
    gsf_status st;
    if ((st = check_dims(d)) || (st = check_ptr(F, 16, "F")) || (st = check_dtype(t, "t")) ||
        (st = check_ptr(mean, 16, "mean")) || (st = check_ptr(stdev, 16, "stdev")) ||
        (st = check_ptr(mask, 8, "mask")))
        return st;
    if (!std::isfinite(k)) return fail(GSF_ERR_INVALID_ARG, "k must be finite");
    const size_t nb = (size_t)(d.nx * d.ny * d.nz) * sizeof(float);
    const size_t fb = (size_t)(d.nx * d.ny * d.nz) * elem_bytes(t);
    const size_t mb = (size_t)to_dims(d).words() * sizeof(uint64_t);
    if (overlaps(mask, mb, F, fb) || overlaps(mask, mb, mean, nb) || overlaps(mask, mb, stdev, nb))
        return fail(GSF_ERR_INVALID_ARG, "mask must not overlap its inputs");
    return device_status(gsf::launch_threshold(F, to_store(t), mean, stdev, to_dims(d), k, mask,
                                               (hipStream_t)stream),
                         "gsf_threshold launch");
}

namespace {

// The core of a cube: its dims less the halo on both sides of each axis.
gsf_dims core_dims(const gsf_cube &q)
{
    return gsf_dims{q.dims.nx - 2 * (int64_t)q.halo[0], q.dims.ny - 2 * (int64_t)q.halo[1],
                    q.dims.nz - 2 * (int64_t)q.halo[2]};
}

gsf_status check_batch(const gsf_cube *cubes, int32_t ncubes, const gsf_filter *f, int32_t nfilt,
                       gsf_box b, gsf_dims *largest)
{
    gsf_status st;
    if (!cubes || ncubes < 1) return fail(GSF_ERR_INVALID_ARG, "need at least one cube");
    if (!f || nfilt < 1) return fail(GSF_ERR_INVALID_ARG, "need at least one filter");
    if ((st = check_box(b))) return st;
    for (int32_t j = 0; j < nfilt; ++j)
        if ((st = check_filter(&f[j]))) return st;
    int64_t best = 0;
    for (int32_t c = 0; c < ncubes; ++c) {
        const gsf_cube &q = cubes[c];
        if ((st = check_dims(q.dims))) return st;
        if ((st = check_dtype(q.dtype, "cube dtype"))) return st;
        if (q.halo[0] < 0 || q.halo[1] < 0 || q.halo[2] < 0)
            return fail(GSF_ERR_INVALID_ARG, "cube %d: negative halo", c);
        const gsf_dims core = core_dims(q);
        if (core.nx < 1 || core.ny < 1 || core.nz < 1)
            return fail(GSF_ERR_INVALID_ARG, "cube %d: halo leaves no core", c);
        const int64_t v = q.dims.nx * q.dims.ny * q.dims.nz;
        if (v > best) { best = v; *largest = q.dims; }
    }
    return GSF_OK;
}

// Independent cubes of a batch run concurrently on up to kSlots library
// streams forked from the caller's stream, each with its own workspace slot;
// a single cube runs on the caller's stream.
// Measured on the 96-sub-cube batch: 4 slots 85 ms per call, 8 slots 78 ms,
// 16 slots 75 ms; with the later kernels 16 slots 71.0 ms, 24 69.7 ms, 32
// 67.8 ms, 48 67.9 ms, 64 68.1 ms.  Each slot holds a workspace for the
// largest cube, so the slot count is also capped at what fits kSlotBudget
// bytes of workspace (at least one slot).
constexpr int kSlots = 32;
constexpr size_t kSlotBudget = (size_t)64 << 30;

// Filters a merged spatial sweep handles together (the compiled forms).
constexpr int kMaxMerge = 3;

// One workspace slot, sized for the batch's largest array:
// [T1 x nT][F x nF][statistics cubes x nS][shift partials x nF][shifts x nF].
// nT is 2 when two spectral-pass groups can share one read of the cube (a
// compiled radius pair), else 1; nF is the largest number of filters that
// share a spectral pass (at most kMaxMerge: larger groups are swept
// kMaxMerge at a time); nS is 2, or 4 when some cube needs the generic
// statistics path.
struct Layout {
    gsf_dims largest;
    int nT;
    int nF;
    int nS;
};

bool same_group(const gsf_filter &a, const gsf_filter &b)
{
    return a.sigma_z == b.sigma_z && a.truncate == b.truncate;
}

// Spectral-pass groups of a filter bank: filters with equal (sigma_z,
// truncate), in order of first appearance, each group's members sorted by
// spatial radius and cut into sweeps of at most kMaxMerge filters.
// Consecutive groups (0, 1), (2, 3), ... whose spectral radii form a compiled
// pair are marked to share one read of the cube.
struct Group {
    int32_t rep;                                  // a member (its sigma_z, truncate)
    std::vector<std::vector<int32_t>> sweeps;
    bool paired_with_next = false;
};

std::vector<Group> filter_groups(const gsf_filter *f, int32_t nfilt)
{
    std::vector<Group> groups;
    std::vector<char> seen((size_t)nfilt, 0);
    for (int32_t g = 0; g < nfilt; ++g) {
        if (seen[g]) continue;
        std::vector<int32_t> m;
        for (int32_t j = g; j < nfilt; ++j)
            if (!seen[j] && same_group(f[g], f[j])) m.push_back(j), seen[j] = 1;
        std::stable_sort(m.begin(), m.end(), [&](int32_t a, int32_t b2) {
            return make_taps(f[a].sigma_xy, f[a].truncate).r <
                   make_taps(f[b2].sigma_xy, f[b2].truncate).r;
        });
        Group gr;
        gr.rep = g;
        for (size_t i = 0; i < m.size(); i += kMaxMerge)
            gr.sweeps.emplace_back(m.begin() + i,
                                   m.begin() + std::min(m.size(), i + (size_t)kMaxMerge));
        groups.push_back(std::move(gr));
    }
    for (size_t i = 0; i + 1 < groups.size(); i += 2) {
        const int ra = make_taps(f[groups[i].rep].sigma_z, f[groups[i].rep].truncate).r;
        const int rb = make_taps(f[groups[i + 1].rep].sigma_z, f[groups[i + 1].rep].truncate).r;
        groups[i].paired_with_next = gsf::zpass_pair(ra, rb) >= 0;
    }
    return groups;
}

Layout find_layout(const gsf_cube *cubes, int32_t ncubes, const gsf_filter *f, int32_t nfilt,
                   gsf_box b, gsf_dims largest)
{
    Layout L{largest, 1, 1, 2};
    for (int32_t g = 0; g < nfilt; ++g) {
        int n = 0;
        for (int32_t j = 0; j < nfilt; ++j) n += same_group(f[g], f[j]) ? 1 : 0;
        L.nF = std::max(L.nF, std::min(n, kMaxMerge));
    }
    for (const Group &g : filter_groups(f, nfilt))
        if (g.paired_with_next) L.nT = 2;
    for (int32_t c = 0; c < ncubes; ++c) {
        const gsf_dims core{cubes[c].dims.nx - 2 * (int64_t)cubes[c].halo[0],
                            cubes[c].dims.ny - 2 * (int64_t)cubes[c].halo[1],
                            cubes[c].dims.nz - 2 * (int64_t)cubes[c].halo[2]};
        L.nS = std::max(L.nS, stats_cubes(b, core));
    }
    return L;
}

size_t slot_ws(const Layout &L)
{
    return (size_t)(L.nT + L.nF + L.nS) * cube_bytes(L.largest) + shift_bytes(L.nF);
}

int find_slots(int32_t ncubes, const Layout &L)
{
    int n = ncubes < kSlots ? ncubes : kSlots;
    const size_t fit = kSlotBudget / slot_ws(L);
    if ((size_t)n > fit) n = fit > 0 ? (int)fit : 1;
    return n;
}

size_t find_ws(const Layout &L, int32_t ncubes)
{
    return (size_t)find_slots(ncubes, L) * slot_ws(L);
}

// Per-device library state, created once per device (gsf_init, or the first
// call that needs it outside a stream capture) and kept until the process
// ends: the batch streams with their fork/join events (default priority).
struct DeviceState {
    bool streams_ready = false;
    hipStream_t stream[kSlots];
    hipEvent_t fork;
    hipEvent_t join[kSlots];
    void *scratch = nullptr;   // this device's copy of `scratch` (gsf_find_noalloc)
};

// The workspace of gsf_find_noalloc: one gsf_find slot in a library-owned
// device array, for callers that cannot allocate.  Each device holds its own
// copy at its own address.  In host code the name `scratch` is a host-side
// stand-in, not device memory: only the address hipGetSymbolAddress returns
// for the current device (DeviceState::scratch) is ever passed to kernels.
// Nothing in it needs clearing: every byte a call reads (the spectral
// intermediate, F, window sums, shift partials and shifts) is written by that
// call's kernels first.
constexpr size_t kScratchBytes = GSF_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_dev_mu;
std::map<int, DeviceState> g_dev;

gsf_status current_device(int *dev)
{
    if (hipGetDevice(dev) != hipSuccess) return fail(GSF_ERR_DEVICE, "hipGetDevice failed");
    return GSF_OK;
}

// Is `s` being captured into a graph?  Streams and symbol addresses are set
// up outside captures only.
bool capturing(hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return false;
    return cs != hipStreamCaptureStatusNone;
}

gsf_status init_streams(DeviceState &ds)
{
    if (ds.streams_ready) return GSF_OK;
    bool good = hipEventCreateWithFlags(&ds.fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < kSlots && good; ++i)
        good = hipStreamCreateWithFlags(&ds.stream[i], hipStreamNonBlocking) == hipSuccess &&
               hipEventCreateWithFlags(&ds.join[i], hipEventDisableTiming) == hipSuccess;
    if (!good) return fail(GSF_ERR_DEVICE, "creating the batch streams failed");
    ds.streams_ready = true;
    return GSF_OK;
}

// Look up this device's scratch address once (the device must be current).
gsf_status init_scratch(DeviceState &ds)
{
    if (ds.scratch) return GSF_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(GSF_ERR_DEVICE, "looking up the scratch address failed: %s",
                    hipGetErrorString(e));
    ds.scratch = p;
    return GSF_OK;
}

// Check every output pointer of a batch against the inputs, the workspace
// and each other; nothing is enqueued.
gsf_status check_outputs(const gsf_cube *cubes, int32_t ncubes, int32_t nfilt,
                         uint64_t *const *masks, void *const *F_out, float *const *mean_out,
                         float *const *std_out, const void *ws, size_t need)
{
    gsf_status st;
    if (!masks) return fail(GSF_ERR_INVALID_ARG, "masks is NULL");
    for (int32_t c = 0; c < ncubes; ++c) {
        const gsf_cube &q = cubes[c];
        if ((st = check_ptr(q.data, 16, "cube data"))) return st;
        const gsf_dims core = core_dims(q);
        const size_t qb = (size_t)(q.dims.nx * q.dims.ny * q.dims.nz) * elem_bytes(q.dtype);
        const size_t nv = (size_t)(core.nx * core.ny * core.nz);   // outputs cover the core
        const size_t nb = nv * sizeof(float);
        const size_t fb = nv * elem_bytes(q.dtype);   // F_out
        const size_t mb = (size_t)to_dims(core).words() * sizeof(uint64_t);
        if (overlaps(ws, need, q.data, qb))
            return fail(GSF_ERR_INVALID_ARG, "cube %d overlaps the workspace", c);
        for (int32_t j = 0; j < nfilt; ++j) {
            const int64_t o = (int64_t)c * nfilt + j;
            if ((st = check_ptr(masks[o], 8, "masks[i]"))) return st;
            const void *outs[4] = {masks[o], F_out ? F_out[o] : nullptr,
                                   mean_out ? mean_out[o] : nullptr, std_out ? std_out[o] : nullptr};
            const size_t sizes[4] = {mb, fb, nb, nb};
            for (int a = 1; a < 4; ++a)
                if (outs[a] && (st = check_ptr(outs[a], 16, "F/mean/std output"))) return st;
            for (int a = 0; a < 4; ++a) {
                if (!outs[a]) continue;
                if (overlaps(outs[a], sizes[a], q.data, qb) || overlaps(outs[a], sizes[a], ws, need))
                    return fail(GSF_ERR_INVALID_ARG, "output of cube %d filter %d overlaps input or ws",
                                c, j);
                for (int b2 = a + 1; b2 < 4; ++b2)
                    if (outs[b2] && overlaps(outs[a], sizes[a], outs[b2], sizes[b2]))
                        return fail(GSF_ERR_INVALID_ARG, "outputs of cube %d filter %d overlap", c, j);
            }
        }
    }
    return GSF_OK;
}

// Enqueue the whole path for a validated batch.  Slot i of `nslots` uses
// bytes [i * slot_ws(L), (i+1) * slot_ws(L)) of ws; with more than one slot
// the cubes run on the device's library streams (ss), forked from and joined
// back to `caller`.
gsf_status find_enqueue(const gsf_cube *cubes, int32_t ncubes, const gsf_filter *f, int32_t nfilt,
                        gsf_box b, double k, uint64_t *const *masks, void *const *F_out,
                        float *const *mean_out, float *const *std_out, void *ws, const Layout &L,
                        int nslots, DeviceState *ss, hipStream_t caller)
{
    // Largest cubes first, each to the slot with the least work so far.
    std::vector<int32_t> order((size_t)ncubes);
    for (int32_t c = 0; c < ncubes; ++c) order[(size_t)c] = c;
    auto vox = [&](int32_t c) { return cubes[c].dims.nx * cubes[c].dims.ny * cubes[c].dims.nz; };
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b2) { return vox(a) > vox(b2); });
    std::vector<int> slot_of((size_t)ncubes, 0);
    std::vector<int64_t> load((size_t)nslots, 0);
    for (int32_t c : order) {
        const int sl = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        slot_of[(size_t)c] = sl;
        load[(size_t)sl] += vox(c);
    }
    const std::vector<Group> groups = filter_groups(f, nfilt);
    if (nslots > 1) {
        if (hipEventRecord(ss->fork, caller) != hipSuccess)
            return fail(GSF_ERR_DEVICE, "gsf_find: fork event failed");
        for (int i = 0; i < nslots; ++i)
            if (hipStreamWaitEvent(ss->stream[i], ss->fork, 0) != hipSuccess)
                return fail(GSF_ERR_DEVICE, "gsf_find: fork wait failed");
    }
    const size_t sws = slot_ws(L);
    const size_t cb = cube_bytes(L.largest);
    const gsf_status run = [&]() -> gsf_status {
    for (int32_t c : order) {
        const int sl = slot_of[(size_t)c];
        const hipStream_t s = nslots > 1 ? ss->stream[sl] : caller;
        char *base = (char *)ws + (size_t)sl * sws;
        void *T1s[2] = {base, L.nT > 1 ? base + cb : nullptr};   // FP32
        char *Fbuf = base + (size_t)L.nT * cb;                   // nF cubes
        const StatsWs w =
            carve_stats(base + (size_t)(L.nT + L.nF) * cb, L.largest, L.nS, L.nF);
        const gsf_cube &q = cubes[c];
        const gsf_dims core = core_dims(q);
        const gsf::Dims dd = to_dims(core);           // the core: F, statistics, masks
        const gsf::Halo h{q.dims.nx, q.dims.ny, q.dims.nz, q.halo[0], q.halo[1], q.halo[2]};
        const gsf::Store sto = to_store(q.dtype);
        const gsf::Tune tune = tune_for(core, q.dtype);
        gsf::set_active_tune(tune);
        bool have_next = false;                       // T1s[1] holds the next group's pass
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            const Group &gr = groups[gi];
            const gsf::Taps tz = make_taps(f[gr.rep].sigma_z, f[gr.rep].truncate);
            void *T1 = T1s[0];
            if (have_next) {
                T1 = T1s[1];
                have_next = false;
            } else {
                hipError_t e = hipErrorInvalidValue;
                if (gr.paired_with_next && tune.pair_spectral && L.nT > 1) {
                    const Group &nx = groups[gi + 1];
                    const gsf::Taps tz2 = make_taps(f[nx.rep].sigma_z, f[nx.rep].truncate);
                    e = gsf::launch_zpass_pair(q.data, T1s[0], T1s[1], sto, dd, h, tz, tz2, s);
                    have_next = e == hipSuccess;
                }
                if (e == hipErrorInvalidValue) e = gsf::launch_zpass(q.data, T1, sto, dd, h, tz, s);
                if (e != hipSuccess) return device_status(e, "gsf_find launch");
            }
            for (const std::vector<int32_t> &sw : gr.sweeps) {
                const int n = (int)sw.size();
                gsf::Taps txy[kMaxMerge];
                void *F[kMaxMerge];
                int r[kMaxMerge];
                for (int i = 0; i < n; ++i) {
                    const int64_t o = (int64_t)c * nfilt + sw[i];
                    txy[i] = make_taps(f[sw[i]].sigma_xy, f[sw[i]].truncate);
                    r[i] = txy[i].r;
                    F[i] = (F_out && F_out[o]) ? F_out[o] : (void *)(Fbuf + (size_t)i * cb);
                }
                const int form = (tune.merge && n >= 2) ? gsf::merged_form(r, n) : -1;
                int nparts[kMaxMerge] = {0, 0, 0};
                hipError_t e = hipSuccess;
                if (form >= 0) {
                    int np = 0;
                    e = gsf::launch_yx_merged(form, tune.merged_shape, T1, F, sto, dd, h, txy,
                                              w.partials, &np, s);
                    for (int i = 0; i < n; ++i) nparts[i] = np;
                }
                if (form < 0 || e == hipErrorInvalidValue) {
                    e = hipSuccess;
                    for (int i = 0; i < n && e == hipSuccess; ++i)
                        e = gsf::launch_yx(T1, F[i], w.w1, sto, dd, h, txy[i],
                                           w.partials + (size_t)i * gsf::kMaxPartials, &nparts[i], s);
                }
                for (int i = 0; i < n && e == hipSuccess; ++i) {
                    const int64_t o = (int64_t)c * nfilt + sw[i];
                    double *parts = w.partials + (size_t)i * gsf::kMaxPartials;
                    double *shift = w.shift + i;
                    e = nparts[i] > 0
                            ? gsf::launch_mean_partials(parts, nparts[i], dd.voxels(), shift, s)
                            : gsf::launch_mean(F[i], sto, dd, parts, shift, s);
                    if (e == hipSuccess)
                        e = gsf::launch_stats(F[i], sto, dd, to_box(b), shift, w.w1, w.w2, w.w3,
                                              w.w4, mean_out ? mean_out[o] : nullptr,
                                              std_out ? std_out[o] : nullptr, masks[o], k, s);
                }
                if (e != hipSuccess) return device_status(e, "gsf_find launch");
            }
        }
    }
    return GSF_OK;
    }();
    if (nslots > 1) {
        // join, also after a failed launch: the caller's stream waits for every slot
        for (int i = 0; i < nslots; ++i)
            if (hipEventRecord(ss->join[i], ss->stream[i]) != hipSuccess ||
                hipStreamWaitEvent(caller, ss->join[i], 0) != hipSuccess)
                return fail(GSF_ERR_DEVICE, "gsf_find: join failed");
    }
    return run != GSF_OK ? run : ok();
}

// Serialises the enqueueing of calls that use the per-device state (the
// batch streams).
std::mutex g_enqueue_mu;

}  // namespace

gsf_status gsf_init(void)
{
    int dev = 0;
    gsf_status st;
    if ((st = current_device(&dev))) return st;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    DeviceState &ds = g_dev[dev];
    if ((st = init_streams(ds)) || (st = init_scratch(ds))) return st;
    return ok();
}

int32_t gsf_size_class(gsf_dims core)
{
    if (check_dims(core) != GSF_OK) return -1;
    return size_class(core);
}

gsf_status gsf_tuning_set(int32_t cls, gsf_dtype t, const gsf_tuning *cfg)
{
    gsf_status st;
    if ((st = check_dtype(t, "dtype")) || (st = check_tuning(cfg))) return st;
    if (cls < -1 || cls >= kSizeClasses)
        return fail(GSF_ERR_INVALID_ARG, "size class must be -1 or in [0, %d)", kSizeClasses);
    gsf::Tune v;
    v.merge = cfg->merge_sweeps;
    v.merged_shape = cfg->merged_shape;
    v.sweep_blocks = cfg->sweep_blocks;
    v.yz_waves = cfg->yz_waves;
    v.pair_spectral = cfg->pair_spectral;
    v.x_exits = cfg->x_exits;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (int c = 0; c < kSizeClasses; ++c)
        if (cls < 0 || c == cls) g_tune[(int)t][c] = v;
    return ok();
}

gsf_status gsf_tuning_get(int32_t cls, gsf_dtype t, gsf_tuning *cfg)
{
    gsf_status st;
    if ((st = check_dtype(t, "dtype"))) return st;
    if (!cfg) return fail(GSF_ERR_INVALID_ARG, "tuning pointer is NULL");
    if (cls < 0 || cls >= kSizeClasses)
        return fail(GSF_ERR_INVALID_ARG, "size class must be in [0, %d)", kSizeClasses);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const gsf::Tune &v = g_tune[(int)t][cls];
    cfg->merge_sweeps = v.merge;
    cfg->merged_shape = v.merged_shape;
    cfg->sweep_blocks = v.sweep_blocks;
    cfg->yz_waves = v.yz_waves;
    cfg->pair_spectral = v.pair_spectral;
    cfg->x_exits = v.x_exits;
    return ok();
}

gsf_status gsf_tuning_reset(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_table.reset();
    return ok();
}

gsf_status gsf_find_workspace_size(const gsf_cube *cubes, int32_t ncubes, const gsf_filter *f,
                                   int32_t nfilt, gsf_box b, size_t *bytes)
{
    gsf_status st;
    gsf_dims largest{};
    if (!bytes) return fail(GSF_ERR_INVALID_ARG, "bytes is NULL");
    if ((st = check_batch(cubes, ncubes, f, nfilt, b, &largest))) return st;
    *bytes = find_ws(find_layout(cubes, ncubes, f, nfilt, b, largest), ncubes);
    return ok();
}

gsf_status gsf_find(const gsf_cube *cubes, int32_t ncubes, const gsf_filter *f, int32_t nfilt,
                    gsf_box b, double k, uint64_t *const *masks, void *const *F_out,
                    float *const *mean_out, float *const *std_out, void *ws, size_t ws_bytes,
                    void *stream)
{
    gsf_status st;
    gsf_dims largest{};
    if ((st = check_batch(cubes, ncubes, f, nfilt, b, &largest))) return st;
    if (!std::isfinite(k)) return fail(GSF_ERR_INVALID_ARG, "k must be finite");
    if (!masks) return fail(GSF_ERR_INVALID_ARG, "masks is NULL");
    const Layout L = find_layout(cubes, ncubes, f, nfilt, b, largest);
    const size_t need = find_ws(L, ncubes);
    if (ws_bytes < need) return fail(GSF_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    if ((st = check_ptr(ws, 16, "ws"))) return st;
    if ((st = check_outputs(cubes, ncubes, nfilt, masks, F_out, mean_out, std_out, ws, need)))
        return st;
    const int nslots = find_slots(ncubes, L);
    const hipStream_t caller = (hipStream_t)stream;
    DeviceState *ss = nullptr;
    std::unique_lock<std::mutex> lock(g_enqueue_mu, std::defer_lock);
    if (nslots > 1) {
        lock.lock();
        int dev = 0;
        if ((st = current_device(&dev))) return st;
        {
            std::lock_guard<std::mutex> lk(g_dev_mu);
            ss = &g_dev[dev];
            if (!ss->streams_ready) {
                if (capturing(caller))
                    return fail(GSF_ERR_UNSUPPORTED,
                                "gsf_find: a batch captured into a graph needs the library "
                                "streams; call gsf_init() before the capture");
                if ((st = init_streams(*ss))) return st;
            }
        }
    }
    return find_enqueue(cubes, ncubes, f, nfilt, b, k, masks, F_out, mean_out, std_out, ws,
                        L, nslots, ss, caller);
}

gsf_status gsf_find_noalloc(const gsf_cube *cubes, int32_t ncubes, const gsf_filter *f,
                            int32_t nfilt, gsf_box b, double k, uint64_t *const *masks,
                            void *const *F_out, float *const *mean_out, float *const *std_out,
                            void *stream)
{
    gsf_status st;
    gsf_dims largest{};
    if ((st = check_batch(cubes, ncubes, f, nfilt, b, &largest))) return st;
    if (!std::isfinite(k)) return fail(GSF_ERR_INVALID_ARG, "k must be finite");
    if (!masks) return fail(GSF_ERR_INVALID_ARG, "masks is NULL");
    const Layout L = find_layout(cubes, ncubes, f, nfilt, b, largest);
    const size_t need = slot_ws(L);
    if (need > kScratchBytes)
        return fail(GSF_ERR_BUDGET,
                    "gsf_find_noalloc: this batch needs %zu bytes of scratch, the library "
                    "holds %zu (GSF_NOALLOC_SCRATCH_BYTES)",
                    need, kScratchBytes);
    const hipStream_t caller = (hipStream_t)stream;
    void *ws = nullptr;
    {
        int dev = 0;
        if ((st = current_device(&dev))) return st;
        std::lock_guard<std::mutex> lk(g_dev_mu);
        DeviceState &ds = g_dev[dev];
        if (!ds.scratch) {
            if (capturing(caller))
                return fail(GSF_ERR_UNSUPPORTED,
                            "gsf_find_noalloc: the scratch address is looked up outside "
                            "captures; call gsf_init() before the capture");
            if ((st = init_scratch(ds))) return st;
        }
        ws = ds.scratch;
    }
    if ((st = check_outputs(cubes, ncubes, nfilt, masks, F_out, mean_out, std_out, ws, need)))
        return st;
    return find_enqueue(cubes, ncubes, f, nfilt, b, k, masks, F_out, mean_out, std_out, ws, L, 1,
                        nullptr, caller);
}

}  // extern "C"
