// Internal interface between the C-ABI layer (gsf_api.cpp) and the kernels
// (gsf_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gsf.h"

namespace gsf {

constexpr int kMaxTaps = 2 * GSF_MAX_RADIUS + 1;

// FP32 taps of one axis, offsets -r..r at g[0..2r].  Passed to kernels by value.
struct Taps {
    float g[kMaxTaps];
    int r;
};

// Storage type of a cube (values as in gsf_dtype); arithmetic is FP32.
enum class Store { F32 = 0, F16 = 1, BF16 = 2 };

inline size_t store_bytes(Store s) { return s == Store::F32 ? 4 : 2; }

// Suffix of kernel timing names for a storage type ("" for FP32).
template <typename St>
constexpr const char *store_suffix()
{
    return sizeof(St) == 4 ? "" : __is_same(St, _Float16) ? ",f16" : ",bf16";
}

struct Dims {
    int64_t nx, ny, nz;
    int64_t voxels() const { return nx * ny * nz; }
    int64_t words() const { return nx * ny * ((nz + 63) / 64); }
};

// Input array of the filter and the core it produces: the array is NX x NY x
// NZ, the core (dims passed alongside as Dims) starts at (hx, hy, hz).  The
// spectral pass writes T1 as NX x NY rows of the core's nz values.
struct Halo {
    int64_t NX, NY, NZ;
    int hx, hy, hz;
};

inline Halo no_halo(Dims d) { return Halo{d.nx, d.ny, d.nz, 0, 0, 0}; }

// Window of length B: offsets [lo, lo + B - 1] with lo = -floor(B/2).
struct Box {
    int bx, by, bz;
};

// Launch configuration of the kernels with more than one compiled shape
// (what the tuning entries of include/gsf.h set; defaults are the measured
// best on the 512x512x1024 cube):
//   merge         1: one merged spatial sweep per sigma_z group where a form is
//                 compiled; 0: one sweep per filter
//   merged_shape  block shape of the merged sweep (kMergedShape index)
//   sweep_blocks  blocks a spatial sweep aims for before it splits x into
//                 chunks (each chunk re-reads 2r planes)
//   yz_waves      waves per block of the yz window kernel (3, 5 or 9; 0: the
//                 one that walks the fewest columns for the cube's depth)
//   pair_spectral 1: two spectral-pass groups with a compiled radius pair
//                 share one read of the cube; 0: one spectral pass each
//   x_exits       1: the x walk's last ring turn stops at the first 16-step
//                 boundary past the end; 0: it runs whole turns
// (the table's defaults per storage type and size class: gsf_api.cpp)
struct Tune {
    int merge = 1;
    int merged_shape = 0;
    int sweep_blocks = 512;
    int yz_waves = 0;
    int pair_spectral = 1;
    int x_exits = 1;
};

// The configuration of the call being enqueued on this thread: the API layer
// sets it per cube before launching; launchers read it (enqueueing is
// synchronous, so a thread-local value cannot be seen by another call).
const Tune &active_tune();
void set_active_tune(const Tune &t);

// Number of per-block partial sums used for the global shift.
constexpr int kShiftBlocks = 1024;

// Kernel timing: a Scope records a start event on construction and a stop
// event on destruction when profiling is enabled; kernels launched inside the
// scope are what it times.
namespace prof {
bool enabled();
struct Scope {
    Scope(const char *name, hipStream_t s);
    ~Scope();
    int slot;
    hipStream_t stream;
};
}  // namespace prof

// Per-block FP64 partial sums of F for the statistics' shift.
constexpr int kMaxPartials = 1 << 16;

// Radii with compiled fast filter paths (gsf_filter.hip); larger radii use
// the generic passes.
constexpr int kMaxFastRz = 32;
constexpr int kMaxFastRxy = 16;
bool zpass_fast(int rz);
// Buffer-addressed kernels need one x-plane below 2^30 bytes.
bool plane_fits(Dims d);
bool yx_fast(int rxy, Dims d);
hipError_t launch_zpass_fast(const void *in, void *T1, Store st, Dims d, const Halo &h,
                             const Taps &tz, hipStream_t s);
// Two spectral passes of different radii from one read of the input (Ta with
// taps ta, Tb with tb); zpass_pair(ra, rb) is the compiled pair's index or
// -1, and launch_zpass_pair returns hipErrorInvalidValue for other radii.
// Bit for bit the results of two launch_zpass_fast calls.
int zpass_pair(int ra, int rb);
hipError_t launch_zpass_pair(const void *in, void *Ta, void *Tb, Store st, Dims d, const Halo &h,
                             const Taps &ta, const Taps &tb, hipStream_t s);
hipError_t launch_yx_fast(const void *T1, void *F, Store st, Dims d, const Halo &h,
                          const Taps &txy, double *partials, int *nparts, hipStream_t s);
// Merged spatial sweeps: one kernel applies the spatial passes of 2 or 3
// filters that share T1 (equal sigma_z).  merged_form(r, nf) returns the
// index of the compiled form for radii r[0] < r[1] (< r[2]), or -1.
// launch_yx_merged writes F[i] for taps txy[i] (radius r[i]) with block
// shape `shape` (an index of kMergedShape: rows per lane and waves per
// block); its shift partials go to partials + i * kMaxPartials (*nparts
// blocks each, 0 if not written).  hipErrorInvalidValue when the form does
// not fit the call.
constexpr int kMaxMergedR = 12;
int merged_form(const int *r, int nf);
hipError_t launch_yx_merged(int form, int shape, const void *T1, void *const *F, Store st,
                            Dims d, const Halo &h, const Taps *txy, double *partials,
                            int *nparts, hipStream_t s);
// FP32 weighted convolution (Eq. 1) pieces, no halo; hipErrorInvalidValue
// when the radius has no compiled form.  T1 = gz * (in * w) along z; and
// F = F / (gxy * (gxy * T1 along y) along x), 0 where the divisor is 0, in
// place (F holds the numerator on entry).
hipError_t launch_zpass_mul_fast(const float *in, const float *w, float *T1, Dims d,
                                 const Taps &tz, hipStream_t s);
hipError_t launch_yx_div_fast(const float *T1, float *F, Dims d, const Taps &txy, hipStream_t s);

// Window lengths with compiled fast statistics paths (gsf_stats.hip): by and
// bx in {8, 16, 32, 64}, bz <= 65, planes of at most 2^27 voxels.  G: two
// cubes of floats (the yz-window sums as interleaved pairs).
bool stats_fast_path(Box b, Dims d);
hipError_t launch_stats_fast(const void *F, Store st, Dims d, Box b, const double *shift,
                             float *G, float *mean, float *stdev, uint64_t *mask, double k,
                             hipStream_t s);

// Kernel launchers.  All enqueue on `s` and return hipGetLastError().
// Cubes passed as void * hold elements of storage type st, except the
// spectral intermediate T1 (and the generic path's tmp), which are FP32.
// Spectral pass: T1 = gz * in along z.  d: the core; h: the input array.
hipError_t launch_zpass(const void *in, void *T1, Store st, Dims d, const Halo &h,
                        const Taps &tz, hipStream_t s);
// Spatial passes: F = gxy * (gxy * T1 along y) along x, F of the core dims d.
// tmp is a scratch cube (NX x ny x nz) used only by the generic path.  If
// partials is non-null, per-block FP64 sums of F may be written there;
// *nparts gets their count (0 if not).
hipError_t launch_yx(const void *T1, void *F, void *tmp, Store st, Dims d, const Halo &h,
                     const Taps &txy, double *partials, int *nparts, hipStream_t s);
// shift[0] = mean of F (FP64), full pass over F with a fixed reduction order.
hipError_t launch_mean(const void *F, Store st, Dims d, double *partials, double *shift,
                       hipStream_t s);
// shift[0] = (sum of n partials) / V, fixed order.
hipError_t launch_mean_partials(const double *partials, int n, int64_t V, double *shift,
                                hipStream_t s);
// Local statistics and (optionally) the mask.  ws1..ws4: four scratch cubes,
// consecutive pieces of one workspace.
hipError_t launch_stats(const void *F, Store st, Dims d, Box b, const double *shift, float *ws1,
                        float *ws2, float *ws3, float *ws4, float *mean, float *stdev,
                        uint64_t *mask, double k, hipStream_t s);
// Weighted convolution pieces: P = d * w; F = N / D (0 where D == 0).
hipError_t launch_mul(const float *d, const float *w, float *P, int64_t n, hipStream_t s);
hipError_t launch_div(const float *N, const float *D, float *F, int64_t n, hipStream_t s);
hipError_t launch_threshold(const void *F, Store st, const float *mean, const float *stdev,
                            Dims d, double k, uint64_t *mask, hipStream_t s);

}  // namespace gsf
