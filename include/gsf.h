/*
 * gsf.h -- C ABI of libgsf, the MI355X (gfx950) hot path of a filter-based
 * HI spectral-line source finder (Westerlund & Harris, "Performance Analysis
 * of GPU-Accelerated Filter-Based Source Finding for HI Spectral Line Image
 * Data", Experimental Astronomy).
 *
 * The path: a bank of separable 3-D Gaussian filters applied to a spectral
 * cube (Eq. 2, §2.1), a per-voxel local mean and standard deviation of each
 * filtered cube over a box around the voxel (§3.3), and the selection of
 * voxels above mean + k * std (§1, §3.3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Layout.  A cube of dims (nx, ny, nz) is one contiguous array, x slowest and
 *   z (the spectral axis) contiguous: voxel (x, y, z) sits at linear index
 *   (x*ny + y)*nz + z (§3.1: X is the major axis and Z the minor axis).
 * Memory.  Every data pointer is a DEVICE pointer on the current HIP device,
 *   owned by the caller: inputs, outputs and workspace.  The library never
 *   allocates or frees device memory in these calls and keeps no pointer
 *   after a call returns.  Data pointers must be 16-byte aligned; mask
 *   pointers 8-byte aligned.
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the null
 *   stream).  Calls validate their arguments synchronously, enqueue kernels on
 *   `stream` and return; results are valid once the stream has been
 *   synchronised.  Calls that overlap on one stream are ordered by it.
 * Errors.  Arguments are checked before anything is enqueued; an invalid
 *   call returns a non-zero gsf_status and leaves every output untouched.
 *   A failed launch returns GSF_ERR_DEVICE.  gsf_last_error() gives a
 *   human-readable detail for the calling thread.  The library never aborts
 *   and never prints.
 * Filters.  Taps per axis are g[o] = exp(-o^2 / (2 sigma^2)) / sum, for
 *   o = -r..r, r = ceil(truncate * sigma) evaluated in FP64 (point-sampled,
 *   unit-sum, box-truncated); the 3-D filter is gxy (x) gxy (x) gz.  The image
 *   is zero outside the cube.  r must not exceed GSF_MAX_RADIUS.
 * Windows.  The statistics window of length B along an axis covers offsets
 *   [-floor(B/2), -floor(B/2) + B - 1] around the voxel, clipped to the cube;
 *   n(v) is the product of the clipped lengths.  Standard deviations are
 *   population values (divide by n).
 * Masks.  One bit per voxel, packed along z: each (x, y) row holds
 *   W = ceil(nz/64) uint64 words, bit j of word w is voxel z = 64*w + j; pad
 *   bits are 0.  Word index of (x, y, w) is (x*ny + y)*W + w.
 */
#ifndef GSF_H
#define GSF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSF_MAX_RADIUS 64     /* largest filter radius r (taps 2r+1 = 129) */
#define GSF_MAX_BOX 4096      /* largest statistics window length per axis */

typedef enum gsf_status {
    GSF_OK = 0,
    GSF_ERR_INVALID_ARG = 1,  /* null/misaligned pointer, bad size, sigma, box, k, overlap */
    GSF_ERR_UNSUPPORTED = 2,  /* valid request the library does not implement */
    GSF_ERR_WORKSPACE = 3,    /* workspace smaller than the *_workspace_size figure */
    GSF_ERR_DEVICE = 4,       /* a HIP call or kernel launch failed */
    GSF_ERR_BUDGET = 5        /* request larger than an imposed memory budget */
} gsf_status;

typedef enum gsf_dtype {
    GSF_F32 = 0,              /* IEEE binary32 */
    GSF_F16 = 1,              /* IEEE binary16, storage only */
    GSF_BF16 = 2              /* bfloat16, storage only */
} gsf_dtype;

typedef struct gsf_dims {
    int64_t nx, ny, nz;       /* x slowest, z contiguous; each >= 1 */
} gsf_dims;

typedef struct gsf_filter {
    double sigma_xy;          /* spatial sigma (x and y), pixels, > 0 */
    double sigma_z;           /* spectral sigma, channels, > 0 */
    double truncate;          /* radius r = ceil(truncate * sigma); 3.0 usual */
} gsf_filter;

typedef struct gsf_box {
    int32_t bx, by, bz;       /* statistics window lengths, 1..GSF_MAX_BOX */
} gsf_box;

typedef struct gsf_cube {
    const void *data;         /* device pointer to the cube */
    gsf_dtype dtype;          /* storage type of data (F32, F16 or BF16) */
    gsf_dims dims;            /* dims of the array at `data` */
    int32_t halo[3];          /* input-only border per side along x, y, z (>= 0) */
} gsf_cube;
/* A cube with a halo is a core of dims - 2*halo voxels surrounded by halo[a]
 * voxels of input on each side of axis a (how a large cube is cut into
 * independently processed sub-cubes, §3.1).  The filter reads the whole array
 * at `data` (zero outside it); F, the local statistics and the mask are
 * produced for the core only, with statistics windows clipped to the core, so
 * every output array of the cube has the core's dims.  halo = 0 is the plain
 * case. */

/* ---- Filtering: Eq. 2 (§2.1), c_u[x][y][z] = sum_o d[x+o_x][y+o_y][z+o_z] f[o] ---- */

/* Bytes of device workspace gsf_filter3d needs for a cube of dims d and
 * filter f.  Pure host computation. */
gsf_status gsf_filter3d_workspace_size(gsf_dims d, const gsf_filter *f, size_t *bytes);

/* out = Eq. 2 applied to `in` with filter *f (zero outside the cube).
 * in, out: nx*ny*nz elements of in_t / out_t, which must be the same type
 * (GSF_F32, GSF_F16 or GSF_BF16; otherwise GSF_ERR_UNSUPPORTED); they must
 * not overlap.  ws: at least gsf_filter3d_workspace_size bytes (may be NULL
 * when that figure is 0).  FP32 arithmetic, taps summed in the fixed order
 * -r..r per axis; the spectral-pass intermediate is FP32 (in ws) whatever
 * the storage type, and a 16-bit output is rounded to nearest even. */
gsf_status gsf_filter3d(const void *in, gsf_dtype in_t, gsf_dims d, const gsf_filter *f,
                        void *out, gsf_dtype out_t, void *ws, size_t ws_bytes, void *stream);

/* ---- Weighted filtering: Eq. 1 (§2.1) ---- */

/* Bytes of device workspace gsf_filter3d_weighted needs.  Pure host. */
gsf_status gsf_filter3d_weighted_workspace_size(gsf_dims d, const gsf_filter *f, size_t *bytes);

/* out = Eq. 1, the weighted convolution of `in` with weights `w`, read as the
 * normalised convolution out = sum(d w f) / sum(w f) over the filter support
 * (zero outside the cube), so that unit weights give Eq. 2 away from the
 * faces; out = 0 where sum(w f) = 0.  in, w, out: nx*ny*nz elements of t
 * (GSF_F32 only; others return GSF_ERR_UNSUPPORTED); none may overlap
 * another or ws.  Computed as Eq. 2 of d*w (FP32 product) over Eq. 2 of w,
 * FP32 arithmetic. */
gsf_status gsf_filter3d_weighted(const void *in, const void *w, gsf_dtype t, gsf_dims d,
                                 const gsf_filter *f, void *out, void *ws, size_t ws_bytes,
                                 void *stream);

/* ---- Local statistics: §3.3, mean and std over a range around each voxel ---- */

/* Bytes of device workspace gsf_local_stats needs.  Pure host computation. */
gsf_status gsf_local_stats_workspace_size(gsf_dims d, gsf_box b, size_t *bytes);

/* mean[v] = (1/n) sum_W F,  stdev[v] = sqrt(max(0, (1/n) sum_W (F-s)^2 - ((1/n) sum_W (F-s))^2))
 * over the clipped window W(v) of box b, s a shift computed on the device
 * from F.  F: nx*ny*nz elements of t (GSF_F32, GSF_F16 or GSF_BF16; 16-bit
 * values are widened exactly).  mean, stdev: nx*ny*nz floats in every case;
 * either may be NULL if not wanted (not both).  The window sums are FP32 or
 * wider whatever t is.  Outputs must not overlap F or each other. */
gsf_status gsf_local_stats(const void *F, gsf_dtype t, gsf_dims d, gsf_box b,
                           float *mean, float *stdev, void *ws, size_t ws_bytes, void *stream);

/* ---- Selection: F > mean + k*std (§1, §3.3) ---- */

/* mask bit of v = F[v] > thr[v], thr = (double)mean[v] + k * (double)stdev[v]
 * evaluated in FP64 with each operation rounded once (no fused multiply-add),
 * comparison strict, F (of type t: GSF_F32, GSF_F16 or GSF_BF16) promoted
 * exactly; mean and stdev are floats.  mask: nx*ny*ceil(nz/64) words
 * (layout above).  Given identical inputs the result is bit-exact. */
gsf_status gsf_threshold(const void *F, gsf_dtype t, const float *mean, const float *stdev,
                         gsf_dims d, double k, uint64_t *mask, void *stream);

/* ---- Library set-up ---- */

/* Create the library's per-device state on the current device, once: the
 * streams a multi-cube gsf_find forks onto and the address of the
 * gsf_find_noalloc scratch.  Optional (they are otherwise set up by the first
 * call that needs them), but required before a graph capture whose first such
 * call is captured: this state is not set up inside a capture (gsf_find and
 * gsf_find_noalloc then return GSF_ERR_UNSUPPORTED).  Idempotent;
 * GSF_ERR_DEVICE if a HIP call fails. */
gsf_status gsf_init(void);

/* ---- The whole path over a batch of cubes and a filter bank ---- */

/* Bytes of device workspace gsf_find needs for this batch: one slot per
 * concurrently processed cube, each sized for the batch's largest array: the
 * FP32 spectral intermediate, one FP32-sized F per filter sharing it (at most
 * 3), two (four if a cube needs the generic statistics path) FP32 cubes of
 * window sums, plus about 0.5 MiB per F; min(ncubes, 32) slots, fewer when
 * that many would exceed 64 GiB (at least one).  Pure host; independent of
 * the tuning. */
gsf_status gsf_find_workspace_size(const gsf_cube *cubes, int32_t ncubes, const gsf_filter *f,
                                   int32_t nfilt, gsf_box b, size_t *bytes);

/* For each cube c and filter j: F = Eq. 2, local mean/std over box b (§3.3),
 * mask = F > mean + k*std, with the same definitions as the three calls
 * above (the mask equals gsf_threshold of the F, mean and std produced here).
 * masks[c*nfilt + j]: mask of cube c, filter j (required).
 * F_out, mean_out, std_out: NULL, or arrays of ncubes*nfilt device pointers
 * (each may be NULL) receiving the filtered cube (in the cube's dtype), local
 * mean and local std (floats).  A cube may be stored as GSF_F32, GSF_F16 or
 * GSF_BF16; F is then stored in that type (the mask is taken from the
 * stored F), while the spectral-pass intermediate and the window sums stay
 * FP32.  ws: at least gsf_find_workspace_size bytes (sized for FP32, enough
 * for every storage type).
 * Cubes are independent: with more than one cube the call forks `stream`
 * into up to 32 library-owned streams (created by gsf_init or on first use
 * per device outside a capture, kept until the process ends, default
 * priority), gives each its own slice of ws,
 * runs the largest cubes first on the least loaded stream, and makes
 * `stream` wait for all of them before returning (also after an error), so
 * the results are ordered on `stream` as for one cube.  Such calls from
 * several host threads are serialized while they enqueue.  Every cube's
 * results are identical to those of a call with that cube alone. */
gsf_status gsf_find(const gsf_cube *cubes, int32_t ncubes, const gsf_filter *f, int32_t nfilt,
                    gsf_box b, double k, uint64_t *const *masks, void *const *F_out,
                    float *const *mean_out, float *const *std_out, void *ws, size_t ws_bytes,
                    void *stream);

/* ---- gsf_find for callers that cannot allocate ---- */

/* Size of the device scratch gsf_find_noalloc works in: a file-scope array of
 * the library, one copy per device, held from the library's first use on that
 * device until the process ends. */
#define GSF_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

/* For callers that cannot allocate device memory (code under graph capture,
 * serving loops, harnesses that forbid hipMalloc): gsf_find with the same
 * arguments, results and definitions, minus the workspace.  The workspace
 * gsf_find would need for ONE slot lives in the library's scratch array
 * instead, and the cubes run one after another on `stream` (no library
 * streams).  The call performs no device allocation or free.
 * Limit: one slot of gsf_find's workspace layout (FP32 spectral
 * intermediate, one FP32-sized F per filter sharing it, two window-sum cubes,
 * shift partials; see gsf_find_workspace_size) must fit in
 * GSF_NOALLOC_SCRATCH_BYTES; otherwise GSF_ERR_BUDGET and nothing is
 * enqueued.  With filters of at most three per sigma_z group that is about
 * 2^23 voxels for the batch's largest array.
 * The scratch is shared by every call on a device and keeps the last call's
 * contents (every scratch byte a call reads is written by that call first):
 * calls that overlap on one device race, so the caller serialises them (one
 * stream, or events).  The scratch address of the current device is looked up
 * by gsf_init or by the first call outside a capture; a first call inside a
 * capture returns GSF_ERR_UNSUPPORTED. */
gsf_status gsf_find_noalloc(const gsf_cube *cubes, int32_t ncubes, const gsf_filter *f,
                            int32_t nfilt, gsf_box b, double k, uint64_t *const *masks,
                            void *const *F_out, float *const *mean_out, float *const *std_out,
                            void *stream);

/* ---- Launch tuning ---- */

/* Launch configuration of the kernels that have several compiled shapes.
 * Every setting gives results within the parity bounds; the filtered values F
 * are bit-identical across settings, the statistics may differ in rounding
 * (a different x split changes the order of the shift's partial sums). */
typedef struct gsf_tuning {
    int32_t merge_sweeps;  /* 1 (default): the filters of a group that shares one
                              spectral pass (equal sigma_z) get one merged spatial
                              sweep where a form is compiled (spatial radii
                              {3,6,12}, {3,6}, {3,12}, {6,12}); 0: one sweep each */
    int32_t merged_shape;  /* merged-sweep block: 0 (default) 1 row per lane x 8
                              waves, 1: 2 rows x 8 waves, 2: 1 row x 16 waves,
                              3: 2 rows x 4 waves */
    int32_t sweep_blocks;  /* blocks a spatial sweep aims for before it splits x
                              into chunks, 64..65536 (default 512) */
    int32_t yz_waves;      /* waves per block of the yz window-sum kernel: 0
                              (default: fewest columns walked for the depth), 3, 5
                              or 9 */
    int32_t pair_spectral; /* 1 (default): two filter groups with different
                              sigma_z whose spectral radii form a compiled pair
                              ({3,6}, {3,12}, {6,12}, {6,24}, {12,24}, {3,24})
                              get both spectral passes from one read of the cube;
                              0: one spectral pass per group */
    int32_t x_exits;       /* 1 (default): the statistics' x walk stops its last
                              ring turn at the first 16-step boundary past the
                              cube (fewer wasted steps, more registers); 0: whole
                              turns */
} gsf_tuning;

/* Size class of a cube core: floor(log2(nx*ny*nz)), 0..40; -1 if invalid. */
int32_t gsf_size_class(gsf_dims core);

/* Set the tuning used for cores of size class `size_class` (-1: every class)
 * stored as `dtype`, by every later call of this process (gsf_filter3d,
 * gsf_filter3d_weighted, gsf_local_stats, gsf_find).  The
 * table is process-wide; calls enqueued concurrently with a change see the
 * old or the new entry.  GSF_ERR_INVALID_ARG for values out of range. */
gsf_status gsf_tuning_set(int32_t size_class, gsf_dtype dtype, const gsf_tuning *cfg);

/* The entry of size class `size_class` (0..40) and `dtype`. */
gsf_status gsf_tuning_get(int32_t size_class, gsf_dtype dtype, gsf_tuning *cfg);

/* Every entry back to the defaults (the values above, except merged_shape 2
 * for FP32 and 3 for 16-bit cores of 2^26 voxels or more). */
gsf_status gsf_tuning_reset(void);

/* ---- Kernel timing (measurement aid) ---- */

/* While enabled (on != 0), every kernel the library enqueues is bracketed by
 * two hipEvents recorded on the stream it runs on, so its duration can be
 * read back afterwards.  Disabled by default; costs two event records per
 * launch when on.  Enabling or disabling does not clear recorded data. */
gsf_status gsf_profile_enable(int on);

/* Drop every recorded launch. */
gsf_status gsf_profile_reset(void);

/* Synchronise the recorded events and aggregate them per kernel name.
 * Returns the number of distinct kernels (0 if nothing was recorded), or -1
 * if a HIP event call failed. */
int32_t gsf_profile_collect(void);

/* Entry i (0 <= i < last collect count) of the aggregate: kernel name
 * (static string), number of launches and summed duration in milliseconds. */
gsf_status gsf_profile_entry(int32_t i, const char **name, int64_t *launches, double *total_ms);

/* ---- Helpers ---- */

/* Number of uint64 mask words for dims d: nx*ny*ceil(nz/64); -1 if invalid. */
int64_t gsf_mask_words(gsf_dims d);

/* Static description of a status code. */
const char *gsf_status_string(gsf_status s);

/* Detail of the last failing call on the calling thread ("" if none). */
const char *gsf_last_error(void);

/* Library version string. */
const char *gsf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GSF_H */
