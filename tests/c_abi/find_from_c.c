/* A plain C caller of libgsf: only include/gsf.h and the HIP runtime API,
 * no Python and no torch.  It runs gsf_find over one seeded cube with three
 * filters (two spectral-pass groups) and compares every voxel of F, the local
 * mean and std and the masks with the FP64 oracle (test infrastructure, linked
 * only into this test program), to the parity bounds the Python tests use:
 * F within 1e-5 max(|F|, sigma_f rms(d)), mean and std within 1e-5 max(std,
 * sigma_f rms(d)) (plus half an FP32 ulp of the mean), masks equal outside
 * the band those bounds span.  It also checks that invalid arguments are
 * refused before anything is enqueued.  Exit status 0 on success. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "gsf.h"

/* the oracle's C entry points (oracle/oracle_gsf.c) */
int oracle_taps(double sigma, double truncate, double *g, int cap);
int oracle_find(const float *d, int64_t nx, int64_t ny, int64_t nz, const double *sigma_xy,
                const double *sigma_z, const double *truncate, int nfilt, int bx, int by, int bz,
                double k, uint8_t *masks, double *F_out, double *mean_out, double *std_out);

#define NX 40
#define NY 36
#define NZ 150
#define NF 3

static int fails = 0;
#define CHECK(c, ...)                                  \
    do {                                               \
        if (!(c)) {                                    \
            fprintf(stderr, "FAIL: " __VA_ARGS__);     \
            fprintf(stderr, "\n");                     \
            ++fails;                                   \
        }                                              \
    } while (0)
#define HIP(x)                                                                  \
    do {                                                                        \
        hipError_t e_ = (x);                                                    \
        if (e_ != hipSuccess) {                                                 \
            fprintf(stderr, "HIP error %s at %s\n", hipGetErrorString(e_), #x); \
            return 2;                                                           \
        }                                                                       \
    } while (0)

/* xorshift64*: seeded uniform noise in [-1, 1) plus a few bright blobs */
static uint64_t state = 0x9E3779B97F4A7C15ull;
static double uniform(void)
{
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return (double)((state * 0x2545F4914F6CDD1Dull) >> 11) / 9007199254740992.0 * 2.0 - 1.0;
}

static double sumsq_taps(double sigma)
{
    double g[128];
    const int r = oracle_taps(sigma, 3.0, g, 128);
    double s = 0.0;
    for (int i = 0; i <= 2 * r; ++i) s += g[i] * g[i];
    return s;
}

int main(void)
{
    const int64_t V = (int64_t)NX * NY * NZ;
    const int64_t W = (NZ + 63) / 64;
    const gsf_filter filt[NF] = {{1.0, 2.0, 3.0}, {2.0, 8.0, 3.0}, {4.0, 2.0, 3.0}};
    const gsf_box box = {16, 16, 32};
    const double k = 4.0;
    float *d = (float *)malloc(sizeof(float) * (size_t)V);
    for (int64_t i = 0; i < V; ++i) d[i] = (float)uniform();
    for (int b = 0; b < 4; ++b) { /* bright compact blobs */
        const int x0 = 5 + 9 * b, y0 = 4 + 8 * b, z0 = 20 + 30 * b;
        for (int x = x0 - 2; x <= x0 + 2; ++x)
            for (int y = y0 - 2; y <= y0 + 2; ++y)
                for (int z = z0 - 6; z <= z0 + 6; ++z)
                    d[((int64_t)x * NY + y) * NZ + z] += 3.0f;
    }
    double rms = 0.0;
    for (int64_t i = 0; i < V; ++i) rms += (double)d[i] * d[i];
    rms = sqrt(rms / (double)V);

    /* device buffers */
    void *dd = NULL, *ws = NULL;
    uint64_t *dm[NF];
    float *dF[NF], *dmu[NF], *dsd[NF];
    HIP(hipMalloc(&dd, sizeof(float) * (size_t)V));
    HIP(hipMemcpy(dd, d, sizeof(float) * (size_t)V, hipMemcpyHostToDevice));
    for (int j = 0; j < NF; ++j) {
        HIP(hipMalloc((void **)&dm[j], sizeof(uint64_t) * (size_t)(NX * NY * W)));
        HIP(hipMalloc((void **)&dF[j], sizeof(float) * (size_t)V));
        HIP(hipMalloc((void **)&dmu[j], sizeof(float) * (size_t)V));
        HIP(hipMalloc((void **)&dsd[j], sizeof(float) * (size_t)V));
    }
    gsf_cube cube;
    memset(&cube, 0, sizeof cube);
    cube.data = dd;
    cube.dtype = GSF_F32;
    cube.dims.nx = NX;
    cube.dims.ny = NY;
    cube.dims.nz = NZ;
    CHECK(gsf_init() == GSF_OK, "gsf_init: %s", gsf_last_error());
    size_t need = 0;
    CHECK(gsf_find_workspace_size(&cube, 1, filt, NF, box, &need) == GSF_OK && need > 0,
          "workspace size: %s", gsf_last_error());
    HIP(hipMalloc(&ws, need));

    /* refused arguments: nothing is enqueued, the status says why */
    uint64_t *const *masks = (uint64_t *const *)dm;
    CHECK(gsf_find(&cube, 0, filt, NF, box, k, masks, NULL, NULL, NULL, ws, need, NULL) ==
              GSF_ERR_INVALID_ARG && strlen(gsf_last_error()) > 0,
          "zero cubes accepted");
    CHECK(gsf_find(&cube, 1, filt, NF, box, k, masks, NULL, NULL, NULL, ws, need - 1, NULL) ==
              GSF_ERR_WORKSPACE,
          "short workspace accepted");
    CHECK(strlen(gsf_status_string(GSF_ERR_BUDGET)) > 0, "status string");

    const gsf_status st = gsf_find(&cube, 1, filt, NF, box, k, masks, (void *const *)dF,
                                   (float *const *)dmu, (float *const *)dsd, ws, need, NULL);
    CHECK(st == GSF_OK, "gsf_find: %s", gsf_last_error());
    HIP(hipDeviceSynchronize());

    /* the oracle on the same host cube */
    double sxy[NF], sz[NF], tr[NF];
    for (int j = 0; j < NF; ++j) sxy[j] = filt[j].sigma_xy, sz[j] = filt[j].sigma_z, tr[j] = 3.0;
    uint8_t *om = (uint8_t *)malloc((size_t)(NF * V));
    double *oF = (double *)malloc(sizeof(double) * (size_t)(NF * V));
    double *omu = (double *)malloc(sizeof(double) * (size_t)(NF * V));
    double *osd = (double *)malloc(sizeof(double) * (size_t)(NF * V));
    CHECK(oracle_find(d, NX, NY, NZ, sxy, sz, tr, NF, box.bx, box.by, box.bz, k, om, oF, omu, osd) ==
              0,
          "oracle");

    float *hF = (float *)malloc(sizeof(float) * (size_t)V);
    float *hmu = (float *)malloc(sizeof(float) * (size_t)V);
    float *hsd = (float *)malloc(sizeof(float) * (size_t)V);
    uint64_t *hm = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(NX * NY * W));
    int64_t total = 0;
    for (int j = 0; j < NF; ++j) {
        HIP(hipMemcpy(hF, dF[j], sizeof(float) * (size_t)V, hipMemcpyDeviceToHost));
        HIP(hipMemcpy(hmu, dmu[j], sizeof(float) * (size_t)V, hipMemcpyDeviceToHost));
        HIP(hipMemcpy(hsd, dsd[j], sizeof(float) * (size_t)V, hipMemcpyDeviceToHost));
        HIP(hipMemcpy(hm, dm[j], sizeof(uint64_t) * (size_t)(NX * NY * W), hipMemcpyDeviceToHost));
        const double sxy2 = sumsq_taps(filt[j].sigma_xy);
        const double sf = sqrt(sxy2 * sxy2 * sumsq_taps(filt[j].sigma_z)) * rms;
        double wf = 0.0, ws_ = 0.0;
        int64_t sel = 0, osel = 0, band = 0, bad = 0;
        for (int64_t i = 0; i < V; ++i) {
            const double Fo = oF[j * V + i], mo = omu[j * V + i], so = osd[j * V + i];
            const double eF = 1e-5 * fmax(fabs(Fo), sf);
            const double es = 1e-5 * fmax(so, sf);
            const double em = es + ldexp(fabs(mo), -24);
            wf = fmax(wf, fabs((double)hF[i] - Fo) / eF);
            ws_ = fmax(ws_, fmax(fabs((double)hmu[i] - mo) / em, fabs((double)hsd[i] - so) / es));
            const int64_t row = i / NZ, z = i % NZ;
            const int bit = (int)((hm[row * W + z / 64] >> (z % 64)) & 1u);
            sel += bit;
            osel += om[j * V + i];
            const double thr = mo + k * so;
            const int inband = fabs(Fo - thr) <= eF + em + k * es;
            band += inband;
            if (!inband && bit != (int)om[j * V + i]) ++bad;
        }
        CHECK(wf <= 1.0, "filter %d: F error %.3g x bound", j, wf);
        CHECK(ws_ <= 1.0, "filter %d: mean/std error %.3g x bound", j, ws_);
        CHECK(bad == 0, "filter %d: %lld mask voxels differ outside the band", j, (long long)bad);
        total += sel;
        printf("filter (%g, %g): F/bound %.3g, stats/bound %.3g, selected %lld (oracle %lld), "
               "band %lld\n",
               filt[j].sigma_xy, filt[j].sigma_z, wf, ws_, (long long)sel, (long long)osel,
               (long long)band);
    }
    CHECK(total > 0, "no filter selected anything");
    if (fails == 0) printf("c consumer ok: %s\n", gsf_version());
    return fails ? 1 : 0;
}
