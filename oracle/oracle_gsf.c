/*
 * oracle_gsf.c -- plain, slow, FP64 CPU oracle for the Gaussian source-finder
 * hot path (Westerlund & Harris, "Performance Analysis of GPU-Accelerated
 * Filter-Based Source Finding for HI Spectral Line Image Data").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code with the HIP path.
 *
 * What it computes, and where each step comes from:
 *   - filter taps: a sampled, unit-sum Gaussian per axis, truncated at
 *     r = ceil(truncate * sigma)  (§2.1: Gaussian filters of radius r_x, r_y,
 *     r_z; the value of r, sampling and normalisation are readings, see the
 *     design notes);
 *   - the unweighted convolution c_u of Eq. 2 (§2.1, with the index ranges of
 *     Eqs. 3-5) with the image taken as zero outside the cube; computed both
 *     directly (the triple sum, `oracle_filter3d_direct*`) and as three 1-D
 *     passes (`oracle_filter3d`), which is the same sum regrouped because the
 *     3-D Gaussian is the outer product of its axis kernels;
 *   - the per-voxel local mean and standard deviation of the filtered cube
 *     over a user-given range around each voxel (§3.3), computed as the
 *     paper describes it: three directional sums (z, then y, then x);
 *     `oracle_local_stats_at` is the plain two-pass definition per voxel;
 *   - the detection threshold mean + k*std and the voxel selection F > thr
 *     (§1 and §3.3: local mean and deviation make the thresholds).
 *
 * All arithmetic is FP64; FP32 inputs are promoted exactly.  Build with
 * -ffp-contract=off so that mean + k*std is rounded twice, as written.
 *
 * Cube layout: x slowest, z (spectral) contiguous, linear index
 * (x*ny + y)*nz + z (§3.1: X major axis, Z minor axis).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORACLE_MAX_TAPS 1025

void oracle_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int oracle_get_threads(void) { return omp_get_max_threads(); }

/* Radius of a truncated Gaussian: r = ceil(truncate * sigma), in FP64. */
int oracle_radius(double sigma, double truncate)
{
    return (int)ceil(truncate * sigma);
}

/* Sampled Gaussian taps g[o + r] = exp(-o^2 / (2 sigma^2)) / sum, o in [-r, r].
 * Returns r, or -1 if 2r+1 exceeds cap or sigma is not positive. */
int oracle_taps(double sigma, double truncate, double *g, int cap)
{
    if (!(sigma > 0.0) || !(truncate > 0.0)) return -1;
    int r = oracle_radius(sigma, truncate);
    if (2 * r + 1 > cap) return -1;
    double sum = 0.0;
    for (int o = -r; o <= r; ++o) {
        double v = exp(-((double)o * (double)o) / (2.0 * sigma * sigma));
        g[o + r] = v;
        sum += v;
    }
    for (int i = 0; i < 2 * r + 1; ++i) g[i] /= sum;
    return r;
}

/* Eq. 2 at one voxel: the triple sum over the filter support of
 * d[x+ox][y+oy][z+oz] * f[ox][oy][oz], f = gxy (x) gxy (x) gz, d = 0 outside. */
static double conv_at(const float *d, int64_t nx, int64_t ny, int64_t nz,
                      const double *gxy, int rxy, const double *gz, int rz,
                      int64_t x, int64_t y, int64_t z)
{
    double c = 0.0;
    for (int ox = -rxy; ox <= rxy; ++ox) {
        int64_t ix = x + ox;
        for (int oy = -rxy; oy <= rxy; ++oy) {
            int64_t iy = y + oy;
            for (int oz = -rz; oz <= rz; ++oz) {
                int64_t iz = z + oz;
                double dv = 0.0;
                if (ix >= 0 && ix < nx && iy >= 0 && iy < ny && iz >= 0 && iz < nz)
                    dv = (double)d[(ix * ny + iy) * nz + iz];
                double f = gxy[ox + rxy] * gxy[oy + rxy] * gz[oz + rz];
                c += dv * f;
            }
        }
    }
    return c;
}

/* Eq. 2 evaluated directly at the listed linear voxel indices. */
int oracle_filter3d_direct_at(const float *d, int64_t nx, int64_t ny, int64_t nz,
                              double sigma_xy, double sigma_z, double truncate,
                              const int64_t *idx, int64_t nidx, double *out)
{
    double gxy[ORACLE_MAX_TAPS], gz[ORACLE_MAX_TAPS];
    int rxy = oracle_taps(sigma_xy, truncate, gxy, ORACLE_MAX_TAPS);
    int rz = oracle_taps(sigma_z, truncate, gz, ORACLE_MAX_TAPS);
    if (rxy < 0 || rz < 0) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nidx; ++i) {
        int64_t v = idx[i];
        int64_t z = v % nz, y = (v / nz) % ny, x = v / (nz * ny);
        out[i] = conv_at(d, nx, ny, nz, gxy, rxy, gz, rz, x, y, z);
    }
    return 0;
}

/* Eq. 2 evaluated directly at every voxel (small cubes only). */
int oracle_filter3d_direct(const float *d, int64_t nx, int64_t ny, int64_t nz,
                           double sigma_xy, double sigma_z, double truncate, double *F)
{
    double gxy[ORACLE_MAX_TAPS], gz[ORACLE_MAX_TAPS];
    int rxy = oracle_taps(sigma_xy, truncate, gxy, ORACLE_MAX_TAPS);
    int rz = oracle_taps(sigma_z, truncate, gz, ORACLE_MAX_TAPS);
    if (rxy < 0 || rz < 0) return -1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t x = 0; x < nx; ++x)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t z = 0; z < nz; ++z)
                F[(x * ny + y) * nz + z] = conv_at(d, nx, ny, nz, gxy, rxy, gz, rz, x, y, z);
    return 0;
}

/* Eq. 2 as three 1-D passes (z, then y, then x), each a sum over the taps in
 * order -r..r with zero outside the cube.  The triple sum factorises because
 * f[ox][oy][oz] = gxy[ox] * gxy[oy] * gz[oz]. */
/* Eq. 2 as z, y and x passes over an FP64 input array (zero outside). */
static int filter3d_f64(const double *d, int64_t nx, int64_t ny, int64_t nz, double sigma_xy,
                        double sigma_z, double truncate, double *F)
{
    double gxy[ORACLE_MAX_TAPS], gz[ORACLE_MAX_TAPS];
    int rxy = oracle_taps(sigma_xy, truncate, gxy, ORACLE_MAX_TAPS);
    int rz = oracle_taps(sigma_z, truncate, gz, ORACLE_MAX_TAPS);
    if (rxy < 0 || rz < 0) return -1;
    const int64_t plane = ny * nz;
    double *T = (double *)malloc(sizeof(double) * (size_t)(nx * plane));
    if (!T) return -2;

    /* z pass: d -> F (F used as the first temporary) */
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t x = 0; x < nx; ++x)
        for (int64_t y = 0; y < ny; ++y) {
            const double *row = d + (x * ny + y) * nz;
            double *o = F + (x * ny + y) * nz;
            for (int64_t z = 0; z < nz; ++z) {
                double c = 0.0;
                for (int oz = -rz; oz <= rz; ++oz) {
                    int64_t iz = z + oz;
                    if (iz >= 0 && iz < nz) c += row[iz] * gz[oz + rz];
                }
                o[z] = c;
            }
        }

    /* y pass: F -> T */
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t x = 0; x < nx; ++x)
        for (int64_t y = 0; y < ny; ++y) {
            double *o = T + (x * ny + y) * nz;
            for (int64_t z = 0; z < nz; ++z) o[z] = 0.0;
            for (int oy = -rxy; oy <= rxy; ++oy) {
                int64_t iy = y + oy;
                if (iy < 0 || iy >= ny) continue;
                const double *src = F + (x * ny + iy) * nz;
                const double g = gxy[oy + rxy];
                for (int64_t z = 0; z < nz; ++z) o[z] += src[z] * g;
            }
        }

    /* x pass: T -> F */
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t x = 0; x < nx; ++x)
        for (int64_t y = 0; y < ny; ++y) {
            double *o = F + (x * ny + y) * nz;
            for (int64_t z = 0; z < nz; ++z) o[z] = 0.0;
            for (int ox = -rxy; ox <= rxy; ++ox) {
                int64_t ix = x + ox;
                if (ix < 0 || ix >= nx) continue;
                const double *src = T + (ix * ny + y) * nz;
                const double g = gxy[ox + rxy];
                for (int64_t z = 0; z < nz; ++z) o[z] += src[z] * g;
            }
        }
    free(T);
    return 0;
}

/* Eq. 2 of an FP32 cube: the values promoted exactly to FP64. */
int oracle_filter3d(const float *d, int64_t nx, int64_t ny, int64_t nz,
                    double sigma_xy, double sigma_z, double truncate, double *F)
{
    const int64_t n = nx * ny * nz;
    double *D = (double *)malloc(sizeof(double) * (size_t)n);
    if (!D) return -2;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) D[i] = (double)d[i];
    int rc = filter3d_f64(D, nx, ny, nz, sigma_xy, sigma_z, truncate, F);
    free(D);
    return rc;
}

/* Eq. 1, the weighted convolution, read as a normalised convolution:
 * F = sum(d w f) / sum(w f) over the filter support (zero outside the cube),
 * i.e. Eq. 2 of the product d*w over Eq. 2 of w; F = 0 where the denominator
 * is 0.  The products of the FP32 inputs are exact in FP64. */
int oracle_filter3d_weighted(const float *d, const float *w, int64_t nx, int64_t ny, int64_t nz,
                             double sigma_xy, double sigma_z, double truncate, double *F)
{
    const int64_t n = nx * ny * nz;
    double *P = (double *)malloc(sizeof(double) * (size_t)n);
    double *W = (double *)malloc(sizeof(double) * (size_t)n);
    double *den = (double *)malloc(sizeof(double) * (size_t)n);
    int rc = (P && W && den) ? 0 : -2;
    if (!rc) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            P[i] = (double)d[i] * (double)w[i];
            W[i] = (double)w[i];
        }
        rc = filter3d_f64(P, nx, ny, nz, sigma_xy, sigma_z, truncate, F);
        if (!rc) rc = filter3d_f64(W, nx, ny, nz, sigma_xy, sigma_z, truncate, den);
        if (!rc) {
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) F[i] = den[i] != 0.0 ? F[i] / den[i] : 0.0;
        }
    }
    free(P);
    free(W);
    free(den);
    return rc;
}

static int64_t window(int64_t i, int64_t n, int B, int64_t *a, int64_t *b)
{
    int64_t lo = i - (int64_t)(B / 2);
    int64_t hi = lo + B;              /* exclusive */
    if (lo < 0) lo = 0;
    if (hi > n) hi = n;
    *a = lo;
    *b = hi;
    return hi > lo ? hi - lo : 0;
}

/* One directional window sum along z, in place, using prefix sums of each row. */
static void dirsum_z(double *A, int64_t nx, int64_t ny, int64_t nz, int B)
{
#pragma omp parallel
    {
        double *P = (double *)malloc(sizeof(double) * (size_t)(nz + 1));
#pragma omp for collapse(2) schedule(static)
        for (int64_t x = 0; x < nx; ++x)
            for (int64_t y = 0; y < ny; ++y) {
                double *row = A + (x * ny + y) * nz;
                P[0] = 0.0;
                for (int64_t z = 0; z < nz; ++z) P[z + 1] = P[z] + row[z];
                for (int64_t z = 0; z < nz; ++z) {
                    int64_t a, b;
                    window(z, nz, B, &a, &b);
                    row[z] = P[b] - P[a];
                }
            }
        free(P);
    }
}

/* Directional window sum along y, in place (prefix over rows of one x-plane). */
static void dirsum_y(double *A, int64_t nx, int64_t ny, int64_t nz, int B)
{
#pragma omp parallel
    {
        double *P = (double *)malloc(sizeof(double) * (size_t)((ny + 1) * nz));
#pragma omp for schedule(static)
        for (int64_t x = 0; x < nx; ++x) {
            double *pl = A + x * ny * nz;
            for (int64_t z = 0; z < nz; ++z) P[z] = 0.0;
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t z = 0; z < nz; ++z)
                    P[(y + 1) * nz + z] = P[y * nz + z] + pl[y * nz + z];
            for (int64_t y = 0; y < ny; ++y) {
                int64_t a, b;
                window(y, ny, B, &a, &b);
                for (int64_t z = 0; z < nz; ++z)
                    pl[y * nz + z] = P[b * nz + z] - P[a * nz + z];
            }
        }
        free(P);
    }
}

/* Directional window sum along x, in place (prefix over x for one y at a time). */
static void dirsum_x(double *A, int64_t nx, int64_t ny, int64_t nz, int B)
{
#pragma omp parallel
    {
        double *P = (double *)malloc(sizeof(double) * (size_t)((nx + 1) * nz));
#pragma omp for schedule(static)
        for (int64_t y = 0; y < ny; ++y) {
            for (int64_t z = 0; z < nz; ++z) P[z] = 0.0;
            for (int64_t x = 0; x < nx; ++x)
                for (int64_t z = 0; z < nz; ++z)
                    P[(x + 1) * nz + z] = P[x * nz + z] + A[(x * ny + y) * nz + z];
            for (int64_t x = 0; x < nx; ++x) {
                int64_t a, b;
                window(x, nx, B, &a, &b);
                for (int64_t z = 0; z < nz; ++z)
                    A[(x * ny + y) * nz + z] = P[b * nz + z] - P[a * nz + z];
            }
        }
        free(P);
    }
}

/* Mean of a cube, summed per x-plane in parallel and then plane by plane in
 * order, so the result does not depend on the thread count. */
double oracle_cube_mean(const double *F, int64_t nx, int64_t ny, int64_t nz)
{
    double *ps = (double *)malloc(sizeof(double) * (size_t)nx);
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < nx; ++x) {
        double s = 0.0;
        const double *pl = F + x * ny * nz;
        for (int64_t i = 0; i < ny * nz; ++i) s += pl[i];
        ps[x] = s;
    }
    double s = 0.0;
    for (int64_t x = 0; x < nx; ++x) s += ps[x];
    free(ps);
    return s / (double)(nx * ny * nz);
}

/* Per-voxel local mean and (population) standard deviation of F over the box
 * window around each voxel, clipped at the cube faces (§3.3).  The sums are
 * three directional sums (z, y, x) of F - s and (F - s)^2, with s the mean of
 * the whole cube; s only changes rounding, since the window mean and variance
 * do not depend on it.  mean = s + S1/n, var = max(0, S2/n - (S1/n)^2). */
int oracle_local_stats(const double *F, int64_t nx, int64_t ny, int64_t nz,
                       int bx, int by, int bz, double *mean, double *stdev)
{
    if (bx < 1 || by < 1 || bz < 1) return -1;
    const int64_t V = nx * ny * nz;
    double s = oracle_cube_mean(F, nx, ny, nz);
    double *A1 = (double *)malloc(sizeof(double) * (size_t)V);
    double *A2 = (double *)malloc(sizeof(double) * (size_t)V);
    if (!A1 || !A2) { free(A1); free(A2); return -2; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < V; ++i) {
        double a = F[i] - s;
        A1[i] = a;
        A2[i] = a * a;
    }
    dirsum_z(A1, nx, ny, nz, bz); dirsum_z(A2, nx, ny, nz, bz);
    dirsum_y(A1, nx, ny, nz, by); dirsum_y(A2, nx, ny, nz, by);
    dirsum_x(A1, nx, ny, nz, bx); dirsum_x(A2, nx, ny, nz, bx);
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t x = 0; x < nx; ++x)
        for (int64_t y = 0; y < ny; ++y) {
            int64_t a, b;
            int64_t cx = window(x, nx, bx, &a, &b);
            int64_t cy = window(y, ny, by, &a, &b);
            for (int64_t z = 0; z < nz; ++z) {
                int64_t cz = window(z, nz, bz, &a, &b);
                double n = (double)(cx * cy * cz);
                int64_t i = (x * ny + y) * nz + z;
                double m1 = A1[i] / n;
                double var = A2[i] / n - m1 * m1;
                if (var < 0.0) var = 0.0;
                mean[i] = s + m1;
                stdev[i] = sqrt(var);
            }
        }
    free(A1);
    free(A2);
    return 0;
}

/* The plain definition at listed voxels: mean = sum(F over W)/n, then
 * var = sum((F - mean)^2 over W)/n, two passes over the clipped window W. */
int oracle_local_stats_at(const double *F, int64_t nx, int64_t ny, int64_t nz,
                          int bx, int by, int bz, const int64_t *idx, int64_t nidx,
                          double *mean, double *stdev)
{
    if (bx < 1 || by < 1 || bz < 1) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nidx; ++i) {
        int64_t v = idx[i];
        int64_t z = v % nz, y = (v / nz) % ny, x = v / (nz * ny);
        int64_t x0, x1, y0, y1, z0, z1;
        int64_t cx = window(x, nx, bx, &x0, &x1);
        int64_t cy = window(y, ny, by, &y0, &y1);
        int64_t cz = window(z, nz, bz, &z0, &z1);
        double n = (double)(cx * cy * cz);
        double s = 0.0;
        for (int64_t a = x0; a < x1; ++a)
            for (int64_t b = y0; b < y1; ++b)
                for (int64_t c = z0; c < z1; ++c) s += F[(a * ny + b) * nz + c];
        double mu = s / n;
        double q = 0.0;
        for (int64_t a = x0; a < x1; ++a)
            for (int64_t b = y0; b < y1; ++b)
                for (int64_t c = z0; c < z1; ++c) {
                    double e = F[(a * ny + b) * nz + c] - mu;
                    q += e * e;
                }
        mean[i] = mu;
        stdev[i] = sqrt(q / n);
    }
    return 0;
}

/* Voxel selection: out[i] = F[i] > mean[i] + k * stdev[i] (strict), FP64. */
void oracle_threshold(const double *F, const double *mean, const double *stdev,
                      int64_t n, double k, uint8_t *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double thr = mean[i] + k * stdev[i];
        out[i] = (uint8_t)(F[i] > thr);
    }
}

/* The same selection on FP32 inputs, each promoted exactly to FP64 first. */
void oracle_threshold_f32(const float *F, const float *mean, const float *stdev,
                          int64_t n, double k, uint8_t *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double thr = (double)mean[i] + k * (double)stdev[i];
        out[i] = (uint8_t)((double)F[i] > thr);
    }
}

/* The whole path for one cube and a bank of filters: for each filter,
 * F = Eq. 2, then local mean/std (§3.3), then the selection mask.
 * masks: nfilt * V bytes.  F_out, mean_out, std_out: nfilt * V doubles each,
 * or NULL when not wanted. */
int oracle_find(const float *d, int64_t nx, int64_t ny, int64_t nz,
                const double *sigma_xy, const double *sigma_z, const double *truncate,
                int nfilt, int bx, int by, int bz, double k,
                uint8_t *masks, double *F_out, double *mean_out, double *std_out)
{
    const int64_t V = nx * ny * nz;
    double *F = NULL, *mu = NULL, *sd = NULL;
    int rc = 0;
    if (!F_out) F = (double *)malloc(sizeof(double) * (size_t)V);
    if (!mean_out) mu = (double *)malloc(sizeof(double) * (size_t)V);
    if (!std_out) sd = (double *)malloc(sizeof(double) * (size_t)V);
    for (int j = 0; j < nfilt && rc == 0; ++j) {
        double *Fj = F_out ? F_out + (int64_t)j * V : F;
        double *mj = mean_out ? mean_out + (int64_t)j * V : mu;
        double *sj = std_out ? std_out + (int64_t)j * V : sd;
        if (!Fj || !mj || !sj) { rc = -2; break; }
        rc = oracle_filter3d(d, nx, ny, nz, sigma_xy[j], sigma_z[j], truncate[j], Fj);
        if (rc) break;
        rc = oracle_local_stats(Fj, nx, ny, nz, bx, by, bz, mj, sj);
        if (rc) break;
        oracle_threshold(Fj, mj, sj, V, k, masks + (int64_t)j * V);
    }
    free(F);
    free(mu);
    free(sd);
    return rc;
}
