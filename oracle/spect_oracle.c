/*
 * spect_oracle.c - plain FP64 CPU oracle for the parallel-hole SPECT system
 * matrix of the paper (Section 2.1.1, Eq. 1) and its transpose.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker: the tests, the smoke
 * check and the CPU-baseline leg of the benchmark load it.  The product path
 * (the HIP library) shares no code with it and never links it.
 *
 * What it computes.  Eq. 1 writes the system matrix as one block per gantry
 * angle n:
 *
 *     H_n = T_fov P_x T_cdr T_att T_trans T_rot
 *
 * applied right to left: rotate the object into the frame of angle n, shift it
 * (identity here: the rotation axis is the grid centre), attenuate, blur with
 * the depth-dependent collimator-detector response, sum along the +x axis of
 * the rotated frame (towards the detector) and mask the field of view (all
 * ones here).  The paper says which operations these are (rotation, photon
 * attenuation, depth-dependent blur, summation) but not their discretisation;
 * the readings used here are:
 *
 *   - rotation: bilinear interpolation per axial slice, zero outside the grid,
 *     rotation centre c = (N-1)/2 in index units; rotated-frame sample
 *     (i', j') sits at X = c + cos(t)(i'-c) - sin(t)(j'-c),
 *     Y = c + sin(t)(i'-c) + cos(t)(j'-c); cos/sin are computed in FP64 and
 *     values below 1e-15 in magnitude are set to 0;
 *   - depth axis i' of the rotated frame points at the detector, which lies
 *     beyond i' = N-1 (the "+x" side);
 *   - attenuation: tau(i') = dx * (mu(i')/2 + sum_{i''>i'} mu(i'')) along the
 *     rotated depth axis (half of the emitting voxel plus every voxel between
 *     it and the detector), factor exp(-tau);
 *   - collimator-detector response at depth i': distance to the detector face
 *     d = max(0, R - (i'-c) dx), Gaussian sigma = a d + b (cm), sampled at
 *     integer pixel offsets, truncated at K = ceil(nsig * sigma/dx - 1e-9),
 *     normalised to unit sum, applied along the detector bin axis and the
 *     axial axis with zero padding; sigma <= 0 means no blur;
 *   - summation: plain sum over i' (no path-length factor).
 *
 * Array layouts (C order, last index fastest):
 *   object      f[i][j][k]   shape (N, N, Nz), i = x, j = y, k = z (axial)
 *   projections p[n][r][k]   shape (A, N, Nz), r = detector bin (= j')
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int n;            /* transverse grid size N */
    int nz;           /* axial size Nz */
    int n_angles;     /* A */
    double voxel_cm;  /* isotropic voxel / detector pixel size dx */
    double psf_a;     /* sigma(d) = psf_a * d + psf_b  (cm) */
    double psf_b;
    double psf_nsigma;
} orc_geom;

/* cos and sin of an angle given in degrees, with tiny values set to zero so
 * that multiples of 90 degrees give exact permutations. */
void orc_trig(double deg, double *c, double *s)
{
    double r = fmod(deg, 360.0);
    if (r < 0) r += 360.0;
    double t = r * (M_PI / 180.0);
    double cc = cos(t), ss = sin(t);
    if (fabs(cc) < 1e-15) cc = 0.0;
    if (fabs(ss) < 1e-15) ss = 0.0;
    *c = cc;
    *s = ss;
}

/* Collimator-detector kernel at rotated depth ip for detector radius R_cm.
 * Writes the one-sided taps g[0..K] (g[m] = g[-m]) and returns K. */
int orc_psf_taps(const orc_geom *g, double radius_cm, int ip, double *taps, int max_k)
{
    double c = 0.5 * (g->n - 1);
    double d = radius_cm - (ip - c) * g->voxel_cm;
    if (d < 0) d = 0;
    double sigma_cm = g->psf_a * d + g->psf_b;
    if (!(sigma_cm > 0)) {
        taps[0] = 1.0;
        return 0;
    }
    double s = sigma_cm / g->voxel_cm;
    double nsig = g->psf_nsigma > 0 ? g->psf_nsigma : 4.0;
    int K = (int)ceil(nsig * s - 1e-9);
    if (K < 0) K = 0;
    if (K > max_k) return -1;
    double sum = 0;
    for (int m = -K; m <= K; ++m) sum += exp(-(double)m * m / (2 * s * s));
    for (int m = 0; m <= K; ++m) taps[m] = exp(-(double)m * m / (2 * s * s)) / sum;
    return K;
}

/* T_rot: rotated[i'][j'][k] = bilinear sample of vol at (X, Y), zero outside. */
void orc_rotate(const double *vol, int N, int Nz, double cs, double sn, double *out)
{
    double c = 0.5 * (N - 1);
    for (int ip = 0; ip < N; ++ip)
        for (int jp = 0; jp < N; ++jp) {
            double X = c + cs * (ip - c) - sn * (jp - c);
            double Y = c + sn * (ip - c) + cs * (jp - c);
            double xf = floor(X), yf = floor(Y);
            int x0 = (int)xf, y0 = (int)yf;
            double fx = X - xf, fy = Y - yf;
            double *o = out + ((size_t)ip * N + jp) * Nz;
            for (int k = 0; k < Nz; ++k) o[k] = 0;
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    int x = x0 + a, y = y0 + b;
                    if (x < 0 || x >= N || y < 0 || y >= N) continue;
                    double w = (a ? fx : 1 - fx) * (b ? fy : 1 - fy);
                    const double *v = vol + ((size_t)x * N + y) * Nz;
                    for (int k = 0; k < Nz; ++k) o[k] += w * v[k];
                }
        }
}

/* Transpose of orc_rotate: spreads each rotated-frame value back onto the four
 * object voxels it was interpolated from, with the same weights. */
void orc_rotate_adjoint(const double *rot, int N, int Nz, double cs, double sn, double *out)
{
    double c = 0.5 * (N - 1);
    memset(out, 0, sizeof(double) * (size_t)N * N * Nz);
    for (int ip = 0; ip < N; ++ip)
        for (int jp = 0; jp < N; ++jp) {
            double X = c + cs * (ip - c) - sn * (jp - c);
            double Y = c + sn * (ip - c) + cs * (jp - c);
            double xf = floor(X), yf = floor(Y);
            int x0 = (int)xf, y0 = (int)yf;
            double fx = X - xf, fy = Y - yf;
            const double *r = rot + ((size_t)ip * N + jp) * Nz;
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    int x = x0 + a, y = y0 + b;
                    if (x < 0 || x >= N || y < 0 || y >= N) continue;
                    double w = (a ? fx : 1 - fx) * (b ? fy : 1 - fy);
                    double *o = out + ((size_t)x * N + y) * Nz;
                    for (int k = 0; k < Nz; ++k) o[k] += w * r[k];
                }
        }
}

/* T_att factors exp(-tau) for a rotated attenuation map murot[i'][j'][k]. */
static void attenuation_factors(const double *murot, int N, int Nz, double dx, double *att)
{
    for (int jp = 0; jp < N; ++jp)
        for (int k = 0; k < Nz; ++k) {
            double beyond = 0; /* sum of mu over voxels between i' and the detector */
            for (int ip = N - 1; ip >= 0; --ip) {
                size_t q = ((size_t)ip * N + jp) * Nz + k;
                double tau = dx * (0.5 * murot[q] + beyond);
                att[q] = exp(-tau);
                beyond += murot[q];
            }
        }
}

/* T_cdr on one depth plane w[r][k] (N x Nz): convolution with the separable
 * kernel g(r) g(k), zero padding.  The 2D kernel is the outer product of the
 * 1D taps, so the 2D convolution is a pass along r followed by a pass along k.
 * tmp has N*Nz entries. */
static void blur_plane(const double *w, int N, int Nz, const double *taps, int K,
                       double *tmp, double *out)
{
    for (int r = 0; r < N; ++r)
        for (int k = 0; k < Nz; ++k) {
            double acc = 0;
            for (int m = -K; m <= K; ++m) {
                int rr = r - m;
                if (rr < 0 || rr >= N) continue;
                acc += taps[abs(m)] * w[(size_t)rr * Nz + k];
            }
            tmp[(size_t)r * Nz + k] = acc;
        }
    for (int r = 0; r < N; ++r)
        for (int k = 0; k < Nz; ++k) {
            double acc = 0;
            for (int l = -K; l <= K; ++l) {
                int kk = k - l;
                if (kk < 0 || kk >= Nz) continue;
                acc += taps[abs(l)] * tmp[(size_t)r * Nz + kk];
            }
            out[(size_t)r * Nz + k] = acc;
        }
}

#define ORC_MAXK 256

static double angle_of(const orc_geom *g, const double *angles_deg, int n)
{
    return angles_deg ? angles_deg[n] : n * 360.0 / g->n_angles;
}

static double radius_of(const orc_geom *g, const double *radius_cm, int n)
{
    return radius_cm ? radius_cm[n] : 0.5 * g->n * g->voxel_cm;
}

/* Forward projection H f for the listed angles:
 * proj[n] = P_x T_cdr T_att T_rot f for n in idx.  Other rows of proj are left
 * untouched.  mu may be NULL (no attenuation).  Returns 0, or -1 when a blur
 * radius exceeds the internal limit. */
int orc_forward(const orc_geom *g, const double *angles_deg, const double *radius_cm,
                const double *f, const double *mu, const int *idx, int n_idx, double *proj)
{
    const int N = g->n, Nz = g->nz;
    const size_t vol = (size_t)N * N * Nz, plane = (size_t)N * Nz;
    int status = 0;
#pragma omp parallel
    {
        double *F = malloc(sizeof(double) * vol);
        double *M = mu ? malloc(sizeof(double) * vol) : NULL;
        double *att = mu ? malloc(sizeof(double) * vol) : NULL;
        double *tmp = malloc(sizeof(double) * plane);
        double *B = malloc(sizeof(double) * plane);
        double *Wp = malloc(sizeof(double) * plane);
        double taps[ORC_MAXK + 1];
#pragma omp for schedule(static)
        for (int t = 0; t < n_idx; ++t) {
            int n = idx[t];
            double cs, sn;
            orc_trig(angle_of(g, angles_deg, n), &cs, &sn);
            double R = radius_of(g, radius_cm, n);
            /* T_rot (T_trans is the identity) */
            orc_rotate(f, N, Nz, cs, sn, F);
            /* T_att */
            if (mu) {
                orc_rotate(mu, N, Nz, cs, sn, M);
                attenuation_factors(M, N, Nz, g->voxel_cm, att);
                for (size_t q = 0; q < vol; ++q) F[q] *= att[q];
            }
            /* T_cdr per depth plane, then P_x (sum over depth); T_fov = 1 */
            double *p = proj + (size_t)n * plane;
            for (size_t q = 0; q < plane; ++q) p[q] = 0;
            for (int ip = 0; ip < N; ++ip) {
                int K = orc_psf_taps(g, R, ip, taps, ORC_MAXK);
                if (K < 0) {
#pragma omp atomic write
                    status = -1;
                    continue;
                }
                memcpy(Wp, F + (size_t)ip * plane, sizeof(double) * plane);
                blur_plane(Wp, N, Nz, taps, K, tmp, B);
                for (size_t q = 0; q < plane; ++q) p[q] += B[q];
            }
        }
        free(F); free(M); free(att); free(tmp); free(B); free(Wp);
    }
    return status;
}

/* Back projection: out = sum_{n in idx} H_n^T proj[n]
 *                      = sum_n T_rot^T T_att T_cdr P_x^T proj[n]
 * (T_att is diagonal and the zero-padded symmetric blur is its own transpose).
 * Angles are split statically over threads and the per-thread partial volumes
 * are added in thread order, so the result does not depend on scheduling. */
int orc_back(const orc_geom *g, const double *angles_deg, const double *radius_cm,
             const double *proj, const double *mu, const int *idx, int n_idx, double *out)
{
    const int N = g->n, Nz = g->nz;
    const size_t vol = (size_t)N * N * Nz, plane = (size_t)N * Nz;
    int status = 0;
    int nthr = 1;
#ifdef _OPENMP
#pragma omp parallel
#pragma omp single
    nthr = omp_get_num_threads();
#endif
    double *partial = calloc((size_t)nthr * vol, sizeof(double));
#pragma omp parallel num_threads(nthr)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *acc = partial + (size_t)tid * vol;
        double *Z = malloc(sizeof(double) * vol);
        double *M = mu ? malloc(sizeof(double) * vol) : NULL;
        double *att = mu ? malloc(sizeof(double) * vol) : NULL;
        double *tmp = malloc(sizeof(double) * plane);
        double *obj = malloc(sizeof(double) * vol);
        double taps[ORC_MAXK + 1];
#pragma omp for schedule(static)
        for (int t = 0; t < n_idx; ++t) {
            int n = idx[t];
            double cs, sn;
            orc_trig(angle_of(g, angles_deg, n), &cs, &sn);
            double R = radius_of(g, radius_cm, n);
            const double *y = proj + (size_t)n * plane;
            /* P_x^T: copy the projection to every depth; T_cdr^T = T_cdr */
            for (int ip = 0; ip < N; ++ip) {
                int K = orc_psf_taps(g, R, ip, taps, ORC_MAXK);
                if (K < 0) {
#pragma omp atomic write
                    status = -1;
                    continue;
                }
                blur_plane(y, N, Nz, taps, K, tmp, Z + (size_t)ip * plane);
            }
            /* T_att^T = T_att */
            if (mu) {
                orc_rotate(mu, N, Nz, cs, sn, M);
                attenuation_factors(M, N, Nz, g->voxel_cm, att);
                for (size_t q = 0; q < vol; ++q) Z[q] *= att[q];
            }
            /* T_rot^T */
            orc_rotate_adjoint(Z, N, Nz, cs, sn, obj);
            for (size_t q = 0; q < vol; ++q) acc[q] += obj[q];
        }
        free(Z); free(M); free(att); free(tmp); free(obj);
    }
    for (size_t q = 0; q < vol; ++q) {
        double s = 0;
        for (int t = 0; t < nthr; ++t) s += partial[(size_t)t * vol + q];
        out[q] = s;
    }
    free(partial);
    return status;
}
