/*
 * srwcr_oracle.c -- plain, slow FP64 CPU oracle for the spatially
 * region-weighted correlation ratio (SRWCR) of Gong et al. (arXiv 1804.05061)
 * and its gradient with respect to cubic B-spline FFD displacements.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file.  The HIP product path shares no
 * code, header, table or helper with it, and never calls it.
 *
 * Every step is the paper's definition written out in double precision:
 *   - intensities normalised to [0, L]                      (Sec. II)
 *   - FFD T(x; Phi), node indexing and B-spline pieces      (Sec. II, eqs 8, 17)
 *   - backward warping of M by trilinear interpolation      (Sec. II-F; reading)
 *   - Parzen window h                                       (eq 5)
 *   - cubic B-spline spatial distribution w(r, x)           (eqs 7, 8)
 *   - full 3-D joint PDF p(a, b, r) and Z                   (eqs 3, 4)
 *   - SRWCR by the Table I loop, and by eqs 9, 11, 12       (Sec. II-D)
 *   - dD/dM by the triple sums of eq 19 (M is B) and eq 21 (M is A),
 *     and, as a second form, by eqs 18 / 20 built from dp/dM of eq 26
 *   - chain rule to the control points                      (eqs 16, 17)
 *   - or, for a dense displacement field, dD/du(x) per voxel  (eq 16)
 *   - RaPTOR (boxcar patches, linear window, frequency moments) and its
 *     gradient, the paper's comparison metric                (eqs 6, 13, 14)
 * The joint PDF is kept literally: R x (L+1) x (L+1) doubles.  Per voxel only
 * the bins where h (or h') can be non-zero are visited, which is exact.
 *
 * Readings where the paper is silent (listed with reasons in the design notes):
 *   - normalisation: linear min-max, evaluated in the IEEE single precision
 *     operations s = fl(fl(I - lo) * fl(L / (hi - lo))), clamped to [0, L];
 *   - spatial lattice: K nodes per axis, spacing (N-1)/(K-3), node j at
 *     (j-1)*spacing;  K == 1 on all axes selects one constant region (test);
 *   - moving sample: trilinear, coordinates clamped to [0, M-1] per axis,
 *     gradient 0 along a clamped axis; grids of other size are mapped by
 *     y = (T + 1/2) * M / N - 1/2;
 *   - derivative of h at its kinks: one-sided, the side that corresponds to
 *     increasing the sample (left derivative in kappa), inward at s = L;
 *   - an empty intensity bin (no mass in region r) contributes nothing; in
 *     eq 21 its conditional mean is the voxel's own B-moment (the one-sided
 *     limit), so that its squared deviation vanishes;
 *   - a region with p(r) == 0, or whose B variance is at most 1e-5 of its
 *     second moment (sigma_r^2 <= 1e-5 E_r[b^2], B constant to 0.3 %),
 *     contributes nothing.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int nf[3];      /* fixed grid (x, y, z), x fastest */
    int nm[3];      /* moving grid */
    int n_bins;     /* L_eps + 1 */
    int K[3];       /* spatial bins per axis (1,1,1 = one constant region) */
    int delta[3];   /* FFD control spacing in fixed voxels */
    int role;       /* 0: the moving image is A (model); 1: it is B (estimated) */
    int dense;      /* 0: displacements are FFD coefficients (eq 17); 1: a dense field
                       u[3][nz][ny][nx] on the fixed grid, T(x) = x + u(x) */
    int at_nodes;   /* 1: the regions are the FFD nodes (the paper's setting, Sec. II-C):
                       K = n_c per axis, spacing delta, cell floor(x / delta) */
} orc_problem;

#define VAR_REL 1e-5   /* degenerate region: sigma_r^2 <= VAR_REL * E_r[b^2] */

/* ---------------------------------------------------------------- eq (5) */
double orc_h(double t)
{
    double u = fabs(t);
    if (u < 0.5) return -1.8 * u * u - 0.1 * u + 1.0;
    if (u < 1.0) return 1.8 * u * u - 3.7 * u + 1.9;
    return 0.0;
}

/* dh/dkappa.  side < 0: left derivative (piece on (k - eps, k]);
 * side > 0: right derivative (piece on [k, k + eps)). */
double orc_dh(double k, int side)
{
    if (side < 0) {
        if (k <= -1.0) return 0.0;
        if (k <= -0.5) return 3.6 * k + 3.7;
        if (k <= 0.0) return -3.6 * k + 0.1;
        if (k <= 0.5) return -3.6 * k - 0.1;
        if (k <= 1.0) return 3.6 * k - 3.7;
        return 0.0;
    }
    if (k < -1.0) return 0.0;
    if (k < -0.5) return 3.6 * k + 3.7;
    if (k < 0.0) return -3.6 * k + 0.1;
    if (k < 0.5) return -3.6 * k - 0.1;
    if (k < 1.0) return 3.6 * k - 3.7;
    return 0.0;
}

/* ---------------------------------------------------------------- eq (8) */
double orc_beta(int l, double t)
{
    switch (l) {
    case 0: return (1.0 - t) * (1.0 - t) * (1.0 - t) / 6.0;
    case 1: return (3.0 * t * t * t - 6.0 * t * t + 4.0) / 6.0;
    case 2: return (-3.0 * t * t * t + 3.0 * t * t + 3.0 * t + 1.0) / 6.0;
    case 3: return t * t * t / 6.0;
    }
    return 0.0;
}

/* ------------------------------------------- Sec. II: normalise to [0, L] */
void orc_normalize(const float *in, long n, double lo, double hi, int n_bins, float *out)
{
    float lo_f = (float)lo;
    float scale_f = (float)((double)(n_bins - 1) / (hi - lo));
    float L = (float)(n_bins - 1);
    for (long i = 0; i < n; ++i) {
        float d = in[i] - lo_f;      /* one IEEE single subtraction */
        float s = d * scale_f;       /* one IEEE single multiplication */
        if (s < 0.0f) s = 0.0f;
        if (s > L) s = L;
        out[i] = s;
    }
}

/* ------------------------------------------------- control grid (eq 17) */
void orc_ctrl_dims(const orc_problem *P, int nc[3])
{
    for (int e = 0; e < 3; ++e) nc[e] = (P->nf[e] - 1) / P->delta[e] + 4;
}

/* ------------------------------------- spatial weights w(r, x), eqs (7, 8)
 * Weights of the K nodes of one axis at voxel coordinate x in [0, N-1]. */
void orc_axis_region_weights(int x, int N, int K, double *w)
{
    for (int j = 0; j < K; ++j) w[j] = 0.0;
    if (K == 1) { w[0] = 1.0; return; }
    long num = (long)x * (long)(K - 3);
    int c = (int)(num / (long)(N - 1));
    if (c > K - 4) c = K - 4;
    double t = (double)(num - (long)c * (long)(N - 1)) / (double)(N - 1);
    for (int l = 0; l < 4; ++l) w[c + l] = orc_beta(l, t);
}

/* Weights of the K = n_c nodes of one axis when the regions sit on the FFD
 * lattice (eq 7 with the control points of eq 17 as region centres): node
 * c + l, c = floor(x / delta), carries beta_l((x mod delta) / delta). */
void orc_axis_node_weights(int x, int delta, int K, double *w)
{
    for (int j = 0; j < K; ++j) w[j] = 0.0;
    int c = x / delta;
    double eta = (double)(x % delta) / delta;
    for (int l = 0; l < 4; ++l) w[c + l] = orc_beta(l, eta);
}

static void axis_weights(const orc_problem *P, int e, int x, double *w)
{
    if (P->at_nodes) orc_axis_node_weights(x, P->delta[e], P->K[e], w);
    else orc_axis_region_weights(x, P->nf[e], P->K[e], w);
}

/* ----------------------------------------------- T(x; Phi), eqs (8, 17)
 * Literal 64-term sum.  ffd holds displacements (fixed-voxel units) as
 * float[3][ncz][ncy][ncx]; stored node index = paper index + 1. */
void orc_ffd_T(const orc_problem *P, const float *ffd, int x, int y, int z, double T[3])
{
    int nc[3];
    orc_ctrl_dims(P, nc);
    long ncell = (long)nc[0] * nc[1] * nc[2];
    int p[3] = {x / P->delta[0], y / P->delta[1], z / P->delta[2]};
    double eta[3] = {(double)(x % P->delta[0]) / P->delta[0],
                     (double)(y % P->delta[1]) / P->delta[1],
                     (double)(z % P->delta[2]) / P->delta[2]};
    T[0] = x; T[1] = y; T[2] = z;
    for (int n = 0; n < 4; ++n)
        for (int m = 0; m < 4; ++m)
            for (int l = 0; l < 4; ++l) {
                double b = orc_beta(l, eta[0]) * orc_beta(m, eta[1]) * orc_beta(n, eta[2]);
                long idx = ((long)(p[2] + n) * nc[1] + (p[1] + m)) * nc[0] + (p[0] + l);
                for (int e = 0; e < 3; ++e) T[e] += b * (double)ffd[e * ncell + idx];
            }
}

/* ------------------------------------- backward warping: trilinear sample
 * y: continuous moving-grid coordinates.  Returns M(y); dsdy gets dM/dy. */
double orc_sample(const orc_problem *P, const float *mov, const double y[3], double dsdy[3])
{
    int i0[3], clamped[3];
    double f[3];
    for (int e = 0; e < 3; ++e) {
        int M = P->nm[e];
        double v = y[e];
        clamped[e] = (v < 0.0 || v > (double)(M - 1));
        if (v < 0.0) v = 0.0;
        if (v > (double)(M - 1)) v = (double)(M - 1);
        int i = (int)floor(v);
        if (i > M - 2) i = M - 2;
        i0[e] = i;
        f[e] = v - i;
    }
    double val = 0.0, g[3] = {0.0, 0.0, 0.0};
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                long idx = ((long)(i0[2] + cz) * P->nm[1] + (i0[1] + cy)) * P->nm[0] + (i0[0] + cx);
                double V = mov[idx];
                double wx = cx ? f[0] : 1.0 - f[0];
                double wy = cy ? f[1] : 1.0 - f[1];
                double wz = cz ? f[2] : 1.0 - f[2];
                val += wx * wy * wz * V;
                g[0] += (cx ? 1.0 : -1.0) * wy * wz * V;
                g[1] += (cy ? 1.0 : -1.0) * wx * wz * V;
                g[2] += (cz ? 1.0 : -1.0) * wx * wy * V;
            }
    for (int e = 0; e < 3; ++e) dsdy[e] = clamped[e] ? 0.0 : g[e];
    return val;
}

/* fixed voxel -> moving coordinates through T, plus dy/dT per axis */
static void map_to_moving(const orc_problem *P, const double T[3], double y[3], double dydT[3])
{
    for (int e = 0; e < 3; ++e) {
        if (P->nm[e] == P->nf[e]) {
            y[e] = T[e];
            dydT[e] = 1.0;
        } else {
            dydT[e] = (double)P->nm[e] / (double)P->nf[e];
            y[e] = (T[e] + 0.5) * dydT[e] - 0.5;
        }
    }
}

/* T(x): the FFD of eq 17, or x + u(x) for a dense displacement field */
static void voxel_T(const orc_problem *P, const float *disp, int x, int y, int z, double T[3])
{
    if (!P->dense) {
        orc_ffd_T(P, disp, x, y, z, T);
        return;
    }
    long nvox = (long)P->nf[0] * P->nf[1] * P->nf[2];
    long idx = ((long)z * P->nf[1] + y) * P->nf[0] + x;
    T[0] = x + (double)disp[idx];
    T[1] = y + (double)disp[nvox + idx];
    T[2] = z + (double)disp[2 * nvox + idx];
}

/* warped, normalised moving intensity at every fixed voxel (clamped to [0, L]) */
static double warped_sample(const orc_problem *P, const float *mov, const float *ffd,
                            int x, int y, int z, double dsdT[3])
{
    double T[3], yy[3], dydT[3], g[3];
    voxel_T(P, ffd, x, y, z, T);
    map_to_moving(P, T, yy, dydT);
    double s = orc_sample(P, mov, yy, g);
    double L = (double)(P->n_bins - 1);
    if (s < 0.0) s = 0.0;
    if (s > L) s = L;
    if (dsdT) for (int e = 0; e < 3; ++e) dsdT[e] = g[e] * dydT[e];
    return s;
}

void orc_warp(const orc_problem *P, const float *mov, const float *ffd, double *out)
{
    for (int z = 0; z < P->nf[2]; ++z)
        for (int y = 0; y < P->nf[1]; ++y)
            for (int x = 0; x < P->nf[0]; ++x)
                out[((long)z * P->nf[1] + y) * P->nf[0] + x] = warped_sample(P, mov, ffd, x, y, z, NULL);
}

/* bins a with possibly non-zero h(a - s) or h'(a - s): floor(s)-1 .. floor(s)+2 */
static int tap_bins(double s, int L, int *bins)
{
    int f = (int)floor(s), n = 0;
    for (int a = f - 1; a <= f + 2; ++a)
        if (a >= 0 && a <= L) bins[n++] = a;
    return n;
}

/* one-sided convention for d/ds: right derivative in s (left in kappa),
 * inward (left in s) at the top of the range s = L */
static int deriv_side(double s, int L) { return (s >= (double)L) ? +1 : -1; }

static int n_regions(const orc_problem *P) { return P->K[0] * P->K[1] * P->K[2]; }

static void voxel_AB(const orc_problem *P, const float *fix, const float *mov, const float *ffd,
                     int x, int y, int z, double *A, double *B, double dsdT[3])
{
    double sF = fix[((long)z * P->nf[1] + y) * P->nf[0] + x];
    double sM = warped_sample(P, mov, ffd, x, y, z, dsdT);
    if (P->role == 0) { *A = sM; *B = sF; }
    else { *A = sF; *B = sM; }
}

/* ------------------------------------------ eq (3): 3-D joint PDF and Z
 * One voxel's unnormalised term of eq (3): q[r][a][b] += w(r, x) h(a - A(x))
 * h(b - B(x)) over the regions with w != 0 and the bins with h != 0 (exact).
 * wx, wy, wz: the voxel's per-axis region weights (eq 8). */
static void voxel_mass(const orc_problem *P, const float *fix, const float *mov, const float *ffd,
                       int x, int y, int z, const double *wx, const double *wy, const double *wz, double *q)
{
    int nb = P->n_bins, L = nb - 1;
    double A, B;
    voxel_AB(P, fix, mov, ffd, x, y, z, &A, &B, NULL);
    int ab[4], bb[4];
    int na = tap_bins(A, L, ab), nbb = tap_bins(B, L, bb);
    for (int k = 0; k < P->K[2]; ++k) {
        if (wz[k] == 0.0) continue;
        for (int j = 0; j < P->K[1]; ++j) {
            if (wy[j] == 0.0) continue;
            for (int i = 0; i < P->K[0]; ++i) {
                if (wx[i] == 0.0) continue;
                double w = wx[i] * wy[j] * wz[k];
                int r = (k * P->K[1] + j) * P->K[0] + i;
                for (int ia = 0; ia < na; ++ia) {
                    double ha = orc_h(ab[ia] - A);
                    if (ha == 0.0) continue;
                    for (int ib = 0; ib < nbb; ++ib) {
                        double hb = orc_h(bb[ib] - B);
                        if (hb == 0.0) continue;
                        q[((long)r * nb + ab[ia]) * nb + bb[ib]] += w * ha * hb;
                    }
                }
            }
        }
    }
}

/* Unnormalised eq (3) mass of the voxels of one box, added to q (R x nb x nb):
 * q[r][a][b] += sum over x in [box0, box1) x [box2, box3) x [box4, box5) of
 * w(r, x) h(a - A(x)) h(b - B(x)).  Serial.  Eq (3) is a plain sum over the
 * voxels, so the masses of the boxes of a partition add up to Z p(a, b, r);
 * the finite-difference checks use this to re-evaluate only the voxels whose
 * warp a control-point perturbation changes. */
void orc_joint_mass_box(const orc_problem *P, const float *fix, const float *mov, const float *ffd,
                        const int box[6], double *q)
{
    double *wx = (double *)malloc(sizeof(double) * P->K[0]);
    double *wy = (double *)malloc(sizeof(double) * P->K[1]);
    double *wz = (double *)malloc(sizeof(double) * P->K[2]);
    for (int z = box[4]; z < box[5]; ++z) {
        axis_weights(P, 2, z, wz);
        for (int y = box[2]; y < box[3]; ++y) {
            axis_weights(P, 1, y, wy);
            for (int x = box[0]; x < box[1]; ++x) {
                axis_weights(P, 0, x, wx);
                voxel_mass(P, fix, mov, ffd, x, y, z, wx, wy, wz, q);
            }
        }
    }
    free(wx); free(wy); free(wz);
}

/* p: R x nb x nb, p[(r * nb + a) * nb + b].  Returns Z. */
double orc_joint_pdf(const orc_problem *P, const float *fix, const float *mov, const float *ffd, double *p)
{
    int R = n_regions(P), nb = P->n_bins;
    long cells = (long)R * nb * nb;
    memset(p, 0, sizeof(double) * cells);
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    double *priv = (double *)calloc((size_t)nthreads * cells, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *pp = priv + (long)tid * cells;
        double *wx = (double *)malloc(sizeof(double) * P->K[0]);
        double *wy = (double *)malloc(sizeof(double) * P->K[1]);
        double *wz = (double *)malloc(sizeof(double) * P->K[2]);
#pragma omp for schedule(static)
        for (int z = 0; z < P->nf[2]; ++z) {
            axis_weights(P, 2, z, wz);
            for (int y = 0; y < P->nf[1]; ++y) {
                axis_weights(P, 1, y, wy);
                for (int x = 0; x < P->nf[0]; ++x) {
                    axis_weights(P, 0, x, wx);
                    voxel_mass(P, fix, mov, ffd, x, y, z, wx, wy, wz, pp);
                }
            }
        }
        free(wx); free(wy); free(wz);
    }
    for (int t = 0; t < nthreads; ++t)            /* fixed merge order */
        for (long c = 0; c < cells; ++c) p[c] += priv[(long)t * cells + c];
    free(priv);
    double Z = 0.0;
    for (long c = 0; c < cells; ++c) Z += p[c];
    if (Z > 0.0)
        for (long c = 0; c < cells; ++c) p[c] /= Z;
    return Z;
}

/* per-region statistics of eqs (4, 10) derived from the normalised PDF */
typedef struct {
    double pr;     /* p(r) */
    double mu;     /* mu_r */
    double var;    /* sigma_r^2 */
    double cr;     /* CR(A, B | r) */
    int ok;        /* p(r) > 0 and sigma_r^2 > VAR_REL E_r[b^2] */
} region_stats;

static void region_statistics(int R, int nb, const double *p, region_stats *st, double *pa, double *mua)
{
    /* pa, mua: R x nb; p_r(a) and mu_r(a) (0 where p_r(a) == 0) */
    for (int r = 0; r < R; ++r) {
        const double *q = p + (long)r * nb * nb;
        double pr = 0.0;
        for (int c = 0; c < nb * nb; ++c) pr += q[c];
        st[r].pr = pr;
        st[r].ok = 0;
        st[r].mu = st[r].var = st[r].cr = 0.0;
        for (int a = 0; a < nb; ++a) { pa[r * nb + a] = 0.0; mua[r * nb + a] = 0.0; }
        if (!(pr > 0.0)) continue;
        double mu = 0.0, m2 = 0.0;
        for (int b = 0; b < nb; ++b) {
            double pb = 0.0;
            for (int a = 0; a < nb; ++a) pb += q[a * nb + b] / pr;
            mu += b * pb;
            m2 += (double)b * b * pb;
        }
        double var = m2 - mu * mu;
        st[r].mu = mu;
        st[r].var = var;
        const double e2 = m2;
        for (int a = 0; a < nb; ++a) {
            double s0 = 0.0, s1 = 0.0;
            for (int b = 0; b < nb; ++b) { s0 += q[a * nb + b] / pr; s1 += b * q[a * nb + b] / pr; }
            pa[r * nb + a] = s0;
            mua[r * nb + a] = (s0 > 0.0) ? s1 / s0 : 0.0;
        }
        if (var <= VAR_REL * e2) continue;
        st[r].ok = 1;
        double c = 0.0;          /* Table I inner double loop */
        for (int a = 0; a < nb; ++a)
            for (int b = 0; b < nb; ++b)
                c += ((double)b * b - mua[r * nb + a] * mua[r * nb + a]) * (q[a * nb + b] / pr) / var;
        st[r].cr = 1.0 - c;
    }
}

/* SRWCR from the joint PDF.  which: 0 Table I loop, 1 eq (9), 2 eq (11), 3 eq (12) */
double orc_srwcr_from_pdf(int R, int nb, const double *p, int which)
{
    double E = 0.0;
    double *pa = (double *)malloc(sizeof(double) * nb), *pb = (double *)malloc(sizeof(double) * nb);
    double *mua = (double *)malloc(sizeof(double) * nb);
    for (int r = 0; r < R; ++r) {
        const double *q = p + (long)r * nb * nb;
        double pr = 0.0;                                  /* eq (4) */
        for (int c = 0; c < nb * nb; ++c) pr += q[c];
        if (!(pr > 0.0)) continue;
        for (int a = 0; a < nb; ++a) { pa[a] = 0.0; pb[a] = 0.0; }
        for (int a = 0; a < nb; ++a)
            for (int b = 0; b < nb; ++b) { pa[a] += q[a * nb + b] / pr; pb[b] += q[a * nb + b] / pr; }
        double mu = 0.0, e2 = 0.0;                        /* eq (10) */
        for (int b = 0; b < nb; ++b) { mu += b * pb[b]; e2 += (double)b * b * pb[b]; }
        double var = e2 - mu * mu;
        if (var <= VAR_REL * e2) continue;
        for (int a = 0; a < nb; ++a) {
            double s1 = 0.0;
            for (int b = 0; b < nb; ++b) s1 += b * q[a * nb + b] / pr;
            mua[a] = (pa[a] > 0.0) ? s1 / pa[a] : 0.0;
        }
        if (which == 0) {                                 /* Table I, lines 11-17 */
            double cr = 0.0;
            for (int a = 0; a < nb; ++a)
                for (int b = 0; b < nb; ++b)
                    cr += ((double)b * b - mua[a] * mua[a]) * (q[a * nb + b] / pr) / var;
            E += pr * cr;
        } else if (which == 1) {                          /* eq (9) */
            double s = 0.0;
            for (int a = 0; a < nb; ++a) {
                if (!(pa[a] > 0.0)) continue;
                double s2 = 0.0;
                for (int b = 0; b < nb; ++b) s2 += (double)b * b * q[a * nb + b] / pr;
                double var_a = s2 / pa[a] - mua[a] * mua[a];
                s += var_a * pa[a];
            }
            E += pr * s / var;
        } else if (which == 2) {                          /* eq (11) */
            double s = 0.0;
            for (int a = 0; a < nb; ++a) s += pa[a] * mua[a] * mua[a];
            E += pr * (e2 - s) / var;
        } else {                                          /* eq (12) */
            for (int a = 0; a < nb; ++a)
                for (int b = 0; b < nb; ++b)
                    E += ((double)b * b - mua[a] * mua[a]) / var * q[a * nb + b];
        }
    }
    free(pa); free(pb); free(mua);
    return E;
}

double orc_value(const orc_problem *P, const float *fix, const float *mov, const float *ffd)
{
    int R = n_regions(P), nb = P->n_bins;
    double *p = (double *)malloc(sizeof(double) * (size_t)R * nb * nb);
    orc_joint_pdf(P, fix, mov, ffd, p);
    double D = orc_srwcr_from_pdf(R, nb, p, 0);
    free(p);
    return D;
}

/* --------------------------------------------- dD/dM at one voxel
 * form 0: eq (19) (M is B) or eq (21) (M is A), literal triple sums.
 * form 1: eq (18) / eq (20) with dp(a,b,r)/dM from eq (26). */
static double dDdM_voxel(const orc_problem *P, int form, double A, double B, double Z,
                         const double *wx, const double *wy, const double *wz,
                         const region_stats *st, const double *pa, const double *mua)
{
    int nb = P->n_bins, L = nb - 1;
    int ab[4], bb[4];
    int na = tap_bins(A, L, ab), nbb = tap_bins(B, L, bb);
    double m1B = 0.0;                              /* sum_b b h(b - B) */
    for (int ib = 0; ib < nbb; ++ib) m1B += bb[ib] * orc_h(bb[ib] - B);
    int sideA = deriv_side(A, L), sideB = deriv_side(B, L);
    double g = 0.0;
    for (int k = 0; k < P->K[2]; ++k) {
        if (wz[k] == 0.0) continue;
        for (int j = 0; j < P->K[1]; ++j) {
            if (wy[j] == 0.0) continue;
            for (int i = 0; i < P->K[0]; ++i) {
                if (wx[i] == 0.0) continue;
                int r = (k * P->K[1] + j) * P->K[0] + i;
                if (!st[r].ok) continue;
                double w = wx[i] * wy[j] * wz[k];
                const region_stats *s = &st[r];
                if (form == 0) {
                    for (int ia = 0; ia < na; ++ia)
                        for (int ib = 0; ib < nbb; ++ib) {
                            int a = ab[ia], b = bb[ib];
                            if (P->role == 1) {            /* eq (19) */
                                double c = ((1.0 - s->cr) * ((double)b * b - 2.0 * b * s->mu)
                                            + 2.0 * b * mua[r * nb + a] - (double)b * b) / s->var;
                                g += c * w * orc_h(a - A) * orc_dh(b - B, sideB) / Z;
                            } else {                       /* eq (21) */
                                double mu_a = (pa[r * nb + a] > 0.0) ? mua[r * nb + a] : m1B;
                                double c = (2.0 * b - mu_a) / s->var * mu_a;
                                g += c * w * orc_h(b - B) * orc_dh(a - A, sideA) / Z;
                            }
                        }
                } else {
                    /* dp(a,b,r)/dM for this voxel, eq (26), on the tap rectangle */
                    double dp[4][4];
                    for (int ia = 0; ia < na; ++ia)
                        for (int ib = 0; ib < nbb; ++ib) {
                            int a = ab[ia], b = bb[ib];
                            if (P->role == 1) dp[ia][ib] = -w * orc_h(a - A) * orc_dh(b - B, sideB) / Z;
                            else dp[ia][ib] = -w * orc_dh(a - A, sideA) * orc_h(b - B) / Z;
                        }
                    double pr = s->pr;
                    if (P->role == 1) {                    /* eq (18) with (22), (23) */
                        double t_b2 = 0.0, t_b1 = 0.0, t_mu = 0.0;
                        for (int ib = 0; ib < nbb; ++ib) {
                            double dpb = 0.0;              /* d p_r(b) / dB */
                            for (int ia = 0; ia < na; ++ia) dpb += dp[ia][ib] / pr;
                            t_b2 += (double)bb[ib] * bb[ib] * dpb;
                            t_b1 += (double)bb[ib] * dpb;
                        }
                        for (int ia = 0; ia < na; ++ia) {
                            int a = ab[ia];
                            double p_a = pa[r * nb + a];
                            if (!(p_a > 0.0)) continue;
                            double dmu = 0.0;              /* eq (23) */
                            for (int ib = 0; ib < nbb; ++ib) dmu += bb[ib] * dp[ia][ib] / pr;
                            dmu /= p_a;
                            t_mu += 2.0 * p_a * mua[r * nb + a] * dmu;
                        }
                        double dvar = t_b2 - 2.0 * s->mu * t_b1;   /* eq (22) */
                        g += pr * ((t_b2 - t_mu) / s->var - dvar / s->var * (1.0 - s->cr));
                    } else {                               /* eq (20) with (28) */
                        double t = 0.0;
                        for (int ia = 0; ia < na; ++ia) {
                            int a = ab[ia];
                            double dpa = 0.0, sb = 0.0;
                            for (int ib = 0; ib < nbb; ++ib) { dpa += dp[ia][ib] / pr; sb += bb[ib] * dp[ia][ib] / pr; }
                            double p_a = pa[r * nb + a];
                            if (p_a > 0.0) {
                                double mu_a = mua[r * nb + a];
                                double dmu = -dpa / p_a * mu_a + sb / p_a;
                                t += 2.0 * p_a * mu_a * dmu + mu_a * mu_a * dpa;
                            } else {
                                t += m1B * m1B * dpa;      /* empty bin: limit mu = m1(B) */
                            }
                        }
                        g += -pr / s->var * t;
                    }
                }
            }
        }
    }
    return g;
}

/* ------------------------------------------------ gradient, eqs (16, 17)
 * grad: float64[3][ncz][ncy][ncx] = dD/d(displacement); for a dense field
 * (P->dense) float64[3][nz][ny][nx] = dD/du(x), eq 16 with dT/du = 1.
 * dDdM_out (optional): dD/dM at every fixed voxel.  Returns D. */
double orc_gradient(const orc_problem *P, const float *fix, const float *mov, const float *ffd,
                    int form, double *grad, double *dDdM_out)
{
    int R = n_regions(P), nb = P->n_bins;
    int nc[3];
    orc_ctrl_dims(P, nc);
    long nvox = (long)P->nf[0] * P->nf[1] * P->nf[2];
    long ncell = P->dense ? nvox : (long)nc[0] * nc[1] * nc[2];
    double *p = (double *)malloc(sizeof(double) * (size_t)R * nb * nb);
    double Z = orc_joint_pdf(P, fix, mov, ffd, p);
    double D = orc_srwcr_from_pdf(R, nb, p, 0);
    region_stats *st = (region_stats *)malloc(sizeof(region_stats) * R);
    double *pa = (double *)malloc(sizeof(double) * R * nb), *mua = (double *)malloc(sizeof(double) * R * nb);
    region_statistics(R, nb, p, st, pa, mua);
    free(p);
    memset(grad, 0, sizeof(double) * 3 * ncell);
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    double *priv = P->dense ? NULL : (double *)calloc((size_t)nthreads * 3 * ncell, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *gg = P->dense ? grad : priv + (long)tid * 3 * ncell;
        double *wx = (double *)malloc(sizeof(double) * P->K[0]);
        double *wy = (double *)malloc(sizeof(double) * P->K[1]);
        double *wz = (double *)malloc(sizeof(double) * P->K[2]);
#pragma omp for schedule(static)
        for (int z = 0; z < P->nf[2]; ++z) {
            axis_weights(P, 2, z, wz);
            for (int y = 0; y < P->nf[1]; ++y) {
                axis_weights(P, 1, y, wy);
                for (int x = 0; x < P->nf[0]; ++x) {
                    axis_weights(P, 0, x, wx);
                    double A, B, dsdT[3];
                    voxel_AB(P, fix, mov, ffd, x, y, z, &A, &B, dsdT);
                    double g = dDdM_voxel(P, form, A, B, Z, wx, wy, wz, st, pa, mua);
                    long vi = ((long)z * P->nf[1] + y) * P->nf[0] + x;
                    if (dDdM_out) dDdM_out[vi] = g;
                    if (P->dense) {                /* eq (16): dT/du = 1 */
                        for (int e = 0; e < 3; ++e) gg[e * nvox + vi] = g * dsdT[e];
                        continue;
                    }
                    if (g == 0.0) continue;
                    /* eq (16) with the Jacobian of eq (17) */
                    int pc[3] = {x / P->delta[0], y / P->delta[1], z / P->delta[2]};
                    double eta[3] = {(double)(x % P->delta[0]) / P->delta[0],
                                     (double)(y % P->delta[1]) / P->delta[1],
                                     (double)(z % P->delta[2]) / P->delta[2]};
                    for (int n = 0; n < 4; ++n)
                        for (int m = 0; m < 4; ++m)
                            for (int l = 0; l < 4; ++l) {
                                double b = orc_beta(l, eta[0]) * orc_beta(m, eta[1]) * orc_beta(n, eta[2]);
                                long idx = ((long)(pc[2] + n) * nc[1] + (pc[1] + m)) * nc[0] + (pc[0] + l);
                                for (int e = 0; e < 3; ++e) gg[e * ncell + idx] += g * dsdT[e] * b;
                            }
                }
            }
        }
        free(wx); free(wy); free(wz);
    }
    if (!P->dense)
        for (int t = 0; t < nthreads; ++t)
            for (long c = 0; c < 3 * ncell; ++c) grad[c] += priv[(long)t * 3 * ncell + c];
    free(priv);
    free(st); free(pa); free(mua);
    return D;
}

/* dD/ds_F: the derivative of D with respect to the normalised fixed intensity
 * at every fixed voxel (a dense field [nz][ny][nx]).  The fixed image is B
 * when the moving image is A and A otherwise, so its derivative is eq (19)
 * (form 0) or eqs (18), (26) (form 1) when it is B, and eq (21) or eqs (20),
 * (26) when it is A; the per-voxel routine takes the formula from the role,
 * so it runs on a copy of the problem with the role flipped while A and B
 * keep their images.  Returns D. */
double orc_gradient_fixed(const orc_problem *P, const float *fix, const float *mov, const float *disp, int form,
                          double *dDdF)
{
    int R = n_regions(P), nb = P->n_bins;
    double *p = (double *)malloc(sizeof(double) * (size_t)R * nb * nb);
    double Z = orc_joint_pdf(P, fix, mov, disp, p);
    double D = orc_srwcr_from_pdf(R, nb, p, 0);
    region_stats *st = (region_stats *)malloc(sizeof(region_stats) * R);
    double *pa = (double *)malloc(sizeof(double) * R * nb), *mua = (double *)malloc(sizeof(double) * R * nb);
    region_statistics(R, nb, p, st, pa, mua);
    free(p);
    orc_problem Pf = *P;
    Pf.role = 1 - P->role;
#pragma omp parallel
    {
        double *wx = (double *)malloc(sizeof(double) * P->K[0]);
        double *wy = (double *)malloc(sizeof(double) * P->K[1]);
        double *wz = (double *)malloc(sizeof(double) * P->K[2]);
#pragma omp for schedule(static)
        for (int z = 0; z < P->nf[2]; ++z) {
            axis_weights(P, 2, z, wz);
            for (int y = 0; y < P->nf[1]; ++y) {
                axis_weights(P, 1, y, wy);
                for (int x = 0; x < P->nf[0]; ++x) {
                    axis_weights(P, 0, x, wx);
                    double A, B;
                    voxel_AB(P, fix, mov, disp, x, y, z, &A, &B, NULL);
                    long vi = ((long)z * P->nf[1] + y) * P->nf[0] + x;
                    dDdF[vi] = dDdM_voxel(&Pf, form, A, B, Z, wx, wy, wz, st, pa, mua);
                }
            }
        }
        free(wx); free(wy); free(wz);
    }
    free(st); free(pa); free(mua);
    return D;
}

/* ------------------------------------------------ RaPTOR, eqs (6), (13), (14)
 * Boxcar patches (eq 6): patches[6 r .. 6 r + 5] = x0, y0, z0, x1, y1, z1, a
 * half-open box on the fixed grid (clipped to it); N_r is its voxel count and
 * N_p = n_patches.  A linear window h(t) = max(0, 1 - |t|) on the A-bins
 * (eq 14); the B-side statistics are plain frequency moments of B (eq 13 and
 * sigma_r^2 = E_r[B^2] - E_r[B]^2 over the patch).  A patch whose B variance
 * is at most VAR_REL of E_r[B^2] contributes nothing.
 * grad (optional): dRaPTOR/d(displacement) in the layout of orc_gradient
 * (FFD coefficients, or a dense field when P->dense); dRds_out (optional):
 * dRaPTOR/ds_M at every fixed voxel.  Returns RaPTOR. */
static double h_lin(double t) { t = fabs(t); return t < 1.0 ? 1.0 - t : 0.0; }

/* one-sided derivative of h_lin(a - s) in s: right derivative (left in the
 * argument a - s), inward at the top of the range s = L */
static double dh_lin_ds(double a, double s, int L)
{
    double k = a - s;                     /* argument of h */
    int side = deriv_side(s, L);          /* -1: left derivative in k, +1: right */
    if (side < 0) {                       /* approach k from below */
        if (k > -1.0 && k <= 0.0) return -1.0;   /* h = 1 + k on (-1, 0]: dh/dk = 1, dk/ds = -1 */
        if (k > 0.0 && k <= 1.0) return 1.0;     /* h = 1 - k on (0, 1]: dh/dk = -1 */
        return 0.0;
    }
    if (k >= -1.0 && k < 0.0) return -1.0;
    if (k >= 0.0 && k < 1.0) return 1.0;
    return 0.0;
}

double orc_raptor(const orc_problem *P, const float *fix, const float *mov, const float *disp, const int *patches,
                  int n_patches, double *grad, double *dRds_out)
{
    int nb = P->n_bins, L = nb - 1;
    long nvox = (long)P->nf[0] * P->nf[1] * P->nf[2];
    int nc[3];
    orc_ctrl_dims(P, nc);
    long ncell = P->dense ? nvox : (long)nc[0] * nc[1] * nc[2];
    int want = grad || dRds_out;
    /* A(x), B(x) (and dM/dT) at every fixed voxel */
    double *Av = (double *)malloc(sizeof(double) * nvox), *Bv = (double *)malloc(sizeof(double) * nvox);
    double *dsdT = want ? (double *)malloc(sizeof(double) * 3 * nvox) : NULL;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < P->nf[2]; ++z)
        for (int y = 0; y < P->nf[1]; ++y)
            for (int x = 0; x < P->nf[0]; ++x) {
                long vi = ((long)z * P->nf[1] + y) * P->nf[0] + x;
                double d3[3];
                voxel_AB(P, fix, mov, disp, x, y, z, &Av[vi], &Bv[vi], d3);
                if (dsdT)
                    for (int e = 0; e < 3; ++e) dsdT[3 * vi + e] = d3[e];
            }
    /* per patch: its box clipped to the grid, N_r, p_r(a) N_r, S1_a, E1, sigma^2, T_r */
    int *box = (int *)malloc(sizeof(int) * 6 * (size_t)(n_patches > 0 ? n_patches : 1));
    double *Pa = (double *)calloc((size_t)n_patches * nb + 1, sizeof(double));
    double *S1 = (double *)calloc((size_t)n_patches * nb + 1, sizeof(double));
    double *Nr = (double *)calloc((size_t)n_patches + 1, sizeof(double));
    double *E1r = (double *)calloc((size_t)n_patches + 1, sizeof(double));
    double *varr = (double *)calloc((size_t)n_patches + 1, sizeof(double));
    double *Tr = (double *)calloc((size_t)n_patches + 1, sizeof(double));
    int *ok = (int *)calloc((size_t)n_patches + 1, sizeof(int));
#pragma omp parallel for schedule(dynamic, 4)
    for (int r = 0; r < n_patches; ++r) {
        int *b = box + 6 * r;
        for (int e = 0; e < 3; ++e) {
            b[e] = patches[6 * r + e] < 0 ? 0 : patches[6 * r + e];
            b[3 + e] = patches[6 * r + 3 + e] > P->nf[e] ? P->nf[e] : patches[6 * r + 3 + e];
        }
        if (b[3] <= b[0] || b[4] <= b[1] || b[5] <= b[2]) continue;      /* clipped away: adds 0 */
        double N = (double)(b[3] - b[0]) * (b[4] - b[1]) * (b[5] - b[2]);
        double sB = 0.0, sB2 = 0.0, *pa = Pa + (long)r * nb, *s1 = S1 + (long)r * nb;
        for (int z = b[2]; z < b[5]; ++z)
            for (int y = b[1]; y < b[4]; ++y)
                for (int x = b[0]; x < b[3]; ++x) {
                    long vi = ((long)z * P->nf[1] + y) * P->nf[0] + x;
                    double A = Av[vi], B = Bv[vi];
                    sB += B;
                    sB2 += B * B;
                    for (int a = 0; a < nb; ++a) {     /* eq (14), every bin */
                        double hw = h_lin(a - A);
                        pa[a] += hw;
                        s1[a] += hw * B;
                    }
                }
        double E1 = sB / N, E2 = sB2 / N, var = E2 - E1 * E1;
        Nr[r] = N;
        E1r[r] = E1;
        varr[r] = var;
        if (!(var > VAR_REL * E2)) continue;
        double Q = 0.0;                               /* sum_a p_r(a) mu_r(a)^2 */
        for (int a = 0; a < nb; ++a)
            if (pa[a] > 0.0) Q += (pa[a] / N) * (s1[a] / pa[a]) * (s1[a] / pa[a]);
        Tr[r] = (E2 - Q) / var;                       /* the patch's term of eq (13) */
        ok[r] = 1;
    }
    double value = 0.0;
    for (int r = 0; r < n_patches; ++r) value += Tr[r];
    value /= (double)n_patches;
    if (want) {
        /* derivative of T_r with respect to A(x) and B(x) for x in patch r */
        double *dRds = (double *)calloc((size_t)nvox, sizeof(double));
#pragma omp parallel for schedule(dynamic, 4)
        for (int r = 0; r < n_patches; ++r) {
            if (!ok[r]) continue;
            const int *b = box + 6 * r;
            double N = Nr[r], E1 = E1r[r], var = varr[r], T = Tr[r];
            const double *pa = Pa + (long)r * nb, *s1 = S1 + (long)r * nb;
            for (int z = b[2]; z < b[5]; ++z)
                for (int y = b[1]; y < b[4]; ++y)
                    for (int x = b[0]; x < b[3]; ++x) {
                        long vi = ((long)z * P->nf[1] + y) * P->nf[0] + x;
                        double A = Av[vi], B = Bv[vi];
                        double dQ_dA = 0.0, dQ_dB = 0.0;
                        for (int a = 0; a < nb; ++a) {
                            double mu = pa[a] > 0.0 ? s1[a] / pa[a] : B;   /* empty bin: the one-sided limit */
                            double d = dh_lin_ds(a, A, L);
                            /* d(S1^2 / P)/dA = (2 mu B - mu^2) dh/dA */
                            dQ_dA += d * (2.0 * mu * B - mu * mu) / N;
                            dQ_dB += 2.0 * h_lin(a - A) * mu / N;
                        }
                        double dT_dA = -dQ_dA / var;
                        double dvar_dB = 2.0 * B / N - 2.0 * E1 / N;
                        double dT_dB = (2.0 * B / N - dQ_dB) / var - T / var * dvar_dB;
                        double t = (P->role == 0 ? dT_dA : dT_dB) / (double)n_patches;
#pragma omp atomic
                        dRds[vi] += t;
                    }
        }
        if (dRds_out) memcpy(dRds_out, dRds, sizeof(double) * nvox);
        if (grad) {
            /* eq (16): the chain rule through dM/dT, then eq (17) to the FFD nodes */
            memset(grad, 0, sizeof(double) * 3 * ncell);
            int nthreads = 1;
#ifdef _OPENMP
            nthreads = omp_get_max_threads();
#endif
            double *priv = P->dense ? NULL : (double *)calloc((size_t)nthreads * 3 * ncell, sizeof(double));
#pragma omp parallel
            {
                int tid = 0;
#ifdef _OPENMP
                tid = omp_get_thread_num();
#endif
                double *gg = P->dense ? grad : priv + (long)tid * 3 * ncell;
#pragma omp for schedule(static)
                for (int z = 0; z < P->nf[2]; ++z)
                    for (int y = 0; y < P->nf[1]; ++y)
                        for (int x = 0; x < P->nf[0]; ++x) {
                            long vi = ((long)z * P->nf[1] + y) * P->nf[0] + x;
                            double g = dRds[vi];
                            const double *d3 = dsdT + 3 * vi;
                            if (P->dense) {
                                for (int e = 0; e < 3; ++e) gg[e * nvox + vi] = g * d3[e];
                                continue;
                            }
                            if (g == 0.0) continue;
                            int pc[3] = {x / P->delta[0], y / P->delta[1], z / P->delta[2]};
                            double eta[3] = {(double)(x % P->delta[0]) / P->delta[0],
                                             (double)(y % P->delta[1]) / P->delta[1],
                                             (double)(z % P->delta[2]) / P->delta[2]};
                            for (int n = 0; n < 4; ++n)
                                for (int m = 0; m < 4; ++m)
                                    for (int l = 0; l < 4; ++l) {
                                        double bw = orc_beta(l, eta[0]) * orc_beta(m, eta[1]) * orc_beta(n, eta[2]);
                                        long idx = ((long)(pc[2] + n) * nc[1] + (pc[1] + m)) * nc[0] + (pc[0] + l);
                                        for (int e = 0; e < 3; ++e) gg[e * ncell + idx] += g * d3[e] * bw;
                                    }
                        }
            }
            if (!P->dense)
                for (int t = 0; t < nthreads; ++t)
                    for (long c = 0; c < 3 * ncell; ++c) grad[c] += priv[(long)t * 3 * ncell + c];
            free(priv);
        }
        free(dRds);
    }
    free(Av); free(Bv); free(dsdT); free(box);
    free(Pa); free(S1); free(Nr); free(E1r); free(varr); free(Tr); free(ok);
    return value;
}

/* number of threads the parallel loops use (reported by the CPU baseline) */
/* threads of the parallel loops (timing only: the results do not depend on it
 * beyond the fixed-order merge of the per-thread PDFs) */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
