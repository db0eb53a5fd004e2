/*
 * tdbem_oracle.c -- CPU reference ("oracle") for the space-time Galerkin discretisation of
 * the sound-hard time-domain boundary integral equation (Veit, Merta, Zapletal, Lukas,
 * arXiv:1503.07221).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU
 * baseline leg load this library.  It shares no code with the GPU library and is written to
 * be read against the paper: plain loops, FP64, no tables, no blocking, no culling beyond the
 * exact support test of psi_{k,i}.
 *
 * Index conventions (0-based throughout):
 *   time nodes t_0 = 0 < ... < t_{N-1} = T, one temporal basis b_i per node (order p = 0),
 *   vertices j, l in [0, M), triangles in [0, E),
 *   A_{k,i}(j,l): test basis (k in time, l in space, x-variable), trial basis (i, j, y-variable),
 *   dense output layout out[((k*N + i)*M + j)*M + l].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------------------------
 * Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n).  Library primitive.
 * ---------------------------------------------------------------------------------------- */
void orc_gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(ORC_PI * (i + 0.75) / (n + 0.5)), pp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int m = 2; m <= n; ++m) {
                double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / m;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            pp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / pp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int m = 2; m <= n; ++m) {
            double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / m;
            p0 = p1;
            p1 = p2;
        }
        pp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;
        w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

/* ------------------------------------------------------------------------------------------
 * Smooth cutoffs F on [0,1] (F = 0 for u <= 0, F = 1 for u >= 1) with F', F''.
 *   cutoff 0 ("bump"): F(u) = beta(u-1) / (beta(u-1) + beta(u)), beta(s) = exp(-1/(1-s^2)):
 *       the two neighbouring node bumps exp(-1/(1-s^2)) normalised to sum to one.
 *       Written as F = 1/(1+exp(g)), g(u) = 1/(u(2-u)) - 1/((1-u)(1+u)).
 *   cutoff 1 ("erf"): the paper's f(s) = erf(2 artanh s)/2 + 1/2 on |s| < 1 (Section 3),
 *       F(u) = f(2u - 1).
 * ---------------------------------------------------------------------------------------- */
static void cutoff_bump(double u, double F[3])
{
    if (u <= 0.0) { F[0] = 0.0; F[1] = 0.0; F[2] = 0.0; return; }
    if (u >= 1.0) { F[0] = 1.0; F[1] = 0.0; F[2] = 0.0; return; }
    double a = u * (2.0 - u), b = (1.0 - u) * (1.0 + u);
    double ap = 2.0 - 2.0 * u, bp = -2.0 * u;          /* a', b' ; a'' = b'' = -2 */
    double g = 1.0 / a - 1.0 / b;
    double gp = -ap / (a * a) + bp / (b * b);
    double gpp = (2.0 * a + 2.0 * ap * ap) / (a * a * a) - (2.0 * b + 2.0 * bp * bp) / (b * b * b);
    double f, s;                                         /* f = 1/(1+e^g), s = f(1-f) */
    if (g > 0.0) { double e = exp(-g); f = e / (1.0 + e); s = e / ((1.0 + e) * (1.0 + e)); }
    else { double e = exp(g); f = 1.0 / (1.0 + e); s = e / ((1.0 + e) * (1.0 + e)); }
    F[0] = f;
    F[1] = -gp * s;
    F[2] = -gpp * s + gp * gp * s * (1.0 - 2.0 * f);
}

static void cutoff_erf(double u, double F[3])
{
    if (u <= 0.0) { F[0] = 0.0; F[1] = 0.0; F[2] = 0.0; return; }
    if (u >= 1.0) { F[0] = 1.0; F[1] = 0.0; F[2] = 0.0; return; }
    double s = 2.0 * u - 1.0;
    double at = 0.5 * log((1.0 + s) / (1.0 - s));       /* artanh s */
    double z = 2.0 * at;
    double om = (1.0 - s) * (1.0 + s);
    double f1 = (2.0 / sqrt(ORC_PI)) * exp(-z * z) / om; /* f'(s) */
    double f2 = f1 * (2.0 * s - 8.0 * at) / om;          /* f''(s) */
    F[0] = 0.5 * erf(z) + 0.5;
    F[1] = 2.0 * f1;
    F[2] = 4.0 * f2;
}

static void cutoff(int kind, double u, double F[3])
{
    if (kind == 1) cutoff_erf(u, F); else cutoff_bump(u, F);
}

void orc_cutoff(int kind, double u, double *out) { cutoff(kind, u, out); }

/* ------------------------------------------------------------------------------------------
 * Partition of unity mu_n and temporal basis b_{n,m} with first and second derivatives
 * (Section 3, construction of f_i, rho_i, mu_i and eq. (BasisFunctions)).
 *   mu_0 = 1 - F((t - t_0)/h_1) on [t_0, t_1];
 *   mu_n = F((t - t_{n-1})/h_n) on [t_{n-1}, t_n], 1 - F((t - t_n)/h_{n+1}) on [t_n, t_{n+1}];
 *   mu_{N-1} = F((t - t_{N-2})/h_{N-1}) on [t_{N-2}, t_{N-1}] and 1 beyond;
 *   every mu_n is 0 for t < 0 (causal extension).  h_n = t_n - t_{n-1}.
 *   b_{n,m} = mu_n P_m(s) with the Legendre polynomial P_m of the support mapped onto [-1, 1]:
 *   s = 2t/h_1 - 1 and the causal factor 8 (t/h_1)^2 for n = 0, s = (t - t_n)/Delta t for the
 *   inner nodes (on a graded grid the affine map of [t_{n-1}, t_{n+1}] onto [-1, 1]), and
 *   s = 2 (t - t_{N-2})/h_{N-1} - 1 for n = N - 1.  m = 0..p; the basis index is j = n (p+1) + m,
 *   L = N (p+1) in all (the numbering of Section 3 read with L = N (p+1)).
 * ---------------------------------------------------------------------------------------- */
void orc_mu(const double *t, int N, int cut, int j, double x, double out[3])
{
    out[0] = out[1] = out[2] = 0.0;
    if (x < 0.0) return;
    double F[3];
    if (j >= 1 && x > t[j - 1] && x <= t[j]) {
        double h = t[j] - t[j - 1];
        cutoff(cut, (x - t[j - 1]) / h, F);
        out[0] = F[0]; out[1] = F[1] / h; out[2] = F[2] / (h * h);
        return;
    }
    if (j <= N - 2 && x >= t[j] && x < t[j + 1]) {
        double h = t[j + 1] - t[j];
        cutoff(cut, (x - t[j]) / h, F);
        out[0] = 1.0 - F[0]; out[1] = -F[1] / h; out[2] = -F[2] / (h * h);
        return;
    }
    if (j == N - 1 && x > t[N - 1]) out[0] = 1.0;
}

/* Legendre polynomial P_m(s) with P_m' and P_m'' (three-term recurrence; the derivatives by
 * P_m' = P_{m-2}' + (2m - 1) P_{m-1} and the same relation once more). */
static void legendre(int m, double s, double P[3])
{
    double p0[3] = {1.0, 0.0, 0.0}, p1[3] = {s, 1.0, 0.0};
    if (m == 0) { P[0] = 1.0; P[1] = P[2] = 0.0; return; }
    for (int q = 2; q <= m; ++q) {
        double v = ((2.0 * q - 1.0) * s * p1[0] - (q - 1.0) * p0[0]) / q;
        double d = p0[1] + (2.0 * q - 1.0) * p1[0];
        double dd = p0[2] + (2.0 * q - 1.0) * p1[1];
        p0[0] = p1[0]; p0[1] = p1[1]; p0[2] = p1[2];
        p1[0] = v; p1[1] = d; p1[2] = dd;
    }
    P[0] = p1[0]; P[1] = p1[1]; P[2] = p1[2];
}

void orc_basis(const double *t, int N, int cut, int p, int j, double x, double out[3])
{
    int n = j / (p + 1), m = j % (p + 1);
    double mu[3], b[3];
    orc_mu(t, N, cut, n, x, mu);
    if (n == 0) {
        if (x <= 0.0) { out[0] = out[1] = out[2] = 0.0; return; }
        double h = t[1] - t[0], u = x / h;
        double q = 8.0 * u * u, qd = 16.0 * u / h, qdd = 16.0 / (h * h);
        b[0] = q * mu[0];
        b[1] = qd * mu[0] + q * mu[1];
        b[2] = qdd * mu[0] + 2.0 * qd * mu[1] + q * mu[2];
    } else {
        b[0] = mu[0]; b[1] = mu[1]; b[2] = mu[2];
    }
    if (m == 0) { out[0] = b[0]; out[1] = b[1]; out[2] = b[2]; return; }
    double lo = n == 0 ? 0.0 : t[n - 1], hi = n == N - 1 ? t[N - 1] : (n == 0 ? t[1] : t[n + 1]);
    double a = 2.0 / (hi - lo), s = a * (x - lo) - 1.0, P[3];
    legendre(m, s, P);
    out[0] = b[0] * P[0];
    out[1] = b[1] * P[0] + b[0] * P[1] * a;
    out[2] = b[2] * P[0] + 2.0 * b[1] * P[1] * a + b[0] * P[2] * a * a;
}

/* ------------------------------------------------------------------------------------------
 * Time kernels (eq. (psis)):
 *   psi_{k,i}(r)  = int_0^T  b_i''(t - r) b_k'(t) dt,
 *   tpsi_{k,i}(r) = int_0^T  b_i(t - r)   b_k'(t) dt.
 * Integration runs over supp b_k' = [t_{k-1}, t_{k+1}] (clipped to [0, T]) intersected with
 * the shifted support of b_i, split at every node and every shifted node t_a + r so that each
 * sub-interval holds a product of two analytic pieces.  On each sub-interval the integrand is
 * flat (C-infinity, not analytic) at the ends, so each one is cut into dyadically graded
 * pieces {0, 1/32, 1/16, 1/8, 1/4, 1/2, 3/4, 7/8, 15/16, 31/32, 1} with 16-point
 * Gauss-Legendre on each.  Accuracy ~1e-13 relative to max |psi| (checked against an
 * arbitrary-precision adaptive integral in the tests).
 * ---------------------------------------------------------------------------------------- */
#define ORC_TQ 16
static double g_tx[ORC_TQ], g_tw[ORC_TQ];
static int g_tq_ready = 0;
static const double g_frac[11] = {0.0, 1.0 / 32, 1.0 / 16, 1.0 / 8, 1.0 / 4, 0.5,
                                  3.0 / 4, 7.0 / 8, 15.0 / 16, 31.0 / 32, 1.0};

/* Filled once when the library is loaded, before any (possibly threaded) call. */
__attribute__((constructor)) static void tq_setup(void)
{
    orc_gauss_legendre(ORC_TQ, g_tx, g_tw);
    g_tq_ready = 1;
}

static void tq_init(void)
{
    if (!g_tq_ready) tq_setup();
}

static int cmp_dbl(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* [lo_k, hi_k] = support of b_k' inside [0, T], k the node */
static void dsupp(const double *t, int N, int k, double *lo, double *hi)
{
    *lo = t[k > 0 ? k - 1 : 0];
    *hi = t[k < N - 1 ? k + 1 : N - 1];
}

/* Open support of psi_{k,i} and tpsi_{k,i} in r >= 0 (Section 3.2), k, i the nodes of the two
 * bases: (t_{k-1} - t_{i+1}, t_{k+1} - t_{i-1}) with t_{-1} := 0 and t_N := T. */
static void node_support(const double *t, int N, int k, int i, double *lo, double *hi)
{
    double tkm = t[k > 0 ? k - 1 : 0], tkp = t[k < N - 1 ? k + 1 : N - 1];
    double tim = t[i > 0 ? i - 1 : 0], tip = t[i < N - 1 ? i + 1 : N - 1];
    double a = tkm - tip;
    *lo = a > 0.0 ? a : 0.0;
    *hi = tkp - tim;
}

void orc_support(const double *t, int N, int p, int k, int i, double *lo, double *hi)
{
    node_support(t, N, k / (p + 1), i / (p + 1), lo, hi);
}

/* The two integrals of eq. (psis) at r, without the support test (at an end of the open
 * support this is the kernel's one-sided limit). */
static void psi_integral(const double *t, int N, int cut, int p, int kb, int ib, double r, double out[2])
{
    tq_init();
    out[0] = out[1] = 0.0;
    int k = kb / (p + 1), i = ib / (p + 1);     /* nodes of the two bases */
    double lo, hi;
    dsupp(t, N, k, &lo, &hi);
    double ilo = r + t[i > 0 ? i - 1 : 0];
    if (ilo > lo) lo = ilo;
    if (i < N - 1) {
        double ihi = r + t[i + 1];
        if (ihi < hi) hi = ihi;
    }
    if (!(hi > lo)) return;
    double pts[8];
    int np = 0;
    pts[np++] = lo;
    pts[np++] = hi;
    if (k > 0 && k < N - 1 && t[k] > lo && t[k] < hi) pts[np++] = t[k];
    for (int a = i - 1; a <= i + 1; ++a) {
        if (a < 0 || a >= N) continue;
        double s = t[a] + r;
        if (s > lo && s < hi) pts[np++] = s;
    }
    qsort(pts, np, sizeof(double), cmp_dbl);
    double ps = 0.0, pt = 0.0;
    for (int s = 0; s + 1 < np; ++s) {
        double a = pts[s], b = pts[s + 1];
        if (!(b > a)) continue;
        for (int g = 0; g < 10; ++g) {
            double pa = a + (b - a) * g_frac[g], pb = a + (b - a) * g_frac[g + 1];
            double hw = 0.5 * (pb - pa), mid = 0.5 * (pa + pb);
            for (int q = 0; q < ORC_TQ; ++q) {
                double tt = mid + hw * g_tx[q], ww = hw * g_tw[q];
                double bi[3], bk[3];
                orc_basis(t, N, cut, p, ib, tt - r, bi);
                orc_basis(t, N, cut, p, kb, tt, bk);
                ps += ww * bi[2] * bk[1];
                pt += ww * bi[0] * bk[1];
            }
        }
    }
    out[0] = ps;
    out[1] = pt;
}

void orc_psi(const double *t, int N, int cut, int p, int k, int i, double r, double out[2])
{
    out[0] = out[1] = 0.0;
    double slo, shi;
    orc_support(t, N, p, k, i, &slo, &shi);
    if (!(r > slo && r < shi)) return;
    psi_integral(t, N, cut, p, k, i, r, out);
}

/* ------------------------------------------------------------------------------------------
 * Fast mode: the oracle's own tabulation of psi_{k,i}, tpsi_{k,i} (a different scheme from the
 * library's piecewise Chebyshev series).  Each kernel's support (lo, hi), cut at rmax (the
 * longest distance on the mesh), carries a uniform grid r_m = lo + m h, m = -ORC_PAD .. n +
 * ORC_PAD, holding the integrals of eq. (psis) without the support test (beyond an end of the
 * support they are the integrals' smooth continuation: zero past a true end, the kernel at
 * negative r below a support cut at r = 0); a value at r inside the open support is the
 * degree-11 polynomial through the 12 grid points around r (barycentric form with the
 * equispaced weights (-1)^j C(11, j)): centred stencils, except next to a support that starts
 * at r = 0, where the stencil keeps to r >= 0; 0 outside.  Checked against the definition in
 * the tests.
 * ---------------------------------------------------------------------------------------- */
#define ORC_LAG 12
#define ORC_PAD 8
typedef struct {
    int N, n;              /* N: basis count L = nodes (p + 1) */
    double *lo, *hi, *h;   /* per (k,i), index k*N + i */
    int64_t *off;          /* first value of (k,i) in val, -1: not tabulated (outside rmax) */
    double *val;           /* 2 (n + 1 + 2 ORC_PAD) per kernel: psi at r_{-ORC_PAD}.., then tpsi */
} orc_tables;

void orc_tables_free(orc_tables *T)
{
    if (!T) return;
    free(T->lo); free(T->hi); free(T->h); free(T->off); free(T->val); free(T);
}

orc_tables *orc_tables_build(const double *t, int Nn, int cut, int p, double rmax, int n)
{
    tq_init();
    if (n < ORC_LAG) n = ORC_LAG;
    int N = Nn * (p + 1);
    orc_tables *T = (orc_tables *)calloc(1, sizeof(orc_tables));
    T->N = N; T->n = n;
    T->lo = (double *)malloc(sizeof(double) * N * N);
    T->hi = (double *)malloc(sizeof(double) * N * N);
    T->h = (double *)malloc(sizeof(double) * N * N);
    T->off = (int64_t *)malloc(sizeof(int64_t) * N * N);
    int64_t tot = 0;
    for (int k = 0; k < N; ++k)
        for (int i = 0; i < N; ++i) {
            int f = k * N + i;
            orc_support(t, Nn, p, k, i, &T->lo[f], &T->hi[f]);
            double end = T->hi[f] < rmax ? T->hi[f] : rmax;
            T->off[f] = -1;
            T->h[f] = 0.0;
            if (T->hi[f] > T->lo[f] && end > T->lo[f]) {
                T->h[f] = (end - T->lo[f]) / n;
                T->off[f] = tot;
                tot += 2 * (int64_t)(n + 1 + 2 * ORC_PAD);
            }
        }
    T->val = (double *)malloc(sizeof(double) * (tot > 0 ? tot : 1));
#pragma omp parallel for schedule(dynamic, 1)
    for (int f = 0; f < N * N; ++f) {
        if (T->off[f] < 0) continue;
        double *v = T->val + T->off[f];
        int np = n + 1 + 2 * ORC_PAD;
        for (int m = 0; m < np; ++m) {
            double o[2];
            psi_integral(t, Nn, cut, p, f / N, f % N, T->lo[f] + (m - ORC_PAD) * T->h[f], o);
            v[m] = o[0];
            v[np + m] = o[1];
        }
    }
    return T;
}

/* psi, tpsi of (k,i) at r from the tables; returns 0 (and zeros) outside the open support. */
static int table_psi(const orc_tables *T, int k, int i, double r, double out[2])
{
    int f = k * T->N + i;
    out[0] = out[1] = 0.0;
    if (!(r > T->lo[f] && r < T->hi[f]) || T->off[f] < 0) return 0;
    const double *v = T->val + T->off[f];
    int np = T->n + 1 + 2 * ORC_PAD;
    double u = (r - T->lo[f]) / T->h[f] + ORC_PAD;     /* grid coordinate, node m at m */
    int a = (int)u - ORC_LAG / 2 + 1;                  /* nodes a .. a + 11 around u */
    if (a > np - ORC_LAG) a = np - ORC_LAG;            /* r at rmax (the mesh's longest distance) */
    /* a support starting at r = 0: the kernels of the first bases are not smooth across r = 0
     * (b_0'' jumps at 0), so the stencil stays on r >= 0 */
    if (T->lo[f] == 0.0 && a < ORC_PAD) a = ORC_PAD;
    double num0 = 0.0, num1 = 0.0, den = 0.0, c = 1.0;   /* c = C(11, j) with alternating sign */
    for (int j = 0; j < ORC_LAG; ++j) {
        double d = u - (a + j);
        if (d == 0.0) { out[0] = v[a + j]; out[1] = v[np + a + j]; return 1; }
        double q = c / d;
        num0 += q * v[a + j];
        num1 += q * v[np + a + j];
        den += q;
        c = -c * (double)(ORC_LAG - 1 - j) / (double)(j + 1);
    }
    out[0] = num0 / den;
    out[1] = num1 / den;
    return 1;
}

void orc_psi_fast(const orc_tables *T, int k, int i, double r, double out[2]) { table_psi(T, k, i, r, out); }

/* ------------------------------------------------------------------------------------------
 * Spatial quadrature.
 * 7-point degree-5 rule on a triangle (Radon; Stroud T2:5-1): centroid with weight 9/40 and
 * the two orbits (a, a, 1-2a), a = (6 -/+ sqrt 15)/21, weights (155 -/+ sqrt 15)/1200
 * (weights normalised to sum to 1, so int_tau f ~ |tau| sum_q w_q f(x_q)).
 * ---------------------------------------------------------------------------------------- */
void orc_rule7(double bary[21], double w[7])
{
    double s15 = sqrt(15.0);
    double a1 = (6.0 - s15) / 21.0, a2 = (6.0 + s15) / 21.0;
    double w1 = (155.0 - s15) / 1200.0, w2 = (155.0 + s15) / 1200.0;
    double B[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3},
                      {a1, a1, 1 - 2 * a1}, {a1, 1 - 2 * a1, a1}, {1 - 2 * a1, a1, a1},
                      {a2, a2, 1 - 2 * a2}, {a2, 1 - 2 * a2, a2}, {1 - 2 * a2, a2, a2}};
    double W[7] = {9.0 / 40, w1, w1, w1, w2, w2, w2};
    for (int q = 0; q < 7; ++q) {
        for (int c = 0; c < 3; ++c) bary[3 * q + c] = B[q][c];
        w[q] = W[q];
    }
}

/* Sauter-Schwab regularising transformations (Sauter & Schwab, Boundary Element Methods,
 * Springer 2011, Sec. 5.2) on the reference triangle {0 <= x2 <= x1 <= 1}.  A physical
 * triangle with ordered vertices (A, B, C) is parametrised as A + x1 (B - A) + x2 (C - B),
 * with barycentric weights (1 - x1, x1 - x2, x2) for (A, B, C).
 *   kind 0, identical triangles: 6 regions, Jacobian xi^3 eta1^2 eta2;
 *   kind 1, common edge A-B in both triangles: 5 regions, Jacobian xi^3 eta1^2 (region 1),
 *           xi^3 eta1^2 eta2 (regions 2-5);
 *   kind 2, common vertex A in both triangles: 2 regions, Jacobian xi^3 eta2.
 * Each region is integrated with an n^4 tensor Gauss-Legendre rule on [0,1]^4.
 * Output rows: (x1, x2, y1, y2, weight); returns the number of points written. */
static void ss_map(int kind, int reg, double xi, double e1, double e2, double e3, double o[5])
{
    double J = 0.0;
    switch (kind) {
    case 0:
        J = xi * xi * xi * e1 * e1 * e2;
        switch (reg) {
        case 0: o[0] = xi; o[1] = xi * (1 - e1 + e1 * e2); o[2] = xi * (1 - e1 * e2 * e3); o[3] = xi * (1 - e1); break;
        case 1: o[0] = xi * (1 - e1 * e2 * e3); o[1] = xi * (1 - e1); o[2] = xi; o[3] = xi * (1 - e1 + e1 * e2); break;
        case 2: o[0] = xi; o[1] = xi * e1 * (1 - e2 + e2 * e3); o[2] = xi * (1 - e1 * e2); o[3] = xi * e1 * (1 - e2); break;
        case 3: o[0] = xi * (1 - e1 * e2); o[1] = xi * e1 * (1 - e2); o[2] = xi; o[3] = xi * e1 * (1 - e2 + e2 * e3); break;
        case 4: o[0] = xi * (1 - e1 * e2 * e3); o[1] = xi * e1 * (1 - e2 * e3); o[2] = xi; o[3] = xi * e1 * (1 - e2); break;
        default: o[0] = xi; o[1] = xi * e1 * (1 - e2); o[2] = xi * (1 - e1 * e2 * e3); o[3] = xi * e1 * (1 - e2 * e3); break;
        }
        break;
    case 1:
        J = xi * xi * xi * e1 * e1 * (reg == 0 ? 1.0 : e2);
        switch (reg) {
        case 0: o[0] = xi; o[1] = xi * e1 * e3; o[2] = xi * (1 - e1 * e2); o[3] = xi * e1 * (1 - e2); break;
        case 1: o[0] = xi; o[1] = xi * e1; o[2] = xi * (1 - e1 * e2 * e3); o[3] = xi * e1 * e2 * (1 - e3); break;
        case 2: o[0] = xi * (1 - e1 * e2); o[1] = xi * e1 * (1 - e2); o[2] = xi; o[3] = xi * e1 * e2 * e3; break;
        case 3: o[0] = xi * (1 - e1 * e2 * e3); o[1] = xi * e1 * e2 * (1 - e3); o[2] = xi; o[3] = xi * e1; break;
        default: o[0] = xi * (1 - e1 * e2 * e3); o[1] = xi * e1 * (1 - e2 * e3); o[2] = xi; o[3] = xi * e1 * e2; break;
        }
        break;
    default:
        J = xi * xi * xi * e2;
        if (reg == 0) { o[0] = xi; o[1] = xi * e1; o[2] = xi * e2; o[3] = xi * e2 * e3; }
        else { o[0] = xi * e2; o[1] = xi * e2 * e3; o[2] = xi; o[3] = xi * e1; }
        break;
    }
    o[4] = J;
}

static const int g_ss_regions[3] = {6, 5, 2};

int orc_ss_rule(int kind, int n, double *out)
{
    double x[64], w[64];
    if (n < 1 || n > 64) return 0;
    orc_gauss_legendre(n, x, w);
    for (int q = 0; q < n; ++q) { x[q] = 0.5 * (x[q] + 1.0); w[q] *= 0.5; }
    int cnt = 0;
    for (int reg = 0; reg < g_ss_regions[kind]; ++reg)
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b)
                for (int c = 0; c < n; ++c)
                    for (int d = 0; d < n; ++d) {
                        double o[5];
                        ss_map(kind, reg, x[a], x[b], x[c], x[d], o);
                        double *r = out + 5 * cnt++;
                        r[0] = o[0]; r[1] = o[1]; r[2] = o[2]; r[3] = o[3];
                        r[4] = o[4] * w[a] * w[b] * w[c] * w[d];
                    }
    return cnt;
}

/* ------------------------------------------------------------------------------------------
 * Triangle geometry.  Unit normal n = (P1-P0)x(P2-P0)/|.|, area |tau|, and the surface curl of
 * the P1 hat of local vertex a: curl_G lambda_a = n x grad lambda_a = -e_a / (2|tau|), where
 * e_a is the edge opposite vertex a traversed counter-clockwise (e_0 = P2-P1, e_1 = P0-P2,
 * e_2 = P1-P0) (tangential rotation as defined after eq. (VarForm)).
 * ---------------------------------------------------------------------------------------- */
typedef struct {
    double P[3][3];
    double n[3];
    double area;
    double curl[3][3];
    int v[3];
} tri_t;

static void tri_build(const double *xyz, const int32_t *tri, int e, tri_t *T)
{
    for (int a = 0; a < 3; ++a) {
        T->v[a] = tri[3 * e + a];
        for (int c = 0; c < 3; ++c) T->P[a][c] = xyz[3 * T->v[a] + c];
    }
    double u[3], w[3], cr[3];
    for (int c = 0; c < 3; ++c) { u[c] = T->P[1][c] - T->P[0][c]; w[c] = T->P[2][c] - T->P[0][c]; }
    cr[0] = u[1] * w[2] - u[2] * w[1];
    cr[1] = u[2] * w[0] - u[0] * w[2];
    cr[2] = u[0] * w[1] - u[1] * w[0];
    double len = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    T->area = 0.5 * len;
    for (int c = 0; c < 3; ++c) T->n[c] = cr[c] / len;
    for (int a = 0; a < 3; ++a) {
        int p = (a + 1) % 3, q = (a + 2) % 3;
        for (int c = 0; c < 3; ++c) T->curl[a][c] = -(T->P[q][c] - T->P[p][c]) / (2.0 * T->area);
    }
}

/* ------------------------------------------------------------------------------------------
 * Local element-pair integrals (eq. (MatrixEntries)) for x in tau (test, index a) and y in
 * sigma (trial, index b):
 *   I_{k,i}[a][b] = 1/(4 pi) int_tau int_sigma [ (n_x.n_y) lam_a(x) lam_b(y) psi_{k,i}(r)
 *                    + (curl lam_a . curl lam_b) tpsi_{k,i}(r) ] / r,   r = |x - y|.
 * The kernel mode replaces (psi, tpsi) for the closed-form tests:
 *   0: the paper's psi_{k,i}, tpsi_{k,i};  1: psi = tpsi = r;  2: psi = tpsi = r^3;
 *   3: psi = tpsi = 1;  4: the paper's kernels, curl-curl term only;  5: the paper's kernels,
 *   n.n term only.  Modes 1-3 use a single (k,i) block (nb = 1).
 * Points are given as lists of (x in tau, y in sigma) with barycentrics and weights; the
 * weight already contains the Jacobians.  Accumulates into loc[(k*nb + i)*9 + 3a + b].
 * ---------------------------------------------------------------------------------------- */
typedef struct {
    const double *t;
    int N, cut, mode;        /* N: time nodes */
    int64_t *count;          /* optional: number of (point pair, k, i) evaluated */
    const orc_tables *tab;   /* fast mode: tabulated kernels (NULL: direct quadrature) */
    int p, L;                /* temporal order, bases L = N (p + 1) */
} tctx_t;

/* Number of (k,i) blocks a kernel mode fills: every (k,i) for the paper's kernels, one for the
 * closed-form test kernels. */
static int mode_blocks(int mode, int N) { return (mode == 0 || mode == 4 || mode == 5) ? N : 1; }

/* For fixed k both ends of the support (t_{k-1} - t_{i+1}, t_{k+1} - t_{i-1}) decrease with i,
 * so {i : r in supp psi_{k,i}} is one range [ia, ib]; binary searches of the two ends. */
static void support_range(const tctx_t *C, int k, double r, int *ia, int *ib)
{
    const orc_tables *T = C->tab;
    int N = C->L, a = 0, b = N;                 /* first i with lo < r */
    while (a < b) { int m = (a + b) / 2; if (T->lo[k * N + m] < r) b = m; else a = m + 1; }
    *ia = a;
    a = 0; b = N;                               /* first i with hi <= r */
    while (a < b) { int m = (a + b) / 2; if (T->hi[k * N + m] <= r) b = m; else a = m + 1; }
    *ib = a - 1;
}

static void accumulate_point(const tctx_t *C, const double *lx, const double *ly,
                             double r, double wgt, double *S1, double *S2)
{
    int nb = mode_blocks(C->mode, C->L);
    if ((C->mode >= 1 && C->mode <= 3) || C->mode == 6) {
        /* closed-form kernels: (psi, tpsi) = (r, r), (r^3, r^3), (1, 1) or (r, r^3) */
        double v1 = C->mode == 1 || C->mode == 6 ? r : C->mode == 2 ? r * r * r : 1.0;
        double v2 = C->mode == 1 ? r : C->mode == 2 || C->mode == 6 ? r * r * r : 1.0;
        double f1 = wgt * v1 / r, f2 = wgt * v2 / r;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) S1[3 * a + b] += f1 * lx[a] * ly[b];
        S2[0] += f2;
        return;
    }
    for (int k = 0; k < C->L; ++k) {
        int ia = 0, ib = C->L - 1;
        if (C->tab) support_range(C, k, r, &ia, &ib);
        for (int i = ia; i <= ib; ++i) {
            double ps[2];
            if (C->tab) {
                if (!table_psi(C->tab, k, i, r, ps)) continue;
            } else {
                double lo, hi;
                orc_support(C->t, C->N, C->p, k, i, &lo, &hi);
                if (!(r > lo && r < hi)) continue;
                orc_psi(C->t, C->N, C->cut, C->p, k, i, r, ps);
            }
            if (C->count) ++*C->count;
            double f1 = C->mode == 4 ? 0.0 : wgt * ps[0] / r;
            double f2 = C->mode == 5 ? 0.0 : wgt * ps[1] / r;
            double *s1 = S1 + 9 * (k * nb + i);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) s1[3 * a + b] += f1 * lx[a] * ly[b];
            S2[k * nb + i] += f2;
        }
    }
}

static void finish_local(const tctx_t *C, const tri_t *X, const tri_t *Y, const double *S1,
                         const double *S2, double *loc)
{
    int nb = mode_blocks(C->mode, C->L);
    double nn = X->n[0] * Y->n[0] + X->n[1] * Y->n[1] + X->n[2] * Y->n[2];
    for (int kb = 0; kb < nb * nb; ++kb)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double cab = X->curl[a][0] * Y->curl[b][0] + X->curl[a][1] * Y->curl[b][1] +
                             X->curl[a][2] * Y->curl[b][2];
                loc[9 * kb + 3 * a + b] = (nn * S1[9 * kb + 3 * a + b] + cab * S2[kb]) / (4.0 * ORC_PI);
            }
}

/* Regular pair (no common vertex): 7 x 7 tensor rule. */
static void local_regular(const tctx_t *C, const tri_t *X, const tri_t *Y, double *S1, double *S2)
{
    double B[21], W[7];
    orc_rule7(B, W);
    for (int q = 0; q < 7; ++q) {
        double x[3];
        for (int c = 0; c < 3; ++c)
            x[c] = B[3 * q] * X->P[0][c] + B[3 * q + 1] * X->P[1][c] + B[3 * q + 2] * X->P[2][c];
        for (int p = 0; p < 7; ++p) {
            double y[3], d2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                y[c] = B[3 * p] * Y->P[0][c] + B[3 * p + 1] * Y->P[1][c] + B[3 * p + 2] * Y->P[2][c];
                d2 += (x[c] - y[c]) * (x[c] - y[c]);
            }
            double wgt = X->area * Y->area * W[q] * W[p];
            accumulate_point(C, &B[3 * q], &B[3 * p], sqrt(d2), wgt, S1, S2);
        }
    }
}

/* Singular pair: kind 0/1/2, permutations px, py give the local vertex index (0..2) of the
 * reference vertices (A, B, C) of X and Y. */
static void local_singular(const tctx_t *C, const tri_t *X, const tri_t *Y, int kind,
                           const int px[3], const int py[3], int order, double *S1, double *S2)
{
    int npts = g_ss_regions[kind] * order * order * order * order;
    double *rule = (double *)malloc(sizeof(double) * 5 * npts);
    orc_ss_rule(kind, order, rule);
    double jac = (2.0 * X->area) * (2.0 * Y->area);
    for (int s = 0; s < npts; ++s) {
        const double *R = rule + 5 * s;
        double lx[3], ly[3], x[3], y[3], d2 = 0.0;
        double bx[3] = {1.0 - R[0], R[0] - R[1], R[1]};
        double by[3] = {1.0 - R[2], R[2] - R[3], R[3]};
        for (int a = 0; a < 3; ++a) { lx[px[a]] = bx[a]; ly[py[a]] = by[a]; }
        for (int c = 0; c < 3; ++c) {
            x[c] = lx[0] * X->P[0][c] + lx[1] * X->P[1][c] + lx[2] * X->P[2][c];
            y[c] = ly[0] * Y->P[0][c] + ly[1] * Y->P[1][c] + ly[2] * Y->P[2][c];
            d2 += (x[c] - y[c]) * (x[c] - y[c]);
        }
        accumulate_point(C, lx, ly, sqrt(d2), jac * R[4], S1, S2);
    }
    free(rule);
}

/* Relation between two triangles: number of shared vertices and the reference orderings.
 * Edge: (A, B) = the shared vertices ordered by global id, C the remaining one.
 * Vertex: A = the shared vertex, (B, C) the next two in the triangle's own cyclic order. */
static int pair_relation(const tri_t *X, const tri_t *Y, int px[3], int py[3])
{
    int sx[3], sy[3], ns = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (X->v[a] == Y->v[b]) { sx[ns] = a; sy[ns] = b; ++ns; }
    if (ns == 3) { for (int a = 0; a < 3; ++a) { px[a] = a; py[a] = a; } return 0; }
    if (ns == 2) {
        int a0 = sx[0], a1 = sx[1], b0 = sy[0], b1 = sy[1];
        if (X->v[a0] > X->v[a1]) { int tmp = a0; a0 = a1; a1 = tmp; tmp = b0; b0 = b1; b1 = tmp; }
        px[0] = a0; px[1] = a1; px[2] = 3 - a0 - a1;
        py[0] = b0; py[1] = b1; py[2] = 3 - b0 - b1;
        return 1;
    }
    if (ns == 1) {
        px[0] = sx[0]; px[1] = (sx[0] + 1) % 3; px[2] = (sx[0] + 2) % 3;
        py[0] = sy[0]; py[1] = (sy[0] + 1) % 3; py[2] = (sy[0] + 2) % 3;
        return 2;
    }
    return 3;
}

/* Local integrals of the ordered pair (X = x-triangle, Y = y-triangle); coincident blocks are
 * symmetrised in (a, b) so that the assembled blocks are exactly symmetric. */
static void pair_local(const tctx_t *C, const tri_t *X, const tri_t *Y, int ss_order, double *loc)
{
    int nb = mode_blocks(C->mode, C->L);
    double *S1 = (double *)calloc((size_t)9 * nb * nb, sizeof(double));
    double *S2 = (double *)calloc((size_t)nb * nb, sizeof(double));
    int px[3], py[3];
    int rel = pair_relation(X, Y, px, py);
    if (rel == 3) local_regular(C, X, Y, S1, S2);
    else local_singular(C, X, Y, rel, px, py, ss_order, S1, S2);
    finish_local(C, X, Y, S1, S2, loc);
    if (rel == 0)
        for (int kb = 0; kb < nb * nb; ++kb)
            for (int a = 0; a < 3; ++a)
                for (int b = a + 1; b < 3; ++b) {
                    double m = 0.5 * (loc[9 * kb + 3 * a + b] + loc[9 * kb + 3 * b + a]);
                    loc[9 * kb + 3 * a + b] = m;
                    loc[9 * kb + 3 * b + a] = m;
                }
    free(S1);
    free(S2);
}

/* Public: local integrals of one ordered triangle pair (used by the closed-form tests). */
void orc_pair_local(const double *xyz, const int32_t *tri, int ex, int ey, const double *t, int N,
                    int cut, int porder, int mode, int ss_order, double *loc)
{
    tctx_t C = {t, N, cut, mode, NULL, NULL, porder, N * (porder + 1)};
    tri_t X, Y;
    tri_build(xyz, tri, ex, &X);
    tri_build(xyz, tri, ey, &Y);
    pair_local(&C, &X, &Y, ss_order, loc);
}

/* ------------------------------------------------------------------------------------------
 * Global blocks A_{k,i}(j,l) = sum over tau containing l and sigma containing j of the local
 * integrals (eq. (integrals)/(MatrixEntries) with the P1 hats phi_l, phi_j).
 * Every unordered pair {p < q} is integrated once with p as the x-triangle and contributes to
 * A(v_b(q), v_a(p)) and, through the symmetry of the kernel in x <-> y, to A(v_a(p), v_b(q));
 * a coincident pair contributes its symmetrised local block once.
 * Dense output out[((k*nb + i)*M + j)*M + l] (zeroed here).  OpenMP over p with per-thread
 * buffers reduced in thread order.
 * ---------------------------------------------------------------------------------------- */
int orc_assemble_dense(const double *xyz, int M, const int32_t *tri, int E, const double *t,
                       int N, int cut, int porder, int mode, int ss_order, const orc_tables *tab, double *out)
{
    int nb = mode_blocks(mode, N * (porder + 1));
    size_t total = (size_t)nb * nb * M * M;
    memset(out, 0, total * sizeof(double));
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    double *buf = (double *)calloc(total * (size_t)nthr, sizeof(double));
    if (!buf) return -1;
    tctx_t C = {t, N, cut, mode, NULL, nb > 1 ? tab : NULL, porder, N * (porder + 1)};
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *mine = buf + total * (size_t)tid;
        double *loc = (double *)malloc(sizeof(double) * 9 * nb * nb);
#pragma omp for schedule(static, 1)
        for (int p = 0; p < E; ++p) {
            tri_t X, Y;
            tri_build(xyz, tri, p, &X);
            for (int q = p; q < E; ++q) {
                tri_build(xyz, tri, q, &Y);
                pair_local(&C, &X, &Y, ss_order, loc);
                for (int kb = 0; kb < nb * nb; ++kb) {
                    double *blk = mine + (size_t)kb * M * M;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) {
                            double v = loc[9 * kb + 3 * a + b];
                            blk[(size_t)Y.v[b] * M + X.v[a]] += v;
                            if (q != p) blk[(size_t)X.v[a] * M + Y.v[b]] += v;
                        }
                }
            }
        }
        free(loc);
    }
    for (int th = 0; th < nthr; ++th)
        for (size_t s = 0; s < total; ++s) out[s] += buf[total * (size_t)th + s];
    free(buf);
    return 0;
}

/* Selected entries: for each requested (j, l), every block A_{k,i}(j,l) is formed from the
 * ordered pairs (tau containing l, sigma containing j), each integrated in the canonical order
 * of the dense assembly.  out[(s*nb + k)*nb + i]. */
int orc_assemble_entries(const double *xyz, int M, const int32_t *tri, int E, const double *t,
                         int N, int cut, int porder, int mode, int ss_order, const orc_tables *tab, int nsel,
                         const int32_t *sel_j, const int32_t *sel_l, double *out)
{
    int nb = mode_blocks(mode, N * (porder + 1));
    (void)M;
    memset(out, 0, sizeof(double) * (size_t)nsel * nb * nb);
    tctx_t C = {t, N, cut, mode, NULL, nb > 1 ? tab : NULL, porder, N * (porder + 1)};
    /* vertex -> triangles */
    int *cnt = (int *)calloc(M, sizeof(int));
    for (int e = 0; e < 3 * E; ++e) cnt[tri[e]]++;
    int *off = (int *)malloc(sizeof(int) * (M + 1));
    off[0] = 0;
    for (int v = 0; v < M; ++v) off[v + 1] = off[v] + cnt[v];
    int *lst = (int *)malloc(sizeof(int) * 3 * E);
    int *fill = (int *)calloc(M, sizeof(int));
    for (int e = 0; e < E; ++e)
        for (int a = 0; a < 3; ++a) { int v = tri[3 * e + a]; lst[off[v] + fill[v]++] = e; }
    /* flatten (s, tau, sigma) work items */
    int nwork = 0;
    for (int s = 0; s < nsel; ++s) nwork += cnt[sel_l[s]] * cnt[sel_j[s]];
    int *work = (int *)malloc(sizeof(int) * 3 * (nwork > 0 ? nwork : 1));
    int w = 0;
    for (int s = 0; s < nsel; ++s)
        for (int u = off[sel_l[s]]; u < off[sel_l[s] + 1]; ++u)
            for (int v = off[sel_j[s]]; v < off[sel_j[s] + 1]; ++v) {
                work[3 * w] = s; work[3 * w + 1] = lst[u]; work[3 * w + 2] = lst[v]; ++w;
            }
    double *res = (double *)calloc((size_t)nwork * nb * nb + 1, sizeof(double));
#pragma omp parallel
    {
        double *loc = (double *)malloc(sizeof(double) * 9 * nb * nb);
#pragma omp for schedule(dynamic, 1)
        for (int it = 0; it < nwork; ++it) {
            int s = work[3 * it], tau = work[3 * it + 1], sig = work[3 * it + 2];
            int j = sel_j[s], l = sel_l[s];
            tri_t X, Y;
            int p = tau < sig ? tau : sig, q = tau < sig ? sig : tau;
            tri_build(xyz, tri, p, &X);
            tri_build(xyz, tri, q, &Y);
            pair_local(&C, &X, &Y, ss_order, loc);
            int al = -1, bj = -1;
            if (tau <= sig) {       /* l is a vertex of X = tau, j a vertex of Y = sigma */
                for (int a = 0; a < 3; ++a) { if (X.v[a] == l) al = a; if (Y.v[a] == j) bj = a; }
                for (int kb = 0; kb < nb * nb; ++kb) res[(size_t)it * nb * nb + kb] = loc[9 * kb + 3 * al + bj];
            } else {                /* j is a vertex of X = sigma, l a vertex of Y = tau */
                for (int a = 0; a < 3; ++a) { if (X.v[a] == j) al = a; if (Y.v[a] == l) bj = a; }
                for (int kb = 0; kb < nb * nb; ++kb) res[(size_t)it * nb * nb + kb] = loc[9 * kb + 3 * al + bj];
            }
        }
        free(loc);
    }
    for (int it = 0; it < nwork; ++it) {
        int s = work[3 * it];
        for (int kb = 0; kb < nb * nb; ++kb) out[(size_t)s * nb * nb + kb] += res[(size_t)it * nb * nb + kb];
    }
    free(res); free(work); free(cnt); free(off); free(lst); free(fill);
    return 0;
}

/* ------------------------------------------------------------------------------------------
 * Right-hand side g_k(l) = int_0^T int_Gamma g(x,t) phi_l(x) b_k'(t) dGamma dt (Section 3),
 * for the plane Gaussian pulse u_inc(x,t) = G(t - t0 - d.x), G(s) = exp(-(s/w)^2):
 *   g = -d u_inc / d n = G'(t - t0 - d.x) (d . n),  G'(s) = -2 s / w^2 exp(-(s/w)^2).
 * Space: the 7-point rule per triangle with the flat-triangle normal.  Time: supp b_k' split
 * at t_k, each half integrated with the graded 16-point composite rule used for psi.
 * Output g[k*M + l].
 * ---------------------------------------------------------------------------------------- */
int orc_rhs_plane_pulse(const double *xyz, int M, const int32_t *tri, int E, const double *t,
                        int N, int cut, int porder, const double d[3], double t0, double width, double *g)
{
    tq_init();
    int L = N * (porder + 1);
    memset(g, 0, sizeof(double) * (size_t)L * M);
    double B[21], W[7];
    orc_rule7(B, W);
    for (int k = 0; k < L; ++k) {
        int kn = k / (porder + 1);
        double lo, hi;
        dsupp(t, N, kn, &lo, &hi);
        double pts[3];
        int np = 0;
        pts[np++] = lo;
        if (kn > 0 && kn < N - 1) pts[np++] = t[kn];
        pts[np++] = hi;
        for (int e = 0; e < E; ++e) {
            tri_t X;
            tri_build(xyz, tri, e, &X);
            double dn = d[0] * X.n[0] + d[1] * X.n[1] + d[2] * X.n[2];
            for (int q = 0; q < 7; ++q) {
                double dx = 0.0;
                for (int c = 0; c < 3; ++c)
                    dx += d[c] * (B[3 * q] * X.P[0][c] + B[3 * q + 1] * X.P[1][c] + B[3 * q + 2] * X.P[2][c]);
                double ti = 0.0;
                for (int s = 0; s + 1 < np; ++s) {
                    double a = pts[s], b = pts[s + 1];
                    for (int gq = 0; gq < 10; ++gq) {
                        double pa = a + (b - a) * g_frac[gq], pb = a + (b - a) * g_frac[gq + 1];
                        double hw = 0.5 * (pb - pa), mid = 0.5 * (pa + pb);
                        for (int m = 0; m < ORC_TQ; ++m) {
                            double tt = mid + hw * g_tx[m];
                            double sarg = tt - t0 - dx;
                            double Gp = -2.0 * sarg / (width * width) * exp(-(sarg / width) * (sarg / width));
                            double bk[3];
                            orc_basis(t, N, cut, porder, k, tt, bk);
                            ti += hw * g_tw[m] * Gp * bk[1];
                        }
                    }
                }
                double f = X.area * W[q] * dn * ti;
                for (int a = 0; a < 3; ++a) g[(size_t)k * M + X.v[a]] += f * B[3 * q + a];
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------
 * Retarded double layer potential of eq. (RetardedPotential) for the discrete density
 * phi(y, t) = sum_i sum_j alpha[i*M + j] b_i(t) phi_j(y):
 *   u(x, t) = -1/(4 pi) int_Gamma (n_y . (x - y)) / r * ( phi(y, t - r) / r^2
 *                                                       + d_t phi(y, t - r) / r ) dGamma_y,
 * r = |x - y|, for points x off Gamma and 0 <= t <= T.  Space: the 7-point rule on every flat
 * triangle; every basis b_i is evaluated at the retarded time (zero outside its support).
 * Output out[s*npts + p] for point p (pts[3p..3p+2]) and time times[s].
 * ---------------------------------------------------------------------------------------- */
int orc_potential_dl(const double *xyz, int M, const int32_t *tri, int E, const double *t, int N, int cut,
                     int porder, const double *alpha, int npts, const double *pts, int ntimes, const double *times,
                     double *out)
{
    int L = N * (porder + 1);
    double B[21], W[7];
    orc_rule7(B, W);
#pragma omp parallel for schedule(dynamic, 1)
    for (int ps = 0; ps < npts * ntimes; ++ps) {
        const int p = ps % npts, s = ps / npts;
        const double *x = pts + 3 * p;
        double u = 0.0;
        for (int e = 0; e < E; ++e) {
            tri_t X;
            tri_build(xyz, tri, e, &X);
            for (int q = 0; q < 7; ++q) {
                double d[3];
                for (int c = 0; c < 3; ++c)
                    d[c] = x[c] - (B[3 * q] * X.P[0][c] + B[3 * q + 1] * X.P[1][c] + B[3 * q + 2] * X.P[2][c]);
                const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                const double nd = X.n[0] * d[0] + X.n[1] * d[1] + X.n[2] * d[2];
                double phi = 0.0, dphi = 0.0;
                for (int i = 0; i < L; ++i) {
                    double bi[3];
                    orc_basis(t, N, cut, porder, i, times[s] - r, bi);
                    if (bi[0] == 0.0 && bi[1] == 0.0) continue;
                    double dens = 0.0;
                    for (int a = 0; a < 3; ++a) dens += B[3 * q + a] * alpha[(size_t)i * M + X.v[a]];
                    phi += bi[0] * dens;
                    dphi += bi[1] * dens;
                }
                u += -X.area * W[q] / (4.0 * ORC_PI) * nd / r * (phi / (r * r) + dphi / r);
            }
        }
        out[(size_t)s * npts + p] = u;
    }
    return 0;
}

/* Quadrature-point count of the method (one unit = one (x_q, y_q', k, i) with r inside the open
 * support of psi_{k,i}), over unordered triangle pairs, computed by brute force.  node_mask
 * (N x N, row = test node) restricts the count to the bases of the node blocks marked nonzero;
 * NULL counts every block. */
int64_t orc_count_quad_evals(const double *xyz, int M, const int32_t *tri, int E, const double *t,
                             int N, int porder, int ss_order, const unsigned char *node_mask)
{
    (void)M;
    int64_t total = 0;
    int L = N * (porder + 1);
    double B[21], W[7];
    orc_rule7(B, W);
    int npmax = 6 * ss_order * ss_order * ss_order * ss_order;
#pragma omp parallel reduction(+ : total)
    {
        double *rule = (double *)malloc(sizeof(double) * 5 * npmax);
#pragma omp for schedule(dynamic, 4)
        for (int p = 0; p < E; ++p) {
            tri_t X, Y;
            tri_build(xyz, tri, p, &X);
            for (int q = p; q < E; ++q) {
                tri_build(xyz, tri, q, &Y);
                int px[3], py[3];
                int rel = pair_relation(&X, &Y, px, py);
                int np;
                if (rel == 3) np = 49;
                else np = orc_ss_rule(rel, ss_order, rule);
                for (int s = 0; s < np; ++s) {
                    double x[3], y[3], d2 = 0.0;
                    if (rel == 3) {
                        int qa = s / 7, qb = s % 7;
                        for (int c = 0; c < 3; ++c) {
                            x[c] = B[3 * qa] * X.P[0][c] + B[3 * qa + 1] * X.P[1][c] + B[3 * qa + 2] * X.P[2][c];
                            y[c] = B[3 * qb] * Y.P[0][c] + B[3 * qb + 1] * Y.P[1][c] + B[3 * qb + 2] * Y.P[2][c];
                        }
                    } else {
                        const double *R = rule + 5 * s;
                        double lx[3], ly[3];
                        double bx[3] = {1.0 - R[0], R[0] - R[1], R[1]};
                        double by[3] = {1.0 - R[2], R[2] - R[3], R[3]};
                        for (int a = 0; a < 3; ++a) { lx[px[a]] = bx[a]; ly[py[a]] = by[a]; }
                        for (int c = 0; c < 3; ++c) {
                            x[c] = lx[0] * X.P[0][c] + lx[1] * X.P[1][c] + lx[2] * X.P[2][c];
                            y[c] = ly[0] * Y.P[0][c] + ly[1] * Y.P[1][c] + ly[2] * Y.P[2][c];
                        }
                    }
                    for (int c = 0; c < 3; ++c) d2 += (x[c] - y[c]) * (x[c] - y[c]);
                    double r = sqrt(d2);
                    for (int k = 0; k < L; ++k)
                        for (int i = 0; i < L; ++i) {
                            double lo, hi;
                            if (node_mask && !node_mask[(k / (porder + 1)) * N + i / (porder + 1)]) continue;
                            orc_support(t, N, porder, k, i, &lo, &hi);
                            if (r > lo && r < hi) ++total;
                        }
                }
            }
        }
        free(rule);
    }
    return total;
}

/* Local integrals of a list of ordered pairs (CPU timing of the method on a sample of a
 * workload): returns the number of (point pair, k, i) evaluations; *checksum receives the sum
 * of all local entries so that nothing is optimised away. */
int64_t orc_local_batch(const double *xyz, const int32_t *tri, int npairs, const int32_t *taus,
                        const int32_t *sigmas, const double *t, int Nn, int cut, int porder, int ss_order,
                        const orc_tables *tab, double *checksum)
{
    int64_t total = 0;
    double sum = 0.0;
    int N = Nn * (porder + 1);
#pragma omp parallel reduction(+ : total, sum)
    {
        int64_t mine = 0;
        tctx_t C = {t, Nn, cut, 0, &mine, tab, porder, N};
        double *loc = (double *)malloc(sizeof(double) * 9 * N * N);
#pragma omp for schedule(dynamic, 1)
        for (int s = 0; s < npairs; ++s) {
            tri_t X, Y;
            tri_build(xyz, tri, taus[s], &X);
            tri_build(xyz, tri, sigmas[s], &Y);
            pair_local(&C, &X, &Y, ss_order, loc);
            for (int m = 0; m < 9 * N * N; ++m) sum += loc[m];
        }
        total += mine;
        free(loc);
    }
    *checksum = sum;
    return total;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
