/* Test infrastructure: drives the CPU oracle (built serially with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitized.py) through every entry point on a
 * 20-triangle sphere, for temporal orders 0 and 1, and checks what holds at any size: block
 * symmetry, the quadrature-point count over a set of node blocks and its complement adding up,
 * finite values.  Returns 0 when every check holds; the sanitizers abort on a memory or
 * undefined-behaviour error. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct orc_tables orc_tables;
orc_tables *orc_tables_build(const double *t, int Nn, int cut, int p, double rmax, int n);
void orc_tables_free(orc_tables *T);
void orc_psi(const double *t, int N, int cut, int p, int k, int i, double r, double out[2]);
void orc_psi_fast(const orc_tables *T, int k, int i, double r, double out[2]);
int orc_assemble_dense(const double *xyz, int M, const int32_t *tri, int E, const double *t, int N, int cut,
                       int porder, int mode, int ss_order, const orc_tables *tab, double *out);
int orc_assemble_entries(const double *xyz, int M, const int32_t *tri, int E, const double *t, int N, int cut,
                         int porder, int mode, int ss_order, const orc_tables *tab, int nsel, const int32_t *sel_j,
                         const int32_t *sel_l, double *out);
int orc_rhs_plane_pulse(const double *xyz, int M, const int32_t *tri, int E, const double *t, int N, int cut,
                        int porder, const double d[3], double t0, double width, double *g);
int orc_potential_dl(const double *xyz, int M, const int32_t *tri, int E, const double *t, int N, int cut,
                     int porder, const double *alpha, int npts, const double *pts, int ntimes, const double *times,
                     double *out);
int64_t orc_count_quad_evals(const double *xyz, int M, const int32_t *tri, int E, const double *t, int N, int porder,
                             int ss_order, const unsigned char *node_mask);
int64_t orc_local_batch(const double *xyz, const int32_t *tri, int npairs, const int32_t *taus,
                        const int32_t *sigmas, const double *t, int Nn, int cut, int porder, int ss_order,
                        const orc_tables *tab, double *checksum);

/* Icosahedron on the unit sphere: vertices (0, +-1, +-phi) and cyclic permutations; faces are the
 * triples at mutual distance 2 (before scaling), oriented with the normal pointing outward. */
static int icosahedron(double *xyz, int32_t *tri)
{
    const double ph = 0.5 * (1.0 + sqrt(5.0));
    int m = 0;
    for (int c = 0; c < 3; ++c)
        for (int s1 = -1; s1 <= 1; s1 += 2)
            for (int s2 = -1; s2 <= 1; s2 += 2) {
                double v[3] = {0.0, s1 * 1.0, s2 * ph};
                xyz[3 * m + c] = v[0];
                xyz[3 * m + (c + 1) % 3] = v[1];
                xyz[3 * m + (c + 2) % 3] = v[2];
                ++m;
            }
    int e = 0;
    for (int a = 0; a < 12; ++a)
        for (int b = a + 1; b < 12; ++b)
            for (int c = b + 1; c < 12; ++c) {
                const int ids[3] = {a, b, c};
                int ok = 1;
                for (int u = 0; u < 3; ++u) {
                    const double *p = xyz + 3 * ids[u], *q = xyz + 3 * ids[(u + 1) % 3];
                    const double d = sqrt((p[0] - q[0]) * (p[0] - q[0]) + (p[1] - q[1]) * (p[1] - q[1]) +
                                          (p[2] - q[2]) * (p[2] - q[2]));
                    ok = ok && fabs(d - 2.0) < 1e-9;
                }
                if (!ok) continue;
                const double *p0 = xyz + 3 * a, *p1 = xyz + 3 * b, *p2 = xyz + 3 * c;
                const double u1[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
                const double u2[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
                const double nrm[3] = {u1[1] * u2[2] - u1[2] * u2[1], u1[2] * u2[0] - u1[0] * u2[2],
                                       u1[0] * u2[1] - u1[1] * u2[0]};
                const double side = nrm[0] * (p0[0] + p1[0] + p2[0]) + nrm[1] * (p0[1] + p1[1] + p2[1]) +
                                    nrm[2] * (p0[2] + p1[2] + p2[2]);
                tri[3 * e] = a;
                tri[3 * e + 1] = side > 0 ? b : c;
                tri[3 * e + 2] = side > 0 ? c : b;
                ++e;
            }
    for (int v = 0; v < 12; ++v) {
        const double r = sqrt(xyz[3 * v] * xyz[3 * v] + xyz[3 * v + 1] * xyz[3 * v + 1] + xyz[3 * v + 2] * xyz[3 * v + 2]);
        for (int c = 0; c < 3; ++c) xyz[3 * v + c] /= r;
    }
    return e;
}

#define CHECK(cond, ...)                                                                       \
    do {                                                                                       \
        if (!(cond)) {                                                                         \
            fprintf(stderr, __VA_ARGS__);                                                      \
            fprintf(stderr, "\n");                                                             \
            return 1;                                                                          \
        }                                                                                      \
    } while (0)

static int run(int p, int cut, const double *t, int N)
{
    double xyz[36];
    int32_t tri[60];
    const int E = icosahedron(xyz, tri), M = 12, L = N * (p + 1);
    CHECK(E == 20, "icosahedron has %d faces", E);
    orc_tables *T = orc_tables_build(t, N, cut, p, 2.1, 256);
    CHECK(T != NULL, "tables");
    double a[2], b[2];
    orc_psi(t, N, cut, p, L - 1, 0, 0.7, a);
    orc_psi_fast(T, L - 1, 0, 0.7, b);
    CHECK(isfinite(a[0]) && isfinite(a[1]) && isfinite(b[0]) && isfinite(b[1]), "psi");
    double *A = malloc(sizeof(double) * (size_t)L * L * M * M);
    CHECK(orc_assemble_dense(xyz, M, tri, E, t, N, cut, p, 0, 3, T, A) == 0, "dense");
    double sc = 0.0;
    for (size_t s = 0; s < (size_t)L * L * M * M; ++s) {
        CHECK(isfinite(A[s]), "finite");
        sc = fmax(sc, fabs(A[s]));
    }
    for (int kb = 0; kb < L * L; ++kb)
        for (int j = 0; j < M; ++j)
            for (int l = 0; l < M; ++l)
                CHECK(fabs(A[((size_t)kb * M + j) * M + l] - A[((size_t)kb * M + l) * M + j]) <= 1e-13 * sc,
                      "symmetry");
    const int32_t sj[3] = {0, 5, 11}, sl[3] = {3, 5, 0};
    double *sel = malloc(sizeof(double) * 3 * L * L);
    CHECK(orc_assemble_entries(xyz, M, tri, E, t, N, cut, p, 0, 3, T, 3, sj, sl, sel) == 0, "entries");
    for (int s = 0; s < 3; ++s)
        for (int kb = 0; kb < L * L; ++kb)
            CHECK(fabs(sel[s * L * L + kb] - A[((size_t)kb * M + sj[s]) * M + sl[s]]) <= 1e-12 * sc, "entries");
    unsigned char *mask = malloc((size_t)N * N), *inv = malloc((size_t)N * N);
    for (int q = 0; q < N * N; ++q) {
        mask[q] = (unsigned char)((q * 7) % 3 == 0);
        inv[q] = (unsigned char)!mask[q];
    }
    const int64_t all = orc_count_quad_evals(xyz, M, tri, E, t, N, p, 3, NULL);
    CHECK(all > 0 && orc_count_quad_evals(xyz, M, tri, E, t, N, p, 3, mask) +
                         orc_count_quad_evals(xyz, M, tri, E, t, N, p, 3, inv) == all, "count");
    double *g = malloc(sizeof(double) * L * M);
    const double d[3] = {0.0, 0.0, 1.0};
    CHECK(orc_rhs_plane_pulse(xyz, M, tri, E, t, N, cut, p, d, 1.2, 0.3, g) == 0, "rhs");
    const double pts[6] = {0.0, 0.0, 2.0, 0.3, -0.4, 1.5};
    const double times[2] = {0.5 * t[N - 1], t[N - 1]};
    double u[4];
    if (p == 0) {
        CHECK(orc_potential_dl(xyz, M, tri, E, t, N, cut, p, g, 2, pts, 2, times, u) == 0, "potential");
        for (int s = 0; s < 4; ++s) CHECK(isfinite(u[s]), "potential finite");
    }
    const int32_t taus[3] = {0, 1, 2}, sigs[3] = {7, 1, 19};
    double chk = 0.0;
    CHECK(orc_local_batch(xyz, tri, 3, taus, sigs, t, N, cut, p, 3, T, &chk) > 0 && isfinite(chk), "batch");
    free(A);
    free(sel);
    free(mask);
    free(inv);
    free(g);
    orc_tables_free(T);
    return 0;
}

int main(void)
{
    const double eq[5] = {0.0, 0.75, 1.5, 2.25, 3.0};
    const double graded[5] = {0.0, 0.4, 1.3, 1.9, 3.0};
    if (run(0, 0, eq, 5) || run(1, 0, graded, 5) || run(0, 1, graded, 5)) return 1;
    printf("oracle sanitized run ok\n");
    return 0;
}
