// Tabulation of the time kernels psi_{k,i}, tilde psi_{k,i} (eq. (psis)) as piecewise Chebyshev
// series (Section 3.1), built on the device: one thread per Chebyshev node computes both kernels
// by quadrature in t, one thread per coefficient forms the interpolant.
#include "tdbem_internal.hpp"

namespace tdbem {

// Both kernels at r by Gauss-Legendre quadrature over t in supp b_k' cap (r + supp b_i), split at
// every node t_k and every shifted node r + t_a and graded dyadically towards each split point.
__device__ void kernels_by_quadrature(const double* t, int N, int p1, int cut, const TimeRule& rule,
                                      int kb, int ib, double r, double& ps, double& pt)
{
    ps = 0.0; pt = 0.0;
    const int k = kb / p1, i = ib / p1;      // the nodes of the two bases
    double lo = t[k > 0 ? k - 1 : 0], hi = t[k < N - 1 ? k + 1 : N - 1];
    const double ilo = r + t[i > 0 ? i - 1 : 0];
    lo = lo > ilo ? lo : ilo;
    if (i < N - 1) {
        const double ihi = r + t[i + 1];
        hi = hi < ihi ? hi : ihi;
    }
    if (!(hi > lo)) return;
    double pts[8];
    int np = 0;
    pts[np++] = lo;
    if (k > 0 && k < N - 1 && t[k] > lo && t[k] < hi) pts[np++] = t[k];
    for (int a = i - 1; a <= i + 1; ++a) {
        if (a < 0 || a >= N) continue;
        const double s = r + t[a];
        if (s > lo && s < hi) pts[np++] = s;
    }
    pts[np++] = hi;
    for (int x = 1; x < np; ++x) {               // insertion sort of at most 6 points
        const double v = pts[x];
        int y = x - 1;
        while (y >= 0 && pts[y] > v) { pts[y + 1] = pts[y]; --y; }
        pts[y + 1] = v;
    }
    double sp = 0.0, st = 0.0;
    for (int s = 0; s + 1 < np; ++s) {
        const double a = pts[s], len = pts[s + 1] - a;
        if (!(len > 0.0)) continue;
        for (int g = 0; g < kTimePieces; ++g) {
            const double pa = a + len * time_grading_edge(g), pb = a + len * time_grading_edge(g + 1);
            const double half = 0.5 * (pb - pa), mid = 0.5 * (pa + pb);
            for (int q = 0; q < kTimeGauss; ++q) {
                const double tt = fma(half, rule.x[q], mid);
                double bv, b1, b2, kv, k1, k2;
                basis_eval(t, N, p1, cut, ib, tt - r, bv, b1, b2);
                basis_eval(t, N, p1, cut, kb, tt, kv, k1, k2);
                const double w = half * rule.w[q] * k1;
                sp = fma(w, b2, sp);
                st = fma(w, bv, st);
            }
        }
    }
    ps = sp;
    pt = st;
}

__global__ void __launch_bounds__(256)
k_table_values(const double* __restrict__ t, int N, int p1, int cut, TimeRule rule, PieceTable pt,
               const int32_t* __restrict__ pc_f, const int32_t* __restrict__ pc_j,
               const int32_t* __restrict__ pc_p, int64_t npieces, const int32_t* __restrict__ f_k,
               const int32_t* __restrict__ f_i, const KernelDesc* __restrict__ desc,
               const double* __restrict__ ivl, double2* __restrict__ values)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= npieces * kNc) return;
    const int64_t pc = gid / kNc;
    const int m = (int)(gid - pc * kNc);
    const int f = pc_f[pc], j = pc_j[pc], p = pc_p[pc];
    const KernelDesc kd = desc[f];
    const double start = ivl[kd.bp_off + 2 * j];
    const double len = 1.0 / ivl[kd.bp_off + 2 * j + 1];
    const double xm = cos(M_PI * (m + 0.5) / kNc);                  // Chebyshev point, first kind
    const double fr = pt.edge[p] + 0.5 * (xm + 1.0) * (pt.edge[p + 1] - pt.edge[p]);
    const double r = start + fr * len;
    double ps, tps;
    kernels_by_quadrature(t, N, p1, cut, rule, f_k[f], f_i[f], r, ps, tps);
    values[gid] = make_double2(ps, tps);
}

__global__ void __launch_bounds__(256)
k_table_coefs(const double2* __restrict__ values, int64_t npieces, double2* __restrict__ coef)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= npieces * kNc) return;
    const int64_t pc = gid / kNc;
    const int m = (int)(gid - pc * kNc);
    const double2* v = values + pc * kNc;
    double a = 0.0, b = 0.0;
    for (int n = 0; n < kNc; ++n) {
        const double c = cos(M_PI * m * (n + 0.5) / kNc);
        a = fma(v[n].x, c, a);
        b = fma(v[n].y, c, b);
    }
    const double s = (m == 0 ? 1.0 : 2.0) / kNc;
    coef[gid] = make_double2(a * s, b * s);
}

__global__ void __launch_bounds__(256)
k_table_eval(TableView tv, int64_t n, const int32_t* __restrict__ k, const int32_t* __restrict__ i,
             const double* __restrict__ r, double* __restrict__ ps, double* __restrict__ tps)
{
    __shared__ PieceTable spt;
    load_piece_table(spt, tv.pt);
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int kk = k[s], ii = i[s];
    double a = 0.0, b = 0.0;
    if (kk >= 0 && kk < tv.N && ii >= 0 && ii < tv.N) {
        const int f = tv.fid[kk * tv.N + ii];
        if (f >= 0) table_eval(tv.desc[f], tv.ivl, tv.coef, spt, r[s], a, b);
    }
    ps[s] = a;
    tps[s] = b;
}

static inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_table_values(const double* t, int N, int p1, int cut, TimeRule rule, PieceTable pt, const int32_t* pc_f,
                         const int32_t* pc_j, const int32_t* pc_p, int64_t npieces, const int32_t* f_k,
                         const int32_t* f_i, const KernelDesc* desc, const double* ivl, double2* values,
                         hipStream_t s)
{
    if (npieces <= 0) return;
    hipLaunchKernelGGL(k_table_values, dim3(grid_for(npieces * kNc, 256)), dim3(256), 0, s, t, N, p1, cut, rule, pt,
                       pc_f, pc_j, pc_p, npieces, f_k, f_i, desc, ivl, values);
}

void launch_table_coefs(const double2* values, int64_t npieces, double2* coef, hipStream_t s)
{
    if (npieces <= 0) return;
    hipLaunchKernelGGL(k_table_coefs, dim3(grid_for(npieces * kNc, 256)), dim3(256), 0, s, values, npieces, coef);
}

void launch_table_eval(TableView tv, int64_t n, const int32_t* k, const int32_t* i, const double* r, double* ps,
                       double* tps, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_table_eval, dim3(grid_for(n, 256)), dim3(256), 0, s, tv, n, k, i, r, ps, tps);
}

}  // namespace tdbem
