// Right-hand side, block matvec and the vector kernels of the FGMRES solver.
#include "tdbem_internal.hpp"

namespace tdbem {

// 7-point rule (identical definition to the assembly's; kept local to this translation unit).
__device__ inline void rhs_rule7(int q, double& l0, double& l1, double& l2, double& w)
{
    const double s15 = 3.872983346207416885;
    const double a1 = (6.0 - s15) / 21.0, a2 = (6.0 + s15) / 21.0;
    const double w1 = (155.0 - s15) / 1200.0, w2 = (155.0 + s15) / 1200.0;
    switch (q) {
    case 0: l0 = 1.0 / 3.0; l1 = 1.0 / 3.0; l2 = 1.0 / 3.0; w = 9.0 / 40.0; break;
    case 1: l0 = a1; l1 = a1; l2 = 1.0 - 2.0 * a1; w = w1; break;
    case 2: l0 = a1; l1 = 1.0 - 2.0 * a1; l2 = a1; w = w1; break;
    case 3: l0 = 1.0 - 2.0 * a1; l1 = a1; l2 = a1; w = w1; break;
    case 4: l0 = a2; l1 = a2; l2 = 1.0 - 2.0 * a2; w = w2; break;
    case 5: l0 = a2; l1 = 1.0 - 2.0 * a2; l2 = a2; w = w2; break;
    default: l0 = 1.0 - 2.0 * a2; l1 = a2; l2 = a2; w = w2; break;
    }
}

// dst = (float) src: the FP32 copy of an FP64 band for the inner products of the preconditioner.
__global__ void __launch_bounds__(256) k_to_f32(const double* __restrict__ src, float* __restrict__ dst, int64_t n)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) dst[s] = (float)src[s];
}

__global__ void __launch_bounds__(256) k_fill(double* __restrict__ x, double v, int64_t n)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) x[s] = v;
}

// g_k(l) = sum_tau |tau| sum_q w_q lam_a(q) (d.n_tau) int b_k'(t) G'(t - t0 - d.x_q) dt with
// G(s) = exp(-(s/w)^2): one lane per (k, tau); the time integral over supp b_k' is split at t_k
// and graded dyadically towards the split points like the kernel quadrature.
__global__ void __launch_bounds__(256)
k_rhs(GeomView g, const double* __restrict__ t, int N, int p1, int cut, TimeRule rule, double d0, double d1,
      double d2, double t0, double width, int M, double* __restrict__ gvec)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int E = g.E;
    if (gid >= (int64_t)N * p1 * E) return;
    const int k = (int)(gid / E), e = (int)(gid - (int64_t)k * E);
    const int kn = k / p1;                       // node of the test basis
    double pts[3];
    int np = 0;
    pts[np++] = t[kn > 0 ? kn - 1 : 0];
    if (kn > 0 && kn < N - 1) pts[np++] = t[kn];
    pts[np++] = t[kn < N - 1 ? kn + 1 : N - 1];
    const double dn = d0 * g.n[e] + d1 * g.n[E + e] + d2 * g.n[2 * E + e];
    const double iw2 = 1.0 / (width * width);
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    for (int q = 0; q < 7; ++q) {
        double l0, l1, l2, wq;
        rhs_rule7(q, l0, l1, l2, wq);
        const double dx = d0 * g.qp[(3 * q) * E + e] + d1 * g.qp[(3 * q + 1) * E + e] + d2 * g.qp[(3 * q + 2) * E + e];
        double ti = 0.0;
        for (int s = 0; s + 1 < np; ++s) {
            const double a = pts[s], len = pts[s + 1] - a;
            for (int gp = 0; gp < kTimePieces; ++gp) {
                const double pa = a + len * time_grading_edge(gp), pb = a + len * time_grading_edge(gp + 1);
                const double half = 0.5 * (pb - pa), mid = 0.5 * (pa + pb);
                for (int m = 0; m < kTimeGauss; ++m) {
                    const double tt = fma(half, rule.x[m], mid);
                    const double sa = tt - t0 - dx;
                    const double Gp = -2.0 * sa * iw2 * exp(-sa * sa * iw2);
                    double bv, b1, b2;
                    basis_eval(t, N, p1, cut, k, tt, bv, b1, b2);
                    ti = fma(half * rule.w[m] * Gp, b1, ti);
                }
            }
        }
        const double f = g.area[e] * wq * dn * ti;
        acc0 = fma(f, l0, acc0);
        acc1 = fma(f, l1, acc1);
        acc2 = fma(f, l2, acc2);
    }
    atomicAdd(gvec + (int64_t)k * M + g.v[e], acc0);
    atomicAdd(gvec + (int64_t)k * M + g.v[E + e], acc1);
    atomicAdd(gvec + (int64_t)k * M + g.v[2 * E + e], acc2);
}

// A load at a wave-uniform index through the constant address space, so that it becomes a
// scalar (SGPR) load: the vector memory pipeline is left to the matrix stream.
__device__ inline double load_uniform(const double* p, int idx)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return ((const __attribute__((address_space(4))) double*)p)[idx];
#else
    return p[idx];
#endif
}

// y = A[k0:k1, i0:i1] x on the lower-triangle band storage.  Block = one 64 x 64 vertex tile
// (rows l, columns j <= l) of one time row k, whose values are one contiguous stretch; wave w
// takes the 16 rows l = 64 tl + w + 4m, lanes the columns.  A stored entry (l, j) serves
// y_k(l) += A x_i(j) and, off the diagonal, y_k(j) += A x_i(l) (block symmetry).  Rows go two
// at a time: the band starts of the next two rows are loaded while the current two are in
// flight, and all their slots are issued before the FMAs.  Row partials are reduced over the
// lanes through LDS, column sums over the 4 waves; both are added atomically into y (zeroed
// before).
template <typename VT>
__global__ void __launch_bounds__(256)
k_matvec_tri(BandView band, const VT* __restrict__ val, int k0, int i0, int i1, const double* __restrict__ x,
             double* __restrict__ y)
{
    const int M = band.M;
    const int k = k0 + blockIdx.y;
    const int t = blockIdx.x;
    const int B = band.B[(int64_t)k * band.nt + t];
    if (B == 0) return;                        // no stored values in this (time row, tile)
    int tl = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((tl + 1) * (tl + 2) / 2 <= t) ++tl;
    while (tl * (tl + 1) / 2 > t) --tl;
    const int tj = t - tl * (tl + 1) / 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = tj * kBT + lane;
    const int16_t* __restrict__ il = band.ilo + ((int64_t)k * band.nt + t) * (kBT * kBT) + lane;
    const VT* __restrict__ vt = val + band.voff[(int64_t)k * band.nt + t] + lane;
    double* __restrict__ yk = y + (int64_t)(k - k0) * M;
    __shared__ double s_row[4][16][65];
    __shared__ double s_col[4][64];
    constexpr int kSlots = 8;    // slots of one row issued together
    // every load below is unconditional at an in-range address (tile entries outside the
    // triangle are stored zeros; lanes without a range read x at block i0, column <= M-1 and are
    // masked out), so the compiler issues the loads of two rows together and waits once
    const int je = j < M ? j : M - 1;
    double col = 0.0;
    int ibA = il[(wave + 0) * kBT], ibB = il[(wave + 4) * kBT];
    for (int m = 0; m < 16; m += 2) {
        const int nA = il[(wave + 4 * (m + 2 < 16 ? m + 2 : 14)) * kBT];
        const int nB = il[(wave + 4 * (m + 3 < 16 ? m + 3 : 15)) * kBT];
        double a[2][kSlots], bj[2][kSlots], bl[2][kSlots];
        int cnt[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int lr = wave + 4 * (m + h);
            const int l = tl * kBT + lr;
            const bool act = l < M && j <= l;
            const int ib = h ? ibB : ibA;
            const int lo = i0 - ib > 0 ? i0 - ib : 0;
            const int hi = i1 - ib < B ? i1 - ib : B;
            cnt[h] = act && hi > lo ? hi - lo : 0;
            const int s0 = cnt[h] ? lo : 0, ibe = cnt[h] ? ib : i0;
            const int top = cnt[h] ? cnt[h] - 1 : 0;
            const int le = l < M ? l : M - 1;
            const VT* __restrict__ v = vt + ((int64_t)lr * B + s0) * kBT;
            const double* __restrict__ xj = x + (int64_t)(ibe + s0 - i0) * M + je;
            // the row's value x_i(l) is the same for every lane when the band start is (the usual
            // case): then it is one scalar load per slot instead of a vector load
            const int ib0 = __builtin_amdgcn_readfirstlane(ibe);
            const int top0 = __builtin_amdgcn_readfirstlane(top);
            const bool uni = __ballot(ibe != ib0 || top != top0) == 0;
            if (uni) {
                const int xo = __builtin_amdgcn_readfirstlane((ib0 + s0 - i0) * M + le);
#pragma unroll
                for (int u = 0; u < kSlots; ++u) {
                    const int su = u < top0 ? u : top0;
                    a[h][u] = (double)v[su * kBT];
                    bj[h][u] = xj[(int64_t)su * M];
                    bl[h][u] = load_uniform(x, xo + su * M);
                }
            } else {
                const double* __restrict__ xl = x + (int64_t)(ibe + s0 - i0) * M + le;
#pragma unroll
                for (int u = 0; u < kSlots; ++u) {
                    const int su = u < top ? u : top;
                    a[h][u] = (double)v[su * kBT];
                    bj[h][u] = xj[(int64_t)su * M];
                    bl[h][u] = xl[(int64_t)su * M];
                }
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int lr = wave + 4 * (m + h);
            const int l = tl * kBT + lr;
            const bool off_diag = j < l;
            double row = 0.0, cl = 0.0;
#pragma unroll
            for (int u = 0; u < kSlots; ++u) {
                const double av = u < cnt[h] ? a[h][u] : 0.0;
                row = fma(av, bj[h][u], row);
                cl = fma(av, bl[h][u], cl);
            }
            // bands wider than kSlots (rare): the remaining slots one at a time
            if (cnt[h] > kSlots) {
                const int ib = h ? ibB : ibA;
                const int lo = i0 - ib > 0 ? i0 - ib : 0;
                const VT* __restrict__ v = vt + (int64_t)lr * B * kBT;
                const double* __restrict__ xj = x + (int64_t)(ib - i0) * M + j;
                const double* __restrict__ xl = x + (int64_t)(ib - i0) * M + l;
                for (int s = lo + kSlots; s < lo + cnt[h]; ++s) {
                    const double av = (double)v[s * kBT];
                    row = fma(av, xj[(int64_t)s * M], row);
                    cl = fma(av, xl[(int64_t)s * M], cl);
                }
            }
            col += off_diag ? cl : 0.0;
            s_row[wave][m + h][lane] = row;
        }
        ibA = nA;
        ibB = nB;
    }
    s_col[wave][lane] = col;
    __syncthreads();
    {
        // row sums: lane = (row m, quarter q) sums 16 lanes of its row, then the 4 quarters
        const int m = lane >> 2, q = lane & 3;
        double rs = 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) rs += s_row[wave][m][16 * q + u];
        rs += __shfl_xor(rs, 1, 64);
        rs += __shfl_xor(rs, 2, 64);
        const int l = tl * kBT + wave + 4 * m;
        if (q == 0 && l < M && rs != 0.0) atomicAdd(yk + l, rs);
    }
    if (wave == 0 && j < M) {
        const double c = s_col[0][lane] + s_col[1][lane] + s_col[2][lane] + s_col[3][lane];
        if (c != 0.0) atomicAdd(yk + j, c);
    }
}

// Partial dot products of w with nvec vectors V[q*ld + .]: block (b, q) sums its chunk.
constexpr int kDotBlock = 256;
constexpr int kDotChunk = 8192;

__global__ void __launch_bounds__(kDotBlock)
k_dots_partial(const double* __restrict__ V, int64_t n, int64_t ld, const double* __restrict__ w,
               double* __restrict__ partial, int nb)
{
    const int q = blockIdx.y;
    const int64_t begin = (int64_t)blockIdx.x * kDotChunk;
    const int64_t end = begin + kDotChunk < n ? begin + kDotChunk : n;
    const double* vq = V + (int64_t)q * ld;
    double acc = 0.0;
    for (int64_t s = begin + threadIdx.x; s < end; s += kDotBlock) acc = fma(vq[s], w[s], acc);
    __shared__ double red[kDotBlock / 64];
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int u = 0; u < kDotBlock / 64; ++u) t += red[u];
        partial[(int64_t)q * nb + blockIdx.x] = t;
    }
}

__global__ void __launch_bounds__(64)
k_dots_final(const double* __restrict__ partial, int nb, double* __restrict__ out)
{
    const int q = blockIdx.x;
    double acc = 0.0;
    for (int s = threadIdx.x; s < nb; s += 64) acc += partial[(int64_t)q * nb + s];
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (threadIdx.x == 0) out[q] = acc;
}

// w += sign * sum_q h[q] V[q*ld + .]
__global__ void __launch_bounds__(256)
k_sub_combination(double* __restrict__ w, const double* __restrict__ V, int nvec, int64_t n, int64_t ld,
                  const double* __restrict__ h, double sign)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    double acc = 0.0;
    for (int q = 0; q < nvec; ++q) acc = fma(h[q], V[(int64_t)q * ld + s], acc);
    w[s] = fma(sign, acc, w[s]);
}

__global__ void __launch_bounds__(256)
k_scale_copy(double* __restrict__ dst, const double* __restrict__ src, double a, int64_t n)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) dst[s] = a * src[s];
}

__global__ void __launch_bounds__(256)
k_axpby(double* __restrict__ y, const double* __restrict__ x, double a, double b, int64_t n)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) y[s] = b == 0.0 ? a * x[s] : fma(a, x[s], b * y[s]);
}

// dst = src / sqrt(*nrm2) (the normalisation of a new Krylov vector without a host round trip)
__global__ void __launch_bounds__(256)
k_scale_inv_sqrt(double* __restrict__ dst, const double* __restrict__ src, const double* __restrict__ nrm2, int64_t n)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double v = *nrm2;
    if (s < n) dst[s] = v > 0.0 ? src[s] / sqrt(v) : 0.0;
}

static inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_scale_inv_sqrt(double* dst, const double* src, const double* nrm2, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale_inv_sqrt, dim3(grid_for(n, 256)), dim3(256), 0, s, dst, src, nrm2, n);
}

void launch_fill(double* x, double v, int64_t n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256)), dim3(256), 0, s, x, v, n);
}

void launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n, 256)), dim3(256), 0, s, src, dst, n);
}

void launch_rhs(GeomView g, const double* t, int N, int p1, int cut, TimeRule rule, double d0, double d1, double d2,
                double t0, double width, int M, double* gvec, hipStream_t s)
{
    const int64_t L = (int64_t)N * p1;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(L * M, 256)), dim3(256), 0, s, gvec, 0.0, L * M);
    hipLaunchKernelGGL(k_rhs, dim3(grid_for(L * g.E, 256)), dim3(256), 0, s, g, t, N, p1, cut, rule, d0, d1, d2, t0,
                       width, M, gvec);
}

void launch_matvec(BandView band, const double* val, const float* valf, int k0, int k1, int i0, int i1,
                   const double* x, double* y, hipStream_t s)
{
    const int64_t M = band.M;
    const int64_t rows = (int64_t)(k1 - k0) * M;
    if (rows <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(rows, 256)), dim3(256), 0, s, y, 0.0, rows);
    const int T = (int)((M + 63) / 64);
    dim3 grid(T * (T + 1) / 2, k1 - k0);
    if (valf)
        hipLaunchKernelGGL(k_matvec_tri<float>, grid, dim3(256), 0, s, band, valf, k0, i0, i1, x, y);
    else
        hipLaunchKernelGGL(k_matvec_tri<double>, grid, dim3(256), 0, s, band, val, k0, i0, i1, x, y);
}

int dots_partial_blocks(int64_t n) { return (int)((n + kDotChunk - 1) / kDotChunk); }

void launch_dots(const double* V, int nvec, int64_t n, int64_t ld, const double* w, double* partial, double* out,
                 hipStream_t s)
{
    const int nb = dots_partial_blocks(n);
    hipLaunchKernelGGL(k_dots_partial, dim3(nb, nvec), dim3(kDotBlock), 0, s, V, n, ld, w, partial, nb);
    hipLaunchKernelGGL(k_dots_final, dim3(nvec), dim3(64), 0, s, partial, nb, out);
}

void launch_sub_combination(double* w, const double* V, int nvec, int64_t n, int64_t ld, const double* h, double sign,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_sub_combination, dim3(grid_for(n, 256)), dim3(256), 0, s, w, V, nvec, n, ld, h, sign);
}

void launch_scale_copy(double* dst, const double* src, double a, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n, 256)), dim3(256), 0, s, dst, src, a, n);
}

void launch_axpby(double* y, const double* x, double a, double b, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(n, 256)), dim3(256), 0, s, y, x, a, b, n);
}

}  // namespace tdbem
