// Retarded double layer potential of eq. (RetardedPotential): the solution u(x, t) off the
// surface from the density phi(y, t) = sum_i sum_j alpha_i(j) b_i(t) phi_j(y),
//   u(x, t) = -1/(4 pi) int_Gamma (n_y . (x - y)) / r * ( phi(y, t - r) / r^2 + d_t phi(y, t - r) / r ),
// r = |x - y|, with the 7-point rule on every flat triangle.  At a retarded time t - r in
// [t_i0, t_i0+1) only b_i0 and b_i0+1 are nonzero (p = 0, one basis per node).
#include "tdbem_internal.hpp"

namespace tdbem {

// The 7-point rule of the assembly (Radon; Stroud T2:5-1), in the same point order as the
// quadrature points of the geometry arrays: centroid weight 9/40, orbits (a,a,1-2a) with
// a = (6 -/+ sqrt 15)/21 and weights (155 -/+ sqrt 15)/1200.
__device__ inline void pot_rule7(int q, double& l0, double& l1, double& l2, double& w)
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

constexpr int kPotTimes = 8;     // evaluation times per lane
constexpr int kPotTri = 64;      // triangles staged in LDS per pass
constexpr int kPotMaxN = 1024;   // time nodes staged in LDS (the entry point rejects more)

// phiq[(e*7 + q)*N + i] = sum_a lam_a(q) alpha[i*M + v_a(e)]: the density of b_i at point q of e.
__global__ void __launch_bounds__(256)
k_potential_density(GeomView g, int N, int M, const double* __restrict__ alpha, double* __restrict__ phiq)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)g.E * 7 * N;
    if (s >= total) return;
    const int i = (int)(s % N);
    const int64_t eq = s / N;
    const int q = (int)(eq % 7), e = (int)(eq / 7);
    double l0, l1, l2, w;
    pot_rule7(q, l0, l1, l2, w);
    const double* ai = alpha + (int64_t)i * M;
    phiq[s] = l0 * ai[g.v[e]] + l1 * ai[g.v[g.E + e]] + l2 * ai[g.v[2 * g.E + e]];
}

// Lane = evaluation point, kPotTimes consecutive times per workgroup column; triangles are
// streamed through LDS (quadrature points, normal, weight -|tau| w_q / (4 pi)).
__global__ void __launch_bounds__(256)
k_potential(GeomView g, const double* __restrict__ tg, int N, int cut, const double* __restrict__ phiq,
            int64_t npts, const double* __restrict__ pts, int ntimes, const double* __restrict__ times,
            double* __restrict__ u)
{
    __shared__ double sy[kPotTri][7][3];
    __shared__ double sc[kPotTri][7];
    __shared__ double sn[kPotTri][3];
    __shared__ double tsh[kPotMaxN];
    for (int z = threadIdx.x; z < N; z += blockDim.x) tsh[z] = tg[z];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int s0 = blockIdx.y * kPotTimes;
    const int E = g.E;
    double x0 = 0.0, x1 = 0.0, x2 = 0.0;
    if (p < npts) { x0 = pts[3 * p]; x1 = pts[3 * p + 1]; x2 = pts[3 * p + 2]; }
    double ts[kPotTimes], acc[kPotTimes];
#pragma unroll
    for (int s = 0; s < kPotTimes; ++s) {
        ts[s] = s0 + s < ntimes ? times[s0 + s] : -1.0;   // past the end: no retarded time >= 0
        acc[s] = 0.0;
    }
    for (int e0 = 0; e0 < E; e0 += kPotTri) {
        __syncthreads();
        for (int z = threadIdx.x; z < kPotTri * 7; z += blockDim.x) {
            const int a = z / 7, q = z % 7, e = e0 + a;
            double y0 = 0.0, y1 = 0.0, y2 = 0.0, c = 0.0;
            if (e < E) {
                y0 = g.qp[(3 * q) * E + e];
                y1 = g.qp[(3 * q + 1) * E + e];
                y2 = g.qp[(3 * q + 2) * E + e];
                double l0, l1, l2, w;
                pot_rule7(q, l0, l1, l2, w);
                c = -g.area[e] * w * 0.07957747154594767;     // -|tau| w_q / (4 pi)
            }
            sy[a][q][0] = y0; sy[a][q][1] = y1; sy[a][q][2] = y2;
            sc[a][q] = c;
        }
        for (int z = threadIdx.x; z < kPotTri * 3; z += blockDim.x) {
            const int a = z / 3, c = z % 3, e = e0 + a;
            sn[a][c] = e < E ? g.n[c * E + e] : 0.0;
        }
        __syncthreads();
        const int ne = E - e0 < kPotTri ? E - e0 : kPotTri;
        for (int a = 0; a < ne; ++a) {
            const double n0 = sn[a][0], n1 = sn[a][1], n2 = sn[a][2];
            for (int q = 0; q < 7; ++q) {
                const double d0 = x0 - sy[a][q][0], d1 = x1 - sy[a][q][1], d2 = x2 - sy[a][q][2];
                const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                const double r = sqrt(r2);
                const double ir = 1.0 / r;
                const double f = sc[a][q] * (n0 * d0 + n1 * d1 + n2 * d2) * ir;
                const double* __restrict__ ph = phiq + ((int64_t)(e0 + a) * 7 + q) * N;
#pragma unroll
                for (int s = 0; s < kPotTimes; ++s) {
                    const double tr = ts[s] - r;
                    if (!(tr > 0.0)) continue;
                    // interval [t_lo, t_lo+1) holding tr (tr < t_{N-1} since r > 0 and t <= T)
                    int lo = 0, hi = N - 1;
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (tsh[mid] <= tr) lo = mid;
                        else hi = mid;
                    }
                    // on that interval b_lo = 1 - F(u) and b_lo+1 = F(u), u = (tr - t_lo)/h, one
                    // cutoff evaluation for both; b_0 carries the causal factor 8 (t/h_1)^2
                    const double ih = 1.0 / (tsh[lo + 1] - tsh[lo]);
                    const double uu = (tr - tsh[lo]) * ih;
                    double F, F1, F2;
                    cutoff_eval(cut, uu, F, F1, F2);
                    double b0 = 1.0 - F, db0 = -F1 * ih;
                    const double b1 = F, db1 = F1 * ih;
                    if (lo == 0) {
                        const double c = 8.0 * uu * uu, c1 = 16.0 * uu * ih;
                        db0 = c1 * b0 + c * db0;
                        b0 = c * b0;
                    }
                    const double pa = ph[lo], pb = ph[lo + 1];
                    const double phi = b0 * pa + b1 * pb, dphi = db0 * pa + db1 * pb;
                    acc[s] = fma(f, (phi * ir + dphi) * ir, acc[s]);
                }
            }
        }
    }
    if (p < npts) {
#pragma unroll
        for (int s = 0; s < kPotTimes; ++s)
            if (s0 + s < ntimes) u[(int64_t)(s0 + s) * npts + p] = acc[s];
    }
}

void launch_potential(GeomView g, const double* t, int N, int cut, int M, const double* alpha, double* phiq,
                      int64_t npts, const double* pts, int ntimes, const double* times, double* u, hipStream_t s)
{
    const int64_t nq = (int64_t)g.E * 7 * N;
    hipLaunchKernelGGL(k_potential_density, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, g, N, M, alpha, phiq);
    dim3 grid((unsigned)((npts + 255) / 256), (unsigned)((ntimes + kPotTimes - 1) / kPotTimes));
    hipLaunchKernelGGL(k_potential, grid, dim3(256), 0, s, g, t, N, cut, phiq, npts, pts, ntimes, times, u);
}

}  // namespace tdbem
