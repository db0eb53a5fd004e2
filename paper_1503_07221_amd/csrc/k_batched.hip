// Block matvec for many right-hand sides at once: Y_r = A X_r, r < nrhs, on the lower-triangle
// band storage (Section 3.2).  The single-vector product streams every stored value from HBM for
// two FMAs; here a value is read once per group of kRC right-hand sides and serves 2 kRC FMAs,
// which moves the product from the HBM bound towards the FP64 ALU bound.
#include "tdbem_internal.hpp"

namespace tdbem {

constexpr int kRC = 8;        // right-hand sides per workgroup pass
constexpr int kSlotChunk = 8; // band slots loaded together

__device__ inline double wave_sum(double v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Workgroup = (vertex tile t, time row k, group of kRC right-hand sides); wave w takes the rows
// l = 64 tl + w + 4m, lanes the columns j.  A stored a = A_{k,i}(l, j), j <= l, adds a X_i(j) to
// the row sum of (k, l) and, off the diagonal, a X_i(l) to the column sum of (k, j), for every
// right-hand side of the group.  Row sums are reduced over the wave (one atomic per row and
// right-hand side), column sums over the 4 waves through LDS.
template <typename VT>
__global__ void __launch_bounds__(256)
k_matvec_multi(BandView band, const VT* __restrict__ val, int nrhs, const double* __restrict__ X, int64_t ldx,
               double* __restrict__ Y, int64_t ldy)
{
    const int M = band.M, N = band.N;
    const int k = blockIdx.y;
    const int t = blockIdx.x;
    const int r0 = blockIdx.z * kRC;
    const int nr = nrhs - r0 < kRC ? nrhs - r0 : kRC;
    const int B = band.B[(int64_t)k * band.nt + t];
    if (B == 0) return;
    int tl = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((tl + 1) * (tl + 2) / 2 <= t) ++tl;
    while (tl * (tl + 1) / 2 > t) --tl;
    const int tj = t - tl * (tl + 1) / 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = tj * kBT + lane;
    const int je = j < M ? j : M - 1;
    const int16_t* __restrict__ il = band.ilo + ((int64_t)k * band.nt + t) * (kBT * kBT) + lane;
    const VT* __restrict__ vt = val + band.voff[(int64_t)k * band.nt + t] + lane;
    __shared__ double s_col[4][kRC][kBT];
    double col[kRC];
#pragma unroll
    for (int rr = 0; rr < kRC; ++rr) col[rr] = 0.0;
    for (int m = 0; m < 16; ++m) {
        const int lr = wave + 4 * m;
        const int l = tl * kBT + lr;
        if (l >= M) break;
        const bool act = j <= l;
        const bool off = j < l;
        const int ib = il[lr * kBT];
        const int lo = ib < 0 ? -ib : 0;
        const int hi = N - ib < B ? N - ib : B;
        const VT* __restrict__ v = vt + (int64_t)lr * B * kBT;
        double row[kRC];
#pragma unroll
        for (int rr = 0; rr < kRC; ++rr) row[rr] = 0.0;
        for (int s0 = 0; s0 < B; s0 += kSlotChunk) {
            double a[kSlotChunk];
            int xi[kSlotChunk];
#pragma unroll
            for (int u = 0; u < kSlotChunk; ++u) {
                const int s = s0 + u;
                const bool in = act && s >= lo && s < hi;
                a[u] = in ? (double)v[(s < B ? s : B - 1) * kBT] : 0.0;
                const int ii = ib + s;
                xi[u] = in ? ii : 0;             // masked slots read block 0 and multiply by 0
            }
#pragma unroll
            for (int rr = 0; rr < kRC; ++rr) {
                if (rr >= nr) break;
                const double* __restrict__ Xr = X + (int64_t)(r0 + rr) * ldx;
                double rs = row[rr], cs = 0.0;
#pragma unroll
                for (int u = 0; u < kSlotChunk; ++u) {
                    const int64_t base = (int64_t)xi[u] * M;
                    rs = fma(a[u], Xr[base + je], rs);
                    cs = fma(a[u], Xr[base + l], cs);
                }
                row[rr] = rs;
                col[rr] += off ? cs : 0.0;
            }
        }
#pragma unroll
        for (int rr = 0; rr < kRC; ++rr) {
            if (rr >= nr) break;
            const double rs = wave_sum(row[rr]);
            if (lane == 0 && rs != 0.0) atomicAdd(Y + (int64_t)(r0 + rr) * ldy + (int64_t)k * M + l, rs);
        }
    }
#pragma unroll
    for (int rr = 0; rr < kRC; ++rr) s_col[wave][rr][lane] = col[rr];
    __syncthreads();
    if (wave == 0 && j < M) {
        for (int rr = 0; rr < nr; ++rr) {
            const double cs = s_col[0][rr][lane] + s_col[1][rr][lane] + s_col[2][rr][lane] + s_col[3][rr][lane];
            if (cs != 0.0) atomicAdd(Y + (int64_t)(r0 + rr) * ldy + (int64_t)k * M + j, cs);
        }
    }
}

__global__ void __launch_bounds__(256)
k_fill_strided(double* __restrict__ Y, int64_t ldy, int64_t n, int nrhs)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n * nrhs) return;
    const int64_t r = s / n;
    Y[r * ldy + (s - r * n)] = 0.0;
}

void launch_matvec_multi(BandView band, const double* val, const float* valf, int nrhs, const double* X, int64_t ldx,
                         double* Y, int64_t ldy, hipStream_t s)
{
    const int64_t n = (int64_t)band.N * band.M;
    if (nrhs <= 0 || n == 0) return;
    hipLaunchKernelGGL(k_fill_strided, dim3((unsigned)((n * nrhs + 255) / 256)), dim3(256), 0, s, Y, ldy, n, nrhs);
    dim3 grid((unsigned)band.nt, (unsigned)band.N, (unsigned)((nrhs + kRC - 1) / kRC));
    if (valf)
        hipLaunchKernelGGL(k_matvec_multi<float>, grid, dim3(256), 0, s, band, valf, nrhs, X, ldx, Y, ldy);
    else
        hipLaunchKernelGGL(k_matvec_multi<double>, grid, dim3(256), 0, s, band, val, nrhs, X, ldx, Y, ldy);
}

}  // namespace tdbem
