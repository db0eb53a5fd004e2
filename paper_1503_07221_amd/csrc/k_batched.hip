// Block matvec for many right-hand sides at once: Y_r = A X_r, r < nrhs, on the lower-triangle
// band storage (Section 3.2).  The single-vector product streams every stored value from HBM for
// two FMAs; here a value is read once per group of RC right-hand sides and serves 2 RC FMAs.
// The trial values of a tile's columns are staged in LDS, whose size ties the group size RC to the
// staged trial range SPAN; tiles with a wider range read them from memory.  Which (RC, SPAN) is
// fastest depends on the operator's band widths, so the host times the variants on the operator
// at hand (4 right-hand sides over 24 indices, 48 KB, on the 5120-triangle sphere: 1.9 ms per
// right-hand side against 3.75 ms for the single product).
#include "tdbem_internal.hpp"

namespace tdbem {


__device__ inline double wave_sum(double v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

constexpr int kSlotGroup = 4; // band slots whose values are loaded together

// One row l of a tile: for every band slot s (values loaded kSlotGroup at a time) and right-hand
// side rr, row[rr] += a X_{ib+s}(j) and col[rr] += a X_{ib+s}(l) off the diagonal.  STAGED: X_i(j)
// from the LDS tile xs[rr][i - ibase][lane]; UNI: the band start is the same on every active lane,
// so the trial index of a slot is wave-uniform and X_i(l) one request per wave.  Right-hand sides
// beyond nr reuse the first one (their sums are dropped by the caller).
template <bool STAGED, bool UNI, typename VT, int RC, int SPAN>
__device__ inline void row_pass(const VT* __restrict__ v, int B, bool act, bool off, int ib, int ib0, int slo, int shi,
                                int ibase, int span, int N, int M, int l, int je, int lane, int nr, int r0,
                                const double* __restrict__ X, int64_t ldx, const double (*xs)[SPAN][kBT],
                                double (&row)[RC], double (&col)[RC])
{
    for (int s0 = 0; s0 < B; s0 += kSlotGroup) {
        double a[kSlotGroup];
        int ii[kSlotGroup];
#pragma unroll
        for (int u = 0; u < kSlotGroup; ++u) {
            const int s = s0 + u;
            const bool in = act && s >= slo && s < shi;
            a[u] = in ? (double)v[(s < B ? s : B - 1) * kBT] : 0.0;
            if (UNI) {
                const int iu = ib0 + s;
                ii[u] = __builtin_amdgcn_readfirstlane(iu < 0 ? 0 : (iu < N ? iu : N - 1));
            } else {
                ii[u] = in ? ib + s : (STAGED ? ibase : 0);   // masked slots: 0 times a valid value
            }
        }
#pragma unroll
        for (int u = 0; u < kSlotGroup; ++u) {
            const double ao = off ? a[u] : 0.0;
            // with UNI every active lane has ib = ib0, so ii is its trial index (a = 0 elsewhere)
            // (masked slots of a uniform row are clamped into the staged rows: 0 times a finite value)
            const int si = STAGED ? (UNI ? (ii[u] - ibase < 0 ? 0 : (ii[u] - ibase < span ? ii[u] - ibase : span - 1))
                                         : ii[u] - ibase)
                                  : 0;
#pragma unroll
            for (int rr = 0; rr < RC; ++rr) {
                const double* __restrict__ Xr = X + (int64_t)(rr < nr ? r0 + rr : r0) * ldx;
                double xj, xl;
                if (STAGED) xj = xs[rr < nr ? rr : 0][si][lane];
                else xj = Xr[(int64_t)ii[u] * M + je];
                // a vector load at a lane-uniform address (one request): a scalar load here would
                // share the LDS counter and serialise the LDS reads of xj behind it
                xl = Xr[(int64_t)ii[u] * M + l];
                row[rr] = fma(a[u], xj, row[rr]);
                col[rr] = fma(ao, xl, col[rr]);
            }
        }
    }
}

// Workgroup = (vertex tile t, time row k, group of RC right-hand sides); wave w takes the rows
// l = 64 tl + w + 4m, lanes the columns j.  A stored a = A_{k,i}(l, j), j <= l, adds a X_i(j) to
// the row sum of (k, l) and, off the diagonal, a X_i(l) to the column sum of (k, j), for every
// right-hand side of the group.  The trial values X_i(j) of the tile's columns over its trial
// range [ibase, ibase + span) are staged in LDS once (span <= SPAN; wider tiles read them from
// memory); X_i(l) is one load at a lane-uniform address.  Row sums are reduced over the wave (one
// atomic per row and right-hand side), column sums over the 4 waves.
template <typename VT, int RC, int SPAN>
__global__ void __launch_bounds__(256)
k_matvec_multi(BandView band, const VT* __restrict__ val, int nrhs, const double* __restrict__ X, int64_t ldx,
               double* __restrict__ Y, int64_t ldy)
{
    const int M = band.M, N = band.N;
    const int k = blockIdx.y;
    const int t = blockIdx.x;
    const int r0 = blockIdx.z * RC;
    const int nr = nrhs - r0 < RC ? nrhs - r0 : RC;
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
    __shared__ double xs[RC][SPAN][kBT];      // after the main loop: the column sums [4][RC][64]
    __shared__ int s_range[4][2];
    // trial range of the tile's stored slots
    int lo = 0x7fffffff, hi = -0x7fffffff;
    for (int m = 0; m < 16; ++m) {
        const int lr = wave + 4 * m;
        const int l = tl * kBT + lr;
        if (l < M && j <= l) {
            const int ib = il[lr * kBT];
            lo = min(lo, max(ib, 0));
            hi = max(hi, min(ib + B, N));
        }
    }
    for (int o = 32; o >= 1; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o, 64));
        hi = max(hi, __shfl_xor(hi, o, 64));
    }
    if (lane == 0) { s_range[wave][0] = lo; s_range[wave][1] = hi; }
    __syncthreads();
    const int ibase = min(min(s_range[0][0], s_range[1][0]), min(s_range[2][0], s_range[3][0]));
    const int itop = max(max(s_range[0][1], s_range[1][1]), max(s_range[2][1], s_range[3][1]));
    const int span = itop - ibase;
    const bool staged = span > 0 && span <= SPAN;
    if (staged) {
        for (int e = threadIdx.x; e < nr * span * kBT; e += 256) {
            const int rr = e / (span * kBT), rest = e - rr * span * kBT, si = rest / kBT, c = rest % kBT;
            const int jj = tj * kBT + c;
            xs[rr][si][c] = jj < M ? X[(int64_t)(r0 + rr) * ldx + (int64_t)(ibase + si) * M + jj] : 0.0;
        }
    }
    __syncthreads();
    double col[RC];
#pragma unroll
    for (int rr = 0; rr < RC; ++rr) col[rr] = 0.0;
    for (int m = 0; m < 16; ++m) {
        const int lr = wave + 4 * m;
        const int l = tl * kBT + lr;
        if (l >= M) break;
        const bool act = j <= l;
        const bool off = j < l;
        const int ib = il[lr * kBT];
        const int slo = ib < 0 ? -ib : 0;
        const int shi = N - ib < B ? N - ib : B;
        const unsigned long long am = __ballot(act);
        if (am == 0) continue;
        const int first = __ffsll((long long)am) - 1;
        const int ib0 = __shfl(ib, first, 64);
        const bool uni = __ballot(act && ib != ib0) == 0;
        const VT* __restrict__ v = vt + (int64_t)lr * B * kBT;
        double row[RC];
#pragma unroll
        for (int rr = 0; rr < RC; ++rr) row[rr] = 0.0;
        // wave-uniform choice of where the trial values come from
        if (staged) {
            if (uni) row_pass<true, true, VT, RC, SPAN>(v, B, act, off, ib, ib0, slo, shi, ibase, span, N, M, l, je, lane, nr, r0, X, ldx, xs, row, col);
            else row_pass<true, false, VT, RC, SPAN>(v, B, act, off, ib, ib0, slo, shi, ibase, span, N, M, l, je, lane, nr, r0, X, ldx, xs, row, col);
        } else {
            if (uni) row_pass<false, true, VT, RC, SPAN>(v, B, act, off, ib, ib0, slo, shi, ibase, span, N, M, l, je, lane, nr, r0, X, ldx, xs, row, col);
            else row_pass<false, false, VT, RC, SPAN>(v, B, act, off, ib, ib0, slo, shi, ibase, span, N, M, l, je, lane, nr, r0, X, ldx, xs, row, col);
        }
#pragma unroll
        for (int rr = 0; rr < RC; ++rr) {
            if (rr >= nr) break;
            const double rs = wave_sum(row[rr]);
            if (lane == 0 && rs != 0.0) atomicAdd(Y + (int64_t)(r0 + rr) * ldy + (int64_t)k * M + l, rs);
        }
    }
    static_assert(RC * SPAN >= 4 * RC, "column sums reuse the staging array");
    double (*s_col)[RC][kBT] = reinterpret_cast<double (*)[RC][kBT]>(&xs[0][0][0]);
    __syncthreads();                             // every wave is done with the staged values
#pragma unroll
    for (int rr = 0; rr < RC; ++rr) s_col[wave][rr][lane] = col[rr];
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

// Variants (right-hand sides per pass RC, staged trial range SPAN), 24-48 KB of LDS each.
struct MultiVariant { int rc, span; };
static const MultiVariant kMultiVariants[] = {{4, 24}, {2, 48}, {8, 12}, {4, 16}, {2, 24}};

int matvec_multi_variants() { return (int)(sizeof(kMultiVariants) / sizeof(kMultiVariants[0])); }
int matvec_multi_variant_rc(int v) { return kMultiVariants[v].rc; }
int matvec_multi_variant_span(int v) { return kMultiVariants[v].span; }

template <int RC, int SPAN>
static void launch_variant(BandView band, const double* val, const float* valf, int nrhs, const double* X, int64_t ldx,
                           double* Y, int64_t ldy, hipStream_t s)
{
    dim3 grid((unsigned)band.nt, (unsigned)band.N, (unsigned)((nrhs + RC - 1) / RC));
    if (valf)
        hipLaunchKernelGGL((k_matvec_multi<float, RC, SPAN>), grid, dim3(256), 0, s, band, valf, nrhs, X, ldx, Y, ldy);
    else
        hipLaunchKernelGGL((k_matvec_multi<double, RC, SPAN>), grid, dim3(256), 0, s, band, val, nrhs, X, ldx, Y, ldy);
}

void launch_matvec_multi(BandView band, const double* val, const float* valf, int nrhs, const double* X, int64_t ldx,
                         double* Y, int64_t ldy, int variant, hipStream_t s)
{
    const int64_t n = (int64_t)band.N * band.M;
    if (nrhs <= 0 || n == 0) return;
    hipLaunchKernelGGL(k_fill_strided, dim3((unsigned)((n * nrhs + 255) / 256)), dim3(256), 0, s, Y, ldy, n, nrhs);
    switch (variant) {
    case 1: launch_variant<2, 48>(band, val, valf, nrhs, X, ldx, Y, ldy, s); break;
    case 2: launch_variant<8, 12>(band, val, valf, nrhs, X, ldx, Y, ldy, s); break;
    case 3: launch_variant<4, 16>(band, val, valf, nrhs, X, ldx, Y, ldy, s); break;
    case 4: launch_variant<2, 24>(band, val, valf, nrhs, X, ldx, Y, ldy, s); break;
    default: launch_variant<4, 24>(band, val, valf, nrhs, X, ldx, Y, ldy, s); break;
    }
}

}  // namespace tdbem
