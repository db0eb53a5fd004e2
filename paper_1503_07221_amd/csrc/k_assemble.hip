// Assembly of the blocks A_{k,i} (eq. (MatrixEntries)) on gfx950.
//
//   k_geometry   per-triangle structure of arrays (normal, area, surface curls, 7 points)
//   k_layout     band layout: per (k, l, j) the first trial index i whose kernel support meets
//                the conservative distance range of the two hats (eq. (SparsitySmallBlock))
//   k_regular    pairs without a common vertex: 7 x 7 point pairs, all (k, i) with r in supp
//   k_singular   coincident / common-edge / common-vertex pairs: Sauter-Schwab rules
// Every unordered pair {tau < sigma} is integrated once with tau as the x-triangle and its local
// 3 x 3 block is added to A(v_b(sigma), v_a(tau)) and, by the symmetry of the kernel in
// x <-> y, to A(v_a(tau), v_b(sigma)); a coincident pair adds its symmetrised block once.  The
// kernels add only the first of the two (a coincident block halved) into P, A = P + P^T, which
// the lower-triangle storage forms on the fly (scatter_half).
#include "tdbem_internal.hpp"

namespace tdbem {

// 7-point degree-5 rule (Radon; Stroud T2:5-1): centroid weight 9/40, orbits (a,a,1-2a) with
// a = (6 -/+ sqrt 15)/21 and weights (155 -/+ sqrt 15)/1200 (weights sum to 1).
__host__ __device__ inline void rule7_point(int q, double& l0, double& l1, double& l2, double& w)
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

__global__ void __launch_bounds__(256)
k_geometry(const double* __restrict__ xyz, const int32_t* __restrict__ tri, int E, double* __restrict__ P,
           double* __restrict__ nrm, double* __restrict__ area, double* __restrict__ curl,
           double* __restrict__ qp, int32_t* __restrict__ vid)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    double X[3][3];
    for (int a = 0; a < 3; ++a) {
        const int v = tri[3 * e + a];
        vid[a * E + e] = v;
        for (int c = 0; c < 3; ++c) {
            X[a][c] = xyz[3 * v + c];
            P[(3 * a + c) * E + e] = X[a][c];
        }
    }
    const double u0 = X[1][0] - X[0][0], u1 = X[1][1] - X[0][1], u2 = X[1][2] - X[0][2];
    const double w0 = X[2][0] - X[0][0], w1 = X[2][1] - X[0][1], w2 = X[2][2] - X[0][2];
    const double c0 = u1 * w2 - u2 * w1, c1 = u2 * w0 - u0 * w2, c2 = u0 * w1 - u1 * w0;
    const double len = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    nrm[e] = c0 / len;
    nrm[E + e] = c1 / len;
    nrm[2 * E + e] = c2 / len;
    const double ar = 0.5 * len;
    area[e] = ar;
    for (int a = 0; a < 3; ++a) {
        const int p = (a + 1) % 3, q = (a + 2) % 3;
        for (int c = 0; c < 3; ++c) curl[(3 * a + c) * E + e] = -(X[q][c] - X[p][c]) / (2.0 * ar);
    }
    for (int q = 0; q < 7; ++q) {
        double l0, l1, l2, w;
        rule7_point(q, l0, l1, l2, w);
        for (int c = 0; c < 3; ++c) qp[(3 * q + c) * E + e] = l0 * X[0][c] + l1 * X[1][c] + l2 * X[2][c];
    }
}

// Band of trial indices i for the time row k and a distance range (dmin, dmax): those with
// lo_{k,i} < dmax and hi_{k,i} > dmin.  Both bounds move right with k (two pointers).  Block
// (j chunk, l); lanes with j > l idle (lower triangle only).
__global__ void __launch_bounds__(256)
k_layout(const double* __restrict__ xyz, const double* __restrict__ rho, int M, const double* __restrict__ t,
         int N, int16_t* __restrict__ ilo, int32_t* __restrict__ Bk)
{
    extern __shared__ int32_t sB[];
    for (int k = threadIdx.x; k < N; k += blockDim.x) sB[k] = 0;
    __syncthreads();
    const int l = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ntri = (int64_t)M * (M + 1) / 2;
    if (j <= l) {
        const double dx = xyz[3 * l] - xyz[3 * j], dy = xyz[3 * l + 1] - xyz[3 * j + 1], dz = xyz[3 * l + 2] - xyz[3 * j + 2];
        const double d = sqrt(dx * dx + dy * dy + dz * dz);
        const double slack = 1e-12 * (1.0 + t[N - 1]);
        const double dmax = d + rho[l] + rho[j] + slack;
        double dmin = d - rho[l] - rho[j] - slack;
        dmin = dmin > 0.0 ? dmin : 0.0;
        int ia = 0, ib = -1;
        for (int k = 0; k < N; ++k) {
            while (ia < N) {
                double lo, hi;
                kernel_support(t, N, k, ia, lo, hi);
                if (lo < dmax) break;
                ++ia;
            }
            while (ib + 1 < N) {
                double lo, hi;
                kernel_support(t, N, k, ib + 1, lo, hi);
                if (!(hi > dmin)) break;
                ++ib;
            }
            const int first = ia < N ? ia : N - 1;
            ilo[(int64_t)k * ntri + tri_index(l, j)] = (int16_t)first;
            const int cnt = ib - ia + 1;
            if (cnt > 0) atomicMax(&sB[k], cnt);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < N; k += blockDim.x)
        if (sB[k] > 0) atomicMax(&Bk[k], sB[k]);
}

__device__ inline double wave_min(double v)
{
    for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline double wave_max(double v)
{
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline unsigned long long wave_sum_u64(unsigned long long v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the 8 lanes of a group (one triangle pair).
__device__ inline double group8_sum(double v)
{
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    return v;
}

// P(l, j) += v for the half P of the assembly (A = P + P^T): in the lower-triangle storage an
// off-diagonal contribution lands at (max, min) and a diagonal one counts twice.
__device__ inline void scatter_half(const BandView& band, double* val, float* valf, int k, int i, int l, int j,
                                    double v)
{
    if (j > l) { const int tmp = j; j = l; l = tmp; }
    if (j == l) v *= 2.0;
    const int s = i - (int)band.ilo[(int64_t)k * band.ntri + tri_index(l, j)];
    const int B = band.B[k];
    if (s < 0 || s >= B) return;   // outside the band: the value is zero (support test)
    const int64_t idx = band_value_index(band, k, l, j, s, B);
    if (valf) atomicAdd(valf + idx, (float)v);
    else atomicAdd(val + idx, v);
}

// Number of keys of the ascending array key[0..n) below v (key < v, or key <= v when le): the
// 64 lanes sample evenly spaced keys and the ballot narrows the range (2 rounds for n <= 4096).
// Every lane returns the same value.
__device__ inline int wave_count_below(const double* key, int n, double v, bool le)
{
    const int lane = threadIdx.x & 63;
    int base = 0, len = n;
    while (len > 64) {
        const int step = (len + 63) / 64;
        const int p = base + lane * step;
        const bool below = p < base + len && (le ? key[p] <= v : key[p] < v);
        const int cnt = __popcll(__ballot(below));
        if (cnt == 0) return base;
        const int lo = base + (cnt - 1) * step + 1;
        const int hi = base + cnt * step < base + len ? base + cnt * step : base + len;
        base = lo;
        len = hi - lo;
    }
    const bool below = lane < len && (le ? key[base + lane] <= v : key[base + lane] < v);
    return base + __popcll(__ballot(below));
}

// One sorted element of the support range: locate its piece, evaluate both series and store
// psi(r) w_q w_q'/r and tpsi(r) w_q w_q'/r at the element's own index.
__device__ inline void eval_sorted_element(const KernelDesc& kd, const double* __restrict__ iv, const TableView& tv,
                                           const PieceTable& spt, double r, int e, double w, double r_far,
                                           double* s_P, double* s_Pt)
{
    int j = 0;
    for (int m = 1; m < kd.nint; ++m) j += r >= iv[2 * m] ? 1 : 0;
    double fr = (r - iv[2 * j]) * iv[2 * j + 1];
    fr = fr < 0.0 ? 0.0 : (fr > 1.0 ? 1.0 : fr);
    int cell = (int)(fr * kLutCells);
    cell = cell < kLutCells ? cell : kLutCells - 1;
    int p = spt.lut[cell];
    if (p + 1 < kPieces && fr >= spt.edge[p + 1]) ++p;
    const double x = 2.0 * (fr - spt.edge[p]) * spt.inv_width[p] - 1.0;
    const int64_t off = kd.coef_off + (int64_t)(j * kPieces + p) * kNc;
    double ps, pt;
    // mixed precision: far-field distances on the middle pieces (away from the flat support
    // edges) evaluate the FP32 copy of the series
    if (r >= r_far && p >= kPieces / 2 - 3 && p < kPieces / 2 + 3) {
        float fps, fpt;
        clenshaw2_f32(tv.coef32 + off, (float)x, fps, fpt);
        ps = fps;
        pt = fpt;
    } else {
        clenshaw2(tv.coef + off, x, ps, pt);
    }
    s_P[e] = ps * w;
    s_Pt[e] = pt * w;
}

// Wave-scope ordering of LDS accesses between lanes of one wave (no block barrier).
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Regular pairs, wave-independent sorted form.  Every wave owns 8 consecutive sigma of one tau
// (392 point pairs), sorts their distances once in its own LDS region, and then runs the
// (k, i) loop on its own: the point pairs inside supp psi_{k,i} are one contiguous range of the
// sorted list, consecutive lanes take consecutive distances (their Chebyshev pieces mostly
// coincide, so the coefficient loads coalesce), the values psi(r) w_q w_q'/r go to LDS in
// element order, and the 8 lanes of each pair (lane q < 7 owns test point x_q) contract them with
// the barycentric weights, reduce lam_a(q) R_b over the group and add entry (a, b) = (m/3, m%3)
// of the pair's 3 x 3 block (lane 0 also entry 8).  Only the half P(v_b(sigma), v_a(tau)) is
// added; the lower-triangle storage receives A = P + P^T directly (scatter_half).  No block
// barrier is taken inside the loop, so the waves of a CU hide each other's latencies.
constexpr int kWavePairs = 8;
constexpr int kWaveEl = kWavePairs * 49;     // 392
constexpr int kWaveSort = 512;
struct WaveLds {
    double key[kWaveSort];
    uint16_t idx[kWaveSort];
    double winv[kWaveEl];
    double P[kWaveEl];
    double Pt[kWaveEl];
    double pmin[kWavePairs], pmax[kWavePairs];
};

__global__ void __launch_bounds__(64)
k_regular_wave(GeomView g, TableView tv, const double* __restrict__ t, BandView band, double* val, float* valf,
               double r_far, unsigned long long* counter)
{
    const int E = g.E;
    const int tau = blockIdx.y;
    const int lane = threadIdx.x;
    const int sig0 = blockIdx.x * kWavePairs;
    if (sig0 + kWavePairs - 1 <= tau) return;            // all sigma <= tau (block = one wave)
    __shared__ PieceTable spt;
    __shared__ WaveLds L;
    load_piece_table(spt, tv.pt);
    __syncthreads();
    const int tv0 = g.v[tau], tv1 = g.v[E + tau], tv2 = g.v[2 * E + tau];
    for (int e = lane; e < kWaveSort; e += 64) {
        if (e < kWaveEl) {
            const int p = e / 49, qq = e - 49 * p, q = qq / 7, qp = qq - 7 * q;
            const int sig = sig0 + p;
            bool ok = sig > tau && sig < E;
            const int sg = ok ? sig : tau;
            if (ok) {
                const int a0 = g.v[sg], a1 = g.v[E + sg], a2 = g.v[2 * E + sg];
                ok = !(a0 == tv0 || a0 == tv1 || a0 == tv2 || a1 == tv0 || a1 == tv1 || a1 == tv2 || a2 == tv0 ||
                       a2 == tv1 || a2 == tv2);
            }
            const double d0 = g.qp[(3 * q) * E + tau] - g.qp[(3 * qp) * E + sg];
            const double d1 = g.qp[(3 * q + 1) * E + tau] - g.qp[(3 * qp + 1) * E + sg];
            const double d2 = g.qp[(3 * q + 2) * E + tau] - g.qp[(3 * qp + 2) * E + sg];
            const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            double la, lb, lc, wq, wp;
            rule7_point(q, la, lb, lc, wq);
            rule7_point(qp, la, lb, lc, wp);
            L.key[e] = ok ? r : INFINITY;
            L.winv[e] = ok ? wq * wp / r : 0.0;
            L.P[e] = 0.0;
            L.Pt[e] = 0.0;
        } else {
            L.key[e] = INFINITY;
        }
        L.idx[e] = (uint16_t)e;
    }
    wave_sync();
    if (lane < kWavePairs) {
        double mn = INFINITY, mx = -INFINITY;
        for (int u = 0; u < 49; ++u) {
            const double r = L.key[lane * 49 + u];
            if (r < INFINITY) { mn = fmin(mn, r); mx = fmax(mx, r); }
        }
        L.pmin[lane] = mn;
        L.pmax[lane] = mx;
    }
    // bitonic sort of (key, idx) inside the wave
    for (int size = 2; size <= kWaveSort; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            wave_sync();
            for (int u = lane; u < kWaveSort / 2; u += 64) {
                const int lo = 2 * stride * (u / stride) + (u % stride);
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const double ka = L.key[lo], kb = L.key[hi];
                if ((ka > kb) == up) {
                    L.key[lo] = kb; L.key[hi] = ka;
                    const uint16_t ia = L.idx[lo];
                    L.idx[lo] = L.idx[hi]; L.idx[hi] = ia;
                }
            }
        }
    }
    wave_sync();
    const int nvalid = wave_count_below(L.key, kWaveSort, INFINITY, false);
    if (nvalid == 0) return;
    const double wmin = L.key[0], wmax = L.key[nvalid - 1];
    const int N = tv.N;
    // contraction lanes: pair gp, test point gq (gq == 7 idles)
    const int gp = lane >> 3, gq = lane & 7;
    const int gsig = sig0 + gp;
    const int gsg = (gsig < E) ? gsig : tau;
    double lqa0, lqa1, lqa2, wdummy;
    rule7_point(gq < 7 ? gq : 0, lqa0, lqa1, lqa2, wdummy);
    if (gq == 7) { lqa0 = lqa1 = lqa2 = 0.0; }
    const int ma = gq / 3, mb = gq % 3;
    const int sv0 = g.v[gsg], sv1 = g.v[E + gsg], sv2 = g.v[2 * E + gsg];
    const int la = ma == 0 ? tv0 : (ma == 1 ? tv1 : tv2), jb = mb == 0 ? sv0 : (mb == 1 ? sv1 : sv2);
    const int mla = gq < 7 ? la : tv2, mjb = gq < 7 ? jb : sv1;
    const double nn = g.n[tau] * g.n[gsg] + g.n[E + tau] * g.n[E + gsg] + g.n[2 * E + tau] * g.n[2 * E + gsg];
    const int ca = gq < 7 ? ma : 2, cb = gq < 7 ? mb : 1;
    const double Cm = g.curl[(3 * ca) * E + tau] * g.curl[(3 * cb) * E + gsg] +
                      g.curl[(3 * ca + 1) * E + tau] * g.curl[(3 * cb + 1) * E + gsg] +
                      g.curl[(3 * ca + 2) * E + tau] * g.curl[(3 * cb + 2) * E + gsg];
    const double C8 = g.curl[6 * E + tau] * g.curl[6 * E + gsg] + g.curl[7 * E + tau] * g.curl[7 * E + gsg] +
                      g.curl[8 * E + tau] * g.curl[8 * E + gsg];
    const double scale = g.area[tau] * g.area[gsg] * 0.07957747154594767;   // |tau||sigma|/(4 pi)
    const double pmn = L.pmin[gp], pmx = L.pmax[gp];
    const bool pair_valid = pmx >= pmn;
    unsigned long long nq = 0;
    int prev0 = 0, prev1 = 0;                 // sorted range written for the previous (k, i)

    int ia = 0, ib = -1;
    for (int k = 0; k < N; ++k) {
        while (ia < N) {
            double lo, hi;
            kernel_support(t, N, k, ia, lo, hi);
            if (lo < wmax) break;
            ++ia;
        }
        while (ib + 1 < N) {
            double lo, hi;
            kernel_support(t, N, k, ib + 1, lo, hi);
            if (!(hi > wmin)) break;
            ++ib;
        }
        for (int i = ia; i <= ib; ++i) {
            const int f = tv.fid[k * N + i];
            if (f < 0) continue;
            const KernelDesc kd = tv.desc[f];
            const int s0 = wave_count_below(L.key, nvalid, kd.lo, true);    // first r > lo
            const int s1 = wave_count_below(L.key, nvalid, kd.hi, false);   // first r >= hi
            if (s1 <= s0) continue;
            // the previous range's values outside the new range become zeros
            const int z0 = prev0 < s0 ? prev0 : s0, z1 = prev1 > s1 ? prev1 : s1;
            for (int s = z0 + lane; s < z1; s += 64)
                if (s < s0 || s >= s1) { const int e = L.idx[s]; L.P[e] = 0.0; L.Pt[e] = 0.0; }
            prev0 = s0;
            prev1 = s1;
            const double* iv = tv.ivl + kd.bp_off;
            for (int base = s0; base < s1; base += 128) {
                const int sa = base + lane, sb = base + 64 + lane;
                if (sa < s1) {
                    const int e = L.idx[sa];
                    eval_sorted_element(kd, iv, tv, spt, L.key[sa], e, L.winv[e], r_far, L.P, L.Pt);
                    ++nq;
                }
                if (sb < s1) {
                    const int e = L.idx[sb];
                    eval_sorted_element(kd, iv, tv, spt, L.key[sb], e, L.winv[e], r_far, L.P, L.Pt);
                    ++nq;
                }
            }
            wave_sync();
            const bool pair_hit = pair_valid && pmx > kd.lo && pmn < kd.hi;
            double R0 = 0.0, R1 = 0.0, R2 = 0.0, T = 0.0;
            if (pair_hit && gq < 7) {
                const int e0 = gp * 49 + gq * 7;
#pragma unroll
                for (int p = 0; p < 7; ++p) {
                    double lb0, lb1, lb2, wp;
                    rule7_point(p, lb0, lb1, lb2, wp);
                    const double P = L.P[e0 + p];
                    R0 = fma(P, lb0, R0);
                    R1 = fma(P, lb1, R1);
                    R2 = fma(P, lb2, R2);
                    T += L.Pt[e0 + p];
                }
            }
            const double s00 = group8_sum(lqa0 * R0), s01 = group8_sum(lqa0 * R1), s02 = group8_sum(lqa0 * R2);
            const double s10 = group8_sum(lqa1 * R0), s11 = group8_sum(lqa1 * R1), s12 = group8_sum(lqa1 * R2);
            const double s20 = group8_sum(lqa2 * R0), s21 = group8_sum(lqa2 * R1), s22 = group8_sum(lqa2 * R2);
            const double sT = group8_sum(gq < 7 ? T : 0.0);
            if (pair_hit) {
                double Sm;
                switch (gq) {
                case 0: Sm = s00; break;
                case 1: Sm = s01; break;
                case 2: Sm = s02; break;
                case 3: Sm = s10; break;
                case 4: Sm = s11; break;
                case 5: Sm = s12; break;
                case 6: Sm = s20; break;
                default: Sm = s21; break;
                }
                scatter_half(band, val, valf, k, i, mla, mjb, (nn * Sm + Cm * sT) * scale);
                if (gq == 0) scatter_half(band, val, valf, k, i, tv2, sv2, (nn * s22 + C8 * sT) * scale);
            }
            wave_sync();
        }
    }
    const unsigned long long tot = wave_sum_u64(nq);
    if (lane == 0 && tot) atomicAdd(counter, tot);
}

// ---------------------------------------------------------------------------------------------
// Singular pairs.  One lane per (pair, k).  pairs[9*s..]: tau, sigma, kind (0 coincident,
// 1 edge, 2 vertex), the local indices of the reference vertices (A, B, C) in tau and in sigma.
// The rule rows are (x1, x2, y1, y2, w) on the reference triangle {0 <= x2 <= x1 <= 1}, the
// physical point A + x1 (B - A) + x2 (C - B) with barycentrics (1 - x1, x1 - x2, x2).
// ---------------------------------------------------------------------------------------------
constexpr int kSingBand = 6;

__global__ void __launch_bounds__(128)
k_singular(GeomView g, TableView tv, const double* __restrict__ t, BandView band, const int32_t* __restrict__ pairs,
           int64_t npairs, const double* __restrict__ rules, const int32_t* __restrict__ roff,
           const int32_t* __restrict__ rcnt, double* val, float* valf, unsigned long long* counter)
{
    __shared__ PieceTable spt;
    load_piece_table(spt, tv.pt);
    __syncthreads();
    const int N = tv.N;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long nq = 0;
    if (gid < npairs * N) {
        const int64_t s = gid / N;
        const int k = (int)(gid - s * N);
        const int E = g.E;
        const int32_t* pr = pairs + 9 * s;
        const int tau = pr[0], sig = pr[1], kind = pr[2];
        int px[3] = {pr[3], pr[4], pr[5]}, py[3] = {pr[6], pr[7], pr[8]};
        double X[3][3], Y[3][3];   // reference vertices A, B, C
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) {
                X[a][c] = g.P[(3 * px[a] + c) * E + tau];
                Y[a][c] = g.P[(3 * py[a] + c) * E + sig];
            }
        double rmax = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const double d0 = X[a][0] - Y[b][0], d1 = X[a][1] - Y[b][1], d2 = X[a][2] - Y[b][2];
                rmax = fmax(rmax, sqrt(d0 * d0 + d1 * d1 + d2 * d2));
            }
        rmax *= 1.0 + 1e-12;
        int ia = 0;
        while (ia < N) {
            double lo, hi;
            kernel_support(t, N, k, ia, lo, hi);
            if (lo < rmax) break;
            ++ia;
        }
        int ib = ia - 1;
        while (ib + 1 < N) {
            double lo, hi;
            kernel_support(t, N, k, ib + 1, lo, hi);
            if (!(hi > 0.0)) break;
            ++ib;
        }
        const double nn = g.n[tau] * g.n[sig] + g.n[E + tau] * g.n[E + sig] + g.n[2 * E + tau] * g.n[2 * E + sig];
        const double jac = 4.0 * g.area[tau] * g.area[sig];
        const double scale = 0.07957747154594767;   // 1/(4 pi)
        // reference-order vertex ids and curl products (static register indices below)
        int vtr[3], vsr[3];
        double Cr[3][3];
        for (int al = 0; al < 3; ++al) {
            vtr[al] = g.v[px[al] * E + tau];
            vsr[al] = g.v[py[al] * E + sig];
        }
        for (int al = 0; al < 3; ++al)
            for (int be = 0; be < 3; ++be)
                Cr[al][be] = g.curl[(3 * px[al]) * E + tau] * g.curl[(3 * py[be]) * E + sig] +
                             g.curl[(3 * px[al] + 1) * E + tau] * g.curl[(3 * py[be] + 1) * E + sig] +
                             g.curl[(3 * px[al] + 2) * E + tau] * g.curl[(3 * py[be] + 2) * E + sig];
        const int npts = rcnt[kind];
        const double* rule = rules + 5 * (int64_t)roff[kind];
        for (int i0 = ia; i0 <= ib; i0 += kSingBand) {
            const int nb = (ib - i0 + 1) < kSingBand ? (ib - i0 + 1) : kSingBand;
            KernelDesc kd[kSingBand];
            bool have[kSingBand];
#pragma unroll
            for (int u = 0; u < kSingBand; ++u) {
                const int f = u < nb ? tv.fid[k * N + i0 + u] : -1;
                have[u] = f >= 0;
                if (have[u]) kd[u] = tv.desc[f];
                else { kd[u].lo = 1.0; kd[u].hi = 0.0; kd[u].nint = 0; kd[u].bp_off = 0; kd[u].coef_off = 0; }
            }
            double S1[kSingBand][9], S2[kSingBand];
#pragma unroll
            for (int u = 0; u < kSingBand; ++u) {
                S2[u] = 0.0;
#pragma unroll
                for (int m = 0; m < 9; ++m) S1[u][m] = 0.0;
            }
            for (int q = 0; q < npts; ++q) {
                const double* R = rule + 5 * q;
                const double x1 = R[0], x2 = R[1], y1 = R[2], y2 = R[3];
                const double w = R[4] * jac;
                const double lx0 = 1.0 - x1, lx1 = x1 - x2, lx2 = x2;
                const double ly0 = 1.0 - y1, ly1 = y1 - y2, ly2 = y2;
                double d2 = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double xc = lx0 * X[0][c] + lx1 * X[1][c] + lx2 * X[2][c];
                    const double yc = ly0 * Y[0][c] + ly1 * Y[1][c] + ly2 * Y[2][c];
                    d2 += (xc - yc) * (xc - yc);
                }
                const double rr = sqrt(d2);
                const double wr = w / rr;
#pragma unroll
                for (int u = 0; u < kSingBand; ++u) {
                    double ps, pt;
                    if (have[u] && table_eval(kd[u], tv.ivl, tv.coef, spt, rr, ps, pt)) {
                        ++nq;
                        const double f1 = ps * wr;
                        const double R0 = f1 * ly0, R1 = f1 * ly1, R2 = f1 * ly2;
                        S1[u][0] = fma(lx0, R0, S1[u][0]); S1[u][1] = fma(lx0, R1, S1[u][1]); S1[u][2] = fma(lx0, R2, S1[u][2]);
                        S1[u][3] = fma(lx1, R0, S1[u][3]); S1[u][4] = fma(lx1, R1, S1[u][4]); S1[u][5] = fma(lx1, R2, S1[u][5]);
                        S1[u][6] = fma(lx2, R0, S1[u][6]); S1[u][7] = fma(lx2, R1, S1[u][7]); S1[u][8] = fma(lx2, R2, S1[u][8]);
                        S2[u] = fma(pt, wr, S2[u]);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < kSingBand; ++u) {
                if (u >= nb || !have[u]) continue;
                const int i = i0 + u;
                double loc[3][3];
#pragma unroll
                for (int al = 0; al < 3; ++al)
#pragma unroll
                    for (int be = 0; be < 3; ++be) loc[al][be] = (nn * S1[u][3 * al + be] + Cr[al][be] * S2[u]) * scale;
                if (kind == 0) {
                    // identical triangles: reference order = local order; symmetrise in (a, b)
#pragma unroll
                    for (int a = 0; a < 3; ++a)
#pragma unroll
                        for (int b = a + 1; b < 3; ++b) {
                            const double m = 0.5 * (loc[a][b] + loc[b][a]);
                            loc[a][b] = m;
                            loc[b][a] = m;
                        }
#pragma unroll
                    for (int a = 0; a < 3; ++a)
#pragma unroll
                        for (int b = 0; b < 3; ++b) scatter_half(band, val, valf, k, i, vtr[a], vsr[b], 0.5 * loc[a][b]);
                } else {
#pragma unroll
                    for (int a = 0; a < 3; ++a)
#pragma unroll
                        for (int b = 0; b < 3; ++b) scatter_half(band, val, valf, k, i, vtr[a], vsr[b], loc[a][b]);
                }
            }
        }
    }
    const unsigned long long tot = wave_sum_u64(nq);
    if ((threadIdx.x & 63) == 0 && tot) atomicAdd(counter, tot);
}

__global__ void __launch_bounds__(256)
k_get_entries(BandView band, const double* __restrict__ val, const float* __restrict__ valf, int64_t n,
              const int32_t* __restrict__ k, const int32_t* __restrict__ i, const int32_t* __restrict__ j,
              const int32_t* __restrict__ l, double* __restrict__ out)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int kk = k[s], ii = i[s];
    int jj = j[s], ll = l[s];
    if (jj > ll) { const int tmp = jj; jj = ll; ll = tmp; }   // symmetric blocks: lower triangle
    double v = 0.0;
    if (kk >= 0 && kk < band.N && ii >= 0 && ii < band.N && jj >= 0 && ll < band.M) {
        const int B = band.B[kk];
        const int sl = ii - (int)band.ilo[(int64_t)kk * band.ntri + tri_index(ll, jj)];
        if (sl >= 0 && sl < B) {
            const int64_t idx = band_value_index(band, kk, ll, jj, sl, B);
            v = valf ? (double)valf[idx] : val[idx];
        }
    }
    out[s] = v;
}

static inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_geometry(const double* xyz, const int32_t* tri, int E, double* geo_P, double* geo_n, double* geo_area,
                     double* geo_curl, double* geo_qp, int32_t* geo_v, hipStream_t s)
{
    hipLaunchKernelGGL(k_geometry, dim3(grid_for(E, 256)), dim3(256), 0, s, xyz, tri, E, geo_P, geo_n, geo_area,
                       geo_curl, geo_qp, geo_v);
}

void launch_layout(const double* xyz, const double* rho, int M, const double* t, int N, int16_t* ilo, int32_t* Bk,
                   hipStream_t s)
{
    hipLaunchKernelGGL(k_layout, dim3(grid_for(M, 256), M), dim3(256), sizeof(int32_t) * N, s, xyz, rho, M, t, N, ilo,
                       Bk);
}

void launch_regular(GeomView g, TableView tv, const double* t, BandView band, double* val, float* valf,
                    double r_far, unsigned long long* counter, hipStream_t s)
{
    dim3 grid(grid_for(g.E, kWavePairs), g.E);
    hipLaunchKernelGGL(k_regular_wave, grid, dim3(64), 0, s, g, tv, t, band, val, valf, r_far, counter);
}

void launch_singular(GeomView g, TableView tv, const double* t, BandView band, const int32_t* pairs, int64_t npairs,
                     const double* ss_rules, const int32_t* ss_off, const int32_t* ss_cnt, double* val, float* valf,
                     unsigned long long* counter, hipStream_t s)
{
    const int64_t n = npairs * tv.N;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_singular, dim3(grid_for(n, 128)), dim3(128), 0, s, g, tv, t, band, pairs, npairs, ss_rules,
                       ss_off, ss_cnt, val, valf, counter);
}

void launch_get_entries(BandView band, const double* val, const float* valf, int64_t n, const int32_t* k,
                        const int32_t* i, const int32_t* j, const int32_t* l, double* out, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_get_entries, dim3(grid_for(n, 256)), dim3(256), 0, s, band, val, valf, n, k, i, j, l, out);
}

}  // namespace tdbem
