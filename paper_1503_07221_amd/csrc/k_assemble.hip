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

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

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
// lo_{k,i} < dmax and hi_{k,i} > dmin.  Both bounds move right with k (two pointers).  Block =
// one 64 x 64 vertex tile t; lane (row l, column j) for 16 rows per wave; pairs with j > l or past
// M idle.  The tile's band width per time row is the maximum over its pairs (LDS), written whole.
__global__ void __launch_bounds__(256)
k_layout(BandView band, const double* __restrict__ xyz, const double* __restrict__ rho,
         const double* __restrict__ t, int16_t* __restrict__ ilo, int32_t* __restrict__ Bt)
{
    const int M = band.M, N = band.N;
    extern __shared__ int32_t sB[];
    for (int k = threadIdx.x; k < N; k += blockDim.x) sB[k] = 0;
    __syncthreads();
    const int tt = blockIdx.x;
    int tl = (int)((sqrt(8.0 * tt + 1.0) - 1.0) * 0.5);
    while ((tl + 1) * (tl + 2) / 2 <= tt) ++tl;
    while (tl * (tl + 1) / 2 > tt) --tl;
    const int tj = tt - tl * (tl + 1) / 2;
    const int j = tj * kBT + (threadIdx.x & 63);
    const double slack = 1e-12 * (1.0 + t[band.nodes - 1]);
    for (int m = 0; m < 16; ++m) {
        const int l = tl * kBT + (threadIdx.x >> 6) + 4 * m;
        if (l >= M || j > l) continue;
        const double dx = xyz[3 * l] - xyz[3 * j], dy = xyz[3 * l + 1] - xyz[3 * j + 1], dz = xyz[3 * l + 2] - xyz[3 * j + 2];
        const double d = sqrt(dx * dx + dy * dy + dz * dz);
        const double dmax = d + rho[l] + rho[j] + slack;
        double dmin = d - rho[l] - rho[j] - slack;
        dmin = dmin > 0.0 ? dmin : 0.0;
        int ia = 0, ib = -1;
        for (int k = 0; k < N; ++k) {
            while (ia < N) {
                double lo, hi;
                kernel_support(t, band.nodes, band.p1, k, ia, lo, hi);
                if (lo < dmax) break;
                ++ia;
            }
            while (ib + 1 < N) {
                double lo, hi;
                kernel_support(t, band.nodes, band.p1, k, ib + 1, lo, hi);
                if (!(hi > dmin)) break;
                ++ib;
            }
            const int first = ia < N ? ia : N - 1;
            ilo[band_ilo_index(band, k, l, j)] = (int16_t)first;
            const int cnt = ib - ia + 1;
            if (cnt > 0) atomicMax(&sB[k], cnt);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < N; k += blockDim.x) Bt[(int64_t)k * band.nt + tt] = sB[k];
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

// Deterministic assembly: a contribution v enters the storage as the 64-bit integer
// round(v * fxs) (fxs a power of two), added with integer atomics, whose sum does not depend on
// the order of the additions (two's complement addition is exact modulo 2^64; the final sums fit).
__device__ inline unsigned long long to_fixed(double v, double fxs)
{
    return (unsigned long long)__double2ll_rn(v * fxs);
}

// P(l, j) += v for the half P of the assembly (A = P + P^T): in the lower-triangle storage an
// off-diagonal contribution lands at (max, min) and a diagonal one counts twice.  fxs > 0: val
// holds the fixed-point integers of the deterministic mode.
__device__ inline void scatter_half(const BandView& band, double* val, float* valf, int k, int i, int l, int j,
                                    double v, double fxs)
{
    if (j > l) { const int tmp = j; j = l; l = tmp; }
    if (j == l) v *= 2.0;
    const int s = i - (int)band.ilo[band_ilo_index(band, k, l, j)];
    const int B = band_width(band, k, l, j);
    if (s < 0 || s >= B) return;   // outside the band: the value is zero (support test)
    const int64_t idx = band_value_index(band, k, l, j, s, B);
    if (fxs > 0.0) atomicAdd(reinterpret_cast<unsigned long long*>(val) + idx, to_fixed(v, fxs));
    else if (valf) atomicAdd(valf + idx, (float)v);
    else atomicAdd(val + idx, v);
}

// Matrix-free form of scatter_half: the contribution v to P(l, j) is applied to x at once,
// y_k(l) += v x_i(j) and y_k(j) += v x_i(l) (A = P + P^T; for l == j the two give 2 v x_i(l)).
struct ProductView {
    const double* x;       // x[i*M + j]
    double* y;             // y[k*M + l]
    int32_t M;
};

__device__ inline void deposit(const BandView& band, double* val, float* valf, const ProductView& pv, int k, int i,
                               int l, int j, double v, double fxs = 0.0)
{
    if (pv.y) {
        atomicAdd(pv.y + (int64_t)k * pv.M + l, v * pv.x[(int64_t)i * pv.M + j]);
        atomicAdd(pv.y + (int64_t)k * pv.M + j, v * pv.x[(int64_t)i * pv.M + l]);
    } else {
        scatter_half(band, val, valf, k, i, l, j, v, fxs);
    }
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

// Both Chebyshev series at x from coefficients held in registers: T_m(x) by the three-term
// recurrence, the two sums accumulated alongside (41 FP64 operations for degree 14).
__device__ inline void cheb_sums(const double2 (&c)[kNc], double x, double& ps, double& pt)
{
    const double x2 = 2.0 * x;
    double tm1 = 1.0, tm = x;
    ps = fma(c[1].x, x, c[0].x);
    pt = fma(c[1].y, x, c[0].y);
#pragma unroll
    for (int m = 2; m < kNc; ++m) {
        const double tn = fma(x2, tm, -tm1);
        ps = fma(c[m].x, tn, ps);
        pt = fma(c[m].y, tn, pt);
        tm1 = tm;
        tm = tn;
    }
}

// 1/r to about one ulp: hardware reciprocal refined by two Newton steps.
__device__ inline double recip(double r)
{
    double y = __builtin_amdgcn_rcp(r);
    double e = fma(-r, y, 1.0);
    y = fma(y, e, y);
    e = fma(-r, y, 1.0);
    return fma(y, e, y);
}

// ---------------------------------------------------------------------------------------------
// Regular pairs, tiled.  One workgroup (8 lanes per triangle pair) owns a tile of TT consecutive
// test triangles tau and TS consecutive trial triangles sigma (the unordered pairs sigma > tau
// without a common vertex: TT TS x 49 point pairs).  It sorts the point-pair distances once; for
// every (k, i) the distances inside supp psi_{k,i} form one range of the sorted list.
//
//   plan     one wave takes up to kPlan candidates (k, i) at once (one per lane): the range
//            [s0, s1) of sorted distances inside the support, and the Chebyshev pieces that
//            range meets.  A round whose range meets more than kStage pieces is cut, at a piece
//            boundary, into segments of at most kStage pieces.  The records go to LDS.
//   stage    the pieces of a record (coefficients and piece records), the interval starts and
//            the support are copied to LDS; the copy for the next record is loaded into
//            registers while the current one is evaluated and contracted, so the inner loop
//            reads LDS only.
//   phase 1  the lanes split the record's range into contiguous chunks; a lane keeps the
//            coefficients of its current piece in registers and moves to the next piece when r
//            passes its end (sorted neighbours share pieces); psi w/r and tpsi w/r of every
//            point pair go to V (one plain store per point pair, each written by one lane).
//   phase 2  after the last segment of a round, the 8 lanes of a triangle pair contract V:
//            lane q sums its row over q' with lam_b(q') into R_b(q) (kept in the row's first
//            two slots), lane (a, b) then sums lam_a(q) R_b(q) over the 7 rows, and the 3 x 3
//            block is merged in an LDS tile over the two vertex sets before one atomic add per
//            (vertex, vertex) entry goes to the band storage.
// Two barriers per record.
// ---------------------------------------------------------------------------------------------
constexpr int kStage = 64;                           // pieces of one record held in LDS
constexpr int kStageSlots = kStage * (kNc + 2) + kMaxIntervals + 1;   // double2 slots
constexpr int kPlan = 64;                            // candidates planned at once (one wave)
constexpr int kSegMax = 3;                           // segments of one round (kMaxIntervals * kPieces pieces)
constexpr int kMaxRec = kSegMax * kPlan;
static_assert((kStage - 1) * (kSegMax - 1) + kStage >= kMaxIntervals * kPieces, "segments cover a kernel");
static_assert(kSegMax == 3, "the record compaction counts three slots");

// Tile shape: TT test x TS trial triangles on THREADS lanes (8 lanes per triangle pair), SORT the
// power of two >= the point pairs that the bitonic sort runs on.  Larger tiles put more point pairs
// behind every record (the fixed cost of a record is its latency chain and two barriers); the LDS
// of the sorted keys and per-point slots bounds the size.  The host times the compiled shapes.
template <int TT, int TS, int THREADS, int SORT>
struct TileShape {
    static constexpr int kT = TT, kS = TS, kThreads = THREADS, kSort = SORT;
    static constexpr int kPairs = TT * TS, kEl = kPairs * 49;
    static constexpr int kVt = 3 * TT, kVs = 3 * TS;
    static constexpr int kStageRegs = (kStageSlots + THREADS - 1) / THREADS;
    static constexpr int kChunkMax = (kEl + THREADS - 1) / THREADS;   // sorted points of one lane
    static constexpr int kDz = (kVt * kVs + THREADS - 1) / THREADS;   // vertex-tile entries of one lane
    static_assert(SORT >= kEl && (SORT & (SORT - 1)) == 0, "bitonic sort size");
    static_assert(kEl < 4096, "a record packs sorted indices in 12 bits");
    static_assert(THREADS == 8 * kPairs && THREADS >= 192 + kPairs, "8 lanes per pair; the setup roles");
};
using TileA = TileShape<4, 8, 256, 2048>;     // 1568 point pairs, 77.9 KB of LDS: 2 workgroups per CU
using TileB = TileShape<8, 8, 512, 4096>;     // 3136 point pairs, 131.7 KB: 1 workgroup (8 waves) per CU

// One record: the sorted range [s0, s1) of a round (k, i) = kernel f, whose pieces
// g0 .. g0 + np - 1 (kernel-local g0l; absolute g0) cover it; last = 1 on a round's last segment.
struct TileRec {
    int32_t f;
    int32_t g0;
    uint32_t s;      // s0 | s1 << 12 | (np - 1) << 24 (s0, s1 <= 4096 point pairs, np <= 64)
    uint32_t ki;     // k | i << 13 | last << 26
    int32_t g0l;     // kernel-local first piece (< 256) | nint << 8
    int32_t bpo;     // the kernel's first interval start in ivl
};

template <class Tile>
struct TileLds {
    double key[Tile::kSort];
    double2 V[Tile::kEl];              // (psi w/r, tpsi w/r) of every point pair; zero off the support
    double2 stage[kStageSlots];      // 15 np coefficients, 2 np piece records, intervals, (lo, hi)
    double acc[Tile::kVt * Tile::kVs];
    double alpha[Tile::kPairs];        // (n_tau . n_sigma) |tau||sigma| / (4 pi)
    double beta[Tile::kPairs * 9];     // C_ab |tau||sigma| / (4 pi), entry e = 3a + b
    double wqq[49];                  // w_q w_q'
    double lam[7 * 3];               // lam_b(q')
    double pmin[Tile::kPairs], pmax[Tile::kPairs];
    TileRec rec[kMaxRec];
    int32_t bcum[Tile::kThreads + 1];  // candidates of the k-block: exclusive prefix over k
    int32_t bia[Tile::kThreads];       // first trial index of each k's band
    uint16_t idx[Tile::kSort];         // point pair p * 49 + 7 q + q' of each sorted distance
    uint16_t aoff[Tile::kPairs * 9];   // entry (v_a(tau), v_b(sigma)) of the merged vertex tile
    int32_t vt[Tile::kVt], vs[Tile::kVs];
    int32_t pok[Tile::kPairs];
    int32_t nvt, nvs, nrec;
    int32_t wtot[Tile::kThreads / 64];
};

// Number of keys <= v (le) or < v among the ascending key[0..n), one lane.
__device__ inline int lane_count_below(const double* key, int n, double v, bool le)
{
    int a = 0, b = n;
    while (a < b) {
        const int m = (a + b) >> 1;
        if (le ? key[m] <= v : key[m] < v) a = m + 1;
        else b = m;
    }
    return a;
}

// Kernel-local piece j * kPieces + p holding r: the interval from its starts, the piece from the
// graded partition (lookup table, one correction).  Rounding can put r one piece early at a
// boundary; callers move on through the piece records.
__device__ inline int piece_local(double r, const double2* iv, int nint, const PieceTable& pt)
{
    int j = 0;
    for (int m = 1; m < nint; ++m) j += r >= iv[m].x ? 1 : 0;
    double fr = (r - iv[j].x) * iv[j].y;
    fr = fr < 0.0 ? 0.0 : (fr > 1.0 ? 1.0 : fr);
    int cell = (int)(fr * kLutCells);
    cell = cell < kLutCells ? cell : kLutCells - 1;
    int p = pt.lut[cell];
    if (p + 1 < kPieces && fr >= pt.edge[p + 1]) ++p;
    return j * kPieces + p;
}

// DPP moves inside groups of 8 lanes: xor 1, xor 2 (quad permutations), mirror within 8.
template <int CTRL>
__device__ inline double dpp_move(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo));
}
__device__ inline double group8_sum_dpp(double v)
{
    v += dpp_move<0xB1>(v);     // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4E>(v);     // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x141>(v);    // row_half_mirror
    return v;
}

// Loads the LDS stage of record R into registers (slot e = tid + threads m).
template <class Tile>
__device__ inline void stage_fetch(const TileRec& R, const TableView& tv, double2 (&st)[Tile::kStageRegs])
{
    const int np = (int)((R.s >> 24) & 63u) + 1, nint = R.g0l >> 8;
    const int nc = kNc * np, nm = nc + 2 * np, ni = nm + nint;
    const double2* meta2 = reinterpret_cast<const double2*>(tv.meta);
    const double2* ivl2 = reinterpret_cast<const double2*>(tv.ivl);
#pragma unroll
    for (int m = 0; m < Tile::kStageRegs; ++m) {
        const int e = threadIdx.x + Tile::kThreads * m;
        double2 v = make_double2(0.0, 0.0);
        if (e < nc) v = tv.coef[(int64_t)R.g0 * kNc + e];
        else if (e < nm) v = meta2[2 * (int64_t)R.g0 + (e - nc)];
        else if (e < ni) v = ivl2[(R.bpo >> 1) + (e - nm)];
        else if (e == ni) v = reinterpret_cast<const double2*>(tv.desc + R.f)[0];
        st[m] = v;
    }
}

template <class Tile>
__device__ inline void stage_store(const TileRec& R, double2* stage, const double2 (&st)[Tile::kStageRegs])
{
    const int np = (int)((R.s >> 24) & 63u) + 1, nint = R.g0l >> 8;
    const int used = (kNc + 2) * np + nint + 1;
#pragma unroll
    for (int m = 0; m < Tile::kStageRegs; ++m) {
        const int e = threadIdx.x + Tile::kThreads * m;
        if (e < used) stage[e] = st[m];
    }
}

// Multi: the tiles of several problems in one launch; the top 8 bits of a tile's test index name
// its problem, whose views replace the launch's own.  Fixed: the deterministic mode (the merged
// vertex tile and the storage hold fixed-point integers of scale fxs, see to_fixed).
template <class Tile, bool Multi, bool Fixed>
__global__ void __launch_bounds__(Tile::kThreads, 2)
k_regular_tile(GeomView g_, TableView tv_, const double* __restrict__ t_, BandView band_, double* val_,
               float* valf_, ProductView pv, const int2* __restrict__ tiles, int64_t ntiles,
               unsigned long long* counter_, const RegularProblem* __restrict__ probs, double fxs)
{
    constexpr int kTileT = Tile::kT, kTileS = Tile::kS, kTilePairs = Tile::kPairs, kTileEl = Tile::kEl, kTileSort = Tile::kSort;
    constexpr int kTileThreads = Tile::kThreads, kTileVt = Tile::kVt, kTileVs = Tile::kVs, kChunkMax = Tile::kChunkMax;
    constexpr int kDz = Tile::kDz, kStageRegs = Tile::kStageRegs;
    // consecutive workgroups go to the 8 XCDs in turn: give each XCD one contiguous range of the
    // tile list (same test rows, shared L2 lines for the output)
    const int64_t per = (ntiles + 7) / 8;
    const int64_t tix = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tix >= ntiles) return;
    int2 tl = tiles[tix];
    GeomView g = g_;
    TableView tv = tv_;
    const double* __restrict__ t = t_;
    BandView band = band_;
    double* val = val_;
    float* valf = valf_;
    unsigned long long* counter = counter_;
    const PieceTable* ptab = &tv_.pt;
    if constexpr (Multi) {
        const RegularProblem& P = probs[(uint32_t)tl.x >> 24];
        ptab = &P.tv.pt;
        g = P.g;
        tv = P.tv;
        t = P.t;
        band = P.band;
        val = P.val;
        valf = P.valf;
        counter = P.counter;
        tl.x &= 0xFFFFFF;
    }
    const int E = g.E;
    const int tau0 = tl.x * kTileT, sig0 = tl.y * kTileS;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    __shared__ PieceTable spt;
    __shared__ TileLds<Tile> L;
    load_piece_table(spt, *ptab);
    if (tid == 0) {
        int n = 0;
        for (int a = 0; a < kTileT && tau0 + a < E; ++a)
            for (int c = 0; c < 3; ++c) {
                const int v = g.v[c * E + tau0 + a];
                bool f = false;
                for (int u = 0; u < n; ++u) f = f || L.vt[u] == v;
                if (!f) L.vt[n++] = v;
            }
        L.nvt = n;
    } else if (tid == 64) {
        int n = 0;
        for (int a = 0; a < kTileS && sig0 + a < E; ++a)
            for (int c = 0; c < 3; ++c) {
                const int v = g.v[c * E + sig0 + a];
                bool f = false;
                for (int u = 0; u < n; ++u) f = f || L.vs[u] == v;
                if (!f) L.vs[n++] = v;
            }
        L.nvs = n;
    } else if (tid >= 128 && tid < 128 + 49) {
        const int qq = tid - 128;
        double l0, l1, l2, wq, wp;
        rule7_point(qq / 7, l0, l1, l2, wq);
        rule7_point(qq % 7, l0, l1, l2, wp);
        L.wqq[qq] = wq * wp;
        if (qq < 7) {
            rule7_point(qq, l0, l1, l2, wp);
            L.lam[3 * qq] = l0;
            L.lam[3 * qq + 1] = l1;
            L.lam[3 * qq + 2] = l2;
        }
    } else if (tid >= 192 && tid < 192 + kTilePairs) {
        const int p = tid - 192;
        const int tau = tau0 + p / kTileS, sig = sig0 + p % kTileS;
        bool ok = tau < E && sig < E && sig > tau;
        if (ok) {
            const int t0 = g.v[tau], t1 = g.v[E + tau], t2 = g.v[2 * E + tau];
            const int a0 = g.v[sig], a1 = g.v[E + sig], a2 = g.v[2 * E + sig];
            ok = !(a0 == t0 || a0 == t1 || a0 == t2 || a1 == t0 || a1 == t1 || a1 == t2 || a2 == t0 || a2 == t1 ||
                   a2 == t2);
        }
        L.pok[p] = ok ? 1 : 0;
    }
    for (int z = tid; z < kTileEl; z += kTileThreads) L.V[z] = make_double2(0.0, 0.0);
    for (int z = tid; z < kTileVt * kTileVs; z += kTileThreads) L.acc[z] = 0.0;
    __syncthreads();
    for (int e = tid; e < kTileSort; e += kTileThreads) {
        double r = INFINITY;
        if (e < kTileEl) {
            const int p = e / 49, qq = e - 49 * p, q = qq / 7, qp = qq - 7 * q;
            if (L.pok[p]) {
                const int tau = tau0 + p / kTileS, sig = sig0 + p % kTileS;
                const double d0 = g.qp[(3 * q) * E + tau] - g.qp[(3 * qp) * E + sig];
                const double d1 = g.qp[(3 * q + 1) * E + tau] - g.qp[(3 * qp + 1) * E + sig];
                const double d2 = g.qp[(3 * q + 2) * E + tau] - g.qp[(3 * qp + 2) * E + sig];
                r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            }
        }
        L.key[e] = r;
        L.idx[e] = (uint16_t)(e < kTileEl ? e : 0);
    }
    __syncthreads();
    // distance range of every pair (8 lanes per pair, lane m < 7 scans the row q = m)
    const int gp = tid >> 3, gm = tid & 7;
    {
        double mn = INFINITY, mx = -INFINITY;
        if (gm < 7)
            for (int u = 0; u < 7; ++u) {
                const double r = L.key[gp * 49 + gm * 7 + u];
                if (r < INFINITY) { mn = fmin(mn, r); mx = fmax(mx, r); }
            }
        for (int o = 1; o < 8; o <<= 1) {
            mn = fmin(mn, __shfl_xor(mn, o, 64));
            mx = fmax(mx, __shfl_xor(mx, o, 64));
        }
        if (gm == 0) { L.pmin[gp] = mn; L.pmax[gp] = mx; }
    }
    // bitonic sort of (key, idx)
    for (int size = 2; size <= kTileSort; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int u = tid; u < kTileSort / 2; u += kTileThreads) {
                const int lo = 2 * stride * (u / stride) + (u % stride);
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const double ka = L.key[lo], kb = L.key[hi];
                if ((ka > kb) == up) {
                    L.key[lo] = kb;
                    L.key[hi] = ka;
                    const uint16_t ia = L.idx[lo];
                    L.idx[lo] = L.idx[hi];
                    L.idx[hi] = ia;
                }
            }
        }
    __syncthreads();
    const int nvalid = __builtin_amdgcn_readfirstlane(wave_count_below(L.key, kTileSort, INFINITY, false));
    if (nvalid == 0) return;                      // uniform: the whole workgroup leaves
    const double wmin = L.key[0], wmax = L.key[nvalid - 1];

    // contraction tables of every pair: lane (pair gp, entry gm = 3a + b; gm == 0 also entry 8)
    {
        const int ctau = tau0 + gp / kTileS, csig = sig0 + gp % kTileS;
        for (int e = gm; e < 9; e += 8) {
            double beta = 0.0;
            int off = 0;
            if (L.pok[gp]) {
                const int ea = e / 3, eb = e % 3;
                const double scale = g.area[ctau] * g.area[csig] * 0.07957747154594767;   // |tau||sigma|/(4 pi)
                beta = (g.curl[(3 * ea) * E + ctau] * g.curl[(3 * eb) * E + csig] +
                        g.curl[(3 * ea + 1) * E + ctau] * g.curl[(3 * eb + 1) * E + csig] +
                        g.curl[(3 * ea + 2) * E + ctau] * g.curl[(3 * eb + 2) * E + csig]) * scale;
                if (e == 0)
                    L.alpha[gp] = (g.n[ctau] * g.n[csig] + g.n[E + ctau] * g.n[E + csig] +
                                   g.n[2 * E + ctau] * g.n[2 * E + csig]) * scale;
                const int vl = g.v[ea * E + ctau], vj = g.v[eb * E + csig];
                int xl = 0, xj = 0;
                for (int u = 0; u < L.nvt; ++u) xl = L.vt[u] == vl ? u : xl;
                for (int u = 0; u < L.nvs; ++u) xj = L.vs[u] == vj ? u : xj;
                off = xl * kTileVs + xj;
            } else if (e == 0) {
                L.alpha[gp] = 0.0;
            }
            L.beta[9 * gp + e] = beta;
            L.aoff[9 * gp + e] = (uint16_t)off;
        }
    }

    const int N = tv.N;
    unsigned long long nq = 0;
    // lam_a(q) of the lane's phase-2 entry (a, b) = (gm / 3, gm % 3)
    double la[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        double l0, l1, l2, w;
        rule7_point(q, l0, l1, l2, w);
        la[q] = gm < 3 ? l0 : (gm < 6 ? l1 : l2);
    }
    // band addresses of the lane's entries z = tid + threads h of the merged vertex tile (time row kcur)
    int kcur = -1;
    int dz_ilo[kDz] = {}, dz_B[kDz] = {}, dz_lj[kDz] = {};
    int64_t dz_vo[kDz] = {};
    for (int kb = 0; kb < N; kb += kTileThreads) {
        // band [ia, ib] of every k of the block: supp psi_{k,i} meets (wmin, wmax); both ends of the
        // support are non-increasing in i, so both ends of the band are binary searches
        {
            const int k = kb + tid;
            int ia = 0, cnt = 0;
            if (k < N) {
                int a = 0, b = N;
                while (a < b) {
                    const int m = (a + b) >> 1;
                    double lo, hi;
                    kernel_support(t, tv.nodes, tv.p1, k, m, lo, hi);
                    if (lo < wmax) b = m;
                    else a = m + 1;
                }
                ia = a;
                a = 0;
                b = N;
                while (a < b) {
                    const int m = (a + b) >> 1;
                    double lo, hi;
                    kernel_support(t, tv.nodes, tv.p1, k, m, lo, hi);
                    if (hi > wmin) a = m + 1;
                    else b = m;
                }
                cnt = a - 1 >= ia ? a - ia : 0;
            }
            // exclusive prefix over the block
            int inc = cnt;
            for (int o = 1; o < 64; o <<= 1) {
                const int v = __shfl_up(inc, o, 64);
                if (lane >= o) inc += v;
            }
            if (lane == 63) L.wtot[wave] = inc;
            __syncthreads();
            int off = 0;
            for (int w = 0; w < wave; ++w) off += L.wtot[w];
            L.bcum[tid] = off + inc - cnt;
            L.bia[tid] = ia;
            if (tid == kTileThreads - 1) L.bcum[kTileThreads] = off + inc;
            __syncthreads();
        }
        const int total = L.bcum[kTileThreads];
        for (int c0 = 0; c0 < total; c0 += kPlan) {
            if (wave == 0) {
                // plan: lane = candidate c0 + lane
                TileRec out[kSegMax];
                bool ok[kSegMax];
#pragma unroll
                for (int m = 0; m < kSegMax; ++m) ok[m] = false;
                const int c = c0 + lane;
                if (c < total) {
                    int a = 0, b = kTileThreads;       // last block slot with bcum <= c
                    while (b - a > 1) {
                        const int m = (a + b) >> 1;
                        if (L.bcum[m] <= c) a = m;
                        else b = m;
                    }
                    const int k = kb + a, i = L.bia[a] + (c - L.bcum[a]);
                    const int f = tv.fid[(int64_t)k * N + i];
                    if (f >= 0) {
                        const KernelDesc kd = tv.desc[f];
                        const int s0 = lane_count_below(L.key, nvalid, kd.lo, true);
                        const int s1 = lane_count_below(L.key, nvalid, kd.hi, false);
                        if (s1 > s0) {
                            const double2* iv = reinterpret_cast<const double2*>(tv.ivl + kd.bp_off);
                            const int base = (int)(kd.coef_off / kNc), npc = kd.nint * kPieces;
                            int ga = piece_local(L.key[s0], iv, kd.nint, spt);
                            int gl = piece_local(L.key[s1 - 1], iv, kd.nint, spt) + 1;
                            gl = gl < npc ? gl : npc - 1;
                            int sa = s0;
                            bool done = false;
#pragma unroll
                            for (int sg = 0; sg < kSegMax; ++sg) {
                                if (done) continue;
                                int sb = s1, np = gl - ga + 1, last = 1;
                                if (np > kStage && sg + 1 < kSegMax) {
                                    np = kStage;
                                    const double rs = tv.meta[base + ga + kStage - 1].x;
                                    sb = lane_count_below(L.key, nvalid, rs, false);
                                    if (sb < s1) last = 0;
                                    else sb = s1;
                                }
                                np = np < kStage ? np : kStage;
                                if (sb > sa) {
                                    TileRec& R = out[sg];
                                    R.f = f;
                                    R.g0 = base + ga;
                                    R.s = (uint32_t)sa | ((uint32_t)sb << 12) | ((uint32_t)(np - 1) << 24);
                                    R.ki = (uint32_t)k | ((uint32_t)i << 13) | ((uint32_t)last << 26);
                                    R.g0l = ga | (kd.nint << 8);
                                    R.bpo = kd.bp_off;
                                    ok[sg] = true;
                                }
                                if (last) {
                                    done = true;
                                } else {
                                    sa = sb;
                                    ga = piece_local(L.key[sa], iv, kd.nint, spt);
                                }
                            }
                        }
                    }
                }
                // order-preserving compaction (at most 3 records a lane: two ballots)
                const int nr = (ok[0] ? 1 : 0) + (ok[1] ? 1 : 0) + (ok[2] ? 1 : 0);
                const uint64_t b0 = __ballot(nr & 1), b1 = __ballot(nr & 2);
                const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
                int pos = __popcll(b0 & below) + 2 * __popcll(b1 & below);
#pragma unroll
                for (int m = 0; m < kSegMax; ++m)
                    if (ok[m]) L.rec[pos++] = out[m];
                if (lane == 0) L.nrec = __popcll(b0) + 2 * __popcll(b1);
            }
            __syncthreads();
            const int nrec = L.nrec;
            if (nrec == 0) {
                __syncthreads();                     // every wave has read nrec before the next plan
                continue;
            }
            double2 st[kStageRegs];
            {
                const TileRec R0 = L.rec[0];
                stage_fetch<Tile>(R0, tv, st);
                stage_store<Tile>(R0, L.stage, st);
            }
            __syncthreads();
            for (int n = 0; n < nrec; ++n) {
                const TileRec R = L.rec[n];
                const int s0 = (int)(R.s & 4095u), s1 = (int)((R.s >> 12) & 4095u);
                const int np = (int)((R.s >> 24) & 63u) + 1, nint = R.g0l >> 8, g0l = R.g0l & 255;
                const int k = (int)(R.ki & 8191u), i = (int)((R.ki >> 13) & 8191u);
                const bool last = (R.ki >> 26) & 1u;
                const double2* sc = L.stage;
                const double2* sm = L.stage + kNc * np;
                const double2* si = sm + 2 * np;
                const double2 lohi = si[nint];
                const bool more = n + 1 < nrec;
                if (more) stage_fetch<Tile>(L.rec[n + 1], tv, st);
                if (!pv.y && k != kcur) {
                    // band addresses of the lane's entries of the merged vertex tile for time row k;
                    // the loads complete while the record is evaluated
                    kcur = k;
#pragma unroll
                    for (int h = 0; h < kDz; ++h) {
                        const int z = tid + h * kTileThreads;
                        dz_B[h] = 0;
                        if (z < kTileVt * kTileVs) {
                            const int a = z / kTileVs, b = z - kTileVs * a;
                            if (a < L.nvt && b < L.nvs) {
                                int l = L.vt[a], j = L.vs[b];
                                if (j > l) { const int tmp = j; j = l; l = tmp; }
                                const int64_t tix = (int64_t)k * band.nt + band_tile(l, j);
                                dz_ilo[h] = band.ilo[band_ilo_index(band, k, l, j)];
                                dz_B[h] = band.B[tix];
                                dz_vo[h] = band.voff[tix];
                                dz_lj[h] = (l % kBT) | ((j % kBT) << 8) | ((l == j ? 1 : 0) << 16);
                            }
                        }
                    }
                }

                // phase 1: the lane's chunk of sorted points, held in registers
                const int npt = s1 - s0;
                const int C = (npt + kTileThreads - 1) / kTileThreads;
                const int u0 = tid * C;
                const int cnt = max(0, min(npt - u0, C));
                double rr[kChunkMax];
                int cd[kChunkMax];
#pragma unroll
                for (int m = 0; m < kChunkMax; ++m) {
                    rr[m] = 0.0;
                    cd[m] = 0;
                    if (m < cnt) {
                        rr[m] = L.key[s0 + u0 + m];
                        cd[m] = L.idx[s0 + u0 + m];
                    }
                }
                if (cnt > 0) {
                    int rel = piece_local(rr[0], si, nint, spt) - g0l;
                    rel = rel < 0 ? 0 : (rel < np ? rel : np - 1);
                    double rhi = sm[2 * rel].x;
                    while (rr[0] >= rhi && rel + 1 < np) rhi = sm[2 * ++rel].x;
                    double rc = sm[2 * rel].y, ra = sm[2 * rel + 1].x;
                    double2 cc[kNc];
                    auto load_piece = [&]() {
#pragma unroll
                        for (int m = 0; m < kNc; ++m) cc[m] = sc[rel * kNc + m];
                    };
                    load_piece();
#pragma unroll
                    for (int m = 0; m < kChunkMax; ++m) {
                        if (m < cnt) {
                            const double r = rr[m];
                            if (r >= rhi && rel + 1 < np) {
                                // sorted neighbours: almost always the next piece, read with its
                                // coefficients in one round trip
                                ++rel;
                                const double2 ma = sm[2 * rel], mb = sm[2 * rel + 1];
                                load_piece();
                                rhi = ma.x;
                                rc = ma.y;
                                ra = mb.x;
                                if (r >= rhi && rel + 1 < np) {
                                    do {
                                        rhi = sm[2 * ++rel].x;
                                    } while (r >= rhi && rel + 1 < np);
                                    rc = sm[2 * rel].y;
                                    ra = sm[2 * rel + 1].x;
                                    load_piece();
                                }
                            }
                            const double x = (r - rc) * ra;
                            double ps, pt;
                            cheb_sums(cc, x, ps, pt);
                            const int code = cd[m];
                            const int qq = code - 49 * (code / 49);
                            const double w = L.wqq[qq] * recip(r);
                            L.V[code] = make_double2(ps * w, pt * w);
                        }
                    }
                    nq += (unsigned long long)cnt;
                }
                __syncthreads();
                if (last) {
                    // phase 2: lane (pair gp, row q = gm < 7) sums its row over q' into
                    // (R_0, R_1, R_2, T)(q), kept in the row's first two slots; lane gm then forms
                    // entry (a, b) = (gm / 3, gm % 3) (lane 0 also entry 8) over the 7 rows.  The
                    // 8 lanes of a pair belong to one wave.
                    const bool act = L.pok[gp] && L.pmax[gp] > lohi.x && L.pmin[gp] < lohi.y;
                    if (act) {
                        double2* prow = L.V + gp * 49;
                        if (gm < 7) {
                            double2* row = prow + gm * 7;
                            double R0 = 0.0, R1 = 0.0, R2 = 0.0, T = 0.0;
#pragma unroll
                            for (int qp = 0; qp < 7; ++qp) {
                                const double2 v = row[qp];
                                double l0, l1, l2, w;
                                rule7_point(qp, l0, l1, l2, w);
                                R0 = fma(l0, v.x, R0);
                                R1 = fma(l1, v.x, R1);
                                R2 = fma(l2, v.x, R2);
                                T += v.y;
                            }
                            row[0] = make_double2(R0, R1);
                            row[1] = make_double2(R2, T);
#pragma unroll
                            for (int qp = 2; qp < 7; ++qp) row[qp] = make_double2(0.0, 0.0);
                        }
                        __threadfence_block();
                        const int eb = gm - 3 * (gm / 3);
                        double S = 0.0, S8 = 0.0, T = 0.0;
#pragma unroll
                        for (int q = 0; q < 7; ++q) {
                            const double* rq = reinterpret_cast<const double*>(prow + q * 7);
                            double l0, l1, l2, w;
                            rule7_point(q, l0, l1, l2, w);
                            S = fma(la[q], rq[eb], S);
                            S8 = fma(l2, rq[2], S8);
                            T += rq[3];
                        }
                        __threadfence_block();
                        if (gm < 7) {
                            double2* row = prow + gm * 7;
                            row[0] = make_double2(0.0, 0.0);
                            row[1] = make_double2(0.0, 0.0);
                        }
                        const double al = L.alpha[gp];
                        if constexpr (Fixed) {
                            unsigned long long* acq = reinterpret_cast<unsigned long long*>(L.acc);
                            atomicAdd(acq + L.aoff[9 * gp + gm], to_fixed(fma(al, S, L.beta[9 * gp + gm] * T), fxs));
                            if (gm == 0)
                                atomicAdd(acq + L.aoff[9 * gp + 8], to_fixed(fma(al, S8, L.beta[9 * gp + 8] * T), fxs));
                        } else {
                            atomicAdd(&L.acc[L.aoff[9 * gp + gm]], fma(al, S, L.beta[9 * gp + gm] * T));
                            if (gm == 0)
                                atomicAdd(&L.acc[L.aoff[9 * gp + 8]], fma(al, S8, L.beta[9 * gp + 8] * T));
                        }
                    }
                }
                // the next record's pieces go to LDS only now (phase 2 does not read them), so their
                // global loads have had phase 1 and phase 2 to arrive
                if (more) stage_store<Tile>(L.rec[n + 1], L.stage, st);
                __syncthreads();
                if (last) {
#pragma unroll
                    for (int h = 0; h < kDz; ++h) {
                        const int z = tid + h * kTileThreads;
                        if constexpr (Fixed) {
                            // integer sums of the tile go to the storage as they are
                            unsigned long long* acq = reinterpret_cast<unsigned long long*>(L.acc);
                            if (z < kTileVt * kTileVs && acq[z] != 0ull) {
                                const unsigned long long q = acq[z];
                                if (dz_B[h] > 0) {
                                    const int s = i - dz_ilo[h];
                                    if (s >= 0 && s < dz_B[h]) {
                                        const int lr = dz_lj[h] & 255, jr = (dz_lj[h] >> 8) & 255;
                                        const int64_t idx = dz_vo[h] + ((int64_t)lr * dz_B[h] + s) * kBT + jr;
                                        atomicAdd(reinterpret_cast<unsigned long long*>(val) + idx,
                                                  (dz_lj[h] >> 16) ? 2ull * q : q);
                                    }
                                }
                                acq[z] = 0ull;
                            }
                            continue;
                        }
                        if (z < kTileVt * kTileVs) {
                            const double v = L.acc[z];
                            if (v != 0.0) {
                                if (pv.y) {
                                    const int a = z / kTileVs, b = z - kTileVs * a;
                                    deposit(band, val, valf, pv, k, i, L.vt[a], L.vs[b], v);
                                } else if (dz_B[h] > 0) {
                                    const int s = i - dz_ilo[h];
                                    if (s >= 0 && s < dz_B[h]) {
                                        const int lr = dz_lj[h] & 255, jr = (dz_lj[h] >> 8) & 255;
                                        const int64_t idx = dz_vo[h] + ((int64_t)lr * dz_B[h] + s) * kBT + jr;
                                        const double vv = (dz_lj[h] >> 16) ? 2.0 * v : v;
                                        if (valf) atomicAdd(valf + idx, (float)vv);
                                        else atomicAdd(val + idx, vv);
                                    }
                                }
                                L.acc[z] = 0.0;
                            }
                        }
                    }
                }
            }
        }
    }
    const unsigned long long tot = wave_sum_u64(nq);
    if ((tid & 63) == 0 && tot) atomicAdd(counter, tot);
}

// ---------------------------------------------------------------------------------------------
// Singular pairs.  pairs[9*s..]: tau, sigma, kind (0 coincident, 1 edge, 2 vertex), the local
// indices of the reference vertices (A, B, C) in tau and in sigma.  The rule rows are
// (x1, x2, y1, y2, w) on the reference triangle {0 <= x2 <= x1 <= 1}, the physical point
// A + x1 (B - A) + x2 (C - B) with barycentrics (1 - x1, x1 - x2, x2).
// One workgroup per pair: the distances of the pair's Sauter-Schwab points are sorted once in
// LDS; the lanes then take (k, i) kernels, each walking the contiguous range of sorted points
// inside its support with the piece record of its current Chebyshev piece in registers (sorted
// distances move through the pieces in order), the nine local sums in registers, and nine
// scatters at the end.
// ---------------------------------------------------------------------------------------------
constexpr int kSingThreads = 256;
constexpr int kSingU = 8;      // trial indices of one time row taken in one round

__global__ void __launch_bounds__(kSingThreads)
k_singular(GeomView g, TableView tv, const double* __restrict__ t, BandView band, const int32_t* __restrict__ pairs,
           const double* __restrict__ rules, const int32_t* __restrict__ roff, const int32_t* __restrict__ rcnt,
           int P, double* val, float* valf, ProductView pv, unsigned long long* counter, double fxs)
{
    extern __shared__ double sing_lds[];
    double* key = sing_lds;                                   // P sorted distances
    uint16_t* idx = reinterpret_cast<uint16_t*>(sing_lds + P);   // their rule rows
    const int tid = threadIdx.x;
    const int E = g.E, N = tv.N;
    const int32_t* pr = pairs + 9 * (int64_t)blockIdx.x;
    const int tau = pr[0], sig = pr[1], kind = pr[2];
    const int px[3] = {pr[3], pr[4], pr[5]}, py[3] = {pr[6], pr[7], pr[8]};
    double X[3][3], Y[3][3];   // reference vertices A, B, C
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) {
            X[a][c] = g.P[(3 * px[a] + c) * E + tau];
            Y[a][c] = g.P[(3 * py[a] + c) * E + sig];
        }
    const int npts = rcnt[kind];
    const double* rule = rules + 5 * (int64_t)roff[kind];
    for (int q = tid; q < P; q += kSingThreads) {
        double r = INFINITY;
        if (q < npts) {
            const double* R = rule + 5 * q;
            const double x1 = R[0], x2 = R[1], y1 = R[2], y2 = R[3];
            const double lx0 = 1.0 - x1, lx1 = x1 - x2, lx2 = x2;
            const double ly0 = 1.0 - y1, ly1 = y1 - y2, ly2 = y2;
            double d2 = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double xc = lx0 * X[0][c] + lx1 * X[1][c] + lx2 * X[2][c];
                const double yc = ly0 * Y[0][c] + ly1 * Y[1][c] + ly2 * Y[2][c];
                d2 += (xc - yc) * (xc - yc);
            }
            r = sqrt(d2);
        }
        key[q] = r;
        idx[q] = (uint16_t)q;
    }
    for (int size = 2; size <= P; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int u = tid; u < P / 2; u += kSingThreads) {
                const int lo = 2 * stride * (u / stride) + (u % stride);
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const double ka = key[lo], kb = key[hi];
                if ((ka > kb) == up) {
                    key[lo] = kb;
                    key[hi] = ka;
                    const uint16_t ia = idx[lo];
                    idx[lo] = idx[hi];
                    idx[hi] = ia;
                }
            }
        }
    __syncthreads();
    const double rmax = key[npts - 1];
    const double nn = g.n[tau] * g.n[sig] + g.n[E + tau] * g.n[E + sig] + g.n[2 * E + tau] * g.n[2 * E + sig];
    const double jac = 4.0 * g.area[tau] * g.area[sig];
    unsigned long long nq = 0;
    for (int c = tid; c < N * kSingU; c += kSingThreads) {
        const int k = c / kSingU, u = c - kSingU * (c / kSingU);
        // first trial index whose support starts below rmax (lo_{k,i} falls as i grows); the
        // supports of trial nodes beyond the test node + 1 are empty
        const int ib = min((k / tv.p1 + 2) * tv.p1, N) - 1;
        int ia = 0, span = ib + 1;
        while (span > 0) {
            const int h = span >> 1;
            double lo, hi;
            kernel_support(t, tv.nodes, tv.p1, k, ia + h, lo, hi);
            if (lo < rmax) span = h;
            else { ia += h + 1; span -= h + 1; }
        }
        for (int i = ia + u; i <= ib; i += kSingU) {
            const int f = tv.fid[k * N + i];
            if (f < 0) continue;
            const KernelDesc kd = tv.desc[f];
            // sorted range inside the open support (lo, hi)
            int s0 = 0, s1 = 0;
            {
                int b = 0, n = npts;
                while (n > 0) { const int h = n >> 1; if (key[b + h] <= kd.lo) { b += h + 1; n -= h + 1; } else n = h; }
                s0 = b;
                b = 0; n = npts;
                while (n > 0) { const int h = n >> 1; if (key[b + h] < kd.hi) { b += h + 1; n -= h + 1; } else n = h; }
                s1 = b;
            }
            if (s1 <= s0) continue;
            double S1[9], S2 = 0.0;
#pragma unroll
            for (int m = 0; m < 9; ++m) S1[m] = 0.0;
            double2 cc[kNc];
            double rhi = -1.0, rc = 0.0, ra = 0.0;
            int64_t gcur = -1;
            for (int sidx = s0; sidx < s1; ++sidx) {
                const double r = key[sidx];
                if (r >= rhi) {
                    int64_t gp;
                    if (gcur < 0) {
                        int cl = (int)((r - kd.lo) * kd.cell_scale);
                        cl = cl < 0 ? 0 : (cl < kCells ? cl : kCells - 1);
                        gp = kd.coef_off / kNc + tv.cell[kd.cell_off + cl];
                    } else {
                        gp = gcur + 1;
                    }
                    double4 mt = tv.meta[gp];
                    while (r >= mt.x) mt = tv.meta[++gp];
                    gcur = gp;
                    rhi = mt.x;
                    rc = mt.y;
                    ra = mt.z;
#pragma unroll
                    for (int m = 0; m < kNc; ++m) cc[m] = tv.coef[gp * kNc + m];
                }
                double ps, pt;
                cheb_sums(cc, (r - rc) * ra, ps, pt);
                const double* R = rule + 5 * idx[sidx];
                const double x1 = R[0], x2 = R[1], y1 = R[2], y2 = R[3];
                const double wr = R[4] * jac / r;
                const double lx0 = 1.0 - x1, lx1 = x1 - x2, lx2 = x2;
                const double ly0 = 1.0 - y1, ly1 = y1 - y2, ly2 = y2;
                const double f1 = ps * wr;
                const double R0 = f1 * ly0, R1 = f1 * ly1, R2 = f1 * ly2;
                S1[0] = fma(lx0, R0, S1[0]); S1[1] = fma(lx0, R1, S1[1]); S1[2] = fma(lx0, R2, S1[2]);
                S1[3] = fma(lx1, R0, S1[3]); S1[4] = fma(lx1, R1, S1[4]); S1[5] = fma(lx1, R2, S1[5]);
                S1[6] = fma(lx2, R0, S1[6]); S1[7] = fma(lx2, R1, S1[7]); S1[8] = fma(lx2, R2, S1[8]);
                S2 = fma(pt, wr, S2);
            }
            nq += (unsigned long long)(s1 - s0);
            const double scale = 0.07957747154594767;   // 1/(4 pi)
            double loc[3][3];
#pragma unroll
            for (int al = 0; al < 3; ++al)
#pragma unroll
                for (int be = 0; be < 3; ++be) {
                    const double C = g.curl[(3 * px[al]) * E + tau] * g.curl[(3 * py[be]) * E + sig] +
                                     g.curl[(3 * px[al] + 1) * E + tau] * g.curl[(3 * py[be] + 1) * E + sig] +
                                     g.curl[(3 * px[al] + 2) * E + tau] * g.curl[(3 * py[be] + 2) * E + sig];
                    loc[al][be] = (nn * S1[3 * al + be] + C * S2) * scale;
                }
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
            }
            const double half = kind == 0 ? 0.5 : 1.0;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    deposit(band, val, valf, pv, k, i, g.v[px[a] * E + tau], g.v[py[b] * E + sig], half * loc[a][b],
                            fxs);
        }
    }
    const unsigned long long tot = wave_sum_u64(nq);
    if ((tid & 63) == 0 && tot) atomicAdd(counter, tot);
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
        const int B = band_width(band, kk, ll, jj);
        const int sl = ii - (int)band.ilo[band_ilo_index(band, kk, ll, jj)];
        if (sl >= 0 && sl < B) {
            const int64_t idx = band_value_index(band, kk, ll, jj, sl, B);
            v = valf ? (double)valf[idx] : val[idx];
        }
    }
    out[s] = v;
}

// Entries of one block A_{k,i} (eqs. (Apartitioned), (SparsitySmallBlock)): one lane per stored
// lower-triangle slot (l, j <= l) of time row k; a slot whose band holds i and whose value is not
// zero gives (l, j) and, off the diagonal, the mirrored (j, l).  Positions come from an atomic
// counter (the host sorts); with row == nullptr only the count is formed.
__global__ void __launch_bounds__(256)
k_block_coo(BandView band, const double* __restrict__ val, const float* __restrict__ valf, int k, int i,
            unsigned long long* __restrict__ count, int32_t* __restrict__ row, int32_t* __restrict__ col,
            double* __restrict__ out, int64_t cap)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= band.nt * kBT * kBT) return;
    const int64_t tt = s / (kBT * kBT);
    const int rem = (int)(s - tt * (kBT * kBT));
    int tl = (int)((sqrt(8.0 * (double)tt + 1.0) - 1.0) * 0.5);
    while ((int64_t)(tl + 1) * (tl + 2) / 2 <= tt) ++tl;
    while ((int64_t)tl * (tl + 1) / 2 > tt) --tl;
    const int tj = (int)(tt - (int64_t)tl * (tl + 1) / 2);
    const int l = tl * kBT + rem / kBT, j = tj * kBT + rem % kBT;
    if (l >= band.M || j > l) return;
    const int B = band_width(band, k, l, j);
    const int sl = i - (int)band.ilo[band_ilo_index(band, k, l, j)];
    if (sl < 0 || sl >= B) return;
    const int64_t idx = band_value_index(band, k, l, j, sl, B);
    const double v = valf ? (double)valf[idx] : val[idx];
    if (v == 0.0) return;
    const unsigned long long pos = atomicAdd(count, j < l ? 2ull : 1ull);
    if (!row) return;
    if ((int64_t)pos < cap) { row[pos] = l; col[pos] = j; out[pos] = v; }
    if (j < l && (int64_t)pos + 1 < cap) { row[pos + 1] = j; col[pos + 1] = l; out[pos + 1] = v; }
}

// Staging of the allocation-free entry query (tdbem_get_entries_noalloc): the four index arrays and
// the results of up to kNoAllocEntries entries, in one statically allocated device array.  Host
// code never passes the array's name to a kernel or a copy: it uses the device address that
// hipGetSymbolAddress returns for the current device (each device holds its own copy).
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(int device, void** ptr)
{
    static std::mutex mu;
    static std::map<int, void*> addr;
    std::lock_guard<std::mutex> lock(mu);
    const auto it = addr.find(device);
    if (it != addr.end()) {
        *ptr = it->second;
        return hipSuccess;
    }
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));   // the caller made `device` current
    if (e != hipSuccess) return e;
    addr[device] = p;
    *ptr = p;
    return hipSuccess;
}

static inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_geometry(const double* xyz, const int32_t* tri, int E, double* geo_P, double* geo_n, double* geo_area,
                     double* geo_curl, double* geo_qp, int32_t* geo_v, hipStream_t s)
{
    hipLaunchKernelGGL(k_geometry, dim3(grid_for(E, 256)), dim3(256), 0, s, xyz, tri, E, geo_P, geo_n, geo_area,
                       geo_curl, geo_qp, geo_v);
}

void launch_layout(BandView band, const double* xyz, const double* rho, const double* t, int16_t* ilo, int32_t* Bt,
                   hipStream_t s)
{
    hipLaunchKernelGGL(k_layout, dim3((unsigned)band.nt), dim3(256), sizeof(int32_t) * band.N, s, band, xyz, rho, t,
                       ilo, Bt);
}

int tile_variants() { return 2; }

void tile_shape(int variant, int* test, int* trial)
{
    *test = variant == 1 ? TileB::kT : TileA::kT;
    *trial = variant == 1 ? TileB::kS : TileA::kS;
}

void launch_regular(GeomView g, TableView tv, const double* t, BandView band, double* val, float* valf,
                    const double* px, double* py, const int2* tiles, int64_t ntiles, int variant,
                    unsigned long long* counter, hipStream_t s, double fxs)
{
    if (ntiles <= 0) return;
    const dim3 grid((unsigned)(8 * ((ntiles + 7) / 8)));
    const ProductView pv{px, py, band.M};
    if (fxs > 0.0) {
        if (variant == 1)
            hipLaunchKernelGGL((k_regular_tile<TileB, false, true>), grid, dim3(TileB::kThreads), 0, s, g, tv, t,
                               band, val, nullptr, pv, tiles, ntiles, counter, nullptr, fxs);
        else
            hipLaunchKernelGGL((k_regular_tile<TileA, false, true>), grid, dim3(TileA::kThreads), 0, s, g, tv, t,
                               band, val, nullptr, pv, tiles, ntiles, counter, nullptr, fxs);
    } else if (variant == 1) {
        hipLaunchKernelGGL((k_regular_tile<TileB, false, false>), grid, dim3(TileB::kThreads), 0, s, g, tv, t, band,
                           val, valf, pv, tiles, ntiles, counter, nullptr, 0.0);
    } else {
        hipLaunchKernelGGL((k_regular_tile<TileA, false, false>), grid, dim3(TileA::kThreads), 0, s, g, tv, t, band,
                           val, valf, pv, tiles, ntiles, counter, nullptr, 0.0);
    }
}

void launch_regular_multi(const RegularProblem* probs, const int2* tiles, int64_t ntiles, hipStream_t s)
{
    if (ntiles <= 0) return;
    const dim3 grid((unsigned)(8 * ((ntiles + 7) / 8)));
    const ProductView pv{nullptr, nullptr, 0};
    hipLaunchKernelGGL((k_regular_tile<TileA, true, false>), grid, dim3(TileA::kThreads), 0, s, GeomView{},
                       TableView{}, nullptr, BandView{}, nullptr, nullptr, pv, tiles, ntiles, nullptr, probs, 0.0);
}

// Tiles (tau tile a, sigma tile b) of the regular-pair kernel holding at least one sigma > tau, in
// Morton (Z) order over squares of triangle index space: the key interleaves the bits of the test
// and trial triangle ranges in units of TS triangles (a TT-triangle test tile is TS / TT of a
// unit).  Each XCD takes one contiguous range of the list, so the workgroups it runs together cover
// a compact patch of (tau, sigma) pairs at similar distances, which need the same Chebyshev
// windows: the stage loads hit its L2 more often.  On the 5120-triangle sphere with 64 bases:
// 1.54 s against 1.60 s in row order (units of TT x TS triangles: 1.58 s; of 2 TS: 1.58 s).
std::vector<int32_t> regular_tiles(int E, int variant)
{
    int TT, TS;
    tile_shape(variant, &TT, &TS);
    const int nA = (E + TT - 1) / TT, nB = (E + TS - 1) / TS, per = TS / TT > 0 ? TS / TT : 1;
    std::vector<std::pair<uint64_t, int64_t>> keyed;
    for (int a = 0; a < nA; ++a)
        for (int b = 0; b < nB; ++b)
            if (b * TS + TS - 1 > a * TT) {
                const uint32_t x = (uint32_t)(a / per), y = (uint32_t)b;
                uint64_t key = 0;
                for (int bit = 0; bit < 21; ++bit)
                    key |= ((uint64_t)((x >> bit) & 1u) << (2 * bit)) | ((uint64_t)((y >> bit) & 1u) << (2 * bit + 1));
                keyed.push_back({key, (int64_t)a * nB + b});
            }
    std::stable_sort(keyed.begin(), keyed.end(),
                     [](const std::pair<uint64_t, int64_t>& p, const std::pair<uint64_t, int64_t>& q) {
                         return p.first < q.first;
                     });
    std::vector<int32_t> out;
    out.reserve(2 * keyed.size());
    for (const auto& kv : keyed) {
        out.push_back((int32_t)(kv.second / nB));
        out.push_back((int32_t)(kv.second % nB));
    }
    return out;
}

void launch_singular(GeomView g, TableView tv, const double* t, BandView band, const int32_t* pairs, int64_t npairs,
                     const double* ss_rules, const int32_t* ss_off, const int32_t* ss_cnt, int max_points, double* val,
                     float* valf, const double* px, double* py, unsigned long long* counter, hipStream_t s,
                     double fxs)
{
    if (npairs <= 0) return;
    int P = 64;
    while (P < max_points) P <<= 1;
    const size_t lds = (size_t)P * (sizeof(double) + sizeof(uint16_t));
    const ProductView pv{px, py, band.M};
    hipLaunchKernelGGL(k_singular, dim3((unsigned)npairs), dim3(kSingThreads), lds, s, g, tv, t, band, pairs, ss_rules,
                       ss_off, ss_cnt, P, val, valf, pv, counter, fxs);
}

void launch_get_entries(BandView band, const double* val, const float* valf, int64_t n, const int32_t* k,
                        const int32_t* i, const int32_t* j, const int32_t* l, double* out, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_get_entries, dim3(grid_for(n, 256)), dim3(256), 0, s, band, val, valf, n, k, i, j, l, out);
}

void launch_block_coo(BandView band, const double* val, const float* valf, int k, int i, unsigned long long* count,
                      int32_t* row, int32_t* col, double* out, int64_t cap, hipStream_t s)
{
    const int64_t n = band.nt * kBT * kBT;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_block_coo, dim3(grid_for(n, 256)), dim3(256), 0, s, band, val, valf, k, i, count, row, col,
                       out, cap);
}

}  // namespace tdbem
