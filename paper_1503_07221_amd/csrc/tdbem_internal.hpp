// Internal definitions shared by the HIP kernels and the host runtime of libtdbem.
//
// Notation (0-based): time nodes t_0 = 0 < ... < t_{N-1} = T with one temporal basis b_i per
// node (p = 0), vertices j, l in [0, M), triangles in [0, E).  A_{k,i}(j, l) is the entry of
// eq. (MatrixEntries): test pair (b_k, phi_l) in x, trial pair (b_i, phi_j) in y.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace tdbem {

// ---------------------------------------------------------------------------------------------
// Piecewise Chebyshev tables of psi_{k,i} and tilde psi_{k,i} (Section 3.1).
// The support of each kernel is cut at every node difference t_c - t_a (the points where the
// kernel stops being analytic) into "intervals"; every interval is cut by one fixed partition
// of [0, 1] that is graded geometrically (ratio 1.6, down to 0.02) towards both ends, where
// the kernels are flat, and uniform (width <= 0.2) in the middle: kPieces pieces.  On each piece
// both kernels are interpolated at kNc Chebyshev points of the first kind (degree kDeg) and
// evaluated with Clenshaw's recurrence.
// ---------------------------------------------------------------------------------------------
constexpr int kDeg = 14;
constexpr int kNc = kDeg + 1;
constexpr int kPieces = 16;
constexpr int kMaxIntervals = 9;   // at most 3 x 3 node differences split a support

struct KernelDesc {
    double lo, hi;        // open support (lo, hi) of psi_{k,i} in r >= 0
    int32_t nint;         // number of intervals
    int32_t bp_off;       // interval starts and inverse lengths: ivl[bp_off + 2*j], ivl[bp_off + 2*j + 1]
    int64_t coef_off;     // first double2 of this kernel: coef[coef_off + (j*kPieces + p)*kNc + m]
    double cell_scale;    // kCells / (length of the tabulated range starting at lo)
    int32_t cell_off;     // first entry of this kernel in the cell table
    int32_t pad;
};

// Per-piece record (piece g = coef offset / kNc): the piece covers r < rhi (and r at or above the
// previous piece's rhi), x = (r - rc) * ra maps it onto [-1, 1]; near = 1 for the pieces of the
// first half of the first interval and the second half of the last one (the flat ends of the
// support).  The cell table splits [lo, end) of every kernel into kCells equal cells and holds
// the first piece (kernel-local index) that meets each cell.
constexpr int kCells = 256;

// Graded partition of [0, 1] into kPieces pieces: edges, inverse widths and a lookup table
// lut[c] = the piece containing c / kLutCells.  Every piece is wider than one cell, so the piece
// of any point is lut[cell] or the next one.  Kernels copy it to LDS.
constexpr int kLutCells = 1024;
struct PieceTable {
    double edge[kPieces + 1];
    double inv_width[kPieces];
    uint8_t lut[kLutCells];
};

__device__ inline void load_piece_table(PieceTable& dst, const PieceTable& src)
{
    for (int s = threadIdx.x; s <= kPieces; s += blockDim.x) dst.edge[s] = src.edge[s];
    for (int s = threadIdx.x; s < kPieces; s += blockDim.x) dst.inv_width[s] = src.inv_width[s];
    for (int s = threadIdx.x; s < kLutCells; s += blockDim.x) dst.lut[s] = src.lut[s];
}

// ---------------------------------------------------------------------------------------------
// Smooth cutoff F on [0, 1] with F', F'' (Section 3).
//   bump: F(u) = beta(u-1) / (beta(u-1) + beta(u)), beta(s) = exp(-1/(1 - s^2)), i.e.
//         F = 1 / (1 + e^g) with g(u) = 1/(u(2-u)) - 1/(1-u^2);
//   erf:  F(u) = f(2u - 1), f(s) = erf(2 artanh s)/2 + 1/2.
// ---------------------------------------------------------------------------------------------
__host__ __device__ inline void cutoff_eval(int kind, double u, double& F, double& F1, double& F2)
{
    if (u <= 0.0) { F = 0.0; F1 = 0.0; F2 = 0.0; return; }
    if (u >= 1.0) { F = 1.0; F1 = 0.0; F2 = 0.0; return; }
    if (kind == 0) {
        const double p = u * (2.0 - u);          // 1 - (u-1)^2
        const double q = (1.0 - u) * (1.0 + u);  // 1 - u^2
        const double dp = 2.0 - 2.0 * u, dq = -2.0 * u;
        const double g = 1.0 / p - 1.0 / q;
        const double g1 = dq / (q * q) - dp / (p * p);
        // d/du (-p'/p^2) = (2 p + 2 p'^2)/p^3 since p'' = -2; same for q with the opposite sign
        const double g2 = (2.0 * p + 2.0 * dp * dp) / (p * p * p) - (2.0 * q + 2.0 * dq * dq) / (q * q * q);
        const double e = exp(-fabs(g));
        const double f = g > 0.0 ? e / (1.0 + e) : 1.0 / (1.0 + e);
        const double s = e / ((1.0 + e) * (1.0 + e));      // f (1 - f)
        F = f;
        F1 = -g1 * s;
        F2 = -g2 * s + g1 * g1 * s * (1.0 - 2.0 * f);
    } else {
        const double s = 2.0 * u - 1.0;
        const double om = (1.0 - s) * (1.0 + s);
        const double at = 0.5 * log((1.0 + s) / (1.0 - s));
        const double z = 2.0 * at;
        const double d1 = 1.1283791670955126 * exp(-z * z) / om;   // f'(s), 2/sqrt(pi)
        F = 0.5 + 0.5 * erf(z);
        F1 = 2.0 * d1;
        F2 = 4.0 * d1 * (2.0 * s - 8.0 * at) / om;
    }
}

// Temporal basis b_j, j = n p1 + m (node n of the N nodes, Legendre degree m < p1 = p + 1), with
// first and second derivative (Section 3, eq. (BasisFunctions)): mu_n from the cutoff on
// [t_{n-1}, t_n] (rising) and [t_n, t_{n+1}] (falling), mu_{N-1} = 1 after T, every basis 0 for
// negative arguments (causality), the causal factor 8 (t/h_1)^2 on node 0, times the Legendre
// polynomial P_m of the support mapped onto [-1, 1]: [0, t_1] for n = 0, [t_{n-1}, t_{n+1}] for the
// inner nodes (the paper's (t - t_n)/Delta t on equidistant grids), [t_{N-2}, T] for n = N - 1.
__host__ __device__ inline void basis_eval(const double* t, int N, int p1, int cut, int j, double x,
                                           double& v, double& d1, double& d2)
{
    v = 0.0; d1 = 0.0; d2 = 0.0;
    if (x < 0.0) return;
    const int n = j / p1, m = j - n * p1;
    double F, F1, F2;
    if (n > 0 && x > t[n - 1] && x <= t[n]) {
        const double h = t[n] - t[n - 1], ih = 1.0 / h;
        cutoff_eval(cut, (x - t[n - 1]) * ih, F, F1, F2);
        v = F; d1 = F1 * ih; d2 = F2 * ih * ih;
    } else if (n < N - 1 && x >= t[n] && x < t[n + 1]) {
        const double h = t[n + 1] - t[n], ih = 1.0 / h;
        cutoff_eval(cut, (x - t[n]) * ih, F, F1, F2);
        v = 1.0 - F; d1 = -F1 * ih; d2 = -F2 * ih * ih;
    } else if (n == N - 1 && x > t[N - 1]) {
        v = 1.0;
    }
    if (n == 0) {
        if (x <= 0.0) { v = d1 = d2 = 0.0; return; }
        const double ih = 1.0 / (t[1] - t[0]);
        const double u = x * ih;
        const double c = 8.0 * u * u, c1 = 16.0 * u * ih, c2 = 16.0 * ih * ih;
        const double nv = c * v, nd1 = c1 * v + c * d1, nd2 = c2 * v + 2.0 * c1 * d1 + c * d2;
        v = nv; d1 = nd1; d2 = nd2;
    }
    if (m == 0) return;
    const double lo = n == 0 ? 0.0 : t[n - 1];
    const double hi = n == N - 1 ? t[N - 1] : (n == 0 ? t[1] : t[n + 1]);
    const double a = 2.0 / (hi - lo), s = a * (x - lo) - 1.0;
    // P_m, P_m', P_m'' by the three-term recurrence and P_q' = P_{q-2}' + (2q - 1) P_{q-1}
    double p0 = 1.0, p0d = 0.0, p0dd = 0.0, q1 = s, q1d = 1.0, q1dd = 0.0;
    for (int q = 2; q <= m; ++q) {
        const double pv = ((2.0 * q - 1.0) * s * q1 - (q - 1.0) * p0) / q;
        const double pd = p0d + (2.0 * q - 1.0) * q1;
        const double pdd = p0dd + (2.0 * q - 1.0) * q1d;
        p0 = q1; p0d = q1d; p0dd = q1dd;
        q1 = pv; q1d = pd; q1dd = pdd;
    }
    const double nv = v * q1, nd1 = d1 * q1 + v * q1d * a, nd2 = d2 * q1 + 2.0 * d1 * q1d * a + v * q1dd * a * a;
    v = nv; d1 = nd1; d2 = nd2;
}

// Open support of psi_{k,i} (Section 3.2) for the bases k, i (nodes k / p1, i / p1):
// (t_{k-1} - t_{i+1}, t_{k+1} - t_{i-1}) cap r > 0 with t_{-1} := 0 and t_N := T.
__host__ __device__ inline void kernel_support(const double* t, int N, int p1, int kb, int ib, double& lo, double& hi)
{
    const int k = kb / p1, i = ib / p1;
    const double tkm = t[k > 0 ? k - 1 : 0], tkp = t[k < N - 1 ? k + 1 : N - 1];
    const double tim = t[i > 0 ? i - 1 : 0], tip = t[i < N - 1 ? i + 1 : N - 1];
    lo = tkm - tip > 0.0 ? tkm - tip : 0.0;
    hi = tkp - tim;
}

// Clenshaw evaluation of two Chebyshev series with interleaved coefficients c[m] = (psi, tpsi).
__device__ inline void clenshaw2(const double2* __restrict__ c, double x, double& ps, double& pt)
{
    const double x2 = 2.0 * x;
    double a1 = 0.0, a2 = 0.0, b1 = 0.0, b2 = 0.0;
#pragma unroll
    for (int m = kDeg; m >= 1; --m) {
        const double2 cm = c[m];
        const double a0 = fma(x2, a1, cm.x - a2);
        const double b0 = fma(x2, b1, cm.y - b2);
        a2 = a1; a1 = a0; b2 = b1; b1 = b0;
    }
    const double2 c0 = c[0];
    ps = fma(x, a1, c0.x - a2);
    pt = fma(x, b1, c0.y - b2);
}

// Device-side table handle (passed by value as a kernel argument).
struct TableView {
    const KernelDesc* desc;   // one per tabulated (k, i)
    const int32_t* fid;       // fid[k*N + i]: index into desc or -1 (identically zero kernel), N = L
    const double* ivl;        // interval starts and inverse lengths
    const double2* coef;      // Chebyshev coefficients (psi, tpsi)
    const double4* meta;      // per-piece record (rhi, rc, ra, near)
    const uint16_t* cell;     // cell table
    int32_t N;                // temporal bases L = nodes (p + 1)
    int32_t nodes, p1;        // time nodes and bases per node
    PieceTable pt;
};

// Gauss-Legendre rule on [-1, 1] used for every time integral of the library.
constexpr int kTimeGauss = 20;
struct TimeRule {
    double x[kTimeGauss];
    double w[kTimeGauss];
};
// Dyadic grading of a smooth sub-interval towards both ends (the integrands are flat there):
// pieces [0,1/64], [1/64,1/32], ..., [1/4,1/2] and mirrored, 12 pieces.
__host__ __device__ inline double time_grading_edge(int g)
{
    // g = 0..12
    const double e[13] = {0.0, 1.0 / 64, 1.0 / 32, 1.0 / 16, 1.0 / 8, 1.0 / 4, 0.5,
                          0.75, 0.875, 0.9375, 0.96875, 63.0 / 64, 1.0};
    return e[g];
}
constexpr int kTimePieces = 12;

// psi_{k,i}(r), tilde psi_{k,i}(r) from the tables; false (and zeros) outside the open support.
// pt lives in LDS.  The interval is found by counting the interval starts below r (the starts
// are the same for all lanes of a wave when (k, i) is wave-uniform).
__device__ inline bool table_eval(const KernelDesc& kd, const double* __restrict__ ivl,
                                  const double2* __restrict__ coef, const PieceTable& pt,
                                  double r, double& ps, double& tps)
{
    ps = 0.0; tps = 0.0;
    if (!(r > kd.lo && r < kd.hi)) return false;
    const double* iv = ivl + kd.bp_off;
    int j = 0;
    for (int m = 1; m < kd.nint; ++m) j += r >= iv[2 * m] ? 1 : 0;
    double fr = (r - iv[2 * j]) * iv[2 * j + 1];
    fr = fr < 0.0 ? 0.0 : (fr > 1.0 ? 1.0 : fr);
    int cell = (int)(fr * kLutCells);
    cell = cell < kLutCells ? cell : kLutCells - 1;
    int p = pt.lut[cell];
    if (p + 1 < kPieces && fr >= pt.edge[p + 1]) ++p;
    const double x = 2.0 * (fr - pt.edge[p]) * pt.inv_width[p] - 1.0;
    clenshaw2(coef + kd.coef_off + (int64_t)(j * kPieces + p) * kNc, x, ps, tps);
    return true;
}

// ---------------------------------------------------------------------------------------------
// Triangle geometry, structure of arrays (lane = triangle).
// ---------------------------------------------------------------------------------------------
struct GeomView {
    const int32_t* v;      // v[a*E + e]: global vertex a of triangle e
    const double* P;       // P[(3*a + c)*E + e]: vertex coordinates
    const double* n;       // n[c*E + e]: unit normal
    const double* area;    // area[e]
    const double* curl;    // curl[(3*a + c)*E + e] = -e_a / (2|tau|) (tangential rotation of lambda_a)
    const double* qp;      // qp[(3*q + c)*E + e]: the 7 quadrature points
    int32_t E;
};

// Band storage of the blocks.  Every block is symmetric in (j, l), so only the lower triangle
// j <= l is kept.  For every vertex pair (l, j <= l) and time row k the trial indices
// i = ilo + s, s < B, are those whose kernel support meets the conservative distance range of the
// two hats (eq. (SparsitySmallBlock)).  The triangle is cut into 64 x 64 vertex tiles
// (tl, tj <= tl), numbered t = tl(tl+1)/2 + tj (nt of them).  Each (time row k, tile t) has its
// own band width B = B[k nt + t] (the widest band of its vertex pairs) and holds
// [row l % 64][slot s][column j % 64] from voff[k nt + t] on, so the values a workgroup of the
// matvec reads form one contiguous stretch:
//   ilo[(k nt + t) 4096 + (l % 64) 64 + j % 64]
//   val[voff[k nt + t] + ((l % 64) B + s) 64 + j % 64]
// Tile entries outside the triangle or past M stay zero.
constexpr int kBT = 64;
__host__ __device__ inline int64_t tri_index(int64_t l, int64_t j) { return l * (l + 1) / 2 + j; }
__host__ __device__ inline int64_t band_tile(int64_t l, int64_t j) { return tri_index(l / kBT, j / kBT); }

// Equal time blocks of an equidistant grid (eq. (relationAtildeBlock)): the bases of the inner
// nodes 1..nodes-2 are translates of one another, so the node block (kn, in) of two inner nodes
// with 2 <= in <= kn equals (kn - in + 1, 1), and the superdiagonal block (kn, kn + 1) with kn >= 2
// equals (1, 2).  Sets (sk, si) and returns true for such a copy; false for the blocks that are
// integrated (the first two columns, the last row, (1, 2) and (nodes - 2, nodes - 1)).  Every
// source is itself integrated.
__host__ __device__ inline bool equal_block_source(int nodes, int kn, int in, int& sk, int& si)
{
    if (kn < 1 || kn > nodes - 2 || in < 2 || in > nodes - 2 || in > kn + 1) return false;
    if (in <= kn) {
        sk = kn - in + 1;
        si = 1;
        return true;
    }
    if (kn == 1) return false;
    sk = 1;
    si = 2;
    return true;
}

struct BandView {
    const int16_t* ilo;    // first trial index of every (k, l, j <= l), tiled as above
    const int32_t* B;      // B[k nt + t]
    const int64_t* voff;   // voff[k nt + t]
    int32_t M, N;          // N: temporal bases L = nodes (p + 1), the time rows of the band
    int64_t nt;            // tiles per time row
    int32_t nodes, p1;     // time nodes and bases per node
};

__host__ __device__ inline int64_t band_ilo_index(const BandView& b, int k, int64_t l, int64_t j)
{
    return ((int64_t)k * b.nt + band_tile(l, j)) * (kBT * kBT) + (l % kBT) * kBT + j % kBT;
}

// Band width and first value of the (k, tile of (l, j)) block.
__device__ inline int band_width(const BandView& b, int k, int64_t l, int64_t j)
{
    return b.B[(int64_t)k * b.nt + band_tile(l, j)];
}

__device__ inline int64_t band_value_index(const BandView& b, int k, int64_t l, int64_t j, int s, int B)
{
    return b.voff[(int64_t)k * b.nt + band_tile(l, j)] + ((l % kBT) * (int64_t)B + s) * kBT + j % kBT;
}

// Learned preconditioner: graph of the space-time nodes n = k*M + j (CSR mesh neighbours of
// every vertex, step-size features feat[2k] = h_k / hbar, feat[2k+1] = h_{k+1} / hbar) and the
// layout of the flat parameter vector: Win (64 x 3), bin (64), per layer W_l (64 x 256) and b_l
// (64), wout (64).
constexpr int kLpHidden = 64;
struct LpGraph {
    const int32_t* ptr;
    const int32_t* idx;
    const float* feat;
    int32_t M, N;
};
inline int64_t lp_off_win() { return 0; }
inline int64_t lp_off_bin() { return 3 * kLpHidden; }
inline int64_t lp_off_w(int l) { return 4 * kLpHidden + (int64_t)l * (4 * kLpHidden * kLpHidden + kLpHidden); }
inline int64_t lp_off_b(int l) { return lp_off_w(l) + 4 * kLpHidden * kLpHidden; }
inline int64_t lp_off_wout(int layers) { return lp_off_w(layers); }
inline int64_t lp_num_params(int layers) { return lp_off_wout(layers) + kLpHidden; }

}  // namespace tdbem

// ---------------------------------------------------------------------------------------------
// Launchers (defined in the .hip files).
// ---------------------------------------------------------------------------------------------
namespace tdbem {
void launch_table_values(const double* t, int N, int p1, int cut, TimeRule rule, PieceTable pt, const int32_t* pc_f,
                         const int32_t* pc_j, const int32_t* pc_p, int64_t npieces, const int32_t* f_k,
                         const int32_t* f_i, const KernelDesc* desc, const double* ivl, double2* values,
                         hipStream_t s);
void launch_table_coefs(const double2* values, int64_t npieces, double2* coef, hipStream_t s);
void launch_table_eval(TableView tv, int64_t n, const int32_t* k, const int32_t* i, const double* r,
                       double* ps, double* tps, hipStream_t s);

void launch_geometry(const double* xyz, const int32_t* tri, int E, double* geo_P, double* geo_n,
                     double* geo_area, double* geo_curl, double* geo_qp, int32_t* geo_v, hipStream_t s);
void launch_layout(BandView band, const double* xyz, const double* rho, const double* t, int16_t* ilo,
                   int32_t* Bk, hipStream_t s);

// Tile shapes of the regular-pair kernel: variant 0 = 4 x 8 triangles on 256 lanes, 1 = 8 x 8 on
// 512; tiles of a shape from regular_tiles(E, variant).
int tile_variants();
void tile_shape(int variant, int* test, int* trial);
// fxs > 0: deterministic mode, val holds fixed-point integers of scale fxs (FP64 storage only).
void launch_regular(GeomView g, TableView tv, const double* t, BandView band, double* val, float* valf,
                    const double* px, double* py, const int2* tiles, int64_t ntiles, int variant,
                    unsigned long long* counter, hipStream_t s, double fxs = 0.0);
std::vector<int32_t> regular_tiles(int E, int variant);
// One launch over the tiles of several problems (shape 0): tile (a, b) of problem q is stored as
// (a | q << 24, b); probs[q] holds that problem's views.
struct RegularProblem {
    GeomView g;
    TableView tv;
    const double* t;
    BandView band;
    double* val;
    float* valf;
    unsigned long long* counter;
};
void launch_regular_multi(const RegularProblem* probs, const int2* tiles, int64_t ntiles, hipStream_t s);
void launch_singular(GeomView g, TableView tv, const double* t, BandView band, const int32_t* pairs,
                     int64_t npairs, const double* ss_rules, const int32_t* ss_off, const int32_t* ss_cnt,
                     int max_points, double* val, float* valf, const double* px, double* py,
                     unsigned long long* counter, hipStream_t s, double fxs = 0.0);
// Copies every block that equal_block_source maps to another one from that block, in place in
// the band storage (all rows k of a node, every basis pair of the node pair).
void launch_block_copy(BandView band, double* val, float* valf, hipStream_t s);
// Deterministic mode: *out = max |val| over n values (out zeroed by the caller), and the in-place
// conversion of fixed-point integers of scale 2^e back to doubles.
void launch_absmax(const double* val, int64_t n, double* out, hipStream_t s);
void launch_fixed_to_double(double* val, int64_t n, int e, hipStream_t s);
// Allocation-free entry query: static device staging of kNoAllocEntries queries (4 int32 index
// arrays and the float64 results); noalloc_scratch returns its address on `device` (current).
constexpr int64_t kNoAllocEntries = 65536;
constexpr size_t kNoAllocScratchBytes = (size_t)kNoAllocEntries * (4 * sizeof(int32_t) + sizeof(double));
hipError_t noalloc_scratch(int device, void** ptr);

void launch_get_entries(BandView band, const double* val, const float* valf, int64_t n, const int32_t* k,
                        const int32_t* i, const int32_t* j, const int32_t* l, double* out, hipStream_t s);

// Entries of block (k, i) as (row l, column j, value) with an atomic position counter; count only
// when row is null.
void launch_block_coo(BandView band, const double* val, const float* valf, int k, int i, unsigned long long* count,
                      int32_t* row, int32_t* col, double* out, int64_t cap, hipStream_t s);

void launch_rhs(GeomView g, const double* t, int N, int p1, int cut, TimeRule rule, double d0, double d1, double d2,
                double t0, double width, int M, double* gvec, hipStream_t s);
void launch_matvec(BandView band, const double* val, const float* valf, int k0, int k1, int i0, int i1,
                   const double* x, double* y, hipStream_t s);

void launch_dots(const double* V, int nvec, int64_t n, int64_t ld, const double* w, double* partial,
                 double* out, hipStream_t s);
void launch_sub_combination(double* w, const double* V, int nvec, int64_t n, int64_t ld, const double* h,
                            double sign, hipStream_t s);
void launch_scale_copy(double* dst, const double* src, double a, int64_t n, hipStream_t s);
void launch_axpby(double* y, const double* x, double a, double b, int64_t n, hipStream_t s);
int dots_partial_blocks(int64_t n);
void launch_scale_inv_sqrt(double* dst, const double* src, const double* nrm2, int64_t n, hipStream_t s);
void launch_fill(double* x, double v, int64_t n, hipStream_t s);
void launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t s);

void launch_lp_round(int64_t P, const float* p, uint16_t* q, hipStream_t s);
// hstride = 0: inference, H holds two ping-pong slots of N*M*64 floats and U is unused;
// hstride = N*M*64: training, H holds layers+1 slots and U (may not be null) holds layers slots.
void launch_lp_forward(LpGraph g, int layers, const float* params, const uint16_t* wq, const double* v,
                       const double* sc, float* H, int64_t hstride, float* U, double* z, hipStream_t st);
// sc[0] = sqrt(vv[0] / n), sc[1] = 1 / sc[0] (0 when vv = 0): the network's scale on the device.
void launch_lp_scale(const double* vv, int64_t n, double* sc, hipStream_t st);
int lp_partial_blocks(int64_t n);
// Adds the gradient of <dz, z> to grad (layout of the parameter vector).  dH2: 2 N*M*64 floats,
// DU: N*M*64, dX: 4 N*M*64, partial: lp_partial_blocks(N*M) * (64*256 + 64) floats.
void launch_lp_backward(LpGraph g, int layers, const uint16_t* wq, const double* v, const double* sc,
                        const float* H, const float* U, const double* dz, float* dH2, float* DU, float* dX,
                        float* partial, float* grad, hipStream_t st);
void launch_lp_adam(int64_t P, float* p, const float* grad, float* m, float* v2, float lr, int64_t step,
                    float gscale, uint16_t* q, hipStream_t s);
void launch_lp_randn(int64_t n, uint64_t seed, uint64_t stream, double* out, hipStream_t s);
void launch_lp_smooth(LpGraph g, const double* x, double* y, hipStream_t s);
void launch_matvec_transpose(BandView band, const double* val, const float* valf, const double* y, double* x,
                             hipStream_t s);
// u[s*npts + p] = retarded double layer potential at pts[3p..] and times[s] (device arrays);
// phiq: workspace of E*7*N doubles.
void launch_potential(GeomView g, const double* t, int N, int cut, int M, const double* alpha, double* phiq,
                      int64_t npts, const double* pts, int ntimes, const double* times, double* u, hipStream_t s);
// Y[r*ldy + .] = A X[r*ldx + .] for r < nrhs (full operator) with kernel variant `variant`
// (0 .. matvec_multi_variants()-1: right-hand sides per pass and staged trial range).
void launch_matvec_multi(BandView band, const double* val, const float* valf, int nrhs, const double* X, int64_t ldx,
                         double* Y, int64_t ldy, int variant, hipStream_t s);
int matvec_multi_variants();
int matvec_multi_variant_rc(int v);
int matvec_multi_variant_span(int v);
}  // namespace tdbem
