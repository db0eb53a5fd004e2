// Host runtime and C ABI of libtdbem (see include/tdbem.h).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "../../include/tdbem.h"
#include "../../include/tdbem_learned.h"
#include "tdbem_internal.hpp"

using namespace tdbem;

namespace {

// Owned device allocation.
struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
    ~DBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t alloc(size_t b)
    {
        release();
        if (b == 0) b = 8;
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) p = nullptr;
        else bytes = b;
        return e;
    }
    template <typename T> T* as() const { return static_cast<T*>(p); }
};

// Gauss-Legendre nodes/weights on [-1, 1] by Newton's method on the three-term recurrence.
void gauss_legendre(int n, double* x, double* w)
{
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int m = 2; m <= n; ++m) {
                const double p2 = ((2 * m - 1) * z * p1 - (m - 1) * p0) / m;
                p0 = p1;
                p1 = p2;
            }
            const double dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int m = 2; m <= n; ++m) {
            const double p2 = ((2 * m - 1) * z * p1 - (m - 1) * p0) / m;
            p0 = p1;
            p1 = p2;
        }
        const double dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Graded partition of [0, 1] used for every tabulated interval: geometric with ratio 1.6 from
// 0.004 until a piece would exceed 1/8, uniform pieces of width <= 1/8 in the middle, mirrored.
PieceTable make_piece_table()
{
    const double q = 1.6, fmin = 0.02, wmax = 0.2;
    std::vector<double> left{fmin};
    double x = fmin;
    while (x * (q - 1.0) < wmax) {
        x *= q;
        left.push_back(x);
    }
    const double xs = left.back();
    const int nm = (int)std::ceil((1.0 - 2.0 * xs) / wmax - 1e-12);
    std::vector<double> e{0.0};
    for (size_t s = 0; s + 1 < left.size(); ++s) e.push_back(left[s]);
    for (int s = 0; s <= nm; ++s) e.push_back(xs + (1.0 - 2.0 * xs) * s / nm);
    for (size_t s = left.size() - 1; s-- > 0;) e.push_back(1.0 - left[s]);
    e.push_back(1.0);
    PieceTable pt;
    if ((int)e.size() != kPieces + 1) {
        std::fprintf(stderr, "tdbem: piece partition has %zu edges, expected %d\n", e.size(), kPieces + 1);
    }
    for (int s = 0; s <= kPieces; ++s) pt.edge[s] = e[std::min<size_t>(s, e.size() - 1)];
    for (int s = 0; s < kPieces; ++s) pt.inv_width[s] = 1.0 / (pt.edge[s + 1] - pt.edge[s]);
    for (int cidx = 0; cidx < kLutCells; ++cidx) {
        const double x = (double)cidx / kLutCells;
        int p = 0;
        while (p + 1 < kPieces && pt.edge[p + 1] <= x) ++p;
        pt.lut[cidx] = (uint8_t)p;
    }
    return pt;
}

// Sauter-Schwab regions on the reference triangle {0 <= x2 <= x1 <= 1} (Sauter & Schwab,
// Boundary Element Methods, Sec. 5.2): identical (6 regions, J = xi^3 e1^2 e2), common edge A-B
// (5 regions, J = xi^3 e1^2 for the first, xi^3 e1^2 e2 for the others), common vertex A
// (2 regions, J = xi^3 e2).  Rows (x1, x2, y1, y2, weight) for an n^4 Gauss rule per region.
void ss_point(int kind, int reg, double xi, double e1, double e2, double e3, double* o)
{
    double J;
    if (kind == 0) {
        J = xi * xi * xi * e1 * e1 * e2;
        const double A = xi, B1 = xi * (1 - e1 + e1 * e2), C1 = xi * (1 - e1 * e2 * e3), D1 = xi * (1 - e1);
        const double B2 = xi * e1 * (1 - e2 + e2 * e3), C2 = xi * (1 - e1 * e2), D2 = xi * e1 * (1 - e2);
        const double C3 = xi * (1 - e1 * e2 * e3), D3 = xi * e1 * (1 - e2 * e3);
        switch (reg) {
        case 0: o[0] = A; o[1] = B1; o[2] = C1; o[3] = D1; break;
        case 1: o[0] = C1; o[1] = D1; o[2] = A; o[3] = B1; break;
        case 2: o[0] = A; o[1] = B2; o[2] = C2; o[3] = D2; break;
        case 3: o[0] = C2; o[1] = D2; o[2] = A; o[3] = B2; break;
        case 4: o[0] = C3; o[1] = D3; o[2] = A; o[3] = D2; break;
        default: o[0] = A; o[1] = D2; o[2] = C3; o[3] = D3; break;
        }
    } else if (kind == 1) {
        J = xi * xi * xi * e1 * e1 * (reg == 0 ? 1.0 : e2);
        switch (reg) {
        case 0: o[0] = xi; o[1] = xi * e1 * e3; o[2] = xi * (1 - e1 * e2); o[3] = xi * e1 * (1 - e2); break;
        case 1: o[0] = xi; o[1] = xi * e1; o[2] = xi * (1 - e1 * e2 * e3); o[3] = xi * e1 * e2 * (1 - e3); break;
        case 2: o[0] = xi * (1 - e1 * e2); o[1] = xi * e1 * (1 - e2); o[2] = xi; o[3] = xi * e1 * e2 * e3; break;
        case 3: o[0] = xi * (1 - e1 * e2 * e3); o[1] = xi * e1 * e2 * (1 - e3); o[2] = xi; o[3] = xi * e1; break;
        default: o[0] = xi * (1 - e1 * e2 * e3); o[1] = xi * e1 * (1 - e2 * e3); o[2] = xi; o[3] = xi * e1 * e2; break;
        }
    } else {
        J = xi * xi * xi * e2;
        if (reg == 0) { o[0] = xi; o[1] = xi * e1; o[2] = xi * e2; o[3] = xi * e2 * e3; }
        else { o[0] = xi * e2; o[1] = xi * e2 * e3; o[2] = xi; o[3] = xi * e1; }
    }
    o[4] = J;
}

}  // namespace

// every kTileSampleStride-th tile of the regular-pair kernel is timed to pick its tile shape
static constexpr int64_t kTileSampleStride = 32;
// The tables reach ~2e-12 of each kernel's maximum for psi (1e-13 for tilde psi); a tolerance
// below this cannot be met.
static constexpr double kPsiTolFloor = 2e-12;

struct tdbem_ctx {
    int device = 0;
    void* scratch = nullptr;      // device address of the allocation-free staging array
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int ss_order = 4;
    bool deterministic = false;   // fixed-point assembly: bitwise the same matrix on every run
    std::string err;

    int M = 0, E = 0, N = 0, cut = 0;   // N: temporal bases L = nodes (p + 1)
    int nodes = 0, p1 = 1;              // time nodes, bases per node (p + 1)
    std::vector<double> xyz, t;
    std::vector<int32_t> tri;
    double diam = 0.0;
    bool have_mesh = false, have_grid = false;

    // mesh on the device
    DBuf d_xyz, d_tri, d_rho, g_P, g_n, g_area, g_curl, g_qp, g_v, d_pairs, d_rules, d_roff, d_rcnt;
    // tiles of the regular-pair kernel per tile shape, and a strided sample of them for the timing
    // that picks the shape (once per mesh and time grid unless a shape is forced)
    DBuf d_tiles[2], d_tiles_sample[2];
    int64_t ntiles[2] = {0, 0}, ntiles_sample[2] = {0, 0};
    int tile_v = -1;
    bool tile_forced = false;
    uint64_t tile_key = ~0ull;
    double tile_ms[2] = {-1.0, -1.0};
    int64_t npairs = 0, npairs_kind[3] = {0, 0, 0};
    // time grid
    DBuf d_t;
    TimeRule rule{};
    PieceTable pieces{};
    // tables
    DBuf d_desc, d_fid, d_ivl, d_coef, d_fk, d_fi, d_meta, d_cell;
    int64_t nfunc = 0;
    // equal blocks of an equidistant grid: the assembly integrates only the kernels of d_fid_asm
    // (copied blocks marked -1) and copies the others afterwards
    bool equidistant = false, reuse = true;
    DBuf d_fid_asm;
    int64_t blocks_reused = 0;
    // band storage
    DBuf d_ilo, d_B, d_voff, d_val, d_counter;
    std::vector<int32_t> Bk;
    std::vector<int64_t> voff;
    int64_t nvals = 0;
    bool assembled = false;
    int prec = 0;
    // solver workspaces, one per recursion depth
    struct Level {
        DBuf V, Z, w, tmp, partial, h;
        int m = 0;
        int64_t n = 0;
    };
    std::vector<Level> levels;
    // FP32 copy of the FP64 band for the preconditioner's inner products (inner_fp32)
    DBuf d_val32;
    uint64_t val32_assembly = ~0ull;
    // DGMRES deflation space of the outer solve: U (orthonormal columns), A U, T^{-1} = (U^T A U)^{-1}
    // on the host, |lambda_max| estimate
    struct Deflation {
        DBuf U, AU, coef;
        int r = 0, rmax = 0;
        int64_t n = 0;
        std::vector<double> T, Tinv;
        double lam = 1.0;
    } defl;
    int64_t matvecs = 0;
    // learned preconditioner: parameters (float32 master, bfloat16 copy, Adam moments), the graph
    // of the current mesh and grid, workspaces
    struct Learned {
        int layers = 0;
        int64_t P = 0, step = 0, samples = 0;
        DBuf params, wq, grad, m1, m2;
        DBuf ptr, idx, feat;
        uint64_t gver = ~0ull;
        DBuf Hinf, dots;
        int64_t ninf = 0, ndots = 0;
        DBuf H, U, DU, dX, dH2, partial, vb, xb, zb, rb, db;
        int64_t ntrain = 0;
        // z = P(v), w = A z captured as one HIP graph on a private stream, replayed on the
        // context's stream; valid while key (operator, network, buffers) is unchanged
        hipStream_t cap = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t gexec = nullptr;
        std::vector<uint64_t> gkey;
        DBuf gv, gz, gw;
        int64_t gn = 0;
    } lp;
    uint64_t assemblies = 0;      // completed assemblies (part of the graph key)
    uint64_t graph_version = 0;   // changes with the mesh and the time grid
    // multi-vector product: variant chosen by timing on the assembled operator (-1: not yet)
    int mm_variant = -1;
    std::vector<double> mm_ms;    // measured time per right-hand side of every variant

    GeomView geom() const
    {
        GeomView g;
        g.v = g_v.as<int32_t>();
        g.P = g_P.as<double>();
        g.n = g_n.as<double>();
        g.area = g_area.as<double>();
        g.curl = g_curl.as<double>();
        g.qp = g_qp.as<double>();
        g.E = E;
        return g;
    }
    TableView tables() const
    {
        TableView tv;
        tv.desc = d_desc.as<KernelDesc>();
        tv.fid = d_fid.as<int32_t>();
        tv.ivl = d_ivl.as<double>();
        tv.coef = d_coef.as<double2>();
        tv.meta = d_meta.as<double4>();
        tv.cell = d_cell.as<uint16_t>();
        tv.N = N;
        tv.nodes = nodes;
        tv.p1 = p1;
        tv.pt = pieces;
        return tv;
    }
    TableView asm_tables() const
    {
        TableView tv = tables();
        if (blocks_reused > 0) tv.fid = d_fid_asm.as<int32_t>();
        return tv;
    }
    BandView band() const
    {
        BandView b;
        b.ilo = d_ilo.as<int16_t>();
        b.B = d_B.as<int32_t>();
        b.voff = d_voff.as<int64_t>();
        b.M = M;
        b.N = N;
        const int64_t T = ((int64_t)M + kBT - 1) / kBT;
        b.nt = T * (T + 1) / 2;
        b.nodes = nodes;
        b.p1 = p1;
        return b;
    }
    const double* valf64() const { return prec == TDBEM_FP64 ? d_val.as<double>() : nullptr; }
    const float* valf32() const { return prec == TDBEM_FP64 ? nullptr : d_val.as<float>(); }
};

#define FAIL(ctx, code, ...)                                                                  \
    do {                                                                                      \
        char _b[512];                                                                         \
        std::snprintf(_b, sizeof(_b), __VA_ARGS__);                                           \
        (ctx)->err = _b;                                                                      \
        return code;                                                                          \
    } while (0)

#define HIPCHK(ctx, expr)                                                                     \
    do {                                                                                      \
        hipError_t _e = (expr);                                                               \
        if (_e != hipSuccess) FAIL(ctx, TDBEM_EHIP, "%s: %s", #expr, hipGetErrorString(_e));  \
    } while (0)

#define ALLOC(ctx, buf, bytes)                                                                \
    do {                                                                                      \
        if ((buf).alloc(bytes) != hipSuccess) {                                               \
            (void)hipGetLastError();                                                          \
            FAIL(ctx, TDBEM_ENOMEM, "device allocation of %zu bytes failed", (size_t)(bytes)); \
        }                                                                                     \
    } while (0)

static tdbem_status set_device(tdbem_ctx* c)
{
    HIPCHK(c, hipSetDevice(c->device));
    return TDBEM_OK;
}

template <typename T>
static tdbem_status upload(tdbem_ctx* c, DBuf& buf, const T* host, size_t n)
{
    ALLOC(c, buf, sizeof(T) * n);
    if (n) HIPCHK(c, hipMemcpyAsync(buf.p, host, sizeof(T) * n, hipMemcpyHostToDevice, c->stream));
    return TDBEM_OK;
}

#define TRY(expr)                                   \
    do {                                            \
        tdbem_status _s = (expr);                   \
        if (_s != TDBEM_OK) return _s;              \
    } while (0)

// Per-triangle structure of arrays (normals, areas, surface curls, quadrature points).
static tdbem_status run_geometry(tdbem_ctx* c)
{
    launch_geometry(c->d_xyz.as<double>(), c->d_tri.as<int32_t>(), c->E, c->g_P.as<double>(), c->g_n.as<double>(),
                    c->g_area.as<double>(), c->g_curl.as<double>(), c->g_qp.as<double>(), c->g_v.as<int32_t>(),
                    c->stream);
    HIPCHK(c, hipGetLastError());
    return TDBEM_OK;
}

extern "C" {

tdbem_status tdbem_create(tdbem_ctx** out, const tdbem_options* opt)
{
    if (!out) return TDBEM_EINVAL;
    *out = nullptr;
    tdbem_ctx* c = new tdbem_ctx();
    c->device = opt ? opt->device : 0;
    c->ss_order = opt && opt->ss_order > 0 ? opt->ss_order : 4;
    if (c->ss_order > 5) { delete c; return TDBEM_EINVAL; }   // <= 6 * 5^4 points per pair (sorted in LDS)
    if (opt && (opt->deterministic < 0 || opt->deterministic > 1)) { delete c; return TDBEM_EINVAL; }
    if (opt && opt->quad_regular != 0 && opt->quad_regular != 7) { delete c; return TDBEM_EINVAL; }
    if (opt && (opt->psi_tol < 0.0 || (opt->psi_tol > 0.0 && opt->psi_tol < kPsiTolFloor))) { delete c; return TDBEM_EINVAL; }
    c->deterministic = opt && opt->deterministic == 1;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || c->device < 0 || c->device >= ndev) {
        (void)hipGetLastError();
        delete c;
        return TDBEM_EHIP;
    }
    if (hipSetDevice(c->device) != hipSuccess) { delete c; return TDBEM_EHIP; }
    // the allocation-free entry point's staging array: its address on this device, once per device
    if (noalloc_scratch(c->device, &c->scratch) != hipSuccess) {
        (void)hipGetLastError();
        c->scratch = nullptr;   // tdbem_get_entries_noalloc then reports TDBEM_EHIP
    }
    if (opt && opt->stream) {
        c->stream = static_cast<hipStream_t>(opt->stream);
    } else {
        if (hipStreamCreate(&c->stream) != hipSuccess) { delete c; return TDBEM_EHIP; }
        c->own_stream = true;
    }
    double x[kTimeGauss], w[kTimeGauss];
    gauss_legendre(kTimeGauss, x, w);
    for (int q = 0; q < kTimeGauss; ++q) { c->rule.x[q] = x[q]; c->rule.w[q] = w[q]; }
    c->pieces = make_piece_table();
    *out = c;
    return TDBEM_OK;
}

void tdbem_destroy(tdbem_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    c->levels.clear();
    if (c->lp.gexec) (void)hipGraphExecDestroy(c->lp.gexec);
    if (c->lp.graph) (void)hipGraphDestroy(c->lp.graph);
    if (c->lp.cap) (void)hipStreamDestroy(c->lp.cap);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char* tdbem_last_error(const tdbem_ctx* c) { return c ? c->err.c_str() : "null context"; }

tdbem_status tdbem_set_mesh(tdbem_ctx* c, const double* xyz, int64_t M, const int32_t* tri, int64_t E)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (!xyz || !tri || M < 3 || E < 1) FAIL(c, TDBEM_EINVAL, "mesh needs M >= 3 vertices and E >= 1 triangles");
    if (M > 32767 * 2048LL || E > (1LL << 30)) FAIL(c, TDBEM_EINVAL, "mesh too large");
    for (int64_t v = 0; v < 3 * M; ++v)
        if (!std::isfinite(xyz[v])) FAIL(c, TDBEM_EMESH, "vertex coordinate %lld is not finite", (long long)v);
    for (int64_t e = 0; e < E; ++e) {
        const int32_t a = tri[3 * e], b = tri[3 * e + 1], d = tri[3 * e + 2];
        if (a < 0 || b < 0 || d < 0 || a >= M || b >= M || d >= M)
            FAIL(c, TDBEM_EMESH, "triangle %lld has a vertex index out of range", (long long)e);
        if (a == b || b == d || a == d) FAIL(c, TDBEM_EMESH, "triangle %lld repeats a vertex", (long long)e);
        const double* P = xyz + 3 * a;
        const double* Q = xyz + 3 * b;
        const double* R = xyz + 3 * d;
        const double u[3] = {Q[0] - P[0], Q[1] - P[1], Q[2] - P[2]}, w[3] = {R[0] - P[0], R[1] - P[1], R[2] - P[2]};
        const double cr[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
        const double ar = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        const double sc = u[0] * u[0] + u[1] * u[1] + u[2] * u[2] + w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
        if (!(ar > 1e-14 * sc)) FAIL(c, TDBEM_EMESH, "triangle %lld is degenerate", (long long)e);
    }
    TRY(set_device(c));
    c->assembled = false;
    c->have_mesh = false;
    c->M = (int)M;
    c->E = (int)E;
    c->xyz.assign(xyz, xyz + 3 * M);
    c->tri.assign(tri, tri + 3 * E);
    // diameter bound: bounding box diagonal
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < M; ++v)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], xyz[3 * v + d]);
            hi[d] = std::max(hi[d], xyz[3 * v + d]);
        }
    c->diam = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                        (hi[2] - lo[2]) * (hi[2] - lo[2]));
    // patch radius of every vertex: farthest vertex of its triangles
    std::vector<double> rho(M, 0.0);
    std::vector<std::vector<int32_t>> vt(M);
    for (int64_t e = 0; e < E; ++e)
        for (int a = 0; a < 3; ++a) {
            const int32_t v = tri[3 * e + a];
            vt[v].push_back((int32_t)e);
            for (int b = 0; b < 3; ++b) {
                const int32_t u = tri[3 * e + b];
                const double dx = xyz[3 * v] - xyz[3 * u], dy = xyz[3 * v + 1] - xyz[3 * u + 1],
                             dz = xyz[3 * v + 2] - xyz[3 * u + 2];
                rho[v] = std::max(rho[v], std::sqrt(dx * dx + dy * dy + dz * dz));
            }
        }
    // singular pairs {tau <= sigma} sharing at least one vertex, grouped by kind
    std::vector<int32_t> pk[3];
    for (int64_t tau = 0; tau < E; ++tau) {
        std::vector<int32_t> cand;
        for (int a = 0; a < 3; ++a)
            for (int32_t s : vt[tri[3 * tau + a]])
                if (s >= tau) cand.push_back(s);
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        for (int32_t sig : cand) {
            int sa[3], sb[3], ns = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    if (tri[3 * tau + a] == tri[3 * sig + b]) { sa[ns] = a; sb[ns] = b; ++ns; }
            int kind, px[3], py[3];
            if (ns == 3) {
                kind = 0;
                for (int a = 0; a < 3; ++a) px[a] = py[a] = a;
            } else if (ns == 2) {
                kind = 1;
                int a0 = sa[0], a1 = sa[1], b0 = sb[0], b1 = sb[1];
                if (tri[3 * tau + a0] > tri[3 * tau + a1]) { std::swap(a0, a1); std::swap(b0, b1); }
                px[0] = a0; px[1] = a1; px[2] = 3 - a0 - a1;
                py[0] = b0; py[1] = b1; py[2] = 3 - b0 - b1;
            } else {
                kind = 2;
                for (int a = 0; a < 3; ++a) { px[a] = (sa[0] + a) % 3; py[a] = (sb[0] + a) % 3; }
            }
            const int32_t row[9] = {(int32_t)tau, sig, kind, px[0], px[1], px[2], py[0], py[1], py[2]};
            pk[kind].insert(pk[kind].end(), row, row + 9);
        }
    }
    std::vector<int32_t> pairs;
    for (int kd = 0; kd < 3; ++kd) {
        c->npairs_kind[kd] = (int64_t)pk[kd].size() / 9;
        pairs.insert(pairs.end(), pk[kd].begin(), pk[kd].end());
    }
    c->npairs = (int64_t)pairs.size() / 9;
    // Sauter-Schwab rules
    const int n = c->ss_order;
    std::vector<double> gx(n), gw(n);
    gauss_legendre(n, gx.data(), gw.data());
    for (int q = 0; q < n; ++q) { gx[q] = 0.5 * (gx[q] + 1.0); gw[q] *= 0.5; }
    std::vector<double> rules;
    int32_t roff[3], rcnt[3];
    const int nreg[3] = {6, 5, 2};
    for (int kd = 0; kd < 3; ++kd) {
        roff[kd] = (int32_t)(rules.size() / 5);
        for (int reg = 0; reg < nreg[kd]; ++reg)
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b)
                    for (int d = 0; d < n; ++d)
                        for (int f = 0; f < n; ++f) {
                            double o[5];
                            ss_point(kd, reg, gx[a], gx[b], gx[d], gx[f], o);
                            o[4] *= gw[a] * gw[b] * gw[d] * gw[f];
                            rules.insert(rules.end(), o, o + 5);
                        }
        rcnt[kd] = (int32_t)(rules.size() / 5) - roff[kd];
    }
    TRY(upload(c, c->d_xyz, c->xyz.data(), c->xyz.size()));
    TRY(upload(c, c->d_tri, c->tri.data(), c->tri.size()));
    TRY(upload(c, c->d_rho, rho.data(), rho.size()));
    TRY(upload(c, c->d_pairs, pairs.data(), pairs.size()));
    for (int v = 0; v < tile_variants(); ++v) {
        const std::vector<int32_t> tiles = regular_tiles((int)E, v);
        c->ntiles[v] = (int64_t)tiles.size() / 2;
        TRY(upload(c, c->d_tiles[v], tiles.data(), tiles.size()));
        std::vector<int32_t> sample;
        for (int64_t q = 0; q < c->ntiles[v]; q += kTileSampleStride) {
            sample.push_back(tiles[2 * q]);
            sample.push_back(tiles[2 * q + 1]);
        }
        c->ntiles_sample[v] = (int64_t)sample.size() / 2;
        TRY(upload(c, c->d_tiles_sample[v], sample.data(), std::max<size_t>(sample.size(), 2)));
    }
    if (!c->tile_forced) c->tile_v = -1;
    TRY(upload(c, c->d_rules, rules.data(), rules.size()));
    TRY(upload(c, c->d_roff, roff, 3));
    TRY(upload(c, c->d_rcnt, rcnt, 3));
    ALLOC(c, c->g_P, sizeof(double) * 9 * E);
    ALLOC(c, c->g_n, sizeof(double) * 3 * E);
    ALLOC(c, c->g_area, sizeof(double) * E);
    ALLOC(c, c->g_curl, sizeof(double) * 9 * E);
    ALLOC(c, c->g_qp, sizeof(double) * 21 * E);
    ALLOC(c, c->g_v, sizeof(int32_t) * 3 * E);
    TRY(run_geometry(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->have_mesh = true;
    ++c->graph_version;
    return TDBEM_OK;
}

tdbem_status tdbem_set_time_grid(tdbem_ctx* c, const double* t, int32_t N, tdbem_cutoff cutoff, int32_t p)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (!t) FAIL(c, TDBEM_EINVAL, "null time grid");
    if (p < 0 || p > 4) FAIL(c, TDBEM_EINVAL, "temporal order p = %d outside 0..4", p);
    if (cutoff != TDBEM_CUTOFF_BUMP && cutoff != TDBEM_CUTOFF_ERF) FAIL(c, TDBEM_EINVAL, "unknown cutoff %d", (int)cutoff);
    if (N < 2 || N > 4096) FAIL(c, TDBEM_EGRID, "need 2 <= N <= 4096 time nodes, got %d", N);
    if ((int64_t)N * (p + 1) > 8192) FAIL(c, TDBEM_EINVAL, "N (p + 1) = %d temporal bases exceed 8192", N * (p + 1));
    if (t[0] != 0.0) FAIL(c, TDBEM_EGRID, "t_0 must be 0");
    for (int s = 0; s < N; ++s)
        if (!std::isfinite(t[s])) FAIL(c, TDBEM_EGRID, "t_%d is not finite", s);
    for (int s = 1; s < N; ++s)
        if (!(t[s] > t[s - 1])) FAIL(c, TDBEM_EGRID, "time grid not strictly increasing at %d", s);
    TRY(set_device(c));
    c->assembled = false;
    c->have_grid = false;
    c->nodes = N;
    c->p1 = p + 1;
    c->N = N * (p + 1);
    c->cut = (int)cutoff;
    c->t.assign(t, t + N);
    // t_n = n T / (N - 1) up to rounding: the inner nodes' bases are translates of one another
    double dev = 0.0;
    for (int s = 0; s < N; ++s) dev = std::max(dev, std::fabs(t[s] - s * (t[N - 1] / (N - 1))));
    c->equidistant = dev <= 1e-12 * t[N - 1];
    TRY(upload(c, c->d_t, c->t.data(), c->t.size()));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->have_grid = true;
    ++c->graph_version;
    return TDBEM_OK;
}

// ---------------------------------------------------------------------------------------------
// Assembly
// ---------------------------------------------------------------------------------------------
static tdbem_status build_tables(tdbem_ctx* c)
{
    const int N = c->N, nodes = c->nodes, p1 = c->p1;     // N: temporal bases
    const double* t = c->t.data();
    const double rcap = c->diam * (1.0 + 1e-9) + 1e-12;
    std::vector<KernelDesc> desc;
    std::vector<int32_t> fid((size_t)N * N, -1), fk, fi;
    std::vector<double> ivl;
    std::vector<double4> meta;
    std::vector<uint16_t> cell;
    std::vector<int32_t> pc_f, pc_j, pc_p;
    int64_t coef_off = 0;
    for (int k = 0; k < N; ++k)
        for (int i = 0; i < N; ++i) {
            double lo, hi;
            kernel_support(t, nodes, p1, k, i, lo, hi);
            if (!(hi > lo) || !(lo < rcap)) continue;
            // node differences t_c - t_a inside the support split it into analytic intervals
            std::vector<double> bp{lo};
            const int kn = k / p1, in = i / p1;
            for (int cc = kn - 1; cc <= kn + 1; ++cc)
                for (int a = in - 1; a <= in + 1; ++a) {
                    if (cc < 0 || cc >= nodes || a < 0 || a >= nodes) continue;
                    const double d = t[cc] - t[a];
                    if (d > lo && d < hi) bp.push_back(d);
                }
            std::sort(bp.begin(), bp.end());
            const double tol = 1e-13 * (1.0 + t[nodes - 1]);
            std::vector<double> uniq;
            for (double b : bp)
                if (uniq.empty() || b - uniq.back() > tol) uniq.push_back(b);
            const double end = std::min(hi, rcap);
            while (uniq.size() > 1 && uniq.back() >= end - tol) uniq.pop_back();
            KernelDesc kd;
            kd.lo = lo;
            kd.hi = hi;
            kd.nint = (int32_t)uniq.size();
            kd.bp_off = (int32_t)ivl.size();
            kd.coef_off = coef_off;
            kd.cell_scale = kCells / (end - lo);
            kd.cell_off = (int32_t)cell.size();
            kd.pad = 0;
            const size_t m0 = meta.size();
            for (size_t s = 0; s < uniq.size(); ++s) {
                const double a = uniq[s], b = s + 1 < uniq.size() ? uniq[s + 1] : end, len = b - a;
                ivl.push_back(a);
                ivl.push_back(1.0 / len);
                for (int p = 0; p < kPieces; ++p) {
                    const double e0 = c->pieces.edge[p], e1 = c->pieces.edge[p + 1];
                    const bool last_interval = s + 1 == uniq.size();
                    double4 r;
                    r.x = p + 1 < kPieces ? a + e1 * len : (last_interval ? INFINITY : uniq[s + 1]);
                    r.y = a + 0.5 * (e0 + e1) * len;
                    r.z = 2.0 / ((e1 - e0) * len);
                    r.w = ((s == 0 && p < kPieces / 2) || (last_interval && p >= kPieces / 2)) ? 1.0 : 0.0;
                    meta.push_back(r);
                }
            }
            for (int cc = 0; cc < kCells; ++cc) {
                const double rc = lo + cc / kd.cell_scale;
                size_t g = m0;
                while (g + 1 < meta.size() && meta[g].x <= rc) ++g;
                cell.push_back((uint16_t)(g - m0));
            }
            const int f = (int)desc.size();
            fid[(size_t)k * N + i] = f;
            desc.push_back(kd);
            fk.push_back(k);
            fi.push_back(i);
            for (int j = 0; j < kd.nint; ++j)
                for (int p = 0; p < kPieces; ++p) {
                    pc_f.push_back(f);
                    pc_j.push_back(j);
                    pc_p.push_back(p);
                }
            coef_off += (int64_t)kd.nint * kPieces * kNc;
        }
    c->nfunc = (int64_t)desc.size();
    const int64_t npieces = (int64_t)pc_f.size();
    TRY(upload(c, c->d_desc, desc.data(), desc.size()));
    TRY(upload(c, c->d_fid, fid.data(), fid.size()));
    c->blocks_reused = 0;
    if (c->reuse && c->equidistant) {
        std::vector<int32_t> fa(fid);
        for (int k = 0; k < N; ++k)
            for (int i = 0; i < N; ++i) {
                int sk, si;
                if (fa[(size_t)k * N + i] >= 0 && equal_block_source(nodes, k / p1, i / p1, sk, si)) {
                    fa[(size_t)k * N + i] = -1;
                    ++c->blocks_reused;
                }
            }
        if (c->blocks_reused > 0) TRY(upload(c, c->d_fid_asm, fa.data(), fa.size()));
    }
    // padding: the regular kernel reads all kMaxIntervals starts of a kernel at once
    ivl.insert(ivl.end(), 2 * kMaxIntervals, 0.0);
    TRY(upload(c, c->d_ivl, ivl.data(), ivl.size()));
    TRY(upload(c, c->d_meta, meta.data(), meta.size()));
    TRY(upload(c, c->d_cell, cell.data(), cell.size()));
    TRY(upload(c, c->d_fk, fk.data(), fk.size()));
    TRY(upload(c, c->d_fi, fi.data(), fi.size()));
    DBuf d_pcf, d_pcj, d_pcp, d_values;
    TRY(upload(c, d_pcf, pc_f.data(), pc_f.size()));
    TRY(upload(c, d_pcj, pc_j.data(), pc_j.size()));
    TRY(upload(c, d_pcp, pc_p.data(), pc_p.size()));
    ALLOC(c, d_values, sizeof(double2) * (size_t)npieces * kNc);
    ALLOC(c, c->d_coef, sizeof(double2) * (size_t)npieces * kNc);
    launch_table_values(c->d_t.as<double>(), nodes, p1, c->cut, c->rule, c->pieces, d_pcf.as<int32_t>(), d_pcj.as<int32_t>(),
                        d_pcp.as<int32_t>(), npieces, c->d_fk.as<int32_t>(), c->d_fi.as<int32_t>(),
                        c->d_desc.as<KernelDesc>(), c->d_ivl.as<double>(), d_values.as<double2>(), c->stream);
    HIPCHK(c, hipGetLastError());
    launch_table_coefs(d_values.as<double2>(), npieces, c->d_coef.as<double2>(), c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));   // the temporaries are released on return
    return TDBEM_OK;
}

static tdbem_status build_layout(tdbem_ctx* c, int prec)
{
    const int64_t M = c->M, N = c->N;
    const int64_t T = (M + kBT - 1) / kBT, nt = T * (T + 1) / 2;
    const int64_t per_k = nt * kBT * kBT;     // tile slots of one time row
    ALLOC(c, c->d_ilo, sizeof(int16_t) * (size_t)(N * per_k));
    HIPCHK(c, hipMemsetAsync(c->d_ilo.p, 0, sizeof(int16_t) * (size_t)(N * per_k), c->stream));
    ALLOC(c, c->d_B, sizeof(int32_t) * (size_t)(N * nt));
    launch_layout(c->band(), c->d_xyz.as<double>(), c->d_rho.as<double>(), c->d_t.as<double>(), c->d_ilo.as<int16_t>(),
                  c->d_B.as<int32_t>(), c->stream);
    HIPCHK(c, hipGetLastError());
    c->Bk.assign((size_t)(N * nt), 0);
    HIPCHK(c, hipMemcpyAsync(c->Bk.data(), c->d_B.p, sizeof(int32_t) * (size_t)(N * nt), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->voff.assign((size_t)(N * nt), 0);
    int64_t tot = 0;
    for (int64_t q = 0; q < N * nt; ++q) {
        c->voff[q] = tot;
        tot += (int64_t)c->Bk[q] * kBT * kBT;
    }
    c->nvals = tot;
    TRY(upload(c, c->d_voff, c->voff.data(), c->voff.size()));
    const size_t esz = prec == TDBEM_FP64 ? sizeof(double) : sizeof(float);
    c->d_val.release();                    // a previous assembly's values count as free memory
    size_t freeb = 0, totb = 0;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemGetInfo(&freeb, &totb));
    const size_t need = esz * (size_t)std::max<int64_t>(tot, 1);
    if (need + (size_t)(1ull << 30) > freeb) {
        FAIL(c, TDBEM_ENOMEM, "band storage needs %.2f GB, %.2f GB free on the device", need / 1e9, freeb / 1e9);
    }
    ALLOC(c, c->d_val, need);
    HIPCHK(c, hipMemsetAsync(c->d_val.p, 0, need, c->stream));
    return TDBEM_OK;
}

// Tile shape of the regular-pair kernel: each shape runs on its strided sample of tiles (after a
// short warm-up launch), timed with events; the faster per tile of the full list is kept for this
// mesh and time grid.  The sample writes into the zeroed storage, which is zeroed again.

static tdbem_status tune_tiles(tdbem_ctx* c, double* v64, float* v32)
{
    if (c->tile_forced || (c->tile_v >= 0 && c->tile_key == c->graph_version)) return TDBEM_OK;
    DBuf scratch_count;
    ALLOC(c, scratch_count, sizeof(unsigned long long));
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    struct Guard {
        hipEvent_t a, b;
        ~Guard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
    } guard{e0, e1};
    int best = 0;
    for (int v = 0; v < tile_variants(); ++v) {
        const int2* smp = c->d_tiles_sample[v].as<int2>();
        launch_regular(c->geom(), c->asm_tables(), c->d_t.as<double>(), c->band(), v64, v32, nullptr, nullptr, smp,
                       std::min<int64_t>(c->ntiles_sample[v], 64), v, scratch_count.as<unsigned long long>(),
                       c->stream);
        HIPCHK(c, hipEventRecord(e0, c->stream));
        launch_regular(c->geom(), c->asm_tables(), c->d_t.as<double>(), c->band(), v64, v32, nullptr, nullptr, smp,
                       c->ntiles_sample[v], v, scratch_count.as<unsigned long long>(), c->stream);
        HIPCHK(c, hipEventRecord(e1, c->stream));
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipEventSynchronize(e1));
        float ms;
        HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
        c->tile_ms[v] = c->ntiles_sample[v] > 0 ? ms * (double)c->ntiles[v] / (double)c->ntiles_sample[v] : 0.0;
        if (c->tile_ms[v] < c->tile_ms[best]) best = v;
    }
    HIPCHK(c, hipMemsetAsync(c->d_val.p, 0, c->d_val.bytes, c->stream));
    c->tile_v = best;
    c->tile_key = c->graph_version;
    return TDBEM_OK;
}

// One assembly in parts, so that a group of problems can share the regular-pair launch:
// asm_begin (geometry, tables, layout, shape timing), the regular-pair launch on the context's
// stream followed by ev[3], asm_tail (singular pairs, copies of equal blocks) and asm_end (wait,
// counts, report).
// (The singular pairs beside the regular ones on a second stream gained nothing: the regular
// kernel's two waves per SIMD hold all of its VGPRs, so the singular waves only ran in its gaps
// and lengthened it by their own time.)
struct AsmRun {
    hipEvent_t ev[6] = {};
    double* v64 = nullptr;
    float* v32 = nullptr;
    AsmRun() = default;
    AsmRun(const AsmRun&) = delete;
    AsmRun& operator=(const AsmRun&) = delete;
    ~AsmRun()
    {
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

static tdbem_status asm_begin(tdbem_ctx* c, tdbem_precision prec, AsmRun& R, bool tune)
{
    c->err.clear();
    if (!c->have_mesh || !c->have_grid) FAIL(c, TDBEM_ESTATE, "set the mesh and the time grid before assembling");
    if (prec != TDBEM_FP64 && prec != TDBEM_MIXED) FAIL(c, TDBEM_EINVAL, "unknown precision %d", (int)prec);
    TRY(set_device(c));
    c->assembled = false;
    c->prec = (int)prec;
    for (auto& e : R.ev) HIPCHK(c, hipEventCreate(&e));
    HIPCHK(c, hipEventRecord(R.ev[0], c->stream));
    TRY(run_geometry(c));
    TRY(build_tables(c));
    HIPCHK(c, hipEventRecord(R.ev[1], c->stream));
    TRY(build_layout(c, (int)prec));
    ALLOC(c, c->d_counter, sizeof(unsigned long long) * 2);
    HIPCHK(c, hipMemsetAsync(c->d_counter.p, 0, sizeof(unsigned long long) * 2, c->stream));
    R.v64 = prec == TDBEM_FP64 ? c->d_val.as<double>() : nullptr;
    R.v32 = prec == TDBEM_FP64 ? nullptr : c->d_val.as<float>();
    if (tune) TRY(tune_tiles(c, R.v64, R.v32));
    HIPCHK(c, hipEventRecord(R.ev[2], c->stream));
    return TDBEM_OK;
}

// Deterministic mode, first pass: the ordinary assembly gives the largest entry, from which the
// fixed-point scale 2^e (every final sum below 2^61) follows; the storage and the counters are
// then cleared for the fixed-point pass.
static tdbem_status fixed_scale(tdbem_ctx* c, AsmRun& R, double* fxs, int* fxe)
{
    launch_regular(c->geom(), c->asm_tables(), c->d_t.as<double>(), c->band(), R.v64, nullptr, nullptr, nullptr,
                   c->d_tiles[c->tile_v].as<int2>(), c->ntiles[c->tile_v], c->tile_v,
                   c->d_counter.as<unsigned long long>(), c->stream);
    const int n4 = c->ss_order * c->ss_order * c->ss_order * c->ss_order;
    launch_singular(c->geom(), c->asm_tables(), c->d_t.as<double>(), c->band(), c->d_pairs.as<int32_t>(), c->npairs,
                    c->d_rules.as<double>(), c->d_roff.as<int32_t>(), c->d_rcnt.as<int32_t>(), 6 * n4, R.v64, nullptr,
                    nullptr, nullptr, c->d_counter.as<unsigned long long>() + 1, c->stream);
    HIPCHK(c, hipGetLastError());
    DBuf d_max;
    ALLOC(c, d_max, sizeof(double));
    HIPCHK(c, hipMemsetAsync(d_max.p, 0, sizeof(double), c->stream));
    launch_absmax(R.v64, c->nvals, d_max.as<double>(), c->stream);
    HIPCHK(c, hipGetLastError());
    double mx = 0.0;
    HIPCHK(c, hipMemcpyAsync(&mx, d_max.p, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *fxe = mx > 0.0 ? std::min(60 - std::ilogb(mx), 1000) : 0;
    *fxs = std::ldexp(1.0, *fxe);
    HIPCHK(c, hipMemsetAsync(c->d_val.p, 0, c->d_val.bytes, c->stream));
    HIPCHK(c, hipMemsetAsync(c->d_counter.p, 0, sizeof(unsigned long long) * 2, c->stream));
    return TDBEM_OK;
}

static tdbem_status asm_tail(tdbem_ctx* c, AsmRun& R, double fxs = 0.0, int fxe = 0)
{
    const int n4 = c->ss_order * c->ss_order * c->ss_order * c->ss_order;
    launch_singular(c->geom(), c->asm_tables(), c->d_t.as<double>(), c->band(), c->d_pairs.as<int32_t>(), c->npairs,
                    c->d_rules.as<double>(), c->d_roff.as<int32_t>(), c->d_rcnt.as<int32_t>(), 6 * n4, R.v64, R.v32,
                    nullptr, nullptr, c->d_counter.as<unsigned long long>() + 1, c->stream, fxs);
    HIPCHK(c, hipGetLastError());
    if (fxs > 0.0) {
        launch_fixed_to_double(R.v64, c->nvals, fxe, c->stream);
        HIPCHK(c, hipGetLastError());
    }
    HIPCHK(c, hipEventRecord(R.ev[4], c->stream));
    if (c->blocks_reused > 0) {
        launch_block_copy(c->band(), R.v64, R.v32, c->stream);
        HIPCHK(c, hipGetLastError());
    }
    HIPCHK(c, hipEventRecord(R.ev[5], c->stream));
    return TDBEM_OK;
}

static tdbem_status asm_end(tdbem_ctx* c, AsmRun& R, tdbem_assembly_report* rep)
{
    HIPCHK(c, hipStreamSynchronize(c->stream));
    unsigned long long counts[2];
    HIPCHK(c, hipMemcpy(counts, c->d_counter.p, sizeof(counts), hipMemcpyDeviceToHost));
    c->assembled = true;
    ++c->assemblies;
    c->mm_variant = -1;
    if (rep) {
        hipEvent_t* ev = R.ev;
        float ms[5], tot;
        for (int s = 0; s < 5; ++s) HIPCHK(c, hipEventElapsedTime(&ms[s], ev[s], ev[s + 1]));
        HIPCHK(c, hipEventElapsedTime(&tot, ev[0], ev[5]));
        rep->quad_evals = (int64_t)(counts[0] + counts[1]);
        rep->quad_evals_regular = (int64_t)counts[0];
        const int64_t E = c->E;
        rep->pairs_coincident = c->npairs_kind[0];
        rep->pairs_edge = c->npairs_kind[1];
        rep->pairs_vertex = c->npairs_kind[2];
        rep->pairs_regular = E * (E - 1) / 2 - c->npairs_kind[1] - c->npairs_kind[2];
        rep->table_functions = c->nfunc;
        rep->bytes_matrix = (int64_t)c->d_val.bytes;
        rep->ms_tables = ms[0];
        rep->ms_layout = ms[1];
        rep->ms_regular = ms[2];
        rep->ms_singular = ms[3];
        rep->ms_reuse = ms[4];
        rep->blocks_reused = c->blocks_reused;
        rep->ms_total = tot;
    }
    return TDBEM_OK;
}

tdbem_status tdbem_assemble(tdbem_ctx* c, tdbem_precision prec, tdbem_assembly_report* rep)
{
    if (!c) return TDBEM_EINVAL;
    if (c->deterministic && prec != TDBEM_FP64) {
        c->err.clear();
        FAIL(c, TDBEM_EINVAL, "the deterministic assembly stores FP64 values (precision TDBEM_FP64)");
    }
    AsmRun R;
    TRY(asm_begin(c, prec, R, true));
    double fxs = 0.0;
    int fxe = 0;
    if (c->deterministic) TRY(fixed_scale(c, R, &fxs, &fxe));
    // both modes evaluate every quadrature point in FP64; the mixed mode rounds the sums into FP32
    // storage
    launch_regular(c->geom(), c->asm_tables(), c->d_t.as<double>(), c->band(), R.v64, R.v32, nullptr, nullptr,
                   c->d_tiles[c->tile_v].as<int2>(), c->ntiles[c->tile_v], c->tile_v,
                   c->d_counter.as<unsigned long long>(), c->stream, fxs);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipEventRecord(R.ev[3], c->stream));
    TRY(asm_tail(c, R, fxs, fxe));
    return asm_end(c, R, rep);
}

tdbem_status tdbem_assemble_group(tdbem_ctx* const* ctxs, int32_t n, tdbem_precision prec,
                                  tdbem_assembly_report* reps)
{
    if (!ctxs || n < 1 || n > 256) return TDBEM_EINVAL;
    for (int a = 0; a < n; ++a) {
        if (!ctxs[a]) return TDBEM_EINVAL;
        for (int b = 0; b < a; ++b)
            if (ctxs[a] == ctxs[b]) FAIL(ctxs[a], TDBEM_EINVAL, "a context appears twice in the group");
        if (ctxs[a]->device != ctxs[0]->device)
            FAIL(ctxs[a], TDBEM_EINVAL, "the contexts of a group must share one device");
        if (ctxs[a]->have_mesh && ctxs[a]->E >= (1 << 24))
            FAIL(ctxs[a], TDBEM_EINVAL, "a group problem may have at most 2^24 - 1 triangles");
    }
    bool any_det = false;
    for (int a = 0; a < n; ++a) any_det = any_det || ctxs[a]->deterministic;
    if (any_det) {
        // the deterministic mode's two passes: each context on its own, side by side
        std::vector<tdbem_status> st(n, TDBEM_OK);
        std::vector<std::thread> th;
        th.reserve(n);
        for (int a = 0; a < n; ++a)
            th.emplace_back([&, a]() { st[a] = tdbem_assemble(ctxs[a], prec, reps ? reps + a : nullptr); });
        for (auto& t : th) t.join();
        for (int a = 0; a < n; ++a)
            if (st[a] != TDBEM_OK) return st[a];
        return TDBEM_OK;
    }
    // every problem's tables and layout on its own stream (one host thread each, so the host work
    // overlaps and the small launches share the device) ...
    std::vector<AsmRun> runs(n);
    std::vector<tdbem_status> st(n, TDBEM_OK);
    {
        std::vector<std::thread> th;
        th.reserve(n);
        for (int a = 0; a < n; ++a) th.emplace_back([&, a]() { st[a] = asm_begin(ctxs[a], prec, runs[a], false); });
        for (auto& t : th) t.join();
    }
    for (int a = 0; a < n; ++a)
        if (st[a] != TDBEM_OK) {
            for (int b = 0; b < n; ++b) (void)hipStreamSynchronize(ctxs[b]->stream);
            return st[a];
        }
    // ... then the regular pairs of all of them in one launch on the first context's stream (each
    // tile tagged with its problem), and each problem's singular pairs and copies on its own stream
    // after it
    tdbem_ctx* c0 = ctxs[0];
    std::vector<int> order(n);
    for (int a = 0; a < n; ++a) order[a] = a;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return ctxs[x]->E > ctxs[y]->E; });
    std::vector<RegularProblem> probs(n);
    std::vector<std::vector<int32_t>> tq(n);
    for (int q = 0; q < n; ++q) {
        tdbem_ctx* c = ctxs[order[q]];
        probs[q] = RegularProblem{c->geom(), c->asm_tables(), c->d_t.as<double>(), c->band(), runs[order[q]].v64,
                                  runs[order[q]].v32, c->d_counter.as<unsigned long long>()};
        tq[q] = regular_tiles(c->E, 0);
        HIPCHK(c0, hipStreamWaitEvent(c0->stream, runs[order[q]].ev[2], 0));
    }
    // the kernel gives XCD x the x-th eighth of the list: every eighth gets the same share of every
    // problem, larger problems first (tiles of different problems cost differently), padded to
    // equal length with tiles past the end of problem 0, which leave at once
    int64_t per = 0;
    for (int x = 0; x < 8; ++x) {
        int64_t cx = 0;
        for (int q = 0; q < n; ++q) {
            const int64_t nq = (int64_t)tq[q].size() / 2;
            cx += nq * (x + 1) / 8 - nq * x / 8;
        }
        per = std::max(per, cx);
    }
    std::vector<int32_t> tiles;
    tiles.reserve((size_t)(16 * per));
    for (int x = 0; x < 8; ++x) {
        for (int q = 0; q < n; ++q) {
            const int64_t nq = (int64_t)tq[q].size() / 2, u0 = nq * x / 8, u1 = nq * (x + 1) / 8;
            for (int64_t u = u0; u < u1; ++u) {
                tiles.push_back((int32_t)((uint32_t)tq[q][2 * u] | ((uint32_t)q << 24)));
                tiles.push_back(tq[q][2 * u + 1]);
            }
        }
        while ((int64_t)tiles.size() < 2 * per * (x + 1)) {
            tiles.push_back(0xFFFFFF);
            tiles.push_back(0);
        }
    }
    DBuf d_probs, d_tiles;
    TRY(set_device(c0));
    if (per > 0) {
        TRY(upload(c0, d_probs, probs.data(), probs.size()));
        TRY(upload(c0, d_tiles, tiles.data(), tiles.size()));
        launch_regular_multi(d_probs.as<RegularProblem>(), d_tiles.as<int2>(), (int64_t)tiles.size() / 2,
                             c0->stream);
        HIPCHK(c0, hipGetLastError());
    }
    hipEvent_t done;
    HIPCHK(c0, hipEventCreate(&done));
    struct Guard {
        hipEvent_t e;
        ~Guard() { (void)hipEventDestroy(e); }
    } guard{done};
    HIPCHK(c0, hipEventRecord(done, c0->stream));
    tdbem_status first = TDBEM_OK;
    for (int a = 0; a < n; ++a) {
        tdbem_ctx* c = ctxs[a];
        TRY(set_device(c));
        HIPCHK(c, hipStreamWaitEvent(c->stream, done, 0));
        HIPCHK(c, hipEventRecord(runs[a].ev[3], c->stream));
        const tdbem_status r = asm_tail(c, runs[a]);
        if (first == TDBEM_OK) first = r;
    }
    for (int a = 0; a < n; ++a) {
        const tdbem_status r = asm_end(ctxs[a], runs[a], reps ? reps + a : nullptr);
        if (first == TDBEM_OK) first = r;
    }
    // the device buffers of the launch are released only when every stream has passed it
    HIPCHK(c0, hipEventSynchronize(done));
    return first;
}

tdbem_status tdbem_matvec_free(tdbem_ctx* c, const double* x, double* y, tdbem_assembly_report* rep)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (!x || !y) FAIL(c, TDBEM_EINVAL, "null vector");
    if (!c->have_mesh || !c->have_grid) FAIL(c, TDBEM_ESTATE, "set the mesh and the time grid before the product");
    TRY(set_device(c));
    hipEvent_t ev[5];
    for (auto& e : ev) HIPCHK(c, hipEventCreate(&e));
    struct EvGuard {
        hipEvent_t* e;
        ~EvGuard() { for (int s = 0; s < 5; ++s) (void)hipEventDestroy(e[s]); }
    } guard{ev};
    HIPCHK(c, hipEventRecord(ev[0], c->stream));
    TRY(run_geometry(c));
    TRY(build_tables(c));
    HIPCHK(c, hipEventRecord(ev[1], c->stream));
    launch_fill(y, 0.0, (int64_t)c->N * c->M, c->stream);
    DBuf counter;
    ALLOC(c, counter, sizeof(unsigned long long) * 2);
    HIPCHK(c, hipMemsetAsync(counter.p, 0, sizeof(unsigned long long) * 2, c->stream));
    HIPCHK(c, hipEventRecord(ev[2], c->stream));
    unsigned long long* cnt = counter.as<unsigned long long>();
    const int tv = c->tile_v >= 0 ? c->tile_v : 0;
    launch_regular(c->geom(), c->tables(), c->d_t.as<double>(), c->band(), nullptr, nullptr, x, y,
                   c->d_tiles[tv].as<int2>(), c->ntiles[tv], tv, cnt, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipEventRecord(ev[3], c->stream));
    const int n4 = c->ss_order * c->ss_order * c->ss_order * c->ss_order;
    launch_singular(c->geom(), c->tables(), c->d_t.as<double>(), c->band(), c->d_pairs.as<int32_t>(), c->npairs,
                    c->d_rules.as<double>(), c->d_roff.as<int32_t>(), c->d_rcnt.as<int32_t>(), 6 * n4, nullptr,
                    nullptr, x, y, cnt + 1, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipEventRecord(ev[4], c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    unsigned long long counts[2];
    HIPCHK(c, hipMemcpy(counts, counter.p, sizeof(counts), hipMemcpyDeviceToHost));
    if (rep) {
        float ms[4];
        for (int s = 0; s < 4; ++s) HIPCHK(c, hipEventElapsedTime(&ms[s], ev[s], ev[s + 1]));
        const int64_t E = c->E;
        rep->quad_evals = (int64_t)(counts[0] + counts[1]);
        rep->quad_evals_regular = (int64_t)counts[0];
        rep->pairs_coincident = c->npairs_kind[0];
        rep->pairs_edge = c->npairs_kind[1];
        rep->pairs_vertex = c->npairs_kind[2];
        rep->pairs_regular = E * (E - 1) / 2 - c->npairs_kind[1] - c->npairs_kind[2];
        rep->table_functions = c->nfunc;
        rep->bytes_matrix = 0;
        rep->ms_tables = ms[0];
        rep->ms_layout = ms[1];
        rep->ms_regular = ms[2];
        rep->ms_singular = ms[3];
        rep->ms_total = ms[0] + ms[1] + ms[2] + ms[3];
        rep->ms_reuse = 0.0;
        rep->blocks_reused = 0;
    }
    return TDBEM_OK;
}

tdbem_status tdbem_get_entries(tdbem_ctx* c, int64_t n, const int32_t* k, const int32_t* i, const int32_t* j,
                               const int32_t* l, double* out)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (n < 0 || (n > 0 && (!k || !i || !j || !l || !out))) FAIL(c, TDBEM_EINVAL, "bad entry query");
    if (!c->assembled) FAIL(c, TDBEM_ESTATE, "assemble before reading entries");
    if (n == 0) return TDBEM_OK;
    TRY(set_device(c));
    DBuf dk, di, dj, dl, dout;
    TRY(upload(c, dk, k, n));
    TRY(upload(c, di, i, n));
    TRY(upload(c, dj, j, n));
    TRY(upload(c, dl, l, n));
    ALLOC(c, dout, sizeof(double) * n);
    launch_get_entries(c->band(), c->valf64(), c->valf32(), n, dk.as<int32_t>(), di.as<int32_t>(), dj.as<int32_t>(),
                       dl.as<int32_t>(), dout.as<double>(), c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(out, dout.p, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return TDBEM_OK;
}

tdbem_status tdbem_get_entries_noalloc(tdbem_ctx* c, int64_t n, const int32_t* k, const int32_t* i, const int32_t* j,
                                       const int32_t* l, double* out)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (n < 0 || (n > 0 && (!k || !i || !j || !l || !out))) FAIL(c, TDBEM_EINVAL, "bad entry query");
    if (n > kNoAllocEntries)
        FAIL(c, TDBEM_EINVAL, "at most %lld entries per allocation-free query, got %lld", (long long)kNoAllocEntries,
             (long long)n);
    if (!c->assembled) FAIL(c, TDBEM_ESTATE, "assemble before reading entries");
    if (!c->scratch) FAIL(c, TDBEM_EHIP, "the staging array has no device address on device %d", c->device);
    if (n == 0) return TDBEM_OK;
    TRY(set_device(c));
    char* base = static_cast<char*>(c->scratch);
    int32_t* sk = reinterpret_cast<int32_t*>(base);
    int32_t* si = sk + kNoAllocEntries;
    int32_t* sj = si + kNoAllocEntries;
    int32_t* sl = sj + kNoAllocEntries;
    double* so = reinterpret_cast<double*>(sl + kNoAllocEntries);
    const size_t b4 = sizeof(int32_t) * (size_t)n;
    HIPCHK(c, hipMemcpyAsync(sk, k, b4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(si, i, b4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(sj, j, b4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(sl, l, b4, hipMemcpyHostToDevice, c->stream));
    launch_get_entries(c->band(), c->valf64(), c->valf32(), n, sk, si, sj, sl, so, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(out, so, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return TDBEM_OK;
}

static tdbem_status block_coo(tdbem_ctx* c, int32_t k, int32_t i, int32_t* row, int32_t* col, double* val,
                              int64_t cap, int64_t* nnz)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (!c->assembled) FAIL(c, TDBEM_ESTATE, "assemble before reading blocks");
    if (k < 0 || k >= c->N || i < 0 || i >= c->N) FAIL(c, TDBEM_EINVAL, "block (%d, %d) outside 0..%d", k, i, c->N - 1);
    TRY(set_device(c));
    DBuf dcount;
    ALLOC(c, dcount, sizeof(unsigned long long));
    HIPCHK(c, hipMemsetAsync(dcount.p, 0, sizeof(unsigned long long), c->stream));
    launch_block_coo(c->band(), c->valf64(), c->valf32(), k, i, dcount.as<unsigned long long>(), nullptr, nullptr,
                     nullptr, 0, c->stream);
    HIPCHK(c, hipGetLastError());
    unsigned long long cnt = 0;
    HIPCHK(c, hipMemcpyAsync(&cnt, dcount.p, sizeof(cnt), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *nnz = (int64_t)cnt;
    if (!row) return TDBEM_OK;
    if ((int64_t)cnt > cap) FAIL(c, TDBEM_EINVAL, "block (%d, %d) has %llu entries, capacity %lld", k, i, cnt, (long long)cap);
    if (cnt == 0) return TDBEM_OK;
    DBuf drow, dcol, dval;
    ALLOC(c, drow, sizeof(int32_t) * cnt);
    ALLOC(c, dcol, sizeof(int32_t) * cnt);
    ALLOC(c, dval, sizeof(double) * cnt);
    HIPCHK(c, hipMemsetAsync(dcount.p, 0, sizeof(unsigned long long), c->stream));
    launch_block_coo(c->band(), c->valf64(), c->valf32(), k, i, dcount.as<unsigned long long>(), drow.as<int32_t>(),
                     dcol.as<int32_t>(), dval.as<double>(), (int64_t)cnt, c->stream);
    HIPCHK(c, hipGetLastError());
    std::vector<int32_t> r(cnt), cl(cnt);
    std::vector<double> v(cnt);
    HIPCHK(c, hipMemcpyAsync(r.data(), drow.p, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(cl.data(), dcol.p, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(v.data(), dval.p, sizeof(double) * cnt, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // the kernel's positions depend on the order of its atomics: sort by (row, column)
    std::vector<int64_t> ord(cnt);
    for (int64_t s = 0; s < (int64_t)cnt; ++s) ord[s] = s;
    std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return r[a] != r[b] ? r[a] < r[b] : cl[a] < cl[b]; });
    for (int64_t s = 0; s < (int64_t)cnt; ++s) {
        row[s] = r[ord[s]];
        col[s] = cl[ord[s]];
        val[s] = v[ord[s]];
    }
    return TDBEM_OK;
}

tdbem_status tdbem_block_nnz(tdbem_ctx* c, int32_t k, int32_t i, int64_t* nnz)
{
    if (!c) return TDBEM_EINVAL;
    if (!nnz) { c->err = "null nnz"; return TDBEM_EINVAL; }
    return block_coo(c, k, i, nullptr, nullptr, nullptr, 0, nnz);
}

tdbem_status tdbem_get_block_coo(tdbem_ctx* c, int32_t k, int32_t i, int32_t* row, int32_t* col, double* val,
                                 int64_t cap)
{
    if (!c) return TDBEM_EINVAL;
    if (!row || !col || !val || cap < 0) { c->err = "null output or negative capacity"; return TDBEM_EINVAL; }
    int64_t nnz = 0;
    return block_coo(c, k, i, row, col, val, cap, &nnz);
}

tdbem_status tdbem_eval_kernels(tdbem_ctx* c, int64_t n, const int32_t* k, const int32_t* i, const double* r,
                                double* psi, double* tpsi)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (n < 0 || (n > 0 && (!k || !i || !r || !psi || !tpsi))) FAIL(c, TDBEM_EINVAL, "bad kernel query");
    if (!c->assembled) FAIL(c, TDBEM_ESTATE, "assemble before evaluating the kernel tables");
    if (n == 0) return TDBEM_OK;
    TRY(set_device(c));
    DBuf dk, di, dr, dp, dt;
    TRY(upload(c, dk, k, n));
    TRY(upload(c, di, i, n));
    TRY(upload(c, dr, r, n));
    ALLOC(c, dp, sizeof(double) * n);
    ALLOC(c, dt, sizeof(double) * n);
    launch_table_eval(c->tables(), n, dk.as<int32_t>(), di.as<int32_t>(), dr.as<double>(), dp.as<double>(),
                      dt.as<double>(), c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(psi, dp.p, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(tpsi, dt.p, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return TDBEM_OK;
}

tdbem_status tdbem_rhs_plane_pulse(tdbem_ctx* c, const double d[3], double t0, double width, double* g)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (!d || !g) FAIL(c, TDBEM_EINVAL, "null argument");
    if (!(width > 0.0) || !std::isfinite(t0)) FAIL(c, TDBEM_EINVAL, "pulse width must be > 0 and t0 finite");
    if (!c->have_mesh || !c->have_grid) FAIL(c, TDBEM_ESTATE, "set the mesh and the time grid first");
    TRY(set_device(c));
    launch_rhs(c->geom(), c->d_t.as<double>(), c->nodes, c->p1, c->cut, c->rule, d[0], d[1], d[2], t0, width, c->M, g,
               c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return TDBEM_OK;
}

static tdbem_status matvec_range(tdbem_ctx* c, int k0, int k1, int i0, int i1, const double* x, double* y)
{
    launch_matvec(c->band(), c->valf64(), c->valf32(), k0, k1, i0, i1, x, y, c->stream);
    HIPCHK(c, hipGetLastError());
    ++c->matvecs;
    return TDBEM_OK;
}

tdbem_status tdbem_matvec_range(tdbem_ctx* c, int32_t k0, int32_t k1, int32_t i0, int32_t i1, const double* x,
                                double* y)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (!x || !y) FAIL(c, TDBEM_EINVAL, "null vector");
    if (!c->assembled) FAIL(c, TDBEM_ESTATE, "assemble before the matvec");
    if (k0 < 0 || k1 > c->N || k0 >= k1 || i0 < 0 || i1 > c->N || i0 >= i1)
        FAIL(c, TDBEM_EINVAL, "bad block range [%d,%d) x [%d,%d)", k0, k1, i0, i1);
    TRY(set_device(c));
    TRY(matvec_range(c, k0, k1, i0, i1, x, y));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return TDBEM_OK;
}

tdbem_status tdbem_matvec(tdbem_ctx* c, const double* x, double* y)
{
    if (!c) return TDBEM_EINVAL;
    return tdbem_matvec_range(c, 0, c->N, 0, c->N, x, y);
}

// ---------------------------------------------------------------------------------------------
// Learned variable preconditioner (not part of the paper): a message-passing network on the
// space-time graph of the unknowns, trained on the residual loss ||A z - v||^2 / ||v||^2.
// ---------------------------------------------------------------------------------------------
namespace {

uint64_t host_splitmix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// Mesh-neighbour lists (vertices sharing an edge) and step-size features of the current mesh
// and grid, rebuilt when either changed.
tdbem_status lp_graph(tdbem_ctx* c)
{
    if (!c->have_mesh || !c->have_grid) FAIL(c, TDBEM_ESTATE, "set the mesh and the time grid first");
    if (c->p1 != 1) FAIL(c, TDBEM_EINVAL, "the learned preconditioner is implemented for p = 0");
    tdbem_ctx::Learned& L = c->lp;
    if (L.gver == c->graph_version) return TDBEM_OK;
    std::vector<std::vector<int32_t>> nb(c->M);
    for (int e = 0; e < c->E; ++e)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                if (a != b) nb[c->tri[3 * e + a]].push_back(c->tri[3 * e + b]);
    std::vector<int32_t> ptr(c->M + 1, 0), idx;
    for (int j = 0; j < c->M; ++j) {
        std::sort(nb[j].begin(), nb[j].end());
        nb[j].erase(std::unique(nb[j].begin(), nb[j].end()), nb[j].end());
        idx.insert(idx.end(), nb[j].begin(), nb[j].end());
        ptr[j + 1] = (int32_t)idx.size();
    }
    std::vector<float> feat(2 * (size_t)c->N, 0.0f);
    const double hbar = c->t[c->N - 1] / (c->N - 1);
    for (int k = 0; k < c->N; ++k) {
        if (k > 0) feat[2 * k] = (float)((c->t[k] - c->t[k - 1]) / hbar);
        if (k + 1 < c->N) feat[2 * k + 1] = (float)((c->t[k + 1] - c->t[k]) / hbar);
    }
    TRY(upload(c, L.ptr, ptr.data(), ptr.size()));
    TRY(upload(c, L.idx, idx.data(), std::max<size_t>(idx.size(), 1)));
    TRY(upload(c, L.feat, feat.data(), feat.size()));
    L.gver = c->graph_version;
    return TDBEM_OK;
}

LpGraph lp_view(const tdbem_ctx* c)
{
    return LpGraph{c->lp.ptr.as<int32_t>(), c->lp.idx.as<int32_t>(), c->lp.feat.as<float>(), c->M, c->N};
}

// Device scalars of the learned preconditioner: dots[0] = the last ||v||^2, dots[2] = s =
// sqrt(||v||^2 / n), dots[3] = 1/s, from dots[4] on the partial sums of the reductions.
tdbem_status lp_dots(tdbem_ctx* c, int64_t n, double** d)
{
    tdbem_ctx::Learned& L = c->lp;
    const int64_t need = dots_partial_blocks(n) + 4;
    if (L.ndots < need) {
        ALLOC(c, L.dots, sizeof(double) * need);
        L.ndots = need;
    }
    *d = L.dots.as<double>();
    return TDBEM_OK;
}

// ||v||^2 of a device vector (synchronises the stream); leaves the scale scalars untouched.
tdbem_status lp_norm2(tdbem_ctx* c, const double* v, int64_t n, double* out)
{
    double* d;
    TRY(lp_dots(c, n, &d));
    launch_dots(v, 1, n, n, v, d + 4, d, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(out, d, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return TDBEM_OK;
}

// The network's scale of v on the device (no host round trip): dots[2..3] from ||v||^2.
tdbem_status lp_scale(tdbem_ctx* c, const double* v, int64_t n, hipStream_t st)
{
    double* d;
    TRY(lp_dots(c, n, &d));
    launch_dots(v, 1, n, n, v, d + 4, d, st);
    launch_lp_scale(d, n, d + 2, st);
    HIPCHK(c, hipGetLastError());
    return TDBEM_OK;
}

tdbem_status lp_need_params(tdbem_ctx* c)
{
    if (c->lp.layers <= 0) FAIL(c, TDBEM_ESTATE, "initialise the learned preconditioner first");
    return TDBEM_OK;
}

tdbem_status lp_need_inference(tdbem_ctx* c)
{
    tdbem_ctx::Learned& L = c->lp;
    const int64_t n = (int64_t)c->N * c->M;
    if (L.ninf < n) {
        ALLOC(c, L.Hinf, sizeof(float) * 2 * (size_t)n * kLpHidden);
        L.ninf = n;
    }
    double* d;
    TRY(lp_dots(c, n, &d));
    return TDBEM_OK;
}

// z = network(v) for device vectors of N*M values, queued on stream st without a host round
// trip (the scale s is formed on the device; v = 0 gives z = 0).
tdbem_status lp_apply_on(tdbem_ctx* c, const double* v, double* z, hipStream_t st)
{
    TRY(lp_need_params(c));
    TRY(lp_graph(c));
    TRY(lp_need_inference(c));
    tdbem_ctx::Learned& L = c->lp;
    const int64_t n = (int64_t)c->N * c->M;
    TRY(lp_scale(c, v, n, st));
    launch_lp_forward(lp_view(c), L.layers, L.params.as<float>(), L.wq.as<uint16_t>(), v, L.dots.as<double>() + 2,
                      L.Hinf.as<float>(), 0, nullptr, z, st);
    HIPCHK(c, hipGetLastError());
    return TDBEM_OK;
}

tdbem_status lp_apply(tdbem_ctx* c, const double* v, double* z) { return lp_apply_on(c, v, z, c->stream); }

// Capture (or reuse) the graph of the preconditioned operator z = P(v), w = A z on the staging
// vectors lp.gv -> lp.gz, lp.gw.  Every allocation happens before the capture.
tdbem_status lp_operator_graph(tdbem_ctx* c)
{
    TRY(lp_need_params(c));
    TRY(lp_graph(c));
    TRY(lp_need_inference(c));
    tdbem_ctx::Learned& L = c->lp;
    const int64_t n = (int64_t)c->N * c->M;
    if (L.gn < n) {
        ALLOC(c, L.gv, sizeof(double) * n);
        ALLOC(c, L.gz, sizeof(double) * n);
        ALLOC(c, L.gw, sizeof(double) * n);
        L.gn = n;
    }
    const std::vector<uint64_t> key{c->graph_version, c->assemblies, (uint64_t)c->prec, (uint64_t)L.layers,
                                    (uint64_t)(uintptr_t)L.params.p, (uint64_t)(uintptr_t)L.Hinf.p,
                                    (uint64_t)(uintptr_t)L.dots.p, (uint64_t)(uintptr_t)L.gv.p, (uint64_t)n};
    if (L.gexec && key == L.gkey) return TDBEM_OK;
    if (L.gexec) { (void)hipGraphExecDestroy(L.gexec); L.gexec = nullptr; }
    if (L.graph) { (void)hipGraphDestroy(L.graph); L.graph = nullptr; }
    if (!L.cap) HIPCHK(c, hipStreamCreateWithFlags(&L.cap, hipStreamNonBlocking));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipStreamBeginCapture(L.cap, hipStreamCaptureModeThreadLocal));
    tdbem_status st = lp_apply_on(c, L.gv.as<double>(), L.gz.as<double>(), L.cap);
    if (st == TDBEM_OK)
        launch_matvec(c->band(), c->valf64(), c->valf32(), 0, c->N, 0, c->N, L.gz.as<double>(), L.gw.as<double>(), L.cap);
    const hipError_t ee = hipStreamEndCapture(L.cap, &L.graph);
    if (st != TDBEM_OK) return st;
    if (ee != hipSuccess) FAIL(c, TDBEM_EHIP, "graph capture failed: %s", hipGetErrorString(ee));
    HIPCHK(c, hipGraphInstantiate(&L.gexec, L.graph, nullptr, nullptr, 0));
    L.gkey = key;
    return TDBEM_OK;
}

// Training buffers of the network of c for graphs of up to n = N*M nodes.
tdbem_status lp_need_train_n(tdbem_ctx* c, int64_t n)
{
    tdbem_ctx::Learned& L = c->lp;
    if (L.ntrain >= n) return TDBEM_OK;
    const size_t f = sizeof(float) * (size_t)n * kLpHidden;
    ALLOC(c, L.H, f * (L.layers + 1));
    ALLOC(c, L.U, f * std::max(L.layers, 1));
    ALLOC(c, L.DU, f);
    ALLOC(c, L.dX, 4 * f);
    ALLOC(c, L.dH2, 2 * f);
    ALLOC(c, L.partial, sizeof(float) * (size_t)lp_partial_blocks(n) * (4 * kLpHidden * kLpHidden + kLpHidden));
    ALLOC(c, L.vb, sizeof(double) * n);
    ALLOC(c, L.xb, sizeof(double) * n);
    ALLOC(c, L.zb, sizeof(double) * n);
    ALLOC(c, L.rb, sizeof(double) * n);
    ALLOC(c, L.db, sizeof(double) * n);
    L.ntrain = n;
    return TDBEM_OK;
}

tdbem_status lp_need_train_buffers(tdbem_ctx* c) { return lp_need_train_n(c, (int64_t)c->N * c->M); }

// Forward pass keeping every layer's input and pre-activation, then add the gradient of <dz, z>
// to lp.grad.  The scale of v must be in dots[2..3] (lp_scale).
tdbem_status lp_forward_backward(tdbem_ctx* c, const double* v, double* z, const double* dz_or_null,
                                 bool backward_now)
{
    tdbem_ctx::Learned& L = c->lp;
    const int64_t n = (int64_t)c->N * c->M;
    const int64_t hs = n * kLpHidden;
    const double* sc = L.dots.as<double>() + 2;
    if (!backward_now) {
        launch_lp_forward(lp_view(c), L.layers, L.params.as<float>(), L.wq.as<uint16_t>(), v, sc, L.H.as<float>(),
                          hs, L.U.as<float>(), z, c->stream);
    } else {
        launch_lp_backward(lp_view(c), L.layers, L.wq.as<uint16_t>(), v, sc, L.H.as<float>(), L.U.as<float>(),
                           dz_or_null, L.dH2.as<float>(), L.DU.as<float>(), L.dX.as<float>(),
                           L.partial.as<float>(), L.grad.as<float>(), c->stream);
    }
    HIPCHK(c, hipGetLastError());
    return TDBEM_OK;
}

}  // namespace

int64_t tdbem_lp_num_params(int32_t layers)
{
    if (layers < 1 || layers > TDBEM_LP_MAX_LAYERS) return -1;
    return lp_num_params(layers);
}

tdbem_status tdbem_lp_init(tdbem_ctx* c, int32_t layers, uint64_t seed)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (layers < 1 || layers > TDBEM_LP_MAX_LAYERS) FAIL(c, TDBEM_EINVAL, "layers must be in 1..%d", TDBEM_LP_MAX_LAYERS);
    TRY(set_device(c));
    const int64_t P = lp_num_params(layers);
    // uniform initialisation: +-1/sqrt(fan_in) for the input and output maps and the biases,
    // +-0.3/sqrt(256) for the layer weights (small residual updates at the start)
    std::vector<float> p(P);
    uint64_t state = host_splitmix64(seed);
    auto unif = [&](double a) {
        state = host_splitmix64(state);
        return (float)(a * (2.0 * ((double)(state >> 11) * 0x1.0p-53) - 1.0));
    };
    for (int64_t s = 0; s < 3 * kLpHidden; ++s) p[lp_off_win() + s] = unif(1.0 / std::sqrt(3.0));
    for (int s = 0; s < kLpHidden; ++s) p[lp_off_bin() + s] = unif(1.0 / std::sqrt(3.0));
    for (int l = 0; l < layers; ++l) {
        for (int64_t s = 0; s < 4 * kLpHidden * kLpHidden; ++s) p[lp_off_w(l) + s] = unif(0.3 / 16.0);
        for (int s = 0; s < kLpHidden; ++s) p[lp_off_b(l) + s] = unif(0.3 / 16.0);
    }
    for (int s = 0; s < kLpHidden; ++s) p[lp_off_wout(layers) + s] = unif(1.0 / 8.0);
    tdbem_ctx::Learned& L = c->lp;
    L.ntrain = 0;
    L.layers = layers;
    L.P = P;
    L.step = 0;
    L.samples = 0;
    ALLOC(c, L.params, sizeof(float) * P);
    ALLOC(c, L.wq, sizeof(uint16_t) * P);
    ALLOC(c, L.grad, sizeof(float) * P);
    ALLOC(c, L.m1, sizeof(float) * P);
    ALLOC(c, L.m2, sizeof(float) * P);
    HIPCHK(c, hipMemcpyAsync(L.params.p, p.data(), sizeof(float) * P, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemsetAsync(L.m1.p, 0, sizeof(float) * P, c->stream));
    HIPCHK(c, hipMemsetAsync(L.m2.p, 0, sizeof(float) * P, c->stream));
    launch_lp_round(P, L.params.as<float>(), L.wq.as<uint16_t>(), c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return TDBEM_OK;
}

tdbem_status tdbem_lp_set_params(tdbem_ctx* c, const float* params, int64_t n)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    TRY(lp_need_params(c));
    if (!params || n != c->lp.P) FAIL(c, TDBEM_EINVAL, "expected %lld parameters", (long long)c->lp.P);
    TRY(set_device(c));
    tdbem_ctx::Learned& L = c->lp;
    HIPCHK(c, hipMemcpyAsync(L.params.p, params, sizeof(float) * n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemsetAsync(L.m1.p, 0, sizeof(float) * n, c->stream));
    HIPCHK(c, hipMemsetAsync(L.m2.p, 0, sizeof(float) * n, c->stream));
    L.step = 0;
    launch_lp_round(n, L.params.as<float>(), L.wq.as<uint16_t>(), c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return TDBEM_OK;
}

tdbem_status tdbem_lp_get_params(tdbem_ctx* c, float* params, int64_t n)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    TRY(lp_need_params(c));
    if (!params || n != c->lp.P) FAIL(c, TDBEM_EINVAL, "expected %lld parameters", (long long)c->lp.P);
    TRY(set_device(c));
    HIPCHK(c, hipMemcpyAsync(params, c->lp.params.p, sizeof(float) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return TDBEM_OK;
}

tdbem_status tdbem_lp_apply(tdbem_ctx* c, const double* v, double* z)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (!v || !z) FAIL(c, TDBEM_EINVAL, "null vector");
    TRY(set_device(c));
    TRY(lp_apply(c, v, z));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return TDBEM_OK;
}

tdbem_status tdbem_lp_gradient(tdbem_ctx* c, const double* v, const double* dz, double* z, float* grad)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (!v || !dz || !z || !grad) FAIL(c, TDBEM_EINVAL, "null argument");
    TRY(lp_need_params(c));
    TRY(set_device(c));
    TRY(lp_graph(c));
    TRY(lp_need_train_buffers(c));
    tdbem_ctx::Learned& L = c->lp;
    const int64_t n = (int64_t)c->N * c->M;
    HIPCHK(c, hipMemsetAsync(L.grad.p, 0, sizeof(float) * L.P, c->stream));
    TRY(lp_scale(c, v, n, c->stream));                 // v = 0: z = 0 and a zero gradient
    TRY(lp_forward_backward(c, v, z, nullptr, false));
    TRY(lp_forward_backward(c, v, z, dz, true));
    HIPCHK(c, hipMemcpyAsync(grad, L.grad.p, sizeof(float) * L.P, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return TDBEM_OK;
}

tdbem_status tdbem_matvec_transpose(tdbem_ctx* c, const double* y, double* x)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (!x || !y) FAIL(c, TDBEM_EINVAL, "null vector");
    if (!c->assembled) FAIL(c, TDBEM_ESTATE, "assemble before the matvec");
    TRY(set_device(c));
    launch_matvec_transpose(c->band(), c->valf64(), c->valf32(), y, x, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return TDBEM_OK;
}

tdbem_status tdbem_lp_train(tdbem_ctx* c, const tdbem_lp_train_opts* o, float* loss_history,
                            tdbem_lp_train_report* rep)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (!o) FAIL(c, TDBEM_EINVAL, "null options");
    if (o->steps < 1 || o->batch < 1 || !(o->lr > 0.0)) FAIL(c, TDBEM_EINVAL, "bad training options");
    TRY(lp_need_params(c));
    if (!c->assembled) FAIL(c, TDBEM_ESTATE, "assemble before training (the loss applies A)");
    TRY(set_device(c));
    TRY(lp_graph(c));
    TRY(lp_need_train_buffers(c));
    const auto t_start = std::chrono::steady_clock::now();
    tdbem_ctx::Learned& L = c->lp;
    const int64_t n = (int64_t)c->N * c->M;
    hipStream_t st = c->stream;
    double* v = L.vb.as<double>();
    double* x = L.xb.as<double>();
    double* z = L.zb.as<double>();
    double* r = L.rb.as<double>();
    double* dz = L.db.as<double>();
    double first = 0.0, last = 0.0;
    for (int step = 0; step < o->steps; ++step) {
        HIPCHK(c, hipMemsetAsync(L.grad.p, 0, sizeof(float) * L.P, st));
        double sum = 0.0;
        int used = 0;
        for (int b = 0; b < o->batch; ++b) {
            // training residual: a normal vector, or A x for a normal x smoothed 0..3 times over
            // the mesh (residuals whose errors are smooth in space)
            const uint64_t sid = (uint64_t)L.samples++;
            const uint64_t h = host_splitmix64(o->seed ^ host_splitmix64(sid));
            if ((h & 1) == 0) {
                launch_lp_randn(n, o->seed, sid, v, st);
            } else {
                launch_lp_randn(n, o->seed, sid, x, st);
                const int q = (int)((h >> 1) & 3);
                for (int u = 0; u < q; ++u) {
                    launch_lp_smooth(lp_view(c), x, z, st);
                    std::swap(x, z);
                }
                TRY(matvec_range(c, 0, c->N, 0, c->N, x, v));
            }
            HIPCHK(c, hipGetLastError());
            double vv;
            TRY(lp_norm2(c, v, n, &vv));
            if (!(vv > 0.0)) continue;
            TRY(lp_scale(c, v, n, st));
            TRY(lp_forward_backward(c, v, z, nullptr, false));
            TRY(matvec_range(c, 0, c->N, 0, c->N, z, r));
            launch_axpby(r, v, -1.0, 1.0, n, st);                   // r = A z - v
            HIPCHK(c, hipGetLastError());
            double rr;
            TRY(lp_norm2(c, r, n, &rr));
            sum += rr / vv;
            ++used;
            launch_matvec_transpose(c->band(), c->valf64(), c->valf32(), r, dz, st);
            launch_scale_copy(dz, dz, 2.0 / vv, n, st);              // d loss / d z = 2 A^T r / |v|^2
            HIPCHK(c, hipGetLastError());
            TRY(lp_forward_backward(c, v, z, dz, true));
        }
        if (used == 0) continue;
        ++L.step;
        launch_lp_adam(L.P, L.params.as<float>(), L.grad.as<float>(), L.m1.as<float>(), L.m2.as<float>(),
                       (float)o->lr, L.step, 1.0f / (float)used, L.wq.as<uint16_t>(), st);
        HIPCHK(c, hipGetLastError());
        const double loss = sum / used;
        if (step == 0) first = loss;
        last = loss;
        if (loss_history) loss_history[step] = (float)loss;
    }
    HIPCHK(c, hipStreamSynchronize(st));
    if (rep) {
        rep->steps = o->steps;
        rep->samples = (int64_t)o->steps * o->batch;
        rep->loss_first = first;
        rep->loss_last = last;
        rep->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    return TDBEM_OK;
}

tdbem_status tdbem_lp_make_pairs(tdbem_ctx* c, int64_t count, uint64_t seed, double* V, double* Z)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (count < 1 || !V || !Z) FAIL(c, TDBEM_EINVAL, "need count >= 1 and two device arrays");
    if (!c->assembled) FAIL(c, TDBEM_ESTATE, "assemble before forming pairs (the residual applies A)");
    TRY(set_device(c));
    TRY(lp_graph(c));
    const int64_t n = (int64_t)c->N * c->M;
    hipStream_t st = c->stream;
    DBuf tmp;
    ALLOC(c, tmp, sizeof(double) * n);
    for (int64_t s = 0; s < count; ++s) {
        // the error: a normal vector smoothed 0..3 times over the mesh (the number of passes from
        // the seed), the residual it leaves: A times it
        double* z = Z + s * n;
        double* v = V + s * n;
        const uint64_t h = host_splitmix64(seed ^ host_splitmix64((uint64_t)s));
        launch_lp_randn(n, seed, (uint64_t)s, z, st);
        const int q = (int)(h & 3);
        for (int u = 0; u < q; ++u) {
            launch_lp_smooth(lp_view(c), z, tmp.as<double>(), st);
            launch_scale_copy(z, tmp.as<double>(), 1.0, n, st);
        }
        HIPCHK(c, hipGetLastError());
        TRY(matvec_range(c, 0, c->N, 0, c->N, z, v));
    }
    HIPCHK(c, hipStreamSynchronize(st));
    return TDBEM_OK;
}

tdbem_status tdbem_lp_train_pairs(tdbem_ctx* c, tdbem_ctx* g, const double* V, const double* Z, int64_t count,
                                  const tdbem_lp_train_opts* o, float* loss_history, tdbem_lp_train_report* rep)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (!g || !V || !Z || !o || count < 1) FAIL(c, TDBEM_EINVAL, "null argument or count < 1");
    if (o->steps < 1 || o->batch < 1 || !(o->lr > 0.0)) FAIL(c, TDBEM_EINVAL, "bad training options");
    TRY(lp_need_params(c));
    if (g->device != c->device) FAIL(c, TDBEM_EINVAL, "the network and the pairs must be on one device");
    if (g != c) {
        g->err.clear();
        TRY(set_device(g));
        const tdbem_status sg = lp_graph(g);
        if (sg != TDBEM_OK) FAIL(c, sg, "geometry of the pairs: %s", g->err.c_str());
        HIPCHK(c, hipStreamSynchronize(g->stream));   // its graph arrays are used on this stream
    }
    TRY(set_device(c));
    if (g == c) TRY(lp_graph(c));
    const int64_t n = (int64_t)g->N * g->M;
    TRY(lp_need_train_n(c, n));
    double* d;
    TRY(lp_dots(c, n, &d));
    const auto t_start = std::chrono::steady_clock::now();
    tdbem_ctx::Learned& L = c->lp;
    hipStream_t st = c->stream;
    const LpGraph gv = lp_view(g);
    const int64_t hs = n * kLpHidden;
    const double* sc = L.dots.as<double>() + 2;
    double* pz = L.zb.as<double>();
    double* r = L.rb.as<double>();
    double* dz = L.db.as<double>();
    // pairs in a seeded random order, reshuffled after every pass over them
    std::vector<int64_t> order(count);
    int64_t pos = count, pass = 0;
    auto next = [&]() {
        if (pos == count) {
            for (int64_t s = 0; s < count; ++s) order[s] = s;
            uint64_t state = host_splitmix64(o->seed ^ host_splitmix64(0x5EEDull + (uint64_t)pass++));
            for (int64_t s = count - 1; s > 0; --s) {
                state = host_splitmix64(state);
                std::swap(order[s], order[(int64_t)(state % (uint64_t)(s + 1))]);
            }
            pos = 0;
        }
        return order[pos++];
    };
    double first = 0.0, last = 0.0;
    for (int step = 0; step < o->steps; ++step) {
        HIPCHK(c, hipMemsetAsync(L.grad.p, 0, sizeof(float) * L.P, st));
        double sum = 0.0;
        int used = 0;
        for (int b = 0; b < o->batch; ++b) {
            const int64_t s = next();
            const double* v = V + s * n;
            const double* z = Z + s * n;
            double zz;
            TRY(lp_norm2(c, z, n, &zz));
            if (!(zz > 0.0)) continue;
            TRY(lp_scale(c, v, n, st));
            launch_lp_forward(gv, L.layers, L.params.as<float>(), L.wq.as<uint16_t>(), v, sc, L.H.as<float>(), hs,
                              L.U.as<float>(), pz, st);
            launch_scale_copy(r, pz, 1.0, n, st);
            launch_axpby(r, z, -1.0, 1.0, n, st);                       // r = P(v) - z
            HIPCHK(c, hipGetLastError());
            double rr;
            TRY(lp_norm2(c, r, n, &rr));
            sum += rr / zz;
            ++used;
            launch_scale_copy(dz, r, 2.0 / zz, n, st);                  // d loss / d P(v)
            launch_lp_backward(gv, L.layers, L.wq.as<uint16_t>(), v, sc, L.H.as<float>(), L.U.as<float>(), dz,
                               L.dH2.as<float>(), L.DU.as<float>(), L.dX.as<float>(), L.partial.as<float>(),
                               L.grad.as<float>(), st);
            HIPCHK(c, hipGetLastError());
            ++L.samples;
        }
        if (used == 0) continue;
        ++L.step;
        launch_lp_adam(L.P, L.params.as<float>(), L.grad.as<float>(), L.m1.as<float>(), L.m2.as<float>(),
                       (float)o->lr, L.step, 1.0f / (float)used, L.wq.as<uint16_t>(), st);
        HIPCHK(c, hipGetLastError());
        const double loss = sum / used;
        if (step == 0) first = loss;
        last = loss;
        if (loss_history) loss_history[step] = (float)loss;
    }
    HIPCHK(c, hipStreamSynchronize(st));
    if (rep) {
        rep->steps = o->steps;
        rep->samples = (int64_t)o->steps * o->batch;
        rep->loss_first = first;
        rep->loss_last = last;
        rep->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    return TDBEM_OK;
}

// ---------------------------------------------------------------------------------------------
// FGMRES (Saad 1993) with the recursive block-Hessenberg preconditioner (Section 4.2, Alg. 1)
// ---------------------------------------------------------------------------------------------
namespace {

// ---------------------------------------------------------------------------------------------
// DGMRES(m, l) (Section 4.1): deflation of the smallest eigenvalues.  The cycle's Hessenberg
// matrix is small (k <= restart), so its eigenvalues are found on the host by the complex QR
// algorithm with Wilkinson shifts, and eigenvectors by inverse iteration.
// ---------------------------------------------------------------------------------------------
using cplx = std::complex<double>;

// Eigenvalues of the k x k upper Hessenberg matrix H (row-major, leading dimension ld).
std::vector<cplx> hessenberg_eigenvalues(const std::vector<double>& H, int k, int ld)
{
    std::vector<cplx> A((size_t)k * k);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) A[(size_t)i * k + j] = j >= i - 1 ? H[(size_t)i * ld + j] : 0.0;
    auto at = [&](int i, int j) -> cplx& { return A[(size_t)i * k + j]; };
    std::vector<cplx> ev(k);
    int hi = k - 1, iter = 0;
    while (hi >= 0) {
        if (hi == 0) { ev[0] = at(0, 0); break; }
        int lo = hi;
        while (lo > 0 && std::abs(at(lo, lo - 1)) > 1e-15 * (std::abs(at(lo - 1, lo - 1)) + std::abs(at(lo, lo)))) --lo;
        if (lo == hi) { ev[hi] = at(hi, hi); --hi; iter = 0; continue; }
        if (iter > 200 * k) { for (int s = lo; s <= hi; ++s) ev[s] = at(s, s); hi = lo - 1; continue; }
        // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block closer to its last entry
        const cplx a = at(hi - 1, hi - 1), b = at(hi - 1, hi), c = at(hi, hi - 1), d = at(hi, hi);
        const cplx tr = a + d, det = a * d - b * c, disc = std::sqrt(tr * tr * 0.25 - det);
        const cplx m1 = tr * 0.5 + disc, m2 = tr * 0.5 - disc;
        cplx mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
        if (iter % 11 == 10) mu = d + std::abs(c);               // exceptional shift
        ++iter;
        for (int s = lo; s <= hi; ++s) at(s, s) -= mu;
        std::vector<cplx> gc(hi - lo), gs(hi - lo);
        for (int j = lo; j < hi; ++j) {                          // R = G^H (A - mu I) row by row
            const cplx x = at(j, j), y = at(j + 1, j);
            const double rr = std::sqrt(std::norm(x) + std::norm(y));
            const cplx cc = rr > 0.0 ? x / rr : 1.0, ss = rr > 0.0 ? y / rr : 0.0;
            gc[j - lo] = cc;
            gs[j - lo] = ss;
            for (int q = j; q <= hi; ++q) {
                const cplx u = at(j, q), v = at(j + 1, q);
                at(j, q) = std::conj(cc) * u + std::conj(ss) * v;
                at(j + 1, q) = -ss * u + cc * v;
            }
        }
        for (int j = lo; j < hi; ++j) {                          // R Q, Q = prod G_j
            const cplx cc = gc[j - lo], ss = gs[j - lo];
            for (int q = lo; q <= std::min(j + 2, hi); ++q) {
                const cplx u = at(q, j), v = at(q, j + 1);
                at(q, j) = cc * u + ss * v;
                at(q, j + 1) = -std::conj(ss) * u + std::conj(cc) * v;
            }
        }
        for (int s = lo; s <= hi; ++s) at(s, s) += mu;
    }
    return ev;
}

// An eigenvector of H (k x k, leading dimension ld) for the eigenvalue lam: two steps of inverse
// iteration with a slightly perturbed shift (Gaussian elimination with partial pivoting).
std::vector<cplx> hessenberg_eigenvector(const std::vector<double>& H, int k, int ld, cplx lam)
{
    const double scale = std::max(1.0, std::abs(lam));
    const cplx shift = lam + cplx(1e-10 * scale, 1e-10 * scale);
    std::vector<cplx> A((size_t)k * k);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) A[(size_t)i * k + j] = (j >= i - 1 ? H[(size_t)i * ld + j] : 0.0) - (i == j ? shift : 0.0);
    std::vector<int> piv(k);
    for (int j = 0; j < k; ++j) {
        int pr = j;
        for (int i = j + 1; i < k; ++i)
            if (std::abs(A[(size_t)i * k + j]) > std::abs(A[(size_t)pr * k + j])) pr = i;
        piv[j] = pr;
        if (pr != j)
            for (int q = 0; q < k; ++q) std::swap(A[(size_t)j * k + q], A[(size_t)pr * k + q]);
        if (std::abs(A[(size_t)j * k + j]) == 0.0) A[(size_t)j * k + j] = 1e-300;
        for (int i = j + 1; i < k; ++i) {
            const cplx f = A[(size_t)i * k + j] / A[(size_t)j * k + j];
            A[(size_t)i * k + j] = f;
            for (int q = j + 1; q < k; ++q) A[(size_t)i * k + q] -= f * A[(size_t)j * k + q];
        }
    }
    std::vector<cplx> y(k, cplx(1.0, 0.5));
    for (int step = 0; step < 2; ++step) {
        for (int j = 0; j < k; ++j) {
            std::swap(y[j], y[piv[j]]);
            for (int i = j + 1; i < k; ++i) y[i] -= A[(size_t)i * k + j] * y[j];
        }
        for (int j = k - 1; j >= 0; --j) {
            for (int q = j + 1; q < k; ++q) y[j] -= A[(size_t)j * k + q] * y[q];
            y[j] /= A[(size_t)j * k + j];
        }
        double nrm = 0.0;
        for (const cplx& v : y) nrm += std::norm(v);
        nrm = std::sqrt(nrm);
        for (cplx& v : y) v /= nrm;
    }
    return y;
}

// Real orthonormal basis (k x cols, column-major) of the invariant subspace of the eigenvalues of
// smallest modulus (l of them, l + 1 when a complex pair would be split), and the largest modulus.
std::vector<double> smallest_invariant_basis(const std::vector<double>& H, int k, int ld, int l, int* cols,
                                             double* lam_max)
{
    std::vector<cplx> ev = hessenberg_eigenvalues(H, k, ld);
    std::vector<int> order(k);
    for (int s = 0; s < k; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return std::abs(ev[a]) < std::abs(ev[b]); });
    *lam_max = 0.0;
    for (const cplx& v : ev) *lam_max = std::max(*lam_max, std::abs(v));
    std::vector<std::vector<double>> vecs;
    int taken = 0;
    for (int idx : order) {
        if (taken >= l) break;
        const cplx lam = ev[idx];
        if (std::fabs(lam.imag()) > 1e-12 * std::max(1.0, std::abs(lam))) {
            if (lam.imag() < 0.0) continue;                      // the partner with Im > 0 gives the pair
            std::vector<cplx> y = hessenberg_eigenvector(H, k, ld, lam);
            std::vector<double> re(k), im(k);
            for (int s = 0; s < k; ++s) { re[s] = y[s].real(); im[s] = y[s].imag(); }
            vecs.push_back(re);
            vecs.push_back(im);
            taken += 2;
        } else {
            std::vector<cplx> y = hessenberg_eigenvector(H, k, ld, cplx(lam.real(), 0.0));
            std::vector<double> re(k);
            for (int s = 0; s < k; ++s) re[s] = y[s].real();
            vecs.push_back(re);
            taken += 1;
        }
    }
    std::vector<double> Q;
    for (auto& v : vecs) {                                       // modified Gram-Schmidt, twice
        for (int pass = 0; pass < 2; ++pass)
            for (size_t c0 = 0; c0 < Q.size() / k; ++c0) {
                double d = 0.0;
                for (int s = 0; s < k; ++s) d += Q[c0 * k + s] * v[s];
                for (int s = 0; s < k; ++s) v[s] -= d * Q[c0 * k + s];
            }
        double nrm = 0.0;
        for (double x : v) nrm += x * x;
        nrm = std::sqrt(nrm);
        if (nrm < 1e-10) continue;
        for (double x : v) Q.push_back(x / nrm);
    }
    *cols = (int)(Q.size() / k);
    return Q;
}

// Inverse of a small dense matrix (row-major) by Gauss-Jordan elimination with partial pivoting.
bool small_inverse(std::vector<double> A, int r, std::vector<double>& inv)
{
    inv.assign((size_t)r * r, 0.0);
    for (int s = 0; s < r; ++s) inv[(size_t)s * r + s] = 1.0;
    for (int j = 0; j < r; ++j) {
        int pr = j;
        for (int i = j + 1; i < r; ++i)
            if (std::fabs(A[(size_t)i * r + j]) > std::fabs(A[(size_t)pr * r + j])) pr = i;
        if (A[(size_t)pr * r + j] == 0.0) return false;
        for (int q = 0; q < r; ++q) {
            std::swap(A[(size_t)j * r + q], A[(size_t)pr * r + q]);
            std::swap(inv[(size_t)j * r + q], inv[(size_t)pr * r + q]);
        }
        const double d = A[(size_t)j * r + j];
        for (int q = 0; q < r; ++q) { A[(size_t)j * r + q] /= d; inv[(size_t)j * r + q] /= d; }
        for (int i = 0; i < r; ++i) {
            if (i == j) continue;
            const double f = A[(size_t)i * r + j];
            if (f == 0.0) continue;
            for (int q = 0; q < r; ++q) { A[(size_t)i * r + q] -= f * A[(size_t)j * r + q]; inv[(size_t)i * r + q] -= f * inv[(size_t)j * r + q]; }
        }
    }
    return true;
}

struct SolveCtx {
    tdbem_ctx* c;
    double tol;
    int restart;
    int levels;
    const int32_t* inner;
    void (*progress)(int32_t, double, void*);
    void* progress_user;
    int kind;               // 0: Algorithm 1 / none, 1: learned network, 2: learned, then Algorithm 1,
                            // 3: deflation (DGMRES)
    int defl_l;             // DGMRES: vectors added to the deflation space after each restart
    bool learned_active;    // the outer iteration currently uses the learned network
    bool graph;             // the learned iteration replays the captured z = P(v), w = A z
    bool inner32;           // Algorithm 1's inner products read the FP32 copy of the band
};

// Block product inside the solver: the outer iteration (depth 0) uses the assembled operator; the
// preconditioner's products (depth >= 1) the FP32 copy when inner32 is set.
tdbem_status solver_matvec(SolveCtx& S, int depth, int k0, int k1, int i0, int i1, const double* x, double* y)
{
    tdbem_ctx* c = S.c;
    if (!(S.inner32 && depth >= 1)) return matvec_range(c, k0, k1, i0, i1, x, y);
    launch_matvec(c->band(), nullptr, c->d_val32.as<float>(), k0, k1, i0, i1, x, y, c->stream);
    HIPCHK(c, hipGetLastError());
    ++c->matvecs;
    return TDBEM_OK;
}

tdbem_status fgmres(SolveCtx& S, int depth, int a, int b, const double* rhs, double* x, int max_it, bool inner,
                    int* its_out, double* rel_out);

// y ~ M^{-1} v for the time-block range [a, b) at recursion level `level` (1-based): split at
// h = a + ceil((b - a)/2), y1 ~ M11^{-1} v1, y2 ~ M22^{-1} (v2 - M21 y1) by inner FGMRES.
tdbem_status apply_precond(SolveCtx& S, int depth, int level, int a, int b, const double* v, double* y)
{
    tdbem_ctx* c = S.c;
    const int64_t M = c->M;
    const int p1 = c->p1;                          // split between the node groups of p + 1 bases
    const int h = a + ((b - a) / p1 + 1) / 2 * p1;
    const int m_it = S.inner[level - 1];
    int its;
    double rel;
    TRY(fgmres(S, depth, a, h, v, y, m_it, true, &its, &rel));
    if (b > h) {
        tdbem_ctx::Level& L = c->levels[depth];
        double* tmp = L.tmp.as<double>();
        TRY(solver_matvec(S, depth, h, b, a, h, y, tmp));                             // M21 y1
        launch_axpby(tmp, v + (int64_t)(h - a) * M, 1.0, -1.0, (int64_t)(b - h) * M, c->stream);   // v2 - M21 y1
        HIPCHK(c, hipGetLastError());
        TRY(fgmres(S, depth, h, b, tmp, y + (int64_t)(h - a) * M, m_it, true, &its, &rel));
    }
    return TDBEM_OK;
}

// z = M^{-1} v = v + U (|lambda| T^{-1} - I) U^T v (Section 4.1) for the outer solve.
tdbem_status apply_deflation(SolveCtx& S, const double* v, double* z, int64_t n, double* part)
{
    tdbem_ctx* c = S.c;
    tdbem_ctx::Deflation& D = c->defl;
    hipStream_t st = c->stream;
    launch_scale_copy(z, v, 1.0, n, st);
    if (D.r == 0) return TDBEM_OK;
    double* dc = D.coef.as<double>();
    launch_dots(D.U.as<double>(), D.r, n, n, v, part, dc, st);
    std::vector<double> cv(D.r), d(D.r);
    HIPCHK(c, hipMemcpyAsync(cv.data(), dc, sizeof(double) * D.r, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    for (int a = 0; a < D.r; ++a) {
        double s = 0.0;
        for (int b = 0; b < D.r; ++b) s += D.Tinv[(size_t)a * D.r + b] * cv[b];
        d[a] = D.lam * s - cv[a];
    }
    HIPCHK(c, hipMemcpyAsync(dc, d.data(), sizeof(double) * D.r, hipMemcpyHostToDevice, st));
    launch_sub_combination(z, D.U.as<double>(), D.r, n, n, dc, 1.0, st);
    HIPCHK(c, hipGetLastError());
    return TDBEM_OK;
}

// After a restart cycle of the outer DGMRES: append the basis V_k S of the invariant subspace of
// the cycle's Hessenberg matrix for its l smallest eigenvalues to U (orthonormalised against U,
// classical Gram-Schmidt twice), with A U and T = U^T A U; |lambda| = the largest eigenvalue
// modulus seen.
tdbem_status update_deflation(SolveCtx& S, const std::vector<double>& Hraw, int k, int ld, const double* V,
                              int64_t n, double* part)
{
    tdbem_ctx* c = S.c;
    tdbem_ctx::Deflation& D = c->defl;
    hipStream_t st = c->stream;
    if (D.r >= D.rmax || k < 2) return TDBEM_OK;
    int cols = 0;
    double lam_max = 0.0;
    const std::vector<double> Sb = smallest_invariant_basis(Hraw, k, ld, std::min(S.defl_l, D.rmax - D.r), &cols, &lam_max);
    D.lam = std::max(D.r > 0 ? D.lam : 0.0, lam_max);
    double* dc = D.coef.as<double>();
    for (int col = 0; col < cols && D.r < D.rmax; ++col) {
        double* u = D.U.as<double>() + (int64_t)D.r * n;
        HIPCHK(c, hipMemcpyAsync(dc, Sb.data() + (size_t)col * k, sizeof(double) * k, hipMemcpyHostToDevice, st));
        launch_fill(u, 0.0, n, st);
        launch_sub_combination(u, V, k, n, n, dc, 1.0, st);
        for (int pass = 0; pass < 2 && D.r > 0; ++pass) {
            launch_dots(D.U.as<double>(), D.r, n, n, u, part, dc, st);
            launch_sub_combination(u, D.U.as<double>(), D.r, n, n, dc, -1.0, st);
        }
        launch_dots(u, 1, n, n, u, part, dc, st);
        double nn = 0.0;
        HIPCHK(c, hipMemcpyAsync(&nn, dc, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        if (!(nn > 1e-20)) continue;                              // already in the span of U
        launch_scale_copy(u, u, 1.0 / std::sqrt(nn), n, st);
        double* au = D.AU.as<double>() + (int64_t)D.r * n;
        TRY(matvec_range(c, 0, c->N, 0, c->N, u, au));
        const int r1 = D.r + 1;
        std::vector<double> colv(r1), rowv(r1);
        launch_dots(D.U.as<double>(), r1, n, n, au, part, dc, st);          // u_a^T A u_new
        HIPCHK(c, hipMemcpyAsync(colv.data(), dc, sizeof(double) * r1, hipMemcpyDeviceToHost, st));
        launch_dots(D.AU.as<double>(), r1, n, n, u, part, dc, st);          // u_new^T A u_b
        HIPCHK(c, hipMemcpyAsync(rowv.data(), dc, sizeof(double) * r1, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        std::vector<double> T((size_t)r1 * r1);
        for (int a = 0; a < D.r; ++a)
            for (int b = 0; b < D.r; ++b) T[(size_t)a * r1 + b] = D.T[(size_t)a * D.r + b];
        for (int a = 0; a < r1; ++a) T[(size_t)a * r1 + D.r] = colv[a];
        for (int b = 0; b < D.r; ++b) T[(size_t)D.r * r1 + b] = rowv[b];
        std::vector<double> Ti;
        if (!small_inverse(T, r1, Ti)) continue;                   // singular T: drop the vector
        D.T.swap(T);
        D.Tinv.swap(Ti);
        D.r = r1;
    }
    return TDBEM_OK;
}

// Solve A[a:b, a:b] x = rhs.  depth indexes the workspace; the preconditioner of a solve at
// depth d (level d in Algorithm 1 numbering, the outer solve being depth 0) runs its inner
// solves at depth d + 1.
// An inner solve of Algorithm 1: a fixed number m of flexible Arnoldi steps from x = 0, queued
// without a host round trip; the Hessenberg columns (both Gram-Schmidt passes and |w|^2) stay on
// the device until the end, where one copy brings them to the host for the Givens rotations and
// the triangular solve.  The result equals the step-by-step form: the solution is taken at the
// first step whose residual estimate meets the tolerance, or at a breakdown (|w| = 0, after which
// the queued steps see zero vectors).
tdbem_status fgmres_fixed(SolveCtx& S, int depth, int a, int b, const double* rhs, double* x, int m, int* its_out,
                          double* rel_out)
{
    tdbem_ctx* c = S.c;
    hipStream_t st = c->stream;
    const int64_t n = (int64_t)(b - a) * c->M;
    tdbem_ctx::Level& L = c->levels[depth];
    const bool alg1 = depth < S.levels && (b - a) > c->p1;
    double* V = L.V.as<double>();
    double* Z = alg1 ? L.Z.as<double>() : V;
    const int hs = 2 * (m + 1) + 1;           // column j: [0, j] h1, [m+1, m+1+j] h2, [2m+2] |w|^2
    double* Hd = L.h.as<double>();
    double* bn2d = Hd + (size_t)m * hs;
    double* part = L.partial.as<double>();
    launch_fill(x, 0.0, n, st);
    launch_dots(rhs, 1, n, n, rhs, part, bn2d, st);
    launch_scale_inv_sqrt(V, rhs, bn2d, n, st);     // v_0 = rhs / ||rhs|| (zero for rhs = 0)
    for (int j = 0; j < m; ++j) {
        double* vj = V + (int64_t)j * n;
        double* zj = Z + (int64_t)j * n;
        double* w = V + (int64_t)(j + 1) * n;
        double* hc = Hd + (size_t)j * hs;
        if (alg1) TRY(apply_precond(S, depth + 1, depth + 1, a, b, vj, zj));
        TRY(solver_matvec(S, depth, a, b, a, b, zj, w));
        launch_dots(V, j + 1, n, n, w, part, hc, st);
        launch_sub_combination(w, V, j + 1, n, n, hc, -1.0, st);
        launch_dots(V, j + 1, n, n, w, part, hc + (m + 1), st);
        launch_sub_combination(w, V, j + 1, n, n, hc + (m + 1), -1.0, st);
        launch_dots(w, 1, n, n, w, part, hc + 2 * (m + 1), st);
        launch_scale_inv_sqrt(w, w, hc + 2 * (m + 1), n, st);
        HIPCHK(c, hipGetLastError());
    }
    std::vector<double> hb((size_t)m * hs + 1);
    HIPCHK(c, hipMemcpyAsync(hb.data(), Hd, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    const double bnorm = std::sqrt(std::max(hb[(size_t)m * hs], 0.0));
    *its_out = 0;
    if (bnorm == 0.0) {
        *rel_out = 0.0;
        return TDBEM_OK;
    }
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), gv(m + 1, 0.0);
    gv[0] = bnorm;
    int jdone = 0;
    for (int j = 0; j < m; ++j) {
        const double* hc = hb.data() + (size_t)j * hs;
        for (int q = 0; q <= j; ++q) H[(size_t)q * m + j] = hc[q] + hc[m + 1 + q];
        const double hn = std::sqrt(std::max(hc[2 * (m + 1)], 0.0));
        H[(size_t)(j + 1) * m + j] = hn;
        for (int q = 0; q < j; ++q) {
            const double t1 = cs[q] * H[(size_t)q * m + j] + sn[q] * H[(size_t)(q + 1) * m + j];
            H[(size_t)(q + 1) * m + j] = -sn[q] * H[(size_t)q * m + j] + cs[q] * H[(size_t)(q + 1) * m + j];
            H[(size_t)q * m + j] = t1;
        }
        const double den = std::hypot(H[(size_t)j * m + j], H[(size_t)(j + 1) * m + j]);
        cs[j] = den != 0.0 ? H[(size_t)j * m + j] / den : 1.0;
        sn[j] = den != 0.0 ? H[(size_t)(j + 1) * m + j] / den : 0.0;
        H[(size_t)j * m + j] = cs[j] * H[(size_t)j * m + j] + sn[j] * H[(size_t)(j + 1) * m + j];
        H[(size_t)(j + 1) * m + j] = 0.0;
        gv[j + 1] = -sn[j] * gv[j];
        gv[j] = cs[j] * gv[j];
        jdone = j + 1;
        if (std::fabs(gv[j + 1]) <= S.tol * bnorm || hn == 0.0) break;
    }
    std::vector<double> y(jdone);
    for (int q = jdone - 1; q >= 0; --q) {
        double s = gv[q];
        for (int u = q + 1; u < jdone; ++u) s -= H[(size_t)q * m + u] * y[u];
        y[q] = s / H[(size_t)q * m + q];
    }
    HIPCHK(c, hipMemcpyAsync(Hd, y.data(), sizeof(double) * jdone, hipMemcpyHostToDevice, st));
    launch_sub_combination(x, Z, jdone, n, n, Hd, 1.0, st);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(st));
    *its_out = jdone;
    *rel_out = std::fabs(gv[jdone]) / bnorm;
    return TDBEM_OK;
}

tdbem_status fgmres(SolveCtx& S, int depth, int a, int b, const double* rhs, double* x, int max_it, bool inner,
                    int* its_out, double* rel_out)
{
    tdbem_ctx* c = S.c;
    hipStream_t st = c->stream;
    const int64_t n = (int64_t)(b - a) * c->M;
    tdbem_ctx::Level& L = c->levels[depth];
    const bool alg1 = depth < S.levels && (b - a) > c->p1;
    const bool precond = alg1 || (depth == 0 && S.kind != 0);
    const int m = inner ? max_it : std::min(S.restart, max_it);
    double* V = L.V.as<double>();
    double* Z = precond ? L.Z.as<double>() : V;
    double* dbuf = L.h.as<double>();          // [0, m+1): h1, [m+1, 2m+2): h2, [2m+2]: |w|^2
    double* part = L.partial.as<double>();
    *its_out = 0;
    if (inner) return fgmres_fixed(S, depth, a, b, rhs, x, m, its_out, rel_out);
    // ||rhs||
    launch_dots(rhs, 1, n, n, rhs, part, dbuf + 2 * (m + 1), st);
    double bn2;
    HIPCHK(c, hipMemcpyAsync(&bn2, dbuf + 2 * (m + 1), sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    const double bnorm = std::sqrt(bn2);
    launch_fill(x, 0.0, n, st);
    if (bnorm == 0.0) {
        *rel_out = 0.0;
        return TDBEM_OK;
    }
    double beta = bnorm;
    const double* r = rhs;   // residual of x = 0
    double* wres = L.w.as<double>();
    int its = 0;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), hbuf(2 * (m + 1) + 1);
    const bool deflate = depth == 0 && S.kind == 3;
    std::vector<double> Hraw(deflate ? (size_t)(m + 1) * m : 0);   // the cycle's Hessenberg matrix, unrotated
    while (true) {
        const int mm = inner ? max_it - its : std::min(m, max_it - its);
        if (mm <= 0 || beta <= S.tol * bnorm) break;
        launch_scale_copy(V, r, 1.0 / beta, n, st);
        std::fill(gv.begin(), gv.end(), 0.0);
        gv[0] = beta;
        int jdone = 0;
        bool done = false;
        for (int j = 0; j < mm; ++j) {
            double* vj = V + (int64_t)j * n;
            double* zj = Z + (int64_t)j * n;
            double* w = V + (int64_t)(j + 1) * n;
            if (depth == 0 && S.learned_active && S.graph) {
                // one graph launch for the preconditioned operator, through the staging vectors
                tdbem_ctx::Learned& Lp = c->lp;
                HIPCHK(c, hipMemcpyAsync(Lp.gv.p, vj, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
                HIPCHK(c, hipGraphLaunch(Lp.gexec, st));
                HIPCHK(c, hipMemcpyAsync(zj, Lp.gz.p, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
                HIPCHK(c, hipMemcpyAsync(w, Lp.gw.p, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
                ++c->matvecs;
            } else {
                if (depth == 0 && S.learned_active) TRY(lp_apply(c, vj, zj));
                else if (deflate) TRY(apply_deflation(S, vj, zj, n, part));
                else if (alg1) TRY(apply_precond(S, depth + 1, depth + 1, a, b, vj, zj));
                else if (precond) launch_scale_copy(zj, vj, 1.0, n, st);
                TRY(solver_matvec(S, depth, a, b, a, b, zj, w));
            }
            // classical Gram-Schmidt, twice
            launch_dots(V, j + 1, n, n, w, part, dbuf, st);
            launch_sub_combination(w, V, j + 1, n, n, dbuf, -1.0, st);
            launch_dots(V, j + 1, n, n, w, part, dbuf + (m + 1), st);
            launch_sub_combination(w, V, j + 1, n, n, dbuf + (m + 1), -1.0, st);
            launch_dots(w, 1, n, n, w, part, dbuf + 2 * (m + 1), st);
            launch_scale_inv_sqrt(w, w, dbuf + 2 * (m + 1), n, st);
            HIPCHK(c, hipGetLastError());
            HIPCHK(c, hipMemcpyAsync(hbuf.data(), dbuf, sizeof(double) * (2 * (m + 1) + 1), hipMemcpyDeviceToHost, st));
            HIPCHK(c, hipStreamSynchronize(st));
            for (int q = 0; q <= j; ++q) H[(size_t)q * m + j] = hbuf[q] + hbuf[m + 1 + q];
            const double hn = std::sqrt(std::max(hbuf[2 * (m + 1)], 0.0));
            H[(size_t)(j + 1) * m + j] = hn;
            if (deflate) {
                for (int q = 0; q <= j + 1; ++q) Hraw[(size_t)q * m + j] = H[(size_t)q * m + j];
            }
            for (int q = 0; q < j; ++q) {
                const double t1 = cs[q] * H[(size_t)q * m + j] + sn[q] * H[(size_t)(q + 1) * m + j];
                H[(size_t)(q + 1) * m + j] = -sn[q] * H[(size_t)q * m + j] + cs[q] * H[(size_t)(q + 1) * m + j];
                H[(size_t)q * m + j] = t1;
            }
            const double den = std::hypot(H[(size_t)j * m + j], H[(size_t)(j + 1) * m + j]);
            cs[j] = den != 0.0 ? H[(size_t)j * m + j] / den : 1.0;
            sn[j] = den != 0.0 ? H[(size_t)(j + 1) * m + j] / den : 0.0;
            H[(size_t)j * m + j] = cs[j] * H[(size_t)j * m + j] + sn[j] * H[(size_t)(j + 1) * m + j];
            H[(size_t)(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            ++its;
            jdone = j + 1;
            if (!inner && S.progress) S.progress(its, std::fabs(gv[j + 1]) / bnorm, S.progress_user);
            if (std::fabs(gv[j + 1]) <= S.tol * bnorm || hn == 0.0) { done = true; break; }
        }
        // y = H^{-1} g (upper triangular), x += Z y
        std::vector<double> y(jdone);
        for (int q = jdone - 1; q >= 0; --q) {
            double s = gv[q];
            for (int u = q + 1; u < jdone; ++u) s -= H[(size_t)q * m + u] * y[u];
            y[q] = s / H[(size_t)q * m + q];
        }
        HIPCHK(c, hipMemcpyAsync(dbuf, y.data(), sizeof(double) * jdone, hipMemcpyHostToDevice, st));
        launch_sub_combination(x, Z, jdone, n, n, dbuf, 1.0, st);
        HIPCHK(c, hipGetLastError());
        if (inner) {
            HIPCHK(c, hipStreamSynchronize(st));
            break;
        }
        // true residual
        TRY(matvec_range(c, a, b, a, b, x, wres));
        launch_axpby(wres, rhs, 1.0, -1.0, n, st);        // rhs - A x
        launch_dots(wres, 1, n, n, wres, part, dbuf + 2 * (m + 1), st);
        double r2;
        HIPCHK(c, hipMemcpyAsync(&r2, dbuf + 2 * (m + 1), sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        beta = std::sqrt(r2);
        r = wres;
        (void)done;
        if (depth == 0 && S.kind == 2) S.learned_active = false;   // fall back to Algorithm 1
        if (beta <= S.tol * bnorm || its >= max_it) break;
        if (deflate) TRY(update_deflation(S, Hraw, jdone, m, V, n, part));
    }
    *its_out = its;
    *rel_out = beta / bnorm;
    return TDBEM_OK;
}

}  // namespace

tdbem_status tdbem_solve(tdbem_ctx* c, const double* g, double* alpha, const tdbem_solve_opts* o,
                         tdbem_solve_report* rep)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (!g || !alpha || !o) FAIL(c, TDBEM_EINVAL, "null argument");
    if (!c->assembled) FAIL(c, TDBEM_ESTATE, "assemble before solving");
    if (o->restart < 1 || o->restart > 5000 || !(o->tol > 0.0) || o->max_it < 1 || o->precond_levels < 0 ||
        o->precond_levels > 8)
        FAIL(c, TDBEM_EINVAL, "bad solver options");
    for (int s = 0; s < o->precond_levels; ++s)
        if (o->precond_inner[s] < 1 || o->precond_inner[s] > 1000) FAIL(c, TDBEM_EINVAL, "bad inner iteration count");
    if (o->precond_kind < 0 || o->precond_kind > 3) FAIL(c, TDBEM_EINVAL, "unknown preconditioner kind %d", o->precond_kind);
    if (o->precond_kind == 3 && (o->deflation_l < 1 || o->deflation_max < o->deflation_l || o->deflation_max > 256 ||
                                 o->precond_levels != 0 || o->use_graph))
        FAIL(c, TDBEM_EINVAL, "deflation needs 1 <= deflation_l <= deflation_max <= 256, no Algorithm 1 levels and no graph");
    if (o->precond_kind == 2 && o->precond_levels < 1)
        FAIL(c, TDBEM_EINVAL, "the learned-then-Algorithm-1 preconditioner needs precond_levels > 0");
    TRY(set_device(c));
    if (o->use_graph != 0 && o->use_graph != 1) FAIL(c, TDBEM_EINVAL, "use_graph must be 0 or 1");
    if (o->use_graph && o->precond_kind == 0)
        FAIL(c, TDBEM_EINVAL, "the captured iteration applies the learned preconditioner (precond_kind 1 or 2)");
    if (o->precond_kind == 1 || o->precond_kind == 2) {
        TRY(lp_need_params(c));
        TRY(lp_graph(c));
    }
    if (o->inner_fp32 != 0 && o->inner_fp32 != 1) FAIL(c, TDBEM_EINVAL, "inner_fp32 must be 0 or 1");
    if (o->inner_fp32 && (c->prec != TDBEM_FP64 || o->precond_levels < 1 || o->precond_kind != 0))
        FAIL(c, TDBEM_EINVAL, "inner_fp32 needs an FP64 assembly and Algorithm 1 (precond_levels > 0)");
    if (o->inner_fp32 && c->val32_assembly != c->assemblies) {
        const int64_t nv = std::max<int64_t>(c->nvals, 1);
        ALLOC(c, c->d_val32, sizeof(float) * (size_t)nv);
        launch_to_f32(c->d_val.as<double>(), c->d_val32.as<float>(), c->nvals, c->stream);
        HIPCHK(c, hipGetLastError());
        c->val32_assembly = c->assemblies;
    }
    if (o->precond_kind == 3) {
        tdbem_ctx::Deflation& D = c->defl;
        const int64_t n = (int64_t)c->N * c->M;
        if (D.rmax < o->deflation_max || D.n != n) {
            ALLOC(c, D.U, sizeof(double) * (size_t)o->deflation_max * n);
            ALLOC(c, D.AU, sizeof(double) * (size_t)o->deflation_max * n);
            ALLOC(c, D.coef, sizeof(double) * (size_t)std::max(o->deflation_max, o->restart) + 8);
        }
        D.rmax = o->deflation_max;
        D.n = n;
        D.r = 0;                                   // a fresh deflation space for every solve
        D.T.clear();
        D.Tinv.clear();
        D.lam = 1.0;
    }
    if (o->use_graph) TRY(lp_operator_graph(c));
    const auto t_start = std::chrono::steady_clock::now();
    const int64_t M = c->M;
    // workspaces: depth 0 is the outer solve; depth d >= 1 holds ranges of <= ceil(N / 2^(d-1)) blocks
    const int depths = o->precond_levels + 1;
    if ((int)c->levels.size() < depths) c->levels.resize(depths);
    int blocks = c->N;
    for (int d = 0; d < depths; ++d) {
        const int m = d == 0 ? o->restart : o->precond_inner[d - 1];
        const int64_t n = (int64_t)blocks * M;
        tdbem_ctx::Level& L = c->levels[d];
        if (L.m < m || L.n < n) {
            ALLOC(c, L.V, sizeof(double) * (size_t)(m + 1) * n);
            ALLOC(c, L.Z, sizeof(double) * (size_t)m * n);
            ALLOC(c, L.w, sizeof(double) * n);
            ALLOC(c, L.tmp, sizeof(double) * n);
            ALLOC(c, L.partial, sizeof(double) * (size_t)(m + 2) * dots_partial_blocks(n));
            // the outer solve keeps one Hessenberg column on the device; an inner solve (a fixed
            // number of steps) keeps all of its columns and ||rhs||^2
            ALLOC(c, L.h, sizeof(double) * ((size_t)(d == 0 ? 1 : m) * (2 * (m + 1) + 1) + 2));
            L.m = m;
            L.n = n;
        }
        blocks = (blocks / c->p1 + 1) / 2 * c->p1;
    }
    SolveCtx S{c,
               o->tol,
               o->restart,
               o->precond_levels,
               o->precond_inner,
               o->progress,
               o->progress_user,
               o->precond_kind,
               o->precond_kind == 3 ? o->deflation_l : 0,
               o->precond_kind == 1 || o->precond_kind == 2,
               o->use_graph != 0,
               o->inner_fp32 != 0};
    c->matvecs = 0;
    int its = 0;
    double rel = 0.0;
    TRY(fgmres(S, 0, 0, c->N, g, alpha, o->max_it, false, &its, &rel));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (rep) {
        rep->iterations = its;
        rep->matvecs = c->matvecs;
        rep->rel_residual = rel;
        rep->ms = ms;
    }
    if (!(rel <= o->tol)) {
        char b[160];
        std::snprintf(b, sizeof(b), "not converged: relative residual %.3e after %d iterations", rel, its);
        c->err = b;
        return TDBEM_NOT_CONVERGED;
    }
    return TDBEM_OK;
}


// ---------------------------------------------------------------------------------------------
// Retarded double layer potential (eq. (RetardedPotential)): the field off the surface.
// ---------------------------------------------------------------------------------------------
tdbem_status tdbem_potential_dl(tdbem_ctx* c, const double* alpha, int64_t npts, const double* pts, int32_t ntimes,
                                const double* times, double* u)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (!alpha || !pts || !times || !u) FAIL(c, TDBEM_EINVAL, "null argument");
    if (!c->have_mesh || !c->have_grid) FAIL(c, TDBEM_ESTATE, "set the mesh and the time grid first");
    if (npts < 1 || ntimes < 1) FAIL(c, TDBEM_EINVAL, "need at least one point and one time");
    if (c->p1 != 1) FAIL(c, TDBEM_EINVAL, "the field evaluation is implemented for p = 0");
    if (c->N > 1024) FAIL(c, TDBEM_EINVAL, "the field evaluation takes at most 1024 time nodes");
    const double T = c->t[c->N - 1];
    for (int s = 0; s < ntimes; ++s)
        if (!(times[s] >= 0.0 && times[s] <= T)) FAIL(c, TDBEM_EINVAL, "time %d = %g outside [0, T]", s, times[s]);
    for (int64_t p = 0; p < 3 * npts; ++p)
        if (!std::isfinite(pts[p])) FAIL(c, TDBEM_EINVAL, "point coordinate %lld is not finite", (long long)p);
    TRY(set_device(c));
    DBuf dp, dt, phiq;
    TRY(upload(c, dp, pts, (size_t)(3 * npts)));
    TRY(upload(c, dt, times, (size_t)ntimes));
    ALLOC(c, phiq, sizeof(double) * (size_t)c->E * 7 * c->N);
    launch_potential(c->geom(), c->d_t.as<double>(), c->N, c->cut, c->M, alpha, phiq.as<double>(), npts,
                     dp.as<double>(), ntimes, dt.as<double>(), u, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return TDBEM_OK;
}

// ---------------------------------------------------------------------------------------------
// Many right-hand sides: one product per iteration serves all of them (the stored operator is
// read once per group of 4 right-hand sides); FGMRES runs per right-hand side on its own Krylov
// basis, with all Gram-Schmidt coefficients of an iteration fetched in one host round trip.
// ---------------------------------------------------------------------------------------------
namespace {
// Autotuning of the multi-vector product: every variant runs twice on 8 vectors of ones over the
// assembled operator, timed with HIP events on the context's stream; the fastest is kept until the
// next assembly.
tdbem_status multi_tune(tdbem_ctx* c)
{
    if (c->mm_variant >= 0) return TDBEM_OK;
    const int64_t n = (int64_t)c->N * c->M;
    const int R = 8;
    DBuf X, Y;
    ALLOC(c, X, sizeof(double) * (size_t)R * n);
    ALLOC(c, Y, sizeof(double) * (size_t)R * n);
    launch_fill(X.as<double>(), 1.0, R * n, c->stream);
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    const int nv = matvec_multi_variants();
    c->mm_ms.assign(nv, 0.0);
    int best = 0;
    for (int v = 0; v < nv; ++v) {
        launch_matvec_multi(c->band(), c->valf64(), c->valf32(), R, X.as<double>(), n, Y.as<double>(), n, v, c->stream);
        (void)hipEventRecord(e0, c->stream);
        for (int rep = 0; rep < 2; ++rep)
            launch_matvec_multi(c->band(), c->valf64(), c->valf32(), R, X.as<double>(), n, Y.as<double>(), n, v,
                                c->stream);
        (void)hipEventRecord(e1, c->stream);
        (void)hipEventSynchronize(e1);
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        c->mm_ms[v] = ms / (2.0 * R);
        if (c->mm_ms[v] < c->mm_ms[best]) best = v;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(c, hipGetLastError());
    c->mm_variant = best;
    return TDBEM_OK;
}
}  // namespace

tdbem_status tdbem_assemble_tuning(tdbem_ctx* c, int32_t* tile_test, int32_t* tile_trial, double* ms)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    int tt = 0, ts = 0;
    if (c->tile_v >= 0 && (c->assembled || c->tile_forced)) tile_shape(c->tile_v, &tt, &ts);
    if (tile_test) *tile_test = tt;
    if (tile_trial) *tile_trial = ts;
    if (ms)
        for (int v = 0; v < tile_variants(); ++v) ms[v] = c->tile_ms[v];
    return TDBEM_OK;
}

tdbem_status tdbem_set_block_reuse(tdbem_ctx* c, int32_t enable)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (enable != 0 && enable != 1) FAIL(c, TDBEM_EINVAL, "block reuse must be 0 or 1, got %d", enable);
    c->reuse = enable == 1;
    return TDBEM_OK;
}

tdbem_status tdbem_assemble_set_tiles(tdbem_ctx* c, int32_t v, int32_t* nvariants)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (nvariants) *nvariants = tile_variants();
    if (v < -1 || v >= tile_variants()) FAIL(c, TDBEM_EINVAL, "tile shape %d outside -1..%d", v, tile_variants() - 1);
    c->tile_forced = v >= 0;
    c->tile_v = v;
    if (v < 0) c->tile_key = ~0ull;
    return TDBEM_OK;
}

tdbem_status tdbem_matvec_multi_tuning(tdbem_ctx* c, int32_t* rhs_per_pass, int32_t* staged_range,
                                       double* ms_per_rhs)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (!c->assembled) FAIL(c, TDBEM_ESTATE, "assemble before tuning the multi-vector product");
    TRY(set_device(c));
    TRY(multi_tune(c));
    if (rhs_per_pass) *rhs_per_pass = matvec_multi_variant_rc(c->mm_variant);
    if (staged_range) *staged_range = matvec_multi_variant_span(c->mm_variant);
    if (ms_per_rhs) *ms_per_rhs = c->mm_ms[c->mm_variant];
    return TDBEM_OK;
}

tdbem_status tdbem_matvec_multi_set_variant(tdbem_ctx* c, int32_t v, int32_t* nvariants)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    const int nv = matvec_multi_variants();
    if (nvariants) *nvariants = nv;
    if (v < -1 || v >= nv) FAIL(c, TDBEM_EINVAL, "variant %d outside -1..%d", v, nv - 1);
    c->mm_variant = v;
    if (v >= 0 && (int)c->mm_ms.size() != nv) c->mm_ms.assign(nv, 0.0);
    return TDBEM_OK;
}

tdbem_status tdbem_matvec_multi(tdbem_ctx* c, int32_t nrhs, const double* X, double* Y)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (!X || !Y) FAIL(c, TDBEM_EINVAL, "null array");
    if (nrhs < 1 || nrhs > 1024) FAIL(c, TDBEM_EINVAL, "need 1 <= nrhs <= 1024, got %d", nrhs);
    if (!c->assembled) FAIL(c, TDBEM_ESTATE, "assemble before the matvec");
    TRY(set_device(c));
    TRY(multi_tune(c));
    const int64_t n = (int64_t)c->N * c->M;
    launch_matvec_multi(c->band(), c->valf64(), c->valf32(), nrhs, X, n, Y, n, c->mm_variant, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return TDBEM_OK;
}

tdbem_status tdbem_solve_multi(tdbem_ctx* c, int32_t nrhs, const double* G, double* Alpha, const tdbem_solve_opts* o,
                               tdbem_solve_report* rep)
{
    if (!c) return TDBEM_EINVAL;
    c->err.clear();
    if (!G || !Alpha || !o) FAIL(c, TDBEM_EINVAL, "null argument");
    if (!c->assembled) FAIL(c, TDBEM_ESTATE, "assemble before solving");
    if (nrhs < 1 || nrhs > 1024) FAIL(c, TDBEM_EINVAL, "need 1 <= nrhs <= 1024, got %d", nrhs);
    if (o->restart < 1 || o->restart > 5000 || !(o->tol > 0.0) || o->max_it < 1)
        FAIL(c, TDBEM_EINVAL, "bad solver options");
    if (o->precond_levels != 0 || (o->precond_kind != 0 && o->precond_kind != 1))
        FAIL(c, TDBEM_EINVAL, "the batched solve takes no preconditioner or the learned one (precond_kind 1)");
    if (o->use_graph) FAIL(c, TDBEM_EINVAL, "the batched solve launches its kernels directly (use_graph 0)");
    TRY(set_device(c));
    const bool learned = o->precond_kind == 1;
    if (learned) {
        TRY(lp_need_params(c));
        TRY(lp_graph(c));
    }
    TRY(multi_tune(c));
    const int mv = c->mm_variant;
    const auto t_start = std::chrono::steady_clock::now();
    hipStream_t st = c->stream;
    const int64_t n = (int64_t)c->N * c->M;
    const int m = std::min(o->restart, o->max_it);
    const int R = nrhs;
    const int np = dots_partial_blocks(n);
    const int hw = 2 * (m + 1) + 2;                       // per right-hand side: h1, h2, |w|^2, spare
    DBuf V, Z, W, part, hb;
    ALLOC(c, V, sizeof(double) * (size_t)R * (m + 1) * n);
    ALLOC(c, Z, sizeof(double) * (size_t)R * m * n);
    ALLOC(c, W, sizeof(double) * (size_t)R * n);
    ALLOC(c, part, sizeof(double) * (size_t)R * (m + 2) * np);
    ALLOC(c, hb, sizeof(double) * (size_t)R * hw);
    double* Vd = V.as<double>();
    double* Zd = Z.as<double>();
    double* Wd = W.as<double>();
    double* Pd = part.as<double>();
    double* Hd = hb.as<double>();
    auto Vr = [&](int r, int q) { return Vd + ((int64_t)r * (m + 1) + q) * n; };
    auto Zr = [&](int r, int q) { return Zd + ((int64_t)r * m + q) * n; };
    auto Pr = [&](int r) { return Pd + (int64_t)r * (m + 2) * np; };
    auto Hr = [&](int r) { return Hd + (int64_t)r * hw; };
    std::vector<double> hhost((size_t)R * hw);
    auto fetch = [&]() -> tdbem_status {
        HIPCHK(c, hipMemcpyAsync(hhost.data(), Hd, sizeof(double) * hhost.size(), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        return TDBEM_OK;
    };
    // ||g_r||
    for (int r = 0; r < R; ++r) launch_dots(G + r * n, 1, n, n, G + r * n, Pr(r), Hr(r) + 2 * (m + 1), st);
    HIPCHK(c, hipGetLastError());
    TRY(fetch());
    std::vector<double> bnorm(R), beta(R);
    std::vector<int> its(R, 0);
    std::vector<char> live(R);
    for (int r = 0; r < R; ++r) {
        bnorm[r] = std::sqrt(hhost[(size_t)r * hw + 2 * (m + 1)]);
        beta[r] = bnorm[r];
        live[r] = bnorm[r] > 0.0;
        launch_fill(Alpha + r * n, 0.0, n, st);
    }
    std::vector<std::vector<double>> H(R, std::vector<double>((size_t)(m + 1) * m)), cs(R, std::vector<double>(m)),
        sn(R, std::vector<double>(m)), gv(R, std::vector<double>(m + 1));
    std::vector<int> jdone(R);
    std::vector<char> run(R);
    int64_t products = 0;
    bool first = true;
    while (true) {
        bool any = false;
        for (int r = 0; r < R; ++r) {
            run[r] = live[r] && its[r] < o->max_it && beta[r] > o->tol * bnorm[r];
            jdone[r] = 0;
            if (!run[r]) continue;
            any = true;
            // the residual of this cycle: g at the start, then W (computed below)
            launch_scale_copy(Vr(r, 0), first ? G + r * n : Wd + r * n, 1.0 / beta[r], n, st);
            std::fill(gv[r].begin(), gv[r].end(), 0.0);
            gv[r][0] = beta[r];
        }
        first = false;
        if (!any) break;
        for (int j = 0; j < m; ++j) {
            bool active = false;
            for (int r = 0; r < R; ++r) {
                if (!run[r]) continue;
                active = true;
                if (learned) TRY(lp_apply(c, Vr(r, j), Zr(r, j)));
                else launch_scale_copy(Zr(r, j), Vr(r, j), 1.0, n, st);
            }
            if (!active) break;
            // w_r = A z_r for every right-hand side (finished ones too: their columns are unused)
            launch_matvec_multi(c->band(), c->valf64(), c->valf32(), R, Zd + (int64_t)j * n, (int64_t)m * n,
                                Vd + (int64_t)(j + 1) * n, (int64_t)(m + 1) * n, mv, st);
            HIPCHK(c, hipGetLastError());
            ++products;
            for (int r = 0; r < R; ++r) {
                if (!run[r]) continue;
                double* w = Vr(r, j + 1);
                double* h = Hr(r);
                launch_dots(Vr(r, 0), j + 1, n, n, w, Pr(r), h, st);
                launch_sub_combination(w, Vr(r, 0), j + 1, n, n, h, -1.0, st);
                launch_dots(Vr(r, 0), j + 1, n, n, w, Pr(r), h + (m + 1), st);
                launch_sub_combination(w, Vr(r, 0), j + 1, n, n, h + (m + 1), -1.0, st);
                launch_dots(w, 1, n, n, w, Pr(r), h + 2 * (m + 1), st);
                launch_scale_inv_sqrt(w, w, h + 2 * (m + 1), n, st);
            }
            HIPCHK(c, hipGetLastError());
            TRY(fetch());
            for (int r = 0; r < R; ++r) {
                if (!run[r]) continue;
                const double* hh = hhost.data() + (size_t)r * hw;
                std::vector<double>& Hm = H[r];
                for (int q = 0; q <= j; ++q) Hm[(size_t)q * m + j] = hh[q] + hh[m + 1 + q];
                const double hn = std::sqrt(std::max(hh[2 * (m + 1)], 0.0));
                Hm[(size_t)(j + 1) * m + j] = hn;
                for (int q = 0; q < j; ++q) {
                    const double t1 = cs[r][q] * Hm[(size_t)q * m + j] + sn[r][q] * Hm[(size_t)(q + 1) * m + j];
                    Hm[(size_t)(q + 1) * m + j] = -sn[r][q] * Hm[(size_t)q * m + j] + cs[r][q] * Hm[(size_t)(q + 1) * m + j];
                    Hm[(size_t)q * m + j] = t1;
                }
                const double den = std::hypot(Hm[(size_t)j * m + j], Hm[(size_t)(j + 1) * m + j]);
                cs[r][j] = den != 0.0 ? Hm[(size_t)j * m + j] / den : 1.0;
                sn[r][j] = den != 0.0 ? Hm[(size_t)(j + 1) * m + j] / den : 0.0;
                Hm[(size_t)j * m + j] = cs[r][j] * Hm[(size_t)j * m + j] + sn[r][j] * Hm[(size_t)(j + 1) * m + j];
                Hm[(size_t)(j + 1) * m + j] = 0.0;
                gv[r][j + 1] = -sn[r][j] * gv[r][j];
                gv[r][j] = cs[r][j] * gv[r][j];
                ++its[r];
                jdone[r] = j + 1;
                if (std::fabs(gv[r][j + 1]) <= o->tol * bnorm[r] || hn == 0.0 || its[r] >= o->max_it) run[r] = 0;
            }
            if (o->progress) {
                double worst = 0.0;
                for (int r = 0; r < R; ++r)
                    if (live[r] && jdone[r] == j + 1) worst = std::max(worst, std::fabs(gv[r][j + 1]) / bnorm[r]);
                o->progress(j + 1, worst, o->progress_user);
            }
        }
        // x_r += Z_r y_r, y_r = H_r^{-1} g_r
        for (int r = 0; r < R; ++r) {
            const int jd = jdone[r];
            if (jd == 0) continue;
            std::vector<double> y(jd);
            for (int q = jd - 1; q >= 0; --q) {
                double s = gv[r][q];
                for (int u = q + 1; u < jd; ++u) s -= H[r][(size_t)q * m + u] * y[u];
                y[q] = s / H[r][(size_t)q * m + q];
            }
            HIPCHK(c, hipMemcpyAsync(Hr(r), y.data(), sizeof(double) * jd, hipMemcpyHostToDevice, st));
            launch_sub_combination(Alpha + r * n, Zr(r, 0), jd, n, n, Hr(r), 1.0, st);
        }
        // true residuals W_r = g_r - A alpha_r
        launch_matvec_multi(c->band(), c->valf64(), c->valf32(), R, Alpha, n, Wd, n, mv, st);
        ++products;
        for (int r = 0; r < R; ++r) {
            launch_axpby(Wd + r * n, G + r * n, 1.0, -1.0, n, st);
            launch_dots(Wd + r * n, 1, n, n, Wd + r * n, Pr(r), Hr(r) + 2 * (m + 1), st);
        }
        HIPCHK(c, hipGetLastError());
        TRY(fetch());
        for (int r = 0; r < R; ++r) beta[r] = std::sqrt(std::max(hhost[(size_t)r * hw + 2 * (m + 1)], 0.0));
    }
    HIPCHK(c, hipStreamSynchronize(st));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    bool all = true;
    for (int r = 0; r < R; ++r) {
        const double rel = bnorm[r] > 0.0 ? beta[r] / bnorm[r] : 0.0;
        all = all && rel <= o->tol;
        if (rep) {
            rep[r].iterations = its[r];
            rep[r].matvecs = products;
            rep[r].rel_residual = rel;
            rep[r].ms = ms;
        }
    }
    if (!all) {
        c->err = "not converged: some right-hand sides are above tol after max_it iterations";
        return TDBEM_NOT_CONVERGED;
    }
    return TDBEM_OK;
}

}  // extern "C"
