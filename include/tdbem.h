/*
 * tdbem.h -- C ABI of the MI355X (gfx950) space-time Galerkin solver for the sound-hard
 * time-domain boundary integral equation of Veit, Merta, Zapletal and Lukas
 * (arXiv:1503.07221).
 *
 * The library assembles the block-Hessenberg system A alpha = g of the space-time Galerkin
 * discretisation of the hypersingular equation W phi = g (Section 2, eqs. (BIE) and
 * (VarForm)) with P1 hats phi_j on flat triangles and one smooth, compactly supported
 * temporal basis b_i per time node (Section 3, eq. (BasisFunctions) with p = 0), and solves it
 * with FGMRES and the recursive block-Hessenberg preconditioner of Section 4.2 (Algorithm 1).
 *
 * Conventions
 *   - Every call returns a tdbem_status; 0 is success, negative values are errors, positive
 *     values are warnings.  Errors never abort: the message is kept and returned by
 *     tdbem_last_error() until the next call on the same context.
 *   - Host arrays passed in are copied; the caller keeps ownership.
 *   - Device pointers (vectors of the solve and the matvec) belong to the caller, must live in
 *     device memory of the context's device and are used in place on the context's stream.
 *   - Vectors follow the block partition of eq. (A): x[i*M + j] multiplies b_i(t) phi_j(x);
 *     row (k, l) of the system is y[k*M + l].  Indices are 0-based.
 *   - A_{k,i}(j, l) is the entry of eq. (MatrixEntries): test functions (b_k, phi_l) in the
 *     x variable, trial functions (b_i, phi_j) in the y variable.
 *   - One context per host thread; calls on one context are not thread safe.
 */
#ifndef TDBEM_H
#define TDBEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tdbem_ctx tdbem_ctx;

typedef enum {
    TDBEM_OK = 0,
    TDBEM_NOT_CONVERGED = 1,     /* warning: the solve stopped at max_it above tol */
    TDBEM_EINVAL = -1,           /* invalid argument (null pointer, bad size or option) */
    TDBEM_EMESH = -2,            /* mesh rejected (bad index, degenerate triangle) */
    TDBEM_EGRID = -3,            /* time grid rejected (t_0 != 0, not increasing, N < 2) */
    TDBEM_ENOMEM = -4,           /* device allocation failed or the matrix exceeds the limit */
    TDBEM_EHIP = -5,             /* HIP runtime error */
    TDBEM_ESTATE = -6            /* call out of order (e.g. matvec before assemble) */
} tdbem_status;

typedef enum {
    TDBEM_CUTOFF_BUMP = 0,       /* F(u) = beta(u-1)/(beta(u-1)+beta(u)), beta = exp(-1/(1-s^2)) */
    TDBEM_CUTOFF_ERF = 1         /* the paper's f(s) = erf(2 artanh s)/2 + 1/2, F(u) = f(2u-1) */
} tdbem_cutoff;

typedef enum {
    TDBEM_FP64 = 0,              /* FP64 quadrature and FP64 matrix storage */
    TDBEM_MIXED = 1              /* FP32 matrix storage (every sum formed in FP64, rounded once);
                                    FP64 tables and solver vectors */
} tdbem_precision;

typedef struct {
    int32_t device;              /* HIP device ordinal */
    void *stream;                /* hipStream_t to run on; NULL: the library creates one */
    int32_t ss_order;            /* Gauss points per direction of the Sauter-Schwab rules, 1..5
                                    (<= 0: 4); larger values give TDBEM_EINVAL */
    int32_t deterministic;       /* 1: every assembly gives bitwise the same matrix on every run
                                    (TDBEM_FP64 only).  The contributions are added as 64-bit
                                    fixed-point integers, whose sums do not depend on the order of
                                    the atomic additions; the scale, a power of two that keeps every
                                    entry below 2^61, comes from a first ordinary pass, so the
                                    assembly takes about twice as long.  Entries differ from the
                                    ordinary assembly by ~1e-16 of the largest.  0: ordinary FP64
                                    atomics (order-dependent in the last bits).  Others: EINVAL */
    int32_t quad_regular;        /* points of the rule on each triangle of a regular pair: 7 (the
                                    degree-5 rule) or 0 for it; other values TDBEM_EINVAL */
    double psi_tol;              /* accuracy asked of the psi tables relative to each kernel's
                                    maximum: 0 (the built-in tables, ~2e-12) or >= 2e-12; a smaller
                                    value cannot be met and gives TDBEM_EINVAL */
} tdbem_options;

typedef struct {
    int64_t quad_evals;          /* (x_q, y_q', k, i) with r inside supp psi_{k,i}, unordered pairs */
    int64_t pairs_regular;       /* unordered triangle pairs without a common vertex */
    int64_t pairs_coincident, pairs_edge, pairs_vertex;
    int64_t table_functions;     /* (k, i) kernels tabulated */
    int64_t bytes_matrix;        /* device bytes of the assembled blocks */
    double ms_tables, ms_layout, ms_regular, ms_singular, ms_total;
    int64_t quad_evals_regular;  /* the part of quad_evals computed by the regular-pair kernel */
    int64_t blocks_reused;       /* nonzero time blocks A_{k,i} (temporal bases k, i) copied from an
                                    equal block instead of integrated (equidistant grids, eq.
                                    (relationAtildeBlock)); quad_evals counts only the integrated
                                    ones.  0 on other grids and with reuse off */
    double ms_reuse;             /* time of those copies (part of ms_total) */
} tdbem_assembly_report;

typedef struct {
    int32_t restart;             /* Krylov dimension between restarts (30) */
    double tol;                  /* relative residual ||g - A alpha|| / ||g|| to reach (1e-8) */
    int32_t max_it;              /* outer iteration limit */
    int32_t precond_levels;      /* 0: none; r > 0: Algorithm 1 with r recursion levels */
    int32_t precond_inner[8];    /* inner FGMRES iterations on each level, e.g. {2, 10} */
    /* optional: called on the calling thread after every outer iteration with the iteration
     * number and the Givens estimate of the relative residual (NULL: no calls) */
    void (*progress)(int32_t iteration, double estimate, void *user);
    void *progress_user;         /* passed to progress unchanged */
    /* preconditioner of the outer iteration: 0 = Algorithm 1 as set by precond_levels (none
     * when 0); 1 = the learned network of tdbem_learned.h (must be initialised); 2 = the learned
     * network during the first restart cycle, then Algorithm 1 (precond_levels > 0) from the
     * iterate reached, the paper's preconditioner serving as the fallback; 3 = DGMRES(restart,
     * deflation_l) of Section 4.1: the deflation M^{-1} = I + U (|lambda_max| T^{-1} - I) U^T,
     * T = U^T A U, where after every restart the eigenvectors of the cycle's Hessenberg matrix for
     * its deflation_l smallest eigenvalues (mapped back through the Krylov basis) are added to U,
     * up to deflation_max columns (precond_levels must be 0) */
    int32_t precond_kind;
    /* 1: with the learned network, run each outer iteration's preconditioned operator
     * (z = P(v), w = A z) as one captured HIP graph, replayed on the context's stream; 0: launch
     * the kernels one by one.  Requires precond_kind 1 or 2. */
    int32_t use_graph;
    int32_t deflation_l;         /* DGMRES: vectors added to U after each restart (precond_kind 3) */
    int32_t deflation_max;       /* DGMRES: largest dimension of U, <= 256 (precond_kind 3); U and
                                    A U take 2 deflation_max N M float64 of device memory */
    /* 1: the products inside Algorithm 1 (its inner FGMRES solves and the coupling block) read an
     * FP32 copy of the FP64 band (made once per assembly, half the bytes of the band), while the
     * outer iteration and its true residual keep the FP64 operator, so the solve still reaches tol
     * on the FP64 system (FGMRES accepts the inexact preconditioner).  Needs an FP64 assembly and
     * precond_levels > 0. */
    int32_t inner_fp32;
} tdbem_solve_opts;

typedef struct {
    int32_t iterations;          /* outer FGMRES iterations */
    int64_t matvecs;             /* block-operator products of any size, outer and inner */
    double rel_residual;         /* true ||g - A alpha|| / ||g|| at return */
    double ms;                   /* wall time of the solve */
} tdbem_solve_report;

/* Create a context on opt->device (opt may be NULL: device 0, own stream, ss_order 4). */
tdbem_status tdbem_create(tdbem_ctx **out, const tdbem_options *opt);

/* Release everything the context owns.  NULL is accepted. */
void tdbem_destroy(tdbem_ctx *ctx);

/* Message of the last error on ctx ("" if none); valid until the next call on ctx. */
const char *tdbem_last_error(const tdbem_ctx *ctx);

/* Surface mesh Gamma (Section 3): M vertices xyz[3*v + c] (host, float64) and E flat
 * triangles tri[3*e + a] (host, int32, 0-based, counter-clockwise seen from the side the
 * normal n of eq. (FullProblem) points to).  Resets any assembled matrix.
 * TDBEM_EMESH for an index out of range, a repeated vertex in a triangle or a zero area. */
tdbem_status tdbem_set_mesh(tdbem_ctx *ctx, const double *xyz, int64_t M, const int32_t *tri, int64_t E);

/* Time grid 0 = t_0 < t_1 < ... < t_{N-1} = T (host, float64) and temporal order p (Section 3,
 * eq. (BasisFunctions): p + 1 bases per node, the node's bump mu_n times the Legendre
 * polynomials P_0..P_p of the node's support mapped to [-1, 1], b_0 with the causal factor
 * 8 (t/h_1)^2; L = N (p + 1) temporal bases, basis n (p + 1) + m).  Resets any assembled matrix.
 * TDBEM_EINVAL unless 0 <= p <= 4 and N (p + 1) <= 8192; TDBEM_EGRID unless 2 <= N <= 4096,
 * t_0 = 0 and t strictly increasing. */
tdbem_status tdbem_set_time_grid(tdbem_ctx *ctx, const double *t, int32_t N, tdbem_cutoff cutoff, int32_t p);

/* Assemble every block A_{k,i} of eq. (MatrixEntries) on the device (Section 3): kernels
 * psi_{k,i}, tilde psi_{k,i} of eq. (psis) tabulated as piecewise Chebyshev series
 * (Section 3.1), 7-point rule for pairs without a common vertex, Sauter-Schwab rules for
 * coincident, edge and vertex pairs, entries kept where supp psi_{k,i} meets the distance
 * range of the two hats (eq. (SparsitySmallBlock)).  On an equidistant grid the blocks that equal
 * another one (eq. (relationAtildeBlock)) are copied, not integrated (tdbem_set_block_reuse); with
 * tdbem_options.deterministic the storage is bitwise reproducible.  rep may be NULL.
 * TDBEM_ESTATE without mesh and grid, TDBEM_ENOMEM if the storage does not fit, TDBEM_EINVAL for
 * TDBEM_MIXED in the deterministic mode. */
tdbem_status tdbem_assemble(tdbem_ctx *ctx, tdbem_precision prec, tdbem_assembly_report *rep);

/* The regular-pair kernel is compiled for two tile shapes (test x trial triangles per workgroup:
 * 4 x 8 on 256 lanes, 8 x 8 on 512).  At the first assembly of a mesh and time grid the library
 * times each shape on every 32nd tile, keeps the faster for that mesh and grid, and zeroes the
 * storage again (the timing is part of that assembly's layout time).  This call reports the
 * shape in use (0 x 0 before any assembly) and, through ms[0..1] when ms is not NULL, each
 * shape's timed estimate for the whole launch (-1 if not timed).  Any pointer may be NULL. */
tdbem_status tdbem_assemble_tuning(tdbem_ctx *ctx, int32_t *tile_test, int32_t *tile_trial, double *ms);

/* Use tile shape v (0: 4 x 8, 1: 8 x 8; the count goes to nvariants when not NULL) for every later
 * assembly instead of the timed choice; v = -1 returns to timing.  TDBEM_EINVAL for another v. */
tdbem_status tdbem_assemble_set_tiles(tdbem_ctx *ctx, int32_t v, int32_t *nvariants);

/* Equal blocks (eq. (relationAtildeBlock), Section 5.1).  On an equidistant grid (every
 * |t_n - n T / (N - 1)| <= 1e-12 T) the bases of the inner nodes 1..N-2 are translates, so the
 * node block of inner nodes (k, i) with 2 <= i <= k equals block (k - i + 1, 1) and the
 * superdiagonal block (k, k + 1), k >= 2, equals (1, 2).  With enable = 1 (the default) such an
 * assembly integrates only the first two block columns, the last block row and the blocks (1, 2),
 * (N - 2, N - 1), and copies the stored values of the others (O(N) instead of O(N^2) blocks
 * integrated; the report's blocks_reused counts the copies).  enable = 0 integrates every
 * block.  Takes effect at the next tdbem_assemble; no effect on other grids or on
 * tdbem_matvec_free.  TDBEM_EINVAL unless enable is 0 or 1. */
tdbem_status tdbem_set_block_reuse(tdbem_ctx *ctx, int32_t enable);

/* Assemble the problems of n distinct contexts (meshes, grids and orders of any sizes, all on one
 * device) together, batching many small problems (Section 3 for each).  One host thread per
 * context builds its tables and layout on its own stream; then the regular pairs of all problems
 * run in ONE launch on the first context's stream (the tiles of the larger problems first, 4 x 8
 * tiles), and each context finishes (singular pairs, equal-block copies, counts) on its stream.
 * Every context then holds the same matrix as after tdbem_assemble; each report's ms_regular
 * spans from the end of that context's layout to the end of the shared launch.  reps: NULL or an array of n reports.  Returns the first
 * non-OK status in context order (its message is in that context); TDBEM_EINVAL for a NULL
 * context, n outside 1..256, a context listed twice, contexts on different devices or a mesh of
 * 2^24 triangles or more. */
tdbem_status tdbem_assemble_group(tdbem_ctx *const *ctxs, int32_t n, tdbem_precision prec,
                                  tdbem_assembly_report *reps);

/* Copy selected entries to the host: out[s] = A_{k[s], i[s]}(j[s], l[s]) for s < n (host
 * arrays).  Entries outside the stored band are zero by eq. (SparsitySmallBlock). */
tdbem_status tdbem_get_entries(tdbem_ctx *ctx, int64_t n, const int32_t *k, const int32_t *i,
                               const int32_t *j, const int32_t *l, double *out);

/* tdbem_get_entries for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same entries, staged through a
 * statically allocated device array instead of allocations made per call.  At most 65536 entries
 * per call (TDBEM_EINVAL beyond); no hipMalloc or hipFree.  Every context on one device shares
 * that device's array, so calls that overlap on one device (several host threads or streams)
 * race; the array keeps the last call's contents.  Host arrays as in tdbem_get_entries. */
tdbem_status tdbem_get_entries_noalloc(tdbem_ctx *ctx, int64_t n, const int32_t *k, const int32_t *i,
                                       const int32_t *j, const int32_t *l, double *out);

/* Number of entries of the assembled block A_{k,i} (the sparse blocks of eq. (Apartitioned), with
 * the pattern of eq. (SparsitySmallBlock)): the non-zero values of the stored band, counted in
 * both triangles (an off-diagonal vertex pair counts twice, the blocks being symmetric).  Written
 * to *nnz (host).  Requires tdbem_assemble; TDBEM_EINVAL for k or i outside 0..N-1. */
tdbem_status tdbem_block_nnz(tdbem_ctx *ctx, int32_t k, int32_t i, int64_t *nnz);

/* The block A_{k,i} in coordinate form (host arrays owned by the caller, cap entries each):
 * row[s] = l (test vertex), col[s] = j (trial vertex), val[s] = A_{k,i}(j, l) for the
 * tdbem_block_nnz(ctx, k, i) entries, sorted by (row, column).  Values are float64 also after a
 * mixed-precision assembly (the stored FP32 values, widened).  TDBEM_EINVAL if cap is smaller than
 * the entry count (the message gives it); nothing is written then. */
tdbem_status tdbem_get_block_coo(tdbem_ctx *ctx, int32_t k, int32_t i, int32_t *row, int32_t *col, double *val,
                                 int64_t cap);

/* Evaluate the tabulated time kernels used by the assembly: psi[s] = psi_{k[s],i[s]}(r[s]) and
 * tpsi[s] = tilde psi_{k[s],i[s]}(r[s]) of eq. (psis) for n host points (host arrays), 0 outside
 * the open support (Section 3.2).  Requires a completed tdbem_assemble. */
tdbem_status tdbem_eval_kernels(tdbem_ctx *ctx, int64_t n, const int32_t *k, const int32_t *i,
                                const double *r, double *psi, double *tpsi);

/* Right-hand side g_k(l) = int_0^T int_Gamma g phi_l b_k' (Section 3) of the plane Gaussian
 * pulse u_inc = exp(-((t - t0 - d.x)/width)^2), g = -d u_inc/d n, written to the device
 * vector g (N*M float64).  d is the propagation direction, a host array of 3 doubles used as
 * given (a unit vector for a plane wave of speed 1). */
tdbem_status tdbem_rhs_plane_pulse(tdbem_ctx *ctx, const double d[3], double t0, double width, double *g);

/* y = A x for device vectors x, y of N*M float64 (the block matvec of Section 3.2). */
tdbem_status tdbem_matvec(tdbem_ctx *ctx, const double *x, double *y);

/* y = A[k0:k1, i0:i1] x for the time-block sub-operator: x holds blocks i0..i1-1
 * ((i1-i0)*M values), y receives blocks k0..k1-1 ((k1-k0)*M values).  Used by Algorithm 1. */
tdbem_status tdbem_matvec_range(tdbem_ctx *ctx, int32_t k0, int32_t k1, int32_t i0, int32_t i1,
                                const double *x, double *y);

/* y = A x in FP64 without storing A, for operators whose band storage does not fit the device:
 * the regular and singular quadrature of eq. (MatrixEntries) runs again and every local block
 * is applied to x as it is formed (its entries with their block-symmetric mirrors, Section 3.2).
 * x, y: device vectors of N*M float64 (y is overwritten).  Needs the mesh and the time grid (no
 * assembly); costs about one assembly.  rep (may be NULL) receives the quadrature counts and
 * times (bytes_matrix = 0). */
tdbem_status tdbem_matvec_free(tdbem_ctx *ctx, const double *x, double *y, tdbem_assembly_report *rep);

/* Solve A alpha = g (device vectors, N*M float64) with FGMRES(restart) (Saad 1993) from
 * alpha = 0, right-preconditioned by Algorithm 1 when opts->precond_levels > 0.  On return
 * alpha holds the iterate; TDBEM_NOT_CONVERGED if the true relative residual is above tol
 * after max_it outer iterations.  rep may be NULL. */
tdbem_status tdbem_solve(tdbem_ctx *ctx, const double *g, double *alpha, const tdbem_solve_opts *opts,
                         tdbem_solve_report *rep);

/* The scattered field off the surface: the retarded double layer potential of eq.
 * (RetardedPotential) of the density phi(y, t) = sum_i sum_j alpha[i*M + j] b_i(t) phi_j(y),
 *   u(x, t) = -1/(4 pi) int_Gamma (n_y.(x - y))/r (phi(y, t - r)/r^2 + d_t phi(y, t - r)/r) dGamma_y,
 * r = |x - y|, with the 7-point rule on every triangle.  alpha: device vector of N*M float64 (e.g.
 * the solution of tdbem_solve); pts: host array of 3*npts coordinates (points off Gamma); times:
 * host array of ntimes values in [0, T]; u: device array of ntimes*npts float64, u[s*npts + p].
 * Needs the mesh and the grid (no assembly).  TDBEM_EINVAL for a time outside [0, T] or more than
 * 1024 time nodes. */
tdbem_status tdbem_potential_dl(tdbem_ctx *ctx, const double *alpha, int64_t npts, const double *pts,
                                int32_t ntimes, const double *times, double *u);

/* Y_r = A X_r for nrhs right-hand sides at once (the block matvec of Section 3.2; every stored
 * value is read once per group of right-hand sides, see tdbem_matvec_multi_tuning): X, Y device
 * arrays of nrhs*N*M float64, vector r at offset r*N*M.  1 <= nrhs <= 1024.  Requires tdbem_assemble. */
tdbem_status tdbem_matvec_multi(tdbem_ctx *ctx, int32_t nrhs, const double *X, double *Y);

/* The multi-vector product has kernel variants (right-hand sides per pass, trial range staged in
 * LDS); on its first use after an assembly the library times each on 8 vectors of the assembled
 * operator and keeps the fastest.  This call runs that tuning if needed and reports the choice
 * and its time per right-hand side in ms (any output pointer may be NULL). */
tdbem_status tdbem_matvec_multi_tuning(tdbem_ctx *ctx, int32_t *rhs_per_pass, int32_t *staged_range,
                                       double *ms_per_rhs);

/* Use variant v (0 <= v < the number of variants, which the call returns through nvariants when
 * not NULL) of the multi-vector product until the next assembly instead of the timed choice;
 * v = -1 returns to timing.  TDBEM_EINVAL for another v. */
tdbem_status tdbem_matvec_multi_set_variant(tdbem_ctx *ctx, int32_t v, int32_t *nvariants);

/* Solve A alpha_r = g_r for nrhs right-hand sides together: FGMRES(restart) from alpha_r = 0 on
 * every right-hand side with its own Krylov basis, sharing one multi-right-hand-side product per
 * iteration (tdbem_matvec_multi).  G, Alpha: device arrays of nrhs*N*M float64 (vector r at
 * offset r*N*M).  Preconditioner: none (precond_kind 0, precond_levels 0) or the learned network
 * of tdbem_learned.h (precond_kind 1); Algorithm 1 is not batched (TDBEM_EINVAL).  progress, if
 * set, receives the iteration and the largest estimate over the right-hand sides still
 * iterating.  rep (may be NULL) is an array of nrhs reports (matvecs = multi-products, ms = the
 * whole batch).  Needs nrhs*(2*restart+2)*N*M*8 bytes of device workspace.  TDBEM_NOT_CONVERGED
 * if any right-hand side ends above tol. */
tdbem_status tdbem_solve_multi(tdbem_ctx *ctx, int32_t nrhs, const double *G, double *Alpha,
                               const tdbem_solve_opts *opts, tdbem_solve_report *rep);

#ifdef __cplusplus
}
#endif

#endif /* TDBEM_H */
