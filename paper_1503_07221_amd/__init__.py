"""Python binding of libtdbem, the MI355X space-time Galerkin TDBIE library (arXiv:1503.07221).

Argument marshalling only: every step of the method runs in the HIP kernels of
``csrc/`` behind the C ABI of ``include/tdbem.h``.  PyTorch provides device memory and the
stream; there is no CPU fallback, and a missing or unloadable library raises at import of the
context.

The learned variable preconditioner of ``include/tdbem_learned.h`` (a message-passing network
trained on the GPU by the library's own kernels) is reached through the ``lp_*`` methods.

Vector layout (eq. (A) block partition): ``x[i*M + j]`` multiplies ``b_i(t) phi_j(x)``.
"""
import ctypes
import os

import numpy as np

from .build import LIB_PATH, build_library

__all__ = ["Context", "TdbemError", "assemble_group", "load_library", "build_library", "LIB_PATH", "EXPORTED_SYMBOLS",
           "FP64", "MIXED", "CUTOFF_BUMP", "CUTOFF_ERF", "PRECOND_ALG1", "PRECOND_LEARNED",
           "PRECOND_LEARNED_THEN_ALG1", "PRECOND_DEFLATION"]

FP64, MIXED = 0, 1
CUTOFF_BUMP, CUTOFF_ERF = 0, 1
STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "EINVAL", -2: "EMESH", -3: "EGRID", -4: "ENOMEM", -5: "EHIP",
          -6: "ESTATE"}

EXPORTED_SYMBOLS = ["tdbem_create", "tdbem_destroy", "tdbem_last_error", "tdbem_set_mesh", "tdbem_set_time_grid",
                    "tdbem_assemble", "tdbem_get_entries", "tdbem_get_entries_noalloc", "tdbem_block_nnz", "tdbem_get_block_coo", "tdbem_eval_kernels", "tdbem_rhs_plane_pulse",
                    "tdbem_matvec", "tdbem_matvec_range", "tdbem_matvec_free", "tdbem_solve",
                    "tdbem_matvec_multi", "tdbem_solve_multi", "tdbem_potential_dl",
                    "tdbem_matvec_multi_tuning", "tdbem_matvec_multi_set_variant", "tdbem_assemble_group",
                    "tdbem_lp_num_params", "tdbem_lp_init", "tdbem_lp_set_params", "tdbem_lp_get_params",
                    "tdbem_lp_apply", "tdbem_lp_gradient", "tdbem_matvec_transpose", "tdbem_lp_train",
                    "tdbem_lp_make_pairs", "tdbem_lp_train_pairs", "tdbem_assemble_tuning", "tdbem_assemble_set_tiles",
                    "tdbem_set_block_reuse"]

# preconditioner kinds of SolveOpts.precond_kind
PRECOND_ALG1, PRECOND_LEARNED, PRECOND_LEARNED_THEN_ALG1, PRECOND_DEFLATION = 0, 1, 2, 3


class TdbemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tdbem {STATUS.get(status, status)}: {msg}")
        self.status = status


class _Options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("stream", ctypes.c_void_p), ("ss_order", ctypes.c_int32),
                ("deterministic", ctypes.c_int32), ("quad_regular", ctypes.c_int32), ("psi_tol", ctypes.c_double)]


class AssemblyReport(ctypes.Structure):
    _fields_ = [("quad_evals", ctypes.c_int64), ("pairs_regular", ctypes.c_int64),
                ("pairs_coincident", ctypes.c_int64), ("pairs_edge", ctypes.c_int64),
                ("pairs_vertex", ctypes.c_int64), ("table_functions", ctypes.c_int64),
                ("bytes_matrix", ctypes.c_int64), ("ms_tables", ctypes.c_double), ("ms_layout", ctypes.c_double),
                ("ms_regular", ctypes.c_double), ("ms_singular", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("quad_evals_regular", ctypes.c_int64), ("blocks_reused", ctypes.c_int64),
                ("ms_reuse", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


PROGRESS = ctypes.CFUNCTYPE(None, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p)


class SolveOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int32), ("tol", ctypes.c_double), ("max_it", ctypes.c_int32),
                ("precond_levels", ctypes.c_int32), ("precond_inner", ctypes.c_int32 * 8),
                ("progress", PROGRESS), ("progress_user", ctypes.c_void_p), ("precond_kind", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("deflation_l", ctypes.c_int32), ("deflation_max", ctypes.c_int32),
                ("inner_fp32", ctypes.c_int32)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class TrainReport(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("samples", ctypes.c_int64), ("loss_first", ctypes.c_double),
                ("loss_last", ctypes.c_double), ("ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class SolveReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("matvecs", ctypes.c_int64), ("rel_residual", ctypes.c_double),
                ("ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load_library(path=LIB_PATH):
    """Load libtdbem.so (built in-tree by build_library())."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch ships its own HIP runtime; loading it first makes libtdbem resolve to the same
    # runtime (one HIP runtime per process), so that torch's device memory and streams are valid
    # handles for the library.
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise ImportError(f"libtdbem.so not found at {path}; run __graft_entry__.build() first")
    L = ctypes.CDLL(path)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    L.tdbem_create.argtypes = [P(vp), P(_Options)]
    L.tdbem_destroy.argtypes = [vp]
    L.tdbem_destroy.restype = None
    L.tdbem_last_error.argtypes = [vp]
    L.tdbem_last_error.restype = ctypes.c_char_p
    L.tdbem_set_mesh.argtypes = [vp, P(dp), i64, P(i32), i64]
    L.tdbem_set_time_grid.argtypes = [vp, P(dp), i32, ctypes.c_int, i32]
    L.tdbem_block_nnz.argtypes = [vp, i32, i32, P(i64)]
    L.tdbem_get_block_coo.argtypes = [vp, i32, i32, P(i32), P(i32), P(dp), i64]
    L.tdbem_assemble.argtypes = [vp, ctypes.c_int, P(AssemblyReport)]
    L.tdbem_get_entries.argtypes = [vp, i64, P(i32), P(i32), P(i32), P(i32), P(dp)]
    L.tdbem_get_entries_noalloc.argtypes = [vp, i64, P(i32), P(i32), P(i32), P(i32), P(dp)]
    L.tdbem_eval_kernels.argtypes = [vp, i64, P(i32), P(i32), P(dp), P(dp), P(dp)]
    L.tdbem_rhs_plane_pulse.argtypes = [vp, P(dp), dp, dp, vp]
    L.tdbem_matvec.argtypes = [vp, vp, vp]
    L.tdbem_matvec_range.argtypes = [vp, i32, i32, i32, i32, vp, vp]
    L.tdbem_matvec_free.argtypes = [vp, vp, vp, P(AssemblyReport)]
    L.tdbem_solve.argtypes = [vp, vp, vp, P(SolveOpts), P(SolveReport)]
    L.tdbem_matvec_multi.argtypes = [vp, i32, vp, vp]
    L.tdbem_assemble_group.argtypes = [P(vp), i32, ctypes.c_int, P(AssemblyReport)]
    L.tdbem_matvec_multi_tuning.argtypes = [vp, P(i32), P(i32), P(dp)]
    L.tdbem_matvec_multi_set_variant.argtypes = [vp, i32, P(i32)]
    L.tdbem_potential_dl.argtypes = [vp, vp, i64, P(dp), i32, P(dp), vp]
    L.tdbem_solve_multi.argtypes = [vp, i32, vp, vp, P(SolveOpts), P(SolveReport)]
    fp = P(ctypes.c_float)
    L.tdbem_lp_num_params.argtypes = [i32]
    L.tdbem_lp_num_params.restype = i64
    L.tdbem_lp_init.argtypes = [vp, i32, ctypes.c_uint64]
    L.tdbem_lp_set_params.argtypes = [vp, fp, i64]
    L.tdbem_lp_get_params.argtypes = [vp, fp, i64]
    L.tdbem_lp_apply.argtypes = [vp, vp, vp]
    L.tdbem_lp_gradient.argtypes = [vp, vp, vp, vp, fp]
    L.tdbem_matvec_transpose.argtypes = [vp, vp, vp]
    L.tdbem_lp_train.argtypes = [vp, P(TrainOpts), fp, P(TrainReport)]
    L.tdbem_lp_make_pairs.argtypes = [vp, i64, ctypes.c_uint64, vp, vp]
    L.tdbem_assemble_tuning.argtypes = [vp, P(i32), P(i32), P(dp)]
    L.tdbem_assemble_set_tiles.argtypes = [vp, i32, P(i32)]
    L.tdbem_set_block_reuse.argtypes = [vp, i32]
    L.tdbem_lp_train_pairs.argtypes = [vp, vp, vp, vp, i64, P(TrainOpts), fp, P(TrainReport)]
    for name in EXPORTED_SYMBOLS:
        if name not in ("tdbem_destroy", "tdbem_last_error", "tdbem_lp_num_params"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def assemble_group(contexts, precision=FP64):
    """Assemble the problems of several contexts together (their regular pairs in one launch);
    returns the list of assembly reports."""
    lib = load_library()
    n = len(contexts)
    hs = (ctypes.c_void_p * n)(*[c.h for c in contexts])
    reps = (AssemblyReport * n)()
    st = lib.tdbem_assemble_group(hs, n, int(precision), reps)
    if st != 0:
        msgs = [c.lib.tdbem_last_error(c.h).decode() for c in contexts]
        raise TdbemError(st, "; ".join(m for m in msgs if m) or "group assembly failed")
    return [r.as_dict() for r in reps]


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class Context:
    """One library context on a HIP device, running on torch's current stream of that device."""

    def __init__(self, device=0, ss_order=4, own_stream=False, deterministic=False):
        """own_stream: run on a new stream of default priority (contexts assembled together with
        assemble_group overlap only on distinct streams) instead of torch's current stream.
        deterministic: assemblies give bitwise the same matrix on every run (FP64 only)."""
        import torch
        self.torch = torch
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("tdbem needs a HIP device (torch.cuda.is_available() is False)")
        self.device = torch.device("cuda", device)
        self.stream = torch.cuda.Stream(self.device) if own_stream else torch.cuda.current_stream(self.device)
        opt = _Options(device, ctypes.c_void_p(self.stream.cuda_stream), ss_order, 1 if deterministic else 0, 7, 0.0)
        h = ctypes.c_void_p()
        st = self.lib.tdbem_create(ctypes.byref(h), ctypes.byref(opt))
        if st != 0:
            raise TdbemError(st, "context creation failed")
        self.h = h
        self.M = self.E = self.N = 0

    def close(self):
        if getattr(self, "h", None):
            self.lib.tdbem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st < 0 or st > 1:
            raise TdbemError(st, self.lib.tdbem_last_error(self.h).decode())
        return st

    def set_mesh(self, xyz, tri):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        self._check(self.lib.tdbem_set_mesh(self.h, _dptr(xyz), xyz.shape[0], _iptr(tri), tri.shape[0]))
        self.M, self.E = xyz.shape[0], tri.shape[0]

    def set_time_grid(self, t, cutoff="bump", p=0):
        t = np.ascontiguousarray(t, dtype=np.float64)
        c = {"bump": CUTOFF_BUMP, "erf": CUTOFF_ERF}[cutoff] if isinstance(cutoff, str) else int(cutoff)
        self._check(self.lib.tdbem_set_time_grid(self.h, _dptr(t), len(t), c, int(p)))
        self.N = len(t) * (int(p) + 1)          # temporal bases L = N (p + 1)

    def block_nnz(self, k, i):
        n = ctypes.c_int64()
        self._check(self.lib.tdbem_block_nnz(self.h, int(k), int(i), ctypes.byref(n)))
        return n.value

    def get_block_coo(self, k, i):
        """Block A_{k,i} as (row l, column j, value) arrays sorted by (row, column)."""
        n = self.block_nnz(k, i)
        row = np.zeros(n, dtype=np.int32); col = np.zeros(n, dtype=np.int32); val = np.zeros(n)
        self._check(self.lib.tdbem_get_block_coo(self.h, int(k), int(i), _iptr(row), _iptr(col), _dptr(val), n))
        return row, col, val

    def assemble(self, precision=FP64):
        rep = AssemblyReport()
        self._check(self.lib.tdbem_assemble(self.h, int(precision), ctypes.byref(rep)))
        return rep.as_dict()

    def assemble_tuning(self):
        """(test, trial) triangles of the regular-pair tile shape in use and the timed estimate of
        every shape (ms per launch, -1 where not timed)."""
        tt, ts = ctypes.c_int32(), ctypes.c_int32()
        ms = (ctypes.c_double * 2)()
        self._check(self.lib.tdbem_assemble_tuning(self.h, ctypes.byref(tt), ctypes.byref(ts), ms))
        return (tt.value, ts.value), [ms[0], ms[1]]

    def assemble_set_tiles(self, v):
        """Force tile shape v (0: 4 x 8, 1: 8 x 8) for later assemblies; -1 returns to timing."""
        n = ctypes.c_int32()
        self._check(self.lib.tdbem_assemble_set_tiles(self.h, int(v), ctypes.byref(n)))
        return n.value

    def set_block_reuse(self, enable):
        """1: copy the equal blocks of an equidistant grid instead of integrating them (default);
        0: integrate every block.  Takes effect at the next assembly."""
        self._check(self.lib.tdbem_set_block_reuse(self.h, int(enable)))

    def get_entries(self, k, i, j, l):
        k, i, j, l = (np.ascontiguousarray(np.broadcast_to(a, np.broadcast(k, i, j, l).shape).ravel(), dtype=np.int32)
                      for a in (k, i, j, l))
        out = np.zeros(len(k))
        self._check(self.lib.tdbem_get_entries(self.h, len(k), _iptr(k), _iptr(i), _iptr(j), _iptr(l), _dptr(out)))
        return out

    def eval_kernels(self, k, i, r):
        k = np.ascontiguousarray(k, dtype=np.int32).ravel()
        i = np.ascontiguousarray(i, dtype=np.int32).ravel()
        r = np.ascontiguousarray(r, dtype=np.float64).ravel()
        ps = np.zeros(len(r)); pt = np.zeros(len(r))
        self._check(self.lib.tdbem_eval_kernels(self.h, len(r), _iptr(k), _iptr(i), _dptr(r), _dptr(ps), _dptr(pt)))
        return ps, pt

    def _vec(self, n=None):
        return self.torch.empty(self.N * self.M if n is None else n, dtype=self.torch.float64, device=self.device)

    def _dev(self, x, n):
        if not (x.is_cuda and x.dtype == self.torch.float64 and x.is_contiguous() and x.numel() == n):
            raise ValueError(f"expected a contiguous float64 device tensor of {n} values")
        return ctypes.c_void_p(x.data_ptr())

    def rhs_plane_pulse(self, direction, t0, width, out=None):
        d = np.ascontiguousarray(direction, dtype=np.float64)
        g = self._vec() if out is None else out
        self._check(self.lib.tdbem_rhs_plane_pulse(self.h, _dptr(d), float(t0), float(width),
                                                   self._dev(g, self.N * self.M)))
        return g

    def matvec(self, x, out=None):
        y = self._vec() if out is None else out
        n = self.N * self.M
        self._check(self.lib.tdbem_matvec(self.h, self._dev(x, n), self._dev(y, n)))
        return y

    def matvec_range(self, k0, k1, i0, i1, x, out=None):
        y = self._vec((k1 - k0) * self.M) if out is None else out
        self._check(self.lib.tdbem_matvec_range(self.h, k0, k1, i0, i1, self._dev(x, (i1 - i0) * self.M),
                                                self._dev(y, (k1 - k0) * self.M)))
        return y

    def matvec_free(self, x, out=None):
        """y = A x in FP64 with the operator formed on the fly (no stored matrix needed)."""
        y = self._vec() if out is None else out
        n = self.N * self.M
        rep = AssemblyReport()
        self._check(self.lib.tdbem_matvec_free(self.h, self._dev(x, n), self._dev(y, n), ctypes.byref(rep)))
        return y, rep.as_dict()

    def solve(self, g, tol=1e-8, restart=30, max_it=10000, precond_inner=(), out=None, progress=None,
              precond_kind=PRECOND_ALG1, use_graph=False, deflation=None, inner_fp32=False):
        """FGMRES(restart) from 0 to ||g - A alpha|| <= tol ||g||, with Algorithm 1 when
        precond_inner lists inner iterations per level (e.g. (2, 10)); progress(iteration,
        estimate) is called after every outer iteration when given.  precond_kind selects the
        learned network (PRECOND_LEARNED) or the network for the first restart cycle and
        Algorithm 1 afterwards (PRECOND_LEARNED_THEN_ALG1); use_graph replays the learned
        iteration's preconditioned operator as one captured HIP graph.  deflation = (l, r_max)
        runs DGMRES(restart, l) with at most r_max deflation vectors (PRECOND_DEFLATION); inner_fp32
        runs Algorithm 1's products on an FP32 copy of the FP64 band."""
        n = self.N * self.M
        alpha = self._vec() if out is None else out
        o = SolveOpts()
        o.restart, o.tol, o.max_it = int(restart), float(tol), int(max_it)
        o.precond_levels = len(precond_inner)
        for s, v in enumerate(precond_inner):
            o.precond_inner[s] = int(v)
        cb = PROGRESS(lambda it, est, user: progress(int(it), float(est))) if progress else PROGRESS()
        o.progress = cb
        o.precond_kind = int(precond_kind)
        o.use_graph = 1 if use_graph else 0
        o.inner_fp32 = 1 if inner_fp32 else 0
        if deflation is not None:
            o.precond_kind = PRECOND_DEFLATION
            o.deflation_l, o.deflation_max = int(deflation[0]), int(deflation[1])
        rep = SolveReport()
        st = self._check(self.lib.tdbem_solve(self.h, self._dev(g, n), self._dev(alpha, n), ctypes.byref(o),
                                              ctypes.byref(rep)))
        d = rep.as_dict()
        d["converged"] = st == 0
        return alpha, d

    def potential_dl(self, alpha, pts, times, out=None):
        """Retarded double layer potential u[s, p] at the points pts (npts x 3, host) and the
        times (host), from the density coefficients alpha (device, N*M)."""
        P = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        T = np.ascontiguousarray(times, dtype=np.float64).ravel()
        u = self.torch.empty(len(T), len(P), dtype=self.torch.float64, device=self.device) if out is None else out
        self._check(self.lib.tdbem_potential_dl(self.h, self._dev(alpha, self.N * self.M), len(P), _dptr(P), len(T),
                                                _dptr(T), ctypes.c_void_p(u.data_ptr())))
        return u

    # --- many right-hand sides ------------------------------------------------------------------------
    def _dev2(self, X):
        n = self.N * self.M
        if not (X.is_cuda and X.dtype == self.torch.float64 and X.is_contiguous() and X.dim() == 2
                and X.shape[1] == n):
            raise ValueError(f"expected a contiguous float64 device tensor of shape (nrhs, {n})")
        return ctypes.c_void_p(X.data_ptr())

    def matvec_multi(self, X, out=None):
        """Y[r] = A X[r] for the rows of X (shape (nrhs, N*M))."""
        Y = self.torch.empty_like(X) if out is None else out
        self._check(self.lib.tdbem_matvec_multi(self.h, X.shape[0], self._dev2(X), self._dev2(Y)))
        return Y

    def matvec_multi_tuning(self):
        """(right-hand sides per pass, staged trial range, ms per right-hand side) of the variant
        of the multi-vector product chosen by timing on the assembled operator."""
        rc, sp, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        self._check(self.lib.tdbem_matvec_multi_tuning(self.h, ctypes.byref(rc), ctypes.byref(sp), ctypes.byref(ms)))
        return rc.value, sp.value, ms.value

    def matvec_multi_set_variant(self, v):
        """Force variant v of the multi-vector product (-1: timed choice); returns the number of
        variants."""
        nv = ctypes.c_int32()
        self._check(self.lib.tdbem_matvec_multi_set_variant(self.h, int(v), ctypes.byref(nv)))
        return nv.value

    def solve_multi(self, G, tol=1e-8, restart=600, max_it=2000, precond_kind=PRECOND_ALG1, out=None,
                    progress=None):
        """Solve A alpha_r = G[r] for every row of G together (one shared product per iteration);
        precond_kind PRECOND_LEARNED uses the learned network, PRECOND_ALG1 here means none."""
        R = G.shape[0]
        A = self.torch.empty_like(G) if out is None else out
        o = SolveOpts()
        o.restart, o.tol, o.max_it = int(restart), float(tol), int(max_it)
        cb = PROGRESS(lambda it, est, user: progress(int(it), float(est))) if progress else PROGRESS()
        o.progress = cb
        o.precond_kind = int(precond_kind)
        reps = (SolveReport * R)()
        st = self._check(self.lib.tdbem_solve_multi(self.h, R, self._dev2(G), self._dev2(A), ctypes.byref(o), reps))
        out_reps = [r.as_dict() for r in reps]
        for d in out_reps:
            d["converged"] = d["rel_residual"] <= tol
        return A, out_reps, st == 0

    # --- learned preconditioner (include/tdbem_learned.h) -----------------------------------------
    def lp_init(self, layers=4, seed=0):
        self._check(self.lib.tdbem_lp_init(self.h, int(layers), int(seed)))
        self.lp_layers = int(layers)

    def lp_num_params(self, layers=None):
        return int(self.lib.tdbem_lp_num_params(int(self.lp_layers if layers is None else layers)))

    def lp_set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        self._check(self.lib.tdbem_lp_set_params(self.h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), p.size))

    def lp_get_params(self):
        p = np.zeros(self.lp_num_params(), dtype=np.float32)
        self._check(self.lib.tdbem_lp_get_params(self.h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), p.size))
        return p

    def lp_apply(self, v, out=None):
        n = self.N * self.M
        z = self._vec() if out is None else out
        self._check(self.lib.tdbem_lp_apply(self.h, self._dev(v, n), self._dev(z, n)))
        return z

    def lp_gradient(self, v, dz):
        """(z, grad): z = P(v) and the gradient of <dz, P(v)> with respect to the parameters."""
        n = self.N * self.M
        z = self._vec()
        grad = np.zeros(self.lp_num_params(), dtype=np.float32)
        self._check(self.lib.tdbem_lp_gradient(self.h, self._dev(v, n), self._dev(dz, n), self._dev(z, n),
                                               grad.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return z, grad

    def matvec_transpose(self, y, out=None):
        x = self._vec() if out is None else out
        n = self.N * self.M
        self._check(self.lib.tdbem_matvec_transpose(self.h, self._dev(y, n), self._dev(x, n)))
        return x

    def lp_make_pairs(self, count, seed=0):
        """(V, Z): count residuals V[s] = A Z[s] of errors Z[s] drawn by the library (device
        tensors of shape (count, N*M))."""
        n = self.N * self.M
        V = self.torch.empty((int(count), n), dtype=self.torch.float64, device=self.device)
        Z = self.torch.empty_like(V)
        self._check(self.lib.tdbem_lp_make_pairs(self.h, int(count), int(seed), self._dev2(V), self._dev2(Z)))
        return V, Z

    def lp_train_pairs(self, geom, V, Z, steps, batch=8, lr=1e-3, seed=0):
        """Train this context's network on the pairs (V[s], Z[s]) of the mesh and grid of `geom`
        (another Context, or self); returns (per-step losses, report dict)."""
        o = TrainOpts(int(steps), int(batch), float(lr), int(seed))
        hist = np.zeros(int(steps), dtype=np.float32)
        rep = TrainReport()
        n = geom.N * geom.M
        if V.shape != Z.shape or V.dim() != 2 or V.shape[1] != n:
            raise ValueError(f"pairs must be two (count, {n}) tensors")
        self._check(self.lib.tdbem_lp_train_pairs(self.h, geom.h, geom._dev2(V), geom._dev2(Z), int(V.shape[0]),
                                                  ctypes.byref(o), hist.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                  ctypes.byref(rep)))
        return hist, rep.as_dict()

    def lp_train(self, steps, batch=8, lr=1e-3, seed=0):
        """Train the network on the assembled operator; returns (per-step losses, report dict)."""
        o = TrainOpts(int(steps), int(batch), float(lr), int(seed))
        hist = np.zeros(int(steps), dtype=np.float32)
        rep = TrainReport()
        self._check(self.lib.tdbem_lp_train(self.h, ctypes.byref(o), hist.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                            ctypes.byref(rep)))
        return hist, rep.as_dict()
