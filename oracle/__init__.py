"""CPU oracle for the space-time Galerkin TDBIE hot path (arXiv:1503.07221).

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_1503_07221_amd``): the heavy loops live in ``tdbem_oracle.c`` (plain C, FP64,
OpenMP over element pairs); the solver (FGMRES and the recursive block-Hessenberg
preconditioner) is plain numpy below.

Vector layout follows the block partition of eq. (A): x[i*M + j] is the coefficient of the
temporal basis b_i and the spatial hat phi_j; row (k, l) of the system is x[k*M + l].
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "tdbem_oracle.c")

CUTOFF = {"bump": 0, "erf": 1}
MODE = {"psi": 0, "r": 1, "r3": 2, "one": 3, "curl": 4, "nn": 5, "r_r3": 6}


def build(force=False):
    """Compile liboracle.so with gcc (-O3, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c99", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        L.orc_gauss_legendre.argtypes = [ctypes.c_int, dp, dp]
        L.orc_cutoff.argtypes = [ctypes.c_int, ctypes.c_double, dp]
        L.orc_mu.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp]
        L.orc_basis.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp]
        L.orc_support.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
        L.orc_psi.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              ctypes.c_double, dp]
        L.orc_rule7.argtypes = [dp, dp]
        L.orc_ss_rule.argtypes = [ctypes.c_int, ctypes.c_int, dp]
        L.orc_ss_rule.restype = ctypes.c_int
        L.orc_pair_local.argtypes = [dp, ip, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        vp = ctypes.c_void_p
        L.orc_assemble_dense.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, dp]
        L.orc_assemble_dense.restype = ctypes.c_int
        L.orc_assemble_entries.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int, ip, ip, dp]
        L.orc_tables_build.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int]
        L.orc_tables_build.restype = vp
        L.orc_tables_free.argtypes = [vp]
        L.orc_psi_fast.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp]
        L.orc_rhs_plane_pulse.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_count_quad_evals.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, vp]
        L.orc_count_quad_evals.restype = ctypes.c_int64
        L.orc_local_batch.argtypes = [dp, ip, ctypes.c_int, ip, ip, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, vp, dp]
        L.orc_local_batch.restype = ctypes.c_int64
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_potential_dl.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_int, dp, dp]
        L.orc_potential_dl.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


# ---------------------------------------------------------------------------------------------
# time basis and time kernels (Section 3, eq. (BasisFunctions), eq. (psis))
# ---------------------------------------------------------------------------------------------
def gauss_legendre(n):
    x = np.zeros(n); w = np.zeros(n)
    xp = x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    wp = w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    lib().orc_gauss_legendre(n, xp, wp)
    return x, w


def cutoff(u, kind="bump"):
    out = np.zeros(3)
    lib().orc_cutoff(CUTOFF[kind], float(u), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def mu(grid, j, t, kind="bump"):
    g, gp = _d(grid)
    out = np.zeros(3)
    lib().orc_mu(gp, len(g), CUTOFF[kind], j, float(t), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def basis(grid, j, t, kind="bump", p=0):
    """(b_j(t), b_j'(t), b_j''(t)) for basis j = n (p + 1) + m (node n, Legendre degree m)."""
    g, gp = _d(grid)
    out = np.zeros(3)
    lib().orc_basis(gp, len(g), CUTOFF[kind], p, j, float(t), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def support(grid, k, i, p=0):
    """Open support (lo, hi) of psi_{k,i} in r >= 0 (Section 3.2)."""
    g, gp = _d(grid)
    lo = ctypes.c_double(); hi = ctypes.c_double()
    lib().orc_support(gp, len(g), p, k, i, ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def psi(grid, k, i, r, kind="bump", p=0):
    """(psi_{k,i}(r), tilde psi_{k,i}(r)) by direct quadrature of eq. (psis)."""
    g, gp = _d(grid)
    out = np.zeros(2)
    lib().orc_psi(gp, len(g), CUTOFF[kind], p, k, i, float(r), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


class Tables:
    """Fast mode: the oracle's own tabulation of psi_{k,i}, tpsi_{k,i} (uniform grid of n + 1
    points over each support cut at rmax, degree-11 local interpolation), built by direct
    quadrature of eq. (psis) at every grid point."""

    def __init__(self, grid, kind="bump", rmax=2.0, n=2048, p=0):
        g, gp = _d(grid)
        self.N, self.p = len(g), p
        self.h = lib().orc_tables_build(gp, len(g), CUTOFF[kind], int(p), float(rmax), int(n))
        if not self.h:
            raise MemoryError("oracle tables")

    def psi(self, k, i, r):
        out = np.zeros(2)
        lib().orc_psi_fast(self.h, k, i, float(r), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return out

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_tables_free(self.h)
            self.h = None


def mesh_diameter(xyz):
    """An upper bound of every distance on the mesh (diagonal of the bounding box)."""
    xyz = np.asarray(xyz)
    return float(np.linalg.norm(xyz.max(axis=0) - xyz.min(axis=0))) * (1 + 1e-9) + 1e-12


def fast_tables(xyz, grid, kind="bump", n=2048, p=0):
    return Tables(grid, kind, mesh_diameter(xyz), n, p)


# ---------------------------------------------------------------------------------------------
# quadrature rules
# ---------------------------------------------------------------------------------------------
def rule7():
    b = np.zeros(21); w = np.zeros(7)
    lib().orc_rule7(b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return b.reshape(7, 3), w


def ss_rule(kind, order):
    """Sauter-Schwab rule rows (x1, x2, y1, y2, weight) on the reference triangle pair;
    kind 0 identical, 1 common edge, 2 common vertex."""
    n = (6, 5, 2)[kind] * order ** 4
    out = np.zeros(5 * n)
    cnt = lib().orc_ss_rule(kind, order, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out[:5 * cnt].reshape(cnt, 5)


# ---------------------------------------------------------------------------------------------
# assembly (eq. (MatrixEntries))
# ---------------------------------------------------------------------------------------------
def pair_local(xyz, tri, ex, ey, grid, kind="bump", mode="psi", ss_order=4, p=0):
    x, xp = _d(xyz); t, tp = _i(tri); g, gp = _d(grid)
    L = len(g) * (p + 1)
    nb = L if MODE[mode] in (0, 4, 5) else 1
    loc = np.zeros(nb * nb * 9)
    lib().orc_pair_local(xp, tp, ex, ey, gp, len(g), CUTOFF[kind], p, MODE[mode], ss_order,
                         loc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return loc.reshape(nb, nb, 3, 3)


def assemble_dense(xyz, tri, grid, kind="bump", mode="psi", ss_order=4, tables=None, p=0):
    """All blocks: returns A[k, i, j, l] = A_{k,i}(j, l) for the L = N (p + 1) bases.  tables: a
    Tables of the same grid, cutoff and p (fast mode), or None (direct quadrature of every
    kernel value)."""
    x, xp = _d(xyz); t, tp = _i(tri); g, gp = _d(grid)
    M, E, N = len(x), len(t), len(g)
    L = N * (p + 1)
    nb = L if MODE[mode] in (0, 4, 5) else 1
    out = np.zeros(nb * nb * M * M)
    rc = lib().orc_assemble_dense(xp, M, tp, E, gp, N, CUTOFF[kind], p, MODE[mode], ss_order,
                                  tables.h if tables is not None else None,
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise MemoryError("oracle dense assembly failed")
    return out.reshape(nb, nb, M, M)


def assemble_entries(xyz, tri, grid, sel_j, sel_l, kind="bump", mode="psi", ss_order=4, tables=None, p=0):
    """Selected entries: returns out[s, k, i] = A_{k,i}(sel_j[s], sel_l[s])."""
    x, xp = _d(xyz); t, tp = _i(tri); g, gp = _d(grid)
    sj, sjp = _i(sel_j); sl, slp = _i(sel_l)
    M, E, N = len(x), len(t), len(g)
    L = N * (p + 1)
    nb = L if MODE[mode] in (0, 4, 5) else 1
    out = np.zeros(len(sj) * nb * nb)
    lib().orc_assemble_entries(xp, M, tp, E, gp, N, CUTOFF[kind], p, MODE[mode], ss_order,
                               tables.h if tables is not None else None, len(sj), sjp, slp,
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out.reshape(len(sj), nb, nb)


def rhs_plane_pulse(xyz, tri, grid, direction, t0, width, kind="bump", p=0):
    """g[k*M + l] for g = -d_n u_inc, u_inc = exp(-((t - t0 - d.x)/w)^2)."""
    x, xp = _d(xyz); t, tp = _i(tri); g, gp = _d(grid); d, dp = _d(direction)
    M, E, N = len(x), len(t), len(g)
    out = np.zeros(N * (p + 1) * M)
    lib().orc_rhs_plane_pulse(xp, M, tp, E, gp, N, CUTOFF[kind], p, dp, float(t0), float(width),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def count_quad_evals(xyz, tri, grid, ss_order=4, p=0, node_blocks=None):
    """Quadrature-point count; node_blocks: optional (N, N) boolean mask of the node blocks
    (test node, trial node) to count."""
    x, xp = _d(xyz); t, tp = _i(tri); g, gp = _d(grid)
    mask = None
    if node_blocks is not None:
        mask = np.ascontiguousarray(node_blocks, dtype=np.uint8)
        assert mask.shape == (len(g), len(g))
    return int(lib().orc_count_quad_evals(xp, len(x), tp, len(t), gp, len(g), p, ss_order,
                                          mask.ctypes.data_as(ctypes.c_void_p) if mask is not None else None))


def local_batch(xyz, tri, taus, sigmas, grid, kind="bump", ss_order=4, tables=None, p=0):
    """Local integrals of the ordered pairs (taus[s], sigmas[s]); returns (quad-evals, checksum)."""
    x, xp = _d(xyz); t, tp = _i(tri); g, gp = _d(grid)
    a, ap = _i(taus); b, bp = _i(sigmas)
    chk = ctypes.c_double()
    n = lib().orc_local_batch(xp, tp, len(a), ap, bp, gp, len(g), CUTOFF[kind], p, ss_order,
                              tables.h if tables is not None else None, ctypes.byref(chk))
    return int(n), chk.value


def potential_dl(xyz, tri, grid, alpha, pts, times, kind="bump", p=0):
    """Retarded double layer potential u(x_p, t_s) of eq. (RetardedPotential) of the density
    sum alpha[i*M + j] b_i(t) phi_j(y); returns an array [len(times), len(pts)]."""
    x, xp = _d(xyz); t, tp = _i(tri); g, gp = _d(grid)
    a, ap = _d(np.ravel(alpha)); P, Pp = _d(np.reshape(pts, (-1, 3))); T, Tp = _d(np.ravel(times))
    out = np.zeros(len(T) * len(P))
    lib().orc_potential_dl(xp, len(x), tp, len(t), gp, len(g), CUTOFF[kind], p, ap, len(P), Pp, len(T), Tp,
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out.reshape(len(T), len(P))


def num_threads():
    return int(lib().orc_num_threads())


def system_matrix(blocks):
    """Dense LM x LM matrix, row (k, l) = k*M + l, column (i, j) = i*M + j."""
    N, _, M, _ = blocks.shape
    return np.ascontiguousarray(blocks.transpose(0, 3, 1, 2).reshape(N * M, N * M))


# ---------------------------------------------------------------------------------------------
# solver: FGMRES (Saad 1993) and the recursive block-Hessenberg preconditioner (Algorithm 1)
# ---------------------------------------------------------------------------------------------
def fgmres(apply_A, b, tol, max_it, restart=30, precond=None, x0=None, inner=False):
    """Right-preconditioned flexible GMRES with modified Gram-Schmidt and Givens rotations.

    Stops when the Givens residual estimate drops to tol*||b||; an outer solve then confirms
    with the true residual ||b - A x|| and restarts if needed.  An inner solve (inner=True)
    runs at most max_it iterations without restart.  Returns (x, iterations, history)."""
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else x0.copy()
    bnorm = np.linalg.norm(b)
    hist = []
    if bnorm == 0.0:
        return x, 0, hist
    its = 0
    r = b - apply_A(x) if x0 is not None else b.copy()
    beta = np.linalg.norm(r)
    while True:
        m = min(restart, max_it - its) if not inner else max_it
        if m <= 0 or beta <= tol * bnorm:
            break
        V = np.zeros((m + 1, n)); Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m); sn = np.zeros(m)
        gvec = np.zeros(m + 1); gvec[0] = beta
        V[0] = r / beta
        jdone = 0
        for j in range(m):
            Z[j] = V[j] if precond is None else precond(V[j])
            w = apply_A(Z[j])
            for q in range(j + 1):
                H[q, j] = np.dot(w, V[q])
                w = w - H[q, j] * V[q]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for q in range(j):
                tmp = cs[q] * H[q, j] + sn[q] * H[q + 1, j]
                H[q + 1, j] = -sn[q] * H[q, j] + cs[q] * H[q + 1, j]
                H[q, j] = tmp
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den if den != 0 else 1.0
            sn[j] = H[j + 1, j] / den if den != 0 else 0.0
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            gvec[j + 1] = -sn[j] * gvec[j]
            gvec[j] = cs[j] * gvec[j]
            its += 1
            jdone = j + 1
            hist.append(abs(gvec[j + 1]) / bnorm)
            if abs(gvec[j + 1]) <= tol * bnorm:
                break
        y = np.linalg.solve(np.triu(H[:jdone, :jdone]), gvec[:jdone]) if jdone > 0 else np.zeros(0)
        x = x + Z[:jdone].T @ y
        if inner:
            break
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        if its >= max_it:
            break
    return x, its, hist


def block_operator(Afull, N, M, k0, k1, i0, i1):
    """Sub-operator of the block system: rows k in [k0,k1), columns i in [i0,i1)."""
    sub = Afull[k0 * M:k1 * M, i0 * M:i1 * M]
    return lambda v: sub @ v


def alg1_preconditioner(Afull, N, M, tol, inner_its, k0=0, k1=None, level=1):
    """Algorithm 1 (ApplyPreconditioner), read with per-call depth: the preconditioner of the
    time-block range [k0,k1) splits it at h = k0 + ceil(n/2); M11 = A[k<h, i<h],
    M21 = A[k>=h, i<h], M22 = A[k>=h, i>=h] (the single block coupling the halves above the
    diagonal is dropped).  y1 ~ M11^{-1} x1 and y2 ~ M22^{-1}(x2 - M21 y1) by inner FGMRES with
    inner_its[level-1] iterations, preconditioned the same way one level deeper while
    level < len(inner_its), unpreconditioned at the last level."""
    if k1 is None:
        k1 = N
    n = k1 - k0
    h = k0 + (n + 1) // 2
    m_it = inner_its[level - 1]
    deeper = level < len(inner_its)
    A11 = block_operator(Afull, N, M, k0, h, k0, h)
    A21 = block_operator(Afull, N, M, h, k1, k0, h)
    A22 = block_operator(Afull, N, M, h, k1, h, k1)
    P1 = alg1_preconditioner(Afull, N, M, tol, inner_its, k0, h, level + 1) if deeper and h - k0 > 1 else None
    P2 = alg1_preconditioner(Afull, N, M, tol, inner_its, h, k1, level + 1) if deeper and k1 - h > 1 else None

    def apply(x):
        x1 = x[:(h - k0) * M]
        x2 = x[(h - k0) * M:]
        y1, _, _ = fgmres(A11, x1, tol, m_it, precond=P1, inner=True)
        y2 = np.zeros(0)
        if k1 > h:
            y2, _, _ = fgmres(A22, x2 - A21(y1), tol, m_it, precond=P2, inner=True)
        return np.concatenate([y1, y2])

    return apply


def solve(Afull, g, N, M, tol=1e-8, restart=30, max_it=5000, alg1_inner=None):
    """FGMRES(restart) on A alpha = g, optionally with the Algorithm 1 preconditioner."""
    P = alg1_preconditioner(Afull, N, M, tol, alg1_inner) if alg1_inner else None
    return fgmres(lambda v: Afull @ v, g, tol, max_it, restart=restart, precond=P)


# ---------------------------------------------------------------------------------------------
# DGMRES(m, l): restarted GMRES preconditioned by deflation (Section 4.1, after Erhel, Burrage
# and Pohl 1996)
# ---------------------------------------------------------------------------------------------
def deflation_inverse(v, U, Tinv, lam):
    """M^{-1} v = v + U (|lambda_LM| T^{-1} - I) U^T v with T = U^T A U (Section 4.1)."""
    if U.shape[1] == 0:
        return v.copy()
    c = U.T @ v
    return v + U @ (lam * (Tinv @ c) - c)


def smallest_invariant_basis(H, l):
    """Real orthonormal basis (k x l', l' = l, or l + 1 to keep a complex pair whole) of the
    invariant subspace of the k x k matrix H belonging to its l eigenvalues of smallest modulus,
    and the largest eigenvalue modulus.  Eigenvectors by a library eigensolver; complex pairs
    contribute their real and imaginary parts."""
    ev, W = np.linalg.eig(H)
    order = np.argsort(np.abs(ev), kind="stable")
    cols, taken = [], 0
    for idx in order:
        if taken >= l:
            break
        if abs(ev[idx].imag) > 1e-14 * max(1.0, abs(ev[idx])):
            if ev[idx].imag < 0:
                continue                          # its conjugate partner supplies the pair
            cols += [W[:, idx].real, W[:, idx].imag]
            taken += 2
        else:
            cols.append(W[:, idx].real)
            taken += 1
    Y = np.array(cols).T if cols else np.zeros((H.shape[0], 0))
    Q, _ = np.linalg.qr(Y)
    return Q, float(np.abs(ev).max())


def dgmres(apply_A, b, tol, max_it, m=50, l=4, rmax=None):
    """DGMRES(m, l): GMRES(m) right-preconditioned by the deflation M^{-1} of Section 4.1.  After
    every cycle the eigenvectors of the cycle's Hessenberg matrix H_m (of the preconditioned
    operator A M^{-1}) for its l smallest eigenvalues, mapped back as V_m S, are orthonormalised
    against U and appended to U until U has rmax columns (default 4 l); |lambda_LM| is estimated
    by the largest eigenvalue modulus of H_m.  Stops at the true residual ||b - A x|| <= tol ||b||.
    Returns (x, iterations, history)."""
    n = b.shape[0]
    rmax = 4 * l if rmax is None else rmax
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    hist = []
    if bnorm == 0.0:
        return x, 0, hist
    U = np.zeros((n, 0)); AU = np.zeros((n, 0)); Tinv = np.zeros((0, 0)); lam = 1.0
    its = 0
    r = b.copy()
    beta = np.linalg.norm(r)
    while its < max_it and beta > tol * bnorm:
        k = min(m, max_it - its)
        V = np.zeros((k + 1, n)); Z = np.zeros((k, n)); H = np.zeros((k + 1, k))
        V[0] = r / beta
        done = 0
        g = np.zeros(k + 1); g[0] = beta
        for j in range(k):
            Z[j] = deflation_inverse(V[j], U, Tinv, lam)
            w = apply_A(Z[j])
            for q in range(j + 1):
                H[q, j] = np.dot(w, V[q])
                w = w - H[q, j] * V[q]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            its += 1
            done = j + 1
            y, *_ = np.linalg.lstsq(H[:j + 2, :j + 1], g[:j + 2], rcond=None)
            res = np.linalg.norm(g[:j + 2] - H[:j + 2, :j + 1] @ y)
            hist.append(res / bnorm)
            if res <= tol * bnorm or H[j + 1, j] == 0.0:
                break
        y, *_ = np.linalg.lstsq(H[:done + 1, :done], g[:done + 1], rcond=None)
        x = x + Z[:done].T @ y
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm or its >= max_it:
            break
        if U.shape[1] < rmax and done >= 2:
            S, lam_c = smallest_invariant_basis(H[:done, :done], min(l, rmax - U.shape[1]))
            lam = max(lam if U.shape[1] else 0.0, lam_c)
            W = V[:done].T @ S
            for _ in range(2):                   # orthonormalise against U, twice
                W = W - U @ (U.T @ W)
            Q, R = np.linalg.qr(W)
            keep = np.abs(np.diag(R)) > 1e-10 * max(1.0, np.abs(np.diag(R)).max(initial=0.0))
            Q = Q[:, keep]
            if Q.shape[1]:
                U = np.hstack([U, Q])
                AU = np.hstack([AU, np.column_stack([apply_A(Q[:, c]) for c in range(Q.shape[1])])])
                Tinv = np.linalg.inv(U.T @ AU)
    return x, its, hist
