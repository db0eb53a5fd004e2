"""Pin of the whole oracle pipeline against the paper's closed-form solutions on the unit sphere
(Section 6.1, eq. (formula_phi) and the explicit solutions for n = 0 and n = 1 below it).

For g(x, t) = g(t) Y_n^0(x) the solution of W phi = g is phi(t) Y_n^0(x).  The discrete
solution of the space-time Galerkin system (oracle assembly in fast mode, dense LU) must approach
it in L2(Gamma_h x [0, T]) under joint refinement of the icosphere and the time grid.  This fixes
every part at once: the temporal bases of eq. (BasisFunctions), psi and tilde psi of eq. (psis)
(n = 1 exercises the curl-curl term, n = 0 does not), the local integrals of eq.
(MatrixEntries), the scatter into the global blocks and the right-hand side of Section 3.

Two readings of the paper are pinned here as well:
  * sign: the closed forms solve W phi = g for the operator whose Laplace symbol is the negative
    of the one of the variational form eq. (VarForm); the discrete solution converges to
    -phi_paper (with +phi_paper the relative error would approach 2);
  * order: with p = 0 (one bump per node) the space reproduces constants only, its time
    derivatives do not converge, and the discrete solution does not approach the closed form
    (relative error ~0.5 at every level); with p = 1 it does (the paper's convergence tests
    use p >= 1).
"""
import math

import numpy as np
import pytest
from scipy import integrate

from workloads import equidistant_grid, icosphere

Y00 = 1.0 / (2.0 * math.sqrt(math.pi))


def _quad(f, a, b):
    return integrate.quad(f, a, b, epsabs=1e-13, epsrel=1e-12, limit=200)[0]


def g_n0(t):
    return math.sin(3 * t) * t * t * math.exp(-t) if t > 0 else 0.0


def dg_n0(t):
    return (3 * math.cos(3 * t) * t * t + 2 * t * math.sin(3 * t) - t * t * math.sin(3 * t)) * math.exp(-t) if t > 0 else 0.0


def phi_paper_n0(t):
    """The paper's n = 0 solution: -2 int_0^t g(t-s) cosh s ds plus the reflection terms
    2 sum_{k=1}^{floor(t/2)} sum_{l=1}^{k} (-1)^{k+1} c_{k,l} int_{2k}^t (s-2k)^{k-l+1} e^{s-2k} g'(t-s) ds,
    c_{k,l} = binom(k-1, l-1) 2^{k-l} / (k-l+1)!."""
    v = -2.0 * _quad(lambda s: g_n0(t - s) * math.cosh(s), 0.0, t)
    for k in range(1, int(t // 2) + 1):
        for l in range(1, k + 1):
            c = math.comb(k - 1, l - 1) * 2.0 ** (k - l) / math.factorial(k - l + 1)
            v += 2.0 * (-1) ** (k + 1) * c * _quad(
                lambda s: (s - 2 * k) ** (k - l + 1) * math.exp(s - 2 * k) * dg_n0(t - s), 2.0 * k, t)
    return v


def g_n1(t):
    return math.sin(2 * math.pi * t) * t ** 3 * math.exp(-2 * t) if t > 0 else 0.0


def phi_paper_n1(t):
    """The paper's n = 1 solution for t < 2: -2 int_0^t g(t-s) cosh(s) cos(s) ds."""
    return -2.0 * _quad(lambda s: g_n1(t - s) * math.cosh(s) * math.cos(s), 0.0, t)


def relative_error(oracle, level, N, n, p, kind="erf"):
    """||phi_h - (-phi_paper) Y_n^0|| / ||phi_paper Y_n^0|| in L2(Gamma_h x [0, T])."""
    T = 6.0 if n == 0 else 2.0
    xyz, tri = icosphere(level)
    grid = equidistant_grid(N, T)
    M, L = len(xyz), N * (p + 1)
    B, W = oracle.rule7()
    P = xyz[tri]
    area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    X = np.einsum("qa,eac->eqc", B, P)                    # 7 points per flat triangle
    Yq = np.full(X.shape[:2], Y00) if n == 0 else math.sqrt(3.0 / (4.0 * math.pi)) * X[..., 2]
    space = np.zeros(M)                                   # int_Gamma Y phi_l
    for a in range(3):
        np.add.at(space, tri[:, a], area * (Yq * B[None, :, a] * W[None, :]).sum(1))
    xg, wg = np.polynomial.legendre.leggauss(24)
    tq = np.concatenate([0.5 * (b - a) * xg + 0.5 * (a + b) for a, b in zip(grid[:-1], grid[1:])])
    wt = np.concatenate([0.5 * (b - a) * wg for a, b in zip(grid[:-1], grid[1:])])
    bas = np.array([[oracle.basis(grid, i, t, kind, p) for t in tq] for i in range(L)])
    gfun = g_n0 if n == 0 else g_n1
    time_part = (bas[:, :, 1] * np.array([gfun(t) for t in tq])[None] * wt[None]).sum(1)   # int g b_k'
    rhs = (time_part[:, None] * space[None, :]).ravel()
    tables = oracle.fast_tables(xyz, grid, kind, p=p)
    A = oracle.system_matrix(oracle.assemble_dense(xyz, tri, grid, kind=kind, tables=tables, p=p))
    alpha = np.linalg.solve(A, rhs).reshape(L, M)
    hq = np.einsum("iea,qa->ieq", alpha[:, tri], B)       # density at the points, per basis
    ref = -np.array([(phi_paper_n0 if n == 0 else phi_paper_n1)(t) for t in tq])
    num = den = 0.0
    for m in range(len(tq)):
        ph = np.einsum("i,ieq->eq", bas[:, m, 0], hq)
        ex = ref[m] * Yq
        num += wt[m] * (area[:, None] * W[None] * (ph - ex) ** 2).sum()
        den += wt[m] * (area[:, None] * W[None] * ex ** 2).sum()
    return math.sqrt(num / den)


def test_closed_form_satisfies_the_reduced_equation():
    """The reading of the sign: on the unit sphere a density f(t) constant in space gives, by
    eq. (VarForm), W f(t) = 1/2 int_0^2 (1 - r^2/2) f''(t - r) dr (n_x.n_y = 1 - r^2/2, dGamma_y =
    2 pi r dr); f = -phi_paper solves W f = g (finite differences of the closed form)."""
    h = 2e-3
    ts = np.arange(0.0, 5.0 + h / 2, h)
    f = -np.array([phi_paper_n0(t) for t in ts])
    fdd = np.zeros_like(f)
    fdd[1:-1] = (f[2:] - 2 * f[1:-1] + f[:-2]) / h ** 2
    for tt in (0.7, 1.7, 2.5, 3.3, 4.5):
        m = int(round(tt / h))
        rs = np.arange(0.0, min(2.0, tt) + h / 2, h)
        vals = 0.5 * (1 - rs ** 2 / 2) * fdd[m - np.round(rs / h).astype(int)]
        Wf = h * (vals.sum() - 0.5 * vals[0] - 0.5 * vals[-1])
        assert abs(Wf - g_n0(tt)) <= 2e-4 * max(1.0, abs(g_n0(tt))), (tt, Wf, g_n0(tt))


def test_convergence_n0_p1(oracle_mod):
    """n = 0, T = 6, p = 1 (Figure 6.1 setting): icosphere level 0 -> 1 with N = 6 -> 12."""
    e0 = relative_error(oracle_mod, 0, 6, 0, 1)
    e1 = relative_error(oracle_mod, 1, 12, 0, 1)
    assert e1 < 0.5 * e0 and e1 < 0.2, (e0, e1)


def test_convergence_n1_p1(oracle_mod):
    """n = 1 (curl-curl term active), T = 2, p = 1: icosphere levels 0 -> 1 -> 2 with
    N = 6 -> 12 -> 24."""
    errs = [relative_error(oracle_mod, lv, N, 1, 1) for lv, N in ((0, 6), (1, 12), (2, 24))]
    assert errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1] and errs[2] < 0.05, errs


def test_p0_space_does_not_converge(oracle_mod):
    """With one bump per node (p = 0) the error stays O(1) under refinement (the space does not
    reproduce linear functions, so the time derivatives in eq. (VarForm) keep an O(1) error)."""
    errs = [relative_error(oracle_mod, lv, N, 1, 0) for lv, N in ((0, 6), (1, 12))]
    assert min(errs) > 0.3, errs
