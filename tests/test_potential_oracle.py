"""Pins of the oracle's retarded double layer potential (eq. (RetardedPotential)).

* Gauss's law: the density 1 (every alpha = 1, so phi(y, t) = sum_i b_i(t) = 1 and its time
  derivative vanishes once every retarded time lies in [t_1, T], by the partition of unity of
  Section 3) gives u = (solid angle of Gamma seen from x) / (4 pi): 1 inside, 0 outside.  The exact
  per-triangle solid angles (Van Oosterom and Strackee 1983) are summed independently; the oracle's
  7-point rule differs from them by its quadrature error only.
* Causality: u(x, t) = 0 exactly while every retarded time t - |x - y| is negative.
* One triangle, a density with both terms active, against adaptive quadrature (scipy) of the same
  integrand: the 7-point rule on the triangle split into 256 congruent pieces (the P1 density
  interpolated at the new vertices is the same linear function) must agree to 1e-9, the rule on
  the whole triangle to its quadrature error (the time bases vary across it).  Catches a dropped
  term, a wrong power of r, a wrong sign or normal.
"""
import numpy as np
from scipy import integrate

from workloads import equidistant_grid, graded_grid, icosphere


def _solid_angles(xyz, tri, x):
    R = xyz[tri] - x
    n = np.linalg.norm(R, axis=2)
    num = np.einsum("ij,ij->i", R[:, 0], np.cross(R[:, 1], R[:, 2]))
    den = (n[:, 0] * n[:, 1] * n[:, 2] + np.einsum("ij,ij->i", R[:, 0], R[:, 1]) * n[:, 2]
           + np.einsum("ij,ij->i", R[:, 0], R[:, 2]) * n[:, 1] + np.einsum("ij,ij->i", R[:, 1], R[:, 2]) * n[:, 0])
    return 2.0 * np.arctan2(num, den)


def test_gauss_law(oracle_mod):
    xyz, tri = icosphere(2)
    grid = equidistant_grid(10, 8.0)
    alpha = np.ones(10 * len(xyz))
    pts = np.array([[0.0, 0.0, 0.0], [0.1, -0.2, 0.25], [2.5, 0.0, 0.0], [0.0, 1.7, 1.7]])
    u = oracle_mod.potential_dl(xyz, tri, grid, alpha, pts, [6.0, 7.5])
    exact = np.array([_solid_angles(xyz, tri, p).sum() / (4 * np.pi) for p in pts])
    assert np.allclose(exact, [1.0, 1.0, 0.0, 0.0], atol=1e-13)
    for s in range(2):
        assert np.all(np.abs(u[s, :2] - 1.0) <= 1e-6), u
        assert np.all(np.abs(u[s, 2:]) <= 1e-9), u


def test_causality(oracle_mod):
    xyz, tri = icosphere(1)
    grid = graded_grid(8, 4.0, seed=1)
    alpha = np.random.default_rng(1).standard_normal(8 * len(xyz))
    pts = np.array([[3.0, 0.0, 0.0], [0.0, -2.5, 1.0]])
    rmin = np.array([np.linalg.norm(xyz - p, axis=1).min() for p in pts]) - 0.05   # below the nearest vertex
    u = oracle_mod.potential_dl(xyz, tri, grid, alpha, pts, [0.5 * rmin.min(), 0.95 * rmin.min()])
    assert np.all(u == 0.0)
    u2 = oracle_mod.potential_dl(xyz, tri, grid, alpha, pts, [rmin.max() + 1.5])
    assert np.all(np.abs(u2) > 0.0)


def test_single_triangle_against_adaptive_quadrature(oracle_mod):
    P = np.array([[0.0, 0.0, 0.0], [0.2, 0.0, 0.05], [0.05, 0.18, 0.0]])
    tri = np.array([[0, 1, 2]], dtype=np.int32)
    grid = equidistant_grid(6, 3.0)
    N = len(grid)
    alpha = np.random.default_rng(2).standard_normal(N * 3)
    x = np.array([0.6, -0.9, 1.1])
    t = 2.3
    u = oracle_mod.potential_dl(P, tri, grid, alpha, x[None, :], [t])[0, 0]
    e1, e2 = P[1] - P[0], P[2] - P[0]
    cr = np.cross(e1, e2)
    area2 = np.linalg.norm(cr)
    nrm = cr / area2

    def f(s2, s1):                      # reference triangle 0 <= s2 <= 1 - s1
        y = P[0] + s1 * e1 + s2 * e2
        lam = np.array([1.0 - s1 - s2, s1, s2])
        d = x - y
        r = np.linalg.norm(d)
        phi = dphi = 0.0
        for i in range(N):
            b = oracle_mod.basis(grid, i, t - r)
            dens = lam @ alpha[i * 3:(i + 1) * 3]
            phi += b[0] * dens
            dphi += b[1] * dens
        return -(nrm @ d) / r * (phi / r ** 2 + dphi / r) / (4 * np.pi) * area2

    ref, _ = integrate.dblquad(f, 0.0, 1.0, 0.0, lambda s1: 1.0 - s1, epsabs=1e-14, epsrel=1e-12)
    assert abs(ref) > 1e-4
    assert abs(u - ref) <= 5e-3 * abs(ref), (u, ref)
    # the same triangle split into n^2 pieces on the barycentric grid
    n = 16
    ids = {}
    verts, dens = [], []
    for a in range(n + 1):
        for b in range(n + 1 - a):
            lam = np.array([1.0 - (a + b) / n, a / n, b / n])
            ids[(a, b)] = len(verts)
            verts.append(lam @ P)
            dens.append([lam @ alpha[i * 3:(i + 1) * 3] for i in range(N)])
    tris = []
    for a in range(n):
        for b in range(n - a):
            tris.append([ids[(a, b)], ids[(a + 1, b)], ids[(a, b + 1)]])
            if a + b + 1 < n:
                tris.append([ids[(a + 1, b)], ids[(a + 1, b + 1)], ids[(a, b + 1)]])
    V = np.array(verts)
    A = np.array(dens).T.reshape(-1)         # alpha[i*M + j]
    uf = oracle_mod.potential_dl(V, np.array(tris, dtype=np.int32), grid, A, x[None, :], [t])[0, 0]
    assert len(tris) == n * n
    assert abs(uf - ref) <= 1e-9 * abs(ref), (uf, ref)
