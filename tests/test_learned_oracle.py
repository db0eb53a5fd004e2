"""Pins of the learned-preconditioner oracle (``oracle.learned``).

The network is defined in that module's docstring.  The pins fix it without comparing the oracle
with itself: hand-chosen weights for which the output has a closed form (neighbour mean, time
shifts, ReLU, the scale s, the time features), invariances (positive homogeneity, relabelling of
the vertices) and central finite differences for the gradient.
"""
import numpy as np
import pytest

from oracle import learned as LP
from workloads import graded_grid, icosphere

H = LP.HIDDEN


def _mesh():
    xyz, tri = icosphere(1)
    return xyz, tri, graded_grid(6, 3.0, seed=3)


def _edges_adjacency(tri, M):
    """Vertex adjacency built from the triangle edges as a dense 0/1 matrix (independent of
    oracle.learned.neighbours)."""
    A = np.zeros((M, M))
    for a, b in ((0, 1), (1, 2), (2, 0)):
        A[tri[:, a], tri[:, b]] = 1.0
        A[tri[:, b], tri[:, a]] = 1.0
    return A


def _zero(layers):
    return np.zeros(LP.num_params(layers), dtype=np.float32)


def test_layout_and_bf16_rounding():
    assert LP.num_params(4) == 256 + 4 * 16448 + 64 == 66112
    o = LP.offsets(2)
    assert o[("W", 0)] == 256 and o[("b", 0)] == 256 + 16384 and o[("W", 1)] == 256 + 16448
    assert o["wout"] == 256 + 2 * 16448
    # bfloat16 keeps 8 significant bits: 1 + 2^-8 is a tie between 1 and 1 + 2^-7 (even: 1),
    # 1 + 3*2^-8 rounds up to 1 + 2^-6, values already on the grid are kept
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 3.0e-3], dtype=np.float32)
    r = LP.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2.0 ** -6 and r[3] == -2.5
    assert abs(r[4] - 3.0e-3) <= 3.0e-3 * 2.0 ** -8


def test_neighbour_mean_closed_form():
    """One layer whose only weight passes the neighbour mean of channel 0 (= v/s):
    z = v + relu(mean of v over the mesh neighbours)."""
    xyz, tri, grid = _mesh()
    M, N = len(xyz), len(grid)
    p = _zero(1); o = LP.offsets(1)
    p[o["Win"] + 0] = 1.0                      # Win[0][0]
    p[o[("W", 0)] + 0 * 4 * H + H + 0] = 1.0   # W[0][agg block, channel 0]
    p[o["wout"] + 0] = 1.0
    v = np.random.default_rng(1).standard_normal(N * M)
    z, _ = LP.forward(p, 1, v, grid, LP.neighbours(tri, M))
    A = _edges_adjacency(tri, M)
    mean = (v.reshape(N, M) @ A.T) / A.sum(1)
    assert np.allclose(z.reshape(N, M), v.reshape(N, M) + np.maximum(mean, 0.0), rtol=0, atol=1e-13)


def test_time_shift_closed_forms():
    """Previous-block weight +1 and next-block weight -1 on channel 0:
    z(k) = v(k) + relu(v(k-1) - v(k+1)) with zero blocks outside 0..N-1."""
    xyz, tri, grid = _mesh()
    M, N = len(xyz), len(grid)
    p = _zero(1); o = LP.offsets(1)
    p[o["Win"]] = 1.0
    p[o[("W", 0)] + 2 * H] = 1.0
    p[o[("W", 0)] + 3 * H] = -1.0
    p[o["wout"]] = 1.0
    v = np.random.default_rng(2).standard_normal((N, M))
    z, _ = LP.forward(p, 1, v.reshape(-1), grid, LP.neighbours(tri, M))
    prev = np.vstack([np.zeros((1, M)), v[:-1]])
    nxt = np.vstack([v[1:], np.zeros((1, M))])
    assert np.allclose(z.reshape(N, M), v + np.maximum(prev - nxt, 0.0), rtol=0, atol=1e-13)


def test_time_features_and_scale():
    """No layers, Win passes the step-size features: z = s * (h_k + 2 h_{k+1}) / hbar + bias
    terms, with s the root mean square of v."""
    xyz, tri, grid = _mesh()
    M, N = len(xyz), len(grid)
    p = _zero(0); o = LP.offsets(0)
    p[o["Win"] + 0 * 3 + 1] = 1.0               # channel 0 <- h_k / hbar
    p[o["Win"] + 1 * 3 + 2] = 1.0               # channel 1 <- h_{k+1} / hbar
    p[o["bin"] + 2] = 0.25                      # channel 2 <- 0.25
    p[o["wout"] + 0] = 1.0; p[o["wout"] + 1] = 2.0; p[o["wout"] + 2] = -4.0
    v = np.random.default_rng(3).standard_normal(N * M) * 3.0
    s = np.sqrt(np.mean(v ** 2))
    z, _ = LP.forward(p, 0, v, grid, LP.neighbours(tri, M))
    h = np.diff(grid); hbar = grid[-1] / (N - 1)
    hk = np.concatenate([[0.0], h]); hk1 = np.concatenate([h, [0.0]])
    ref = s * ((hk + 2 * hk1) / hbar - 1.0)
    assert np.allclose(z.reshape(N, M), ref[:, None], rtol=0, atol=1e-13)
    z0, c0 = LP.forward(p, 0, np.zeros(N * M), grid, LP.neighbours(tri, M))
    assert not z0.any() and not LP.backward(c0, np.ones(N * M)).any()


def _random_params(layers, seed, scale=0.15):
    return (np.random.default_rng(seed).standard_normal(LP.num_params(layers)) * scale).astype(np.float32)


def test_positive_homogeneity_and_relabelling():
    xyz, tri, grid = _mesh()
    M, N = len(xyz), len(grid)
    p = _random_params(3, 4)
    v = np.random.default_rng(5).standard_normal(N * M)
    z, _ = LP.forward(p, 3, v, grid, LP.neighbours(tri, M))
    z2, _ = LP.forward(p, 3, 7.5 * v, grid, LP.neighbours(tri, M))
    assert np.allclose(z2, 7.5 * z, rtol=1e-13, atol=1e-13 * np.abs(z).max())
    perm = np.random.default_rng(6).permutation(M)       # new label of old vertex j is perm[j]
    inv = np.argsort(perm)
    tri2 = perm[tri]
    v2 = v.reshape(N, M)[:, inv].reshape(-1)
    z3, _ = LP.forward(p, 3, v2, grid, LP.neighbours(tri2, M))
    assert np.allclose(z3.reshape(N, M), z.reshape(N, M)[:, inv], rtol=1e-13, atol=1e-13 * np.abs(z).max())


def test_gradient_finite_differences():
    """Analytic gradient of <dz, z(params)> against central differences (exact parameters)."""
    xyz, tri, grid = icosphere(0)[0], icosphere(0)[1], graded_grid(5, 2.0, seed=1)
    M, N = len(xyz), len(grid)
    L = 2
    nb = LP.neighbours(tri, M)
    p = LP.bf16_round(_random_params(L, 7, 0.3)).astype(np.float64)
    rng = np.random.default_rng(8)
    v = rng.standard_normal(N * M)
    dz = rng.standard_normal(N * M)
    _, cache = LP.forward(p, L, v, grid, nb, exact=True)
    g = LP.backward(cache, dz)
    o = LP.offsets(L)
    idx = list(rng.choice(LP.num_params(L), 60, replace=False))
    idx += [o["Win"] + 5, o["bin"] + 3, o[("b", 1)] + 7, o["wout"] + 11, o[("W", 1)] + 3 * H + 9]
    eps = 1e-6
    checked = 0
    for q in idx:
        pp = p.copy(); pp[q] += eps
        pm = p.copy(); pm[q] -= eps
        fp = dz @ LP.forward(pp, L, v, grid, nb, exact=True)[0]
        fm = dz @ LP.forward(pm, L, v, grid, nb, exact=True)[0]
        fd = (fp - fm) / (2 * eps)
        assert abs(fd - g[q]) <= 1e-6 * max(1.0, abs(g[q])), (q, fd, g[q])
        checked += 1
    assert checked == len(idx)
    assert np.abs(g).max() > 1e-3
