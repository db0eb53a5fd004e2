"""Arbitrary-precision reference values for the oracle pins (mpmath, 30 digits).

Written independently of the oracle: the bump cutoff is taken in its Shepard form
beta(u-1)/(beta(u-1)+beta(u)), derivatives of every basis come from mpmath's numerical
differentiation, and the time integrals use mpmath's tanh-sinh quadrature.
"""
import mpmath as mp

mp.mp.dps = 30


def beta(s):
    s = mp.mpf(s)
    if abs(s) >= 1:
        return mp.mpf(0)
    return mp.exp(-1 / (1 - s * s))


def F_bump(u):
    u = mp.mpf(u)
    if u <= 0:
        return mp.mpf(0)
    if u >= 1:
        return mp.mpf(1)
    return beta(u - 1) / (beta(u - 1) + beta(u))


def F_erf(u):
    u = mp.mpf(u)
    if u <= 0:
        return mp.mpf(0)
    if u >= 1:
        return mp.mpf(1)
    return mp.erf(2 * mp.atanh(2 * u - 1)) / 2 + mp.mpf(1) / 2


def make_basis(grid, kind):
    G = [mp.mpf(x) for x in grid]
    N = len(G)
    F = F_bump if kind == "bump" else F_erf

    def mu(j, t):
        if t < 0:
            return mp.mpf(0)
        if j >= 1 and G[j - 1] < t <= G[j]:
            return F((t - G[j - 1]) / (G[j] - G[j - 1]))
        if j <= N - 2 and G[j] <= t < G[j + 1]:
            return 1 - F((t - G[j]) / (G[j + 1] - G[j]))
        if j == N - 1 and t > G[N - 1]:
            return mp.mpf(1)
        return mp.mpf(0)

    def b(j, t):
        t = mp.mpf(t)
        if j == 0:
            if t <= 0:
                return mp.mpf(0)
            return 8 * (t / (G[1] - G[0])) ** 2 * mu(0, t)
        return mu(j, t)

    return G, mu, b


def psi_ref(grid, k, i, r, kind="bump"):
    """(psi_{k,i}(r), tilde psi_{k,i}(r)) = int_0^T (b_i''(t-r), b_i(t-r)) b_k'(t) dt."""
    G, mu, b = make_basis(grid, kind)
    N = len(G)
    r = mp.mpf(r)
    pts = {mp.mpf(0), G[-1]}
    for a in range(N):
        pts.add(G[a])
        if 0 < G[a] + r < G[-1]:
            pts.add(G[a] + r)
    if 0 < r < G[-1]:
        pts.add(r)
    pts = sorted(pts)
    lo = G[max(k - 1, 0)]
    hi = G[min(k + 1, N - 1)]
    pts = [p for p in pts if lo <= p <= hi]
    d1 = lambda j, t: mp.diff(lambda s: b(j, s), t)
    d2 = lambda j, t: mp.diff(lambda s: b(j, s), t, 2)
    ps = mp.quad(lambda t: d2(i, t - r) * d1(k, t), pts)
    pt = mp.quad(lambda t: b(i, t - r) * d1(k, t), pts)
    return float(ps), float(pt)
