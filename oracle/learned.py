"""CPU oracle of the learned variable preconditioner (not part of the paper).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: it shares no code with the GPU library.

Flexible GMRES (Saad 1993), which the paper adopts in Section 4.2 so that its block-Hessenberg
preconditioner may change from one iteration to the next, accepts any variable preconditioner.
This module defines one: a small message-passing network on the space-time graph of the
discretisation.  Its nodes are the unknowns (k, j) of the
block partition of eq. (A) (time basis b_k, spatial hat phi_j; vector index k*M + j).  A node
exchanges messages with its mesh neighbours (vertices sharing an edge) in the same time block and
with the nodes (k-1, j) and (k+1, j) of the neighbouring time blocks.

Definition (all arithmetic here in float64; the parameters are given as float32 and used after
rounding to bfloat16, as the GPU stores them):

    s        = sqrt(mean_n v_n^2)                          (the map is positively homogeneous)
    x_(k,j)  = [ v_(k,j) / s,  h_k / hbar,  h_{k+1} / hbar ]     h_k = t_k - t_{k-1} (0 outside),
                                                                 hbar = t_{N-1} / (N - 1)
    H0       = x Win^T + bin                                 Win: 64 x 3, bin: 64
    for layer l = 1..L:
      X      = [ H, mean over mesh neighbours of H, H at (k-1, j) (0 for k = 0),
                 H at (k+1, j) (0 for k = N-1) ]             256 features per node
      U      = X W_l^T + b_l                                 W_l: 64 x 256, b_l: 64
      H      = H + relu(U)
    z        = s * (H wout)                                  wout: 64

Parameter vector layout (float32, P = 256 + L*16448 + 64 entries): Win (row-major 64 x 3), bin,
then for every layer W_l (row-major 64 x 256, feature blocks in the order above) and b_l, then
wout.  The weight matrices and wout are rounded to bfloat16 before use; the biases are not.
"""
import numpy as np

HIDDEN = 64
FEATURES = 3


def num_params(layers):
    return HIDDEN * FEATURES + HIDDEN + layers * (HIDDEN * 4 * HIDDEN + HIDDEN) + HIDDEN


def offsets(layers):
    """Start of every parameter group in the flat vector."""
    o = {"Win": 0, "bin": HIDDEN * FEATURES}
    p = HIDDEN * FEATURES + HIDDEN
    for l in range(layers):
        o[("W", l)] = p
        o[("b", l)] = p + HIDDEN * 4 * HIDDEN
        p += HIDDEN * 4 * HIDDEN + HIDDEN
    o["wout"] = p
    return o


def bf16_round(a):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params, layers, exact=False):
    """Parameter groups as float64 arrays: weights bfloat16-rounded from float32, biases float32.
    exact=True takes the given values as they are (float64, no rounding)."""
    if exact:
        p = np.asarray(params, dtype=np.float64)
        rnd = lambda a: a.astype(np.float64)
    else:
        p = np.asarray(params, dtype=np.float32)
        rnd = bf16_round
    assert p.shape == (num_params(layers),)
    o = offsets(layers)
    g = {"Win": rnd(p[o["Win"]:o["Win"] + HIDDEN * FEATURES]).reshape(HIDDEN, FEATURES),
         "bin": p[o["bin"]:o["bin"] + HIDDEN].astype(np.float64),
         "wout": rnd(p[o["wout"]:o["wout"] + HIDDEN])}
    for l in range(layers):
        a = o[("W", l)]
        g[("W", l)] = rnd(p[a:a + HIDDEN * 4 * HIDDEN]).reshape(HIDDEN, 4 * HIDDEN)
        g[("b", l)] = p[o[("b", l)]:o[("b", l)] + HIDDEN].astype(np.float64)
    return g


def neighbours(tri, M):
    """Mesh neighbours of every vertex (vertices sharing an edge), sorted."""
    nb = [set() for _ in range(M)]
    for t in np.asarray(tri):
        for a in range(3):
            for b in range(3):
                if a != b:
                    nb[int(t[a])].add(int(t[b]))
    return [sorted(s) for s in nb]


def time_features(grid):
    t = np.asarray(grid, dtype=np.float64)
    N = len(t)
    hbar = t[-1] / (N - 1)
    f = np.zeros((N, 2))
    f[1:, 0] = np.diff(t) / hbar
    f[:-1, 1] = np.diff(t) / hbar
    return f


def _neighbour_mean(Hn, nbrs):
    """Hn: [N, M, C] -> mean over the mesh neighbours of every vertex."""
    out = np.zeros_like(Hn)
    for j, lst in enumerate(nbrs):
        if lst:
            out[:, j] = Hn[:, lst].mean(axis=1)
    return out


def _features(Hn, nbrs):
    N = Hn.shape[0]
    prev = np.zeros_like(Hn)
    nxt = np.zeros_like(Hn)
    if N > 1:
        prev[1:] = Hn[:-1]
        nxt[:-1] = Hn[1:]
    return np.concatenate([Hn, _neighbour_mean(Hn, nbrs), prev, nxt], axis=2)


def forward(params, layers, v, grid, nbrs, exact=False):
    """z = network(v) for one vector v of N*M values; returns (z, cache for backward).
    exact=True uses the parameters without bfloat16 rounding (for derivative checks)."""
    g = unpack(params, layers, exact)
    N, M = len(grid), len(nbrs)
    v = np.asarray(v, dtype=np.float64).reshape(N, M)
    s = np.sqrt(np.mean(v * v))
    if s == 0.0:
        return np.zeros(N * M), {"layers": layers, "zero": True}
    f = time_features(grid)
    x = np.concatenate([(v / s)[:, :, None], np.broadcast_to(f[:, None, :], (N, M, 2))], axis=2)
    H = x @ g["Win"].T + g["bin"]
    cache = {"g": g, "s": s, "x": x, "H": [H], "U": [], "nbrs": nbrs, "layers": layers}
    for l in range(layers):
        X = _features(H, nbrs)
        U = X @ g[("W", l)].T + g[("b", l)]
        H = H + np.maximum(U, 0.0)
        cache["U"].append(U)
        cache["H"].append(H)
    z = s * (H @ g["wout"])
    return z.reshape(-1), cache


def backward(cache, dz):
    """Gradient of <dz, z(params)> with respect to the flat parameter vector (float64).

    The scale s depends on v only, so it is a constant here; the bfloat16 rounding is treated
    as the identity (straight-through), so the gradient is taken at the rounded values."""
    layers = cache["layers"]
    grad = np.zeros(num_params(layers))
    if cache.get("zero"):
        return grad
    o = offsets(layers)
    g, s, nbrs = cache["g"], cache["s"], cache["nbrs"]
    Hs, Us = cache["H"], cache["U"]
    N, M = Hs[0].shape[:2]
    dzr = np.asarray(dz, dtype=np.float64).reshape(N, M)
    grad[o["wout"]:o["wout"] + HIDDEN] = np.einsum("km,kmc->c", s * dzr, Hs[-1])
    dH = (s * dzr)[:, :, None] * g["wout"][None, None, :]
    for l in reversed(range(layers)):
        H = Hs[l]
        X = _features(H, nbrs)
        dU = dH * (Us[l] > 0.0)
        a = o[("W", l)]
        grad[a:a + HIDDEN * 4 * HIDDEN] = np.einsum("kmo,kmc->oc", dU, X).reshape(-1)
        grad[o[("b", l)]:o[("b", l)] + HIDDEN] = dU.sum(axis=(0, 1))
        dX = dU @ g[("W", l)]                     # [N, M, 256]
        C = HIDDEN
        dHin = dH + dX[:, :, 0:C]
        dagg = dX[:, :, C:2 * C]
        for j, lst in enumerate(nbrs):            # agg(k, j) = mean_{j' in nbrs(j)} H(k, j')
            if lst:
                dHin[:, lst] += dagg[:, j][:, None, :] / len(lst)
        if N > 1:
            dHin[:-1] += dX[1:, :, 2 * C:3 * C]   # prev(k, j) = H(k-1, j)
            dHin[1:] += dX[:-1, :, 3 * C:4 * C]   # next(k, j) = H(k+1, j)
        dH = dHin
    grad[o["Win"]:o["Win"] + HIDDEN * FEATURES] = np.einsum("kmc,kmf->cf", dH, cache["x"]).reshape(-1)
    grad[o["bin"]:o["bin"] + HIDDEN] = dH.sum(axis=(0, 1))
    return grad


def residual_loss(apply_A, z, v):
    """Training loss of the preconditioner for one residual v: ||A z - v||^2 / ||v||^2."""
    r = apply_A(z) - v
    return float(r @ r) / float(v @ v)
