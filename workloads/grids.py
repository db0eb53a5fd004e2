"""Time grids t_0 = 0 < t_1 < ... < t_{N-1} = T (N nodes, one temporal basis per node)."""
import numpy as np


def equidistant_grid(N, T):
    """t_i = i T / (N - 1)."""
    t = np.linspace(0.0, T, N)
    t[-1] = T
    return t


def graded_grid(N, T, seed, ratio=4.0):
    """Nonequidistant grid whose step sizes span exactly a factor `ratio`.

    u_1..u_{N-1} ~ U(0,1) i.i.d. (numpy PCG64, `seed`), rescaled affinely to span [0,1];
    h_j = ratio**u_j; the steps are then scaled to sum to T."""
    rng = np.random.default_rng(seed)
    u = rng.random(N - 1)
    u = (u - u.min()) / (u.max() - u.min())
    h = ratio ** u
    h *= T / h.sum()
    t = np.concatenate([[0.0], np.cumsum(h)])
    t[-1] = T
    return t
