"""The seeded synthetic inputs: closed, outward-oriented meshes of the stated sizes, graded grids."""
import numpy as np
import pytest

from workloads import geodesic_sphere, graded_grid, icosphere, torus


def _closed_outward(xyz, tri):
    edges = {}
    for a, b, c in tri:
        for u, v in ((a, b), (b, c), (c, a)):
            edges[(u, v)] = edges.get((u, v), 0) + 1
    closed = all(n == 1 for n in edges.values()) and all((v, u) in edges for (u, v) in edges)
    P = xyz[tri]
    vol = np.einsum("ij,ij->i", P[:, 0], np.cross(P[:, 1], P[:, 2])).sum() / 6.0
    return closed, vol


@pytest.mark.parametrize("nu", [1, 4, 5, 7, 12])
def test_geodesic_sphere(nu):
    xyz, tri = geodesic_sphere(nu)
    assert len(tri) == 20 * nu * nu and len(xyz) == 10 * nu * nu + 2
    assert np.allclose(np.linalg.norm(xyz, axis=1), 1.0, atol=1e-15)
    closed, vol = _closed_outward(xyz, tri)
    assert closed and 0.6 * 4.18879 < vol < 4.18879          # inscribed, positive (outward) volume
    if nu == 4:                                              # the same surface as two 4-way refinements
        x2, t2 = icosphere(2)
        assert len(t2) == len(tri)
        d = np.linalg.norm(xyz[:, None, :] - x2[None, :, :], axis=2).min(axis=1)
        assert d.max() < 0.06                                # same vertex count, nearby (not identical) points


def test_icosphere_and_torus_closed():
    for xyz, tri in (icosphere(2), torus(16, 8)):
        closed, vol = _closed_outward(xyz, tri)
        assert closed and vol > 0.0


def test_graded_grid_ratio():
    t = graded_grid(64, 8.0, seed=2)
    h = np.diff(t)
    assert t[0] == 0.0 and abs(t[-1] - 8.0) < 1e-12 and np.all(h > 0)
    assert abs(h.max() / h.min() - 4.0) < 1e-9


def test_bench_refuses_several_gpus():
    """The benchmark measures one GPU: --gpus 2 ends at once with a message and status 2, before
    anything touches a device."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=300)
    assert res.returncode == 2
    assert "one GPU" in json.loads(res.stdout.strip().splitlines()[-1])["error"]
