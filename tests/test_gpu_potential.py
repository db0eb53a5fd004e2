"""Retarded double layer potential (eq. (RetardedPotential)) on the GPU against the CPU oracle.

Same 7-point rule and time bases on both sides, so the values agree to rounding: 1e-12 of the
largest |u| of the case (the sums over triangles and points change order).  Point counts are not
multiples of the kernel's 256-point workgroups, time counts not multiples of its 8-time columns;
the times include 0 (u = 0) and T.
"""
import numpy as np
import pytest

from tests.conftest import gpu_available
from workloads import get_config, graded_grid, icosphere

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tb():
    if not gpu_available():
        pytest.skip("no HIP device")
    import paper_1503_07221_amd as tb
    tb.load_library()
    return tb


@pytest.fixture(scope="module")
def ctx(tb):
    c = tb.Context(0)
    yield c
    c.close()


def _points(rng, n):
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rad = np.where(rng.random(n) < 0.5, rng.uniform(0.0, 0.7, n), rng.uniform(1.3, 3.0, n))
    return d * rad[:, None]


def test_potential_small(ctx, oracle_mod):
    import torch
    xyz, tri = icosphere(2)
    grid = graded_grid(12, 6.0, seed=5)
    M, N = len(xyz), len(grid)
    ctx.set_mesh(xyz, tri); ctx.set_time_grid(grid)
    rng = np.random.default_rng(51)
    alpha = rng.standard_normal(N * M)
    pts = _points(rng, 40)
    times = np.concatenate([[0.0], np.sort(rng.uniform(0.0, 6.0, 11)), [6.0]])
    u = ctx.potential_dl(torch.from_numpy(alpha).cuda(), pts, times).cpu().numpy()
    ur = oracle_mod.potential_dl(xyz, tri, grid, alpha, pts, times)
    assert np.all(u[0] == 0.0)
    assert np.abs(u - ur).max() <= 1e-12 * np.abs(ur).max(), np.abs(u - ur).max() / np.abs(ur).max()


def test_potential_full_size_sampled(ctx, oracle_mod):
    import torch
    c = get_config("sphere5120_graded64")
    xyz, tri = c["mesh"]
    grid = c["grid"]
    M, N = len(xyz), len(grid)
    ctx.set_mesh(xyz, tri); ctx.set_time_grid(grid, c["cutoff"])
    rng = np.random.default_rng(52)
    alpha = rng.standard_normal(N * M)
    pts = _points(rng, 300)
    times = np.sort(rng.uniform(0.5, 8.0, 9))
    u = ctx.potential_dl(torch.from_numpy(alpha).cuda(), pts, times).cpu().numpy()
    pick = [0, 77, 150, 299]
    ur = oracle_mod.potential_dl(xyz, tri, grid, alpha, pts[pick], times)
    assert np.abs(u[:, pick] - ur).max() <= 1e-12 * np.abs(ur).max(), np.abs(u[:, pick] - ur).max() / np.abs(ur).max()


def test_potential_errors(ctx, tb):
    import torch
    xyz, tri = icosphere(1)
    grid = graded_grid(5, 2.0, seed=1)
    ctx.set_mesh(xyz, tri); ctx.set_time_grid(grid)
    a = torch.zeros(5 * len(xyz), dtype=torch.float64, device="cuda")
    with pytest.raises(tb.TdbemError) as e:
        ctx.potential_dl(a, np.zeros((2, 3)) + 3.0, [2.5])
    assert e.value.status == -1
