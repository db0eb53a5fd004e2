"""GPU path (libtdbem through its C ABI) against the CPU oracle on the same seeded inputs.

Tolerances: blocks of eq. (MatrixEntries) to 1e-11 relative per block (max norm); the time
kernel tables to 1e-11 (psi) and 1e-12 (tilde psi) of each kernel's maximum; RHS and matvec to
1e-13; solves to their residual tolerance.  Integer work (quadrature-point counts) is exact.
The mixed-precision form (FP64 quadrature, FP32 storage of the assembled entries, FP64 solver) is
held to MIXED_TOL relative per block.
"""
import numpy as np
import pytest

from tests.conftest import gpu_available, integrated_node_blocks
from workloads import equidistant_grid, graded_grid, get_config, icosphere, torus

pytestmark = pytest.mark.gpu

BLOCK_TOL = 1e-11
# FP32 storage rounds the contributions of every tile into its entries (2^-24 relative each, a
# few dozen FP32 additions per entry): ~1e-6 of the block maximum at worst
MIXED_TOL = 2e-6


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


def gpu_blocks(ctx, N, M):
    K, I, J, L = np.meshgrid(np.arange(N), np.arange(N), np.arange(M), np.arange(M), indexing="ij")
    return ctx.get_entries(K.ravel(), I.ravel(), J.ravel(), L.ravel()).reshape(N, N, M, M)


def assert_blocks_close(G, A, tol=BLOCK_TOL):
    N = A.shape[0]
    worst = 0.0
    for k in range(N):
        for i in range(N):
            sc = np.abs(A[k, i]).max()
            if sc == 0.0:
                assert np.all(G[k, i] == 0.0), (k, i)
                continue
            worst = max(worst, np.abs(G[k, i] - A[k, i]).max() / sc)
    assert worst <= tol, worst
    return worst


# --- time kernels ----------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["eq10", "graded64", "eq5erf"])
def test_kernel_tables_against_oracle(ctx, oracle_mod, name):
    """Piecewise Chebyshev tables (Section 3.1) against direct quadrature of eq. (psis),
    including points outside the support (exact zeros) and next to the support ends."""
    grid, kind = {"eq10": (equidistant_grid(10, 4.0), "bump"), "graded64": (graded_grid(64, 8.0, seed=2), "bump"),
                  "eq5erf": (equidistant_grid(5, 3.0), "erf")}[name]
    xyz, tri = icosphere(1)
    ctx.set_mesh(xyz, tri)
    ctx.set_time_grid(grid, kind)
    ctx.assemble()
    N = len(grid)
    rng = np.random.default_rng(10)
    ks, is_, rs = [], [], []
    while len(rs) < 400:
        k = int(rng.integers(0, N)); i = int(rng.integers(max(0, k - 6), min(N, k + 3)))
        lo, hi = oracle_mod.support(grid, k, i)
        top = min(hi, 2.0) if hi > lo else 2.0
        u = rng.random()
        r = rng.uniform(lo, top) if u < 0.8 else (lo + 1e-7 * rng.random() if u < 0.9 else rng.uniform(top, top + 0.3))
        ks.append(k); is_.append(i); rs.append(r)
    ref = np.array([oracle_mod.psi(grid, k, i, r, kind) for k, i, r in zip(ks, is_, rs)])
    ps, pt = ctx.eval_kernels(ks, is_, rs)
    scale = {}
    for k, i in set(zip(ks, is_)):
        lo, hi = oracle_mod.support(grid, k, i)
        if hi <= lo:
            scale[(k, i)] = (1.0, 1.0)
            continue
        v = np.abs([oracle_mod.psi(grid, k, i, x, kind) for x in np.linspace(lo, min(hi, 2.0), 60)[1:-1]]).max(0)
        scale[(k, i)] = (max(v[0], 1e-300), max(v[1], 1e-300))
    for s in range(len(rs)):
        sc = scale[(ks[s], is_[s])]
        assert abs(ps[s] - ref[s, 0]) <= 1e-11 * sc[0], (ks[s], is_[s], rs[s], ps[s], ref[s])
        assert abs(pt[s] - ref[s, 1]) <= 1e-12 * sc[1], (ks[s], is_[s], rs[s], pt[s], ref[s])
        lo, hi = oracle_mod.support(grid, ks[s], is_[s])
        if not (lo < rs[s] < hi):      # outside the open support both sides are exact zeros
            assert ps[s] == 0.0 and pt[s] == 0.0 and ref[s, 0] == 0.0 and ref[s, 1] == 0.0


# --- assembled blocks ------------------------------------------------------------------------
def _two_triangles(kind):
    """Two flat triangles sharing an edge, a vertex, or nothing; a single triangle."""
    P = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.3, 0.9, 0.1], [1.2, 0.8, 0.4], [1.9, 0.1, 0.3],
                  [2.6, 0.9, -0.2], [2.0, 1.7, 0.5]])
    if kind == "single":
        return P[:3], np.array([[0, 1, 2]])
    if kind == "edge":
        return P[:4], np.array([[0, 1, 2], [1, 3, 2]])
    if kind == "vertex":
        return P[:5], np.array([[0, 1, 2], [1, 4, 3]])
    return P, np.array([[0, 1, 2], [4, 5, 6]])


@pytest.mark.parametrize("kind", ["single", "edge", "vertex", "apart"])
def test_two_triangle_blocks(ctx, oracle_mod, kind):
    """Each Sauter-Schwab kind and the regular rule in isolation (N = 4 graded, bump)."""
    xyz, tri = _two_triangles(kind)
    grid = graded_grid(4, 2.5, seed=21)
    ctx.set_mesh(xyz, tri)
    ctx.set_time_grid(grid, "bump")
    ctx.assemble()
    A = oracle_mod.assemble_dense(xyz, tri, grid)
    assert_blocks_close(gpu_blocks(ctx, len(grid), len(xyz)), A)


@pytest.mark.parametrize("case", ["sphere20_eq5_erf", "torus24_graded5_ss3"])
def test_small_meshes_every_block(tb, oracle_mod, case):
    """Every entry of every block on closed meshes small enough for the dense oracle."""
    if case == "sphere20_eq5_erf":
        c = get_config("sphere20_eq5_erf")
        xyz, tri = c["mesh"]; grid = c["grid"]; kind = "erf"; order = 4
    else:
        xyz, tri = torus(4, 3)
        grid = graded_grid(5, 2.5, seed=22); kind = "bump"; order = 3
    ctx = tb.Context(0, ss_order=order)
    ctx.set_mesh(xyz, tri)
    ctx.set_time_grid(grid, kind)
    rep = ctx.assemble()
    A = oracle_mod.assemble_dense(xyz, tri, grid, kind=kind, ss_order=order)
    G = gpu_blocks(ctx, len(grid), len(xyz))
    assert_blocks_close(G, A)
    # the method's quadrature-point count, by brute force on the CPU
    assert rep["quad_evals"] == oracle_mod.count_quad_evals(xyz, tri, grid, ss_order=order,
                                                            node_blocks=integrated_node_blocks(grid))
    ctx.close()


def test_tile_shapes_every_block(tb, oracle_mod):
    """Both tile shapes of the regular-pair kernel (4 x 8 and 8 x 8 triangles), forced in turn, on a
    70-triangle torus (ragged in both shapes): every block against the oracle, the exact
    quadrature-point count; then the timed choice reports an estimate for each shape."""
    xyz, tri = torus(7, 5)
    grid = graded_grid(6, 3.0, seed=23)
    T = oracle_mod.fast_tables(xyz, grid, "bump")
    A = oracle_mod.assemble_dense(xyz, tri, grid, tables=T)
    count = oracle_mod.count_quad_evals(xyz, tri, grid)
    ctx = tb.Context(0)
    ctx.set_mesh(xyz, tri)
    ctx.set_time_grid(grid, "bump")
    blocks = {}
    for v, shape in ((0, (4, 8)), (1, (8, 8))):
        assert ctx.assemble_set_tiles(v) == 2
        rep = ctx.assemble()
        assert ctx.assemble_tuning()[0] == shape
        blocks[v] = gpu_blocks(ctx, len(grid), len(xyz))
        assert_blocks_close(blocks[v], A)
        assert rep["quad_evals"] == count and rep["blocks_reused"] == 0
    assert np.abs(blocks[0] - blocks[1]).max() <= 1e-13 * np.abs(blocks[0]).max()
    ctx.assemble_set_tiles(-1)
    ctx.assemble()
    shape, ms = ctx.assemble_tuning()
    assert shape in ((4, 8), (8, 8)) and min(ms) > 0.0
    with pytest.raises(tb.TdbemError) as e:
        ctx.assemble_set_tiles(2)
    assert e.value.status == -1
    ctx.close()


@pytest.mark.parametrize("case", ["sphere320_eq10", "sphere80_eq7_p1"])
def test_equal_block_reuse(tb, oracle_mod, case):
    """Equidistant grids, where the assembly copies equal blocks (eq. (relationAtildeBlock)) instead
    of integrating them: every block against the oracle (which integrates every block), the
    quadrature-point count over the integrated node blocks only, the same blocks as an assembly
    with the copies switched off (which counts every block), and FP32 storage with copies."""
    if case == "sphere320_eq10":
        c = get_config("sphere320_eq10")
        (xyz, tri), grid, p = c["mesh"], c["grid"], 0
    else:
        (xyz, tri), grid, p = icosphere(1), equidistant_grid(7, 3.0), 1
    L, M = len(grid) * (p + 1), len(xyz)
    A = oracle_mod.assemble_dense(xyz, tri, grid, tables=oracle_mod.fast_tables(xyz, grid, p=p), p=p)
    ctx = tb.Context(0)
    ctx.set_mesh(xyz, tri)
    ctx.set_time_grid(grid, "bump", p=p)
    rep = ctx.assemble()
    assert rep["blocks_reused"] > 0
    G = gpu_blocks(ctx, L, M)
    assert_blocks_close(G, A)
    assert rep["quad_evals"] == oracle_mod.count_quad_evals(xyz, tri, grid, p=p,
                                                            node_blocks=integrated_node_blocks(grid))
    ctx.set_block_reuse(0)
    rep0 = ctx.assemble()
    assert rep0["blocks_reused"] == 0
    assert rep0["quad_evals"] == oracle_mod.count_quad_evals(xyz, tri, grid, p=p) > rep["quad_evals"]
    G0 = gpu_blocks(ctx, L, M)
    assert np.abs(G - G0).max() <= 1e-13 * np.abs(G0).max()
    ctx.set_block_reuse(1)
    repm = ctx.assemble(tb.MIXED)
    assert repm["blocks_reused"] == rep["blocks_reused"]
    assert_blocks_close(gpu_blocks(ctx, L, M), A, tol=MIXED_TOL)
    with pytest.raises(tb.TdbemError) as e:
        ctx.set_block_reuse(2)
    assert e.value.status == -1
    ctx.close()


def test_deterministic_assembly(tb, oracle_mod):
    """The deterministic mode (fixed-point integer atomics): two assemblies give bitwise the same
    storage, every block matches the oracle (1e-11) and the ordinary assembly (1e-13 of the largest
    entry), with the exact count; on the 5120/64 workload 200000 sampled entries are bitwise equal
    between two runs and within 1e-13 of the ordinary assembly, while two ordinary runs agree to
    1e-14.  FP32 storage is refused in this mode."""
    xyz, tri = torus(7, 5)
    grid = graded_grid(6, 3.0, seed=23)
    A = oracle_mod.assemble_dense(xyz, tri, grid, tables=oracle_mod.fast_tables(xyz, grid, "bump"))
    det = tb.Context(0, deterministic=True)
    ordi = tb.Context(0)
    for c in (det, ordi):
        c.set_mesh(xyz, tri)
        c.set_time_grid(grid, "bump")
    r1 = det.assemble()
    G1 = gpu_blocks(det, len(grid), len(xyz))
    r2 = det.assemble()
    G2 = gpu_blocks(det, len(grid), len(xyz))
    assert np.array_equal(G1.view(np.int64), G2.view(np.int64))
    assert r1["quad_evals"] == r2["quad_evals"] == oracle_mod.count_quad_evals(xyz, tri, grid)
    assert_blocks_close(G1, A)
    ordi.assemble()
    G0 = gpu_blocks(ordi, len(grid), len(xyz))
    assert np.abs(G1 - G0).max() <= 1e-13 * np.abs(G0).max()
    with pytest.raises(tb.TdbemError) as e:
        det.assemble(tb.MIXED)
    assert e.value.status == -1
    c5 = get_config("sphere5120_graded64")
    (xyz, tri), grid = c5["mesh"], c5["grid"]
    for c in (det, ordi):
        c.set_mesh(xyz, tri)
        c.set_time_grid(grid, c5["cutoff"])
    rng = np.random.default_rng(71)
    M, N = len(xyz), len(grid)
    K = rng.integers(0, N, 200000); I = np.clip(K - rng.integers(-1, 6, 200000), 0, N - 1)
    J = rng.integers(0, M, 200000); L = rng.integers(0, M, 200000)
    e = []
    for c in (det, det, ordi, ordi):
        c.assemble()
        e.append(c.get_entries(K, I, J, L))
    sc = np.abs(e[2]).max()
    assert np.array_equal(e[0].view(np.int64), e[1].view(np.int64))
    assert np.abs(e[0] - e[2]).max() <= 1e-13 * sc
    assert np.abs(e[2] - e[3]).max() <= 1e-14 * sc
    det.close()
    ordi.close()


def _sample_pairs(xyz, tri, rng, n_far):
    """Vertex pairs (j, l): the diagonal, edge neighbours, one at distance ~1, far ones."""
    l0 = int(tri[0][0])
    d = np.linalg.norm(xyz - xyz[l0], axis=1)
    js = [l0, int(tri[0][1]), int(np.argmin(np.abs(d - 1.0))), int(np.argmax(d))]
    js += [int(x) for x in rng.integers(0, len(xyz), n_far)]
    return np.array(js), np.full(len(js), l0)


@pytest.mark.parametrize("name", ["sphere320_eq10", "sphere5120_graded64"])
def test_sampled_entries_full_size(ctx, oracle_mod, name):
    """Full-size workloads (the benchmark's assembly launch): all (k, i) blocks at sampled vertex
    pairs, each entry formed by the oracle from its triangle pairs one by one."""
    c = get_config(name)
    xyz, tri = c["mesh"]; grid = c["grid"]
    ctx.set_mesh(xyz, tri)
    ctx.set_time_grid(grid, c["cutoff"])
    ctx.assemble()
    N = len(grid)
    sj, sl = _sample_pairs(xyz, tri, np.random.default_rng(5), 2 if name == "sphere320_eq10" else 0)
    if name == "sphere5120_graded64":
        sj, sl = sj[:3], sl[:3]
    ref = oracle_mod.assemble_entries(xyz, tri, grid, sj, sl, kind=c["cutoff"])
    K, I = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    for s in range(len(sj)):
        got = ctx.get_entries(K.ravel(), I.ravel(), sj[s], sl[s]).reshape(N, N)
        sc = np.abs(ref[s]).max()
        assert np.abs(got - ref[s]).max() <= BLOCK_TOL * sc, (sj[s], sl[s])
        # block symmetry (exact) and the Hessenberg zeros
        got_t = ctx.get_entries(K.ravel(), I.ravel(), sl[s], sj[s]).reshape(N, N)
        assert np.array_equal(got, got_t)
        assert np.all(got[np.triu_indices(N, 2)] == 0.0)


@pytest.mark.parametrize("name", ["sphere320_eq10", "sphere5120_graded64"])
def test_mixed_sampled_entries(ctx, tb, oracle_mod, name):
    """Mixed precision against the FP64 oracle at sampled vertex pairs of every (k, i) block,
    with the exact block symmetry and Hessenberg zeros kept."""
    c = get_config(name)
    xyz, tri = c["mesh"]; grid = c["grid"]
    ctx.set_mesh(xyz, tri)
    ctx.set_time_grid(grid, c["cutoff"])
    ctx.assemble(tb.MIXED)
    N = len(grid)
    sj, sl = _sample_pairs(xyz, tri, np.random.default_rng(6), 4 if name == "sphere320_eq10" else 2)
    if name == "sphere5120_graded64":
        sj, sl = sj[:3], sl[:3]
    ref = oracle_mod.assemble_entries(xyz, tri, grid, sj, sl, kind=c["cutoff"])
    K, I = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    worst = 0.0
    for s in range(len(sj)):
        got = ctx.get_entries(K.ravel(), I.ravel(), sj[s], sl[s]).reshape(N, N)
        sc = np.abs(ref[s]).max()
        worst = max(worst, np.abs(got - ref[s]).max() / sc)
        got_t = ctx.get_entries(K.ravel(), I.ravel(), sl[s], sj[s]).reshape(N, N)
        assert np.array_equal(got, got_t)
        assert np.all(got[np.triu_indices(N, 2)] == 0.0)
    assert worst <= MIXED_TOL, worst


def test_mixed_torus_full_size(ctx, tb, oracle_mod):
    """The 20480-triangle torus with 128 graded bases in mixed precision (about 210 GB of FP32
    band storage, one launch of each assembly kernel): all (k, i) blocks at sampled vertex
    pairs against the FP64 oracle, Hessenberg zeros exact."""
    c = get_config("torus20480_graded128")
    xyz, tri = c["mesh"]; grid = c["grid"]
    ctx.set_mesh(xyz, tri)
    ctx.set_time_grid(grid, c["cutoff"])
    rep = ctx.assemble(tb.MIXED)
    assert rep["quad_evals"] > 4e12
    N = len(grid)
    l0 = int(tri[0][0])
    d = np.linalg.norm(xyz - xyz[l0], axis=1)
    sj = np.array([int(tri[0][1]), int(np.argmin(np.abs(d - 1.0))), int(np.argmax(d))])
    sl = np.full(len(sj), l0)
    ref = oracle_mod.assemble_entries(xyz, tri, grid, sj, sl, kind=c["cutoff"])
    K, I = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    for s in range(len(sj)):
        got = ctx.get_entries(K.ravel(), I.ravel(), sj[s], sl[s]).reshape(N, N)
        assert np.abs(got - ref[s]).max() <= MIXED_TOL * np.abs(ref[s]).max(), (sj[s], sl[s])
        assert np.all(got[np.triu_indices(N, 2)] == 0.0)
    ctx.set_mesh(*icosphere(0))            # release the band storage
    ctx.set_time_grid(equidistant_grid(3, 2.0))
    ctx.assemble()


def test_mixed_solve_config1(ctx, tb):
    """The mixed operator's solution of the 320-triangle workload to 1e-8 (its own residual),
    then its residual against the FP64 operator and its distance to the FP64 solution."""
    import torch
    c = get_config("sphere320_eq10")
    xyz, tri = c["mesh"]
    ctx.set_mesh(xyz, tri); ctx.set_time_grid(c["grid"], "bump")
    ctx.assemble(tb.MIXED)
    g = ctx.rhs_plane_pulse(c["direction"], c["t0"], c["width"])
    a32, rep = ctx.solve(g, tol=1e-8, precond_inner=(2, 10), max_it=4000)
    assert rep["converged"]
    ctx.assemble(tb.FP64)
    a64, rep = ctx.solve(g, tol=1e-8, precond_inner=(2, 10), max_it=4000)
    assert rep["converged"]
    r = g - ctx.matvec(a32)
    assert torch.linalg.norm(r).item() <= 1e-5 * torch.linalg.norm(g).item()
    assert torch.linalg.norm(a32 - a64).item() <= 1e-4 * torch.linalg.norm(a64).item()


# --- RHS, matvec, solve ----------------------------------------------------------------------
@pytest.fixture(scope="module")
def small_system(tb, oracle_mod):
    c = get_config("sphere20_eq5_erf")
    xyz, tri = c["mesh"]
    A = oracle_mod.assemble_dense(xyz, tri, c["grid"], kind="erf")
    g = oracle_mod.rhs_plane_pulse(xyz, tri, c["grid"], c["direction"], c["t0"], c["width"], kind="erf")
    return c, A, g


def test_rhs_and_matvec(ctx, oracle_mod, small_system):
    import torch
    c, A, g_ref = small_system
    xyz, tri = c["mesh"]; N, M = len(c["grid"]), len(xyz)
    ctx.set_mesh(xyz, tri); ctx.set_time_grid(c["grid"], "erf"); ctx.assemble()
    g = ctx.rhs_plane_pulse(c["direction"], c["t0"], c["width"]).cpu().numpy()
    assert np.abs(g - g_ref).max() <= 1e-13 * np.abs(g_ref).max()
    Af = oracle_mod.system_matrix(A)
    x = torch.from_numpy(np.random.default_rng(3).standard_normal(N * M)).cuda()
    y = ctx.matvec(x).cpu().numpy()
    yr = Af @ x.cpu().numpy()
    assert np.linalg.norm(y - yr) <= 1e-13 * np.linalg.norm(yr)
    for (k0, k1, i0, i1) in [(1, 3, 0, 2), (2, 5, 2, 5), (0, 5, 4, 5)]:
        xs = x[i0 * M:i1 * M].contiguous()
        ys = ctx.matvec_range(k0, k1, i0, i1, xs).cpu().numpy()
        ysr = Af[k0 * M:k1 * M, i0 * M:i1 * M] @ xs.cpu().numpy()
        assert np.linalg.norm(ys - ysr) <= 1e-13 * max(np.linalg.norm(ysr), 1e-300)


def test_matvec_free(ctx, tb, oracle_mod, small_system):
    """The matrix-free FP64 product against the oracle's dense system, and at full size against
    the stored FP64 operator (same quadrature, other summation order)."""
    import torch
    c, A, g_ref = small_system
    xyz, tri = c["mesh"]; N, M = len(c["grid"]), len(xyz)
    ctx.set_mesh(xyz, tri); ctx.set_time_grid(c["grid"], "erf")
    Af = oracle_mod.system_matrix(A)
    x = torch.from_numpy(np.random.default_rng(4).standard_normal(N * M)).cuda()
    y, rep = ctx.matvec_free(x)
    yr = Af @ x.cpu().numpy()
    assert np.linalg.norm(y.cpu().numpy() - yr) <= 1e-13 * np.linalg.norm(yr)
    assert rep["quad_evals"] == oracle_mod.count_quad_evals(xyz, tri, c["grid"]) and rep["bytes_matrix"] == 0
    c2 = get_config("sphere5120_graded64")
    ctx.set_mesh(*c2["mesh"]); ctx.set_time_grid(c2["grid"], c2["cutoff"])
    ctx.assemble(tb.FP64)
    n = len(c2["grid"]) * len(c2["mesh"][0])
    x = torch.from_numpy(np.random.default_rng(5).standard_normal(n)).cuda()
    y_stored = ctx.matvec(x).clone()
    y_free, _ = ctx.matvec_free(x)
    assert torch.linalg.norm(y_free - y_stored).item() <= 1e-12 * torch.linalg.norm(y_stored).item()


def test_rhs_config1(ctx, oracle_mod):
    c = get_config("sphere320_eq10")
    xyz, tri = c["mesh"]
    ctx.set_mesh(xyz, tri); ctx.set_time_grid(c["grid"], "bump")
    g = ctx.rhs_plane_pulse(c["direction"], c["t0"], c["width"]).cpu().numpy()
    ref = oracle_mod.rhs_plane_pulse(xyz, tri, c["grid"], c["direction"], c["t0"], c["width"])
    assert np.abs(g - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("inner", [(), (2, 10), (5,)])
def test_solve_against_lu(ctx, oracle_mod, small_system, inner):
    """FGMRES (plain and with Algorithm 1) reaches the LU solution of the oracle's system."""
    import torch
    c, A, g_ref = small_system
    xyz, tri = c["mesh"]
    ctx.set_mesh(xyz, tri); ctx.set_time_grid(c["grid"], "erf"); ctx.assemble()
    Af = oracle_mod.system_matrix(A)
    ref = np.linalg.solve(Af, g_ref)
    kappa = np.linalg.cond(Af)
    alpha, rep = ctx.solve(torch.from_numpy(g_ref).cuda(), tol=1e-10, precond_inner=inner)
    a = alpha.cpu().numpy()
    assert rep["converged"] and rep["rel_residual"] <= 1e-10
    assert np.linalg.norm(g_ref - Af @ a) <= 1.01e-10 * np.linalg.norm(g_ref)
    assert np.linalg.norm(a - ref) <= kappa * 1e-10 * np.linalg.norm(ref)


def test_solve_progress(ctx):
    """The progress callback sees every outer iteration, with Givens estimates that never grow
    within one restart cycle."""
    c = get_config("sphere320_eq10")
    xyz, tri = c["mesh"]
    ctx.set_mesh(xyz, tri); ctx.set_time_grid(c["grid"], "bump"); ctx.assemble()
    g = ctx.rhs_plane_pulse(c["direction"], c["t0"], c["width"])
    seen = []
    alpha, rep = ctx.solve(g, tol=1e-8, restart=1000, precond_inner=(2, 10), max_it=500,
                           progress=lambda it, est: seen.append((it, est)))
    assert rep["converged"]
    assert [it for it, _ in seen] == list(range(1, rep["iterations"] + 1))
    est = [e for _, e in seen]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(est, est[1:]))
    assert est[-1] <= 1e-8


def test_solve_config1_to_1e8(ctx):
    """The 320-triangle, 10-basis workload solved to 1e-8 with Algorithm 1 (2 levels, (2, 10))."""
    import torch
    c = get_config("sphere320_eq10")
    xyz, tri = c["mesh"]
    ctx.set_mesh(xyz, tri); ctx.set_time_grid(c["grid"], "bump"); ctx.assemble()
    g = ctx.rhs_plane_pulse(c["direction"], c["t0"], c["width"])
    for inner in [(), (2, 10)]:
        alpha, rep = ctx.solve(g, tol=1e-8, precond_inner=inner, max_it=4000)
        r = g - ctx.matvec(alpha)
        assert rep["converged"]
        assert torch.linalg.norm(r).item() <= 1.01e-8 * torch.linalg.norm(g).item()


# --- error handling --------------------------------------------------------------------------
def test_error_paths(tb):
    import torch
    with pytest.raises(tb.TdbemError) as e:
        tb.Context(0, ss_order=6)            # Sauter-Schwab rules beyond 5 points per direction
    assert e.value.status == -1
    ctx = tb.Context(0)
    xyz, tri = icosphere(0)
    with pytest.raises(tb.TdbemError) as e:
        ctx.assemble()
    assert e.value.status == -6
    with pytest.raises(tb.TdbemError) as e:
        ctx.set_mesh(xyz, np.array([[0, 1, 99]]))
    assert e.value.status == -2
    with pytest.raises(tb.TdbemError) as e:
        ctx.set_mesh(xyz, np.array([[0, 1, 1]]))
    assert e.value.status == -2
    bad = xyz.copy(); bad[2] = bad[0] + 0.5 * (bad[1] - bad[0])
    with pytest.raises(tb.TdbemError) as e:
        ctx.set_mesh(bad, np.array([[0, 1, 2]]))
    assert e.value.status == -2
    with pytest.raises(tb.TdbemError) as e:
        ctx.set_time_grid(np.array([0.0, 1.0, 1.0]))
    assert e.value.status == -3
    with pytest.raises(tb.TdbemError) as e:
        ctx.set_time_grid(np.array([0.1, 1.0]))
    assert e.value.status == -3
    with pytest.raises(tb.TdbemError) as e:
        ctx.set_time_grid(np.array([0.0]))
    assert e.value.status == -3
    ctx.set_mesh(xyz, tri)
    ctx.set_time_grid(equidistant_grid(3, 2.0))
    x = torch.zeros(3 * len(xyz), dtype=torch.float64, device="cuda")
    with pytest.raises(tb.TdbemError) as e:
        ctx.matvec(x)
    assert e.value.status == -6
    ctx.assemble()
    import ctypes
    xp = ctypes.c_void_p(x.data_ptr())
    assert ctx.lib.tdbem_matvec_range(ctx.h, 2, 1, 0, 1, xp, xp) == -1      # empty k range
    assert ctx.lib.tdbem_matvec_range(ctx.h, 0, 4, 0, 1, xp, xp) == -1      # k1 > N
    assert ctx.lib.tdbem_matvec(ctx.h, None, xp) == -1
    g = ctx.rhs_plane_pulse([0.0, 0.0, 1.0], 1.0, 0.3)
    alpha, rep = ctx.solve(g, tol=1e-14, max_it=1)
    assert not rep["converged"] and rep["iterations"] == 1
    # zero right-hand side: alpha = 0 immediately
    alpha, rep = ctx.solve(torch.zeros_like(g), tol=1e-8)
    assert rep["converged"] and torch.count_nonzero(alpha).item() == 0
    ctx.close()
    ctx.close()   # double close is harmless
