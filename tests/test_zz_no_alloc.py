"""The allocation-free entry query (tdbem_get_entries_noalloc) against tdbem_get_entries, through
the C ABI: two calls in a row, the second with fewer entries, results identical (the same kernel
on the same stored values), and the size limit."""
import ctypes

import numpy as np
import pytest

from tests.conftest import gpu_available
from workloads import get_config

pytestmark = pytest.mark.gpu


def _call(ctx, fn, k, i, j, l):
    P = ctypes.POINTER
    out = np.full(len(k), np.nan)
    arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in (k, i, j, l)]
    st = fn(ctx.h, len(k), *[a.ctypes.data_as(P(ctypes.c_int32)) for a in arrs], out.ctypes.data_as(P(ctypes.c_double)))
    return st, out


def test_noalloc_entries_match_allocating_query():
    if not gpu_available():
        pytest.skip("no HIP device")
    import paper_1503_07221_amd as tb
    c = get_config("sphere320_eq10")
    ctx = tb.Context(0)
    ctx.set_mesh(*c["mesh"]); ctx.set_time_grid(c["grid"], c["cutoff"]); ctx.assemble(tb.FP64)
    N, M = len(c["grid"]), len(c["mesh"][0])
    rng = np.random.default_rng(17)
    for n in (40000, 123):
        k = rng.integers(0, N, n); i = np.clip(k - rng.integers(-1, 4, n), 0, N - 1)
        j = rng.integers(0, M, n); l = rng.integers(0, M, n)
        st1, ref = _call(ctx, ctx.lib.tdbem_get_entries, k, i, j, l)
        st2, got = _call(ctx, ctx.lib.tdbem_get_entries_noalloc, k, i, j, l)
        assert st1 == 0 and st2 == 0
        assert np.array_equal(got, ref)
        assert np.count_nonzero(ref) > n // 10
    n = 65537
    z = np.zeros(n, dtype=np.int32)
    st, _ = _call(ctx, ctx.lib.tdbem_get_entries_noalloc, z, z, z, z)
    assert st == -1 and "65536" in ctx.lib.tdbem_last_error(ctx.h).decode()
    ctx.close()
