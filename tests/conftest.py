import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build()
    return oracle


def integrated_node_blocks(grid):
    """Node blocks (test node, trial node) that an assembly integrates when it copies equal blocks
    (eq. (relationAtildeBlock), Section 5.1): on an equidistant grid the first two block columns,
    the last block row and the blocks (1, 2) and (N-2, N-1), 0-based (the blocks above the first
    superdiagonal are zero and count as integrated); None (every block) on any other grid."""
    import numpy as np
    g = np.asarray(grid, dtype=float)
    N = len(g)
    if N < 2 or np.abs(g - np.arange(N) * (g[-1] / (N - 1))).max() > 1e-12 * g[-1]:
        return None
    k, i = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    m = (i <= 1) | (k == N - 1) | (i > k + 1)
    if N >= 3:
        m[1, 2] = True
        m[N - 2, N - 1] = True
    return m
