"""Pin of the oracle's cell sort against library routines: the permutation is
numpy's stable argsort and cell_start is the prefix sum of numpy's bincount."""
import numpy as np
import pytest

import oracle as O
from paper_2305_05600_amd import workloads as W


@pytest.mark.parametrize("ncell,n,seed", [(1, 10, 0), (35, 1000, 1), (1024, 65536, 2),
                                          (4096, 3, 3), (10, 0, 4)])
def test_sort_matches_stable_argsort(ncell, n, seed):
    cfg = W.Config(name="s", ndim=2, nx=ncell, ny=1, nz=1, dx=1, dy=1, dz=1, dt=1, nsub=1)
    rng = np.random.Generator(np.random.PCG64(seed))
    key = rng.integers(0, ncell, n).astype(np.int32)
    if n > 100:
        key[: n // 2] = np.sort(key[: n // 2])  # long runs of equal keys
    perm, cs = O.sort(cfg, key)
    assert np.array_equal(perm, np.argsort(key, kind="stable"))
    expect = np.concatenate([[0], np.cumsum(np.bincount(key, minlength=ncell))])
    assert np.array_equal(cs, expect)
