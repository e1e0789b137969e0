"""The allocation-free sort (polypic_sort_noalloc) against polypic_sort, through the C ABI.

Both sorts must give the same keys and permutation bit for bit (the sort is integer
work).  Two calls in a row share the library's static workspace: the first at the
largest size it accepts, the second smaller, so a stale word of the first call would
show in the second.  The smaller one is also checked against the oracle's stable
argsort.
"""
import numpy as np
import pytest
import torch

from oracle import polypic_oracle as O
from tests.gpu_util import dev, host, note, oracle_grid, require_gpu

pytestmark = pytest.mark.gpu


def _positions(seed, n_cells, P):
    rng = np.random.default_rng(seed)
    dx = 1.0 / n_cells
    return (2 * dx + rng.random((3, P)) * (n_cells * dx)).astype(np.float32), dx


def _both(pp, g, x):
    P = x.shape[1]
    xd = dev(x)
    keys_ref = torch.empty(P, dtype=torch.int32, device="cuda")
    perm_ref = torch.empty(P, dtype=torch.int32, device="cuda")
    ws = torch.empty(pp.ops.polypic_sort_workspace_bytes(g, P), dtype=torch.uint8, device="cuda")
    st_ref = torch.zeros(1, dtype=torch.int32, device="cuda")
    pp.ops.polypic_sort(g, xd, keys_ref, perm_ref, ws, st_ref)
    keys = torch.full((P,), -1, dtype=torch.int32, device="cuda")
    perm = torch.full((P,), -1, dtype=torch.int32, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    pp.ops.polypic_sort_noalloc(g, xd, keys, perm, st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and int(st_ref.item()) == 0
    return host(keys), host(perm), host(keys_ref), host(perm_ref)


def test_noalloc_sort_equals_sort_two_calls():
    pp = require_gpu()
    cap = pp._lib.POLYPIC_SORT_NOALLOC_MAX_P
    sizes = [(0, 128, cap), (1, 64, 40_001)]
    for seed, n_cells, P in sizes:
        note(f"noalloc sort: seed={seed} cells={n_cells} P={P}")
        x, dx = _positions(seed, n_cells, P)
        g = pp.make_grid((n_cells + 4,) * 3, dx)
        k, p, k_ref, p_ref = _both(pp, g, x)
        assert np.array_equal(k, k_ref)
        assert np.array_equal(p, p_ref)
        if P < 100_000:
            kref, pref = O.sort_keys(oracle_grid(g), x)
            assert np.array_equal(k.view(np.uint32), kref)
            assert np.array_equal(p, pref)


def test_noalloc_sort_rejects_above_the_cap():
    pp = require_gpu()
    cap = pp._lib.POLYPIC_SORT_NOALLOC_MAX_P
    g = pp.make_grid((36, 36, 36), 1 / 32)
    x = torch.full((3, cap + 1), 0.5, dtype=torch.float32, device="cuda")
    keys = torch.empty(cap + 1, dtype=torch.int32, device="cuda")
    perm = torch.empty(cap + 1, dtype=torch.int32, device="cuda")
    with pytest.raises(pp.PolyPICError, match="workspace"):
        pp.ops.polypic_sort_noalloc(g, x, keys, perm)
