"""Particle-order permutations on the device (polypic_gather_rows,
polypic_scatter_rows, polypic_invert_permutation) against numpy indexing:
bit-exact, since they only move 4-byte elements."""
import numpy as np
import pytest
import torch

from tests.gpu_util import note, require_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("P,rows", [(1, 1), (255, 3), (1000, 13), (4099, 81)])
@pytest.mark.parametrize("dtype", [np.float32, np.int32])
def test_gather_rows_equals_indexing(P, rows, dtype):
    pp = require_gpu()
    rng = np.random.default_rng(P * 100 + rows)
    src = rng.standard_normal((rows, P)).astype(np.float32)
    if dtype == np.int32:
        src = rng.integers(-2**31, 2**31 - 1, size=(rows, P), dtype=np.int64).astype(np.int32)
    idx = rng.permutation(P).astype(np.int32)
    note(f"gather_rows P={P} rows={rows} {np.dtype(dtype).name}")
    s = torch.from_numpy(src).cuda()
    d = torch.empty_like(s)
    pp.ops.polypic_gather_rows(s, d, torch.from_numpy(idx).cuda())
    torch.cuda.synchronize()
    out = d.cpu().numpy()
    assert np.array_equal(out.view(np.uint32), src[:, idx].view(np.uint32))


@pytest.mark.parametrize("P,rows", [(1, 1), (255, 3), (1000, 13), (4099, 81)])
def test_scatter_rows_equals_indexed_assignment(P, rows):
    pp = require_gpu()
    rng = np.random.default_rng(P * 7 + rows)
    src = rng.standard_normal((rows, P)).astype(np.float32)
    idx = rng.permutation(P).astype(np.int32)
    note(f"scatter_rows P={P} rows={rows}")
    d = torch.empty(rows, P, device="cuda")
    pp.ops.polypic_scatter_rows(torch.from_numpy(src).cuda(), d, torch.from_numpy(idx).cuda())
    torch.cuda.synchronize()
    ref = np.empty_like(src)
    ref[:, idx] = src
    assert np.array_equal(d.cpu().numpy(), ref)


def test_gather_rows_clamps_bad_indices_and_repeats():
    pp = require_gpu()
    P, rows = 300, 2
    src = np.arange(rows * P, dtype=np.float32).reshape(rows, P)
    idx = np.array([(-7 if i % 5 == 0 else (P + 3 if i % 7 == 0 else i // 2)) for i in range(P)],
                   dtype=np.int32)
    d = torch.empty(rows, P, device="cuda")
    pp.ops.polypic_gather_rows(torch.from_numpy(src).cuda(), d, torch.from_numpy(idx).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy(), src[:, np.clip(idx, 0, P - 1)])


@pytest.mark.parametrize("P", [1, 257, 5000])
def test_invert_permutation(P):
    pp = require_gpu()
    perm = np.random.default_rng(P).permutation(P).astype(np.int32)
    inv = torch.full((P,), -1, dtype=torch.int32, device="cuda")
    pp.ops.polypic_invert_permutation(torch.from_numpy(perm).cuda(), inv)
    torch.cuda.synchronize()
    ref = np.empty(P, np.int32)
    ref[perm] = np.arange(P, dtype=np.int32)
    assert np.array_equal(inv.cpu().numpy(), ref)


def test_empty_permutation_calls():
    pp = require_gpu()
    e = torch.empty(3, 0, device="cuda")
    pp.ops.polypic_gather_rows(e, torch.empty_like(e), torch.empty(0, dtype=torch.int32,
                                                                    device="cuda"))
    pp.ops.polypic_scatter_rows(e, torch.empty_like(e), torch.empty(0, dtype=torch.int32,
                                                                     device="cuda"))
    z = torch.empty(0, dtype=torch.int32, device="cuda")
    pp.ops.polypic_invert_permutation(z, torch.empty_like(z))
    torch.cuda.synchronize()
