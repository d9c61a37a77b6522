"""The sort entry point that allocates nothing (fixed device scratch) against
the workspace sort it shares its kernels with: two calls in a row, the
second on a smaller input, bit for bit, and both against a stable argsort."""

import numpy as np
import pytest
import torch

from gpu_helpers import say

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")


def _inputs(n, cap, bits, seed):
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, 1 << bits, n, dtype=np.int64).view(np.uint64)
    keys = keys[rng.integers(0, max(1, n // 3), n)]          # equal keys: stability matters
    k = torch.zeros(cap, dtype=torch.int64, device=DEV)
    v = torch.zeros(cap, dtype=torch.int32, device=DEV)
    k[:n] = torch.as_tensor(keys.view(np.int64), device=DEV)
    v[:n] = torch.arange(n, dtype=torch.int32, device=DEV)
    cnt = torch.tensor([n], dtype=torch.int32, device=DEV)
    return keys, k, v, cnt


def test_noalloc_sort_matches_the_workspace_sort_on_consecutive_calls():
    from paper_2601_17354_amd import _lib
    from paper_2601_17354_amd import binding as B
    cases = [(600_000, _lib.SORT_NOALLOC_MAX_PAIRS, 46, 1), (70_001, 100_000, 40, 2)]
    for n, cap, bits, seed in cases:
        say(f"[no-alloc sort] n={n} capacity={cap} bits={bits}")
        keys, k0, v0, cnt = _inputs(n, cap, bits, seed)
        k1, v1 = k0.clone(), v0.clone()
        ws = torch.empty(B.pgs_sort_workspace(cap), dtype=torch.uint8, device=DEV)
        B.pgs_sort_pairs(k0, v0, cnt, cap, bits, ws)
        B.pgs_sort_pairs_noalloc(k1, v1, cnt, cap, bits)
        torch.cuda.synchronize()
        assert torch.equal(k0, k1) and torch.equal(v0, v1)
        order = np.argsort(keys, kind="stable")
        np.testing.assert_array_equal(k1[:n].cpu().numpy().view(np.uint64), keys[order])
        np.testing.assert_array_equal(v1[:n].cpu().numpy().astype(np.int64), order)
        del ws


def test_noalloc_sort_rejects_a_capacity_beyond_its_scratch():
    from paper_2601_17354_amd import _lib
    from paper_2601_17354_amd import binding as B
    cap = _lib.SORT_NOALLOC_MAX_PAIRS + 1
    k = torch.zeros(cap, dtype=torch.int64, device=DEV)
    v = torch.zeros(cap, dtype=torch.int32, device=DEV)
    cnt = torch.tensor([cap], dtype=torch.int32, device=DEV)
    with pytest.raises(_lib.PgsError, match="exceeds"):
        B.pgs_sort_pairs_noalloc(k, v, cnt, cap, 40)
