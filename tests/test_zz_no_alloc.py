"""pivco_decode_noalloc (no device allocation, library-held scratch) must
give exactly what pivco_decode gives with a caller workspace, on two calls in
a row (the second smaller, so stale scratch from the first is exercised), and
refuse a stream that needs more workspace than the fixed array holds."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2606_05765_amd.pivco")


def _stream(x, block_size, ans_mode):
    return torch.from_numpy(oracle.encode(x, block_size, ans_mode=ans_mode)).cuda()


def _noalloc(stream, n):
    out = torch.full((n,), 0xA5, dtype=torch.uint8, device="cuda")
    status = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    P.pivco_decode_noalloc(stream, out, status)
    torch.cuda.synchronize()
    return out, int(status.cpu()[0])


def test_noalloc_matches_workspace_decode_twice():
    rng = np.random.default_rng(21)
    big = W.skew256m(seed=2, scale=256).jobs[0]                  # 1 MiB, rANS nodes
    small = W.draw(rng, W.zipf_p(1.1, rng), 150_001)             # ragged, split-free
    cases = [(big, 128 << 10, 1), (small, 64 << 10, 0)]
    for x, bs, am in cases:
        print("case", x.size, bs, am, flush=True)
        s = _stream(x, bs, am)
        ref, st = P.pivco_decode(s)
        torch.cuda.synchronize()
        assert st == 0
        got, st2 = _noalloc(s, x.size)
        assert st2 == 0
        assert torch.equal(got, ref)
        assert np.array_equal(got.cpu().numpy(), x)


def test_noalloc_split_blocks_and_constant():
    # a block decoded as tiles (boundary tables in the scratch), then a
    # constant block, in a row
    rng = np.random.default_rng(22)
    x1 = W.draw(rng, W.geometric_p(0.9), (1 << 20) + 77)
    x2 = np.full(5000, 3, np.uint8)
    for x, bs in [(x1, 1 << 20), (x2, 4096)]:
        s = _stream(x, bs, 1)
        ref, st = P.pivco_decode(s)
        torch.cuda.synchronize()
        got, st2 = _noalloc(s, x.size)
        assert st == 0 and st2 == 0
        assert torch.equal(got, ref)


def test_noalloc_rejects_oversized_workspace():
    # 8000 blocks of 64 symbols need ~45 MB of per-block records alone
    rng = np.random.default_rng(23)
    x = rng.integers(0, 7, size=64 * 8000).astype(np.uint8)
    s = _stream(x, 64, 0)
    out = torch.empty(x.size, dtype=torch.uint8, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert P.pivco_decode_workspace([s], [out]) > P.NOALLOC_SCRATCH_BYTES
    with pytest.raises(P.PivcoError) as e:
        P.pivco_decode_noalloc(s, out, status)
    assert e.value.code == P.E_CAPACITY
