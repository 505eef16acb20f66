"""GPU encode parity: the HIP encoder's stream must be byte-identical to the
oracle's stream for the same input and options, and must decode back."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_cases import cases, mix_jobs

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2606_05765_amd.pivco")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


_CASES = cases() + mix_jobs(n_blocks=12)


def _first_diff(a, b):
    n = min(a.size, b.size)
    d = np.flatnonzero(a[:n] != b[:n])
    return int(d[0]) if d.size else n


@pytest.mark.parametrize("case", _CASES, ids=[c[0] for c in _CASES])
def test_encode_matches_oracle(case):
    name, data, bs, mode, tree = case
    print("case", name, data.size, flush=True)
    want = O.encode(data, bs, ans_mode=mode, tree_len=tree)
    got = P.pivco_encode(dev(data), bs, ans_mode=mode, tree=tree)
    torch.cuda.synchronize()
    g = got.cpu().numpy()
    assert g.size == want.size and np.array_equal(g, want), \
        f"{name}: sizes {g.size}/{want.size}, first difference at byte {_first_diff(g, want)}"
    out, st = P.pivco_decode(got)
    torch.cuda.synchronize()
    assert st == 0 and np.array_equal(out.cpu().numpy(), data)


def test_encode_empty_input():
    got = P.pivco_encode(torch.empty(0, dtype=torch.uint8, device="cuda"), 4096)
    want = O.encode(np.zeros(0, np.uint8), 4096)
    assert np.array_equal(got.cpu().numpy(), want)


def test_encode_rejects_tree_missing_symbol():
    lens = np.zeros(256, np.uint8)
    lens[0] = lens[1] = 1
    with pytest.raises(P.PivcoError) as e:
        P.pivco_encode(dev(np.array([0, 1, 2], np.uint8)), 16, tree=lens)
    assert e.value.code == P.E_ARG


def test_encode_deterministic_large():
    x = W.zipf256m(seed=4, scale=64).jobs[0]                  # 4 MiB, 64 blocks
    a = P.pivco_encode(dev(x), 64 << 10).cpu().numpy()
    b = P.pivco_encode(dev(x), 64 << 10).cpu().numpy()
    assert np.array_equal(a, b)
    for blk in [0, 17, 63]:
        ref = O.decode_blocks(a, blk, blk + 1)
        assert np.array_equal(ref, x[blk * 65536:(blk + 1) * 65536])
