"""Top-down decode (partition/scatter, Sec. 2.1), the ablation of the
bottom-up merge: the same oracle-written streams must decode to exactly the
oracle's bytes, whole blocks and tiles of split blocks alike, and corrupt
streams must be flagged without touching the clean job beside them."""
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


def test_topdown_matches_oracle_in_one_batch():
    cs = cases() + mix_jobs()
    streams = [dev(O.encode(d, bs, ans_mode=m, tree_len=t)) for _, d, bs, m, t in cs]
    outs = [torch.full((c[1].size,), 0xAB, dtype=torch.uint8, device="cuda") for c in cs]
    print("batch of", len(cs), flush=True)
    got, status = P.pivco_decode_topdown(streams, outs)
    torch.cuda.synchronize()
    assert (status == 0).all(), status
    for c, o in zip(cs, got):
        assert np.array_equal(o.cpu().numpy(), c[1]), c[0]


@pytest.mark.parametrize("mode", [0, 2])
def test_topdown_corrupt_streams_flagged(mode):
    rng = np.random.default_rng(31 + mode)
    x = W.draw(rng, W.zipf_p(1.05, rng), 300_000)
    good = O.encode(x, 1 << 17, ans_mode=mode)
    off0 = int(np.frombuffer(good[48:56].tobytes(), np.uint64)[0])
    muts = []
    for _ in range(10):
        b = good.copy()
        p = int(rng.integers(off0 + 200, len(good)))
        b[p] ^= np.uint8(1 << int(rng.integers(0, 8)))
        muts.append(b)
    streams = [dev(good)] + [dev(m) for m in muts]
    outs = [torch.empty(x.size, dtype=torch.uint8, device="cuda") for _ in streams]
    got, status = P.pivco_decode_topdown(streams, outs)
    torch.cuda.synchronize()
    assert status[0] == 0 and np.array_equal(got[0].cpu().numpy(), x)
    for m, s in zip(muts, status[1:]):
        try:
            ok = np.array_equal(O.decode(m, n=x.size), x)
        except O.OracleError:
            ok = False
        if not ok:
            assert s != 0
