"""PivCo-Golomb (App. G) on the GPU: the encoder must write exactly the
oracle's stream and the decoder must return the oracle's values, on geometric
sources over the code lengths the appendix measures, ragged and full-range
blocks; corrupt streams are flagged."""
import numpy as np
import pytest
import torch

import oracle as O

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2606_05765_amd.pivco")


def _geo(rng, mean_len, n):
    # unary code length v + 1 with v geometric: mean length 1 / (1 - q)
    q = 1.0 - 1.0 / mean_len
    return np.minimum(rng.geometric(1.0 - q, size=n) - 1, 255).astype(np.uint8)


def _cases():
    rng = np.random.default_rng(41)
    out = []
    for L in (1.25, 1.5, 2, 3, 4, 5):
        out.append((f"geo_len{L}", _geo(rng, L, 200_003), 1 << 16))
    out.append(("full_range", rng.integers(0, 256, size=50_001).astype(np.uint8), 20_000))
    out.append(("zeros", np.zeros(70_000, np.uint8), 1 << 16))
    out.append(("tiny", np.array([0, 2, 1, 0, 3], np.uint8), 16))
    out.append(("one", np.array([255], np.uint8), 8))
    out.append(("big_block", _geo(rng, 3, 1_000_000), 1 << 20))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_golomb_encode_decode_match_oracle(case):
    name, x, bs = case
    print("case", name, x.size, bs, flush=True)
    want = O.golomb_encode(x, bs)
    got = P.pivco_golomb_encode(torch.from_numpy(x).cuda(), bs)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want)
    outs, st = P.pivco_golomb_decode([torch.from_numpy(want).cuda()])
    torch.cuda.synchronize()
    assert st[0] == 0
    assert np.array_equal(outs[0].cpu().numpy(), x)


def test_golomb_batch_and_corruption():
    rng = np.random.default_rng(42)
    x = _geo(rng, 3, 120_000)
    good = O.golomb_encode(x, 1 << 15)
    streams, flags = [torch.from_numpy(good).cuda()], [True]
    for _ in range(12):
        b = good.copy()
        p = int(rng.integers(80, len(good)))
        b[p] ^= np.uint8(1 << int(rng.integers(0, 8)))
        try:
            ok = np.array_equal(O.golomb_decode(b, n=x.size), x)
        except O.OracleError:
            ok = False
        streams.append(torch.from_numpy(b).cuda())
        flags.append(ok)
    outs = [torch.empty(x.size, dtype=torch.uint8, device="cuda") for _ in streams]
    got, st = P.pivco_golomb_decode(streams, outs)
    torch.cuda.synchronize()
    assert st[0] == 0 and np.array_equal(got[0].cpu().numpy(), x)
    for ok, s in zip(flags[1:], st[1:]):
        if not ok:
            assert s != 0
