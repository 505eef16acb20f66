"""Seeded random sweep of encode options and inputs: for each case the HIP
encoder's stream must equal the oracle's byte for byte, the HIP decoder must
return the input from the oracle's stream (alone and with every other case
in one batched launch), and the oracle's own decode must return the input.
Bit-exact throughout (integer work)."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2606_05765_amd.pivco")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _random_cases(seed=20261203, count=40):
    """(name, data, block_size, ans_mode, max_len, chunk_log2): sizes
    log-uniform in 1..400K symbols, block sizes from 1 Ki to 256 Ki symbols
    (ragged tails, one or many blocks, whole and split blocks), the mixed
    families plus one-symbol-dominated and few-symbol sources, every rANS
    mode, code length limits 8..12 and rANS chunks of 2^10..2^16 bits."""
    r = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = W.log_uniform_size(r, 1, 400_000)
        kind = int(r.integers(0, 5))
        if kind < 3:
            lab, p = W.family_p(r)
        elif kind == 3:
            lab, p = "skew", W.skew_p()
        else:
            k = int(r.integers(2, 6))
            lab, p = f"few(k={k})", np.concatenate([np.ones(k), np.zeros(256 - k)])
        data = W.draw(r, p, n)
        bs = int(2 ** r.integers(10, 19))
        mode = int(r.integers(0, 3))
        max_len = int(r.integers(8, 13))
        clog = int(r.choice([10, 12, 16]))
        out.append((f"r{i}_{lab}_n{n}_bs{bs}_m{mode}_L{max_len}_c{clog}", data, bs, mode, max_len, clog))
    return out


_CASES = _random_cases()


@pytest.mark.parametrize("case", _CASES, ids=[c[0] for c in _CASES])
def test_random_encode_decode(case):
    name, data, bs, mode, max_len, clog = case
    print("case", name, flush=True)
    want = O.encode(data, bs, max_len=max_len, ans_mode=mode, chunk_log2=clog)
    assert np.array_equal(O.decode(want), data)
    got = P.pivco_encode(dev(data), bs, max_len=max_len, ans_mode=mode, chunk_log2=clog)
    torch.cuda.synchronize()
    g = got.cpu().numpy()
    assert g.size == want.size and np.array_equal(g, want), f"{name}: encoder bytes differ"
    out, status = P.pivco_decode(dev(want))
    torch.cuda.synchronize()
    assert status == 0
    assert np.array_equal(out.cpu().numpy(), data), f"{name}: decoded bytes differ"


def test_random_cases_in_one_batch():
    streams = [dev(O.encode(d, bs, max_len=L, ans_mode=m, chunk_log2=c)) for _, d, bs, m, L, c in _CASES]
    outs = [torch.empty(c[1].size, dtype=torch.uint8, device="cuda") for c in _CASES]
    plan = P.BatchPlan(streams, outs, tune=P.pivco_autotune(streams, outs))
    for o in outs:
        o.fill_(0xAB)
    torch.cuda.synchronize()
    plan.launch()
    torch.cuda.synchronize()
    assert (plan.statuses() == 0).all()
    for c, o in zip(_CASES, outs):
        assert np.array_equal(o.cpu().numpy(), c[1]), c[0]
    plan.close()
