"""Parity at full workload sizes, in the launch configuration the benchmark
times (autotuned batch plan, HIP-graph replay): the GPU stream must be
byte-identical to the oracle's stream (whole stream, or sampled blocks for
the 2.3 GB mixed workload), every decoded byte must equal the input, and the
oracle must decode sampled blocks of the GPU stream to the same bytes."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2606_05765_amd.pivco")


def _say(*a):
    print(*a, flush=True)


def _sample(n, k, seed):
    rng = np.random.default_rng(seed)
    picks = set(int(i) for i in rng.choice(n, size=min(k, n), replace=False))
    picks.update({0, n - 1})
    return sorted(picks)


def _first_diff(a, b):
    m = min(a.size, b.size)
    d = np.flatnonzero(a[:m] != b[:m])
    return int(d[0]) if d.size else m


def _plan_decode(streams, outs, reps=2):
    """Decode as bench.py does: autotune, then graph replays."""
    tune = P.pivco_autotune(streams, outs)
    plan = P.BatchPlan(streams, outs, tune=tune)
    for _ in range(reps):
        for o in outs:
            o.fill_(0xAB)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        assert (plan.statuses() == 0).all()
        yield tune
    plan.close()


def _single_stream(w, sample_blocks=24, ans_mode=None):
    x = w.jobs[0]
    mode = w.ans_mode if ans_mode is None else ans_mode
    _say("workload", w.name, x.size, "bytes, block", w.block_size, "ans_mode", mode)
    d_x = torch.from_numpy(x).cuda()
    st = P.pivco_encode(d_x, w.block_size, ans_mode=mode)
    torch.cuda.synchronize()
    g = st.cpu().numpy()
    _say("gpu stream", g.size, "bytes; oracle encode ...")
    want = O.encode(x, w.block_size, ans_mode=mode)
    assert g.size == want.size and np.array_equal(g, want), \
        f"stream sizes {g.size}/{want.size}, first difference at byte {_first_diff(g, want)}"
    _say("stream identical; batched decode ...")
    out = torch.empty(x.size, dtype=torch.uint8, device="cuda")
    for tune in _plan_decode([st], [out]):
        assert torch.equal(out, d_x), tune.as_dict()
    _say("decode identical with", tune.as_dict())
    nb = O.stream_info(g)["n_blocks"]
    for b in _sample(nb, sample_blocks, 5):
        dec = O.decode_blocks(g, b, b + 1)
        lo = b * w.block_size
        assert np.array_equal(dec, x[lo:lo + dec.size]), b
    _say("oracle decode of sampled blocks identical")


@pytest.mark.timeout(120)
def test_geo1m_full():
    w = W.geo1m(seed=1)
    _single_stream(w)
    x = w.jobs[0]
    assert np.array_equal(O.decode(O.encode(x, w.block_size)), x)


@pytest.mark.timeout(300)
def test_zipf256m_full():
    _single_stream(W.zipf256m(seed=1))


@pytest.mark.timeout(300)
def test_skew256m_full():
    _single_stream(W.skew256m(seed=1))


@pytest.mark.timeout(300)
def test_skew256m_full_selective_tans():
    # the same workload with the selective tANS of Sec. 5.2 (ans_mode 3)
    _single_stream(W.skew256m(seed=1), ans_mode=3)


@pytest.mark.timeout(400)
def test_mix4096_full():
    w = W.mix4096(seed=1)
    _say("mix4096:", len(w.jobs), "blocks,", w.total, "bytes")
    d_in = [torch.from_numpy(x).cuda() for x in w.jobs]
    streams = []
    for i, d in enumerate(d_in):
        streams.append(P.pivco_encode(d, max(d.numel(), 1), ans_mode=w.ans_mode))
        if i % 512 == 0:
            _say("encoded", i)
    torch.cuda.synchronize()
    for i in _sample(len(w.jobs), 32, 7):
        want = O.encode(w.jobs[i], max(w.jobs[i].size, 1), ans_mode=w.ans_mode)
        g = streams[i].cpu().numpy()
        assert g.size == want.size and np.array_equal(g, want), (i, w.labels[i])
    _say("sampled streams identical; batched decode ...")
    outs = [torch.empty_like(d) for d in d_in]
    for tune in _plan_decode(streams, outs):
        bad = [i for i in range(len(outs)) if not torch.equal(outs[i], d_in[i])]
        assert not bad, (bad[:5], tune.as_dict())
    _say("decode identical with", tune.as_dict())
    for i in _sample(len(w.jobs), 16, 9):
        assert np.array_equal(O.decode(streams[i].cpu().numpy()), w.jobs[i]), i
    _say("oracle decode of sampled jobs identical")
