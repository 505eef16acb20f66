"""GPU decode parity: the HIP library decodes oracle-written streams; every
output byte must equal the oracle's decode (which the CPU tests pin to the
input).  Integer work, so the bar is bit-exact."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_cases import cases, mix_jobs

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2606_05765_amd.pivco")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def oracle_stream(case):
    name, data, bs, mode, tree = case
    return O.encode(data, bs, ans_mode=mode, tree_len=tree)


_CASES = cases()


@pytest.mark.parametrize("case", _CASES, ids=[c[0] for c in _CASES])
def test_decode_matches_oracle(case):
    print("case", case[0], len(case[1]), flush=True)
    st = oracle_stream(case)
    want = O.decode(st)
    assert np.array_equal(want, case[1])
    out, status = P.pivco_decode(dev(st))
    torch.cuda.synchronize()
    assert status == 0
    got = out.cpu().numpy()
    assert got.size == want.size
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, f"{bad.size} bytes differ, first at {bad[:5]}"


def _batch():
    cs = _CASES + mix_jobs()
    streams = [dev(oracle_stream(c)) for c in cs]
    wants = [c[1] for c in cs]
    return cs, streams, wants


def test_batch_and_plain_and_graph_agree():
    cs, streams, wants = _batch()
    print("batch of", len(cs), flush=True)
    outs, status = P.pivco_decode_batch(streams)
    torch.cuda.synchronize()
    assert (status == 0).all(), status
    for c, o, w in zip(cs, outs, wants):
        assert np.array_equal(o.cpu().numpy(), w), c[0]
    pouts, pstatus = P.pivco_decode_plain(streams)
    torch.cuda.synchronize()
    assert (pstatus == 0).all()
    for c, o, w in zip(cs, pouts, wants):
        assert np.array_equal(o.cpu().numpy(), w), c[0]
    gouts = [torch.empty_like(o) for o in outs]
    plan = P.BatchPlan(streams, gouts)
    for rep in range(3):
        for o in gouts:
            o.fill_(0xAB)                       # eager work between replays
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        assert (plan.statuses() == 0).all()
        for c, o, w in zip(cs, gouts, wants):
            assert np.array_equal(o.cpu().numpy(), w), (rep, c[0])
    plan.close()


def test_every_merge_variant():
    cs, streams, wants = _batch()
    outs = [torch.empty(w.size, dtype=torch.uint8, device="cuda") for w in wants]
    nv = len(P.pivco_merge_variants())
    # every variant on the persistent queue, then every variant as one
    # non-persistent launch with a workgroup per work item
    for v, mode in [(v, m) for m in (0, 1) for v in range(nv)]:
        print("variant", v, "grid_mode", mode, flush=True)
        t = P.Tune()
        t.merge_variant = v
        t.merge_grid = 64
        t.rans_grid = 32
        t.grid_mode = mode
        plan = P.BatchPlan(streams, outs, tune=t)
        for o in outs:
            o.fill_(0xAB)                       # a byte left unwritten cannot match by chance
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        assert (plan.statuses() == 0).all()
        for c, o, w in zip(cs, outs, wants):
            assert np.array_equal(o.cpu().numpy(), w), (v, mode, c[0])
        plan.close()


def test_autotune_choice_is_correct():
    cs, streams, wants = _batch()
    outs = [torch.empty(w.size, dtype=torch.uint8, device="cuda") for w in wants]
    P.pivco_autotune_cache_clear()
    t = P.pivco_autotune(streams, outs)
    assert t.merge_variant < len(P.pivco_merge_variants()) and t.merge_grid >= 1
    again = P.pivco_autotune(streams, outs)               # the same bucket: cached choice
    assert again.as_dict() == t.as_dict()
    plan = P.BatchPlan(streams, outs, tune=t)
    plan.launch()
    torch.cuda.synchronize()
    assert (plan.statuses() == 0).all()
    for c, o, w in zip(cs, outs, wants):
        assert np.array_equal(o.cpu().numpy(), w), c[0]
    plan.close()


def _corruptions(st):
    off0 = int(np.frombuffer(st[48:56].tobytes(), np.uint64)[0])
    muts = []
    b = st.copy(); b[0] ^= 1; muts.append(("magic", b))
    b = st.copy(); b[off0 + 12] = (b[off0 + 12] & 0xF0) | 1; muts.append(("kraft", b))
    b = st.copy(); b[off0 + 4] ^= 1; muts.append(("block_n", b))
    b = st.copy(); b[off0 + 140 + 1] ^= 0x40; muts.append(("kind_or_count", b))
    b = st.copy(); b[-9] ^= 0x10; muts.append(("body_bit", b))
    muts.append(("truncated", st[:len(st) // 2].copy()))
    b = st.copy(); b[56:64] = np.frombuffer(np.uint64(len(st) + 4096).tobytes(), np.uint8)
    muts.append(("offset_past_end", b))
    # last rANS offset (the table's final entry) past the stream's total of
    # scratch words
    b = st.copy(); b[off0 - 8:off0] = np.frombuffer(np.uint64(1 << 20).tobytes(), np.uint8)
    muts.append(("ans_offset_past_total", b))
    return muts


def test_corrupt_streams_flagged_and_isolated():
    rng = np.random.default_rng(21)
    import workloads as W
    x = W.draw(rng, W.zipf_p(1.1, rng), 150_000)
    good = O.encode(x, 1 << 15, ans_mode=1)
    muts = _corruptions(good)
    streams = [dev(good)] + [dev(m) for _, m in muts]
    outs = [torch.empty(x.size, dtype=torch.uint8, device="cuda") for _ in streams]
    got, status = P.pivco_decode_batch(streams, outs)
    torch.cuda.synchronize()
    assert status[0] == 0 and np.array_equal(got[0].cpu().numpy(), x)
    for (name, m), s in zip(muts, status[1:]):
        try:
            O.decode(m, n=x.size)
            oracle_ok = True
        except O.OracleError:
            oracle_ok = False
        if oracle_ok:
            continue                        # a flip the format cannot detect
        assert s != 0, name


def test_small_output_capacity_rejected():
    x = np.arange(1000, dtype=np.uint8) % 7
    st = O.encode(x, 256)
    outs, status = P.pivco_decode_batch([dev(st)], [torch.empty(999, dtype=torch.uint8, device="cuda")])
    torch.cuda.synchronize()
    assert status[0] == P.E_CAPACITY


def test_corrupt_split_blocks_flagged_and_isolated():
    """Bit flips inside blocks decoded as tiles: the boundary pass must flag
    every stream the oracle rejects, and the clean stream beside them must
    still decode exactly."""
    rng = np.random.default_rng(22)
    import workloads as W
    x = W.draw(rng, W.zipf_p(1.05, rng), 600_000)
    for mode in (0, 2):
        good = O.encode(x, 1 << 18, ans_mode=mode)
        off0 = int(np.frombuffer(good[48:56].tobytes(), np.uint64)[0])
        muts = []
        for k in range(12):
            b = good.copy()
            pos = int(rng.integers(off0 + 200, len(good)))
            b[pos] ^= np.uint8(1 << int(rng.integers(0, 8)))
            muts.append((f"flip_{pos}", b))
        streams = [dev(good)] + [dev(m) for _, m in muts]
        outs = [torch.empty(x.size, dtype=torch.uint8, device="cuda") for _ in streams]
        got, status = P.pivco_decode_batch(streams, outs)
        torch.cuda.synchronize()
        assert status[0] == 0 and np.array_equal(got[0].cpu().numpy(), x), mode
        for (name, m), s in zip(muts, status[1:]):
            try:
                ok = np.array_equal(O.decode(m, n=x.size), x)
            except O.OracleError:
                ok = False
            if not ok:
                assert s != 0, (mode, name)



def test_corrupt_entropy_coded_bodies_match_oracle():
    """Single-bit flips in the second half of forced-rANS streams (whole
    blocks: where the entropy-coded bodies lie), each decoded in one batch
    with the intact stream: the plan kernel reserves a block's chunk slots
    before it walks the bodies, and a body found corrupt must leave empty
    chunks behind.  Every flipped stream gets the oracle's verdict: rejected,
    or decoded to exactly the oracle's bytes; the intact one decodes."""
    rng = np.random.default_rng(33)
    import workloads as W
    x = W.draw(rng, W.geometric_p(0.85), 200_000)
    good = O.encode(x, 1 << 15, ans_mode=2)
    muts = []
    for _ in range(60):
        b = good.copy()
        pos = int(rng.integers(good.size // 2, good.size))
        b[pos] ^= np.uint8(1 << int(rng.integers(0, 8)))
        muts.append((f"flip_{pos}", b))
    streams = [dev(good)] + [dev(m) for _, m in muts]
    outs = [torch.empty(x.size, dtype=torch.uint8, device="cuda") for _ in streams]
    got, status = P.pivco_decode_batch(streams, outs)
    torch.cuda.synchronize()
    assert status[0] == 0 and np.array_equal(got[0].cpu().numpy(), x)
    for (name, m), s, o in zip(muts, status[1:], got[1:]):
        try:
            want = O.decode(m, n=x.size)
        except O.OracleError:
            want = None
        if want is None:
            assert s != 0, name
        else:
            assert s == 0 and np.array_equal(o.cpu().numpy(), want), name
