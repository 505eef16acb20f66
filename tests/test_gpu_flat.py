"""GPU parity for v2 streams (flat subtrees, Sec. 2.2.3-2.2.4; merge_flat_D,
Sec. 3.2): the HIP decoder must reproduce the oracle's bytes on oracle-written
v2 streams -- whole blocks held in LDS, streamed blocks, tiles of split
blocks, rANS nodes beside flat ones, every merge variant -- and the HIP
encoder must write the oracle's v2 stream byte for byte."""
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


def flat_cases():
    r = np.random.default_rng(77)
    out = list(cases())
    # every symbol of length 8: the root is one flat node of depth 8 (64 KiB
    # blocks are streamed: their bodies exceed the LDS budget), also split
    u = np.tile(np.arange(256, dtype=np.uint8), 4096)
    r.shuffle(u)
    out.append(("flat_root_d8_stream", u[:(256 << 10) + 3], 64 << 10, 0, None))
    out.append(("flat_root_d8_split", u, 1 << 20, 0, None))
    # four equally frequent symbols: a root flat node of depth 2
    out.append(("flat_root_d2", r.integers(0, 4, size=100_003).astype(np.uint8) * 60, 1 << 15, 0, None))
    # 200 symbols: lengths 7 (56 symbols) and 8 (144): groups of 32, 16, 8
    # and 128, 16
    v = np.tile(np.arange(200, dtype=np.uint8), 3000)
    r.shuffle(v)
    out.append(("flat_mixed_D", v, 1 << 16, 0, None))
    out.append(("flat_mixed_D_split", v, v.size, 1, None))
    # flat nodes beside rANS-coded binary nodes
    sk = W.draw(r, W.geometric_p(0.6), 400_000)
    out.append(("flat_with_rans", np.where(r.random(sk.size) < 0.3, r.integers(0, 64, sk.size), sk).astype(np.uint8),
                1 << 17, 2, None))
    return out


_CASES = flat_cases()


def _stream(case):
    name, data, bs, mode, tree = case
    return O.encode(data, bs, ans_mode=mode, tree_len=tree, flat=True)


@pytest.mark.parametrize("case", _CASES, ids=[c[0] for c in _CASES])
def test_flat_decode_matches_oracle(case):
    print("case", case[0], len(case[1]), flush=True)
    st = _stream(case)
    want = O.decode(st, merge=True)
    assert np.array_equal(want, case[1])
    out, status = P.pivco_decode(dev(st))
    torch.cuda.synchronize()
    assert status == 0
    got = out.cpu().numpy()
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, f"{bad.size} bytes differ, first at {bad[:5]}"


def test_flat_every_merge_variant_with_v1_beside():
    cs = _CASES + mix_jobs(n_blocks=12)
    streams = [dev(_stream(c)) for c in cs] + [dev(O.encode(c[1], c[2], ans_mode=c[3], tree_len=c[4]))
                                               for c in cs[:6]]
    wants = [c[1] for c in cs] + [c[1] for c in cs[:6]]
    outs = [torch.empty(w.size, dtype=torch.uint8, device="cuda") for w in wants]
    nv = len(P.pivco_merge_variants())
    for v, mode in [(v, m) for m in (0, 1) for v in range(nv)]:
        print("variant", v, "grid_mode", mode, flush=True)
        t = P.Tune()
        t.merge_variant = v
        t.merge_grid = 64
        t.rans_grid = 32
        t.grid_mode = mode
        plan = P.BatchPlan(streams, outs, tune=t)
        for o in outs:
            o.fill_(0xAB)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        assert (plan.statuses() == 0).all()
        for i, (o, w) in enumerate(zip(outs, wants)):
            assert np.array_equal(o.cpu().numpy(), w), (v, mode, i)
        plan.close()


_ENC = [c for c in _CASES if c[1].size <= (4 << 20) + 1] + mix_jobs(n_blocks=8)


@pytest.mark.parametrize("case", _ENC, ids=[c[0] for c in _ENC])
def test_flat_encode_matches_oracle(case):
    name, data, bs, mode, tree = case
    print("case", name, data.size, flush=True)
    want = _stream(case)
    got = P.pivco_encode(dev(data), bs, ans_mode=mode, tree=tree, flat=True).cpu().numpy()
    torch.cuda.synchronize()
    n = min(got.size, want.size)
    d = np.flatnonzero(got[:n] != want[:n])
    assert got.size == want.size and d.size == 0, \
        f"{name}: sizes {got.size}/{want.size}, first difference at {d[:3] if d.size else n}"


def test_flat_topdown_unsupported():
    x = np.tile(np.arange(16, dtype=np.uint8), 1000)
    st = dev(O.encode(x, 4096, flat=True))
    outs, status = P.pivco_decode_topdown([st], [torch.empty(x.size, dtype=torch.uint8, device="cuda")])
    torch.cuda.synchronize()
    assert status[0] == P.E_UNSUPPORTED


def _flat_block_fields(st, b):
    """Offsets of block b's kind bytes, count fields and the first flat node."""
    nb = int.from_bytes(st[20:24].tobytes(), "little")
    off = int.from_bytes(st[48 + 8 * b:56 + 8 * b].tobytes(), "little")
    info = O.block_info(st, b)
    I, cw = info["n_internal"], int(st[off + 10])
    kb = (I + 7) // 8
    flat = [i for i in range(I) if info["flat"][i]]
    return off, I, cw, kb, flat, info, nb


@pytest.mark.parametrize("bs", [1 << 15, 1 << 18])
def test_flat_corruption_flagged(bs):
    r = np.random.default_rng(5)
    v = np.tile(np.arange(200, dtype=np.uint8), 1500)
    r.shuffle(v)
    good = O.encode(v, bs, flat=True)
    off, I, cw, kb, flat, info, nb = _flat_block_fields(good, 0)
    assert flat
    f = flat[0]
    muts = []
    b = good.copy(); b[off + 140 + kb + cw * f] ^= 1; muts.append(("flat_count", b))
    b = good.copy(); b[off + 140 + f // 8] |= 1 << (f % 8); muts.append(("flat_kind", b))
    streams = [dev(good)] + [dev(m) for _, m in muts]
    outs = [torch.empty(v.size, dtype=torch.uint8, device="cuda") for _ in streams]
    got, status = P.pivco_decode_batch(streams, outs)
    torch.cuda.synchronize()
    assert status[0] == 0 and np.array_equal(got[0].cpu().numpy(), v)
    for (name, m), s in zip(muts, status[1:]):
        with pytest.raises(O.OracleError):
            O.decode(m)
        assert s != 0, name
