"""GPU tests of the asynchronous encode (pivco_encode_async): streams
byte-identical to the oracle's with the code lengths built on the device
(package-merge with the format's tie rules), lengths and statuses left in
device memory, many encodes enqueued without a host wait, replays of a
captured HIP graph, and the errors that only the data reveal (a supplied
tree that misses a present symbol, a stream larger than out_cap)."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2606_05765_amd.pivco")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _buffers(n, bs, **kw):
    cap = P.pivco_encode_bound(n, bs, **{k: v for k, v in kw.items() if k != "tree"})
    wsb = P.pivco_encode_workspace(n, bs, **{k: v for k, v in kw.items() if k != "tree"})
    out = torch.full((max(cap, 16),), 0xAB, dtype=torch.uint8, device="cuda")
    ws = torch.empty(max(wsb, 256), dtype=torch.uint8, device="cuda")
    ln = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    return out, ws, ln, st


def _count_cases():
    """Inputs whose histograms stress the device package-merge: many equal
    counts (ties between singles and packages), every symbol, two symbols,
    counts that force the 11-bit limit, and random mixes."""
    r = np.random.default_rng(31)
    out = []
    out.append(("ties", np.repeat(np.arange(200, dtype=np.uint8), 37)))
    out.append(("all256_equal", np.tile(np.arange(256, dtype=np.uint8), 64)))
    out.append(("two", (r.random(50_000) < 0.2).astype(np.uint8)))
    fib = [1, 1]
    while len(fib) < 30:
        fib.append(fib[-1] + fib[-2])
    p = np.zeros(256)
    p[:30] = fib[::-1]
    out.append(("fib_limit", W.draw(r, p, 400_000)))
    for i in range(6):
        k = int(r.integers(2, 257))
        w = r.pareto(1.0 + i * 0.3, k) + 1e-3
        pp = np.zeros(256)
        pp[r.choice(256, k, replace=False)] = w
        out.append((f"pareto_{i}", W.draw(r, pp, int(r.integers(3000, 300_000)))))
    return out


_CASES = _count_cases()


@pytest.mark.parametrize("case", _CASES, ids=[c[0] for c in _CASES])
@pytest.mark.parametrize("max_len", [11, 9])
def test_async_encode_matches_oracle(case, max_len):
    name, data = case
    m = int(np.count_nonzero(np.bincount(data, minlength=256)))
    if m > (1 << max_len):
        pytest.skip("more symbols than codes of this length")
    bs = 1 << 16
    print("case", name, data.size, max_len, flush=True)
    want = O.encode(data, bs, max_len=max_len, ans_mode=1)
    out, ws, ln, st = _buffers(data.size, bs, max_len=max_len, ans_mode=1)
    P.pivco_encode_async(dev(data), out, ln, st, ws, bs, max_len=max_len, ans_mode=1)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    n = int(ln.item())
    got = out[:n].cpu().numpy()
    assert n == want.size and np.array_equal(got, want)


def test_many_encodes_without_a_host_wait():
    r = np.random.default_rng(5)
    datas = [W.draw(r, W.geometric_p(float(r.uniform(0.5, 0.95))), int(r.integers(1, 200_000)))
             for _ in range(48)]
    bufs = [_buffers(d.size, 1 << 15, ans_mode=1) for d in datas]
    ins = [dev(d) for d in datas]
    torch.cuda.synchronize()
    for d, (out, ws, ln, st) in zip(ins, bufs):
        P.pivco_encode_async(d, out, ln, st, ws, 1 << 15, ans_mode=1)
    torch.cuda.synchronize()
    for d, (out, ws, ln, st) in zip(datas, bufs):
        want = O.encode(d, 1 << 15, ans_mode=1)
        assert int(st.item()) == 0
        assert np.array_equal(out[:int(ln.item())].cpu().numpy(), want)


def test_captured_graph_replays():
    r = np.random.default_rng(9)
    data = W.draw(r, W.zipf_p(1.1, r), 300_000)
    want = O.encode(data, 1 << 16, ans_mode=1)
    d = dev(data)
    out, ws, ln, st = _buffers(data.size, 1 << 16, ans_mode=1)
    P.pivco_encode_async(d, out, ln, st, ws, 1 << 16, ans_mode=1)    # eager run first
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            P.pivco_encode_async(d, out, ln, st, ws, 1 << 16, ans_mode=1)
    torch.cuda.synchronize()
    for rep in range(3):
        out.fill_(0xAB)
        ln.fill_(-1)
        st.fill_(99)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(st.item()) == 0, rep
        assert int(ln.item()) == want.size, rep
        assert np.array_equal(out[:want.size].cpu().numpy(), want), rep
        x = torch.arange(1 << 20, device="cuda").sum()    # eager work between replays
        torch.cuda.synchronize()
        del x


def test_errors_found_in_the_data():
    data = np.tile(np.arange(8, dtype=np.uint8), 5000)
    # a supplied tree without a code for symbol 7
    lens = np.zeros(256, np.uint8)
    lens[:6] = 3
    lens[6] = 2
    out, ws, ln, st = _buffers(data.size, 4096, tree=lens)
    P.pivco_encode_async(dev(data), out, ln, st, ws, 4096, tree=lens)
    torch.cuda.synchronize()
    assert int(st.item()) == P.E_ARG
    with pytest.raises(P.PivcoError):
        P.pivco_encode(dev(data), 4096, tree=lens)
    # out_cap too small: the needed length, nothing written
    want = O.encode(data, 4096)
    out, ws, ln, st = _buffers(data.size, 4096)
    small = out[:want.size - 1]
    P.pivco_encode_async(dev(data), small, ln, st, ws, 4096)
    torch.cuda.synchronize()
    assert int(st.item()) == P.E_CAPACITY
    assert int(ln.item()) == want.size
    assert bool((out == 0xAB).all())
    # empty input
    want = O.encode(np.zeros(0, np.uint8), 4096, ans_mode=3)
    out, ws, ln, st = _buffers(0, 4096, ans_mode=3)
    P.pivco_encode_async(torch.zeros(0, dtype=torch.uint8, device="cuda"), out, ln, st, ws, 4096, ans_mode=3)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and int(ln.item()) == want.size
    assert np.array_equal(out[:want.size].cpu().numpy(), want)
