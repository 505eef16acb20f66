"""Pins of the PivCo-Golomb oracle (App. G): a hand-derived worked example,
brute force over every short input, closed forms of the bitmap sizes, an
independent pure-Python reader of the format, and corruption detection."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _read_blocks(stream):
    """Independent reader: bitmaps of every block as Python bit lists."""
    b = bytes(stream)
    assert b[:4] == b"PVG1" and b[4] == 1
    n_total = int.from_bytes(b[8:16], "little")
    nb = int.from_bytes(b[20:24], "little")
    offs = [int.from_bytes(b[32 + 8 * i:40 + 8 * i], "little") for i in range(nb + 1)]
    blocks = []
    for i in range(nb):
        p = b[offs[i]:offs[i + 1]]
        n = int.from_bytes(p[4:8], "little")
        K = int.from_bytes(p[8:10], "little")
        nk = [n] + [int.from_bytes(p[12 + 4 * j:16 + 4 * j], "little") for j in range(K - 1)]
        o = 12 + 4 * (K - 1) if K else 12
        bms = []
        for k in range(K):
            nbytes = (nk[k] + 7) // 8
            bits = [(p[o + j // 8] >> (j % 8)) & 1 for j in range(nk[k])]
            bms.append(bits)
            o += nbytes
        blocks.append((n, K, nk, bms))
    return n_total, blocks


def _python_decode(stream):
    """Reads every value's code: 0-bits until the first 1-bit, one bitmap
    after the other (a cursor per bitmap)."""
    _, blocks = _read_blocks(stream)
    out = []
    for n, K, nk, bms in blocks:
        cur = [0] * K
        for _ in range(n):
            k = 0
            while True:
                bit = bms[k][cur[k]]
                cur[k] += 1
                if bit:
                    break
                k += 1
            out.append(k)
    return np.array(out, dtype=np.uint8)


def test_worked_example():
    g = json.load(open(os.path.join(HERE, "golden", "golomb_small.json")))
    x = np.array(g["values"], np.uint8)
    st = O.golomb_encode(x, 16)
    block = st[48:48 + len(g["block_hex"]) // 2].tobytes().hex()
    assert block == g["block_hex"]
    _, blocks = _read_blocks(st)
    assert sum(blocks[0][2]) == g["code_bits_total"]
    assert np.array_equal(O.golomb_decode(st), x) and np.array_equal(O.golomb_decode_merge(st), x)


def test_brute_force_short_inputs():
    for n in range(1, 7):
        for seq in itertools.product(range(4), repeat=n):
            x = np.array(seq, np.uint8)
            st = O.golomb_encode(x, 4)
            assert np.array_equal(O.golomb_decode(st), x), seq
            assert np.array_equal(O.golomb_decode_merge(st), x), seq
    st = O.golomb_encode(np.zeros(0, np.uint8), 4)
    assert st.size == 40 and O.golomb_decode(st, n=0).size == 0


def test_bitmap_sizes_closed_forms():
    # bitmap k holds exactly the values >= k; all bitmaps together hold
    # sum(v + 1) bits (the unary code lengths); the last one is all ones
    rng = np.random.default_rng(3)
    for q in (0.2, 0.5, 0.8, 0.95):
        x = np.minimum(rng.geometric(1 - q, size=20000) - 1, 255).astype(np.uint8)
        st = O.golomb_encode(x, 5000)
        _, blocks = _read_blocks(st)
        for b, (n, K, nk, bms) in enumerate(blocks):
            xb = x[5000 * b:5000 * (b + 1)].astype(np.int64)
            assert K == xb.max() + 1
            assert nk == [int((xb >= k).sum()) for k in range(K)]
            assert sum(nk) == int((xb + 1).sum())
            assert all(bms[-1])
            for k in range(K):
                assert sum(bms[k]) == int((xb == k).sum())
        assert np.array_equal(_python_decode(st), x)
        assert np.array_equal(O.golomb_decode(st), x)
        assert np.array_equal(O.golomb_decode_merge(st), x)


def test_full_range_and_ragged_blocks():
    rng = np.random.default_rng(4)
    x = rng.integers(0, 256, size=3001).astype(np.uint8)
    x[17] = 255
    st = O.golomb_encode(x, 1000)
    assert np.array_equal(O.golomb_decode(st), x)
    assert np.array_equal(O.golomb_decode_merge(st), x)
    assert np.array_equal(_python_decode(st), x)


def test_corruption_detected():
    rng = np.random.default_rng(5)
    x = np.minimum(rng.geometric(0.4, size=4000) - 1, 255).astype(np.uint8)
    st = O.golomb_encode(x, 4000)
    caught = 0
    for _ in range(40):
        b = st.copy()
        p = int(rng.integers(48 + 12, len(st)))
        b[p] ^= np.uint8(1 << int(rng.integers(0, 8)))
        try:
            same = np.array_equal(O.golomb_decode(b, n=x.size), x)
        except O.OracleError:
            caught += 1
            continue
        assert not same or b[p] == st[p]
    assert caught >= 30
    with pytest.raises(O.OracleError):
        O.golomb_decode(st[:-4], n=x.size)
