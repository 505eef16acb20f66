"""Pins for the CPU oracle: every check compares it with something other than
itself -- values the paper prints, brute force, textbook Huffman, closed-form
invariants, or the independent pure-Python reader in ``independent.py``."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from independent import brute_min_cost, canonical, decode_stream, huffman_cost

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def counts_of(data):
    return np.bincount(np.frombuffer(bytes(data), dtype=np.uint8), minlength=256).astype(np.uint64)


def cost(counts, lens):
    return int(sum(int(c) * int(l) for c, l in zip(counts, lens)))


# --------------------------------------------------------------------------
# worked examples printed in the paper
# --------------------------------------------------------------------------

def test_huffman_word_tree():
    fx = golden("huffman.json")
    word = fx["word"].encode()
    c = counts_of(word)
    lens = O.lengths(c)
    present = [int(lens[s]) for s in range(256) if c[s]]
    assert sorted(present) == [2, 2, 3, 3, 3, 3]
    assert cost(c, lens) == 18 == brute_min_cost([int(x) for x in c if x], 4)
    assert lens[ord("h")] == fx["h_code_bits"]
    st = O.encode(np.frombuffer(word, np.uint8), 64)
    bi = O.block_info(st, 0)
    assert bi["n_internal"] == 5 and int(bi["n_v"][0]) == 7


def test_huffman_supplied_tree_reproduces_printed_code():
    fx = golden("huffman.json")
    word = np.frombuffer(fx["word"].encode(), np.uint8)
    lens = np.zeros(256, np.uint8)
    for ch, l in fx["supplied_lengths"].items():
        lens[ord(ch)] = l
    code = O.codes(lens)
    assert format(int(code[ord("h")]), "03b") == fx["h_code_printed"]
    st = O.encode(word, 64, tree_len=lens)
    assert bytes(O.decode(st)) == word.tobytes()
    assert decode_stream(st) == word.tobytes()
    # the classical stream starts with the code of 'h', the first letter
    bits, nbits = O.pivoted_to_classical(st, 64)
    first3 = "".join(str((bits[0] >> (7 - i)) & 1) for i in range(3))
    assert first3 == fx["h_code_printed"]


def test_coconut_papaya_bits():
    fx = golden("coconut_papaya.json")
    s = fx["string"].encode()
    c = counts_of(s)
    lens = O.lengths(c)
    total = cost(c, lens)
    assert total == fx["derived_total_code_bits"]
    assert round((total + len(s)) / len(s), 3) == fx["ops_per_byte_printed"]
    assert total == huffman_cost([int(x) for x in c if x])
    st = O.encode(np.frombuffer(s, np.uint8), 64)
    bi = O.block_info(st, 0)
    assert int(bi["n_v"].sum()) == total          # one bitmap bit per code bit


def test_proba80_like_statistics():
    fx = golden("proba80.json")
    x = W.proba80_like(seed=3, n=1 << 20)
    c = counts_of(x)
    lens = O.lengths(c)
    used = lens[c > 0]
    assert int((c > 0).sum()) == fx["symbols"]
    assert int(used.min()) == fx["min_len"] and int(used.max()) == fx["max_len"]
    lbar = cost(c, lens) / x.size
    assert abs(lbar - fx["huffman_bits"]) < 0.005
    p = c[c > 0] / x.size
    h = float(-(p * np.log2(p)).sum())
    assert abs(h - fx["entropy_bits"]) < 0.01
    st = O.encode(x, 1 << 20)
    bi = O.block_info(st, 0)
    assert bi["n_internal"] == fx["naive_nodes"]
    # ops/B of a naive tree equals the mean code length (Table 7)
    assert abs(int(bi["n_v"].sum()) / x.size - lbar) < 1e-12


# --------------------------------------------------------------------------
# optimality and structure of the code-length builder
# --------------------------------------------------------------------------

def test_brute_force_optimal_lengths():
    rng = np.random.default_rng(7)
    for _ in range(300):
        m = int(rng.integers(2, 7))
        L = int(rng.integers(max(1, math.ceil(math.log2(m))), 5))
        w = rng.integers(1, 50, size=m)
        c = np.zeros(256, np.uint64)
        syms = rng.choice(256, size=m, replace=False)
        c[syms] = w
        lens = O.lengths(c, max_len=L)
        assert int(lens.max()) <= L
        assert cost(c, lens) == brute_min_cost(list(w), L)


def test_unlimited_equals_textbook_huffman():
    rng = np.random.default_rng(8)
    for _ in range(200):
        m = int(rng.integers(2, 80))
        c = np.zeros(256, np.uint64)
        c[rng.choice(256, size=m, replace=False)] = rng.integers(1, 10000, size=m)
        lens = O.lengths(c, max_len=15)
        # 15 bits suffice for these weights whenever the Huffman depth fits
        assert cost(c, lens) <= huffman_cost([int(x) for x in c if x])
        assert cost(c, lens) >= huffman_cost([int(x) for x in c if x])


def test_length_limit_and_kraft():
    fib = [1, 1]
    while len(fib) < 30:
        fib.append(fib[-1] + fib[-2])
    c = np.zeros(256, np.uint64)
    c[:30] = fib
    lens = O.lengths(c, max_len=11)
    assert int(lens.max()) == 11                      # the limit binds
    assert sum(2.0 ** -int(l) for l in lens if l) == 1.0
    assert cost(c, lens) >= huffman_cost(fib)
    # monotone: a more frequent symbol never gets a longer code
    for a in range(30):
        for b in range(30):
            if c[a] > c[b]:
                assert lens[a] <= lens[b]


def test_canonical_codes_prefix_free():
    rng = np.random.default_rng(9)
    for _ in range(50):
        m = int(rng.integers(2, 257))
        c = np.zeros(256, np.uint64)
        c[rng.choice(256, size=m, replace=False)] = rng.integers(1, 1 << 20, size=m)
        lens = O.lengths(c)
        code = O.codes(lens)
        want = canonical([int(x) for x in lens])
        for s, (cd, l) in want.items():
            assert int(code[s]) == cd and int(lens[s]) == l
        strs = sorted(format(cd, f"0{l}b") for cd, l in want.values())
        for a, b in zip(strs, strs[1:]):
            assert not b.startswith(a)


# --------------------------------------------------------------------------
# codec round trips and invariants
# --------------------------------------------------------------------------

def test_all_short_strings_roundtrip():
    n_checked = 0
    for length in range(1, 9):
        for t in itertools.product(b"abc", repeat=length):
            x = np.frombuffer(bytes(t), np.uint8)
            st = O.encode(x, 4)                          # several tiny blocks
            assert bytes(O.decode(st)) == x.tobytes()
            if length <= 6:
                assert bytes(O.decode(st, merge=True)) == x.tobytes()
                assert decode_stream(st) == x.tobytes()
            n_checked += 1
    assert n_checked == sum(3 ** k for k in range(1, 9))


def test_forced_rans_small_strings_independent_reader():
    rng = np.random.default_rng(10)
    for n in [1, 2, 31, 32, 33, 63, 64, 65, 200, 1000]:
        for k in [2, 3, 7, 40]:
            x = rng.integers(0, k, size=n).astype(np.uint8)
            if len(set(x.tolist())) < 2:
                continue
            st = O.encode(x, 1 << 20, ans_mode=2)
            assert decode_stream(st) == x.tobytes()
            assert bytes(O.decode(st)) == x.tobytes()


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_invariants_on_workload_blocks(mode):
    x = W.zipf256m(seed=2, scale=1024).jobs[0]                 # 256 KiB
    y = W.skew256m(seed=2, scale=512).jobs[0]                  # 512 KiB
    for data, bs in [(x, 64 << 10), (y, 128 << 10)]:
        st = O.encode(data, bs, ans_mode=mode)
        assert np.array_equal(O.decode(st), data)
        assert np.array_equal(O.decode(st, merge=True), data)
        info = O.stream_info(st)
        aw = 0
        for b in range(info["n_blocks"]):
            blk = data[b * bs:(b + 1) * bs]
            c = counts_of(blk)
            bi = O.block_info(st, b)
            lens = bi["len"]
            m = int((c > 0).sum())
            assert bi["n_internal"] == m - 1                     # Table 7: nodes = #syms - 1
            assert sum(2.0 ** -int(l) for l in lens if l) == 1.0  # Kraft equality
            assert int(bi["n_v"].sum()) == cost(c, lens)          # bits = sum count x len
            assert int(bi["n_v"][0]) == blk.size
            for i in range(bi["n_internal"]):
                want = O.select_ans(mode, int(bi["n_v"][i]), int(bi["n_right"][i]))
                assert bool(bi["kind"][i]) == want
                if bi["kind"][i]:
                    aw += (int(bi["n_v"][i]) + 31) // 32
        assert info["ans_words"] == aw


def test_classical_listing1_crosscheck():
    rng = np.random.default_rng(11)
    for n in [2, 10, 1000, 50000]:
        x = W.draw(rng, W.zipf_p(1.1, rng), n)
        if len(set(x.tolist())) < 2:
            continue
        st = O.encode(x, 1 << 20)
        lens = O.block_info(st, 0)["len"]
        bits, nbits = O.classical_encode(x, lens)
        assert np.array_equal(O.classical_decode(bits, nbits, lens, n), x)
        pbits, pnbits = O.pivoted_to_classical(st, bits.size + 8)
        assert pnbits == nbits and np.array_equal(pbits, bits)


def test_constant_empty_and_ragged_blocks():
    for n, bs in [(0, 16), (1, 16), (17, 16), (4097, 4096), (100, 7)]:
        x = np.full(n, 42, np.uint8)
        st = O.encode(x, bs)
        assert np.array_equal(O.decode(st, n=n), x)
    x = np.array([1, 2] * 50 + [3], np.uint8)
    for bs in [1, 2, 3, 64, 101, 1000]:
        st = O.encode(x, bs)
        assert np.array_equal(O.decode(st), x)
        assert decode_stream(st) == x.tobytes()


# --------------------------------------------------------------------------
# binary rANS
# --------------------------------------------------------------------------

def _binary_entropy(p):
    return 0.0 if p <= 0 or p >= 1 else -(p * math.log2(p) + (1 - p) * math.log2(1 - p))


@pytest.mark.parametrize("nbits", [0, 1, 31, 32, 33, 1000, 65535, 65536, 65537, 300000])
def test_rans_roundtrip(nbits):
    rng = np.random.default_rng(nbits)
    for p in [0.02, 0.3, 0.5, 0.97]:
        bits = (rng.random(nbits) < p).astype(np.uint8)
        packed = np.packbits(bits, bitorder="little").tobytes()
        q = O.p1q(max(nbits, 1), int(bits.sum()))
        body = O.rans_encode(packed, nbits, q)
        assert O.rans_decode(body, nbits, q) == packed


def test_rans_size_near_entropy():
    rng = np.random.default_rng(12)
    nbits = 1 << 20
    for p in [0.05, 0.1, 0.5, 0.93]:
        bits = (rng.random(nbits) < p).astype(np.uint8)
        ones = int(bits.sum())
        q = O.p1q(nbits, ones)
        body = O.rans_encode(np.packbits(bits, bitorder="little").tobytes(), nbits, q)
        pq = q / 4096.0
        ideal = -(ones * math.log2(pq) + (nbits - ones) * math.log2(1 - pq))
        chunks = nbits >> 16
        overhead = chunks * (132 + 3) * 8 + 32 * 32 * chunks
        assert len(body) * 8 <= ideal * 1.005 + overhead
        assert len(body) * 8 >= nbits * _binary_entropy(ones / nbits) * 0.99
    bits = (rng.random(nbits) < 0.5).astype(np.uint8)
    body = O.rans_encode(np.packbits(bits, bitorder="little").tobytes(), nbits, 2048)
    assert abs(len(body) * 8 / nbits - 1.0) < 0.02


def test_rans_corruption_detected():
    rng = np.random.default_rng(13)
    nbits = 5000
    bits = (rng.random(nbits) < 0.08).astype(np.uint8)
    packed = np.packbits(bits, bitorder="little").tobytes()
    q = O.p1q(nbits, int(bits.sum()))
    body = bytearray(O.rans_encode(packed, nbits, q))
    bad = bytearray(body)
    bad[4] ^= 0x10                                          # a lane's initial state
    with pytest.raises(O.OracleError):
        assert O.rans_decode(bytes(bad), nbits, q) == packed and False
    bad = bytearray(body)
    bad[0] = (bad[0] + 1) & 0xFF                             # word count
    with pytest.raises(O.OracleError):
        O.rans_decode(bytes(bad), nbits, q)


def test_selection_rule_boundaries():
    # one-bit fraction strictly below 0.1 or strictly above 0.9
    assert O.select_ans(1, 100, 9) and not O.select_ans(1, 100, 10)
    assert not O.select_ans(1, 100, 90) and O.select_ans(1, 100, 91)
    assert O.select_ans(1, 1, 0) and O.select_ans(1, 1, 1)
    assert not O.select_ans(0, 100, 0) and O.select_ans(2, 100, 50)
    assert not O.select_ans(2, 0, 0)
    for n in [1, 2, 3, 10, 4095, 1 << 20]:
        qs = [O.p1q(n, r) for r in range(0, n + 1, max(1, n // 50))]
        assert all(1 <= q <= 4095 for q in qs) and qs == sorted(qs)
    assert O.p1q(1 << 20, 1 << 19) == 2048


def test_p1q_rounds_to_nearest():
    # The rANS probability of a 1 bit is the node's one-bit fraction in 12-bit
    # fixed point, rounded to nearest and clamped to [1, 4095] (the reading of
    # the 12-bit binary coder written down for this format).  Values worked
    # out by hand; truncation would give the numbers in the comments.
    assert O.p1q(3, 2) == 2731        # 8192 / 3 = 2730.67 (floor: 2730)
    assert O.p1q(5, 3) == 2458        # 12288 / 5 = 2457.6 (floor: 2457)
    assert O.p1q(9, 7) == 3186        # 28672 / 9 = 3185.78 (floor: 3185)
    assert O.p1q(3, 1) == 1365        # 4096 / 3 = 1365.33 rounds down
    assert O.p1q(2, 1) == 2048        # exactly one half
    assert O.p1q(8193, 1) == 1        # 0.4999 rounds to 0, clamped up to 1
    assert O.p1q(10000, 9999) == 4095  # 4095.59 + 0.5 = 4096.09: 4096, clamped down
    assert O.p1q(7, 0) == 1 and O.p1q(7, 7) == 4095


# --------------------------------------------------------------------------
# corrupt streams are rejected
# --------------------------------------------------------------------------

def test_corrupt_streams_rejected():
    rng = np.random.default_rng(14)
    x = W.draw(rng, W.zipf_p(1.1, rng), 20000)
    st = O.encode(x, 8192, ans_mode=1)
    assert np.array_equal(O.decode(st), x)
    info = O.stream_info(st)

    def expect_bad(buf):
        with pytest.raises(O.OracleError) as e:
            O.decode(buf, n=x.size)
        assert e.value.code in (O.E_CORRUPT, O.E_CAPACITY)

    expect_bad(st[:-5])                                      # truncated
    b = st.copy(); b[0] ^= 1; expect_bad(b)                 # magic
    off0 = int(np.frombuffer(st[48:56].tobytes(), np.uint64)[0])
    b = st.copy(); b[off0 + 12] = (b[off0 + 12] & 0xF0) | 0x1; expect_bad(b)  # Kraft
    b = st.copy(); b[off0 + 12 + 128 + 1] ^= 0x01; expect_bad(b)  # n_right / kinds
    b = st.copy(); b[off0 + 4] ^= 0x01; expect_bad(b)       # block length
    assert info["n_blocks"] == 3
