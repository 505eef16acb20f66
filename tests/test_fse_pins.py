"""Pins of the selective tANS of bitmap bytes (Sec. 5.2, App. D's FSE marker,
App. F's cursors; the readings are written out in oracle/fse_ref.c): tables
against an exact-rational construction and the tANS closed form, the coded
size between the entropy and the table's cost, the selection rule's
constants and depth limits from an independent cost, the XOR marker, an
independent reader, corruption, and whole streams (ans_mode 3)."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from independent import decode_stream, fse_body_bits, fse_table


def _bits(rng, n, p):
    return (rng.random(n) < p).astype(np.uint8)


def _pack(bits):
    return np.packbits(bits, bitorder="little")


@pytest.mark.parametrize("t", [1, 2, 13, 14, 26, 41, 46, 50])
def test_tables_match_exact_construction(t):
    norm = O.fse_norm(t)
    assert int(norm.sum()) == 2048 and int(norm.min()) >= 1
    ref, table = fse_table(t)
    assert list(norm) == ref
    if t == 1:
        assert set(norm.tolist()) == {8}                 # s = 1/2: every byte 2^11 / 256
    else:
        assert int(norm[0xFF]) == int(norm.max())        # the all-ones byte is (one of) the likeliest
    # tANS closed form: each symbol's states (k = n_b .. 2 n_b - 1) cover the
    # next-state range [0, 2^11) exactly once with their bit-read intervals
    for b in (0, 0x0F, 0xFF):
        cover = sorted((base, base + (1 << nb)) for (s, nb, base) in table if s == b)
        assert cover[0][0] == 0 and cover[-1][1] == 2048
        assert all(cover[i][1] == cover[i + 1][0] for i in range(len(cover) - 1))


def _cost(t):
    """Expected bits per bitmap bit of table t at its own skew (numpy)."""
    norm = np.array(fse_table(t)[0], dtype=np.float64)
    s = (t + 49) / 100
    k = np.array([bin(b).count("1") for b in range(256)])
    p = s ** k * (1 - s) ** (8 - k)
    return float((p * (11 - np.log2(norm))).sum() / 8)


@pytest.mark.parametrize("p", [0.7, 0.9, 0.97])
def test_coded_size_between_entropy_and_table_cost(p):
    rng = np.random.default_rng(int(p * 100))
    n = 1 << 20
    bits = _bits(rng, n, p)
    sel, m = O.fse_select(n, int(bits.sum()), 0)
    assert sel and not m & 0x80
    t = m & 0x7F
    assert t == round(100 * bits.mean()) - 49
    body = O.fse_encode(_pack(bits), n, m)
    per_bit = 8 * body.size / n
    h = -(p * math.log2(p) + (1 - p) * math.log2(1 - p))
    headers = 8 * 128 * (n >> 16) / n                    # cursor states and lengths per chunk
    assert h < per_bit < _cost(t) + headers + 0.01
    assert abs(O.fse_cost(t) - _cost(t)) < 1e-9


def test_selection_rule_constants():
    # fewer than 256 bits (32 bytes): never
    assert not O.fse_select(255, 250, 0)[0]
    assert O.fse_select(256, 250, 0)[0]
    # skew 0.625 exactly is not above the threshold
    assert not O.fse_select(800, 500, 0)[0]
    # table choice rounds 100 * skew, halves up: 0.645 -> 65 -> table 16
    sel, m = O.fse_select(1000, 645, 0)
    assert sel and m == 16
    # more zeros than ones: the complemented bitmap's table and the XOR marker
    sel, m = O.fse_select(1000, 100, 0)
    assert sel and m == (90 - 49) | 0x80


@pytest.mark.parametrize("t", [15, 20, 27, 33, 41, 44, 46])
def test_depth_limit_from_benefit_ratio(t):
    h = _cost(t)
    dmax = max(d for d in range(16) if (d + h) / (d + 1) < 0.95)
    n = 100_000
    ones = round(n * (t + 49) / 100)
    assert O.fse_select(n, ones, dmax)[0]
    assert not O.fse_select(n, ones, dmax + 1)[0]


def test_xor_marker_is_the_complement():
    rng = np.random.default_rng(3)
    bits = _bits(rng, 50_000, 0.92)
    a = O.fse_encode(_pack(bits), bits.size, 43)
    b = O.fse_encode(_pack(1 - bits), bits.size, 43 | 0x80)
    assert np.array_equal(a, b)
    assert np.array_equal(O.fse_decode(b, bits.size, 43 | 0x80), _pack(1 - bits))


@pytest.mark.parametrize("cl", [8, 11, 16])
def test_round_trip_and_independent_reader(cl):
    rng = np.random.default_rng(cl)
    for n in [1, 7, 8, 9, 255, 256, 257, 4095, 33333]:
        for t in (1, 30, 50):
            bits = _bits(rng, n, 0.8)
            m = t | (0x80 if n % 2 else 0)
            body = O.fse_encode(_pack(bits), n, m, cl)
            assert np.array_equal(O.fse_decode(body, n, m, cl), _pack(bits))
            assert fse_body_bits(bytes(body), n, m, cl) == bits.tolist()


def test_corruption_is_detected():
    rng = np.random.default_rng(9)
    bits = _bits(rng, 70_000, 0.9)
    m = 41
    body = O.fse_encode(_pack(bits), bits.size, m)
    caught = 0
    for k in range(40):
        bad = body.copy()
        pos = int(rng.integers(128, bad.size))
        bad[pos] ^= np.uint8(1 << int(rng.integers(0, 8)))
        try:
            out = O.fse_decode(bad, bits.size, m)
            caught += int(not np.array_equal(out, _pack(bits)))    # undetected and wrong: counted below
        except O.OracleError:
            caught += 1
    assert caught == 40
    bad = body.copy(); bad[0] ^= 1                                # a cursor's first state
    with pytest.raises(O.OracleError):
        O.fse_decode(bad, bits.size, m)


def test_streams_with_selective_tans():
    x = W.skew256m(seed=4, scale=1024).jobs[0]
    for flat in (False, True):
        st = O.encode(x, 1 << 16, ans_mode=3, flat=flat)
        assert int.from_bytes(st[6:8].tobytes(), "little") == 1
        assert np.array_equal(O.decode(st), x) and np.array_equal(O.decode(st, merge=True), x)
        assert decode_stream(st) == x.tobytes()
        kinds = [O.block_info(st, b)["kind"] for b in range(4)]
        assert any(k.any() for k in kinds)
    # coded no larger than the binary-rANS stream by more than the chunk headers
    a = O.encode(x, 1 << 16, ans_mode=1)
    b = O.encode(x, 1 << 16, ans_mode=3)
    assert b.size < a.size * 1.05
