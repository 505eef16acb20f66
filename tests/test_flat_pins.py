"""Pins of the flat-subtree trees (v2 streams; Sec. 2.2.3-2.2.4, Sec. 3.1-3.2,
Table 7): a hand-derived worked example, the proba80 row of Table 7, closed
forms of the node count and ops/B, brute force over short inputs, an
independent pure-Python reader, and corruption detection."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from independent import decode_stream, flat_tree

HERE = os.path.dirname(os.path.abspath(__file__))


def golden(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return json.load(f)


def lens_of(d):
    lens = np.zeros(256, np.uint8)
    for ch, l in d.items():
        lens[ord(ch)] = l
    return lens


def block_at(st, b):
    nb = int.from_bytes(st[20:24].tobytes(), "little")
    offs = [int.from_bytes(st[48 + 8 * i:56 + 8 * i].tobytes(), "little") for i in range(nb + 1)]
    return st[offs[b]:offs[b + 1]]


def test_worked_example():
    fx = golden("coconut_papaya_flat.json")
    x = np.frombuffer(fx["string"].encode(), np.uint8)
    lens = lens_of(fx["code_lengths"])
    st = O.encode(x, 64, tree_len=lens, flat=True)
    assert int.from_bytes(st[4:6].tobytes(), "little") == 2
    blk = block_at(st, 0)
    comp = int.from_bytes(blk[0:4].tobytes(), "little")
    assert blk[140:comp].tobytes().hex() == fx["after_length_table_hex"]
    bi = O.block_info(st, 0)
    assert bi["n_internal"] == fx["n_internal"]
    for k in ("depth", "flat", "n_v", "n_right"):
        assert bi[k].tolist() == fx[k], k
    assert int(bi["n_v"].sum()) == fx["ops_flat"]
    for merge in (False, True):
        assert O.decode(st, merge=merge).tobytes() == x.tobytes()
    # the same lengths in a v1 stream: 8 binary nodes and ops/B = mean code length
    st1 = O.encode(x, 64, tree_len=lens)
    b1 = O.block_info(st1, 0)
    assert b1["n_internal"] == 8 and int(b1["n_v"].sum()) == fx["ops_canonical"]


def test_proba80_row_of_table7():
    # Table 7: proba80 keeps 5 nodes and ops/B 1.251 under every tree optimization
    fx = golden("proba80.json")
    x = W.proba80_like(seed=3, n=1 << 20)
    b1 = O.block_info(O.encode(x, 1 << 20), 0)
    b2 = O.block_info(O.encode(x, 1 << 20, flat=True), 0)
    assert b1["n_internal"] == b2["n_internal"] == fx["naive_nodes"]
    assert int(b2["n_v"].sum()) == int(b1["n_v"].sum())
    assert not b2["flat"].any()


def _flat_closed_forms(lens, counts):
    """Nodes and ops of the regrouped tree from the class sizes alone: a
    class of c symbols of length l splits by the binary digits of c; a digit
    D >= 2 turns 2^D - 1 binary nodes into one flat node, through which its
    symbols pass once instead of D times."""
    m = int((lens > 0).sum())
    nodes, ops, flats = m - 1, 0, []
    for l in range(1, 16):
        syms = [s for s in range(256) if lens[s] == l]
        pos = 0
        for d in range(8, -1, -1):
            if len(syms) >> d & 1:
                grp = syms[pos:pos + (1 << d)]
                pos += 1 << d
                c = sum(int(counts[s]) for s in grp)
                if d >= 2:
                    nodes -= (1 << d) - 2
                    ops += c * (l - d + 1)
                    flats.append(d)
                else:
                    ops += c * l
    return nodes, ops, sorted(flats)


@pytest.mark.parametrize("seed", range(12))
def test_closed_forms_random(seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(2, 257))
    alpha = float(rng.choice([0.05, 0.3, 1.0, 10.0]))
    p = rng.dirichlet(np.ones(k) * alpha)
    x = rng.choice(rng.permutation(256)[:k], size=20000, p=p).astype(np.uint8)
    counts = np.bincount(x, minlength=256)
    if int((counts > 0).sum()) < 2:
        return
    st1 = O.encode(x, 1 << 20)
    st2 = O.encode(x, 1 << 20, flat=True)
    b1, b2 = O.block_info(st1, 0), O.block_info(st2, 0)
    lens = b2["len"]
    assert np.array_equal(lens, b1["len"])              # same code lengths
    nodes, ops, flats = _flat_closed_forms(lens, counts)
    assert b2["n_internal"] == nodes
    assert int(b2["n_v"].sum()) == ops
    assert sorted(int(d) for d in b2["flat"] if d) == flats
    # body bits: one per code bit, as in v1 (a flat node holds D per symbol)
    bits2 = sum(int(v) * max(int(d), 1) for v, d in zip(b2["n_v"], b2["flat"]))
    assert bits2 == int((counts * lens.astype(np.int64)).sum()) == int(b1["n_v"].sum())
    assert ops <= int(b1["n_v"].sum())
    for merge in (False, True):
        assert np.array_equal(O.decode(st2, merge=merge), x)


def test_tree_shapes_by_hand():
    # four symbols of length 2: the root itself is a flat node of depth 2
    lens = np.zeros(256, np.uint8); lens[[3, 7, 9, 200]] = 2
    nodes, leaf, groups = flat_tree(lens)
    assert nodes == {(0, 0): 2} and groups[(0, 0)] == [3, 7, 9, 200] and not leaf
    x = np.array([200, 3, 9, 7, 7, 200], np.uint8)
    st = O.encode(x, 16, tree_len=lens, flat=True)
    bi = O.block_info(st, 0)
    assert bi["n_internal"] == 1 and bi["flat"].tolist() == [2]
    # indices in (3, 7, 9, 200): 3 0 2 1 1 3; 2-bit fields LSB first:
    # byte 0 = 3 | 0 << 2 | 2 << 4 | 1 << 6 = 0x63, byte 1 = 1 | 3 << 2 = 0x0D
    q = [3, 0, 2, 1, 1, 3]
    want = bytearray(2)
    for j, v in enumerate(q):
        for k in range(2):
            if v >> k & 1:
                want[(2 * j + k) // 8] |= 1 << ((2 * j + k) % 8)
    blk = block_at(st, 0)
    assert blk[140 + 1 + 2:140 + 1 + 2 + 2].tobytes() == bytes(want) == bytes([0x63, 0x0D])
    for merge in (False, True):
        assert np.array_equal(O.decode(st, merge=merge), x)
    # two symbols of length 2 and four of length 3: a flat node of depth 2 on
    # the left of the root, a two-leaf binary node on the right
    lens = np.zeros(256, np.uint8); lens[[1, 2]] = 2; lens[[10, 11, 12, 13]] = 3
    nodes, leaf, groups = flat_tree(lens)
    assert nodes == {(0, 0): 0, (1, 0): 2, (1, 1): 0}
    assert groups[(1, 0)] == [10, 11, 12, 13] and leaf == {(2, 2): 1, (2, 3): 2}


def test_brute_force_short_inputs():
    # every string of length 1..5 over 4 symbols under three length vectors
    shapes = [{1: 2, 2: 2, 3: 2, 4: 2}, {1: 1, 2: 2, 3: 3, 4: 3}, {1: 2, 2: 2, 3: 3, 4: 3, 5: 3, 6: 3}]
    for shape in shapes:
        lens = np.zeros(256, np.uint8)
        for s, l in shape.items():
            lens[s] = l
        alphabet = sorted(shape)[:4]
        for n in range(1, 6):
            for t in itertools.product(alphabet, repeat=n):
                x = np.array(t, np.uint8)
                st = O.encode(x, 3, tree_len=lens, flat=True)
                assert np.array_equal(O.decode(st), x)
                assert np.array_equal(O.decode(st, merge=True), x)
                assert decode_stream(st) == x.tobytes()


@pytest.mark.parametrize("ans_mode", [0, 1, 2])
def test_independent_reader_agrees(ans_mode):
    rng = np.random.default_rng(100 + ans_mode)
    for _ in range(25):
        k = int(rng.integers(2, 60))
        p = rng.dirichlet(np.ones(k) * float(rng.choice([0.1, 1.0, 8.0])))
        x = rng.choice(rng.permutation(256)[:k], size=int(rng.integers(1, 4000)), p=p).astype(np.uint8)
        st = O.encode(x, int(rng.integers(1, 1500)), ans_mode=ans_mode, flat=True)
        assert decode_stream(st) == x.tobytes()
        assert np.array_equal(O.decode(st, merge=True), x)


def _corrupt(st, off, fn):
    b = st.copy()
    b[off] = fn(int(b[off]))
    return b


def test_corruption_is_rejected():
    fx = golden("coconut_papaya_flat.json")
    x = np.frombuffer(fx["string"].encode(), np.uint8)
    st = O.encode(x, 64, tree_len=lens_of(fx["code_lengths"]), flat=True)
    b0 = int.from_bytes(st[48:56].tobytes(), "little")
    cases = [
        b0 + 140, lambda v: v | 0x02,          # kind bit on flat node 1
        b0 + 141 + 2, lambda v: v | 1,         # n_right of flat node 1 nonzero
    ]
    # padding bits of the flat copy body (14 of 16 bits used)
    body = b0 + 141 + 8 + 2
    cases += [body + 1, lambda v: v | 0x80]
    for i in range(0, len(cases), 2):
        bad = _corrupt(st, cases[i], cases[i + 1])
        for merge in (False, True):
            with pytest.raises(O.OracleError):
                O.decode(bad, merge=merge)
    # a v2 stream is not a v1 stream: declaring version 1 changes the tree
    v1 = st.copy(); v1[4] = 1
    try:
        y = O.decode(v1)
    except O.OracleError:
        y = None
    assert y is None or not np.array_equal(y, x)
