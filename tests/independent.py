"""Pure-Python checks written from textbook definitions, used to pin the C
oracle.  They share nothing with ``oracle/`` or the GPU library and are only
fast enough for small inputs.

* ``huffman_cost``      textbook Huffman (two-smallest merge with a heap)
* ``brute_min_cost``    exhaustive search over length vectors obeying Kraft
* ``canonical``         canonical code numbering (ref. [5] of the paper)
* ``decode_stream``     a second reader of the v1 wire format that walks the
                        code tree bit by bit as in Listing 1 (Sec. 1.1), with
                        its own binary-rANS reader for entropy-coded nodes;
                        v2 streams (flat subtrees, Sec. 2.2.3-2.2.4) through
                        ``flat_tree``
* ``flat_tree``         the regrouped tree from code lengths: each length
                        class split by the binary digits of its size
* ``fse_table``         the selective-tANS tables of the format (exact
                        rationals) and a reader of such node bodies
"""
import heapq
import itertools
import struct


def huffman_cost(weights):
    w = [x for x in weights if x > 0]
    if len(w) < 2:
        return 0
    heapq.heapify(w)
    cost = 0
    while len(w) > 1:
        a = heapq.heappop(w)
        b = heapq.heappop(w)
        cost += a + b
        heapq.heappush(w, a + b)
    return cost


def brute_min_cost(weights, max_len):
    w = [x for x in weights if x > 0]
    best = None
    for lens in itertools.product(range(1, max_len + 1), repeat=len(w)):
        if sum(2.0 ** -l for l in lens) <= 1.0 + 1e-12:
            c = sum(a * b for a, b in zip(w, lens))
            best = c if best is None else min(best, c)
    return best


def canonical(lens):
    """{symbol: (code, length)} with codes numbered by (length, symbol)."""
    order = sorted((l, s) for s, l in enumerate(lens) if l)
    out, code, prev = {}, 0, None
    for i, (l, s) in enumerate(order):
        if i:
            code = (code + 1) << (l - prev)
        out[s] = (code, l)
        prev = l
    return out


def _rans_bits(body, nbits, p1q, chunk_log2):
    f = [4096 - p1q, p1q]
    c = [0, 4096 - p1q]
    bits, o, C = [], 0, 1 << chunk_log2
    for start in range(0, nbits, C):
        cl = min(C, nbits - start)
        nw = struct.unpack_from("<I", body, o)[0]
        x = list(struct.unpack_from("<32I", body, o + 4))
        words = struct.unpack_from(f"<{nw}H", body, o + 132)
        chunk, pos = [0] * cl, 0
        for k in range((cl + 31) // 32):
            for lane in range(32):
                j = 32 * k + lane
                if j >= cl:
                    continue
                slot = x[lane] & 4095
                b = 1 if slot >= f[0] else 0
                x[lane] = f[b] * (x[lane] >> 12) + slot - c[b]
                if x[lane] < 65536:
                    x[lane] = (x[lane] << 16) | words[pos]
                    pos += 1
                chunk[j] = b
        assert pos == nw and all(v == 65536 for v in x)
        bits += chunk
        o += (132 + 2 * nw + 3) & ~3
    return bits


def flat_tree(lens):
    """The flat-subtree tree of a length vector.

    Returns (nodes, leaf): nodes maps (depth, prefix) -> D for every node
    (0 for a binary node, D >= 2 for a flat one; a group of two symbols is a
    binary node), and leaf maps (depth, prefix) -> symbol for the leaves
    that hang below binary nodes.  A flat node's symbols are listed in
    ``groups[(depth, prefix)]`` (third value returned)."""
    by_len = {}
    for sym, l in enumerate(lens):
        if l:
            by_len.setdefault(l, []).append(sym)
    items = []                                   # (depth, -D, symbols)
    for l, syms in by_len.items():
        pos = 0
        for d in range(8, -1, -1):               # binary digits of the class size, high first
            if len(syms) >> d & 1:
                items.append((l - d, -d, syms[pos:pos + (1 << d)]))
                pos += 1 << d
    items.sort(key=lambda t: (t[0], t[1]))
    nodes, leaf, groups = {}, {}, {}
    code, prev = 0, None
    for i, (m, negd, syms) in enumerate(items):
        if i:
            code = (code + 1) << (m - prev)
        prev = m
        for k in range(m):
            nodes[(k, code >> (m - k))] = 0
        d = -negd
        if d == 0:
            leaf[(m, code)] = syms[0]
        elif d == 1:
            nodes[(m, code)] = 0
            leaf[(m + 1, 2 * code)] = syms[0]
            leaf[(m + 1, 2 * code + 1)] = syms[1]
        else:
            nodes[(m, code)] = d
            groups[(m, code)] = syms
    return nodes, leaf, groups


def fse_table(t):
    """tANS table t (1..50) from the format's readings, written afresh:
    counts by largest remainder over P(b) = s^k (1-s)^(8-k), s = (t+49)/100,
    the spread with step 1283, and the decoding entries (symbol, bits read,
    base of the next state)."""
    from fractions import Fraction
    s = Fraction(t + 49, 100)
    exact = [s ** bin(b).count("1") * (1 - s) ** (8 - bin(b).count("1")) * 2048 for b in range(256)]
    norm = [max(1, int(e)) for e in exact]
    frac = [e - int(e) if int(e) >= 1 else Fraction(0) for e in exact]
    while sum(norm) < 2048:
        b = max(range(256), key=lambda i: (frac[i], -i))
        norm[b] += 1
        frac[b] = Fraction(0)
    if sum(norm) > 2048:
        b = max(range(256), key=lambda i: (norm[i], -i))
        norm[b] -= sum(norm) - 2048
    spread, pos = [0] * 2048, 0
    for b in range(256):
        for _ in range(norm[b]):
            spread[pos] = b
            pos = (pos + 1283) % 2048
    nxt = list(norm)
    table = []
    for X in range(2048):
        b = spread[X]
        k = nxt[b]
        nxt[b] += 1
        nb = 11 - (k.bit_length() - 1)
        table.append((b, nb, (k << nb) - 2048))
    return norm, table


def fse_body_bits(body, nbits, marker, chunk_log2):
    """Bitmap bits of a selective-tANS node body (32 cursors per chunk)."""
    _, table = fse_table(marker & 0x7F)
    flip = 0xFF if marker & 0x80 else 0
    nbytes, cb = (nbits + 7) // 8, (1 << chunk_log2) // 8
    out, o = bytearray(nbytes), 0
    for c0 in range(0, nbytes, cb):
        n = min(cb, nbytes - c0)
        x0 = struct.unpack_from("<32H", body, o)
        lens = struct.unpack_from("<32H", body, o + 64)
        so = o + 128
        for lane in range(32):
            X, p = x0[lane], 0
            stream = body[so:so + lens[lane]]
            for i in range((n - lane + 31) // 32 if n > lane else 0):
                b, nb, base = table[X]
                v = sum(((stream[(p + k) >> 3] >> ((p + k) & 7)) & 1) << k for k in range(nb))
                p += nb
                X = base + v
                out[c0 + lane + 32 * i] = b ^ flip
            assert X == 0 and (p + 7) // 8 == lens[lane]
            so += lens[lane]
        o = (so + 3) & ~3
    return [(out[j >> 3] >> (j & 7)) & 1 for j in range(nbits)]


def decode_stream(stream):
    """Decode a v1 or v2 stream (small inputs only)."""
    s = bytes(stream)
    magic, ver, flags, n_total, bs, nb, max_len, cl2 = struct.unpack_from("<IHHQIIBB", s, 0)
    assert magic == 0x31435650 and ver in (1, 2) and flags in (0, 1)
    offs = struct.unpack_from(f"<{nb + 1}Q", s, 48)
    out = bytearray()
    for b in range(nb):
        p = offs[b]
        comp, n, mode, csym, cw, _ = struct.unpack_from("<IIBBBB", s, p)
        if mode == 1:
            out += bytes([csym]) * n
            continue
        lens = []
        for j in range(128):
            lens += [s[p + 12 + j] & 15, s[p + 12 + j] >> 4]
        if ver == 1:
            codes = canonical(lens)
            # the code tree: internal nodes keyed by (depth, prefix)
            nodes = {(d, code >> (l - d)): 0 for code, l in codes.values() for d in range(l)}
            leaf = {(l, code): sym for sym, (code, l) in codes.items()}
            groups = {}
        else:
            nodes, leaf, groups = flat_tree(lens)
        internal = sorted(nodes)
        I = len(internal)
        q = p + 140
        kind = [(s[q + i // 8] >> (i % 8)) & 1 for i in range(I)]
        q += (I + 7) // 8
        fmt = "<H" if cw == 2 else "<I"
        n_right = [struct.unpack_from(fmt, s, q + cw * i)[0] for i in range(I)]
        q += cw * I
        nv = {internal[0]: n}
        for i, (d, pre) in enumerate(internal):
            v = nv[(d, pre)]
            if nodes[(d, pre)]:
                assert n_right[i] == 0 and kind[i] == 0
                continue
            nv[(d + 1, 2 * pre)] = v - n_right[i]
            nv[(d + 1, 2 * pre + 1)] = n_right[i]
        bitmaps = {}
        for i, node in enumerate(internal):
            if kind[i]:
                continue
            nbits = nv[node] * max(nodes[node], 1)
            bitmaps[node] = [(s[q + j // 8] >> (j % 8)) & 1 for j in range(nbits)]
            q += (nbits + 7) // 8
        for i, node in enumerate(internal):
            if not kind[i]:
                continue
            q = (q + 3) & ~3
            p1q, _, blen = struct.unpack_from("<HHI", s, q)
            if flags:                            # selective tANS on bytes
                bitmaps[node] = fse_body_bits(s[q + 8:q + 8 + blen], nv[node], p1q & 0xFF, cl2)
            else:
                bitmaps[node] = _rans_bits(s[q + 8:q + 8 + blen], nv[node], p1q, cl2)
            q += 8 + blen
        cursor = {node: 0 for node in internal}
        for _ in range(n):                       # Listing 1
            d, pre = 0, 0
            while (d, pre) not in leaf:
                D = nodes[(d, pre)]
                c = cursor[(d, pre)]
                cursor[(d, pre)] += 1
                if D:                            # flat node: a D-bit index, LSB first
                    bits = bitmaps[(d, pre)][D * c:D * c + D]
                    out.append(groups[(d, pre)][sum(b << k for k, b in enumerate(bits))])
                    break
                bit = bitmaps[(d, pre)][c]
                d, pre = d + 1, 2 * pre + bit
            else:
                out.append(leaf[(d, pre)])
    return bytes(out)
