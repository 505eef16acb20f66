"""Pure-Python checks written from textbook definitions, used to pin the C
oracle.  They share nothing with ``oracle/`` or the GPU library and are only
fast enough for small inputs.

* ``huffman_cost``      textbook Huffman (two-smallest merge with a heap)
* ``brute_min_cost``    exhaustive search over length vectors obeying Kraft
* ``canonical``         canonical code numbering (ref. [5] of the paper)
* ``decode_stream``     a second reader of the v1 wire format that walks the
                        code tree bit by bit as in Listing 1 (Sec. 1.1), with
                        its own binary-rANS reader for entropy-coded nodes
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


def decode_stream(stream):
    """Decode a v1 stream (small inputs only)."""
    s = bytes(stream)
    magic, ver, flags, n_total, bs, nb, max_len, cl2 = struct.unpack_from("<IHHQIIBB", s, 0)
    assert magic == 0x31435650 and ver == 1 and flags == 0
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
        codes = canonical(lens)
        # the code tree: internal nodes keyed by (depth, prefix)
        internal = sorted({(d, code >> (l - d)) for code, l in codes.values() for d in range(l)})
        leaf = {(l, code): sym for sym, (code, l) in codes.items()}
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
            nv[(d + 1, 2 * pre)] = v - n_right[i]
            nv[(d + 1, 2 * pre + 1)] = n_right[i]
        bitmaps = {}
        for i, node in enumerate(internal):
            if kind[i]:
                continue
            m = (nv[node] + 7) // 8
            bitmaps[node] = [(s[q + j // 8] >> (j % 8)) & 1 for j in range(nv[node])]
            q += m
        for i, node in enumerate(internal):
            if not kind[i]:
                continue
            q = (q + 3) & ~3
            p1q, _, blen = struct.unpack_from("<HHI", s, q)
            bitmaps[node] = _rans_bits(s[q + 8:q + 8 + blen], nv[node], p1q, cl2)
            q += 8 + blen
        cursor = {node: 0 for node in internal}
        for _ in range(n):                       # Listing 1
            d, pre = 0, 0
            while (d, pre) not in leaf:
                bit = bitmaps[(d, pre)][cursor[(d, pre)]]
                cursor[(d, pre)] += 1
                d, pre = d + 1, 2 * pre + bit
            out.append(leaf[(d, pre)])
    return bytes(out)
