"""Seeded decode/encode parity cases shared by the GPU tests (data only)."""
import numpy as np

import workloads as W


def _rng(seed):
    return np.random.default_rng(seed)


def cases():
    """(name, data, block_size, ans_mode, tree_len or None) tuples.  Sizes keep
    the oracle at a few seconds while spanning several decode tiles, ragged
    tails, the resident and the streaming paths, and both rANS modes."""
    out = []
    g = W.geo1m(seed=1, scale=8).jobs[0]
    out.append(("geo_1block_ragged", g[:len(g) - 37], 1 << 20, 0, None))
    z = W.zipf256m(seed=1, scale=1024).jobs[0]                 # 256 KiB
    out.append(("zipf_64k_ragged", np.concatenate([z, z[:13]]), 64 << 10, 0, None))
    s = W.skew256m(seed=1, scale=512).jobs[0]                  # 512 KiB
    out.append(("skew_128k_ans", s, 128 << 10, 1, None))
    out.append(("zipf_forced_ans", z[:200_000], 64 << 10, 2, None))
    r = _rng(5)
    u = r.integers(0, 256, size=(256 << 10) + 5).astype(np.uint8)
    out.append(("uniform256_64k", u, 64 << 10, 0, None))       # 8-bit codes: streaming path
    big = W.draw(r, W.geometric_p(0.97), 3 << 20)
    out.append(("geo97_3m_block", big, 3 << 20, 1, None))       # one big block, many tiles
    # split-block limits: 128 tiles of 32Ki (the most a block is split
    # into), one symbol more (decoded whole), and just above the split size
    g4 = W.draw(r, W.geometric_p(0.9), (4 << 20) + 1)
    out.append(("geo_4m_128_tiles", g4[:4 << 20], 4 << 20, 0, None))
    out.append(("geo_4m_plus1_whole", g4, (4 << 20) + 1, 1, None))
    out.append(("zipf_split_min_plus1", np.concatenate([z, z])[:(64 << 10) + 1], (64 << 10) + 1, 0, None))
    for n in [1, 2, 3, 31, 32, 33, 255, 256, 257, 4095, 4096, 4097, 70000]:
        k = int(r.integers(2, 40))
        out.append((f"tiny_{n}", r.integers(0, k, size=n).astype(np.uint8), 1 << 16, 0, None))
    out.append(("tiny_forced_1000", r.integers(0, 5, size=1000).astype(np.uint8), 333, 2, None))
    out.append(("constant", np.full(100_000, 7, np.uint8), 40_000, 0, None))
    out.append(("constant_split", np.full(200_000, 9, np.uint8), 1 << 17, 0, None))
    out.append(("two_symbols", (r.random(150_000) < 0.03).astype(np.uint8), 1 << 16, 1, None))
    # the first 32Ki-output tile holds only the most frequent symbol (a
    # 1-bit code): every level below the root has no work in it, whole and split
    tail = W.draw(r, W.geometric_p(0.97), 60_000)
    front = np.concatenate([np.zeros(40_000, np.uint8), tail])
    out.append(("front_loaded_whole", front[:1 << 16], 1 << 16, 0, None))
    out.append(("front_loaded_split", front, front.size, 0, None))
    # deepest codes: Fibonacci-like counts reach the 11-bit limit
    fib = [1, 1]
    while len(fib) < 24:
        fib.append(fib[-1] + fib[-2])
    p = np.zeros(256)
    p[:24] = fib[::-1]
    out.append(("deep_11", W.draw(r, p, 300_000), 1 << 17, 0, None))
    # a caller-supplied tree (the paper's "huffman" shape) on a 3-symbol source
    lens = np.zeros(256, np.uint8)
    for ch, l in {"f": 2, "u": 2, "a": 3, "h": 3, "m": 3, "n": 3}.items():
        lens[ord(ch)] = l
    src = np.frombuffer(b"huffman", np.uint8)
    out.append(("supplied_tree", np.tile(src, 5000), 4096, 0, lens))
    return out


def mix_jobs(seed=3, n_blocks=24, hi=1 << 20):
    """Independent single-block streams with the mixed family workload."""
    w = W.mix4096(seed=seed, n_blocks=n_blocks, hi=hi)
    return [(f"mix_{i}_{lab}", d, max(d.size, 1), 1, None) for i, (d, lab) in
            enumerate(zip(w.jobs, w.labels))]
