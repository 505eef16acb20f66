"""Seeded sweep wider than test_gpu_random: per seed 150 inputs (sizes
log-uniform in 1 B .. 3 MB, block sizes 4 Ki .. 4 Mi symbols, so whole,
streamed and split blocks, the mixed families, skewed, few-symbol and
uniform-256 sources), every encoder mode (raw, rANS by the rule, forced
rANS, selective tANS), canonical and flat-subtree trees, code length limits
9..11 and rANS chunks of 2^12 or 2^16 bits.  The HIP encoder's stream must
equal the oracle's byte for byte, and every merge variant must decode all
the oracle's streams of a seed, in one batched launch, back to the input.
Bit-exact throughout (integer work)."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2606_05765_amd.pivco")


def _cases(seed, count=150):
    r = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = W.log_uniform_size(r, 1, 3_000_000)
        kind = int(r.integers(0, 6))
        if kind < 3:
            lab, p = W.family_p(r)
        elif kind == 3:
            lab, p = "skew", W.skew_p()
        elif kind == 4:
            k = int(r.integers(2, 6))
            lab, p = f"few{k}", np.concatenate([np.ones(k), np.zeros(256 - k)])
        else:
            lab, p = "uni256", np.ones(256)
        data = W.draw(r, p, n)
        bs = int(2 ** r.integers(12, 23))
        mode = int(r.integers(0, 4))
        flat = bool(r.integers(0, 2))
        max_len = int(r.integers(9, 12))
        clog = int(r.choice([12, 16])) if mode != 3 else 16
        out.append((f"s{seed}_{i}_{lab}_n{n}_bs{bs}_m{mode}_f{int(flat)}_L{max_len}_c{clog}",
                    data, bs, mode, flat, max_len, clog))
    return out


@pytest.mark.parametrize("seed", [7, 11])
def test_sweep_encode_and_every_variant(seed):
    cases = _cases(seed)
    print("seed", seed, "cases", len(cases), flush=True)
    streams = []
    for name, data, bs, mode, flat, L, c in cases:
        want = O.encode(data, bs, max_len=L, ans_mode=mode, chunk_log2=c, flat=flat)
        got = P.pivco_encode(torch.from_numpy(data).cuda(), bs, max_len=L, ans_mode=mode,
                             chunk_log2=c, flat=flat)
        torch.cuda.synchronize()
        g = got.cpu().numpy()
        assert g.size == want.size and np.array_equal(g, want), f"{name}: encoder bytes differ"
        streams.append(torch.from_numpy(want).cuda())
    outs = [torch.empty(max(c[1].size, 1), dtype=torch.uint8, device="cuda")[:c[1].size] for c in cases]
    for v in range(len(P.pivco_merge_variants())):
        print("variant", v, flush=True)
        t = P.Tune()
        t.merge_variant = v
        t.merge_grid = 256
        t.rans_grid = 256
        for o in outs:
            o.fill_(0xAB)
        plan = P.BatchPlan(streams, outs, tune=t)
        plan.launch()
        torch.cuda.synchronize()
        st = plan.statuses()
        for c, o, s in zip(cases, outs, st):
            assert s == 0, f"variant {v} {c[0]}: status {int(s)}"
            assert np.array_equal(o.cpu().numpy(), c[1]), f"variant {v} {c[0]}: decoded bytes differ"
        plan.close()
