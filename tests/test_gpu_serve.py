"""Serving loop: requests decoded inside a Poisson mix must give exactly the
bytes they give alone (and the input), admission must respect the memory
budget, and batches must overlap (continuous batching, not a queue)."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2606_05765_amd.pivco")


def _requests(n_req=40, hi=2 << 20, seed=7):
    w = W.serve_requests(seed=seed, n_req=n_req, hi=hi)
    streams = [P.pivco_encode(torch.from_numpy(x).cuda(), w.block_size, ans_mode=w.ans_mode)
               for x in w.jobs]
    torch.cuda.synchronize()
    return w, streams


def test_results_same_alone_and_in_mix():
    w, streams = _requests()
    sv = P.Server(mem_budget=1 << 30, slots=4, max_batch=8, keep_outputs=True)
    ids = [sv.register(s) for s in streams]
    n = 3 * len(ids)                                   # every request three times
    order = np.random.default_rng(3).permutation(np.repeat(ids, 3))
    arrivals = W.poisson_arrivals(5, 4000.0, n)
    pool = torch.empty(sum(int(w.jobs[i].size) for i in order) + 256 * n + (1 << 20),
                       dtype=torch.uint8, device="cuda")
    res, stats = sv.run(arrivals, order, pool)
    torch.cuda.synchronize()
    print("stats", stats, flush=True)
    alone = {}
    for i, s in enumerate(streams):
        out, st = P.pivco_decode(s)
        assert st == 0
        alone[i] = out.cpu().numpy()
        assert np.array_equal(alone[i], w.jobs[i])
    for k, r in enumerate(res):
        assert r["status"] == 0, (k, r)
        got = P.view_output(pool, r["d_out"], r["n_out"]).cpu().numpy()
        assert np.array_equal(got, alone[int(order[k])]), k
        assert r["t_done"] >= r["t_admit"] >= r["arrival"] - 1e-6
    assert stats["batches"] < n                         # requests shared batches
    assert stats["max_batch"] > 1
    sv.close()


def test_budget_admission_and_rejection():
    w, streams = _requests(n_req=12, hi=4 << 20, seed=9)
    sizes = [int(x.size) for x in w.jobs]
    budget = sorted(sizes)[-2] + 4096                  # the largest request cannot fit
    sv = P.Server(mem_budget=budget, slots=2, max_batch=4, keep_outputs=False)
    ids = [sv.register(s) for s in streams]
    arrivals = np.linspace(0, 0.01, len(ids))
    pool = torch.empty(budget, dtype=torch.uint8, device="cuda")
    res, stats = sv.run(arrivals, ids, pool)
    torch.cuda.synchronize()
    for k, r in enumerate(res):
        if (sizes[k] + 255) // 256 * 256 > budget:
            assert r["status"] == P.E_BUDGET, (k, r)
        else:
            assert r["status"] == 0, (k, r)
    assert any(r["status"] == P.E_BUDGET for r in res)
    assert stats["peak_pool_bytes"] <= budget
    sv.close()
