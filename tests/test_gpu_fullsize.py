"""Cross-checks at the full sizes of the benchmark workloads that do not go through the oracle's
Simulate: at the fixed point of Alg. 2 a vertex's register j is the largest rank of Eq. (sketch-add)
over the vertices reachable from it in sample j (the vertex itself included), so the oracle's reach
search from a vertex (its Monte-Carlo reach routine on an empty blocked set) yields the exact register
row of that vertex.  On the 2^24-vertex weighted-cascade graph (R = 256) and the 2^20-vertex IC graph
(p = 0.01, R = 256), in the benchmark's configuration:

* register rows and their estimates (Eq. sketch-estimate, binary32) of sampled vertices whose reach
  the oracle enumerates in seconds;
* the Monte-Carlo reach (the reach search the greedy steps run) of sampled seed sets, through the
  influence evaluator on the same samples: the reached pairs equal the oracle's.

The whole runs (all registers, traces, seeds and step records) are compared with the oracle's
recorded outputs in test_gpu_golden.py.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

J = 256
MAX_PAIRS = 1 << 20  # sampled vertices whose oracle reach is larger are not checked row by row


@pytest.fixture(scope="module")
def hf():
    import torch

    assert torch.cuda.is_available(), "the GPU tests need a visible MI355X"
    import paper_2105_04023_amd as hf

    hf._binding.load()
    return hf


WORKLOADS = {"rmat24_wc": synth.workload_rmat24_wc, "rmat20_p0.01": synth.workload_rmat20}


@pytest.fixture(scope="module", params=sorted(WORKLOADS))
def full(hf, request):
    import torch

    w = WORKLOADS[request.param]()
    g, model, p = w.graph, w.model, w.p
    thr = oracle.edge_thresholds(g, model, np.float32(p))
    deg = np.diff(g.xadj)
    rng = np.random.default_rng(24)
    sample = [int(u) for u in rng.choice(np.nonzero(deg > 0)[0], 8, replace=False)]
    seed_sets = [sample[:1], sample[1:3], sample[3:6]]
    ctx = hf.Context(0)
    xd, ad = torch.from_numpy(g.xadj).cuda(), torch.from_numpy(g.adj).cuda()
    sk = hf.im_build_sketches(ctx, xd, ad, g.n, J, model=model, p=p)
    try:
        M = sk.registers(0)
        est = {u: hf.im_estimate(sk, [u]) for u in sample}
    finally:
        sk.free()
    evals = [hf.im_evaluate_influence(ctx, xd, ad, g.n, s, J, model=model, p=p) for s in seed_sets]
    del xd, ad
    return g, thr, M, est, sample, seed_sets, evals


def _reach(g, thr, seeds):
    blk = np.zeros((g.n, J), dtype=np.uint8)
    pairs = 0
    for s in seeds:
        pairs += oracle.reach_add(g, thr, J, 0, blk, int(s))
    return blk, pairs


def test_sampled_register_rows_and_estimates(full):
    g, thr, M, est, sample, seed_sets, evals = full
    checked = 0
    for u in sample:
        blk, pairs = _reach(g, thr, [u])
        if pairs > MAX_PAIRS:
            continue
        row = np.zeros(J, dtype=np.uint8)
        for v in np.nonzero(blk.view(np.uint64).any(axis=1))[0]:
            ranks = np.array([oracle.rank(int(v), j) for j in range(J)], dtype=np.uint8)
            row = np.maximum(row, np.where(blk[v] != 0, ranks, 0).astype(np.uint8))
        assert np.array_equal(M[u], row), u
        assert est[u] == np.float32(oracle.estimate(row)), u
        checked += 1
    assert checked >= 4


def test_reach_of_sampled_seed_sets(full):
    g, thr, M, est, sample, seed_sets, evals = full
    for s, (sigma, reached) in zip(seed_sets, evals):
        _, pairs = _reach(g, thr, s)
        assert reached == pairs, s
        assert sigma == pairs / J
