"""Parity at the full sizes of the benchmark workloads, in the configuration the benchmark
times (default build options), on outputs the oracle can compute one by one.

At the fixed point of Alg. 2 a vertex's register j is the largest rank of Eq. (sketch-add) over
the vertices reachable from it in sample j (the vertex itself included), so the oracle's reach
search from a vertex (its Monte-Carlo reach routine on an empty blocked set) yields the exact
register row of that vertex.  On the 2^24-vertex weighted-cascade graph (R = 256) and the
2^20-vertex IC graph (p = 0.01, R = 256):

* register rows and their estimates (Eq. sketch-estimate, binary32) of sampled vertices;
* the first greedy step of Alg. 1 over all rows: the seed is the row with the largest
  register sum (lowest id on ties) and its score is that sum;
* the Monte-Carlo reach (the reach search the greedy steps run) of sampled seed sets, through
  the influence evaluator on the same samples: the reached pairs equal the oracle's.

(The first seed's own reach on the 2^24 graph, 63 M pairs, takes the oracle about 100 s, so
reach is checked on sampled seeds instead.)  On the 64-job batch workload (R = 128, K = 20),
the autotuned one-launch batch returns, for every job, the seeds and step records of the
single-graph path.
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
        seeds, steps, _ = hf.im_select_seeds(sk, 1)
    finally:
        sk.free()
    evals = [hf.im_evaluate_influence(ctx, xd, ad, g.n, s, J, model=model, p=p) for s in seed_sets]
    del xd, ad
    return g, thr, M, est, list(seeds), steps, sample, seed_sets, evals


def _reach(g, thr, seeds):
    blk = np.zeros((g.n, J), dtype=np.uint8)
    pairs = 0
    for s in seeds:
        pairs += oracle.reach_add(g, thr, J, 0, blk, int(s))
    return blk, pairs


def test_sampled_register_rows_and_estimates(full):
    g, thr, M, est, seeds, steps, sample, seed_sets, evals = full
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


def test_first_greedy_step_is_the_largest_register_sum(full):
    g, thr, M, est, seeds, steps, sample, seed_sets, evals = full
    sums = M.sum(axis=1, dtype=np.int64)
    s0 = int(np.argmax(sums))  # the first (lowest) id of the maximum
    assert seeds[0] == s0
    assert steps[0].score == int(sums[s0])


def test_reach_of_sampled_seed_sets(full):
    g, thr, M, est, seeds, steps, sample, seed_sets, evals = full
    for s, (sigma, reached) in zip(seed_sets, evals):
        _, pairs = _reach(g, thr, s)
        assert reached == pairs, s
        assert sigma == pairs / J


def test_batch_workload_matches_single_graph_path(hf):
    import torch

    Jb, K = 128, 20
    graphs = [(synth.rmat(scale, draws, seed=seed), p) for scale, draws, p, seed in synth.batch_recipe()]
    dev = [(torch.from_numpy(g.xadj).cuda(), torch.from_numpy(g.adj).cuda(), g, p) for g, p in graphs]
    ctx = hf.Context(0)
    b = hf.im_batch_create(ctx, [hf.BatchJob(x, a, g.n, Jb, K, model="const", p=p) for x, a, g, p in dev],
                           autotune=True)
    try:
        b.run()
        res = [b.result(i) for i in range(len(dev))]
    finally:
        b.free()
    for (x, a, g, p), (bseeds, bsteps, cnt) in zip(dev, res):
        sk = hf.im_build_sketches(ctx, x, a, g.n, Jb, model="const", p=p)
        try:
            info = sk.info()
            seeds, steps, stats = hf.im_select_seeds(sk, K)
        finally:
            sk.free()
        assert list(bseeds) == list(seeds)
        assert cnt["build_sweeps"] == info["sweeps"] and cnt["build_visits"] == info["visits"]
        assert cnt["rebuilds"] == stats["rebuilds"]
        for u, v in zip(bsteps, steps):
            assert u == v
