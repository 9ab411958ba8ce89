"""Reach-search level ids of the greedy loop restart with cleared vertex stamps when they would run
past their limit (forced small here through HFR_LEVEL_ID_LIMIT, which the library reads at every
selection call), and the seeds and step records still equal the oracle's (Alg. 1).  Every selection
call also starts its level ids afresh, so a sketch that serves many requests never runs them out."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(300)]


@pytest.fixture(scope="module")
def hf():
    import torch

    assert torch.cuda.is_available(), "the GPU tests need a visible MI355X"
    import paper_2105_04023_amd as hf

    hf._binding.load()
    return hf


@pytest.mark.parametrize("limit", ["3", None])
def test_level_ids_restart_when_forced(hf, monkeypatch, limit):
    if limit is None:
        monkeypatch.delenv("HFR_LEVEL_ID_LIMIT", raising=False)
    else:
        monkeypatch.setenv("HFR_LEVEL_ID_LIMIT", limit)
    g = synth.rmat(11, 16 << 11, seed=44)
    J, K = 64, 12
    thr = oracle.edge_thresholds(g, "const", np.float32(0.1))
    ref = oracle.greedy(g, thr, J, K)
    ctx = hf.Context(0)
    sk = hf.im_build_sketches(ctx, g.xadj, g.adj, g.n, J, model="const", p=0.1)
    try:
        for _ in range(3):  # repeated calls on one resident sketch
            seeds, steps, stats = hf.im_select_seeds(sk, K)
            assert list(seeds) == ref["seeds"]
            for s, r in zip(steps, ref["steps"]):
                assert (s.reach, s.e, s.rebuilt, s.sweeps, s.visits) == (
                    r["reach"], r["e"], r["rebuilt"], r["sweeps"], r["visits"])
        assert stats["bfs_levels"] > K  # several levels per step, so a limit of 3 restarts every step
    finally:
        sk.free()
        ctx.close()
