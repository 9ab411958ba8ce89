"""The independent Monte-Carlo evaluator (im_evaluate_influence) against the oracle's reach.

The oracle blocks the reach of every seed, one seed after the other, in R samples drawn with the
evaluation's hash seed; the number of blocked (vertex, sample) pairs is the size of the union of
the seeds' reach sets, which the device's single multi-source search must reproduce exactly.
With the selection's own hash seed the evaluation equals the greedy loop's final sigma.
"""
from __future__ import annotations

import struct

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def f32(x):
    return struct.unpack("<f", struct.pack("<f", x))[0]


@pytest.fixture(scope="module")
def hf():
    import torch

    assert torch.cuda.is_available(), "the GPU tests need a visible MI355X"
    import paper_2105_04023_amd as hf

    hf._binding.load()
    return hf


@pytest.fixture(scope="module")
def ctx(hf):
    return hf.Context(0)


GRAPHS = {
    "er300": synth.erdos_renyi(300, 2400, seed=41),
    "rmat11": synth.rmat(11, 16 << 11, seed=42),
    "star": synth.from_edges(600, [(0, v) for v in range(1, 600)] + [(v, 0) for v in range(1, 600, 7)]),
}


def _oracle_reach(g, thr, R, seed, seeds):
    blk = np.zeros((g.n, R), dtype=np.uint8)
    return sum(oracle.reach_add(g, thr, R, seed, blk, int(s)) for s in seeds)


@pytest.mark.parametrize("gname,model,p,R,seed", [
    ("er300", "const", 0.1, 64, 1234),
    ("rmat11", "wc", 0.0, 256, 99),
    ("rmat11", "const", 0.05, 128, 7),
    ("star", "const", 0.3, 32, 5),
    ("rmat11", "const", 0.02, 12, 3),
])
def test_evaluate_matches_oracle(hf, ctx, gname, model, p, R, seed):
    g = GRAPHS[gname]
    thr = oracle.edge_thresholds(g, model, f32(p))
    rng = np.random.default_rng(R)
    for size in [1, 3, 17]:
        seeds = rng.choice(g.n, size, replace=False)
        seeds = np.concatenate([seeds, seeds[:1]])  # a repeated seed adds nothing
        ref = _oracle_reach(g, thr, R, seed, seeds)
        sigma, reach = hf.im_evaluate_influence(ctx, g.xadj, g.adj, g.n, seeds, R, model=model, p=p, hash_seed=seed)
        assert reach == ref
        assert sigma == ref / R


def test_evaluate_with_selection_seed_equals_greedy_sigma(hf, ctx):
    g = GRAPHS["rmat11"]
    sk = hf.im_build_sketches(ctx, g.xadj, g.adj, g.n, 64, model="const", p=0.05)
    try:
        seeds, steps, _ = hf.im_select_seeds(sk, 10)
    finally:
        sk.free()
    sigma, reach = hf.im_evaluate_influence(ctx, g.xadj, g.adj, g.n, seeds, 64, model="const", p=0.05)
    assert reach == steps[-1].reach and sigma == steps[-1].sigma


def test_evaluate_rejects_bad_seeds(hf, ctx):
    g = GRAPHS["er300"]
    with pytest.raises(hf.ImError):
        hf.im_evaluate_influence(ctx, g.xadj, g.adj, g.n, [g.n], 64, p=0.1)
    with pytest.raises(hf.ImError):
        hf.im_evaluate_influence(ctx, g.xadj, g.adj, g.n, [], 64, p=0.1)
