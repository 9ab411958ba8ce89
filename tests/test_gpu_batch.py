"""Parity of the batched solver (one persistent launch for many jobs) with the CPU oracle and
with the single-graph path, through the C ABI.

Every job of a batch must reproduce, bit for bit, what the oracle's Alg. 1 computes for it
alone: seeds, every step record (integers exact, FP64 fields exactly equal since both sides
evaluate the same IEEE operations), the build's sweep and visit counts, and the registers of
the build and at the end of the greedy loop.  The work decomposition (lanes per row, tile
sizes, split rows, grid size) and the order of jobs in a batch must not change any result.
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


def _per_edge(g, seed=5):
    rng = np.random.default_rng(seed)
    return rng.random(g.m, dtype=np.float32) * np.float32(0.6)


def _graphs():
    return {
        "er40": synth.erdos_renyi(40, 200, seed=21),
        "er300": synth.erdos_renyi(300, 2400, seed=22),
        "rmat10": synth.rmat(10, 16 << 10, seed=23),
        "rmat11": synth.rmat(11, 24 << 11, seed=24),
        "path": synth.from_edges(50, [(i, i + 1) for i in range(49)] + [(49, 20), (10, 0)]),
        "star": synth.from_edges(600, [(0, v) for v in range(1, 600)] + [(v, 0) for v in range(1, 600, 7)]),
        "isolated": synth.from_edges(70, [(3, 4), (4, 5)]),
    }


GRAPHS = _graphs()

# (graph, model, p, R, K, eps_g, eps_l, eps_c, hash_seed)
MIX = [
    ("er300", "const", 0.1, 64, 10, 0.01, 0.3, 0.0, 0),
    ("rmat10", "wc", 0.0, 128, 12, 0.01, 0.3, 0.0, 0),
    ("rmat11", "const", 0.05, 256, 8, 0.01, 0.3, 0.0, 7),
    ("star", "edge", 0.0, 32, 6, 0.01, 0.3, 0.0, 0),
    ("path", "const", 0.5, 12, 5, 0.0, 0.0, 0.0, 3),
    ("isolated", "const", 0.5, 16, 70, 0.01, 0.3, 0.0, 0),
    ("er40", "wc", 0.0, 4, 7, float("inf"), float("inf"), 0.0, 0),
    ("rmat10", "const", 0.2, 64, 9, 0.01, 0.3, 0.05, 11),
]


def _job(hf, spec):
    gname, model, p, R, K, eg, el, ec, seed = spec
    g = GRAPHS[gname]
    pe = _per_edge(g) if model == "edge" else None
    return hf.BatchJob(g.xadj, g.adj, g.n, R, K, model=model, p=p, per_edge=pe, hash_seed=seed, eps_c=ec,
                       eps_g=eg, eps_l=el)


def _oracle(spec):
    gname, model, p, R, K, eg, el, ec, seed = spec
    g = GRAPHS[gname]
    pe = _per_edge(g) if model == "edge" else None
    thr = oracle.edge_thresholds(g, model, f32(p), per_edge=pe)
    return oracle.greedy(g, thr, R, K, seed=seed, eps_g=eg, eps_l=el, eps_c=ec)


ORACLE = {}


def _ref(spec):
    if spec not in ORACLE:
        ORACLE[spec] = _oracle(spec)
    return ORACLE[spec]


def _compare(res, seeds, steps, K):
    assert list(seeds) == res["seeds"]
    for k in range(K):
        o, s = res["steps"][k], steps[k]
        for f in ("seed", "rebuilt", "fresh", "sweeps", "score", "reach", "visits", "e", "sigma", "delta", "err_l",
                  "err_g"):
            assert getattr(s, f) == o[f], (k, f, getattr(s, f), o[f])


def _check_batch(b, specs):
    for i, spec in enumerate(specs):
        ref = _ref(spec)
        K = spec[4]
        seeds, steps, cnt = b.result(i)
        assert cnt["status"] == 0
        _compare(ref, seeds, steps, K)
        assert cnt["build_sweeps"] == ref["build_sweeps"]
        assert cnt["build_visits"] == ref["build_visits"]
        assert cnt["rebuilds"] == sum(s["rebuilt"] for s in ref["steps"])
        assert np.array_equal(b.registers(i, 1), ref["M"])


@pytest.mark.parametrize("cfg", [
    dict(),
    dict(lanes_per_row=64),
    dict(tile_edges=256, heavy_degree=16, piece_edges=8, workgroups=64),
    dict(tile_edges=64, heavy_degree=4, piece_edges=3, workgroups=7),
    dict(pin_edges=-1),
    dict(pin_edges=1 << 30, tile_edges=128),
    dict(pin_edges=3000, workgroups=40),
])
def test_mixed_batch_matches_oracle(hf, ctx, cfg):
    """Uneven graphs, all three edge models, R from 4 to 256 and K up to n in one launch."""
    b = hf.im_batch_create(ctx, [_job(hf, s) for s in MIX], **cfg)
    try:
        st = b.run()
        assert st["phases"] > 0 and st["tiles"] > 0
        _check_batch(b, MIX)
        # a replay of the captured launch reproduces everything
        b.run()
        _check_batch(b, MIX)
    finally:
        b.free()


def test_build_registers_match_oracle(hf, ctx):
    specs = MIX[:4]
    b = hf.im_batch_create(ctx, [_job(hf, s) for s in specs], heavy_degree=8, piece_edges=5)
    try:
        b.run()
        for i, (gname, model, p, R, K, eg, el, ec, seed) in enumerate(specs):
            g = GRAPHS[gname]
            pe = _per_edge(g) if model == "edge" else None
            thr = oracle.edge_thresholds(g, model, f32(p), per_edge=pe)
            M, sweeps, tl, te = oracle.simulate(g, thr, R, seed=seed, eps_c=ec)
            assert np.array_equal(b.registers(i, 0), M)
            assert b.result(i)[2]["build_sweeps"] == sweeps
    finally:
        b.free()


def test_job_order_does_not_matter(hf, ctx):
    specs = list(reversed(MIX))
    b = hf.im_batch_create(ctx, [_job(hf, s) for s in specs], tile_edges=512)
    try:
        b.run()
        _check_batch(b, specs)
    finally:
        b.free()


def test_autotune_agrees_and_reports(hf, ctx):
    specs = MIX[:3]
    b = hf.im_batch_create(ctx, [_job(hf, s) for s in specs], autotune=True)
    try:
        st = b.run()
        assert st["candidates"] >= 2
        assert st["lanes_per_row"] in (32, 64) and st["workgroups"] > 0
        _check_batch(b, specs)
    finally:
        b.free()


def test_batch_matches_single_graph_path(hf, ctx):
    """Larger R-MAT graphs with hub rows split into pieces: batch == im_build_sketches + im_select_seeds."""
    rng = np.random.default_rng(9)
    graphs = [synth.rmat(s, int(d) << s, seed=100 + s) for s, d in [(13, 20), (12, 8), (14, 12), (12, 32)]]
    models = [("const", 0.05), ("wc", 0.0), ("const", 0.01), ("const", 0.005)]
    jobs, plain = [], []
    for g, (model, p) in zip(graphs, models):
        K = int(rng.integers(5, 15))
        jobs.append(hf.BatchJob(g.xadj, g.adj, g.n, 128, K, model=model, p=p))
        sk = hf.im_build_sketches(ctx, g.xadj, g.adj, g.n, 128, model=model, p=p)
        try:
            info = sk.info()
            seeds, steps, stats = hf.im_select_seeds(sk, K)
            plain.append((info, list(seeds), steps, stats, sk.registers(1)))
        finally:
            sk.free()
    b = hf.im_batch_create(ctx, jobs, heavy_degree=64, piece_edges=48)
    try:
        b.run()
        for i, (info, seeds, steps, stats, M) in enumerate(plain):
            bs, bsteps, cnt = b.result(i)
            assert list(bs) == seeds
            assert cnt["build_sweeps"] == info["sweeps"] and cnt["build_visits"] == info["visits"]
            assert cnt["rebuilds"] == stats["rebuilds"] and cnt["bfs_levels"] == stats["bfs_levels"]
            assert cnt["rebuild_sweeps"] == stats["rebuild_sweeps"]
            assert cnt["rebuild_visits"] == stats["rebuild_visits"]
            for a, c in zip(bsteps, steps):
                assert a == c
            assert np.array_equal(b.registers(i, 1), M)
    finally:
        b.free()


def test_batch_from_device_csr(hf, ctx):
    import torch

    g = GRAPHS["rmat10"]
    job = hf.BatchJob(torch.from_numpy(g.xadj).cuda(), torch.from_numpy(g.adj).cuda(), g.n, 64, 6, model="wc")
    b = hf.im_batch_create(ctx, [job])
    try:
        b.run()
        ref = oracle.greedy(g, oracle.edge_thresholds(g, "wc"), 64, 6)
        seeds, steps, _ = b.result(0)
        _compare(ref, seeds, steps, 6)
    finally:
        b.free()


def test_batch_invalid_inputs(hf, ctx):
    g = GRAPHS["er40"]
    bad = [
        hf.BatchJob(g.xadj, g.adj, g.n, 260, 3),          # R above 256
        hf.BatchJob(g.xadj, g.adj, g.n, 6, 3),            # R not a multiple of 4
        hf.BatchJob(g.xadj, g.adj, g.n, 16, 0),           # K = 0
        hf.BatchJob(g.xadj, g.adj, g.n, 16, g.n + 1),     # K > n
        hf.BatchJob(g.xadj, g.adj, g.n, 16, 3, p=1.5),    # p outside [0, 1]
    ]
    for j in bad:
        with pytest.raises(hf.ImError) as e:
            hf.im_batch_create(ctx, [j])
        assert e.value.status == -1
    adj = g.adj.copy()
    adj[5] = g.n
    with pytest.raises(hf.ImError) as e:
        hf.im_batch_create(ctx, [hf.BatchJob(g.xadj, adj, g.n, 16, 3)])
    assert e.value.status == -2
    pe = _per_edge(g)
    pe[2] = -0.5
    with pytest.raises(hf.ImError) as e:
        hf.im_batch_create(ctx, [hf.BatchJob(g.xadj, g.adj, g.n, 16, 3, model="edge", per_edge=pe)])
    assert e.value.status == -1


def test_batch_budget(hf):
    g = GRAPHS["rmat10"]
    small = hf.Context(0, hbm_budget=1 << 16)
    with pytest.raises(hf.ImError) as e:
        hf.im_batch_create(small, [hf.BatchJob(g.xadj, g.adj, g.n, 64, 4)])
    assert e.value.status == -3
    assert small.bytes_in_use() == 0


def test_uneven_pinned_batch_with_short_watchdog(hf, ctx, monkeypatch):
    """Every job pinned to one XCD, one job far larger than the rest: the XCDs that hold only small
    jobs finish long before the large one.  Their waves leave instead of reading the unchanged claim
    words of finished jobs as a stall, and the waves that keep waiting see the tiles completed on
    other XCDs; with the watchdog period forced down to 20 ms the batch still completes and every
    job equals the single-graph path."""
    monkeypatch.setenv("HFR_BATCH_TIMEOUT_MS", "20")
    big = synth.rmat(15, 16 << 15, seed=61)
    small = [synth.rmat(8, 12 << 8, seed=62 + i) for i in range(15)]
    specs = [(big, "const", 0.05, 12)] + [(g, ("const", "wc")[i % 2], 0.1, 5) for i, g in enumerate(small)]
    jobs, plain = [], []
    for g, model, p, K in specs:
        jobs.append(hf.BatchJob(g.xadj, g.adj, g.n, 128, K, model=model, p=p))
        sk = hf.im_build_sketches(ctx, g.xadj, g.adj, g.n, 128, model=model, p=p)
        try:
            seeds, steps, _ = hf.im_select_seeds(sk, K)
            plain.append((list(seeds), steps))
        finally:
            sk.free()
    b = hf.im_batch_create(ctx, jobs, pin_edges=1 << 30)
    try:
        for _ in range(2):
            b.run()
            for i, (seeds, steps) in enumerate(plain):
                bs, bsteps, _ = b.result(i)
                assert list(bs) == seeds, i
                for a, c in zip(bsteps, steps):
                    assert a == c
    finally:
        b.free()
