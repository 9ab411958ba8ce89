"""The serving engine (im_server_*): requests that overlap on the device give, each one, the result
the same request gives alone; resident sketches are reused; the HBM budget admits and evicts.

"Alone" is the single-graph path on a fresh sketch (im_build_sketches + im_select_seeds, checked
against the CPU oracle for the small graphs), so every served result is pinned to the oracle.
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


GRAPHS = [synth.erdos_renyi(300, 2400, seed=31), synth.rmat(10, 16 << 10, seed=32), synth.rmat(13, 16 << 13, seed=33),
          synth.rmat(12, 12 << 12, seed=34)]

# (graph, model, p, R, K, hash_seed)
REQS = [(0, "const", 0.1, 64, 10, 0), (1, "wc", 0.0, 256, 12, 0), (2, "const", 0.01, 64, 20, 3),
        (3, "const", 0.1, 256, 15, 0), (1, "const", 0.05, 128, 8, 1), (2, "wc", 0.0, 128, 25, 0),
        (0, "wc", 0.0, 32, 30, 2), (3, "const", 0.01, 64, 9, 5)]


def _alone(hf, ctx, req):
    gi, model, p, R, K, seed = req
    g = GRAPHS[gi]
    sk = hf.im_build_sketches(ctx, g.xadj, g.adj, g.n, R, model=model, p=p, hash_seed=seed)
    try:
        seeds, _, _ = hf.im_select_seeds(sk, K)
    finally:
        sk.free()
    return list(map(int, seeds))


@pytest.fixture(scope="module")
def alone(hf):
    ctx = hf.Context(0)
    return {r: _alone(hf, ctx, r) for r in REQS}


def test_alone_results_match_oracle(alone):
    for req in REQS[:2]:
        gi, model, p, R, K, seed = req
        g = GRAPHS[gi]
        ref = oracle.greedy(g, oracle.edge_thresholds(g, model, f32(p)), R, K, seed=seed)
        assert alone[req] == ref["seeds"]


def _server(hf, slots=3, budget=0, max_copies=0):
    sv = hf.Server(0, slots=slots, hbm_budget=budget, max_copies=max_copies)
    for g in GRAPHS:
        sv.add_graph(g.xadj, g.adj, g.n)
    return sv


def test_mix_equals_alone(hf, alone):
    """All requests submitted at once over 3 slots, one copy per sketch: they overlap, each equals its
    result alone, and the second round reuses every sketch of the first (on whichever slot runs it)."""
    sv = _server(hf, max_copies=1)
    try:
        tickets = [(r, sv.submit(r[0], r[3], r[4], model=r[1], p=r[2], hash_seed=r[5])) for r in REQS * 2]
        slots = set()
        for req, t in tickets:
            seeds, resp = sv.wait(t)
            assert resp["status"] == 0
            assert list(map(int, seeds)) == alone[req], req
            slots.add(resp["slot"])
            assert resp["latency_ms"] >= resp["select_ms"]
        assert len(slots) > 1
        st = sv.stats()
        assert st["completed"] == 2 * len(REQS) and st["failed"] == 0
        # the second round reused every sketch of the first
        assert st["sketches_built"] == len(REQS)
    finally:
        sv.close()


def test_sketch_reuse_and_prefixes(hf, alone):
    sv = _server(hf, slots=2)
    try:
        gi, model, p, R, K, seed = REQS[2]
        s1, r1 = sv.wait(sv.submit(gi, R, K, model=model, p=p, hash_seed=seed))
        s2, r2 = sv.wait(sv.submit(gi, R, 5, model=model, p=p, hash_seed=seed))
        s3, r3 = sv.wait(sv.submit(gi, R, K, model=model, p=p, hash_seed=seed))
        assert r1["sketch_reused"] == 0 and r2["sketch_reused"] == 1 and r3["sketch_reused"] == 1
        assert r2["build_ms"] == 0.0
        assert list(s1) == alone[REQS[2]] and list(s3) == list(s1)
        assert list(s2) == list(s1[:5])
    finally:
        sv.close()


def test_growing_and_repeated_K_on_one_sketch(hf):
    """One slot, one copy: requests of one key with K growing, shrinking and repeated are answered
    from, or continue, the greedy run the sketch holds; each equals the same K run alone."""
    gi, model, p, R, _, seed = REQS[2]
    g = GRAPHS[gi]
    ks = [5, 20, 12, 35, 35, 3, 40]
    ctx = hf.Context(0)
    sk = hf.im_build_sketches(ctx, g.xadj, g.adj, g.n, R, model=model, p=p, hash_seed=seed)
    try:
        ref = {K: (list(map(int, r[0])), r[2]["rebuilds"]) for K in set(ks)
               for r in [hf.im_select_seeds(sk, K)]}
    finally:
        sk.free()
    sv = _server(hf, slots=1, max_copies=1)
    try:
        for K in ks:
            seeds, resp = sv.wait(sv.submit(gi, R, K, model=model, p=p, hash_seed=seed))
            assert (list(map(int, seeds)), resp["rebuilds"]) == ref[K], K
        assert sv.stats()["sketches_built"] == 1
    finally:
        sv.close()


def test_budget_evicts_and_rejects(hf, alone):
    ctx = hf.Context(0)
    g = GRAPHS[2]
    one = ctx.bytes_needed(g.n, g.m, 256)
    graphs = sum(8 * (x.n + 1) + 4 * x.m for x in GRAPHS)
    # one slot that holds a single large sketch: alternating keys evict each other
    sv = _server(hf, slots=1, budget=graphs + int(one * 1.5))
    try:
        order = [REQS[3], REQS[2], REQS[3], REQS[5], REQS[2]]
        for req in order:
            seeds, resp = sv.wait(sv.submit(req[0], req[3], req[4], model=req[1], p=req[2], hash_seed=req[5]))
            assert list(map(int, seeds)) == alone[req]
        assert sv.stats()["evictions"] >= 2
    finally:
        sv.close()
    # a budget below one sketch rejects the request and keeps serving
    small = ctx.bytes_needed(GRAPHS[0].n, GRAPHS[0].m, 4)
    assert small < one
    sv = _server(hf, slots=1, budget=graphs + (small + one) // 2)
    try:
        t = sv.submit(2, 256, 5, model="const", p=0.1)
        with pytest.raises(hf.ImError) as e:
            sv.wait(t)
        assert e.value.status == -3
        t = sv.submit(0, 4, 3, model="const", p=0.1)
        seeds, resp = sv.wait(t)
        assert resp["status"] == 0
    finally:
        sv.close()


def test_invalid_requests(hf):
    sv = _server(hf, slots=1)
    try:
        with pytest.raises(hf.ImError):
            sv.submit(7, 64, 3)          # unknown graph
        with pytest.raises(hf.ImError):
            sv.submit(0, 66, 3)          # R not a multiple of 4
        with pytest.raises(hf.ImError):
            sv.submit(0, 64, 0)          # K = 0
        with pytest.raises(hf.ImError):
            sv.submit(0, 64, 3, p=2.0)   # p outside [0, 1]
        with pytest.raises(ValueError):
            sv.submit(0, 64, 3, model="edge")
    finally:
        sv.close()


def test_second_copies_under_contention(hf, alone):
    """Many requests of two keys at once over 4 slots with up to 2 copies per key: more than one copy
    of a key may be built, never more than 2, and every result equals the request alone."""
    sv = _server(hf, slots=4, max_copies=2)
    try:
        reqs = [REQS[1], REQS[3]] * 6
        tickets = [(r, sv.submit(r[0], r[3], r[4], model=r[1], p=r[2], hash_seed=r[5])) for r in reqs]
        for req, t in tickets:
            seeds, _ = sv.wait(t)
            assert list(map(int, seeds)) == alone[req]
        st = sv.stats()
        assert 2 <= st["sketches_built"] <= 4 and st["resident_sketches"] == st["sketches_built"]
    finally:
        sv.close()


def test_cancel_queued_requests(hf, alone):
    """One slot: requests queue behind the first; cancelled ones report IM_ERR_STATE and never run,
    and the results of the others are unchanged."""
    sv = _server(hf, slots=1)
    try:
        order = [REQS[5], REQS[0], REQS[2], REQS[4], REQS[7], REQS[1]]
        tickets = [(r, sv.submit(r[0], r[3], r[4], model=r[1], p=r[2], hash_seed=r[5])) for r in order]
        cancelled = {tickets[2][1], tickets[4][1]}
        assert all(sv.cancel(t) for t in cancelled)
        for req, t in tickets:
            if t in cancelled:
                with pytest.raises(hf.ImError) as e:
                    sv.wait(t)
                assert e.value.status == -5
            else:
                seeds, resp = sv.wait(t)
                assert list(map(int, seeds)) == alone[req]
                assert not sv.cancel(t)  # finished
        assert sv.stats()["completed"] == len(order)
    finally:
        sv.close()


def test_oversized_request_evicts_nothing(hf, alone):
    """A request whose sketch cannot fit the budget even alone fails at once and leaves the resident
    sketches in place; a failed request does not change the results of the others."""
    ctx = hf.Context(0)
    graphs = sum(8 * (x.n + 1) + 4 * x.m for x in GRAPHS)
    small = ctx.bytes_needed(GRAPHS[0].n, GRAPHS[0].m, 64)
    big = ctx.bytes_needed(GRAPHS[2].n, GRAPHS[2].m, 1024)
    assert big > 2 * small
    sv = _server(hf, slots=2, budget=graphs + 2 * small)
    try:
        req = REQS[0]
        s1, _ = sv.wait(sv.submit(req[0], req[3], req[4], model=req[1], p=req[2], hash_seed=req[5]))
        assert sv.stats()["resident_sketches"] == 1
        with pytest.raises(hf.ImError) as e:
            sv.wait(sv.submit(2, 1024, 5, model="const", p=0.1))
        assert e.value.status == -3
        st = sv.stats()
        assert st["resident_sketches"] == 1 and st["evictions"] == 0
        s2, r2 = sv.wait(sv.submit(req[0], req[3], req[4], model=req[1], p=req[2], hash_seed=req[5]))
        assert r2["sketch_reused"] == 1 and list(map(int, s1)) == list(map(int, s2)) == alone[req]
    finally:
        sv.close()
