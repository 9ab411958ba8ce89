"""CSR offsets of 32 bits at the C ABI (im_csr.offset_bits = 32): the library widens them to its
own int64 copy, so every result equals the one from int64 offsets and the oracle's (Sec. 3.3 CSR).
Host arrays and device tensors, the single-graph path, the batched solver, the serving pool and the
influence evaluator; an unsupported offset_bits is refused."""
from __future__ import annotations

import ctypes
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


G = synth.rmat(11, 16 << 11, seed=71)
J, K = 128, 8


@pytest.fixture(scope="module")
def ref():
    thr = oracle.edge_thresholds(G, "wc", 0.0)
    return oracle.greedy(G, thr, J, K), thr


@pytest.mark.parametrize("where", ["host", "device"])
def test_single_graph_int32_offsets(hf, ref, where):
    import torch

    res, _ = ref
    x32 = G.xadj.astype(np.int32)
    xadj, adj = (x32, G.adj) if where == "host" else (torch.from_numpy(x32).cuda(), torch.from_numpy(G.adj).cuda())
    ctx = hf.Context(0)
    sk = hf.im_build_sketches(ctx, xadj, adj, G.n, J, model="wc")
    try:
        assert sk.info()["sweeps"] == oracle.simulate(G, ref[1], J)[1]
        seeds, steps, _ = hf.im_select_seeds(sk, K)
        assert list(map(int, seeds)) == res["seeds"]
        assert np.array_equal(sk.registers(1), res["M"])
    finally:
        sk.free()
        ctx.close()


def test_batch_server_evaluator_int32_offsets(hf, ref):
    res, thr = ref
    x32 = G.xadj.astype(np.int32)
    ctx = hf.Context(0)
    b = hf.im_batch_create(ctx, [hf.BatchJob(x32, G.adj, G.n, J, K, model="wc")])
    try:
        b.run()
        assert list(map(int, b.result(0)[0])) == res["seeds"]
    finally:
        b.free()
    sv = hf.Server(0, slots=2)
    try:
        gid = sv.add_graph(x32, G.adj, G.n)
        seeds, _ = sv.wait(sv.submit(gid, J, K, model="wc"))
        assert list(map(int, seeds)) == res["seeds"]
    finally:
        sv.close()
    sigma, reached = hf.im_evaluate_influence(ctx, x32, G.adj, G.n, res["seeds"][:3], J, model="wc")
    blk = np.zeros((G.n, J), dtype=np.uint8)
    pairs = sum(oracle.reach_add(G, thr, J, 0, blk, s) for s in res["seeds"][:3])
    assert reached == pairs
    ctx.close()


def test_unsupported_offset_bits_refused(hf):
    B = hf._binding
    lib = B.load()
    ctx = hf.Context(0)
    x = np.ascontiguousarray(G.xadj)
    a = np.ascontiguousarray(G.adj)
    probs = B.im_probs(B.IM_PROB_CONSTANT, ctypes.c_float(0.1), None)
    for bits, status in [(16, B.IM_ERR_INVALID_ARG), (8, B.IM_ERR_INVALID_ARG)]:
        g = B.im_csr(G.n, G.m, x.ctypes.data, a.ctypes.data, 0, bits)
        out = ctypes.c_void_p()
        st = lib.im_build_sketches(ctx.handle, ctypes.byref(g), ctypes.byref(probs), 64, 0, None, ctypes.byref(out))
        assert st == status and not out.value
        assert b"offset_bits" in lib.im_last_error()
    ctx.close()
