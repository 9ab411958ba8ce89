"""The allocation-free selection (im_select_seeds_noalloc) against im_select_seeds, through the C ABI.

Two calls in a row on the shared per-device scratch, the second with a smaller input (a smaller
graph and a smaller K): seeds, step records and the registers in force at the end must equal those
of the allocating entry point exactly; K beyond the scratch's limit is refused before any device work.
"""
from __future__ import annotations

import numpy as np
import pytest

import synth

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(300)]


@pytest.fixture(scope="module")
def hf():
    import torch

    assert torch.cuda.is_available(), "the GPU tests need a visible MI355X"
    import paper_2105_04023_amd as hf

    hf._binding.load()
    return hf


def _both(hf, ctx, g, J, K, model, p):
    sk = hf.im_build_sketches(ctx, g.xadj, g.adj, g.n, J, model=model, p=p)
    try:
        a = hf.im_select_seeds(sk, K)
        Ma = sk.registers(1)
        b = hf.im_select_seeds(sk, K, noalloc=True)
        Mb = sk.registers(1)
        c = hf.im_select_seeds(sk, K)
    finally:
        sk.free()
    return a, Ma, b, Mb, c


def test_noalloc_equals_allocating_two_calls(hf):
    ctx = hf.Context(0)
    try:
        cases = [(synth.rmat(12, 16 << 12, seed=41), 128, 24, "const", 0.05),
                 (synth.erdos_renyi(600, 4000, seed=42), 64, 7, "wc", 0.0)]
        for g, J, K, model, p in cases:
            print(f"[noalloc] n={g.n} m={g.m} J={J} K={K} model={model}", flush=True)
            a, Ma, b, Mb, c = _both(hf, ctx, g, J, K, model, p)
            assert list(a[0]) == list(b[0]) == list(c[0])
            assert a[1] == b[1] == c[1]
            assert a[2]["rebuilds"] == b[2]["rebuilds"]
            assert np.array_equal(Ma, Mb)
        g = synth.erdos_renyi(300, 2000, seed=43)
        sk = hf.im_build_sketches(ctx, g.xadj, g.adj, g.n, 16)
        try:
            with pytest.raises(hf.ImError) as ei:
                hf.im_select_seeds(sk, hf._binding.IM_NOALLOC_MAX_K + 1, noalloc=True)
            assert "IM_ERR_INVALID_ARG" in str(ei.value)
            seeds, _, _ = hf.im_select_seeds(sk, 5, noalloc=True)  # the sketch is still usable
            assert len(seeds) == 5
        finally:
            sk.free()
    finally:
        ctx.close()
