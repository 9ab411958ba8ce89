"""MI355X (gfx950) library for sketch-based influence maximisation (arXiv 2105.04023).

Python names mirror the C ABI of include/im.h: ``im_build_sketches``, ``im_estimate``,
``im_estimate_all`` and ``im_select_seeds``.  This module only marshals arguments; the
sampling, register propagation, estimates, reach and greedy decisions all run in the HIP
library.  PyTorch provides the device, the stream and (by default) the device allocator.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _binding as B

__all__ = ["Context", "Sketch", "Batch", "BatchJob", "Server", "im_build_sketches", "im_estimate", "im_estimate_all",
           "im_select_seeds", "im_batch_create", "im_evaluate_influence", "ImError"]

ImError = B.ImError
_KIND = {"const": B.IM_PROB_CONSTANT, "wc": B.IM_PROB_WEIGHTED_CASCADE, "edge": B.IM_PROB_PER_EDGE}


def _torch():
    import torch

    return torch


class Context:
    """A device, a HIP stream and an optional device-memory budget (bytes, 0 = none)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, stream=None, torch_allocator: bool = True):
        torch = _torch()
        self.lib = B.load()
        torch.cuda.set_device(device)
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._keep = []
        if torch_allocator:
            dev, st = device, self.stream

            def _alloc(nbytes, _user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, st)
                except Exception:  # out of memory: the library reports IM_ERR_OUT_OF_BUDGET
                    return None

            def _free(ptr, _user):
                torch.cuda.caching_allocator_delete(ptr)

            af, ff = B.ALLOC_FN(_alloc), B.FREE_FN(_free)
        else:
            af, ff = B.ALLOC_FN(), B.FREE_FN()
        self._keep += [af, ff]
        h = ctypes.c_void_p()
        B.check(self.lib.im_ctx_create(device, ctypes.c_void_p(self.stream.cuda_stream), hbm_budget, af, ff, None,
                                       ctypes.byref(h)))
        self.handle = h

    def bytes_in_use(self) -> int:
        return int(self.lib.im_ctx_bytes_in_use(self.handle))

    def bytes_needed(self, n: int, m: int, R: int, model: str = "const") -> int:
        return int(self.lib.im_sketch_bytes_needed(n, m, R, _KIND[model]))

    def close(self):
        if self.handle:
            self.lib.im_ctx_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Step:
    seed: int
    rebuilt: int
    fresh: int
    sweeps: int
    score: int
    reach: int
    e: float
    sigma: float
    delta: float
    err_l: float
    err_g: float
    visits: int


class Sketch:
    """Handle of a built sketch (graph copy + registers) on the device."""

    def __init__(self, ctx: Context, handle, n: int, R: int):
        self.ctx, self.handle, self.n, self.R = ctx, handle, n, R
        self.lib = ctx.lib

    def info(self) -> dict:
        i = B.im_sketch_info()
        B.check(self.lib.im_sketch_get_info(self.handle, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in B.im_sketch_info._fields_}

    def trace(self):
        """(|L_t| for t = 0..sweeps, edges with a live head per sweep)."""
        cap = self.info()["sweeps"] + 1
        live = np.zeros(cap, dtype=np.int64)
        vis = np.zeros(cap, dtype=np.int64)
        w = ctypes.c_int32()
        B.check(self.lib.im_sketch_get_trace(self.handle, live.ctypes.data, vis.ctypes.data, cap, ctypes.byref(w)))
        return live[: w.value], vis[: w.value - 1]

    def sweep_log(self, clear: bool = False) -> list:
        """One record per launched sweep (needs time_sweeps at build)."""
        cap = 1 << 16
        buf = (B.im_sweep_rec * cap)()
        k = self.lib.im_sketch_get_sweep_log(self.handle, ctypes.cast(buf, ctypes.c_void_p), cap)
        out = [{f: getattr(buf[i], f) for f, _ in B.im_sweep_rec._fields_} for i in range(k)]
        if clear:
            self.lib.im_sketch_clear_sweep_log(self.handle)
        return out

    def registers(self, which: int = 0) -> np.ndarray:
        out = np.empty((self.n, self.R), dtype=np.uint8)
        B.check(self.lib.im_sketch_get_registers(self.handle, which, out.ctypes.data))
        return out

    def blocked(self) -> np.ndarray:
        out = np.empty((self.n, self.R), dtype=np.uint8)
        B.check(self.lib.im_sketch_get_blocked(self.handle, out.ctypes.data))
        return out

    def free(self):
        if self.handle:
            self.lib.im_sketch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _ptr_and_residency(a, dtype):
    """Returns (pointer, on_device, keepalive) for a numpy array or a torch tensor."""
    torch = _torch()
    if isinstance(a, torch.Tensor):
        if a.dtype != dtype[1]:
            raise TypeError(f"expected {dtype[1]}, got {a.dtype}")
        a = a.contiguous()
        return a.data_ptr(), int(a.is_cuda), a
    arr = np.ascontiguousarray(a, dtype=dtype[0])
    return arr.ctypes.data, 0, arr


def _offsets(xadj):
    """(pointer, on_device, keepalive, offset_bits) of CSR offsets: int32 arrays and tensors are passed as
    they are (offset_bits 32), anything else as int64."""
    torch = _torch()
    if isinstance(xadj, torch.Tensor):
        if xadj.dtype == torch.int32:
            t = xadj.contiguous()
            return t.data_ptr(), int(t.is_cuda), t, 32
        p, d, k = _ptr_and_residency(xadj, (np.int64, torch.int64))
        return p, d, k, 64
    if np.asarray(xadj).dtype == np.int32:
        arr = np.ascontiguousarray(xadj, dtype=np.int32)
        return arr.ctypes.data, 0, arr, 32
    p, d, k = _ptr_and_residency(xadj, (np.int64, torch.int64))
    return p, d, k, 64


def im_build_sketches(ctx: Context, xadj, adj, n: int, R: int, model: str = "const", p: float = 0.0,
                      per_edge=None, hash_seed: int = 0, eps_c: float = 0.0, heavy_degree: int = 0,
                      piece_edges: int = 0, sparse_div: int = 0, time_sweeps=False,
                      in_place: bool = False, atomic_reverse: bool = False) -> Sketch:
    """Alg. 1 initialisation + Alg. 2: builds the per-vertex rank registers of R samples.
    time_sweeps: True times every kernel of every sweep (IM_BUILD_TIME_SWEEPS), "pieces" the
    split-row piece kernel only (IM_BUILD_TIME_PIECES);
    in_place selects in-place sweeps (IM_BUILD_IN_PLACE) for the build and every rebuild;
    atomic_reverse the atomic reverse-CSR construction (IM_BUILD_ATOMIC_REVERSE)."""
    if time_sweeps not in (False, True, "pieces"):
        raise ValueError("time_sweeps must be False, True or 'pieces'")
    torch = _torch()
    xp, xdev, xk, xbits = _offsets(xadj)
    ap, adev, ak = _ptr_and_residency(adj, (np.int32, torch.int32))
    if xdev != adev:
        raise ValueError("xadj and adj must both be host arrays or both device tensors")
    m = int(len(adj)) if not isinstance(adj, torch.Tensor) else int(adj.numel())
    g = B.im_csr(n, m, xp, ap, xdev, xbits)
    keep = [xk, ak]
    pe_ptr = None
    if model == "edge":
        pp, pdev, pk = _ptr_and_residency(per_edge, (np.float32, torch.float32))
        if pdev != xdev:
            raise ValueError("per-edge probabilities must reside where the CSR resides")
        pe_ptr = pp
        keep.append(pk)
    probs = B.im_probs(_KIND[model], float(p), pe_ptr)
    timing = (B.IM_BUILD_TIME_PIECES if time_sweeps == "pieces" else
              B.IM_BUILD_TIME_SWEEPS if time_sweeps else 0)
    flags = (timing | (B.IM_BUILD_IN_PLACE if in_place else 0) |
             (B.IM_BUILD_ATOMIC_REVERSE if atomic_reverse else 0))
    opts = B.im_build_opts(eps_c, heavy_degree, piece_edges, sparse_div, flags)
    h = ctypes.c_void_p()
    B.check(ctx.lib.im_build_sketches(ctx.handle, ctypes.byref(g), ctypes.byref(probs), R, hash_seed & 0xFFFFFFFF,
                                      ctypes.byref(opts), ctypes.byref(h)))
    del keep
    return Sketch(ctx, h, n, R)


def im_evaluate_influence(ctx: Context, xadj, adj, n: int, seeds, R: int, model: str = "const", p: float = 0.0,
                          per_edge=None, hash_seed: int = 0):
    """Monte-Carlo influence of a seed set over R fresh samples: (sigma, reached pairs)."""
    torch = _torch()
    xp, xdev, xk, xbits = _offsets(xadj)
    ap, adev, ak = _ptr_and_residency(adj, (np.int32, torch.int32))
    if xdev != adev:
        raise ValueError("xadj and adj must both be host arrays or both device tensors")
    m = int(len(adj)) if not isinstance(adj, torch.Tensor) else int(adj.numel())
    keep = [xk, ak]
    pe_ptr = None
    if model == "edge":
        pp, pdev, pk = _ptr_and_residency(per_edge, (np.float32, torch.float32))
        if pdev != xdev:
            raise ValueError("per-edge probabilities must reside where the CSR resides")
        pe_ptr = pp
        keep.append(pk)
    sv = np.ascontiguousarray(seeds, dtype=np.int32).ravel()
    sigma, reach = ctypes.c_double(), ctypes.c_int64()
    B.check(ctx.lib.im_evaluate_influence(ctx.handle, ctypes.byref(B.im_csr(n, m, xp, ap, xdev, xbits)),
                                          ctypes.byref(B.im_probs(_KIND[model], float(p), pe_ptr)), R,
                                          hash_seed & 0xFFFFFFFF, sv.ctypes.data, len(sv), ctypes.byref(sigma),
                                          ctypes.byref(reach)))
    del keep
    return sigma.value, reach.value


def im_estimate(sk: Sketch, verts) -> float:
    """Eq. (sketch-estimate) of the merged sketch of a vertex set, as binary32."""
    v = np.ascontiguousarray(verts, dtype=np.int32).ravel()
    out = ctypes.c_float()
    B.check(sk.lib.im_estimate(sk.handle, v.ctypes.data, len(v), ctypes.byref(out)))
    return float(out.value)


def im_estimate_all(sk: Sketch, out=None):
    """Per-vertex estimates (binary32).  `out` may be a float32 CUDA tensor of n elements."""
    torch = _torch()
    if out is not None and isinstance(out, torch.Tensor):
        if out.dtype != torch.float32 or out.numel() != sk.n or not out.is_cuda:
            raise ValueError("out must be a float32 CUDA tensor of n elements")
        B.check(sk.lib.im_estimate_all(sk.handle, out.data_ptr(), 1))
        return out
    res = np.empty(sk.n, dtype=np.float32)
    B.check(sk.lib.im_estimate_all(sk.handle, res.ctypes.data, 0))
    return res


def im_select_seeds(sk: Sketch, K: int, eps_g: float = 0.01, eps_l: float = 0.3, noalloc: bool = False,
                    resume: bool = False):
    """Alg. 1 greedy loop with error-adaptive rebuild.  Returns (seeds, steps, stats).

    noalloc selects im_select_seeds_noalloc (no device allocation in the call; K <= 4096);
    resume selects im_select_seeds_resume (reuses or continues the sketch's last run)."""
    if noalloc and resume:
        raise ValueError("noalloc and resume select different entry points")
    seeds = np.zeros(K, dtype=np.int32)
    steps = (B.im_step * K)()
    stats = B.im_select_stats()
    opts = B.im_select_opts(eps_g, eps_l)
    fn = (sk.lib.im_select_seeds_noalloc if noalloc else
          sk.lib.im_select_seeds_resume if resume else sk.lib.im_select_seeds)
    B.check(fn(sk.handle, K, ctypes.byref(opts), seeds.ctypes.data, ctypes.cast(steps, ctypes.c_void_p),
               ctypes.byref(stats)))
    st = [Step(**{f: getattr(s, f) for f, _ in B.im_step._fields_}) for s in steps]
    return seeds, st, {f: getattr(stats, f) for f, _ in B.im_select_stats._fields_}


@dataclass
class BatchJob:
    """One problem of a batched solve (see im_batch_create).  xadj/adj/per_edge are numpy
    arrays or device tensors (all of one kind)."""
    xadj: object
    adj: object
    n: int
    R: int
    K: int
    model: str = "const"
    p: float = 0.0
    per_edge: object = None
    hash_seed: int = 0
    eps_c: float = 0.0
    eps_g: float = 0.01
    eps_l: float = 0.3


class Batch:
    """Handle of a batched solve: every job's graph resident on the device, one captured launch."""

    def __init__(self, ctx: Context, handle, jobs):
        self.ctx, self.handle, self.lib = ctx, handle, ctx.lib
        self.ns = [j.n for j in jobs]
        self.Rs = [j.R for j in jobs]
        self.Ks = [j.K for j in jobs]

    def run(self) -> dict:
        st = B.im_batch_stats()
        B.check(self.lib.im_batch_run(self.handle, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in B.im_batch_stats._fields_}

    def result(self, job: int):
        """(seeds, steps, counters) of job `job` from the last run."""
        K = self.Ks[job]
        seeds = np.zeros(K, dtype=np.int32)
        steps = (B.im_step * K)()
        res = B.im_batch_job_result()
        B.check(self.lib.im_batch_get_result(self.handle, job, seeds.ctypes.data, ctypes.cast(steps, ctypes.c_void_p),
                                             ctypes.byref(res)))
        st = [Step(**{f: getattr(s, f) for f, _ in B.im_step._fields_}) for s in steps]
        return seeds, st, {f: getattr(res, f) for f, _ in B.im_batch_job_result._fields_}

    def registers(self, job: int, which: int = 0) -> np.ndarray:
        out = np.empty((self.ns[job], self.Rs[job]), dtype=np.uint8)
        B.check(self.lib.im_batch_get_registers(self.handle, job, which, out.ctypes.data))
        return out

    def device_bytes(self) -> int:
        return int(self.lib.im_batch_device_bytes(self.handle))

    def free(self):
        if self.handle:
            self.lib.im_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def im_batch_create(ctx: Context, jobs, autotune: bool = False, lanes_per_row: int = 0, tile_edges: int = 0,
                    heavy_degree: int = 0, piece_edges: int = 0, workgroups: int = 0, pin_edges: int = 0) -> Batch:
    """Uploads every job and captures the persistent launch (Alg. 1 + Alg. 2 per job)."""
    torch = _torch()
    arr = (B.im_batch_job * len(jobs))()
    keep = []
    for i, j in enumerate(jobs):
        xp, xdev, xk, xbits = _offsets(j.xadj)
        ap, adev, ak = _ptr_and_residency(j.adj, (np.int32, torch.int32))
        if xdev != adev:
            raise ValueError("xadj and adj must both be host arrays or both device tensors")
        m = int(len(j.adj)) if not isinstance(j.adj, torch.Tensor) else int(j.adj.numel())
        keep += [xk, ak]
        pe_ptr = None
        if j.model == "edge":
            pp, pdev, pk = _ptr_and_residency(j.per_edge, (np.float32, torch.float32))
            if pdev != xdev:
                raise ValueError("per-edge probabilities must reside where the CSR resides")
            pe_ptr = pp
            keep.append(pk)
        arr[i].graph = B.im_csr(j.n, m, xp, ap, xdev, xbits)
        arr[i].probs = B.im_probs(_KIND[j.model], float(j.p), pe_ptr)
        arr[i].R, arr[i].K, arr[i].hash_seed = j.R, j.K, j.hash_seed & 0xFFFFFFFF
        arr[i].eps_c, arr[i].eps_g, arr[i].eps_l = j.eps_c, j.eps_g, j.eps_l
    opts = B.im_batch_opts(1 if autotune else 0, lanes_per_row, tile_edges, heavy_degree, piece_edges, workgroups,
                           pin_edges)
    h = ctypes.c_void_p()
    B.check(ctx.lib.im_batch_create(ctx.handle, len(jobs), ctypes.cast(arr, ctypes.c_void_p), ctypes.byref(opts),
                                    ctypes.byref(h)))
    del keep
    return Batch(ctx, h, jobs)


class Server:
    """Serving engine of the library (im_server_*): resident graphs, concurrent slots, sketch reuse,
    admission by an HBM budget.  submit() returns a ticket; wait() blocks for its seeds and response."""

    def __init__(self, device: int = 0, slots: int = 4, hbm_budget: int = 0, max_copies: int = 0):
        self.lib = B.load()
        h = ctypes.c_void_p()
        B.check(self.lib.im_server_create(device, ctypes.byref(B.im_server_opts(slots, max_copies, hbm_budget)),
                                          ctypes.byref(h)))
        self.handle = h
        self._ns = []
        self._pending = {}

    def add_graph(self, xadj, adj, n: int) -> int:
        torch = _torch()
        xp, xdev, xk, xbits = _offsets(xadj)
        ap, adev, ak = _ptr_and_residency(adj, (np.int32, torch.int32))
        if xdev != adev:
            raise ValueError("xadj and adj must both be host arrays or both device tensors")
        m = int(len(adj)) if not isinstance(adj, torch.Tensor) else int(adj.numel())
        gid = ctypes.c_int32()
        B.check(self.lib.im_server_add_graph(self.handle, ctypes.byref(B.im_csr(n, m, xp, ap, xdev, xbits)),
                                             ctypes.byref(gid)))
        self._ns.append(n)
        return gid.value

    def submit(self, graph: int, R: int, K: int, model: str = "const", p: float = 0.0, hash_seed: int = 0,
               eps_c: float = 0.0, eps_g: float = 0.01, eps_l: float = 0.3) -> int:
        if model not in ("const", "wc"):
            raise ValueError("requests take model 'const' or 'wc'")
        seeds = np.zeros(K, dtype=np.int32)
        rq = B.im_request(graph, _KIND[model], p, R, K, hash_seed & 0xFFFFFFFF, eps_c, eps_g, eps_l)
        t = ctypes.c_int64()
        B.check(self.lib.im_server_submit(self.handle, ctypes.byref(rq), seeds.ctypes.data, ctypes.byref(t)))
        self._pending[t.value] = seeds
        return t.value

    def wait(self, ticket: int):
        """(seeds, response dict); raises ImError if the request failed."""
        resp = B.im_response()
        st = self.lib.im_server_wait(self.handle, ticket, ctypes.byref(resp))
        seeds = self._pending.pop(ticket)
        B.check(st)
        return seeds, {f: getattr(resp, f) for f, _ in B.im_response._fields_}

    def cancel(self, ticket: int) -> bool:
        """Cancels a request that has not started; False if it started, finished or is unknown."""
        st = self.lib.im_server_cancel(self.handle, ticket)
        if st == B.IM_OK:
            return True
        if st == B.IM_ERR_STATE:
            return False
        B.check(st)

    def stats(self) -> dict:
        s = B.im_server_stats()
        B.check(self.lib.im_server_get_stats(self.handle, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in B.im_server_stats._fields_}

    def close(self):
        if self.handle:
            self.lib.im_server_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
