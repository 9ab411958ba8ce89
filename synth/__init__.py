"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module synthesises graphs only; it contains none of the influence-maximisation
arithmetic (no hashing, thresholds, registers or estimates).  Graphs are directed, in CSR
form over out-neighbours (the layout of the paper's implementation section): ``xadj``
(int64, n+1 offsets) and ``adj`` (int32 targets, each row sorted, no duplicates, no
self-loops).

The paper evaluates on twelve real networks (Table NetProps) that are not available here;
R-MAT and Erdos-Renyi graphs with the same degree range stand in for them.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgraphgen.so")
_SRC = os.path.join(_HERE, "graphgen.c")
_lock = threading.Lock()
_lib = None

RMAT_ABC = (0.57, 0.19, 0.19)  # quadrant probabilities a, b, c (d = 0.05)


def build(force: bool = False) -> str:
    """Compile the generator library with gcc (OpenMP, -O3)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_SO):
                build()
            lib = ctypes.CDLL(_SO)
            i64, u64, p = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
            lib.gg_rmat_draw.argtypes = [ctypes.c_int, i64, ctypes.c_double, ctypes.c_double, ctypes.c_double, u64, p, p]
            lib.gg_rmat_draw.restype = i64
            lib.gg_keys_to_csr.argtypes = [p, i64, i64, p, p, p]
            lib.gg_keys_to_csr.restype = i64
            lib.gg_er_draw.argtypes = [i64, i64, u64, p]
            lib.gg_er_draw.restype = i64
            lib.gg_rand64.argtypes = [u64, u64]
            lib.gg_rand64.restype = u64
            _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


@dataclass
class Graph:
    """A directed graph in CSR over out-neighbours."""

    n: int
    xadj: np.ndarray  # int64[n+1]
    adj: np.ndarray  # int32[m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.xadj[-1])

    def in_degree(self) -> np.ndarray:
        return np.bincount(self.adj, minlength=self.n).astype(np.int64)


def _keys_to_graph(keys: np.ndarray, n: int, name: str) -> Graph:
    xadj = np.empty(n + 1, dtype=np.int64)
    adj = np.empty(max(len(keys), 1), dtype=np.int32)
    tmp = np.empty(n + 1, dtype=np.int64)
    m = _load().gg_keys_to_csr(_ptr(keys), len(keys), n, _ptr(xadj), _ptr(adj), _ptr(tmp))
    return Graph(n=n, xadj=xadj, adj=adj[:m].copy(), name=name)


def rmat(scale: int, draws: int, seed: int, abc=RMAT_ABC) -> Graph:
    """R-MAT graph on 2^scale vertices from `draws` edge draws; self-loops and duplicates dropped."""
    n = 1 << scale
    keys = np.empty(max(draws, 1), dtype=np.uint64)
    keep = np.empty(max(draws, 1), dtype=np.uint8)
    a, b, c = abc
    k = _load().gg_rmat_draw(scale, draws, a, b, c, seed, _ptr(keys), _ptr(keep))
    del keep
    return _keys_to_graph(keys[:k], n, f"rmat{scale}_d{draws}_s{seed}")


def erdos_renyi(n: int, m: int, seed: int) -> Graph:
    """m distinct uniform ordered pairs (u != v) by rejection."""
    keys = np.empty(max(m, 1), dtype=np.uint64)
    k = _load().gg_er_draw(n, m, seed, _ptr(keys))
    if k < 0:
        raise ValueError("m exceeds n(n-1)")
    return _keys_to_graph(keys[:k], n, f"er{n}_m{m}_s{seed}")


def from_edges(n: int, edges) -> Graph:
    """Small hand-made graphs (tests): list of (u, v) pairs."""
    e = np.asarray(list(edges), dtype=np.uint64).reshape(-1, 2)
    keys = (e[:, 0] << np.uint64(32)) | e[:, 1]
    keys = keys[e[:, 0] != e[:, 1]]
    return _keys_to_graph(np.ascontiguousarray(keys), n, "custom")


def rand64(seed: int, ctr: int) -> int:
    return int(_load().gg_rand64(seed, ctr))


# --------------------------------------------------------------------------------------
# Workload recipes.  Graph seed = 1 + workload index; hash seed 0.
# --------------------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    graph: Graph
    model: str  # "const" or "wc"
    p: float  # constant IC probability (ignored for "wc")
    J: int
    K: int
    eps_g: float = 0.01
    eps_l: float = 0.3
    eps_c: float = 0.0
    hash_seed: int = 0


def workload_er_small() -> Workload:
    """Directed ER, n=1000, m=10000, IC p=0.1, J=64, K=10."""
    return Workload("er_n1000_m10000_p0.1_J64_K10", erdos_renyi(1000, 10000, seed=1), "const", 0.1, 64, 10)


def workload_rmat20() -> Workload:
    """R-MAT scale 20, 16*2^20 draws, IC p=0.01, J=256, K=50."""
    return Workload("rmat20_p0.01_J256_K50", rmat(20, 16 << 20, seed=2), "const", 0.01, 256, 50)


def workload_rmat24_wc() -> Workload:
    """R-MAT scale 24, 16*2^24 draws, weighted cascade, J=256, K=50."""
    return Workload("rmat24_wc_J256_K50", rmat(24, 16 << 24, seed=3), "wc", 0.0, 256, 50)


def workload_scaled(scale: int, model: str = "const", p: float = 0.01, J: int = 256, K: int = 50,
                    seed: int = 2, edge_factor: int = 16) -> Workload:
    """R-MAT at a reduced scale with the same recipe (tests at sizes the oracle finishes quickly)."""
    g = rmat(scale, edge_factor << scale, seed=seed)
    return Workload(f"rmat{scale}_{model}_J{J}_K{K}", g, model, p, J, K)


def batch_recipe(master_seed: int = 4, count: int = 64):
    """Parameters of the batched workload: per graph (scale, draws, p, seed).

    log2 n uniform over the integers 12..18, average degree uniform in [8, 32],
    p uniform over {0.005, 0.01, 0.05}; J=128, K=20.  Draws come from the counter generator.
    """
    out = []
    for i in range(count):
        r0 = rand64(master_seed, 4 * i)
        r1 = rand64(master_seed, 4 * i + 1)
        r2 = rand64(master_seed, 4 * i + 2)
        scale = 12 + int(r0 % 7)
        deg = 8.0 + 24.0 * ((r1 >> 11) / float(1 << 53))
        p = (0.005, 0.01, 0.05)[int(r2 % 3)]
        out.append((scale, int(round(deg * (1 << scale))), p, 1000 * master_seed + i))
    return out


def serving_recipe(master_seed: int = 5, graphs: int = 16, requests: int = 2000, rate: float = 200.0):
    """The serving workload: a pool of R-MAT graphs and a Poisson request stream.

    Graphs: log2 n uniform over the integers 14..22, average degree 16 (draws = 16 n),
    graph seed 100 * master_seed + index.  Requests: exponential inter-arrival gaps
    with mean 1/rate seconds; graph uniform over the pool; model uniform over
    {IC p=0.01, IC p=0.1, weighted cascade}; R uniform over {64, 256}; K uniform
    over the integers 10..100.  Returns (pool, stream) with pool entries
    (scale, draws, seed) and stream entries (arrival_s, graph, model, p, R, K).
    """
    pool = []
    for i in range(graphs):
        scale = 14 + int(rand64(master_seed, i) % 9)
        pool.append((scale, 16 << scale, 100 * master_seed + i))
    stream, t = [], 0.0
    base = graphs
    for i in range(requests):
        r = [rand64(master_seed, base + 5 * i + k) for k in range(5)]
        u = (r[0] >> 11) / float(1 << 53)
        t += -math.log1p(-u) / rate
        model, p = [("const", 0.01), ("const", 0.1), ("wc", 0.0)][int(r[2] % 3)]
        stream.append((t, int(r[1] % graphs), model, p, (64, 256)[int(r[3] % 2)], 10 + int(r[4] % 91)))
    return pool, stream
