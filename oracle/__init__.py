"""CPU oracle for the sketch-based influence-maximisation method (arXiv 2105.04023).

TEST INFRASTRUCTURE ONLY.  This package is the plain, single-threaded reference the GPU
library is checked against; only the tests, the smoke check and the benchmark's CPU-baseline
leg may import it.  It shares no code with the GPU library.  The arithmetic lives in
``hfr_oracle.c`` (plain C, IEEE double, ``-ffp-contract=off``); this module marshals numpy
arrays into it.

Functions follow the paper's sections: Eq. (hash) and Eq. (hash_prob) for sampling
(Sec. 3.1), Eqs. (sketch-add), (sketch-merge) and (sketch-estimate) for the registers
(Sec. 2.2), Alg. 2 for Simulate and Alg. 1 for the greedy loop with error-adaptive rebuild
(Sec. 3.2, 3.2.1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "hfr_oracle.c")
_lock = threading.Lock()
_lib = None

PHI = 0.77351  # Eq. (sketch-estimate) correction factor
H_MAX = 2**31 - 1  # largest value of the 31-bit edge hash, Eq. (hash)


class Step(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_int32),
        ("rebuilt", ctypes.c_int32),
        ("fresh", ctypes.c_int32),
        ("sweeps", ctypes.c_int32),
        ("score", ctypes.c_int64),
        ("reach", ctypes.c_int64),
        ("e", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("delta", ctypes.c_double),
        ("err_l", ctypes.c_double),
        ("err_g", ctypes.c_double),
        ("visits", ctypes.c_int64),
    ]


# int obs(k, const uint8_t* M, const uint8_t* blk, const orc_step* st, int64_t sweeps,
#         const int64_t* trace_live, const int64_t* trace_edges, void* user)
_OBSERVER = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                             ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc: -O2, no FMA contraction, no fast-math."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC", "-o", tmp, _SRC,
             "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_SO):
                build()
            lib = ctypes.CDLL(_SO)
            p, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
            lib.orc_murmur3_32.argtypes = [p, ctypes.c_uint64, u32]
            lib.orc_murmur3_32.restype = u32
            lib.orc_edge_hash.argtypes = [i32, i32, u32]
            lib.orc_edge_hash.restype = u32
            lib.orc_sim_word.argtypes = [i32, u32]
            lib.orc_sim_word.restype = u32
            lib.orc_rank.argtypes = [i32, i32, u32]
            lib.orc_rank.restype = ctypes.c_uint8
            lib.orc_threshold.argtypes = [ctypes.c_float]
            lib.orc_threshold.restype = u32
            lib.orc_live.argtypes = [u32, u32, u32]
            lib.orc_live.restype = ctypes.c_int
            lib.orc_edge_thresholds.argtypes = [i64, p, p, ctypes.c_int, ctypes.c_float, p, p]
            lib.orc_edge_thresholds.restype = ctypes.c_int
            lib.orc_simulate.argtypes = [i64, p, p, p, i32, u32, p, ctypes.c_double, i64, p, p, p, i64]
            lib.orc_simulate.restype = i64
            lib.orc_estimate.argtypes = [p, i32]
            lib.orc_estimate.restype = ctypes.c_double
            lib.orc_reach_add.argtypes = [i64, p, p, p, i32, u32, p, i32]
            lib.orc_reach_add.restype = i64
            lib.orc_greedy.argtypes = [i64, p, p, p, i32, u32, i32, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, p, p, p, p, p]
            lib.orc_greedy.restype = ctypes.c_int
            lib.orc_greedy_observed.argtypes = [i64, p, p, p, i32, u32, i32, ctypes.c_double, ctypes.c_double,
                                                ctypes.c_double, p, p, p, p, p, _OBSERVER, p]
            lib.orc_greedy_observed.restype = ctypes.c_int
            _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _csr(graph):
    xadj = np.ascontiguousarray(graph.xadj, dtype=np.int64)
    adj = np.ascontiguousarray(graph.adj, dtype=np.int32)
    if len(adj) == 0:
        adj = np.zeros(1, dtype=np.int32)
    return xadj, adj


# ---- Sec. 3.1: hash-based fused sampling ----------------------------------------------

def murmur3_32(data: bytes, seed: int) -> int:
    buf = np.frombuffer(bytes(data) + b"\0", dtype=np.uint8)
    return int(_load().orc_murmur3_32(buf.ctypes.data, len(data), seed & 0xFFFFFFFF))


def edge_hash(u: int, v: int, seed: int = 0) -> int:
    """Eq. (hash): Murmur3(LE32(u) || LE32(v)) mod 2^31."""
    return int(_load().orc_edge_hash(u, v, seed & 0xFFFFFFFF))


def sim_word(j: int, seed: int = 0) -> int:
    """X_j of Eq. (hash_prob)."""
    return int(_load().orc_sim_word(j, seed & 0xFFFFFFFF))


def rank(v: int, j: int, seed: int = 0) -> int:
    """Initial register value clz(hash(v) xor hash(j)) (Alg. 1 initialisation)."""
    return int(_load().orc_rank(v, j, seed & 0xFFFFFFFF))


def threshold(w: float) -> int:
    """Integer live threshold of binary32 weight w (0xFFFFFFFF if w is not in [0, 1])."""
    return int(_load().orc_threshold(ctypes.c_float(w)))


def live(h: int, x: int, thr: int) -> bool:
    return bool(_load().orc_live(h, x, thr))


def edge_thresholds(graph, model: str, p: float = 0.0, per_edge=None) -> np.ndarray:
    """Per-edge integer thresholds for constant IC ("const"), weighted cascade ("wc") or per-edge weights ("edge")."""
    xadj, adj = _csr(graph)
    m = int(xadj[-1])
    out = np.zeros(max(m, 1), dtype=np.uint32)
    kind = {"const": 0, "wc": 1, "edge": 2}[model]
    pe = None if per_edge is None else np.ascontiguousarray(per_edge, dtype=np.float32)
    rc = _load().orc_edge_thresholds(graph.n, _p(xadj), _p(adj), kind, ctypes.c_float(p), _p(pe), _p(out))
    if rc != 0:
        raise ValueError("edge weight outside [0, 1]")
    return out


# ---- Alg. 2: Simulate --------------------------------------------------------------------

def simulate(graph, thr: np.ndarray, J: int, seed: int = 0, blk=None, eps_c: float = 0.0, max_sweeps: int = -1):
    """Returns (M uint8[n, J], sweeps, live_trace int64[sweeps+1], edge_trace int64[sweeps])."""
    xadj, adj = _csr(graph)
    n = graph.n
    M = np.zeros((n, J), dtype=np.uint8)
    cap = n + 2
    tl = np.zeros(cap, dtype=np.int64)
    te = np.zeros(cap, dtype=np.int64)
    b = None if blk is None else np.ascontiguousarray(blk, dtype=np.uint8)
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    sw = _load().orc_simulate(n, _p(xadj), _p(adj), _p(thr), J, seed & 0xFFFFFFFF, _p(b), eps_c, max_sweeps,
                              _p(M), _p(tl), _p(te), cap)
    if sw < 0:
        raise MemoryError("oracle simulate")
    return M, int(sw), tl[: sw + 1].copy(), te[:sw].copy()


# ---- Eq. (sketch-estimate) ---------------------------------------------------------------

def estimate(row: np.ndarray) -> float:
    r = np.ascontiguousarray(row, dtype=np.uint8)
    return float(_load().orc_estimate(_p(r), len(r)))


# ---- Alg. 1: reach of the seed set and the greedy loop ----------------------------------

def reach_add(graph, thr: np.ndarray, J: int, seed: int, blk: np.ndarray, s: int) -> int:
    """Blocks the reach of s in every sample (in place on blk uint8[n, J]); returns the number of new pairs."""
    xadj, adj = _csr(graph)
    assert blk.dtype == np.uint8 and blk.flags.c_contiguous
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    return int(_load().orc_reach_add(graph.n, _p(xadj), _p(adj), _p(thr), J, seed & 0xFFFFFFFF, _p(blk), s))


def greedy(graph, thr: np.ndarray, J: int, K: int, seed: int = 0, eps_g: float = 0.01, eps_l: float = 0.3,
           eps_c: float = 0.0, want_blk: bool = False, observer=None):
    """Alg. 1.  Returns a dict: seeds, steps (list of dicts), M (final registers), blk, build_sweeps, build_visits.

    observer (optional) is called as observer(k, M, blk, step, trace_live, trace_edges) with numpy views
    of the oracle's own buffers (valid during the call only): k = 0 once after the build (M = the build's
    registers, trace_live[t] = |L_t| for t = 0..sweeps, trace_edges[t] = visits of sweep t, blk and step
    None), then k = 1..K after each step, before its rebuild (M = registers the step used, blk = blocked
    pairs after it, step = its record as a dict, with, for k >= 2, the completed record of step k - 1 under
    "previous": its rebuild, if any, has ended): the final state of a run with K = k.  A true return value
    ends the run; the result then holds the steps done ("stopped_after").
    """
    xadj, adj = _csr(graph)
    n = graph.n
    if not (1 <= K <= n):
        raise ValueError("K must be in [1, n]")
    M = np.zeros((n, J), dtype=np.uint8)
    blk = np.zeros((n, J), dtype=np.uint8) if want_blk else None
    steps = (Step * K)()
    bs = ctypes.c_int64()
    bv = ctypes.c_int64()
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    last = [0]

    def _obs(k, pM, pblk, pst, sweeps, ptl, pte, user):
        def view(ptr, count, dt):
            return np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(dt)), shape=(count,))
        Mv = view(pM, n * J, ctypes.c_uint8).reshape(n, J)
        last[0] = k
        if k == 0:
            tl = view(ptl, sweeps + 1, ctypes.c_int64).copy()
            te = view(pte, max(sweeps, 1), ctypes.c_int64)[:sweeps].copy()
            return int(bool(observer(0, Mv, None, None, tl, te)))
        st = ctypes.cast(pst, ctypes.POINTER(Step)).contents
        rec = {f: getattr(st, f) for f, _ in Step._fields_}
        if k >= 2:
            rec["previous"] = {f: getattr(steps[k - 2], f) for f, _ in Step._fields_}
        return int(bool(observer(k, Mv, view(pblk, n * J, ctypes.c_uint8).reshape(n, J), rec, None, None)))

    cb = _OBSERVER(_obs) if observer is not None else _OBSERVER()
    rc = _load().orc_greedy_observed(n, _p(xadj), _p(adj), _p(thr), J, seed & 0xFFFFFFFF, K, eps_g, eps_l, eps_c,
                                     _p(M), _p(blk), ctypes.cast(steps, ctypes.c_void_p), ctypes.byref(bs),
                                     ctypes.byref(bv), cb, None)
    if rc < 0:
        raise MemoryError("oracle greedy")
    done = K if rc == 0 else last[0]
    recs = [{f: getattr(s, f) for f, _ in Step._fields_} for s in steps[:done]]
    return {
        "seeds": [r["seed"] for r in recs],
        "steps": recs,
        "M": M,
        "blk": blk,
        "build_sweeps": bs.value,
        "build_visits": bv.value,
        "stopped_after": None if rc == 0 else done,
    }
