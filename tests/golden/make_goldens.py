"""Writes the expected outputs of the benchmark workloads, computed by the CPU oracle only.

Run on a CPU host:  python tests/golden/make_goldens.py {er1000,rmat20,rmat24_wc,batch64,serve_sample}

For each workload the seeded input generator builds the graph, the oracle runs Alg. 1 with
Alg. 2 (build, then the greedy loop with error-adaptive rebuild) and this script records:

* the input's fingerprint (sha256 of xadj and adj), so a reader can check it compares the
  same graph;
* the build: sweep count, |L_t| trace, edge-visit trace, sha256 of the n x J register array
  (vertex-major, as the C ABI returns it), a digest per 1/64 of the vertices, and the full
  register rows of the largest in-degree vertices, the largest out-degree vertices and a
  seeded random sample;
* every greedy step's record (seed, score, e, sigma, delta, err_l, err_g, fresh, rebuilt,
  rebuild sweeps and visits) with sha256 of the registers the step used and of the blocked
  pairs after it.  After step k these are the final outputs of a run with K = k (no rebuild
  follows the last step), so a file holding k steps is the expected result of K = k.

The 2^24-vertex run is long (the build alone is over 10^12 edge visits on one core): the file
is rewritten after the build and after every step, and the greedy prefix it holds is the
number of steps done when the run was stopped ("K_done").  Nothing here runs GPU code.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

CHUNKS = 64


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).data).hexdigest()


def chunk_digests(M: np.ndarray) -> list:
    n = M.shape[0]
    return [sha(M[c * n // CHUNKS:(c + 1) * n // CHUNKS])[:16] for c in range(CHUNKS)]


def sample_rows(g) -> list:
    """Vertices whose register rows are stored in full: hubs by in- and out-degree, and a random sample."""
    indeg = g.in_degree()
    outdeg = np.diff(g.xadj)
    k = min(8, g.n)
    pick = list(np.argsort(-indeg, kind="stable")[:k]) + list(np.argsort(-outdeg, kind="stable")[:k])
    rng = np.random.default_rng(24)
    nz = np.nonzero(outdeg > 0)[0]
    if len(nz):
        pick += list(rng.choice(nz, min(8, len(nz)), replace=False))
    out = []
    for v in pick:
        if int(v) not in out:
            out.append(int(v))
    return out


def fingerprint(g) -> dict:
    return {"n": int(g.n), "m": int(g.m), "xadj_sha256": sha(g.xadj), "adj_sha256": sha(g.adj[: g.m])}


def solve(g, model, p, J, K, eps_g=0.01, eps_l=0.3, eps_c=0.0, hash_seed=0, out_path=None, meta=None, log=None):
    """Runs the oracle's greedy loop on one problem and returns the record (written to out_path as it grows)."""
    t0 = time.time()
    thr = oracle.edge_thresholds(g, model, np.float32(p))
    rows = sample_rows(g)
    rec = dict(meta or {})
    rec.update({"graph": fingerprint(g), "model": model, "p": float(np.float32(p)), "J": J, "K": K,
                "eps_g": eps_g, "eps_l": eps_l, "eps_c": eps_c, "hash_seed": hash_seed,
                "host_cpu": _cpu_model(), "K_done": 0, "steps": []})

    def flush():
        rec["oracle_wall_s"] = round(time.time() - t0, 1)
        if out_path:
            tmp = out_path + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(rec, fh, indent=1)
            os.replace(tmp, out_path)

    def obs(k, M, blk, st, tl, te):
        if k == 0:
            rec["build"] = {"sweeps": int(len(te)), "visits": int(te.sum()), "live_trace": [int(x) for x in tl],
                            "visit_trace": [int(x) for x in te], "M_sha256": sha(M), "M_chunks": chunk_digests(M),
                            "rows": {str(v): M[v].tobytes().hex() for v in rows},
                            "wall_s": round(time.time() - t0, 1)}
        else:
            st = dict(st)
            prev = st.pop("previous", None)
            if prev is not None:  # the rebuild after step k - 1 has ended: complete its record
                for f in ("rebuilt", "sweeps", "visits"):
                    rec["steps"][-1][f] = prev[f]
            st["M_sha256"] = sha(M)
            st["blk_sha256"] = sha(blk)
            st["wall_s"] = round(time.time() - t0, 1)
            rec["steps"].append(st)
            rec["K_done"] = k
        flush()
        if log:
            print(f"[golden] {rec.get('name', '')} k={k} t={time.time() - t0:.0f}s", file=log, flush=True)
        return False

    res = oracle.greedy(g, thr, J, K, seed=hash_seed, eps_g=eps_g, eps_l=eps_l, eps_c=eps_c, observer=obs)
    # the records of steps that rebuilt are completed after the observer saw them
    for st, full in zip(rec["steps"], res["steps"]):
        for f in ("rebuilt", "sweeps", "visits"):
            st[f] = full[f]
    rec["seeds"] = [int(s) for s in res["seeds"]]
    flush()
    return rec


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def path_of(name: str) -> str:
    return os.path.join(HERE, f"oracle_{name}.json")


def run_workload(w, log):
    meta = {"name": w.name}
    return solve(w.graph, w.model, w.p, w.J, w.K, w.eps_g, w.eps_l, w.eps_c, w.hash_seed, path_of(w.name), meta, log)


def _batch_job(args):
    i, (scale, draws, p, seed) = args
    g = synth.rmat(scale, draws, seed=seed)
    meta = {"name": f"job{i}", "scale": scale, "draws": draws, "graph_seed": seed}
    return solve(g, "const", p, 128, 20, meta=meta)


def serve_sample(pool, stream, limit=400):
    """Requests of the serving stream's first `limit` arrivals checked against the oracle, in arrival order:
    the first one of every (graph size, model, p, R) class on the pool's graphs of at most 2^15 vertices, and
    the first one of each R with IC p = 0.01 on its 2^18-vertex graph."""
    seen, out = set(), []
    for i, (t, gi, model, p, R, K) in enumerate(stream[:limit]):
        scale = pool[gi][0]
        key = (scale, model, p, R)
        if (scale <= 15 or (scale == 18 and model == "const" and p == 0.01)) and key not in seen:
            seen.add(key)
            out.append(i)
    return out


def _serve_job(args):
    i, (t, gi, model, p, R, K), (scale, draws, gseed) = args
    g = synth.rmat(scale, draws, seed=gseed)
    meta = {"name": f"request{i}", "request": i, "pool_graph": gi, "scale": scale, "draws": draws,
            "graph_seed": gseed}
    return solve(g, model, p, R, K, meta=meta)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["er1000", "rmat20", "rmat24_wc", "batch64", "serve_sample"])
    ap.add_argument("--procs", type=int, default=4, help="worker processes for the batch and serving sets")
    a = ap.parse_args()
    log = sys.stdout
    if a.workload == "er1000":
        run_workload(synth.workload_er_small(), log)
    elif a.workload == "rmat20":
        run_workload(synth.workload_rmat20(), log)
    elif a.workload == "rmat24_wc":
        run_workload(synth.workload_rmat24_wc(), log)
    else:
        from multiprocessing import Pool
        if a.workload == "batch64":
            tasks = list(enumerate(synth.batch_recipe()))
            fn, name = _batch_job, "batch64_rmat_J128_K20"
        else:
            pool, stream = synth.serving_recipe()
            tasks = [(i, stream[i], pool[stream[i][1]]) for i in serve_sample(pool, stream)]
            fn, name = _serve_job, "serve_sample"
        t0 = time.time()
        with Pool(a.procs) as pp:
            recs = []
            for r in pp.imap(fn, tasks):
                recs.append(r)
                print(f"[golden] {name} {r['name']} done t={time.time() - t0:.0f}s", flush=True)
        out = {"name": name, "host_cpu": _cpu_model(), "procs": a.procs, "oracle_wall_s": round(time.time() - t0, 1),
               "jobs": recs}
        with open(path_of(name) + ".tmp", "w") as fh:
            json.dump(out, fh, indent=1)
        os.replace(path_of(name) + ".tmp", path_of(name))


if __name__ == "__main__":
    main()
