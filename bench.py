"""Benchmark of the sketch-based influence-maximisation path on one MI355X.

One step = the whole path on one synthetic graph already resident in HBM: build the
sketches (edge hashing, thresholds, register init, synchronous sweeps to the fixed point)
and select K seeds with error-adaptive rebuild.  The headline value is edge*simulation
visits per second of sketch build (visits = R * edges with a live head, summed over the
build's sweeps); the K-seed IM time is reported beside it.

Prints one JSON line.  `--gpus N` with N > 1 is refused: this path runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


WORKLOADS = {
    "rmat24_wc_J256_K50": lambda s: s.workload_rmat24_wc(),
    "rmat20_p0.01_J256_K50": lambda s: s.workload_rmat20(),
    "er_n1000_m10000_p0.1_J64_K10": lambda s: s.workload_er_small(),
}


def heavy_launch_bytes(rec, J, wc, m_heavy, npieces):
    """Algorithmic HBM bytes of one launch of the split-row piece kernel (k_sweep_heavy).

    Per merged edge (a visited edge live in some sample): the neighbour's row (J bytes) and,
    for the weighted cascade, the edge's threshold (4); the edge's hash is recomputed from
    its two ids, and an edge live in no sample is known to be so from its id (flag bit),
    which costs nothing more.  Edge
    ids: a dense launch reads every split-row out-edge id (4 m_heavy) and the piece table
    (20 B per piece), a sparse launch the ids of the edges it visits (4 each).  The partial
    rows and flags written (J + 4 bytes per run of a row's pieces with a live edge) are not
    counted: how many there were is not logged, and they are under 1% of the bytes.  A
    launch past the stopping rule moves nothing.
    """
    if not rec["ran"]:
        return 0
    hv = rec["visits"] - rec["light_visits"]
    hm = rec["merged"] - rec["light_merged"]
    b = hm * (J + (4 if wc else 0))
    if rec["sparse"]:
        b += 4 * hv
    else:
        b += 4 * m_heavy + 20 * npieces
    return b


def heavy_launch_visit_bytes(rec, J, wc, m_heavy, npieces):
    """The same launch priced by the per-sweep formula of the measurement plan, which charges the
    neighbour's row (and threshold) for EVERY visited edge (E_t * J + ...), live in some sample or
    not.  The kernel reads nothing for an edge live in no sample, so this fraction can exceed 1."""
    if not rec["ran"]:
        return 0
    hv = rec["visits"] - rec["light_visits"]
    b = hv * (J + (4 if wc else 0))
    b += 4 * hv if rec["sparse"] else 4 * m_heavy + 20 * npieces
    return b


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweep_heavy__rmat24_wc_J256_K50__traffic.md")
KERNEL_SOURCES = ["paper_2105_04023_amd/csrc/hfr_kernels.hip", "paper_2105_04023_amd/csrc/hfr_device.h",
                  "paper_2105_04023_amd/csrc/hfr_internal.h", "paper_2105_04023_amd/csrc/hfr_api.hip"]
COPY_BYTES = 1 << 30


def kernel_source_hash() -> str:
    """sha256 over the sources the sweep kernels and their launches are built from."""
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per k_sweep_heavy launch from the committed counter summary, or None when the
    summary is missing or was taken from other kernel sources."""
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                kv[k.strip()] = v.strip().strip("`")
        if kv.get("source_sha256") != kernel_source_hash():
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def summarize_pmc(fetch_dir: str, write_dir: str, command: str):
    """Writes the traffic summary from two rocprofv3 --pmc runs of the same command (FETCH_SIZE, then
    WRITE_SIZE; KiB per dispatch).  Each counter is scaled by what it reads for the 1 GiB device copy
    that bench.py --calibrate-copy performs: factor = copied bytes / (counter KiB * 1024)."""
    import csv

    def per_dispatch(d):
        out = {}
        path = os.path.join(d, "run_counter_collection.csv")
        for r in csv.DictReader(open(path)):
            k = int(r["Dispatch_Id"])
            e = out.setdefault(k, {"name": r["Kernel_Name"], "v": 0.0})
            e["v"] += float(r["Counter_Value"])
        return out

    res = {}
    for tag, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        disp = per_dispatch(d)
        heavy = [e["v"] for e in disp.values() if e["name"].startswith("void hfr::k_sweep_heavy<")]
        copies = [e["v"] for e in disp.values() if "copyBuffer" in e["name"]]
        if not heavy or not copies:
            raise SystemExit(f"{d}: no k_sweep_heavy or copy dispatches")
        cal = max(copies)  # the 1 GiB calibration copy is the largest copy
        factor = COPY_BYTES / (cal * 1024.0)
        res[tag] = (sum(heavy) / len(heavy), len(heavy), cal, factor)
    fetch_kib, n_f, cal_f, fac_f = res["FETCH_SIZE"]
    write_kib, n_w, cal_w, fac_w = res["WRITE_SIZE"]
    traffic = fetch_kib * 1024 * fac_f + write_kib * 1024 * fac_w
    lines = [
        "# k_sweep_heavy on rmat24_wc_J256_K50: HBM traffic from counters",
        "",
        "Commands (run from the repository root on an MI355X, `cd /tmp && export TMPDIR=/tmp` first):",
        "",
        f"    {command.format(counter='FETCH_SIZE', out=fetch_dir)}",
        f"    {command.format(counter='WRITE_SIZE', out=write_dir)}",
        "",
        f"k_sweep_heavy dispatches: {n_f} (FETCH_SIZE run), {n_w} (WRITE_SIZE run); averages per dispatch:",
        f"FETCH_SIZE {fetch_kib:.1f} KiB, WRITE_SIZE {write_kib:.1f} KiB.",
        f"Calibration: a {COPY_BYTES} B device copy read FETCH_SIZE {cal_f:.1f} KiB and WRITE_SIZE {cal_w:.1f} KiB,",
        f"so the factors are {fac_f:.4f} (fetch) and {fac_w:.4f} (write).",
        "",
        f"- fetch_bytes_per_launch: {fetch_kib * 1024 * fac_f:.0f}",
        f"- write_bytes_per_launch: {write_kib * 1024 * fac_w:.0f}",
        f"- traffic_bytes_per_launch: {traffic:.0f}",
        f"- source_sha256: `{kernel_source_hash()}`",
    ]
    return "\n".join(lines) + "\n"


def host_cpu() -> dict:
    """CPU model and the cores this process may run on."""
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"host_cpu": model, "host_nproc": os.cpu_count(), "host_usable_cores": usable}


def recorded_oracle_runs() -> list:
    """Wall times of the oracle's full runs on the configured workloads, as recorded (with the host's CPU
    model) when tests/golden/make_goldens.py wrote the expected values: one core per run."""
    out = []
    gdir = os.path.join(ROOT, "tests", "golden")
    for name in ("er_n1000_m10000_p0.1_J64_K10", "rmat20_p0.01_J256_K50", "rmat24_wc_J256_K50"):
        try:
            rec = json.load(open(os.path.join(gdir, f"oracle_{name}.json")))
        except (OSError, ValueError):
            continue
        b = rec.get("build")
        if not b:
            continue
        J = rec["J"]
        item = {"workload": name, "host_cpu": rec.get("host_cpu"), "cores": 1,
                "build_s": b["wall_s"], "build_visits": b["visits"] * J,
                "build_visits_per_s": b["visits"] * J / b["wall_s"] if b["wall_s"] > 0 else None,
                "greedy_steps_done": rec["K_done"], "K": rec["K"], "total_s": rec.get("oracle_wall_s")}
        out.append(item)
    try:
        rec = json.load(open(os.path.join(gdir, "oracle_batch64_rmat_J128_K20.json")))
        out.append({"workload": rec["name"], "host_cpu": rec.get("host_cpu"), "cores": rec.get("procs"),
                    "jobs": len(rec["jobs"]), "total_s": rec.get("oracle_wall_s"),
                    "job_s_sum": sum(j.get("oracle_wall_s", 0.0) for j in rec["jobs"])})
    except (OSError, ValueError, KeyError):
        pass
    return out


def cpu_baseline(max_sweeps: int = 1):
    """The oracle, single-threaded, on a bounded sample of the configured workloads: the 2^20-vertex IC
    workload's build Simulate for its first `max_sweeps` sweeps (the full build is ~200 s on one core),
    and the 1000-vertex ER workload's whole run (build and K = 10 greedy steps)."""
    import oracle
    import synth

    w = synth.workload_rmat20()
    g = w.graph
    thr = oracle.edge_thresholds(g, w.model, w.p)
    t0 = time.perf_counter()
    M, sweeps, tl, te = oracle.simulate(g, thr, w.J, max_sweeps=max_sweeps)
    dt = time.perf_counter() - t0
    visits = int(te.sum()) * w.J
    e = synth.workload_er_small()
    ethr = oracle.edge_thresholds(e.graph, e.model, e.p)
    t1 = time.perf_counter()
    res = oracle.greedy(e.graph, ethr, e.J, e.K)
    dt_er = time.perf_counter() - t1
    out = {"value": visits / dt, "unit": "edge·simulation visits/s", "cores": 1, "kind": "oracle",
           "sample": f"{w.name} (n={g.n}, m={g.m}): the build Simulate's first {sweeps} sweeps ({visits} visits) "
                     f"in {dt:.1f} s on one host core",
           "er1000_whole_run_s": dt_er, "er1000_build_visits": res["build_visits"] * e.J,
           "recorded_full_runs": recorded_oracle_runs()}
    out.update(host_cpu())
    return out


def batch_leg(hf, ctx, steps: int, warmup: int):
    """64 independent R-MAT jobs (log2 n uniform in 12..18, average degree uniform in [8, 32], p in
    {0.005, 0.01, 0.05}, R=128, K=20): one persistent graph-captured launch (autotuned decomposition)
    against the same jobs solved one graph per call back-to-back (im_build_sketches + im_select_seeds),
    both from device-resident CSRs.  Every job's seeds must agree between the two."""
    import torch

    import synth

    J, K = 128, 20
    t = time.perf_counter()
    recipe = synth.batch_recipe()
    graphs = [(synth.rmat(scale, draws, seed=seed), p) for scale, draws, p, seed in recipe]
    dev = [(torch.from_numpy(g.xadj).cuda(), torch.from_numpy(g.adj).cuda(), g, p) for g, p in graphs]
    torch.cuda.synchronize()
    n_tot = sum(g.n for g, _ in graphs)
    m_tot = sum(g.m for g, _ in graphs)
    log(f"batch workload: {len(graphs)} graphs, n={n_tot} m={m_tot}, generated in {time.perf_counter() - t:.1f} s")
    jobs = [hf.BatchJob(x, a, g.n, J, K, model="const", p=p) for x, a, g, p in dev]
    t = time.perf_counter()
    b = hf.im_batch_create(ctx, jobs, autotune=True)
    create_s = time.perf_counter() - t
    try:
        for _ in range(warmup):
            b.run()
        runs = [b.run() for _ in range(steps)]
        res = [b.result(i) for i in range(len(jobs))]
        batch_seeds = [list(map(int, r[0])) for r in res]
        build_visits = sum(r[2]["build_visits"] for r in res)
        rebuild_visits = sum(r[2]["rebuild_visits"] for r in res)
        tune = {k: runs[-1][k] for k in ("lanes_per_row", "tile_edges", "heavy_degree", "piece_edges", "workgroups",
                                          "candidates")}
        phases, tiles = runs[-1]["phases"], runs[-1]["tiles"]
    finally:
        b.free()

    def plain_pass():
        out = []
        for x, a, g, p in dev:
            sk = hf.im_build_sketches(ctx, x, a, g.n, J, model="const", p=p)
            try:
                seeds, _, _ = hf.im_select_seeds(sk, K)
            finally:
                sk.free()
            out.append(list(map(int, seeds)))
        return out

    for _ in range(warmup):
        plain_pass()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        plain_seeds = plain_pass()
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t) * 1e3 / steps
    batch_ms = sum(r["wall_ms"] for r in runs) / len(runs)
    batch_dev_ms = sum(r["device_ms"] for r in runs) / len(runs)
    log(f"batched {batch_ms:.1f} ms (device {batch_dev_ms:.1f} ms, {tune}), plain {plain_ms:.1f} ms")
    return {
        "workload": "batch64_rmat_log2n12-18_deg8-32_p{0.005,0.01,0.05}_J128_K20",
        "jobs": len(jobs), "n_total": n_tot, "m_total": m_tot, "R": J, "K": K,
        "batched_ms": batch_ms, "batched_device_ms": batch_dev_ms, "plain_ms": plain_ms,
        "speedup_vs_plain": plain_ms / batch_ms,
        "batched_build_visits_per_s": build_visits * J / (batch_ms * 1e-3),
        "build_visits": build_visits * J, "rebuild_visits": rebuild_visits * J,
        "seeds_equal_to_plain": batch_seeds == plain_seeds,
        "create_s": create_s, "decomposition": tune, "phases": phases, "tiles": tiles,
    }


def _replay(hf, graphs, stream, slots: int, budget_gb: int, max_copies: int = 0):
    """Replays a request stream in real time against a fresh serving engine; latency is
    submit-to-completion and service time build + selection, as the engine measures them."""
    import numpy as np

    sv = hf.Server(0, slots=slots, hbm_budget=budget_gb << 30, max_copies=max_copies)
    try:
        for g in graphs:
            sv.add_graph(g.xadj, g.adj, g.n)
        t0 = time.perf_counter()
        tickets = []
        for i, (arr, gi, model, p, R, K) in enumerate(stream):
            delay = t0 + arr - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tickets.append(sv.submit(gi, R, K, model=model, p=p))
            if (i + 1) % 500 == 0:
                log(f"serving: {i + 1} submitted")
        lat, svc, qms, reused = [], [], [], 0
        for i, tk in enumerate(tickets):
            _, resp = sv.wait(tk)
            lat.append(resp["latency_ms"])
            svc.append(resp["build_ms"] + resp["select_ms"])
            qms.append(resp["queue_ms"])
            reused += resp["sketch_reused"]
            if (i + 1) % 500 == 0:
                log(f"serving: {i + 1} completed")
        wall = time.perf_counter() - t0
        st = sv.stats()
    finally:
        sv.close()
    lat, svc = np.asarray(lat), np.asarray(svc)
    return {
        "requests": len(stream), "offered_req_s": len(stream) / stream[-1][0],
        "throughput_req_s": len(stream) / wall, "wall_s": wall,
        "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
        "latency_ms_mean": float(lat.mean()), "queue_ms_p50": float(np.percentile(qms, 50)),
        "service_ms_p50": float(np.percentile(svc, 50)), "service_ms_p99": float(np.percentile(svc, 99)),
        "sketch_reuse_frac": reused / len(stream), "sketches_built": st["sketches_built"],
        "evictions": st["evictions"], "peak_resident_sketches": st["resident_sketches"],
    }


def serve_leg(hf, n_requests: int, slots: int = 8, budget_gb: int = 200, low_rate: float = 3.0,
              low_requests: int = 60, max_copies: int = 0):
    """Poisson stream (mean 200 requests/s, seed 5) over 16 resident R-MAT graphs (log2 n in 14..22,
    degree 16); each request: IC p=0.01, IC p=0.1 or weighted cascade, R in {64, 256}, K in 10..100.
    The stream is replayed in real time against the library's serving engine under a 200 GB budget.
    The offered load is far above what one GPU sustains, so its latencies are mostly queueing;
    the first low_requests requests of the same recipe at low_rate requests/s (below capacity)
    are replayed as well, on a fresh engine, to report latency without a standing queue."""
    import synth

    t = time.perf_counter()
    pool, stream = synth.serving_recipe(requests=n_requests)
    graphs = [synth.rmat(scale, draws, seed=seed) for scale, draws, seed in pool]
    log(f"serving workload: {len(graphs)} graphs (n={sum(g.n for g in graphs)}, m={sum(g.m for g in graphs)}), "
        f"{len(stream)} requests over {stream[-1][0]:.1f} s, generated in {time.perf_counter() - t:.1f} s")
    out = {"workload": "serve_16rmat_log2n14-22_deg16_poisson200_" + str(n_requests), "slots": slots,
           "max_copies": max_copies or 1, "hbm_budget_gb": budget_gb}
    out.update(_replay(hf, graphs, stream, slots, budget_gb, max_copies))
    if low_requests > 0:
        _, low = synth.serving_recipe(requests=low_requests, rate=low_rate)
        log(f"serving at low load: {len(low)} requests over {low[-1][0]:.1f} s")
        r = _replay(hf, graphs, low, slots, budget_gb, max_copies)
        out["low_load"] = {k: r[k] for k in ("requests", "offered_req_s", "throughput_req_s", "latency_ms_p50",
                                             "latency_ms_p99", "service_ms_p50", "service_ms_p99",
                                             "sketch_reuse_frac")}
    return out


def quality_leg(hf, ctx, eval_R: int = 1024, eval_seed: int = 0x5EED):
    """Seed quality against rebuild policy on the 2^20-vertex R-MAT (IC p = 0.01, R = 256, K = 50):
    error-adaptive rebuild (eps_g = 0.01, eps_l = 0.3) against rebuilding after every step
    (eps = 0) and never rebuilding (eps = inf).  Each seed set is scored by the independent
    Monte-Carlo evaluator on eval_R fresh samples (hash seed eval_seed)."""
    import torch

    import synth

    w = synth.workload_rmat20()
    g = w.graph
    xd = torch.from_numpy(g.xadj).cuda()
    ad = torch.from_numpy(g.adj).cuda()
    sk = hf.im_build_sketches(ctx, xd, ad, g.n, w.J, model=w.model, p=w.p)
    out = {"workload": w.name, "eval_R": eval_R, "eval_hash_seed": eval_seed, "modes": {}}
    try:
        for name, (eg, el) in (("adaptive", (w.eps_g, w.eps_l)), ("always_rebuild", (0.0, 0.0)),
                               ("never_rebuild", (float("inf"), float("inf")))):
            t0 = time.perf_counter()
            seeds, steps, stats = hf.im_select_seeds(sk, w.K, eps_g=eg, eps_l=el)
            sel_ms = (time.perf_counter() - t0) * 1e3
            sigma_eval, _ = hf.im_evaluate_influence(ctx, xd, ad, g.n, seeds, eval_R, model=w.model, p=w.p,
                                                     hash_seed=eval_seed)
            out["modes"][name] = {"sigma_eval": sigma_eval, "sigma_sketch_samples": steps[-1].sigma,
                                  "rebuilds": stats["rebuilds"], "select_ms": sel_ms}
            log(f"quality {name}: sigma {sigma_eval:.1f} (fresh samples), rebuilds {stats['rebuilds']}, "
                f"select {sel_ms:.0f} ms")
    finally:
        sk.free()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat24_wc_J256_K50", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain comparison")
    ap.add_argument("--no-quality", action="store_true", help="skip the rebuild-policy quality comparison")
    ap.add_argument("--serve-slots", type=int, default=8, help="concurrent slots of the serving engine")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving leg and print its object")
    ap.add_argument("--serve-max-copies", type=int, default=0,
                    help="resident copies one sketch key may have in the serving leg (0: the library's default, 1)")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests of the serving leg (the full stream has 2000; 0 skips the leg)")
    ap.add_argument("--K", type=int, default=0, help="override K")
    ap.add_argument("--sparse-div", type=int, default=0)
    ap.add_argument("--heavy-degree", type=int, default=0)
    ap.add_argument("--piece-edges", type=int, default=0)
    ap.add_argument("--dump-sweeps", default="",
                    help="write the sweep log of the last warm-up step (every kernel timed) to this JSON file")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="start with one 1 GiB device copy (the counter calibration of the traffic summary)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print the traffic summary of two rocprofv3 --pmc output folders and exit")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched-vs-plain comparison and print its object (for profiling)")
    args = ap.parse_args()
    if args.summarize_pmc:
        cmd = ("timeout -s KILL 600 rocprofv3 --kernel-trace --pmc {counter} --output-format csv -d {out} -o run "
               "-- python3 bench.py --steps 1 --warmup 0 --no-batch --no-quality --serve-requests 0 "
               "--no-cpu-baseline --calibrate-copy")
        sys.stdout.write(summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], cmd))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this path runs on one GPU: --gpus above 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2105_04023_amd as hf

    if args.batch_only:
        print(json.dumps({"batched": batch_leg(hf, hf.Context(0), args.steps, args.warmup)}), flush=True)
        return
    if args.serve_only:
        print(json.dumps({"serving": serve_leg(hf, args.serve_requests, slots=args.serve_slots,
                                               max_copies=args.serve_max_copies)}), flush=True)
        return
    import synth

    t = time.perf_counter()
    w = WORKLOADS[args.workload](synth)
    g = w.graph
    K = args.K or w.K
    log(f"workload {w.name}: n={g.n} m={g.m} generated in {time.perf_counter() - t:.1f} s")
    deg = np.diff(g.xadj)
    heavy_deg = args.heavy_degree or 64  # the library's default split threshold
    m_heavy = int(deg[deg > heavy_deg].sum())
    xd = torch.from_numpy(g.xadj).cuda()
    ad = torch.from_numpy(g.adj).cuda()
    if args.calibrate_copy:
        a = torch.ones(COPY_BYTES // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    torch.cuda.synchronize()
    ctx = hf.Context(0)

    def step(timed):
        t0 = time.perf_counter()
        sk = hf.im_build_sketches(ctx, xd, ad, g.n, w.J, model=w.model, p=w.p, eps_c=w.eps_c,
                                  sparse_div=args.sparse_div, heavy_degree=args.heavy_degree,
                                  piece_edges=args.piece_edges,
                                  time_sweeps="pieces" if timed else True)
        t1 = time.perf_counter()
        seeds, steps, stats = hf.im_select_seeds(sk, K, eps_g=w.eps_g, eps_l=w.eps_l)
        t2 = time.perf_counter()
        info = sk.info()
        swl = sk.sweep_log()
        sk.free()
        return {"build_s": t1 - t0, "select_s": t2 - t1, "info": info, "stats": stats, "seeds": list(map(int, seeds)),
                "sweep_log": swl, "sigma": steps[-1].sigma}

    warm_log = []  # every kernel of every sweep timed, in the last warm-up step
    for i in range(args.warmup):
        r = step(False)
        warm_log = r["sweep_log"]
        log(f"warmup {i}: build {r['build_s'] * 1e3:.1f} ms select {r['select_s'] * 1e3:.1f} ms "
            f"sweeps {r['info']['sweeps']} rebuilds {r['stats']['rebuilds']}")
    torch.cuda.synchronize()
    results = []
    tstart = time.perf_counter()
    for i in range(args.steps):
        r = step(True)
        results.append(r)
        log(f"step {i}: build {r['build_s'] * 1e3:.1f} ms select {r['select_s'] * 1e3:.1f} ms "
            f"sweeps {r['info']['sweeps']} rebuilds {r['stats']['rebuilds']} sigma {r['sigma']:.1f}")
    torch.cuda.synchronize()
    total_s = time.perf_counter() - tstart

    J = w.J
    visits = sum(r["info"]["visits"] for r in results) * J
    build_s = sum(r["build_s"] for r in results)
    select_s = sum(r["select_s"] for r in results)
    sim_ms = sum(r["info"]["build_ms"] for r in results)
    # roofline of the dominant kernel (the split-row piece kernel) over every timed launch
    # of the timed steps (build and rebuild sweeps, including launches past the stopping rule)
    recs = [rec for r in results for rec in r["sweep_log"]]
    wc = w.model == "wc"
    npieces = results[-1]["info"]["heavy_pieces"]
    assert results[-1]["info"]["heavy_rows"] == int((deg > heavy_deg).sum()), "split threshold mismatch"
    tot_bytes = sum(heavy_launch_bytes(rec, J, wc, m_heavy, npieces) for rec in recs)
    tot_visit_bytes = sum(heavy_launch_visit_bytes(rec, J, wc, m_heavy, npieces) for rec in recs)
    heavy_visits = sum(rec["visits"] - rec["light_visits"] for rec in recs if rec["ran"])
    heavy_merged = sum(rec["merged"] - rec["light_merged"] for rec in recs if rec["ran"])
    tot_ms = sum(rec["heavy_ms"] for rec in recs)
    nlaunch = len(recs)
    achieved = tot_bytes / (tot_ms * 1e-3) / 1e9 if tot_ms > 0 else 0.0
    # the row kernel, from the warm-up step's full sweep timing (the timed steps record only the
    # piece kernel's events, two per sweep instead of six)
    row_ms = sum(rec["kernel_ms"] for rec in warm_log)
    row_bytes = sum(rec["light_visits"] * 4 + rec["light_merged"] * (J + (4 if wc else 0))
                    for rec in warm_log if rec["ran"])
    out = {
        "metric": "edge\u00b7simulation visits/s in sketch build + K=50 IM time, batched vs plain",
        "value": visits / build_s,
        "unit": "edge\u00b7simulation visits/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_s * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": w.name, "n": g.n, "m": g.m, "R": J, "K": K, "model": w.model, "p": w.p,
                   "eps_g": w.eps_g, "eps_l": w.eps_l, "eps_c": w.eps_c, "hash_seed": w.hash_seed},
        "im_time_ms": select_s * 1e3 / args.steps,
        "build_ms": build_s * 1e3 / args.steps,
        "simulate_device_ms": sim_ms / args.steps,
        "visits_per_step": visits // args.steps,
        "sweeps": results[-1]["info"]["sweeps"],
        "rebuilds": results[-1]["stats"]["rebuilds"],
        "rebuild_sweeps": results[-1]["stats"]["rebuild_sweeps"],
        "bfs_levels": results[-1]["stats"]["bfs_levels"],
        "sigma": results[-1]["sigma"],
        "seeds_head": results[-1]["seeds"][:8],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(), "traffic_unit": "bytes/launch",
                     "kernel": "k_sweep_heavy",
                     "launches": nlaunch, "avg_launch_ms": tot_ms / max(nlaunch, 1),
                     "algorithmic_bytes_per_launch": tot_bytes / max(nlaunch, 1),
                     # the same launches priced per visited edge (every visit's row charged)
                     "visit_model_bytes_per_launch": tot_visit_bytes / max(nlaunch, 1),
                     "frac_visit_model": (tot_visit_bytes / (tot_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
                                          if tot_ms > 0 else 0.0),
                     "heavy_edge_visits_per_step": heavy_visits // args.steps,
                     "heavy_edges_merged_per_step": heavy_merged // args.steps},
        "row_kernel": ({"kernel": "k_sweep_rows64", "ms_per_step": row_ms, "measured_on": "warm-up step",
                        "visit_bytes_GBs": row_bytes / (row_ms * 1e-3) / 1e9}
                       if row_ms > 0 else None),
    }
    if not args.no_batch:
        out["batched"] = batch_leg(hf, ctx, args.steps, args.warmup)
    if args.serve_requests > 0:
        out["serving"] = serve_leg(hf, args.serve_requests, slots=args.serve_slots, max_copies=args.serve_max_copies)
    if not args.no_quality:
        out["quality"] = quality_leg(hf, ctx)
    if args.dump_sweeps:
        with open(args.dump_sweeps, "w") as fh:
            json.dump(warm_log or results[-1]["sweep_log"], fh)
    if not args.no_cpu_baseline:
        log("timing the oracle on the CPU sample")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
