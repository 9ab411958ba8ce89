"""Pins of the CPU oracle against facts fixed outside it.

Each test checks the oracle against something it does not compute itself: published
hash test values, exact rational arithmetic, closed-form distributions, brute-force graph
search on the explicit sample graphs, or the worked example of the paper's Fig.
(hf-processing).  A plausible slip in the oracle (a dropped term, a wrong index, an
in-place instead of synchronous sweep, a missing block) fails at least one of them.
"""
from __future__ import annotations

import math
import os
import struct
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle
import synth
from tests import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def f32(x: float) -> float:
    return struct.unpack("<f", struct.pack("<f", x))[0]


# ---------------------------------------------------------------- Murmur3 (Eq. hash)

def _golden_murmur():
    rows = []
    with open(os.path.join(GOLDEN, "murmur3_x86_32_vectors.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            key, seed, h = line.rstrip("\n").split("\t")
            key = b"" if key == '""' else key.replace("\\0", "\0").encode()
            rows.append((key, int(seed, 16), int(h, 16)))
    return rows


def test_murmur3_published_vectors():
    rows = _golden_murmur()
    assert len(rows) == 8
    for key, seed, h in rows:
        assert oracle.murmur3_32(key, seed) == h, (key, seed)


def test_edge_hash_is_31_bit_murmur_of_concatenation():
    # Eq. (hash): Murmur3(u || v) mod 2^31, u and v as little-endian 32-bit words.
    for u, v, seed in [(0, 0, 0), (1, 2, 0), (123456, 7, 99), (2**31 - 1, 5, 3)]:
        full = oracle.murmur3_32(struct.pack("<II", u, v), seed)
        assert oracle.edge_hash(u, v, seed) == full % 2**31
        assert oracle.edge_hash(u, v, seed) < 2**31


def test_sim_word_and_rank_definitions():
    for j in range(5):
        assert oracle.sim_word(j, 7) == oracle.murmur3_32(struct.pack("<I", j), 9) % 2**31
    for v, j in [(0, 0), (5, 3), (999, 63)]:
        x = oracle.murmur3_32(struct.pack("<I", v), 1) ^ oracle.murmur3_32(struct.pack("<I", j), 3)
        expect = 32 if x == 0 else 32 - x.bit_length()
        assert oracle.rank(v, j, 0) == expect


# ---------------------------------------------------------------- thresholds (Eq. hash_prob)

def _exact_thr(w: float) -> int:
    # #{integers x >= 0 : x < w * h_max} = ceil(w * h_max)
    return math.ceil(Fraction(w) * (2**31 - 1))


def test_threshold_matches_exact_rational():
    rng = np.random.default_rng(0)
    bits = rng.integers(0, 0x3F800001, size=4000, dtype=np.uint32)  # all binary32 in [0, 1]
    ws = [float(x) for x in bits.view(np.float32)]
    ws += [0.0, 1.0, f32(0.005), f32(0.01), f32(0.1), f32(0.05), 1.4e-45, f32(1.0 - 2**-24)]
    ws += [f32(1.0 / d) for d in range(1, 200)]
    for w in ws:
        assert oracle.threshold(w) == _exact_thr(w), w


def test_threshold_rejects_out_of_range():
    for w in [-1e-30, 1.0000001, float("nan"), float("inf")]:
        assert oracle.threshold(w) == 0xFFFFFFFF


def test_live_rule_boundaries():
    # live iff (X xor h) / h_max < w: the largest live XOR value is thr - 1.
    thr = oracle.threshold(f32(0.25))
    assert oracle.live(thr - 1, 0, thr) and not oracle.live(thr, 0, thr)
    assert not oracle.live(0, 0, oracle.threshold(0.0))  # w = 0: never live
    # w = 1: every XOR value except h_max itself is live (strict "<")
    t1 = oracle.threshold(1.0)
    assert oracle.live(2**31 - 2, 0, t1) and not oracle.live(2**31 - 1, 0, t1)


# ---------------------------------------------------------------- statistical pins of sampling

def _xor_values(num_edges=4000, J=256, seed=0):
    X = np.array([oracle.sim_word(j, seed) for j in range(J)], dtype=np.uint64)
    rng = np.random.default_rng(1)
    uv = rng.integers(0, 1 << 24, size=(num_edges, 2))
    H = np.array([oracle.edge_hash(int(u), int(v), seed) for u, v in uv], dtype=np.uint64)
    return H[:, None] ^ X[None, :]


def test_hash_prob_is_uniform_ks():
    # Fig. (prob-cdf) analogue: P(u,v)_r = (X_r xor h)/h_max is close to U[0, 1].
    P = (_xor_values(3000).astype(np.float64) / (2**31 - 1)).ravel()
    res = stats.kstest(P, "uniform")
    assert res.pvalue > 1e-4, res


@pytest.mark.parametrize("w", [0.005, 0.01, 0.1, 0.5])
def test_live_fraction_matches_weight(w):
    V = _xor_values(3000)
    thr = oracle.threshold(f32(w))
    frac = float((V < thr).mean())
    N = V.size
    sd = math.sqrt(w * (1 - w) / N)
    assert abs(frac - w) < 5 * sd + 1e-6, (frac, w)


def test_capture_rate_in_256_samples():
    # Sec. 4.4: at w = 0.005 an edge is live in at least one of 256 samples with
    # probability 1 - (1 - 0.005)^256 = 0.72.
    V = _xor_values(6000, J=256)
    thr = oracle.threshold(f32(0.005))
    cap = float((V < thr).any(axis=1).mean())
    p = 1 - (1 - 0.005) ** 256
    assert abs(p - 0.7228) < 1e-4
    sd = math.sqrt(p * (1 - p) / V.shape[0])
    assert abs(cap - p) < 5 * sd, (cap, p)


def test_weighted_cascade_activation_probability():
    # Sec. 2.1 (WC): with l active in-neighbours, v activates with probability 1 - (1 - 1/d_v)^l.
    d, ell = 5, 3
    n = d + 1
    g = synth.from_edges(n, [(u, d) for u in range(d)])  # v = d has in-degree d
    thr = oracle.edge_thresholds(g, "wc")
    assert all(int(t) == oracle.threshold(f32(1.0 / d)) for t in thr)
    J = 4096
    X = np.array([oracle.sim_word(j, 0) for j in range(J)], dtype=np.uint64)
    H = np.array([oracle.edge_hash(u, d, 0) for u in range(ell)], dtype=np.uint64)
    act = ((H[:, None] ^ X[None, :]) < np.uint64(thr[0])).any(axis=0).mean()
    p = 1 - (1 - 1 / d) ** ell
    assert abs(act - p) < 5 * math.sqrt(p * (1 - p) / J)


def test_rank_distribution_geometric():
    # Eq. (sketch-add): a leading-zero count of a uniform word has P(rank = k) = 2^-(k+1).
    vs = np.arange(3000)
    R = np.array([[oracle.rank(int(v), j, 0) for j in range(64)] for v in vs]).ravel()
    K = 12
    obs = np.bincount(np.minimum(R, K), minlength=K + 1)
    exp = np.array([2.0 ** -(k + 1) for k in range(K)] + [2.0 ** -K]) * R.size
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert chi2 < stats.chi2.ppf(0.9999, K), (obs, exp)


# ---------------------------------------------------------------- Simulate (Alg. 2) vs brute force

def _tiny_graphs():
    out = []
    for i, (n, m) in enumerate([(12, 30), (20, 60), (30, 120), (25, 40)]):
        out.append(synth.erdos_renyi(n, m, seed=100 + i))
    out.append(synth.rmat(5, 160, seed=7))
    # a long directed path plus a cycle: stresses iteration counts
    out.append(synth.from_edges(16, [(i, i + 1) for i in range(15)] + [(15, 8), (3, 0)]))
    return out


@pytest.mark.parametrize("gi", range(6))
@pytest.mark.parametrize("model,p,J", [("const", 0.3, 8), ("const", 0.9, 4), ("wc", 0.0, 16), ("const", 0.05, 64)])
def test_simulate_fixed_point_equals_bruteforce_reach(gi, model, p, J):
    g = _tiny_graphs()[gi]
    thr = oracle.edge_thresholds(g, model, f32(p))
    M, sweeps, tl, te = oracle.simulate(g, thr, J)
    gs = bf.sample_graphs(g, thr, J)
    rk = bf.ranks(g.n, J)
    assert np.array_equal(M.astype(np.int64), bf.fixed_point(gs, rk))


@pytest.mark.parametrize("gi", [0, 2, 4, 5])
def test_simulate_with_blocked_pairs(gi):
    g = _tiny_graphs()[gi]
    J = 8
    thr = oracle.edge_thresholds(g, "const", f32(0.4))
    gs = bf.sample_graphs(g, thr, J)
    rk = bf.ranks(g.n, J)
    rng = np.random.default_rng(gi)
    # (a) blocked = reach of a seed set (what Alg. 1 passes); (b) an arbitrary blocked pattern
    S = [int(x) for x in rng.choice(g.n, 2, replace=False)]
    reach = bf.reach_sets(gs, S)
    arb = [set(int(x) for x in np.nonzero(rng.random(g.n) < 0.3)[0]) for _ in range(J)]
    for blocked in (reach, arb):
        blk = np.zeros((g.n, J), dtype=np.uint8)
        for j, b in enumerate(blocked):
            for v in b:
                blk[v, j] = 1
        M, *_ = oracle.simulate(g, thr, J, blk=blk)
        assert np.array_equal(M.astype(np.int64), bf.fixed_point(gs, rk, blocked))


@pytest.mark.parametrize("gi", [1, 4, 5])
def test_sweep_states_counts_and_traces(gi):
    """Synchronous sweeps: after t sweeps a register holds the max rank within t live hops.

    The sweep count is 1 + the last sweep that changes a register, |L_t| counts the
    vertices whose rows changed in sweep t-1, and the edge trace counts edges whose head
    is in L_t.
    """
    g = _tiny_graphs()[gi]
    J = 8
    thr = oracle.edge_thresholds(g, "const", f32(0.5))
    gs = bf.sample_graphs(g, thr, J)
    rk = bf.ranks(g.n, J)
    M, sweeps, tl, te = oracle.simulate(g, thr, J)
    states = [bf.hop_state(gs, rk, t) for t in range(sweeps + 1)]
    for t in range(sweeps + 1):
        Mt, *_ = oracle.simulate(g, thr, J, max_sweeps=t)
        assert np.array_equal(Mt.astype(np.int64), states[t]), t
    last_change = max([t for t in range(1, sweeps + 1) if not np.array_equal(states[t], states[t - 1])], default=0)
    assert sweeps == last_change + 1
    assert tl[0] == g.n
    for t in range(1, sweeps + 1):
        changed = (states[t] != states[t - 1]).any(axis=1)
        assert tl[t] == changed.sum()
    Lsets = [np.ones(g.n, bool)] + [(states[t] != states[t - 1]).any(axis=1) for t in range(1, sweeps + 1)]
    for t in range(sweeps):
        assert te[t] == int(Lsets[t][g.adj].sum())
    assert tl[sweeps] == 0
    # iteration bound: at most the largest sample diameter (in hops) + 1 detection sweep
    import networkx as nx
    dmax = 0
    for h in gs:
        for u in range(g.n):
            d = nx.single_source_shortest_path_length(h, u)
            dmax = max(dmax, max(d.values()))
    assert sweeps <= dmax + 1


def _bf_blocked_trace(g, gs, rk, blocked):
    """Sweep count, |L_t| and edge-visit traces of Simulate on the residual graph, from the brute-force
    sweep states: L_0 = V, L_t = rows changed by sweep t-1, and sweep t visits the edges (u, v) with v in
    L_t whose source u is not blocked in every sample (reading 11: such a row holds zeros and cannot
    change, so its edges are not visited)."""
    J = len(gs)
    full = np.array([all(u in blocked[j] for j in range(J)) for u in range(g.n)])
    states = [bf.hop_state(gs, rk, 0, blocked)]
    while True:
        states.append(bf.hop_state(gs, rk, len(states), blocked))
        if np.array_equal(states[-1], states[-2]):
            break
    sweeps = len(states) - 1  # the last sweep changes nothing and detects the fixed point
    L = [np.ones(g.n, bool)] + [(states[t] != states[t - 1]).any(axis=1) for t in range(1, sweeps + 1)]
    src = np.repeat(np.arange(g.n), np.diff(g.xadj))
    te = [int((L[t][g.adj] & ~full[src]).sum()) for t in range(sweeps)]
    return sweeps, [int(x.sum()) for x in L], te, states[-1]


@pytest.mark.parametrize("gi", [0, 2, 4, 5])
def test_edge_trace_under_blocking(gi):
    """Reading 11 on Simulate(blocked): with (a) the reach of a seed set, whose seeds are blocked in every
    sample, and (b) an arbitrary pattern with some vertices blocked in every sample, the sweep count, the
    |L_t| trace and the per-sweep edge visits equal their definitions on the brute-force sweep states."""
    g = _tiny_graphs()[gi]
    J = 8
    thr = oracle.edge_thresholds(g, "const", f32(0.45))
    gs = bf.sample_graphs(g, thr, J)
    rk = bf.ranks(g.n, J)
    rng = np.random.default_rng(50 + gi)
    S = [int(x) for x in rng.choice(g.n, 2, replace=False)]
    arb = [set(int(x) for x in np.nonzero(rng.random(g.n) < 0.25)[0]) for _ in range(J)]
    everywhere = [int(x) for x in rng.choice(g.n, 3, replace=False)]
    for b in arb:
        b.update(everywhere)
    for blocked in (bf.reach_sets(gs, S), arb):
        blk = np.zeros((g.n, J), dtype=np.uint8)
        for j, b in enumerate(blocked):
            for v in b:
                blk[v, j] = 1
        assert blk.all(axis=1).any()  # reading 11 is exercised
        M, sweeps, tl, te = oracle.simulate(g, thr, J, blk=blk)
        bsw, btl, bte, bM = _bf_blocked_trace(g, gs, rk, blocked)
        assert sweeps == bsw
        assert list(tl) == btl
        assert list(te) == bte
        assert np.array_equal(M.astype(np.int64), bM)
        # the unblocked count differs whenever a fully blocked row has an out-edge into L_0 = V
        src_full = blk.all(axis=1)[np.repeat(np.arange(g.n), np.diff(g.xadj))]
        if src_full.any():
            assert te[0] == g.m - int(src_full.sum())


@pytest.mark.parametrize("gi,model,p", [(1, "const", 0.3), (4, "const", 0.2), (2, "wc", 0.0)])
def test_rebuild_visits_and_sweeps(gi, model, p):
    """Always-rebuild greedy: each step's rebuild runs Simulate on the residual graph of the seeds so far;
    its sweep count and its edge visits (summed over its sweeps, reading 11) equal the brute-force ones."""
    g = _tiny_graphs()[gi]
    J, K = 8, 5
    thr = oracle.edge_thresholds(g, model, f32(p))
    gs = bf.sample_graphs(g, thr, J)
    rk = bf.ranks(g.n, J)
    res = oracle.greedy(g, thr, J, K, eps_g=0.0, eps_l=0.0)
    _, bsw0, _, bte0, _ = (None,) + _bf_blocked_trace(g, gs, rk, [set() for _ in range(J)])
    assert res["build_sweeps"] == bsw0 and res["build_visits"] == sum(bte0)
    for k in range(K - 1):
        st = res["steps"][k]
        bsw, _, bte, _ = _bf_blocked_trace(g, gs, rk, bf.reach_sets(gs, res["seeds"][: k + 1]))
        assert st["rebuilt"] == 1
        assert st["sweeps"] == bsw, k
        assert st["visits"] == sum(bte), k


def test_early_exit_threshold():
    # eps_c: stop as soon as |L| <= eps_c * n (Sec. 3.2).
    g = _tiny_graphs()[5]
    thr = oracle.edge_thresholds(g, "const", f32(0.9))
    _, sweeps_full, tl, _ = oracle.simulate(g, thr, 4)
    eps = (tl[2] + 0.5) / g.n  # first t with |L_t| <= eps*n is t = 2 (or earlier)
    _, sw, tl2, _ = oracle.simulate(g, thr, 4, eps_c=eps)
    first = min(t for t in range(len(tl)) if tl[t] <= eps * g.n)
    assert sw == first <= sweeps_full


def test_worked_example_live_set_sequence():
    """Fig. (hf-processing): two simulations on a 4-vertex toy graph.

    Edge (1,4) is live in both simulations, edge (4,3) only in the second, and vertex 3's
    second register is 5; the live sets are {1,4} after the first iteration and {1} after
    the second, then nothing changes.  The figure image is missing, so the remaining register
    values are not pinned; a hash seed and per-edge weights are searched that realise
    the narrated conditions (vertices 1..4 are ids 0..3, simulations 1, 2 are j = 0, 1).
    """
    edges = [(0, 3), (3, 2), (1, 0), (2, 1), (1, 2), (0, 1)]
    g = synth.from_edges(4, edges)
    order = {(int(u), int(g.adj[e])): e for u in range(4) for e in range(g.xadj[u], g.xadj[u + 1])}
    found = None
    for seed in range(5000):
        r = [[oracle.rank(v, j, seed) for j in range(2)] for v in range(4)]
        if not (r[2][1] == 5 and r[3][1] < 5 and r[0][1] < 5):
            continue
        if not any(r[3][j] > r[0][j] for j in range(2)):
            continue
        x0, x1 = oracle.sim_word(0, seed), oracle.sim_word(1, seed)
        h = oracle.edge_hash(3, 2, seed)
        lo, hi = x1 ^ h, x0 ^ h  # need lo < thr <= hi
        if hi - lo < 1000:
            continue
        if (x0 ^ oracle.edge_hash(0, 3, seed)) == 2**31 - 1 or (x1 ^ oracle.edge_hash(0, 3, seed)) == 2**31 - 1:
            continue
        w43 = f32(((lo + hi) / 2) / (2**31 - 1))
        t43 = oracle.threshold(w43)
        if not (lo < t43 <= hi):
            continue
        found = (seed, w43)
        break
    assert found is not None
    seed, w43 = found
    w = np.zeros(len(g.adj), dtype=np.float32)
    w[order[(0, 3)]] = 1.0
    w[order[(3, 2)]] = w43
    thr = oracle.edge_thresholds(g, "edge", per_edge=w)
    M, sweeps, tl, te = oracle.simulate(g, thr, 2, seed=seed)
    M1, *_ = oracle.simulate(g, thr, 2, seed=seed, max_sweeps=1)
    M0, *_ = oracle.simulate(g, thr, 2, seed=seed, max_sweeps=0)
    changed1 = {v for v in range(4) if (M1[v] != M0[v]).any()}
    assert changed1 == {0, 3}
    assert M1[3, 1] == 5
    M2, *_ = oracle.simulate(g, thr, 2, seed=seed, max_sweeps=2)
    assert {v for v in range(4) if (M2[v] != M1[v]).any()} == {0}
    assert M2[0, 1] == 5
    assert sweeps == 3 and list(tl) == [4, 2, 1, 0]


# ---------------------------------------------------------------- estimate (Eq. sketch-estimate)

def test_estimate_matches_high_precision_value():
    getcontext().prec = 50
    rng = np.random.default_rng(3)
    for J in [4, 64, 100, 256, 1024]:
        for _ in range(30):
            row = rng.integers(0, 33, size=J).astype(np.uint8)
            s = int(row.sum())
            exact = (Decimal(2) ** (Decimal(s) / Decimal(J))) / Decimal("0.77351")
            got = oracle.estimate(row)
            assert abs(Decimal(got) - exact) / exact < Decimal("4e-16"), (J, s)
    assert oracle.estimate(np.zeros(8, np.uint8)) == 1 / 0.77351


def test_register_mean_matches_closed_form():
    """For a fixed set of c vertices, a register is the max of c geometric ranks:
    P(M <= k) = (1 - 2^-(k+1))^c, so E[M] = sum_{k>=1} 1 - (1 - 2^-k)^c.  The mean over
    J = 256 registers of the oracle's ranks must match it within the sampling error, and
    the estimate 2^mean / phi is then about 1.63 c (the estimator's bias as printed)."""
    c, J, trials = 1000, 256, 12
    rk = np.array([[oracle.rank(v, j, 0) for j in range(J)] for v in range(c * trials)], dtype=np.int64)
    means = [rk[t * c:(t + 1) * c].max(axis=0).mean() for t in range(trials)]
    ks = np.arange(0, 34)
    cdf = (1 - 2.0 ** -(ks + 1)) ** c
    pmf = np.diff(np.concatenate([[0.0], cdf]))
    EM = float((ks * pmf).sum())
    VarM = float((ks ** 2 * pmf).sum() - EM ** 2)
    assert abs(EM - 10.299) < 0.01
    sd_mean = math.sqrt(VarM / J / trials)
    assert abs(np.mean(means) - EM) < 5 * sd_mean, (np.mean(means), EM)
    assert abs(np.std(means, ddof=1) - math.sqrt(VarM / J)) < 0.6 * math.sqrt(VarM / J)
    ratio = 2 ** EM / 0.77351 / c
    assert 1.55 < ratio < 1.70


# ---------------------------------------------------------------- reach and greedy (Alg. 1)

@pytest.mark.parametrize("gi", [0, 2, 4])
def test_reach_add_equals_bfs(gi):
    g = _tiny_graphs()[gi]
    J = 16
    thr = oracle.edge_thresholds(g, "const", f32(0.3))
    gs = bf.sample_graphs(g, thr, J)
    blk = np.zeros((g.n, J), dtype=np.uint8)
    total = 0
    S = []
    for s in [0, 3, 7]:
        S.append(s)
        total += oracle.reach_add(g, thr, J, 0, blk, s)
        reach = bf.reach_sets(gs, S)
        expect = np.zeros_like(blk)
        for j, r in enumerate(reach):
            for v in r:
                expect[v, j] = 1
        assert np.array_equal(blk, expect)
        assert total == int(expect.sum())


def _bf_gain_registers(gs, rk, S):
    reach = bf.reach_sets(gs, S) if S else [set() for _ in gs]
    return bf.fixed_point(gs, rk, reach), reach


@pytest.mark.parametrize("gi,model,p", [(1, "const", 0.3), (4, "const", 0.2), (2, "wc", 0.0)])
def test_greedy_always_rebuild_is_exact_marginal_sketch_argmax(gi, model, p):
    """eps_l = eps_g = 0 rebuilds after every seed (Sec. 3.2.1).  Then each seed is the
    argmax over v not in S of sum_j max rank over Reach_j(v) minus Reach_j(S), lowest id
    on ties, and sigma is the exact mean reach of S over the samples."""
    g = _tiny_graphs()[gi]
    J, K = 8, 5
    thr = oracle.edge_thresholds(g, model, f32(p))
    gs = bf.sample_graphs(g, thr, J)
    rk = bf.ranks(g.n, J)
    res = oracle.greedy(g, thr, J, K, eps_g=0.0, eps_l=0.0)
    S = []
    for k in range(K):
        Mg, _ = _bf_gain_registers(gs, rk, S)
        score = Mg.sum(axis=1)
        score[S] = -1
        s = int(np.argmax(score))  # numpy argmax returns the first (lowest id) maximum
        assert res["seeds"][k] == s, k
        st = res["steps"][k]
        assert st["score"] == score[s]
        assert st["e"] == pytest.approx(2 ** (score[s] / J) / 0.77351, rel=1e-12)
        S.append(s)
        reach = bf.reach_sets(gs, S)
        R = sum(len(r) for r in reach)
        assert st["reach"] == R
        assert st["sigma"] == R / J
        assert st["rebuilt"] == (1 if k < K - 1 else 0)
    assert np.array_equal(res["M"].astype(np.int64), _bf_gain_registers(gs, rk, S[:-1])[0])


def test_greedy_never_rebuild_uses_merged_seed_registers():
    """eps = infinity never rebuilds: scores use max(M_S', M_v) over the initial registers."""
    g = _tiny_graphs()[4]
    J, K = 16, 6
    thr = oracle.edge_thresholds(g, "const", f32(0.25))
    gs = bf.sample_graphs(g, thr, J)
    rk = bf.ranks(g.n, J)
    M0 = bf.fixed_point(gs, rk)
    res = oracle.greedy(g, thr, J, K, eps_g=math.inf, eps_l=math.inf)
    MS = np.zeros(J, dtype=np.int64)
    S = []
    for k in range(K):
        sc = np.maximum(MS[None, :], M0).sum(axis=1)
        sc[S] = -1
        s = int(np.argmax(sc))
        assert res["seeds"][k] == s
        assert res["steps"][k]["rebuilt"] == 0
        MS = np.maximum(MS, M0[s])
        S.append(s)
    assert np.array_equal(res["M"].astype(np.int64), M0)


def test_greedy_error_adaptive_decisions():
    """Default thresholds: sigma and delta from brute-force reach counts, e from the registers
    of the brute-force sketch in force at each step, and a rebuild exactly when neither
    error is below its threshold (steps 1..K-1)."""
    g = synth.erdos_renyi(50, 250, seed=14)
    J, K = 16, 8
    thr = oracle.edge_thresholds(g, "const", f32(0.4))
    gs = bf.sample_graphs(g, thr, J)
    rk = bf.ranks(g.n, J)
    res = oracle.greedy(g, thr, J, K, eps_g=0.01, eps_l=0.3)
    S, MS, last_S, R_last = [], np.zeros(J, np.int64), [], 0
    M = bf.fixed_point(gs, rk)
    for k in range(K):
        st = res["steps"][k]
        s = st["seed"]
        merged = np.maximum(MS, M[s])
        assert st["e"] == pytest.approx(2 ** (merged.sum() / J) / 0.77351, rel=1e-12)
        S.append(s)
        R = sum(len(r) for r in bf.reach_sets(gs, S))
        sigma, delta = R / J, (R - R_last) / J
        assert st["sigma"] == sigma and st["delta"] == delta
        fresh = (abs((st["e"] - delta) / delta) < 0.3 if delta else False) or abs((st["e"] - delta) / sigma) < 0.01
        assert st["fresh"] == int(fresh)
        if k < K - 1 and not fresh:
            assert st["rebuilt"] == 1
            M = bf.fixed_point(gs, rk, bf.reach_sets(gs, S))
            MS = np.zeros(J, np.int64)
            R_last = R
        else:
            assert st["rebuilt"] == 0
            if k < K - 1:
                MS = merged
    assert any(s["rebuilt"] for s in res["steps"]) and any(s["fresh"] for s in res["steps"][:-1])


def test_greedy_observer_sees_completed_previous_steps():
    """The observer of a run gets, from step 2 on, the record of the step before as the finished
    run reports it (rebuild flag, sweep and visit counts included), and each step's own record
    before its rebuild; a run stopped by the observer after step k reports the first k steps of
    the full run, the last without a rebuild."""
    g = synth.erdos_renyi(50, 250, seed=14)
    J, K = 16, 8
    thr = oracle.edge_thresholds(g, "const", f32(0.4))
    full = oracle.greedy(g, thr, J, K, eps_g=0.01, eps_l=0.3)
    assert any(s["rebuilt"] for s in full["steps"][:-1])
    seen = {}

    def obs(k, M, blk, st, tl, te):
        if k >= 1:
            seen[k] = dict(st)
        return k == 5

    part = oracle.greedy(g, thr, J, K, eps_g=0.01, eps_l=0.3, observer=obs)
    assert part["stopped_after"] == 5
    for k in range(2, 6):
        assert seen[k]["previous"] == full["steps"][k - 2], k
    for k in range(1, 6):
        own = {f: v for f, v in seen[k].items() if f != "previous"}
        assert own == dict(full["steps"][k - 1], rebuilt=0, sweeps=0, visits=0), k
    assert part["steps"][:4] == full["steps"][:4]
    assert part["steps"][4] == dict(full["steps"][4], rebuilt=0, sweeps=0, visits=0)
