"""Brute-force references for tiny graphs, independent of the oracle's Simulate/greedy code.

Each sample graph G_j is materialised explicitly: edge (u, v) is in G_j when the
oracle's (separately pinned) live predicate says so.  Reachability then comes from
networkx, so the propagation, blocking, reach and greedy logic are checked against
plain graph search rather than against themselves.
"""
from __future__ import annotations

import networkx as nx
import numpy as np

import oracle


def sample_graphs(graph, thr, J, seed=0):
    """List of J networkx DiGraphs, G_j = live edges of sample j (Eq. hash_prob)."""
    X = [oracle.sim_word(j, seed) for j in range(J)]
    gs = [nx.DiGraph() for _ in range(J)]
    for g in gs:
        g.add_nodes_from(range(graph.n))
    for u in range(graph.n):
        for e in range(graph.xadj[u], graph.xadj[u + 1]):
            v = int(graph.adj[e])
            h = oracle.edge_hash(u, v, seed)
            for j in range(J):
                if oracle.live(h, X[j], int(thr[e])):
                    gs[j].add_edge(u, v)
    return gs


def ranks(n, J, seed=0):
    return np.array([[oracle.rank(v, j, seed) for j in range(J)] for v in range(n)], dtype=np.int64)


def reach_sets(gs, sources):
    """Per sample j: the set of vertices reachable from `sources` (sources included)."""
    out = []
    for g in gs:
        r = set()
        for s in sources:
            r |= {s} | nx.descendants(g, s)
        out.append(r)
    return out


def fixed_point(gs, rk, blocked=None):
    """M[u][j] = max rank over the vertices u reaches in G_j through unblocked vertices; 0 if u is blocked.

    When the blocked set is the reach of a seed set (closed under live edges) this is
    the reach of u in G_j minus the reach of S.
    """
    n, J = rk.shape
    M = np.zeros((n, J), dtype=np.int64)
    for j, g in enumerate(gs):
        bl = blocked[j] if blocked is not None else set()
        h = g.subgraph([v for v in range(n) if v not in bl])
        for u in range(n):
            if u in bl:
                continue
            rs = {u} | nx.descendants(h, u)
            M[u, j] = max(rk[w, j] for w in rs)
    return M


def hop_state(gs, rk, t, blocked=None):
    """Registers after t synchronous sweeps: max rank over vertices within <= t live hops (residual graph)."""
    n, J = rk.shape
    M = np.zeros((n, J), dtype=np.int64)
    for j, g in enumerate(gs):
        bl = blocked[j] if blocked is not None else set()
        h = g.subgraph([v for v in range(n) if v not in bl])
        for u in range(n):
            if u in bl:
                continue
            d = nx.single_source_shortest_path_length(h, u, cutoff=t)
            M[u, j] = max(rk[w, j] for w in d)
    return M
