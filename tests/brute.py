"""Brute-force references written straight from the paper's definitions.

Pure Python / numpy, for tiny graphs only.  They share nothing with the oracle
or the GPU library; tests use them to pin both.

* clique_degrees  -- Definition 3 by testing every h-subset of vertices.
* core_fixpoint   -- Definition 6: R_k is what remains after repeatedly
                     deleting vertices whose clique-degree (Definition 3, in
                     the current subgraph) is below k; core(v) = max k with v in R_k.
* densest         -- Problem 1 by trying every non-empty vertex subset.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def adjacency_sets(n, edges):
    adj = [set() for _ in range(n)]
    for u, v in edges:
        u, v = int(u), int(v)
        if u != v:
            adj[u].add(v)
            adj[v].add(u)
    return adj


def cliques(n, edges, h, vertices=None):
    adj = adjacency_sets(n, edges)
    vs = sorted(range(n) if vertices is None else vertices)
    out = []
    for S in itertools.combinations(vs, h):
        if all(b in adj[a] for a, b in itertools.combinations(S, 2)):
            out.append(S)
    return out


def clique_degrees(n, edges, h, vertices=None):
    deg = [0] * n
    cl = cliques(n, edges, h, vertices)
    for S in cl:
        for v in S:
            deg[v] += 1
    return deg, len(cl)


def core_fixpoint(n, edges, h):
    core = [0] * n
    k = 0
    while True:
        alive = set(range(n))
        while True:
            deg, _ = clique_degrees(n, edges, h, alive)
            drop = {v for v in alive if deg[v] < k}
            if not drop:
                break
            alive -= drop
        if not alive:
            break
        for v in alive:
            core[v] = k
        k += 1
    return core


def densest(n, edges, h):
    """max over non-empty S of mu(S)/|S|, and every maximiser (as bitmasks)."""
    cl = cliques(n, edges, h)
    if n == 0:
        return Fraction(0), []
    masks = np.array([sum(1 << v for v in S) for S in cl], dtype=np.int64)
    allS = np.arange(1, 1 << n, dtype=np.int64)
    mu = np.zeros(allS.size, dtype=np.int64)
    for c in masks:
        mu += ((allS & c) == c)
    size = np.zeros(allS.size, dtype=np.int64)
    for v in range(n):
        size += (allS >> v) & 1
    ratio = mu / size
    top = ratio.max()
    best = max(Fraction(int(mu[i]), int(size[i])) for i in np.nonzero(ratio >= top - 1e-9)[0])
    arg = allS[np.nonzero(mu * best.denominator == best.numerator * size)[0]].tolist()
    if best == 0:
        arg = []
    return best, arg


def random_graph(n, p, seed):
    rng = np.random.default_rng(seed)
    return [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]


def elementary_symmetric(values, r):
    """e_r(values): the sum, over all r-element subsets, of their products."""
    e = [1] + [0] * r
    for a in values:
        for j in range(r, 0, -1):
            e[j] += e[j - 1] * a
    return e[r]


def multipartite_closed_form(parts, h):
    """Clique-degrees and clique-core numbers, per part, of the complete
    multipartite graph with the given part sizes.

    An h-clique takes one vertex from each of h distinct parts, so a vertex of
    part i lies in e_{h-1}(a_j : j != i) of them.  The vertices of a part are
    alike and pairwise non-adjacent, so a peel removes a part whole: the part
    of least remaining clique-degree (the largest part left) goes at level
    k = max(k, its degree), and every part whose degree then drops to k or
    below follows at the same level."""
    p = len(parts)
    deg = [elementary_symmetric([parts[j] for j in range(p) if j != i], h - 1) for i in range(p)]
    core = [0] * p
    alive = set(range(p))
    k = 0
    while alive:
        cur = {i: elementary_symmetric([parts[j] for j in alive if j != i], h - 1) for i in alive}
        k = max(k, min(cur.values()))
        for i in [i for i in alive if cur[i] <= k]:
            core[i] = k
            alive.remove(i)
    return deg, core


def pattern_instances(n, edges, pattern, x=0, vertices=None):
    """Instances of a special pattern as (members) tuples, by testing vertex
    subsets: an x-star (pattern 1) is a centre adjacent to x other chosen
    vertices; a 4-loop (pattern 2) is one of the three cyclic orders of a
    4-set whose four edges all exist.  Subgraphs, not necessarily induced."""
    adj = adjacency_sets(n, edges)
    vs = sorted(range(n) if vertices is None else vertices)
    out = []
    if pattern == 1:
        for S in itertools.combinations(vs, x + 1):
            for c in S:
                if all(u in adj[c] for u in S if u != c):
                    out.append(S)
    else:
        for a, b, c, d in itertools.combinations(vs, 4):
            for p, q, r, s in ((a, b, c, d), (a, b, d, c), (a, c, b, d)):
                if q in adj[p] and r in adj[q] and s in adj[r] and p in adj[s]:
                    out.append((a, b, c, d))
    return out


def pattern_degrees(n, edges, pattern, x=0, vertices=None):
    deg = [0] * n
    inst = pattern_instances(n, edges, pattern, x, vertices)
    for S in inst:
        for v in S:
            deg[v] += 1
    return deg, len(inst)


def pattern_core_fixpoint(n, edges, pattern, x=0):
    """core(v) = max k with v in the largest set whose every vertex lies in
    >= k pattern instances inside it (recounted from scratch each pass)."""
    core = [0] * n
    k = 0
    while True:
        alive = set(range(n))
        while True:
            deg, _ = pattern_degrees(n, edges, pattern, x, alive)
            drop = {v for v in alive if deg[v] < k}
            if not drop:
                break
            alive -= drop
        if not alive:
            break
        for v in alive:
            core[v] = k
        k += 1
    return core
