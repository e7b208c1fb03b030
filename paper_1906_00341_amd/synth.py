"""Seeded synthetic graph generators (inputs only).

This module draws edge lists; it holds none of the densest-subgraph
arithmetic.  Both the HIP path and the CPU oracle consume its output, which is
a raw list of undirected vertex pairs: duplicates and self-loops may be present
and each consumer removes them itself (the paper's data model is a simple
undirected graph, Section 3 "Data model").

The generators stand in for the paper's datasets (Section 8, dataset table),
which are not available here:

* ``er_planted``   -- Erdos-Renyi G(n, m) plus one planted dense block, shaped like
                      the small graphs the paper solves exactly.
* ``chung_lu``     -- power-law expected-degree graph (exponent beta) with planted
                      dense blocks, shaped like the large power-law graphs.
* ``rmat``         -- Graph500-style recursive matrix graph (the paper's own
                      synthetic R-MAT family, scaled up).
* ``batch_graphs`` -- a mixture of small Chung-Lu graphs of uneven size.

Every function is deterministic in its ``seed`` and returns
``(n, src, dst)`` with ``src``/``dst`` int32 numpy arrays of equal length.
Vertex ids are randomly permuted so that id order carries no structure.
"""
from __future__ import annotations

import numpy as np

__all__ = ["er_planted", "chung_lu", "rmat", "batch_specs", "batch_graph",
           "plant_block", "complete_graph", "from_edges"]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def from_edges(n: int, edges) -> tuple[int, np.ndarray, np.ndarray]:
    """Wrap an explicit edge list (tests, fixtures)."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    return int(n), e[:, 0].astype(np.int32), e[:, 1].astype(np.int32)


def complete_graph(n: int) -> tuple[int, np.ndarray, np.ndarray]:
    iu, ju = np.triu_indices(n, 1)
    return int(n), iu.astype(np.int32), ju.astype(np.int32)


def complete_multipartite(parts, seed: int = 0) -> tuple[int, np.ndarray, np.ndarray]:
    """Complete multipartite graph with the given part sizes: every pair of
    vertices in different parts is an edge.  Vertex ids are a seeded random
    permutation, so parts are not contiguous id ranges.  Returns the edge
    list and, as a fourth value, the part index of every vertex."""
    sizes = [int(a) for a in parts]
    n = sum(sizes)
    part = np.repeat(np.arange(len(sizes)), sizes)
    perm = np.random.default_rng(seed).permutation(n)
    part_of = np.empty(n, dtype=np.int64)
    part_of[perm] = part
    iu, ju = np.triu_indices(n, 1)
    keep = part_of[iu] != part_of[ju]
    return int(n), iu[keep].astype(np.int32), ju[keep].astype(np.int32), part_of


def plant_block(rng: np.random.Generator, n: int, size: int, p: float,
                exclude: np.ndarray | None = None):
    """Pick ``size`` distinct vertex ids (avoiding ``exclude``) and keep each of
    their C(size, 2) pairs independently with probability ``p``."""
    if exclude is not None and exclude.size:
        pool = np.setdiff1d(np.arange(n, dtype=np.int64), exclude)
        ids = rng.choice(pool, size=size, replace=False)
    else:
        ids = rng.choice(n, size=size, replace=False)
    iu, ju = np.triu_indices(size, 1)
    keep = rng.random(iu.size) < p
    return ids.astype(np.int64), ids[iu[keep]].astype(np.int64), ids[ju[keep]].astype(np.int64)


def er_planted(n: int = 2000, m: int = 10000, plant: int = 60, p: float = 0.4,
               seed: int = 1):
    """G(n, m): exactly ``m`` distinct uniform pairs without self-loops, then a
    planted block of ``plant`` random ids whose pairs are added with prob. p
    (union with the ER edges)."""
    rng = _rng(seed)
    if n < 2:
        return n, np.zeros(0, np.int32), np.zeros(0, np.int32)
    m = min(m, n * (n - 1) // 2)
    chosen = np.zeros(0, dtype=np.int64)
    while chosen.size < m:
        need = m - chosen.size
        a = rng.integers(0, n, size=2 * need + 16, dtype=np.int64)
        b = rng.integers(0, n, size=2 * need + 16, dtype=np.int64)
        ok = a != b
        a, b = a[ok], b[ok]
        key = np.minimum(a, b) * n + np.maximum(a, b)
        allk = np.concatenate([chosen, key])
        _, first = np.unique(allk, return_index=True)
        first.sort()
        chosen = allk[first][:m]
    src = chosen // n
    dst = chosen % n
    if plant > 0:
        _, ps, pd = plant_block(rng, n, min(plant, n), p)
        src = np.concatenate([src, ps])
        dst = np.concatenate([dst, pd])
    return n, src.astype(np.int32), dst.astype(np.int32)


def _chung_lu_weights(n: int, avg_deg: float, beta: float, i0: float = 1.0):
    """Expected degrees w_i proportional to (i + i0)^(-1/(beta-1)), capped at
    sqrt(sum w) and rescaled to mean ``avg_deg`` (cap and rescale repeated a few
    times so that both hold approximately)."""
    i = np.arange(n, dtype=np.float64)
    w = (i + i0) ** (-1.0 / (beta - 1.0))
    w *= avg_deg * n / w.sum()
    for _ in range(8):
        cap = np.sqrt(w.sum())
        w = np.minimum(w, cap)
        w *= avg_deg * n / w.sum()
    return w


def chung_lu(n: int = 1_000_000, avg_deg: float = 20.0, beta: float = 2.1,
             planted: int = 5, plant_size: int = 200, p: float = 0.7,
             seed: int = 1):
    """Chung-Lu graph: n*avg_deg/2 endpoint pairs, each endpoint drawn
    independently with probability proportional to its weight; ids permuted;
    then ``planted`` disjoint random blocks with pair probability ``p``."""
    rng = _rng(seed)
    w = _chung_lu_weights(n, avg_deg, beta)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    M = int(round(n * avg_deg / 2))
    src = np.searchsorted(cdf, rng.random(M), side="right").astype(np.int64)
    dst = np.searchsorted(cdf, rng.random(M), side="right").astype(np.int64)
    np.minimum(src, n - 1, out=src)
    np.minimum(dst, n - 1, out=dst)
    perm = rng.permutation(n).astype(np.int64)
    src = perm[src]
    dst = perm[dst]
    parts_s, parts_d = [src], [dst]
    used = np.zeros(0, dtype=np.int64)
    for _ in range(planted):
        ids, ps, pd = plant_block(rng, n, plant_size, p, exclude=used)
        used = np.concatenate([used, ids])
        parts_s.append(ps)
        parts_d.append(pd)
    return n, np.concatenate(parts_s).astype(np.int32), np.concatenate(parts_d).astype(np.int32)


def rmat(scale: int = 22, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 1, chunk: int = 1 << 24):
    """R-MAT: edge_factor * 2^scale draws; at each of ``scale`` levels the
    quadrant is (a, b, c, d=1-a-b-c); no per-level noise; ids permuted."""
    rng = _rng(seed)
    n = 1 << scale
    M = edge_factor * n
    src = np.empty(M, dtype=np.int32)
    dst = np.empty(M, dtype=np.int32)
    ab = a + b
    abc = a + b + c
    for lo in range(0, M, chunk):
        hi = min(M, lo + chunk)
        k = hi - lo
        s = np.zeros(k, dtype=np.int64)
        d = np.zeros(k, dtype=np.int64)
        for _ in range(scale):
            r = rng.random(k)
            sbit = r >= ab                     # quadrants c, d: lower half
            dbit = ((r >= a) & (r < ab)) | (r >= abc)  # quadrants b, d: right half
            s = (s << 1) | sbit
            d = (d << 1) | dbit
        src[lo:hi] = s
        dst[lo:hi] = d
    perm = rng.permutation(n).astype(np.int32)
    return n, perm[src], perm[dst]


def batch_specs(count: int = 8192, seed: int = 7):
    """Per-graph parameters of the batched mixture: n log-uniform in
    [100, 50000], Chung-Lu exponent U[2, 3], average degree U[4, 40],
    h uniform in {2, 3, 4}; graph i is drawn with seed ``seed*1000003 + i``."""
    rng = _rng(seed)
    n = np.rint(np.exp(rng.uniform(np.log(100), np.log(50000), size=count))).astype(np.int64)
    beta = rng.uniform(2.0, 3.0, size=count)
    avg = rng.uniform(4.0, 40.0, size=count)
    h = rng.integers(2, 5, size=count)
    return [dict(n=int(n[i]), beta=float(beta[i]), avg_deg=float(avg[i]), h=int(h[i]),
                 seed=int(seed) * 1000003 + i) for i in range(count)]


def batch_graph(spec: dict):
    """One graph of the batched mixture (Chung-Lu, no planted blocks)."""
    return chung_lu(n=spec["n"], avg_deg=min(spec["avg_deg"], spec["n"] - 1),
                    beta=spec["beta"], planted=0, seed=spec["seed"])
