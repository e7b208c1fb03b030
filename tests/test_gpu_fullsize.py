"""Parity at the benchmark's full size, in the configuration bench.py times.

Chung-Lu, n = 10^6, average degree 20, exponent 2.1, five planted 200-vertex
blocks at pair probability 0.7, h = 3: clique-degrees, core numbers and the
k_max-core are compared with the CPU oracle element by element over the whole
graph.  The oracle's exact step (Dinic on 128-bit capacities) would take many
minutes here, so CoreExact's answer is checked by properties that hold for
every densest subgraph: its density is the returned rho_opt (counted by the
oracle), it lies in the ceil(rho_opt)-core (Lemma 7), and rho_opt lies between
the density of the k_max-core and k_max (Lemma 8 and Theorem 1).  PeelApp (every
minimum-degree vertex per round) is compared with the oracle exactly: member
set, density, rounds and the round of the answer; its density is also at least
rho' (every level set R_k is one of its residual graphs) and within Lemma 10's
factor h of rho_opt.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1906_00341_amd import dsd, synth

pytestmark = pytest.mark.gpu

CHUNG_LU_1E6 = dict(n=1_000_000, avg_deg=20.0, beta=2.1, planted=5, plant_size=200, p=0.7)


def induced_mu(og, h, mask):
    off, adj = og.adjacency()
    rows = np.repeat(np.arange(og.n), np.diff(off))
    e = mask[rows] & mask[adj] & (rows < adj)
    sub = oracle.Graph(og.n, rows[e].astype(np.int32), adj[e].astype(np.int32))
    return sub.clique_degrees(h)[1]


@pytest.fixture(scope="module")
def chung_lu_1e6():
    """The benchmark's Chung-Lu graph on the GPU (edge list read from device
    memory, as the benchmark does) and in the oracle, with the oracle's core
    numbers at h = 3 (computed once for the tests below)."""
    torch = pytest.importorskip("torch")
    n, s, d = synth.chung_lu(seed=1, **CHUNG_LU_1E6)
    g = dsd.build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda())
    og = oracle.Graph(n, s, d)
    core_o, km_o = og.core_decomposition(3)
    return n, g, og, core_o, km_o


@pytest.mark.timeout(600)
def test_chung_lu_1e6_triangles_whole_graph(chung_lu_1e6):
    h = 3
    n, g, og, core_o, km_o = chung_lu_1e6
    deg_g, mu_g = dsd.clique_degrees(g, h)
    core_g, km_g = dsd.clique_core(g, h)
    mem_app, km_app, dens_app = dsd.core_app(g, h)
    mem_x, rho = dsd.core_exact(g, h)
    mem_p, rho_p, rounds_p, best_p = dsd.peel_app(g, h)
    print(f"gpu: mu={mu_g} kmax={km_g} rho_app={dens_app} rho_opt={rho} "
          f"peel_app={rho_p} rounds={rounds_p} best_round={best_p}", flush=True)

    deg_o, mu_o = og.clique_degrees(h)
    assert mu_g == mu_o
    np.testing.assert_array_equal(deg_g, deg_o)
    assert km_g == km_o
    np.testing.assert_array_equal(core_g, core_o)

    top = core_o == km_o
    assert km_app == km_o
    np.testing.assert_array_equal(mem_app.astype(bool), top)
    assert dens_app == Fraction(induced_mu(og, h, top), int(top.sum()))

    sel = mem_x.astype(bool)
    assert sel.any()
    assert Fraction(induced_mu(og, h, sel), int(sel.sum())) == rho
    assert (core_o[sel] >= math.ceil(rho)).all()
    assert dens_app <= rho <= km_o

    mem_po, rho_po, steps_po, best_po = og.peel_app(h, rounds=True)
    assert (rho_p, rounds_p, best_p) == (rho_po, steps_po, best_po)
    np.testing.assert_array_equal(mem_p.astype(bool), mem_po)
    lv, rs, rm = og.level_table(h, core_o)
    rho1 = max(Fraction(int(m), int(z)) for m, z in zip(rm, rs) if z)
    assert rho1 <= rho_p <= rho <= h * rho_p


@pytest.mark.timeout(900)
def test_chung_lu_1e6_core_exact_certified(chung_lu_1e6):
    """CoreExact's rho_opt on the benchmark graph, pinned exactly.

    The locate step's figures (Pruning1/2, Section 6.1: rho', k', rho'',
    k'', the number of components of R_{k'}) must equal the oracle's locate
    on the oracle's core numbers.  Then one strict test of the oracle
    (Algorithm 1's network, Lemma 14) on G[R_c], c = ceil(rho), at alpha =
    rho must find nothing denser: by Lemma 7 every subgraph denser than rho
    would have its densest subgraph inside R_{ceil(rho_opt)}, which lies in
    R_c.  With the returned set attaining rho, rho = rho_opt."""
    h = 3
    n, g, og, core_o, km_o = chung_lu_1e6
    mem_x, rho = dsd.core_exact(g, h)
    st = g.stats()
    loc = og.locate(h, core_o)
    print(f"gpu locate: rho'={st['locate_rho1_num']}/{st['locate_rho1_den']} k'={st['locate_k1']} "
          f"rho''={st['locate_rho2_num']}/{st['locate_rho2_den']} k''={st['locate_k2']} "
          f"components={st['locate_components']} located={st['located_vertices']}; oracle {loc['rho1']} "
          f"{loc['k1']} {loc['rho2']} {loc['k2']} {loc['ncomp']}", flush=True)
    assert Fraction(st["locate_rho1_num"], st["locate_rho1_den"]) == loc["rho1"]
    assert st["locate_k1"] == loc["k1"]
    assert Fraction(st["locate_rho2_num"], st["locate_rho2_den"]) == loc["rho2"]
    assert st["locate_k2"] == loc["k2"]
    assert st["locate_components"] == loc["ncomp"]
    assert st["located_vertices"] == int((core_o >= loc["k2"]).sum())

    sel = mem_x.astype(bool)
    assert Fraction(induced_mu(og, h, sel), int(sel.sum())) == rho
    c = math.ceil(rho)
    mask = core_o >= c
    assert not (sel & ~mask).any()
    idx, s2, d2 = induced(og, mask)
    sub = oracle.Graph(idx.size, s2, d2)
    found, _ = sub.denser_than(h, rho)
    print(f"certificate: G[R_{c}] has {idx.size} vertices, {sub.m} edges; denser than {rho}: {found}", flush=True)
    assert not found


# ------------------------------------------------------------------ R-MAT scale 22, h = 4 and 5

RMAT_22 = dict(scale=22, edge_factor=16, seed=1)


@pytest.fixture(scope="module")
def rmat22():
    torch = pytest.importorskip("torch")
    n, s, d = synth.rmat(**RMAT_22)
    og = oracle.Graph(n, s, d)
    g = dsd.build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda())
    return n, og, g


def induced(og, mask):
    """Edges of the subgraph induced by mask, relabelled 0 .. |mask| - 1."""
    off, adj = og.adjacency()
    rows = np.repeat(np.arange(og.n, dtype=np.int32), np.diff(off))
    e = mask[rows] & mask[adj] & (rows < adj)
    idx = np.nonzero(mask)[0]
    new = np.full(og.n, -1, dtype=np.int64)
    new[idx] = np.arange(idx.size)
    return idx, new[rows[e]].astype(np.int32), new[adj[e]].astype(np.int32)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("h", [4, 5])
def test_rmat22_higher_order_cliques(rmat22, h):
    """R-MAT scale 22 (n = 4,194,304, 67,108,864 edge draws): the oracle
    cannot list its 10^11 - 10^13 cliques, so the decomposition is checked by
    what pins it at any size.
      * sum of degrees = h mu, core <= degree;
      * clique-degrees across the whole degree range: 48 sampled vertices of
        degree <= 1,500 against the oracle; the 20 largest hubs and 20
        vertices sampled from degree ranks 20 .. 20,000 against the
        (h-1)-cliques of their induced neighbourhoods, counted by a separate
        enumeration (another graph, another h), with the oracle recounting
        those of at most 2*10^7;
      * every level set R_c = {core >= c} of the top region (at h = 4 every
        level whose R_c has at most 30,000 vertices, up to 300 levels; at
        h = 5, where every R_c holds the 10^12 cliques of the k_max-core,
        the 12 highest levels of at most 4,000 vertices) has least
        clique-degree exactly c
        inside itself (so R_c is a c-core and c is the degree at which its
        level opens), counted by a separate enumeration of its induced
        subgraph; for sampled levels the oracle recounts the vertex of least
        degree; at h = 4 CoreApp returns exactly the k_max-core with the
        density that separate count gives it."""
    n, og, g = rmat22
    deg_g, mu_g = dsd.clique_degrees(g, h)
    core_g, km = dsd.clique_core(g, h)
    print(f"rmat22 h={h}: mu={mu_g} kmax={km} levels={np.unique(core_g).size}", flush=True)
    assert int(deg_g.sum()) == h * mu_g
    assert (core_g <= deg_g).all()
    assert int(core_g.max()) == km

    off, adj = og.adjacency()
    deg = np.diff(off)
    rows = np.repeat(np.arange(og.n, dtype=np.int32), deg)
    rng = np.random.default_rng(100 + h)
    sample = rng.choice(np.nonzero((deg >= 1) & (deg <= 1500))[0], 48, replace=False)
    for v in sample:
        assert og.clique_degree_of(h, int(v)) == int(deg_g[v]), int(v)

    # hubs: the h-cliques through v are the (h-1)-cliques of G[N(v)]
    by_deg = np.argsort(-deg, kind="stable")
    hubs = np.concatenate([by_deg[:20], by_deg[rng.choice(np.arange(20, 20_000), 20, replace=False)]])
    oracle_hubs = 0
    upper = rows < adj
    for v in hubs:
        nb = adj[off[v]:off[v + 1]]
        inn = np.zeros(og.n, bool)
        inn[nb] = True
        e = upper & inn[rows] & inn[adj]
        loc = np.full(og.n, -1, np.int64)
        loc[nb] = np.arange(nb.size)
        s2, d2 = loc[rows[e]].astype(np.int32), loc[adj[e]].astype(np.int32)
        sub = dsd.build_csr(nb.size, s2, d2)
        _, mu_nb = dsd.clique_degrees(sub, h - 1)
        sub.free()
        assert mu_nb == int(deg_g[v]), (int(v), int(deg[v]))
        if mu_nb <= 20_000_000:
            assert oracle.Graph(nb.size, s2, d2).clique_degrees(h - 1)[1] == mu_nb, int(v)
            oracle_hubs += 1
    print(f"  hubs: {hubs.size} checked (max degree {int(deg[by_deg[0]])}), {oracle_hubs} recounted by the oracle",
          flush=True)

    mem_app = dens_app = None
    if h == 4:
        mem_app, km_app, dens_app = dsd.core_app(g, h)
        np.testing.assert_array_equal(mem_app.astype(bool), core_g == km)
        assert km_app == km

    # the top region: the highest levels, each R_c of at most 4,000 vertices
    lv, cnt = np.unique(core_g, return_counts=True)
    levels, sizes = lv[::-1], np.cumsum(cnt[::-1])
    ntop, vmax = (300, 30_000) if h == 4 else (12, 4_000)
    top = levels[:ntop][sizes[:ntop] <= vmax]
    assert top.size >= 1 and top[0] == km
    region = core_g >= top[-1]
    ridx = np.nonzero(region)[0]
    e = upper & region[rows] & region[adj]
    rl = np.full(og.n, -1, np.int64)
    rl[ridx] = np.arange(ridx.size)
    rs, rd = rl[rows[e]], rl[adj[e]]
    rcore = core_g[ridx]
    checked = 0
    picks = set(np.linspace(0, top.size - 1, 4).astype(int).tolist())
    for i, c in enumerate(top):
        keep = rcore >= c
        ke = keep[rs] & keep[rd]
        sub_idx = np.nonzero(keep)[0]
        sl = np.full(ridx.size, -1, np.int64)
        sl[sub_idx] = np.arange(sub_idx.size)
        s2, d2 = sl[rs[ke]].astype(np.int32), sl[rd[ke]].astype(np.int32)
        sub = dsd.build_csr(sub_idx.size, s2, d2)
        d_in, mu_in = dsd.clique_degrees(sub, h)
        sub.free()
        j = int(np.argmin(d_in))
        # R_c is a c-core, and c is the smallest degree when its level opens
        assert int(d_in[j]) == int(c), int(c)
        if h == 4 and c == km:
            assert dens_app == Fraction(mu_in, sub_idx.size)
        if i in picks and int(d_in[j]) <= 200_000_000:
            assert oracle.Graph(sub_idx.size, s2, d2).clique_degree_of(h, j) == int(d_in[j])
            checked += 1
    print(f"  top region: {top.size} level sets of up to {ridx.size} vertices checked, {checked} oracle recounts",
          flush=True)
    # sampled level sets below the top region, each a c-core
    low = levels[levels < top[-1]]
    for c in low[np.linspace(0, low.size - 1, 5).astype(int)[1:-1]]:
        mask = core_g >= c
        idx, s2, d2 = induced(og, mask)
        sub = dsd.build_csr(idx.size, s2, d2)
        d_in, mu_in = dsd.clique_degrees(sub, h)
        sub.free()
        print(f"  R_{int(c)}: {idx.size} vertices, least degree {int(d_in.min())}", flush=True)
        assert int(d_in.min()) == int(c), int(c)
