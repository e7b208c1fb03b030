"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Integer results (clique-degrees, core numbers, k_max, member sets of the
k_max-core) must match bit for bit; densities are compared as exact
rationals.  Densest subgraphs need not be unique, so for CoreExact the
returned set must attain rho_opt and lie inside the ceil(rho_opt)-core
(Lemma 7 holds for every densest subgraph).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1906_00341_amd import dsd, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    dsd.load()          # fails loudly when the library is missing


def both(n, s, d):
    return oracle.Graph(n, s, d), dsd.build_csr(n, np.ascontiguousarray(s, np.int32), np.ascontiguousarray(d, np.int32))


def density_of(og: oracle.Graph, h: int, member) -> Fraction:
    idx = np.nonzero(np.asarray(member))[0]
    if idx.size == 0:
        return Fraction(0)
    off, adj = og.adjacency()
    keep = np.zeros(og.n, dtype=bool)
    keep[idx] = True
    rows = np.repeat(np.arange(og.n), np.diff(off))
    e = keep[rows] & keep[adj] & (rows < adj)
    sub = oracle.Graph(og.n, rows[e].astype(np.int32), adj[e].astype(np.int32))
    _, mu = sub.clique_degrees(h)
    return Fraction(mu, idx.size)


def check_all(n, s, d, h, exact=True, app=True):
    og, gg = both(n, s, d)
    deg_o, mu_o = og.clique_degrees(h)
    deg_g, mu_g = dsd.clique_degrees(gg, h)
    assert mu_g == mu_o
    np.testing.assert_array_equal(deg_g, deg_o)
    core_o, km_o = og.core_decomposition(h)
    core_g, km_g = dsd.clique_core(gg, h)
    assert km_g == km_o
    np.testing.assert_array_equal(core_g, core_o)
    if app:
        mem_o, km2, dens_o = og.inc_app(h)
        mem_g, km3, dens_g = dsd.core_app(gg, h)
        assert km3 == km2 and dens_g == dens_o
        np.testing.assert_array_equal(mem_g.astype(bool), mem_o)
    if exact:
        _, rho_o, _ = og.exact(h, "core")
        mem_g, rho_g = dsd.core_exact(gg, h)
        assert rho_g == rho_o
        if rho_o > 0:
            assert density_of(og, h, mem_g) == rho_o
            kk = math.ceil(rho_o)
            assert (core_o[mem_g.astype(bool)] >= kk).all()
        else:
            assert not mem_g.any()
    return gg


# ------------------------------------------------------------------ fixtures

@pytest.mark.parametrize("name", ["F1", "F2", "F4"])
@pytest.mark.parametrize("h", [2, 3, 4])
def test_paper_examples(fixtures, name, h):
    f = fixtures[name]
    e = np.asarray(f["edges"], np.int32)
    check_all(f["n"], e[:, 0], e[:, 1], h)


def test_fig1_values(fixtures):
    f = fixtures["F1"]
    e = np.asarray(f["edges"], np.int32)
    g = dsd.build_csr(f["n"], e[:, 0], e[:, 1])
    mem, rho = dsd.core_exact(g, 2)
    assert rho == Fraction(11, 7) and np.nonzero(mem)[0].tolist() == f["expect"]["h2_cds"]
    mem, rho = dsd.core_exact(g, 3)
    assert rho == Fraction(1, 2) and np.nonzero(mem)[0].tolist() == f["expect"]["h3_cds"]
    deg, _ = dsd.clique_degrees(g, 3)
    A, B, C = f["labels"]["A"], f["labels"]["B"], f["labels"]["C"]
    assert [int(deg[A]), int(deg[B]), int(deg[C])] == [2, 1, 2]


# ------------------------------------------------------------------ random small graphs

@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("h", [2, 3, 4, 5, 6])
def test_random_small(seed, h):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(20, 160))
    p = float(rng.uniform(0.05, 0.45))
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < p
    check_all(n, iu[keep].astype(np.int32), ju[keep].astype(np.int32), h, exact=(n <= 80 or h <= 3))


@pytest.mark.parametrize("n", [0, 1, 2, 5])
@pytest.mark.parametrize("h", [2, 3, 6])
def test_tiny_and_empty(n, h):
    z = np.zeros(0, np.int32)
    g = dsd.build_csr(n, z, z)
    assert g.info() == (n, 0)
    if n == 0:
        return
    deg, mu = dsd.clique_degrees(g, h)
    assert mu == 0 and not deg.any()
    core, km = dsd.clique_core(g, h)
    assert km == 0 and not core.any()
    mem, km, dens = dsd.core_app(g, h)
    assert km == 0 and dens == 0 and not mem.any()
    mem, rho = dsd.core_exact(g, h)
    assert rho == 0 and not mem.any()


def test_duplicates_and_self_loops_are_dropped():
    s = np.array([0, 1, 1, 2, 2, 3, 0, 0, 2], np.int32)
    d = np.array([1, 0, 1, 0, 2, 3, 2, 1, 1], np.int32)
    g = dsd.build_csr(4, s, d)
    assert g.info() == (4, 3)
    deg, mu = dsd.clique_degrees(g, 3)
    assert mu == 1 and deg.tolist() == [1, 1, 1, 0]


@pytest.mark.parametrize("h", [2, 3, 4, 5, 6])
def test_complete_graph(h):
    n, s, d = synth.complete_graph(40)
    g = dsd.build_csr(n, s, d)
    deg, mu = dsd.clique_degrees(g, h)
    assert mu == math.comb(40, h) and (deg == math.comb(39, h - 1)).all()
    core, km = dsd.clique_core(g, h)
    assert km == math.comb(39, h - 1) and (core == km).all()
    mem, rho = dsd.core_exact(g, h)
    assert rho == Fraction(math.comb(40, h), 40) and mem.all()


@pytest.mark.parametrize("n,h", [(300, 4), (800, 4), (1281, 4), (1700, 4), (2049, 4), (300, 5), (100, 6)])
def test_complete_graph_wide_neighbourhoods(n, h):
    # out-neighbourhoods up to n - 1 vertices: every bitmap class of the
    # engine, up to its 2048-vertex limit (the hub class: 1281 .. 2048)
    _, s, d = synth.complete_graph(n)
    g = dsd.build_csr(n, s, d)
    deg, mu = dsd.clique_degrees(g, h)
    assert mu == math.comb(n, h) and (deg == math.comb(n - 1, h - 1)).all()
    core, km = dsd.clique_core(g, h)
    assert km == math.comb(n - 1, h - 1) and (core == km).all()
    mem, km2, dens = dsd.core_app(g, h)
    assert km2 == km and mem.all() and dens == Fraction(math.comb(n, h), n)


def test_out_degree_limit():
    n, s, d = synth.complete_graph(2050)
    g = dsd.build_csr(n, s, d)
    with pytest.raises(dsd.DsdError) as e:
        dsd.clique_degrees(g, 4)
    assert e.value.status == -5
    deg, mu = dsd.clique_degrees(g, 3)      # h <= 3 has no such limit
    assert mu == math.comb(2050, 3) and (deg == math.comb(2049, 2)).all()


def test_hub_with_sparse_out_neighbourhood():
    """A hub whose 1,400 neighbours all rank above it (each also has 1,401
    leaves of its own) and are joined to each other sparsely: the hub's
    out-neighbourhood of 1,400 takes the 1,281 .. 2,048 class of the
    enumeration and of the per-vertex peel counting at h = 4, 5, 6, with few
    cliques, against the oracle."""
    rng = np.random.default_rng(3)
    k, leaves = 1400, 1401
    hub = 0
    sat = np.arange(1, k + 1)
    src = [np.full(k, hub), ]
    dst = [sat]
    # sparse random pairs among the satellites, plus a few dense spots
    a = rng.integers(1, k + 1, size=6 * k)
    b = rng.integers(1, k + 1, size=6 * k)
    src.append(a)
    dst.append(b)
    blk = rng.choice(sat, size=12, replace=False)
    iu, ju = np.triu_indices(12, 1)
    src.append(blk[iu])
    dst.append(blk[ju])
    base = k + 1
    for i, x in enumerate(sat):
        src.append(np.full(leaves, x))
        dst.append(np.arange(base, base + leaves))
        base += leaves
    n = base
    s = np.concatenate(src).astype(np.int32)
    d = np.concatenate(dst).astype(np.int32)
    g = dsd.build_csr(n, s, d)
    og = oracle.Graph(n, s, d)
    for h in (4, 5, 6):
        deg, mu = dsd.clique_degrees(g, h)
        deg_o, mu_o = og.clique_degrees(h)
        assert mu == mu_o
        np.testing.assert_array_equal(deg, deg_o)
        core, km = dsd.clique_core(g, h)
        core_o, km_o = og.core_decomposition(h)
        assert km == km_o
        np.testing.assert_array_equal(core, core_o)


@pytest.mark.parametrize("k", [2400, 3500, 4500])
def test_hub_rows_beyond_2048(k):
    """A hub whose row holds k entries is removed while that row is long: k - 4
    of its neighbours have no clique and leave in the first round (before
    any compaction of the adjacency), and the other four, which with the hub
    form a K5, also belong to a K10 and so outlast it; the hub leaves next,
    alone, with its whole row.  At h = 4 a row of up to 4,096 entries takes
    the sliced counting with 64-word bitmap rows, a longer one a single
    workgroup; at h = 5 every row beyond 2,048 entries takes a single
    workgroup.  Clique-degrees, cores and CoreApp against the oracle."""
    hub = 0
    sat = np.arange(1, k + 1)
    extra = np.arange(k + 1, k + 7)                  # 6 more vertices of the K10
    src, dst = [np.full(k, hub)], [sat]
    quad = sat[:4]
    ten = np.concatenate([quad, extra])
    iu, ju = np.triu_indices(ten.size, 1)
    src.append(ten[iu])
    dst.append(ten[ju])
    n = k + 7
    s = np.concatenate(src).astype(np.int32)
    d = np.concatenate(dst).astype(np.int32)
    perm = np.random.default_rng(k).permutation(n).astype(np.int32)
    s, d = perm[s], perm[d]
    g = dsd.build_csr(n, s, d)
    og = oracle.Graph(n, s, d)
    for h in (4, 5):
        deg, mu = dsd.clique_degrees(g, h)
        deg_o, mu_o = og.clique_degrees(h)
        assert mu == mu_o
        np.testing.assert_array_equal(deg, deg_o)
        core, km = dsd.clique_core(g, h)
        core_o, km_o = og.core_decomposition(h)
        assert km == km_o
        np.testing.assert_array_equal(core, core_o)
        # the hub left at its own level, below the K10's
        assert 0 < core_o[perm[hub]] < km_o
        mem, km2, dens = dsd.core_app(g, h)
        mem_o, km2_o, dens_o = og.inc_app(h)
        assert km2 == km2_o and dens == dens_o
        np.testing.assert_array_equal(mem.astype(bool), mem_o)


@pytest.mark.parametrize("h", [4])
def test_hub_class_k1500_plus_noise(h):
    """A 1,500-vertex clique (every root of out-degree 1,281 .. 1,499 takes
    the hub class of the engine and of the per-vertex peel counting) beside a
    sparse ER graph with a planted block: clique-degrees and core numbers are
    the closed form C(1499, h-1) on the clique and the oracle's on the rest;
    CoreApp returns the clique."""
    k = 1500
    _, s1, d1 = synth.complete_graph(k)
    n2, s2, d2 = synth.er_planted(n=3000, m=20000, plant=40, p=0.6, seed=h)
    n = k + n2
    perm = np.random.default_rng(h).permutation(n).astype(np.int32)
    s = perm[np.concatenate([s1, s2 + k])]
    d = perm[np.concatenate([d1, d2 + k])]
    g = dsd.build_csr(n, s, d)
    og = oracle.Graph(n2, s2, d2)
    deg_o, mu_o = og.clique_degrees(h)
    core_o, _ = og.core_decomposition(h)
    in_k = np.zeros(n, bool)
    in_k[perm[:k]] = True
    want_deg = np.zeros(n, np.uint64)
    want_deg[perm[:k]] = math.comb(k - 1, h - 1)
    want_deg[perm[k:]] = deg_o
    want_core = np.zeros(n, np.uint64)
    want_core[perm[:k]] = math.comb(k - 1, h - 1)
    want_core[perm[k:]] = core_o
    deg, mu = dsd.clique_degrees(g, h)
    assert mu == math.comb(k, h) + mu_o
    np.testing.assert_array_equal(deg, want_deg)
    core, km = dsd.clique_core(g, h)
    assert km == math.comb(k - 1, h - 1)
    np.testing.assert_array_equal(core, want_core)
    mem, km2, dens = dsd.core_app(g, h)
    assert km2 == km
    np.testing.assert_array_equal(mem.astype(bool), in_k)
    assert dens == Fraction(math.comb(k, h), k)


@pytest.mark.parametrize("parts,hs", [([400, 300, 250, 200, 100], (2, 3, 4)),
                                      ([40, 30, 30, 20, 10, 5], (5, 6)),
                                      ([600, 90, 90, 80], (3, 4))])
def test_complete_multipartite(parts, hs):
    from tests import brute
    n, s, d, part = synth.complete_multipartite(parts, seed=len(parts))
    g = dsd.build_csr(n, s, d)
    for h in hs:
        deg, core = brute.multipartite_closed_form(parts, h)
        got, mu = dsd.clique_degrees(g, h)
        assert mu == brute.elementary_symmetric(parts, h)
        np.testing.assert_array_equal(got, np.asarray(deg, np.uint64)[part])
        got, km = dsd.clique_core(g, h)
        assert km == max(core)
        np.testing.assert_array_equal(got, np.asarray(core, np.uint64)[part])
        top = [i for i in range(len(parts)) if core[i] == km]
        mem, km2, dens = dsd.core_app(g, h)
        assert km2 == km
        np.testing.assert_array_equal(mem.astype(bool), np.isin(part, top))
        assert dens == Fraction(brute.elementary_symmetric([parts[i] for i in top], h),
                                sum(parts[i] for i in top))


@pytest.mark.parametrize("h", [3, 4])
def test_union_of_complete_graphs(h):
    # one core level per clique size, out-neighbourhoods up to 1280 vertices
    sizes = [1281, 900, 500, 300, 70, 5]
    src, dst, size_of, base = [], [], [], 0
    for a in sizes:
        _, s, d = synth.complete_graph(a)
        src.append(s + base)
        dst.append(d + base)
        size_of += [a] * a
        base += a
    perm = np.random.default_rng(7).permutation(base).astype(np.int32)
    s, d = perm[np.concatenate(src)], perm[np.concatenate(dst)]
    size_of = np.asarray(size_of)[np.argsort(perm)]
    g = dsd.build_csr(base, s, d)
    want = np.array([math.comb(a - 1, h - 1) for a in size_of], np.uint64)
    deg, mu = dsd.clique_degrees(g, h)
    assert mu == sum(math.comb(a, h) for a in sizes)
    np.testing.assert_array_equal(deg, want)
    core, km = dsd.clique_core(g, h)
    np.testing.assert_array_equal(core, want)
    mem, km2, dens = dsd.core_app(g, h)
    assert km2 == km == math.comb(1280, h - 1)
    np.testing.assert_array_equal(mem.astype(bool), size_of == 1281)
    assert dens == Fraction(math.comb(1281, h), 1281)


@pytest.mark.parametrize("h", [2, 3, 4])
def test_exact_with_every_min_cut_on_the_gpu(fixtures, monkeypatch, h):
    # every network of the exact step goes to the device push-relabel
    monkeypatch.setenv("DSD_FLOW_GPU_MIN_ARCS", "0")
    cases = []
    for name in ("F1", "F4"):
        e = np.asarray(fixtures[name]["edges"], np.int32)
        cases.append((int(fixtures[name]["n"]), e[:, 0], e[:, 1]))
    for seed in range(4):
        cases.append(synth.er_planted(n=300, m=1500, plant=25, p=0.6, seed=40 + seed))
    cases.append(synth.er_planted(seed=2))
    if h == 3:
        # nodes with more than 4096 residual arcs take the block-per-node kernels
        n, s, d = synth.complete_graph(110)
        keep = np.random.default_rng(3).random(len(s)) < 0.97
        cases.append((n, s[keep], d[keep]))
    gpu_cuts = 0
    for n, s, d in cases:
        og = oracle.Graph(n, s, d)
        gg = dsd.build_csr(n, np.ascontiguousarray(s, np.int32), np.ascontiguousarray(d, np.int32))
        _, rho_o, _ = og.exact(h, "core")
        mem_g, rho_g = dsd.core_exact(gg, h)
        st = gg.stats()
        assert st["flow_gpu_calls"] == st["flow_calls"]
        gpu_cuts += st["flow_gpu_calls"]
        assert rho_g == rho_o
        if rho_o > 0:
            assert density_of(og, h, mem_g) == rho_o
            core_o, _ = og.core_decomposition(h)
            assert (core_o[mem_g.astype(bool)] >= math.ceil(rho_o)).all()
    assert gpu_cuts > 0


def _exact_cases(fixtures, extra_dense):
    cases = []
    for name in ("F1", "F4"):
        e = np.asarray(fixtures[name]["edges"], np.int32)
        cases.append((int(fixtures[name]["n"]), e[:, 0], e[:, 1]))
    for seed in range(4):
        cases.append(synth.er_planted(n=300, m=1500, plant=25, p=0.6, seed=40 + seed))
    cases.append(synth.er_planted(seed=2))
    if extra_dense:
        n, s, d = synth.complete_graph(110)
        keep = np.random.default_rng(3).random(len(s)) < 0.97
        cases.append((n, s[keep], d[keep]))
    return cases


@pytest.mark.parametrize("cut", ["gpu", "host"])
def test_triangle_networks_built_on_the_device(fixtures, monkeypatch, cut):
    # every h = 3 network of the exact step is built on the device (bitmap
    # triangle listing, residual CSR there); its minimum cuts run on the
    # device, or on the host from the arcs copied back
    monkeypatch.setenv("DSD_NET_GPU_MIN_EDGES", "0")
    monkeypatch.setenv("DSD_FLOW_GPU_MIN_ARCS", "0" if cut == "gpu" else "-1")
    h = 3
    nets = 0
    for n, s, d in _exact_cases(fixtures, True):
        og = oracle.Graph(n, s, d)
        gg = dsd.build_csr(n, np.ascontiguousarray(s, np.int32), np.ascontiguousarray(d, np.int32))
        _, rho_o, _ = og.exact(h, "core")
        mem_g, rho_g = dsd.core_exact(gg, h)
        st = gg.stats()
        nets += st["flow_gpu_networks"]
        assert st["flow_gpu_calls"] == (st["flow_calls"] if cut == "gpu" else 0)
        assert rho_g == rho_o
        if rho_o > 0:
            assert density_of(og, h, mem_g) == rho_o
    assert nets > 0


@pytest.mark.parametrize("h", [2, 3])
@pytest.mark.parametrize("case", ["chung_lu", "er_planted", "rmat", "multipartite"])
def test_tail_engine_matches_round_kernels(monkeypatch, case, h):
    # the single-workgroup tail engine (the last alive vertices of an h = 3
    # peel over triangle lists, or of an h = 2 peel over the adjacency)
    # against the per-round kernels: the same core numbers, rounds, levels,
    # and the same exact answer from the level table; the third run hands
    # every round with a pair to the grid kernel (the engine stops and
    # resumes around each), the default hands over rounds of more than 2^18
    # pairs (the multipartite graph's last level)
    if case == "chung_lu":
        n, s, d = synth.chung_lu(n=60000, avg_deg=14, beta=2.1, planted=2, plant_size=80, p=0.6, seed=5)
    elif case == "er_planted":
        n, s, d = synth.er_planted(seed=2)
    elif case == "rmat":
        n, s, d = synth.rmat(scale=15, seed=3)
    else:
        n, s, d, _ = synth.complete_multipartite([30, 40, 50, 60, 70], seed=4)
    s = np.ascontiguousarray(s, np.int32)
    d = np.ascontiguousarray(d, np.int32)
    res, grid = {}, {}
    for mode, flag, heavy in (("rounds", "0", None), ("engine", "1", None), ("grid", "1", "0")):
        monkeypatch.setenv("DSD_TAIL_ENGINE", flag)
        if heavy is None:
            monkeypatch.delenv("DSD_TE_GRID_PAIRS", raising=False)
        else:
            monkeypatch.setenv("DSD_TE_GRID_PAIRS", heavy)
        g = dsd.build_csr(n, s, d)
        core, km = dsd.clique_core(g, h)
        st = g.stats()
        grid[mode] = (st["k4_tail_launches"], st["k4_tail_grid_rounds"])
        mem, rho = dsd.core_exact(g, h)
        _, km_app, dens_app = dsd.core_app(g, h)
        res[mode] = (core, km, st["peel_rounds"], st["peel_levels"], rho, km_app, dens_app)
    for mode in ("engine", "grid"):
        np.testing.assert_array_equal(res["rounds"][0], res[mode][0])
        assert res["rounds"][1:] == res[mode][1:]
    assert grid["rounds"] == (0, 0)
    launches, rounds = grid["grid"]
    assert launches == rounds + 1 and rounds > 0
    if case == "multipartite" and h == 3:
        assert grid["engine"][1] > 0


def test_h2_large_rounds_match_oracle():
    # the first rounds of this classic core decomposition remove more than
    # 16,384 vertices and a sixteenth of the alive ones each, so the peel
    # counts them from the alive side; core numbers, k_max and the level
    # count against the oracle's bucket-queue peel
    n, s, d = synth.chung_lu(n=200000, avg_deg=10, beta=2.3, planted=2, plant_size=50, p=0.6, seed=11)
    s = np.ascontiguousarray(s, np.int32)
    d = np.ascontiguousarray(d, np.int32)
    og = oracle.Graph(n, s, d)
    core_o, km_o = og.core_decomposition(2)
    g = dsd.build_csr(n, s, d)
    core_g, km_g = dsd.clique_core(g, 2)
    assert km_g == km_o
    np.testing.assert_array_equal(core_g, core_o)
    _, km_app, _ = dsd.core_app(g, 2)
    assert km_app == km_o


def test_bad_arguments():
    g = dsd.build_csr(3, np.array([0, 1], np.int32), np.array([1, 2], np.int32))
    for h in (0, 1, 7):
        with pytest.raises(dsd.DsdError) as e:
            dsd.clique_degrees(g, h)
        assert e.value.status == -1
    with pytest.raises(dsd.DsdError) as e:
        dsd.build_csr(3, np.array([0, 3], np.int32), np.array([1, 2], np.int32))
    assert e.value.status == -1
    with pytest.raises(dsd.DsdError) as e:
        dsd.build_csr(3, np.array([0, -1], np.int32), np.array([1, 2], np.int32))
    assert e.value.status == -1


# ------------------------------------------------------------------ configuration-shaped graphs

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_er_planted_config(seed):
    n, s, d = synth.er_planted(seed=seed)
    for h in (2, 3):
        check_all(n, s, d, h)


@pytest.mark.parametrize("seed", [1, 2])
def test_chung_lu_medium(seed):
    n, s, d = synth.chung_lu(n=30000, avg_deg=12, beta=2.1, planted=2, plant_size=60, p=0.7, seed=seed)
    check_all(n, s, d, 3)
    check_all(n, s, d, 4, exact=False)


@pytest.mark.parametrize("scale,h", [(11, 4), (11, 5), (12, 4), (10, 6)])
def test_rmat_small(scale, h):
    n, s, d = synth.rmat(scale=scale, edge_factor=16, seed=scale)
    check_all(n, s, d, h, exact=False)


def test_device_buffers():
    torch = pytest.importorskip("torch")
    n, s, d = synth.er_planted(seed=4)
    og = oracle.Graph(n, s, d)
    ts, td = torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda()
    g = dsd.build_csr(n, ts, td)
    out = torch.zeros(n, dtype=torch.uint64, device="cuda")
    dsd.clique_degrees(g, 3, out=out)
    deg_o, _ = og.clique_degrees(3)
    np.testing.assert_array_equal(out.cpu().numpy(), deg_o)
    dsd.clique_core(g, 3, out=out)
    core_o, _ = og.core_decomposition(3)
    np.testing.assert_array_equal(out.cpu().numpy(), core_o)
    mem = torch.zeros(n, dtype=torch.uint8, device="cuda")
    _, km, _ = dsd.core_app(g, 3, out=mem)
    m_o, km_o, _ = og.inc_app(3)
    assert km == km_o
    np.testing.assert_array_equal(mem.cpu().numpy().astype(bool), m_o)


def test_repeat_calls_are_identical():
    n, s, d = synth.chung_lu(n=20000, avg_deg=10, beta=2.3, planted=1, plant_size=50, p=0.6, seed=9)
    g = dsd.build_csr(n, s, d)
    ref = [dsd.clique_degrees(g, 3)[0].copy(), dsd.clique_core(g, 3)[0].copy()]
    for _ in range(3):
        np.testing.assert_array_equal(dsd.clique_degrees(g, 3)[0], ref[0])
        np.testing.assert_array_equal(dsd.clique_core(g, 3)[0], ref[1])


# ------------------------------------------------------------------ h = 3 without triangle lists

@pytest.mark.parametrize("case", ["er", "chung_lu", "multipartite", "random"])
def test_triangle_peel_without_lists(monkeypatch, case):
    # DSD_TRI_LIST=0: the h = 3 peel intersects neighbourhoods (hashes, chunk
    # and wide items) instead of walking triangle lists; same results
    monkeypatch.setenv("DSD_TRI_LIST", "0")
    if case == "er":
        n, s, d = synth.er_planted(seed=2)
    elif case == "chung_lu":
        n, s, d = synth.chung_lu(n=30000, avg_deg=12, beta=2.1, planted=2, plant_size=60, p=0.7, seed=3)
    elif case == "multipartite":
        n, s, d, _ = synth.complete_multipartite([40, 30, 25, 20, 10], seed=1)
    else:
        rng = np.random.default_rng(77)
        e = np.asarray([(u, v) for u in range(60) for v in range(u + 1, 60) if rng.random() < 0.3], np.int32)
        n, s, d = 60, e[:, 0].copy(), e[:, 1].copy()
    gg = check_all(n, s, d, 3, exact=(case != "chung_lu"))
    og = oracle.Graph(n, s, d)
    mem_o, rho_o, steps_o, best_o = og.peel_app(3)
    mem_g, rho_g, rounds_g, best_g = dsd.peel_app(gg, 3)
    assert (rho_g, rounds_g, best_g) == (rho_o, steps_o, best_o)
    np.testing.assert_array_equal(mem_g.astype(bool), mem_o)
