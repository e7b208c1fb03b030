"""Batches and the server (through the C ABI) against the CPU oracle and
against the single-graph entry points.

A batch peels its graphs as one disjoint union with a level per graph, so
every graph's results must equal the oracle's, and the batch must take
exactly as many peel rounds as its slowest graph takes alone.
"""
from __future__ import annotations

import math
import time
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1906_00341_amd import dsd, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    dsd.load()


def mixed_graphs(seed=0, count=24):
    """Small graphs of the batch workload's family plus degenerate ones."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = i % 6
        if kind == 0:
            out.append(synth.er_planted(n=int(rng.integers(60, 400)), m=int(rng.integers(200, 2000)), plant=20,
                                        p=0.6, seed=seed * 100 + i))
        elif kind in (1, 2):
            out.append(synth.chung_lu(n=int(rng.integers(200, 3000)), avg_deg=float(rng.uniform(4, 16)),
                                      beta=float(rng.uniform(2.0, 3.0)), planted=1, plant_size=20, p=0.7,
                                      seed=seed * 100 + i))
        elif kind == 3:
            out.append(synth.complete_graph(int(rng.integers(3, 25))))
        elif kind == 4:
            n = int(rng.integers(0, 3))                      # empty, single vertex, or one edge
            s = np.array([0], np.int32) if n == 2 else np.zeros(0, np.int32)
            d = np.array([1], np.int32) if n == 2 else np.zeros(0, np.int32)
            out.append((n, s, d))
        else:
            n = int(rng.integers(10, 200))                   # a tree: no triangles
            s = np.arange(1, n, dtype=np.int32)
            d = (rng.integers(0, np.arange(1, n))).astype(np.int32)
            out.append((n, s, d))
    return out


def build_all(graphs):
    return [dsd.build_csr(n, s, d) for n, s, d in graphs]


def density_of(og, h, member):
    idx = np.nonzero(np.asarray(member))[0]
    if idx.size == 0:
        return Fraction(0)
    off, adj = og.adjacency()
    keep = np.zeros(og.n, dtype=bool)
    keep[idx] = True
    rows = np.repeat(np.arange(og.n), np.diff(off))
    e = keep[rows] & keep[adj] & (rows < adj)
    return Fraction(oracle.Graph(og.n, rows[e].astype(np.int32), adj[e].astype(np.int32)).clique_degrees(h)[1],
                    idx.size)


@pytest.mark.parametrize("seed", [1, 2])
def test_batch_core_and_degrees_match_oracle(seed):
    graphs = mixed_graphs(seed)
    hs = [2 + (i % 3) for i in range(len(graphs))]
    handles = build_all(graphs)
    degs = [np.zeros(max(n, 1), np.uint64) for n, _, _ in graphs]
    res = dsd.batch_run(handles, hs, "degrees", outs=degs)
    for (n, s, d), h, r, out in zip(graphs, hs, res, degs):
        og = oracle.Graph(n, s, d)
        deg_o, mu_o = og.clique_degrees(h)
        assert r["status"] == 0 and r["num_cliques"] == mu_o
        np.testing.assert_array_equal(out[:n], deg_o)
    cores = [np.zeros(max(n, 1), np.uint64) for n, _, _ in graphs]
    res = dsd.batch_run(handles, hs, "core", outs=cores)
    for (n, s, d), h, r, out in zip(graphs, hs, res, cores):
        core_o, km_o = oracle.Graph(n, s, d).core_decomposition(h)
        assert r["status"] == 0 and r["kmax"] == km_o
        np.testing.assert_array_equal(out[:n], core_o)


def test_batch_rounds_are_those_of_the_slowest_graph():
    graphs = mixed_graphs(3, count=12)
    h = 3
    alone = []
    for n, s, d in graphs:
        g = dsd.build_csr(n, s, d)
        dsd.clique_core(g, h)
        alone.append(g.stats()["peel_rounds"])
    handles = build_all(graphs)
    res = dsd.batch_run(handles, h, "core")
    assert all(r["status"] == 0 for r in res)
    assert max(r["peel_rounds"] for r in res) == max(alone)


@pytest.mark.parametrize("h", [2, 3, 4])
def test_batch_app_and_exact_match_oracle(h):
    graphs = mixed_graphs(4, count=18)
    handles = build_all(graphs)
    mems = [np.zeros(max(n, 1), np.uint8) for n, _, _ in graphs]
    res = dsd.batch_run(handles, h, "app", outs=mems)
    for (n, s, d), r, out in zip(graphs, res, mems):
        mem_o, km_o, dens_o = oracle.Graph(n, s, d).inc_app(h)
        assert r["status"] == 0 and r["kmax"] == km_o and r["density"] == dens_o
        np.testing.assert_array_equal(out[:n].astype(bool), mem_o)
        assert r["members"] == int(np.count_nonzero(mem_o))
    handles = build_all(graphs)
    mems = [np.zeros(max(n, 1), np.uint8) for n, _, _ in graphs]
    res = dsd.batch_run(handles, h, "exact", outs=mems)
    for (n, s, d), r, out in zip(graphs, res, mems):
        og = oracle.Graph(n, s, d)
        _, rho_o, _ = og.exact(h, "core")
        assert r["status"] == 0 and r["density"] == rho_o
        assert density_of(og, h, out[:n]) == rho_o
        assert r["members"] == int(np.count_nonzero(out[:n]))


@pytest.mark.parametrize("h", [2, 3, 4])
def test_batch_peel_app_matches_oracle(h):
    # every graph of the union removes its own minimum-degree vertices each
    # round; its answer, member set and round count are those of a graph alone
    graphs = mixed_graphs(5, count=24)
    handles = build_all(graphs)
    mems = [np.full(max(n, 1), 9, np.uint8) for n, _, _ in graphs]
    res = dsd.batch_run(handles, h, "peel", outs=mems)
    for (n, s, d), r, out in zip(graphs, res, mems):
        mem_o, rho_o, steps_o, _ = oracle.Graph(n, s, d).peel_app(h, rounds=True)
        assert r["status"] == 0 and r["density"] == rho_o and r["peel_rounds"] == steps_o
        np.testing.assert_array_equal(out[:n].astype(bool), mem_o)
        assert r["members"] == int(np.count_nonzero(mem_o))


def test_batch_device_outputs_and_cached_decomposition():
    torch = pytest.importorskip("torch")
    graphs = mixed_graphs(5, count=10)
    handles = build_all(graphs)
    outs = [torch.zeros(max(n, 1), dtype=torch.uint64, device="cuda") for n, _, _ in graphs]
    res = dsd.batch_run(handles, 3, "core", outs=outs)
    assert all(r["status"] == 0 for r in res)
    for (n, s, d), g, out in zip(graphs, handles, outs):
        og = oracle.Graph(n, s, d)
        core_o, _ = og.core_decomposition(3)
        np.testing.assert_array_equal(out.cpu().numpy()[:n], core_o)
        # the handle keeps the batch's decomposition: single-graph calls reuse it
        core_g, _ = dsd.clique_core(g, 3)
        np.testing.assert_array_equal(core_g, core_o)
        mem, rho = dsd.core_exact(g, 3)
        assert rho == og.exact(3, "core")[1]


def test_batch_argument_errors():
    graphs = mixed_graphs(6, count=3)
    handles = build_all(graphs)
    with pytest.raises(dsd.DsdError) as e:
        dsd.batch_run([handles[0], handles[0]], 3, "core")
    assert e.value.status == -1
    with pytest.raises(dsd.DsdError) as e:
        dsd.batch_run(handles, [3, 7, 3], "core")
    assert e.value.status == -1
    assert dsd.batch_run([], 3, "core") == []


def test_batch_of_chung_lu_graphs_matches_single_calls():
    # the batch workload's generator: n log-uniform, exponent and degree drawn per graph
    specs = synth.batch_specs(count=40, seed=11)
    graphs = [synth.batch_graph(sp) for sp in specs]
    hs = [sp["h"] for sp in specs]
    handles = build_all([(n, s, d) for n, s, d in graphs])
    cores = [np.zeros(max(n, 1), np.uint64) for n, _, _ in graphs]
    res = dsd.batch_run(handles, hs, "core", outs=cores)
    for (n, s, d), h, r, out in zip(graphs, hs, res, cores):
        g = dsd.build_csr(n, s, d)
        core1, km1 = dsd.clique_core(g, h)
        assert r["status"] == 0 and r["kmax"] == km1
        np.testing.assert_array_equal(out[:n], core1)


# ------------------------------------------------------------------ server

def test_server_results_match_single_calls():
    graphs = mixed_graphs(7, count=16)
    handles = build_all(graphs)
    srv = dsd.Server(1 << 34, 64)
    ops = ["degrees", "core", "app", "exact", "peel"]
    tickets, outs = [], []
    for i, g in enumerate(handles):
        n = graphs[i][0]
        op = ops[i % len(ops)]
        out = np.zeros(max(n, 1), np.uint64 if op in ("degrees", "core") else np.uint8)
        outs.append(out)
        tickets.append(srv.submit(g, 3, op, out))
    for i, t in enumerate(tickets):
        st, r = srv.wait(t)
        assert st == 0 and r["status"] == 0
        n, s, d = graphs[i]
        og = oracle.Graph(n, s, d)
        op = ops[i % len(ops)]
        if op == "degrees":
            np.testing.assert_array_equal(outs[i][:n], og.clique_degrees(3)[0])
        elif op == "core":
            np.testing.assert_array_equal(outs[i][:n], og.core_decomposition(3)[0])
        elif op == "app":
            np.testing.assert_array_equal(outs[i][:n].astype(bool), og.inc_app(3)[0])
        elif op == "peel":
            mem_o, rho_o, _, _ = og.peel_app(3)
            assert r["density"] == rho_o
            np.testing.assert_array_equal(outs[i][:n].astype(bool), mem_o)
        else:
            assert r["density"] == og.exact(3, "core")[1]
    with pytest.raises(dsd.DsdError):          # a completed ticket is released by its wait
        srv.wait(tickets[0], 0)
    srv.close()


def test_server_admission_slots_timeout_and_cancel():
    n, s, d = synth.chung_lu(n=200_000, avg_deg=16, beta=2.2, planted=2, plant_size=100, p=0.6, seed=3)
    big = [dsd.build_csr(n, s, d) for _ in range(2)]         # above 2^20 edges: the large-graph worker
    assert big[0].info()[1] >= 1 << 20
    small = [dsd.build_csr(*synth.complete_graph(10)) for _ in range(3)]
    # a request whose footprint exceeds the whole budget is refused
    tiny = dsd.Server(1 << 20, 8)
    with pytest.raises(dsd.DsdError) as e:
        tiny.submit(big[0], 3, "core")
    assert e.value.status == -2
    tiny.close()
    # one slot: taken until the running request completes
    srv = dsd.Server(1 << 34, 1)
    t0 = srv.submit(big[0], 3, "exact")
    with pytest.raises(dsd.DsdError) as e:
        srv.submit(small[0], 3, "core")
    assert e.value.status == dsd.DSD_EBUSY
    st, _ = srv.wait(t0, 0)
    assert st in (0, dsd.DSD_ETIMEDOUT)
    if st == dsd.DSD_ETIMEDOUT:
        st, r = srv.wait(t0)
        assert st == 0 and r["status"] == 0
    t1 = srv.submit(small[1], 3, "core")                     # the slot is free again
    st, r = srv.wait(t1)
    assert st == 0 and r["kmax"] == math.comb(9, 2)
    srv.close()
    # large requests run one at a time: the second waits in the queue and can be cancelled
    srv = dsd.Server(1 << 34, 8)
    ta = srv.submit(big[0], 3, "exact")
    tb = srv.submit(big[1], 3, "core")
    tc = srv.submit(small[2], 3, "core")                     # the small-graph worker is not blocked
    st, r = srv.wait(tc)
    assert st == 0 and r["kmax"] == math.comb(9, 2)
    c = srv.cancel(tb)
    stb, _ = srv.wait(tb)
    if c == 0:
        assert stb == dsd.DSD_ECANCELED
    else:
        assert c == dsd.DSD_EBUSY and stb == 0
    st, r = srv.wait(ta)
    assert st == 0 and r["status"] == 0
    srv.close()


def test_batch_triangles_without_lists(monkeypatch):
    # DSD_TRI_LIST=0: the union's h = 3 peel intersects neighbourhoods instead
    # of walking triangle lists; same results
    monkeypatch.setenv("DSD_TRI_LIST", "0")
    graphs = mixed_graphs(6, count=18)
    handles = build_all(graphs)
    cores = [np.zeros(max(n, 1), np.uint64) for n, _, _ in graphs]
    res = dsd.batch_run(handles, 3, "core", outs=cores)
    for (n, s, d), r, out in zip(graphs, res, cores):
        core_o, km_o = oracle.Graph(n, s, d).core_decomposition(3)
        assert r["status"] == 0 and r["kmax"] == km_o
        np.testing.assert_array_equal(out[:n], core_o)
    mems = [np.zeros(max(n, 1), np.uint8) for n, _, _ in graphs]
    res = dsd.batch_run(build_all(graphs), 3, "peel", outs=mems)
    for (n, s, d), r, out in zip(graphs, res, mems):
        mem_o, rho_o, steps_o, _ = oracle.Graph(n, s, d).peel_app(3)
        assert r["status"] == 0 and r["density"] == rho_o and r["peel_rounds"] == steps_o
        np.testing.assert_array_equal(out[:n].astype(bool), mem_o)


def test_server_staggered_arrivals_match_single_calls_and_oracle():
    """Continuous batching: requests of mixed h (2, 3, 4), op and size arrive
    one by one while earlier ones run on the server's workers (each with its
    own stream).  Every result must be the one the request's single-graph
    entry point gives alone, and the oracle's."""
    import threading
    rng = np.random.default_rng(11)
    graphs = mixed_graphs(5, count=30)
    # two graphs above 2^20 edges: they run alone, beside the small groups
    for k in range(2):
        graphs.append(synth.chung_lu(n=150_000, avg_deg=16, beta=2.3, planted=1, plant_size=60, p=0.7, seed=40 + k))
    ops = ["core", "app", "exact", "degrees", "peel"]
    reqs = []
    for i, (n, s, d) in enumerate(graphs):
        h = int(rng.integers(2, 5))
        op = ops[i % len(ops)]
        if n >= 100_000 and op in ("exact", "peel", "degrees"):
            op = "core"
        reqs.append((i, h, op))
    handles = build_all(graphs)
    outs = [np.zeros(max(graphs[i][0], 1), np.uint64 if op in ("degrees", "core") else np.uint8)
            for i, h, op in reqs]
    srv = dsd.Server(1 << 36, 64)
    tickets = [None] * len(reqs)

    def submitter():
        for j, (i, h, op) in enumerate(reqs):
            tickets[j] = srv.submit(handles[i], h, op, outs[j])
            time.sleep(float(rng.uniform(0.0, 0.01)))

    th = threading.Thread(target=submitter)
    th.start()
    results = [None] * len(reqs)
    for j in range(len(reqs)):
        while tickets[j] is None:
            time.sleep(0.001)
        st, r = srv.wait(tickets[j])
        assert st == 0 and r["status"] == 0, (j, reqs[j], r)
        results[j] = r
    th.join()
    srv.close()
    for j, (i, h, op) in enumerate(reqs):
        n, s, d = graphs[i]
        g1 = dsd.build_csr(n, s, d)                 # the single call, alone, on a fresh handle
        r = results[j]
        if op == "degrees":
            deg1, mu1 = dsd.clique_degrees(g1, h)
            np.testing.assert_array_equal(outs[j][:n], deg1[:n])
            assert r["num_cliques"] == mu1
        elif op == "core":
            core1, km1 = dsd.clique_core(g1, h)
            np.testing.assert_array_equal(outs[j][:n], core1[:n])
            assert r["kmax"] == km1
        elif op == "app":
            mem1, km1, dens1 = dsd.core_app(g1, h)
            np.testing.assert_array_equal(outs[j][:n], mem1[:n])
            assert (r["kmax"], r["density"]) == (km1, dens1)
        elif op == "peel":
            mem1, rho1, rounds1, _ = dsd.peel_app(g1, h)
            np.testing.assert_array_equal(outs[j][:n], mem1[:n])
            assert r["density"] == rho1
        else:
            _, rho1 = dsd.core_exact(g1, h)
            assert r["density"] == rho1
        if n >= 100_000:
            continue                                  # the oracle below: small graphs only
        og = oracle.Graph(n, s, d)
        if op == "degrees":
            np.testing.assert_array_equal(outs[j][:n], og.clique_degrees(h)[0])
        elif op == "core":
            np.testing.assert_array_equal(outs[j][:n], og.core_decomposition(h)[0])
        elif op == "app":
            np.testing.assert_array_equal(outs[j][:n].astype(bool), og.inc_app(h)[0])
        elif op == "peel":
            assert r["density"] == og.peel_app(h)[1]
        else:
            assert r["density"] == og.exact(h, "core")[1]
