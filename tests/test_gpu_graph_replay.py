"""The peel's rounds replayed from a captured HIP graph (DSD_PEEL_GRAPH=1).

Every round of a peel is the same kernel sequence reading its state from
the device, so the library can capture one round once (again after every
compaction of the adjacency, a kernel argument) and replay it round after
round, with the host's own synchronisations (the alive count it polls
between batches of rounds) and eager work (compaction, tail mode) in
between.  Each case runs eagerly and with replays and must give identical
core numbers, k_max, level counts, CoreApp sets and batch results; the
eager results are the oracle's (Algorithm 3, Definition 6).
"""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
from paper_1906_00341_amd import dsd, synth

pytestmark = pytest.mark.gpu


def _both(fn):
    old = os.environ.pop("DSD_PEEL_GRAPH", None)
    try:
        eager = fn()
        os.environ["DSD_PEEL_GRAPH"] = "1"
        replayed = fn()
    finally:
        os.environ.pop("DSD_PEEL_GRAPH", None)
        if old is not None:
            os.environ["DSD_PEEL_GRAPH"] = old
    return eager, replayed


@pytest.mark.parametrize("h", [2, 3, 4, 5, 6])
def test_rmat_cores_replayed(h):
    n, s, d = synth.rmat(scale=12, seed=h)

    def run():
        g = dsd.build_csr(n, s, d)
        core, km = dsd.clique_core(g, h)
        st = g.stats()
        mem, km2, dens = dsd.core_app(g, h)
        g.free()
        return core, km, st["peel_rounds"], st["peel_levels"], mem, dens

    a, b = _both(run)
    np.testing.assert_array_equal(a[0], b[0])
    assert a[1:4] == b[1:4]
    np.testing.assert_array_equal(a[4], b[4])
    assert a[5] == b[5]
    core_o, km_o = oracle.Graph(n, s, d).core_decomposition(h)
    np.testing.assert_array_equal(a[0], core_o)
    assert a[1] == km_o


def test_compaction_and_tail_replayed():
    """A Chung-Lu graph large enough to compact its adjacency several times
    and to switch to tail mode: both graphs are captured, the plain one more
    than once."""
    n, s, d = synth.chung_lu(n=60_000, avg_deg=12.0, beta=2.2, planted=2, plant_size=80, p=0.6, seed=3)
    for h in (2, 4):
        def run():
            g = dsd.build_csr(n, s, d)
            core, km = dsd.clique_core(g, h)
            rounds = g.stats()["peel_rounds"]
            g.free()
            return core, km, rounds
        a, b = _both(run)
        np.testing.assert_array_equal(a[0], b[0])
        assert a[1:] == b[1:]


def test_batch_replayed():
    specs = synth.batch_specs(count=64, seed=11)[:48]
    graphs = [synth.batch_graph(sp) for sp in specs]
    hs = [sp["h"] for sp in specs]

    def run():
        hd = [dsd.build_csr(n, s, d) for n, s, d in graphs]
        res = dsd.batch_run(hd, hs, "core")
        out = [(r["status"], r["kmax"], r["num_cliques"], r["peel_rounds"]) for r in res]
        for g in hd:
            g.free()
        return out

    a, b = _both(run)
    assert a == b
    assert all(x[0] == 0 for x in a)
