"""Recycled device memory: handles freed one after another leave their chunks
to the next handle (stale contents must never show), and dsd_release_cache
hands the cache back to the device."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1906_00341_amd import dsd, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    dsd.load()


def _graphs():
    return [synth.chung_lu(n=30000, avg_deg=12, beta=2.2, planted=2, plant_size=60, p=0.6, seed=21),
            synth.er_planted(n=4000, m=30000, plant=80, p=0.5, seed=22),
            synth.chung_lu(n=30000, avg_deg=12, beta=2.2, planted=2, plant_size=60, p=0.6, seed=23)]


def _run(n, s, d, h):
    g = dsd.build_csr(n, np.ascontiguousarray(s, np.int32), np.ascontiguousarray(d, np.int32))
    core, km = dsd.clique_core(g, h)
    _, km_app, dens = dsd.core_app(g, h)
    _, rho = dsd.core_exact(g, h)
    g.free()
    return core, km, km_app, dens, rho


@pytest.mark.parametrize("h", [2, 3])
def test_recycled_memory_between_handles(h):
    graphs = _graphs()
    want = []
    for n, s, d in graphs:
        og = oracle.Graph(n, s, d)
        core_o, km_o = og.core_decomposition(h)
        _, rho_o, _ = og.exact(h, "core")
        want.append((core_o, km_o, rho_o))
    first = []
    for (n, s, d), (core_o, km_o, rho_o) in zip(graphs, want):
        core, km, km_app, dens, rho = _run(n, s, d, h)
        np.testing.assert_array_equal(core, core_o)
        assert km == km_o and km_app == km_o and rho == rho_o
        first.append((core, km, km_app, dens, rho))
    dsd.release_cache()
    # the same graphs again, in the other order, on fresh and then recycled memory
    for i in (2, 0, 1):
        n, s, d = graphs[i]
        core, km, km_app, dens, rho = _run(n, s, d, h)
        np.testing.assert_array_equal(core, first[i][0])
        assert (km, km_app, dens, rho) == first[i][1:]
