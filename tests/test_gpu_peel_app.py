"""GPU parity of PeelApp (Algorithm 2, every minimum-degree vertex per round)
through the C ABI against the CPU oracle's round-synchronous PeelApp.

The process is deterministic, so the member set, the density (an exact
rational), the number of rounds and the round before which the answer was
seen must all match exactly.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1906_00341_amd import dsd, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    dsd.load()          # fails loudly when the library is missing


def check(n, s, d, hs):
    s = np.ascontiguousarray(s, np.int32)
    d = np.ascontiguousarray(d, np.int32)
    og = oracle.Graph(n, s, d)
    gg = dsd.build_csr(n, s, d)
    for h in hs:
        mem_o, rho_o, steps_o, best_o = og.peel_app(h, rounds=True)
        mem_g, rho_g, rounds_g, best_g = dsd.peel_app(gg, h)
        assert (rho_g, rounds_g, best_g) == (rho_o, steps_o, best_o), h
        np.testing.assert_array_equal(mem_g.astype(bool), mem_o)
    return og, gg


@pytest.mark.parametrize("name", ["F1", "F2", "F4"])
def test_paper_examples(fixtures, name):
    f = fixtures[name]
    e = np.asarray(f["edges"], np.int32)
    check(f["n"], e[:, 0], e[:, 1], (2, 3, 4))


def test_fig6_trace(fixtures):
    # the residual graph before round 1 (the pendant edge gone) is the 3-core, 25/12
    f = fixtures["F4"]
    e = np.asarray(f["edges"], np.int32)
    g = dsd.build_csr(f["n"], e[:, 0].copy(), e[:, 1].copy())
    mem, rho, rounds, best = dsd.peel_app(g, 2)
    assert (rho, rounds, best) == (Fraction(25, 12), 5, 1)
    assert np.nonzero(mem)[0].tolist() == list(range(12))


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("h", [2, 3, 4, 5, 6])
def test_random_small(seed, h):
    rng = np.random.default_rng(700 + seed)
    n = 40
    pairs = [(u, v) for u, v in itertools.combinations(range(n), 2) if rng.random() < 0.35]
    e = np.asarray(pairs, np.int32)
    check(n, e[:, 0], e[:, 1], (h,))


@pytest.mark.parametrize("n", [0, 1, 2, 5])
def test_tiny_and_empty(n):
    e = np.asarray(list(itertools.combinations(range(n), 2)) or np.zeros((0, 2)), np.int32).reshape(-1, 2)
    check(n, e[:, 0], e[:, 1], (2, 3, 6))


def test_graph_without_cliques():
    # a path: no triangle anywhere, so no residual graph has positive density
    n = 50
    s = np.arange(n - 1, dtype=np.int32)
    g = dsd.build_csr(n, s, s + 1)
    mem, rho, rounds, best = dsd.peel_app(g, 3)
    assert rho == 0 and best == -1 and not mem.any() and rounds == 1
    check(n, s, s + 1, (2, 3))


@pytest.mark.parametrize("h", [2, 3, 5])
def test_complete_graph(h):
    n, s, d = synth.complete_graph(30)
    check(n, s, d, (h,))


@pytest.mark.parametrize("parts", [[40, 30, 25, 20, 10], [18, 18, 12, 12, 3]])
def test_complete_multipartite(parts):
    # a part leaves whole; equal parts leave in the same round
    n, s, d, _ = synth.complete_multipartite(parts, seed=3)
    check(n, s, d, (2, 3, 4))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_er_planted_config(seed):
    n, s, d = synth.er_planted(seed=seed)
    check(n, s, d, (2, 3))


@pytest.mark.parametrize("seed", [1, 2])
def test_chung_lu_medium(seed):
    # hubs of degree > 64 take the chunked h = 3 path
    n, s, d = synth.chung_lu(n=30000, avg_deg=12, beta=2.1, planted=2, plant_size=60, p=0.7, seed=seed)
    check(n, s, d, (2, 3, 4))


@pytest.mark.parametrize("scale,h", [(11, 4), (11, 5), (10, 6)])
def test_rmat_small(scale, h):
    n, s, d = synth.rmat(scale=scale, edge_factor=16, seed=scale)
    check(n, s, d, (h,))


def test_device_buffers_and_repeat():
    torch = pytest.importorskip("torch")
    n, s, d = synth.er_planted(seed=4)
    og = oracle.Graph(n, s, d)
    g = dsd.build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda())
    mem_o, rho_o, steps_o, best_o = og.peel_app(3)
    for _ in range(3):
        mem = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
        _, rho, rounds, best = dsd.peel_app(g, 3, out=mem)
        assert (rho, rounds, best) == (rho_o, steps_o, best_o)
        np.testing.assert_array_equal(mem.cpu().numpy().astype(bool), mem_o)
