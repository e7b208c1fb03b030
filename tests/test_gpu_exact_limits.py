"""The exact step's size limit (Algorithm 4's networks are bounded before they
are built): with the limit lowered through DSD_EXACT_MAX_CLIQUES, a graph
that is one component, and a query on it, are refused with DSD_EUNSUPPORTED
instead of building the network; with the default limit the same calls give
the closed form of the complete graph (rho = C(n, h) / n)."""
from __future__ import annotations

from fractions import Fraction
from math import comb

import numpy as np
import pytest

from paper_1906_00341_amd import dsd, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("h", [2, 3, 4])
def test_limit_refuses_one_component_and_query(h, monkeypatch):
    n, s, d = synth.complete_graph(9)
    g = dsd.build_csr(n, s, d)
    monkeypatch.setenv("DSD_EXACT_MAX_CLIQUES", "5")
    if h >= 3:   # h = 2 networks carry no clique nodes
        with pytest.raises(dsd.DsdError) as e:
            dsd.core_exact(g, h)
        assert e.value.status == -5
        with pytest.raises(dsd.DsdError) as e:
            dsd.core_exact_query(g, h, [3])
        assert e.value.status == -5
    monkeypatch.delenv("DSD_EXACT_MAX_CLIQUES")
    mem, rho = dsd.core_exact(g, h)
    assert rho == Fraction(comb(9, h), 9)
    assert mem.astype(bool).all()
    mem, rho = dsd.core_exact_query(g, h, [3])
    assert rho == Fraction(comb(9, h), 9)
