"""The R-MAT family at h = 4 and 5, element by element against the oracle.

R-MAT graphs of scales 16 and 18 (edge factor 16, (a, b, c, d) = (0.57, 0.19,
0.19, 0.05), the generator of the scale-22 benchmark graph; the paper's own
synthetic R-MAT graph, section 8, scaled).  The oracle needs minutes to
hours to list their 10^8 - 10^10 cliques one by one, so its outputs are
stored by tests/golden/make_rmat_goldens.py (which calls only the oracle);
each file carries the SHA-256 of the edge list it was computed from, checked
here before the file is trusted.

Compared exactly: every clique-degree and mu (Definition 3), every core
number and k_max (Definition 6, Algorithm 3), CoreApp's member set and
density (Algorithm 6: the whole (k_max, Psi)-core), and the locate step of
CoreExact (Pruning1/2, section 6.1: rho', k', rho'', k'', the number of
components of R_{k'} and |R_{k''}|).  Their located cores hold 10^8 and more
cliques, beyond the exact step's limit, which refuses them with
DSD_EUNSUPPORTED after the locate step; the refusal is checked too.
"""
from __future__ import annotations

import glob
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_1906_00341_amd import dsd, synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = sorted(glob.glob(os.path.join(HERE, "golden", "rmat*_h*.npz")))


def _edge_hash(s, d):
    import hashlib
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(s, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(d, dtype=np.int32).tobytes())
    return h.hexdigest()


_graphs = {}


def _graph(meta):
    key = (meta["scale"], meta["seed"])
    if key not in _graphs:
        torch = pytest.importorskip("torch")
        n, s, d = synth.rmat(scale=meta["scale"], edge_factor=meta["edge_factor"], a=meta["a"], b=meta["b"],
                             c=meta["c"], seed=meta["seed"])
        assert n == meta["n"]
        assert _edge_hash(s, d) == meta["edges_sha256"], "generator output differs from the stored oracle run"
        _graphs.clear()
        _graphs[key] = dsd.build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda())
    return _graphs[key]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("path", GOLDEN, ids=[os.path.basename(p)[:-4] for p in GOLDEN])
def test_rmat_family_against_oracle(path):
    z = np.load(path, allow_pickle=False)
    meta = json.loads(str(z["meta"]))
    h = meta["h"]
    print(f"{os.path.basename(path)}: n={meta['n']} m={meta['m']} mu={meta['mu']} kmax={meta['kmax']}", flush=True)
    g = _graph(meta)
    assert g.info()[1] == meta["m"]

    deg, mu = dsd.clique_degrees(g, h)
    assert mu == meta["mu"]
    np.testing.assert_array_equal(deg, z["deg"])

    core, km = dsd.clique_core(g, h)
    assert km == meta["kmax"]
    np.testing.assert_array_equal(core, z["core"])

    mem, km2, dens = dsd.core_app(g, h)
    assert km2 == meta["kmax"]
    np.testing.assert_array_equal(mem.astype(bool), z["core"] == meta["kmax"])
    assert dens == Fraction(*meta["app_density"])

    try:
        mem_x, rho = dsd.core_exact(g, h)
        refused = False
    except dsd.DsdError as e:
        assert e.status == -5, e
        refused = True
    st = g.stats()
    print(f"  locate: rho'={st['locate_rho1_num']}/{st['locate_rho1_den']} k''={st['locate_k2']} "
          f"located={st['located_vertices']} exact={'refused' if refused else rho}", flush=True)
    assert Fraction(st["locate_rho1_num"], st["locate_rho1_den"]) == Fraction(*meta["rho1"])
    assert st["locate_k1"] == meta["k1"]
    assert Fraction(st["locate_rho2_num"], st["locate_rho2_den"]) == Fraction(*meta["rho2"])
    assert st["locate_k2"] == meta["k2"]
    assert st["locate_components"] == meta["ncomp"]
    assert st["located_vertices"] == int((z["core"] >= meta["k2"]).sum())
    if not refused and "rho_opt" in meta:
        assert rho == Fraction(*meta["rho_opt"])
