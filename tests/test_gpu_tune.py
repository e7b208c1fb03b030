"""Launch tuning of the clique enumeration (dsd_autotune): every class of
roots present is timed under several grid caps, the fastest kept per
(architecture, h, class) and written to a JSON file; clique-degrees with the
tuned caps, with caps loaded back from the file, and with extreme caps must
equal the built-in ones' and the oracle's (Definition 3)."""
from __future__ import annotations

import json

import numpy as np
import pytest

import oracle
from paper_1906_00341_amd import dsd, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("h", [3, 4, 5])
def test_tuned_caps_give_identical_results(tmp_path, h):
    n, s, d = synth.rmat(scale=12, seed=20 + h)
    g = dsd.build_csr(n, s, d)
    dsd.tune_load(None)
    deg0, mu0 = dsd.clique_degrees(g, h)
    deg_o, mu_o = oracle.Graph(n, s, d).clique_degrees(h)
    np.testing.assert_array_equal(deg0, deg_o)
    assert mu0 == mu_o

    path = tmp_path / "tune.json"
    res = dsd.autotune(g, h, str(path))
    assert res, "no class measured"
    for r in res:
        assert r["roots"] > 0 and r["cap_best"] >= 1 and r["ms_best"] <= r["ms_default"] + 1e-9
    table = json.loads(path.read_text())
    keys = [k for k in table if k.endswith(tuple(f"/h{h}/c{r['cls']}" for r in res))]
    assert len(keys) == len(res)
    deg1, mu1 = dsd.clique_degrees(g, h)                  # the tuned table is in use
    np.testing.assert_array_equal(deg1, deg0)
    assert mu1 == mu0

    dsd.tune_load(None)
    dsd.tune_load(str(path))                              # back from the file
    deg2, mu2 = dsd.clique_degrees(g, h)
    np.testing.assert_array_equal(deg2, deg0)

    # extreme caps: one workgroup per class, and far more than the roots
    arch = next(iter(table)).split("/")[0]
    for cap in (1, 60000):
        path.write_text(json.dumps({f"{arch}/h{h}/c{c}": cap for c in range(5)}))
        dsd.tune_load(str(path))
        deg3, mu3 = dsd.clique_degrees(g, h)
        np.testing.assert_array_equal(deg3, deg0)
        core3, _ = dsd.clique_core(dsd.build_csr(n, s, d), h)
        core_o, _ = oracle.Graph(n, s, d).core_decomposition(h)
        np.testing.assert_array_equal(core3, core_o)
    dsd.tune_load(None)
    g.free()


def test_tune_merges_into_existing_file(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text('{"otherarch/h4/c1": 77}')
    n, s, d = synth.rmat(scale=11, seed=3)
    g = dsd.build_csr(n, s, d)
    dsd.autotune(g, 4, str(path))
    table = json.loads(path.read_text())
    assert table["otherarch/h4/c1"] == 77
    assert any(k.endswith("/h4/c0") for k in table)
    dsd.tune_load(None)
    with pytest.raises(dsd.DsdError):
        dsd.autotune(g, 2, None)
    g.free()
