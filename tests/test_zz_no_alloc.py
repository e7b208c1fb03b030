"""The allocation-free entry point dsd_clique_degrees_noalloc against
dsd_clique_degrees and the oracle (Definition 3): two calls in a row, the
second on a smaller graph, must both give every clique-degree and mu exactly;
the calls must not change the device's free memory; a graph beyond the fixed
scratch is refused with DSD_EINVAL."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1906_00341_amd import dsd, synth

pytestmark = pytest.mark.gpu


def _pair(g, og, h, device_out=False):
    torch = pytest.importorskip("torch")
    n, _ = g.info()
    if device_out:
        buf = torch.zeros(max(n, 1), dtype=torch.int64, device="cuda")
        _, mu_na = dsd.clique_degrees_noalloc(g, h, out=buf)
        deg_na = buf.cpu().numpy().view(np.uint64)[:n]
    else:
        deg_na, mu_na = dsd.clique_degrees_noalloc(g, h)
    deg_ref, mu_ref = dsd.clique_degrees(g, h)
    deg_o, mu_o = og.clique_degrees(h)
    assert mu_na == mu_ref == mu_o
    np.testing.assert_array_equal(deg_na, deg_ref)
    np.testing.assert_array_equal(deg_na, deg_o)


@pytest.mark.parametrize("h", [2, 3, 4, 5])
def test_two_calls_second_smaller(h):
    n1, s1, d1 = synth.rmat(scale=12, seed=3)
    n2, s2, d2 = synth.er_planted(n=2000, m=10000, plant=60, p=0.4, seed=2)
    g1, g2 = dsd.build_csr(n1, s1, d1), dsd.build_csr(n2, s2, d2)
    o1, o2 = oracle.Graph(n1, s1, d1), oracle.Graph(n2, s2, d2)
    print(f"noalloc h={h}: rmat12 then er2000", flush=True)
    _pair(g1, o1, h)
    _pair(g2, o2, h, device_out=True)
    # the first graph again after the smaller one: nothing stale in the array
    _pair(g1, o1, h, device_out=True)


@pytest.mark.parametrize("k", [900, 1500])
def test_global_bitmap_classes(k):
    """K_900 and K_1500: the roots of out-degree 769 .. 1,280 and 1,281 ..
    2,048 take the kernels whose bitmaps live in the fixed array (their grids
    capped to fit)."""
    n, s, d = synth.complete_graph(k)
    g = dsd.build_csr(n, s, d)
    from math import comb
    for h in ((4, 5) if k < 1281 else (4,)):
        deg, mu = dsd.clique_degrees_noalloc(g, h)
        assert mu == comb(k, h)
        assert (deg == comb(k - 1, h - 1)).all()


def test_no_device_allocation():
    torch = pytest.importorskip("torch")
    n, s, d = synth.rmat(scale=13, seed=5)
    dsd.release_cache()
    g = dsd.build_csr(n, s, d)
    out = torch.zeros(n, dtype=torch.int64, device="cuda")
    dsd.clique_degrees_noalloc(g, 4, out=out)       # first call: the array's address is taken
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for h in (3, 4, 5):
        dsd.clique_degrees_noalloc(g, h, out=out)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0


def test_limit_and_errors():
    n = (1 << 22) + 1
    g = dsd.build_csr(n, np.array([0], np.int32), np.array([1], np.int32))
    with pytest.raises(dsd.DsdError) as e:
        dsd.clique_degrees_noalloc(g, 3)
    assert e.value.status == -1
    g0 = dsd.build_csr(0, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert dsd.clique_degrees_noalloc(g0, 3)[1] == 0
    with pytest.raises(dsd.DsdError) as e:
        dsd.clique_degrees_noalloc(g0, 7)
    assert e.value.status == -1
