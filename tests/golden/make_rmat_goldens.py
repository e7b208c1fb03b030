"""Write the oracle's expected values for the R-MAT family (scales 16 and 18).

The oracle takes minutes to hours on these graphs (it lists every clique one
by one, single-threaded), so its outputs are computed once by this script and
stored beside it; the GPU parity tests compare the library with them element
by element.  Only ``oracle/`` computes anything here; ``synth`` draws the
edge list.  Every file records what it was computed from: generator,
parameters, seed, h, and a SHA-256 of the generated edge list, which the tests
recompute before trusting the file.

    python tests/golden/make_rmat_goldens.py --scale 16 --h 4 [--exact]

Output: ``tests/golden/rmat{scale}_h{h}.npz`` holding
  deg, core      -- uint64[n] clique-degrees (Def. 3) and core numbers (Def. 6, Alg. 3)
  levels, rsize, rmu -- the level table: every distinct core value k, |R_k|, mu(R_k)
  label          -- int32[n] component of R_{k'} (Pruning2), -1 outside
  meta           -- a JSON string: mu, kmax, rho', k', rho'', k'', CoreApp's
                    (IncApp's) density, and, with --exact, rho_opt (Alg. 4)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1906_00341_amd import synth  # noqa: E402

GEN = dict(edge_factor=16, a=0.57, b=0.19, c=0.19, seed=1)


def edge_hash(s: np.ndarray, d: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(s, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(d, dtype=np.int32).tobytes())
    return h.hexdigest()


def path_for(scale: int, h: int) -> str:
    return os.path.join(HERE, f"rmat{scale}_h{h}.npz")


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--scale", type=int, required=True)
    ap.add_argument("--h", type=int, required=True)
    ap.add_argument("--exact", action="store_true", help="also run the oracle's CoreExact (Alg. 4)")
    a = ap.parse_args()
    t0 = time.time()
    n, s, d = synth.rmat(scale=a.scale, **GEN)
    og = oracle.Graph(n, s, d)
    meta = dict(generator="rmat", scale=a.scale, **GEN, h=a.h, n=n, m=int(og.m), edges_sha256=edge_hash(s, d))
    deg, mu = og.clique_degrees(a.h)
    print(f"degrees mu={mu} {time.time() - t0:.0f}s", flush=True)
    core, kmax = og.core_decomposition(a.h)
    print(f"cores kmax={kmax} {time.time() - t0:.0f}s", flush=True)
    levels, rsize, rmu = og.level_table(a.h, core)
    loc = og.locate(a.h, core)
    mem, km2, dens = og.inc_app(a.h)
    assert km2 == kmax
    meta.update(mu=int(mu), kmax=int(kmax), nlevels=int(levels.size),
                rho1=[loc["rho1"].numerator, loc["rho1"].denominator], k1=loc["k1"],
                rho2=[loc["rho2"].numerator, loc["rho2"].denominator], k2=loc["k2"],
                ncomp=loc["ncomp"], app_density=[dens.numerator, dens.denominator],
                app_size=int(mem.sum()))
    print(f"locate {meta['rho1']} {meta['rho2']} {time.time() - t0:.0f}s", flush=True)

    def save():
        meta["oracle_seconds"] = round(time.time() - t0, 1)
        np.savez_compressed(path_for(a.scale, a.h), deg=deg.astype(np.uint64), core=core.astype(np.uint64),
                            levels=levels.astype(np.uint64), rsize=rsize.astype(np.uint64),
                            rmu=rmu.astype(np.uint64), label=loc["label"].astype(np.int32),
                            meta=np.array(json.dumps(meta)))
        print(json.dumps(meta), flush=True)

    save()
    if a.exact:
        mem_x, rho, calls = og.exact(a.h, "core")
        meta.update(rho_opt=[rho.numerator, rho.denominator], cds_size=int(mem_x.sum()))
        print(f"exact {rho} {time.time() - t0:.0f}s", flush=True)
        save()
    return 0


if __name__ == "__main__":
    sys.exit(main())
