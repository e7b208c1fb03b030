#!/usr/bin/env python3
"""Benchmark of the whole densest-subgraph hot path on one MI355X.

One step = one pass of every stage over one synthetic graph whose edge list
is already resident in HBM: CSR build and degree-ordered orientation, clique
enumeration (clique-degrees), the (k, Psi)-core peel, CoreApp, and CoreExact
(locating on the GPU, exact minimum cuts on the host).  CoreExact reuses the
decomposition the handle already holds from the clique-core call.  The workload is a
Chung-Lu power-law graph, n = 1,000,000, average degree 20, exponent 2.1,
with 5 planted 200-vertex blocks at pair probability 0.7, and the triangle
(h = 3) as the clique.

Prints one JSON line.  ``value`` is whole-pass throughput in h-cliques/s
(mu(G, Psi) divided by the time of one step).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "h-cliques/s + peel edges/s on 1 GPU, %HBM peak; batched & served vs plain"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # the configuration the metric is quoted on
    "chung_lu_1e6": dict(gen="chung_lu", h=3, kw=dict(n=1_000_000, avg_deg=20.0, beta=2.1, planted=5,
                                                     plant_size=200, p=0.7)),
    # the small configuration (quick runs)
    "er_2000": dict(gen="er_planted", h=2, kw=dict(n=2000, m=10000, plant=60, p=0.4)),
}


def make_graph(name: str, seed: int):
    from paper_1906_00341_amd import synth
    w = WORKLOADS[name]
    return getattr(synth, w["gen"])(seed=seed, **w["kw"]), w["h"]


def k3_bytes(st: dict) -> float:
    """Algorithmic bytes of one whole-graph clique-degree pass (h = 3): every
    directed 2-path r -> v -> x reads one out-list entry (4 B), plus per edge
    the row pointers / staged out-list / flushed counters (24 B) and 8 B of
    output per vertex."""
    return 4.0 * st["w2"] + 24.0 * st["m"] + 8.0 * st["n"]


def k4_bytes(st: dict, h: int) -> float:
    """Algorithmic bytes of one full peel: h = 3 reads the out-list of every
    neighbour of every removed vertex (4 B per entry of sum_v deg(v) d+(v)),
    stages N(v) (8 B per edge) and decrements survivors (16 B per edge);
    h = 2 touches every edge from both ends (32 B per edge)."""
    if h == 2:
        return 32.0 * st["m"]
    return 4.0 * st["s2"] + 24.0 * st["m"]


# the peel's main kernel by the kind the library reports
MAIN_KERNEL = {1: "k_process_h2", 2: "k_h3_probe", 3: "k_tl_process", 4: "k_star_front"}


def main_kernel_bytes(st: dict) -> float:
    """Algorithmic bytes of the peel's main kernel over one peel, from the
    work it counted.  Triangle lists (k_tl_process): every walked pair
    (a, b) costs itself and the removal stamps of a and b (8 + 4 + 4 B),
    every row item its descriptor and the row's two offsets (8 + 16 B).
    Triangle probe (k_h3_probe): every probed out-list entry costs 4 B,
    every expanded neighbour w its column entry and the two row offsets of
    N+(w) (4 + 8 + 8 B).  Edge pass (k_process_h2, h = 2): every walked
    adjacency entry costs its column entry, the neighbour's stamp and an
    8-byte read-modify-write of its degree (4 + 4 + 16 B), every frontier
    vertex its two row offsets (16 B)."""
    kind = st["k4_main_kind"]
    if kind == 1:
        return 24.0 * st["k4_main_pairs"] + 16.0 * st["k4_main_nbrs"]
    if kind == 3:
        return 16.0 * st["k4_main_pairs"] + 24.0 * st["k4_main_nbrs"]
    return 4.0 * st["k4_main_pairs"] + 20.0 * st["k4_main_nbrs"]


TAIL_KERNEL = "k_tail_engine"


def tail_kernel_bytes(st: dict) -> float:
    """Algorithmic bytes of the h = 3 tail engine over one peel: every pair it
    walks is one 4-byte word of the rewritten rows; every tail vertex costs its
    degree and id in (8 + 4 B), its two row offsets (16 B), its id again and
    its core number out (4 + 8 B); every round handed to the grid costs each
    tail vertex its degree and state out (5 B) and back in with its row start
    (13 B).  The degrees and states stay in LDS while the engine runs."""
    return (4.0 * st["k4_tail_pairs"] + 40.0 * st["k4_tail_vertices"]
            + 18.0 * st["k4_tail_vertices"] * st["k4_tail_grid_rounds"])


PEEL_SOURCE = os.path.join(ROOT, "paper_1906_00341_amd", "csrc", "peel.hip")


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of kernel on workload from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of
    known size), or None when there is none or the peel's source has changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", "|", " ")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    sha = hashlib.sha256(open(PEEL_SOURCE, "rb").read()).hexdigest()
    if fields.get("kernel_source_sha256") != sha or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def cpu_baseline(workload: str, seed: int):
    """The CPU oracle, single-threaded, on a bounded sample of the same
    workload.  Chung-Lu: the same generator at n = 600,000 (same degree law
    and planted blocks), clique-degrees + core decomposition + CoreApp; the
    oracle's exact step (Dinic on 128-bit capacities over the whole located
    core) alone runs for many minutes on this graph family, so it is left out
    of the sample.  ER: the whole 2,000-vertex graph and the whole path."""
    import oracle
    from paper_1906_00341_amd import synth
    w = WORKLOADS[workload]
    h = w["h"]
    if workload == "er_2000":
        n, s, d = synth.er_planted(seed=seed, **w["kw"])
        stages = "clique-degrees + core decomposition + CoreApp + CoreExact"
    else:
        kw = dict(w["kw"], n=600_000)
        n, s, d = synth.chung_lu(seed=seed, **kw)
        stages = "clique-degrees + core decomposition + CoreApp"
    g = oracle.Graph(n, s, d)
    t0 = time.perf_counter()
    _, mu = g.clique_degrees(h)
    g.core_decomposition(h)
    g.core_app(h)
    if workload == "er_2000":
        g.exact(h, "core")
    t = time.perf_counter() - t0
    return {"value": mu / t, "unit": "h-cliques/s", "cores": 1, "kind": "oracle",
            "sample": f"{workload} generator at n={n} (m={g.m}, mu={mu}); {stages}; {t:.2f} s, one thread"}


def batch_leg(n_graphs: int, seed: int):
    """Batched vs plain on a bounded sample of the batched mixture (n
    log-uniform in [100, 50000], Chung-Lu exponent U[2, 3], average degree
    U[4, 40], h in {2, 3, 4}): the first n_graphs graphs of the 8192-graph
    mixture.  Op: the (k, Psi)-core decomposition.  Plain = one
    dsd_clique_core call per graph; batched = one dsd_batch_run."""
    import torch
    from paper_1906_00341_amd import dsd, synth
    specs = synth.batch_specs(count=8192, seed=seed)[:n_graphs]
    graphs = [synth.batch_graph(sp) for sp in specs]
    hs = [sp["h"] for sp in specs]
    handles = []
    for n, s, d in graphs:
        handles.append(dsd.build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda()))
    torch.cuda.synchronize()
    mu = 0
    t0 = time.perf_counter()
    for g, h in zip(handles, hs):
        _, km = dsd.clique_core(g, h)
        mu += g.stats()["num_cliques"]
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    res = dsd.batch_run(handles, hs, "core")
    t_batch = time.perf_counter() - t0
    assert all(r["status"] == 0 for r in res)
    assert sum(r["num_cliques"] for r in res) == mu
    m = sum(g.info()[1] for g in handles)
    for g in handles:
        g.free()
    return {"graphs": n_graphs, "of": 8192, "edges": m, "h_cliques": mu, "op": "core",
            "plain_s": t_plain, "batched_s": t_batch,
            "plain_graphs_per_s": n_graphs / t_plain, "batched_graphs_per_s": n_graphs / t_batch,
            "plain_h_cliques_per_s": mu / t_plain, "batched_h_cliques_per_s": mu / t_batch,
            "speedup": t_plain / t_batch,
            "peel_rounds_batched": max(r["peel_rounds"] for r in res)}


def serve_leg(n_requests: int, seed: int):
    """The server under load: requests drawn 95 % from the batched mixture and
    5 % from R-MAT scale 20 (a = 0.57, b = c = 0.19), h in {2, 3, 4}, ops 70 %
    CoreApp, 20 % core decomposition, 10 % CoreExact (R-MAT requests: CoreApp
    only, whose cost does not depend on the located core).  Pass 1 submits
    everything at once (saturation throughput); pass 2 submits with Poisson
    arrivals at half that rate and records each request's latency.  Plain =
    the same requests as sequential single-graph calls."""
    import concurrent.futures as cf
    import numpy as np
    import torch
    from paper_1906_00341_amd import dsd, synth
    rng = np.random.default_rng(seed)
    specs = synth.batch_specs(count=8192, seed=seed + 1)
    n_rmat = max(1, n_requests // 20)
    reqs = []
    rn, rs, rd = synth.rmat(scale=20, edge_factor=16, seed=seed)
    rmat_graph = (rn, rs, rd)
    for i in range(n_requests):
        if i < n_rmat:
            reqs.append((rmat_graph, int(rng.integers(2, 5)), "app"))
        else:
            sp = specs[i]
            u = rng.random()
            op = "app" if u < 0.7 else ("core" if u < 0.9 else "exact")
            reqs.append((synth.batch_graph(sp), sp["h"], op))
    order = rng.permutation(n_requests)
    reqs = [reqs[i] for i in order]

    def build():
        return [dsd.build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda()) for (n, s, d), _, _ in reqs]

    handles = build()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g, (_, h, op) in zip(handles, reqs):
        {"app": dsd.core_app, "core": dsd.clique_core, "exact": dsd.core_exact}[op](g, h)
    t_plain = time.perf_counter() - t0
    for g in handles:
        g.free()

    srv = dsd.Server(64 << 30, 4 * n_requests)

    def run(rate):
        hs = build()
        torch.cuda.synchronize()
        lat = [0.0] * n_requests
        with cf.ThreadPoolExecutor(max_workers=64) as pool:
            futs = []
            start = time.perf_counter()
            t_next = start
            for i, (g, (_, h, op)) in enumerate(zip(hs, reqs)):
                if rate:
                    t_next += rng.exponential(1.0 / rate)
                    delay = t_next - time.perf_counter()
                    if delay > 0:
                        time.sleep(delay)
                t_sub = time.perf_counter()
                tk = srv.submit(g, h, op)

                def waiter(tk=tk, t_sub=t_sub, i=i):
                    st, r = srv.wait(tk)
                    lat[i] = time.perf_counter() - t_sub
                    return st, r

                futs.append(pool.submit(waiter))
            outs = [f.result() for f in futs]
            total = time.perf_counter() - start
        assert all(st == 0 and r["status"] in (0, -5) for st, r in outs)
        for g in hs:
            g.free()
        return total, lat

    t_sat, _ = run(None)
    qps_sat = n_requests / t_sat
    t_half, lat = run(0.5 * qps_sat)
    srv.close()
    lat_ms = np.sort(np.asarray(lat)) * 1000.0
    return {"requests": n_requests, "rmat20_requests": n_rmat, "mix": "70% app / 20% core / 10% exact",
            "plain_qps": n_requests / t_plain, "served_qps_saturation": qps_sat,
            "offered_qps": 0.5 * qps_sat, "served_qps_at_offered": n_requests / t_half,
            "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99))}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="chung_lu_1e6", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-graphs", type=int, default=512,
                    help="graphs of the batched mixture in the batched-vs-plain leg (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=192,
                    help="requests in the serving leg (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path is not sharded "
              f"across GPUs", file=sys.stderr)
        return 2
    import numpy as np
    import torch

    from paper_1906_00341_amd import dsd

    (n, src, dst), h = make_graph(args.workload, args.seed)
    dev = torch.device("cuda:0")
    ts = torch.from_numpy(np.ascontiguousarray(src, np.int32)).to(dev)
    td = torch.from_numpy(np.ascontiguousarray(dst, np.int32)).to(dev)
    core_t = torch.zeros(n, dtype=torch.uint64, device=dev)
    app_t = torch.zeros(n, dtype=torch.uint8, device=dev)
    exact_t = torch.zeros(n, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def step(time_kernels=False):
        rec = {}
        g = dsd.build_csr(n, ts, td)
        rec["build"] = g.stats()
        g.set_kernel_timing(time_kernels)
        _, km = dsd.clique_core(g, h, out=core_t)
        rec["core"] = g.stats()
        rec["kmax"] = km
        _, km2, dens = dsd.core_app(g, h, out=app_t)
        rec["app"] = g.stats()
        _, rho = dsd.core_exact(g, h, out=exact_t)
        rec["exact"] = g.stats()
        rec["rho"] = rho
        rec["m"] = g.info()[1]
        g.free()
        return rec

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        recs.append(step())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1000.0 * wall / args.steps
    # one more step, right after the timed ones, with every launch of the
    # peel's main kernel bracketed by HIP events on the graph's stream (each
    # bracketed launch costs the host ~20 us, so the timed steps run without)
    inst = step(time_kernels=True)["core"]

    core = recs[-1]["core"]
    mu = core["num_cliques"]
    avg = lambda key, stage: sum(r[stage][key] for r in recs) / len(recs)
    k3_ms = avg("k3_ms", "core")
    k4_ms = avg("k4_ms", "core")
    # roofline of the peel's dominant kernel (the round kernels' main kernel or
    # the tail engine, whichever took longer), every launch of the instrumented
    # step timed with HIP events; the other one beside it
    def roof(kernel, total_ms, launches, total_bytes):
        launches = max(launches, 1)
        bytes_call = total_bytes / launches
        ms_call = total_ms / launches
        achieved = bytes_call / (ms_call / 1e3) / 1e9 if ms_call > 0 else 0.0
        return {"kernel": kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kernel, args.workload),
                "bytes_per_launch": bytes_call, "ms_per_launch": ms_call, "launches_per_step": launches,
                "timing": "HIP events around every launch of one extra step after the timed ones"}

    main_roof = roof(MAIN_KERNEL.get(inst["k4_main_kind"]), inst["k4_main_ms"], inst["k4_main_launches"],
                     main_kernel_bytes(inst))
    main_roof.update({"pairs_per_step": inst["k4_main_pairs"], "nbrs_per_step": inst["k4_main_nbrs"]})
    tail_roof = roof(TAIL_KERNEL, inst["k4_tail_ms"], inst["k4_tail_launches"], tail_kernel_bytes(inst))
    tail_roof.update({"pairs_per_step": inst["k4_tail_pairs"], "tail_vertices": inst["k4_tail_vertices"],
                      "grid_rounds": inst["k4_tail_grid_rounds"], "grid_pairs": inst["k4_tail_grid_pairs"],
                      "grid_ms": inst["k4_tail_grid_ms"]})
    if inst["k4_tail_ms"] > inst["k4_main_ms"]:
        dominant, other = tail_roof, main_roof
    else:
        dominant, other = main_roof, tail_roof
    out = {
        "metric": METRIC,
        "value": mu / (ms_per_step / 1e3),
        "unit": "h-cliques/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": args.workload, "h": h, "n": n, "m": recs[-1]["m"], "seed": args.seed,
                   "num_cliques": mu, "kmax": recs[-1]["kmax"], "rho_opt": str(recs[-1]["rho"])},
        "stages_ms": {
            "build_orient": avg("t_total_ms", "build"),
            "clique_degrees": avg("t_enum_ms", "core"),
            "peel": avg("t_peel_ms", "core"),
            "core_app": avg("t_total_ms", "app"),
            "core_exact_locate_gpu": avg("t_locate_ms", "exact"),
            "core_exact_host_network": avg("t_flow_build_ms", "exact"),
            "core_exact_host_maxflow": avg("t_flow_ms", "exact"),
            "core_exact_flow_setup": avg("t_flow_setup_ms", "exact"),
            "core_exact_search": avg("t_exact_ms", "exact"),
            "core_exact_total": avg("t_total_ms", "exact"),
        },
        "kernel_rates": {
            "enum_h_cliques_per_s": mu / (k3_ms / 1e3) if k3_ms else None,
            "peel_edges_per_s": recs[-1]["m"] / (k4_ms / 1e3) if k4_ms else None,
            "peel_rounds": core["peel_rounds"], "peel_levels": core["peel_levels"],
            "enum_hbm_frac": k3_bytes(core) / (k3_ms / 1e3) / 1e9 / HBM_PEAK_GBS if k3_ms else None,
            "peel_hbm_frac": k4_bytes(core, h) / (k4_ms / 1e3) / 1e9 / HBM_PEAK_GBS if k4_ms else None,
        },
        "roofline": dominant,
        "roofline_other": other,
    }
    if args.batch_graphs > 0:
        out["batch"] = batch_leg(args.batch_graphs, 7)
    if args.serve_requests > 0:
        out["serve"] = serve_leg(args.serve_requests, 5)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload, args.seed)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
