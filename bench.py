#!/usr/bin/env python3
"""Benchmark of the whole densest-subgraph hot path on one MI355X.

One step = one pass of every stage over one synthetic graph whose edge list
is already resident in HBM: CSR build and degree-ordered orientation, clique
enumeration (clique-degrees), the (k, Psi)-core peel, CoreApp, and CoreExact
(locating on the GPU, then the exact search with minimum cuts).  CoreExact
reuses the decomposition the handle already holds from the clique-core call.

The headline workload is the largest single-GPU configuration: an R-MAT graph
of scale 22 (4,194,304 vertices, 67,108,864 edge draws, (a, b, c, d) =
(0.57, 0.19, 0.19, 0.05), duplicates and self-loops removed) with the
4-clique as the pattern.  Its located core holds about 3.4e10 4-cliques, so
the exact step's flow network (about four arcs per clique) cannot be built
in device memory; the library refuses it with DSD_EUNSUPPORTED after the
locate step, and the step records that refusal.

Further legs: the Chung-Lu graph (n = 10^6, h = 3, where CoreExact runs to
the end), the batched mixture (8,192 graphs, batched vs a plain per-graph
loop), the server under load, the CPU oracle on a bounded sample of the
headline family and the OpenMP enumeration beside it, and the same R-MAT
graph at h = 5: one step (about 80 s), without warm-up or per-launch
timing.

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
    # the largest single-GPU configuration: the headline
    "rmat22_h4": dict(gen="rmat", h=4, kw=dict(scale=22, edge_factor=16)),
    "rmat22_h5": dict(gen="rmat", h=5, kw=dict(scale=22, edge_factor=16)),
    # triangle density on a power-law graph
    "chung_lu_1e6": dict(gen="chung_lu", h=3, kw=dict(n=1_000_000, avg_deg=20.0, beta=2.1, planted=5,
                                                     plant_size=200, p=0.7)),
    # the small configuration (quick runs)
    "er_2000": dict(gen="er_planted", h=2, kw=dict(n=2000, m=10000, plant=60, p=0.4)),
}

# the paper's own figures, quoted with the hardware it states (context only:
# other machine, other graphs; the paper prints no absolute time for h >= 3)
PAPER_FIGURES = {
    "hardware": "Java; Intel Xeon 3.40 GHz, 16 cores, 125 GB RAM (section 8, setup)",
    "core_app_h2_s": {"DBLP": 0.077, "Cit-Patents": 1.021, "Friendster": 2.986, "Enwiki-2017": 8.139,
                      "UK-2002": 5.825},
    "core_app_vs_peel_app_triangle": {"SSCA n=1e5": 20, "R-MAT n=1e5": 201},
    "note": "CoreApp wall times at h = 2 from the paper's EMcore comparison table; speed-ups from section 8",
}


def say(msg: str):
    """A progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_graph(name: str, seed: int):
    from paper_1906_00341_amd import synth
    w = WORKLOADS[name]
    return getattr(synth, w["gen"])(seed=seed, **w["kw"]), w["h"]


def k3_bytes(st: dict) -> float:
    """Algorithmic bytes of one whole-graph clique-degree pass: every
    directed 2-path r -> v -> x reads one out-list entry (4 B), plus per edge
    the row pointers / staged out-list / flushed counters (24 B) and 8 B of
    output per vertex.  The same bytes hold for h >= 4: the deeper levels run
    in LDS bitmaps built from those reads."""
    return 4.0 * st["w2"] + 24.0 * st["m"] + 8.0 * st["n"]


# the peel's main kernel by the kind the library reports
MAIN_KERNEL = {1: "k_process_h2", 2: "k_h3_probe", 3: "k_tl_process", 4: "k_star_front", 6: "k_root_edges"}
MAIN2_KERNEL = {6: "k_root_count"}


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
    vertex its two row offsets (16 B).  Arc discovery of h >= 4
    (k_root_edges): every row entry of a removed vertex its column entry and
    the neighbour's stamp (4 + 4 B), every member of a candidate set C_v its
    two row offsets (16 B), every probed out-list entry 4 B."""
    kind = st["k4_main_kind"]
    if kind == 1:
        return 24.0 * st["k4_main_pairs"] + 16.0 * st["k4_main_nbrs"]
    if kind == 3:
        return 16.0 * st["k4_main_pairs"] + 24.0 * st["k4_main_nbrs"]
    if kind == 6:
        return 8.0 * st["k4_main_entries"] + 16.0 * st["k4_main_nbrs"] + 4.0 * st["k4_main_pairs"]
    return 4.0 * st["k4_main_pairs"] + 20.0 * st["k4_main_nbrs"]


# Integer ALU peak for the counting kernel's unit of work, one 64-bit bitmap
# word ANDed and counted: two 32-bit ANDs and two 32-bit popcounts (each
# adding into the running count), 4 VALU operations per lane; 256 CUs x 4
# SIMDs x 16 lanes issue 64 lane-operations per CU per clock at 2.4 GHz.
ALU_WORD_PEAK = 256 * 64 * 2.4e9 / 4 / 1e12     # 9.83 Tword/s


def roof_alu(kernel, total_ms, launches, words):
    """Roofline of a kernel bound by integer ALU work on bitmap words."""
    launches = max(launches, 1)
    words_call = words / launches
    ms_call = total_ms / launches
    achieved = words_call / (ms_call / 1e3) / 1e12 if ms_call > 0 else 0.0
    return {"kernel": kernel, "bound": "alu", "achieved": achieved, "peak": ALU_WORD_PEAK,
            "unit": "Tword/s (64-bit AND + popcount)", "frac": achieved / ALU_WORD_PEAK, "traffic": None,
            "words_per_launch": words_call, "ms_per_launch": ms_call, "launches_per_step": launches,
            "ms_per_step": total_ms,
            "timing": "HIP events around every launch of one extra step after the timed ones"}


def k4_bytes(st: dict, h: int) -> float:
    """Algorithmic bytes of one full peel (the stage rate): h = 2 touches
    every edge from both ends (32 B per edge); h = 3 reads the out-list of
    every neighbour of every removed vertex (4 B per entry of
    sum_v deg(v) d+(v)) and decrements survivors (24 B per edge); h >= 4
    the arc-discovery kernel's bytes above, plus, for the counting kernel,
    every member's stamp and an 8-byte read-modify-write of its degree
    (20 B; its bitmap rows are the arc kernel's output, read from L2)."""
    if h == 2:
        return 32.0 * st["m"]
    if h >= 4 and st["k4_main_kind"] == 6:
        return main_kernel_bytes(st) + 20.0 * st["k4_main_nbrs"]
    return 4.0 * st["s2"] + 24.0 * st["m"]


TAIL_KERNEL = "k_tail_engine"


def tail_kernel_bytes(st: dict) -> float:
    """Algorithmic bytes of the tail engine (h = 2, 3) over one peel: every
    pair it walks is one 4-byte word of the rewritten rows; every tail vertex
    costs its degree and id in (8 + 4 B), its two row offsets (16 B), its id
    again and its core number out (4 + 8 B); every round handed to the grid
    costs each tail vertex its degree and state out (5 B) and back in with
    its row start (13 B)."""
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


def roof(kernel, workload, total_ms, launches, total_bytes):
    launches = max(launches, 1)
    bytes_call = total_bytes / launches
    ms_call = total_ms / launches
    achieved = bytes_call / (ms_call / 1e3) / 1e9 if ms_call > 0 else 0.0
    return {"kernel": kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kernel, workload),
            "bytes_per_launch": bytes_call, "ms_per_launch": ms_call, "launches_per_step": launches,
            "ms_per_step": total_ms,
            "timing": "HIP events around every launch of one extra step after the timed ones"}


def run_workload(name: str, seed: int, steps: int, warmup: int, instrument: bool = True):
    """Timed steps of one workload; returns the record of the bench line.
    instrument=False skips the step with per-launch kernel timing (no
    roofline then)."""
    import numpy as np
    import torch

    from paper_1906_00341_amd import dsd

    (n, src, dst), h = make_graph(name, seed)
    dev = torch.device("cuda:0")
    ts = torch.from_numpy(np.ascontiguousarray(src, np.int32)).to(dev)
    td = torch.from_numpy(np.ascontiguousarray(dst, np.int32)).to(dev)
    del src, dst
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
        rec["app_density"] = dens
        try:
            _, rho = dsd.core_exact(g, h, out=exact_t)
            rec["rho"] = str(rho)
        except dsd.DsdError as e:
            if e.status != -5:
                raise
            rec["rho"] = None
        rec["exact"] = g.stats()
        rec["m"] = g.info()[1]
        g.free()
        return rec

    def progress(what, t):
        say(f"{name} {what}: {1000.0 * (time.perf_counter() - t):.0f} ms")

    for i in range(warmup):
        t = time.perf_counter()
        step()
        progress(f"warmup step {i + 1}/{warmup}", t)
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for i in range(steps):
        recs.append(step())
        # one line per step, after it (the host already waited for its results)
        progress(f"timed step {i + 1}/{steps}", t0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1000.0 * wall / steps
    # one more step, right after the timed ones, with every launch of the
    # peel's main kernels bracketed by HIP events on the graph's stream (each
    # bracketed launch costs the host ~20 us, so the timed steps run without)
    if instrument:
        t = time.perf_counter()
        inst = step(time_kernels=True)["core"]
        progress("step with per-launch kernel timing", t)
    else:
        inst = recs[-1]["core"]

    core = recs[-1]["core"]
    ex = recs[-1]["exact"]
    mu = core["num_cliques"]
    avg = lambda key, stage: sum(r[stage][key] for r in recs) / len(recs)
    k3_ms = avg("k3_ms", "core")
    k4_ms = avg("k4_ms", "core")
    kind = inst["k4_main_kind"]
    cands = [] if not instrument else [roof(MAIN_KERNEL.get(kind), name, inst["k4_main_ms"], inst["k4_main_launches"],
                  main_kernel_bytes(inst))]
    if cands:
        cands[0].update({"pairs_per_step": inst["k4_main_pairs"], "members_per_step": inst["k4_main_nbrs"],
                         "row_entries_per_step": inst["k4_main_entries"]})
    if instrument and kind in MAIN2_KERNEL:
        # k_root_count: the bitmap words it ANDs and counts (its first level:
        # all of its work at h = 4) against the ALU peak
        r2 = roof_alu(MAIN2_KERNEL[kind], inst["k4_main2_ms"], inst["k4_main2_launches"], inst["k4_main2_words"])
        r2.update({"members_per_step": inst["k4_main_nbrs"]})
        cands.append(r2)
    if instrument and inst["k4_tail_launches"]:
        t = roof(TAIL_KERNEL, name, inst["k4_tail_ms"], inst["k4_tail_launches"], tail_kernel_bytes(inst))
        t.update({"pairs_per_step": inst["k4_tail_pairs"], "tail_vertices": inst["k4_tail_vertices"],
                  "grid_rounds": inst["k4_tail_grid_rounds"], "grid_pairs": inst["k4_tail_grid_pairs"],
                  "grid_ms": inst["k4_tail_grid_ms"]})
        cands.append(t)
    cands.sort(key=lambda r: -r["ms_per_step"])
    located = {"vertices": ex["located_vertices"],
               "rho1": f"{ex['locate_rho1_num']}/{ex['locate_rho1_den']}", "k1": ex["locate_k1"],
               "rho2": f"{ex['locate_rho2_num']}/{ex['locate_rho2_den']}", "k2": ex["locate_k2"],
               "components": ex["locate_components"]}
    return {
        "value": mu / (ms_per_step / 1e3),
        "ms_per_step": ms_per_step,
        "config": {"workload": name, "h": h, "n": n, "m": recs[-1]["m"], "seed": seed, "num_cliques": mu,
                   "kmax": recs[-1]["kmax"], "rho_app": str(recs[-1]["app_density"]),
                   "rho_opt": recs[-1]["rho"] if recs[-1]["rho"] is not None else
                   "refused: the located core's flow network does not fit (DSD_EUNSUPPORTED)",
                   "located": located},
        "stages_ms": {
            "build_orient": avg("t_total_ms", "build"),
            "clique_degrees": avg("t_enum_ms", "core"),
            "peel": avg("t_peel_ms", "core"),
            "core_app": avg("t_total_ms", "app"),
            "core_exact_locate_gpu": avg("t_locate_ms", "exact"),
            "core_exact_network": avg("t_flow_build_ms", "exact"),
            "core_exact_maxflow": avg("t_flow_ms", "exact"),
            "core_exact_flow_setup": avg("t_flow_setup_ms", "exact"),
            "core_exact_search": avg("t_exact_ms", "exact"),
            "core_exact_total": avg("t_total_ms", "exact"),
        },
        "kernel_rates": {
            "enum_h_cliques_per_s": mu / (k3_ms / 1e3) if k3_ms else None,
            "peel_edges_per_s": recs[-1]["m"] / (k4_ms / 1e3) if k4_ms else None,
            "peel_cliques_per_s": mu / (k4_ms / 1e3) if k4_ms else None,
            "peel_rounds": core["peel_rounds"], "peel_levels": core["peel_levels"],
            "enum_hbm_frac": k3_bytes(core) / (k3_ms / 1e3) / 1e9 / HBM_PEAK_GBS if k3_ms else None,
            "peel_hbm_frac": k4_bytes(inst, h) / (k4_ms / 1e3) / 1e9 / HBM_PEAK_GBS if k4_ms else None,
        },
        "roofline": cands[0] if cands else None,
        "roofline_other": cands[1:],
    }


def cpu_baseline(workload: str, seed: int):
    """The CPU oracle, single-threaded, on a bounded sample of the workload's
    family.  R-MAT: the same generator at scale 15 (32,768 vertices; about
    20 s of one core), clique-degrees + core decomposition + CoreApp at the
    workload's h.
    Chung-Lu: the same generator at n = 600,000, the same stages.  ER: the
    whole 2,000-vertex graph and the whole path."""
    import oracle
    from paper_1906_00341_amd import synth
    w = WORKLOADS[workload]
    h = w["h"]
    if workload == "er_2000":
        n, s, d = synth.er_planted(seed=seed, **w["kw"])
        stages = "clique-degrees + core decomposition + CoreApp + CoreExact"
    elif w["gen"] == "rmat":
        n, s, d = synth.rmat(seed=seed, **dict(w["kw"], scale=15))
        stages = "clique-degrees + core decomposition + CoreApp"
    else:
        n, s, d = synth.chung_lu(seed=seed, **dict(w["kw"], n=600_000))
        stages = "clique-degrees + core decomposition + CoreApp"
    g = oracle.Graph(n, s, d)
    say(f"cpu baseline: oracle on n={n}, h={h}")
    t0 = time.perf_counter()
    _, mu = g.clique_degrees(h)
    g.core_decomposition(h)
    g.core_app(h)
    if workload == "er_2000":
        g.exact(h, "core")
    t = time.perf_counter() - t0
    say(f"cpu baseline: {t:.1f} s")
    out = {"value": mu / t, "unit": "h-cliques/s", "cores": 1, "kind": "oracle",
           "sample": f"{w['gen']} generator of {workload} at n={n} (m={g.m}, h={h}, mu={mu}); {stages}; "
                     f"{t:.2f} s, one thread"}
    if w["gen"] == "rmat":
        # the secondary CPU line: the oracle's listing on OpenMP threads,
        # clique-degrees only, on a larger graph of the same family
        n2, s2, d2 = synth.rmat(seed=seed, **dict(w["kw"], scale=18))
        g2 = oracle.Graph(n2, s2, d2)
        say(f"cpu baseline: OpenMP clique-degrees on n={n2}, h={h}")
        t0 = time.perf_counter()
        _, mu2, nt = oracle.clique_degrees_omp(g2, h)
        t2 = time.perf_counter() - t0
        say(f"cpu baseline: OpenMP {t2:.1f} s on {nt} threads")
        out["openmp"] = {"value": mu2 / t2, "unit": "h-cliques/s", "cores": nt,
                         "kind": "secondary CPU line: the oracle's clique listing on OpenMP threads (oracle/omp_enum.c)",
                         "sample": f"rmat generator at scale 18 (n={n2}, m={g2.m}, h={h}, mu={mu2}); "
                                   f"clique-degrees only; {t2:.2f} s"}
    return out


def _batch_graphs(specs, threads=16):
    import concurrent.futures as cf
    from paper_1906_00341_amd import synth
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(synth.batch_graph, specs))


def batch_leg(n_graphs: int, seed: int):
    """Batched vs plain on the batched mixture (n log-uniform in [100,
    50000], Chung-Lu exponent U[2, 3], average degree U[4, 40], h in {2, 3,
    4}): the first n_graphs graphs of the 8192-graph mixture.  Op: the (k,
    Psi)-core decomposition.  Plain = one dsd_clique_core call per graph;
    batched = one dsd_batch_run over all of them."""
    import torch
    from paper_1906_00341_amd import dsd, synth
    specs = synth.batch_specs(count=8192, seed=seed)[:n_graphs]
    hs = [sp["h"] for sp in specs]
    t0 = time.perf_counter()
    graphs = _batch_graphs(specs)
    t_gen = time.perf_counter() - t0
    handles = []
    for n, s, d in graphs:
        handles.append(dsd.build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda()))
    del graphs
    torch.cuda.synchronize()
    mu = 0
    t0 = time.perf_counter()
    for g, h in zip(handles, hs):
        dsd.clique_core(g, h)
        mu += g.stats()["num_cliques"]
    t_plain = time.perf_counter() - t0
    say(f"batch leg: plain loop over {n_graphs} graphs {t_plain:.2f} s")
    # every graph again, from scratch: the batch must not reuse the plain
    # loop's cached decompositions
    for g in handles:
        g.free()
    handles = []
    graphs = _batch_graphs(specs)
    for n, s, d in graphs:
        handles.append(dsd.build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda()))
    del graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = dsd.batch_run(handles, hs, "core")
    t_batch = time.perf_counter() - t0
    say(f"batch leg: one batch {t_batch:.2f} s")
    assert all(r["status"] == 0 for r in res)
    assert sum(r["num_cliques"] for r in res) == mu
    m = sum(g.info()[1] for g in handles)
    for g in handles:
        g.free()
    return {"graphs": n_graphs, "of": 8192, "edges": m, "h_cliques": mu, "op": "core",
            "plain_s": t_plain, "batched_s": t_batch,
            "plain_graphs_per_s": n_graphs / t_plain, "batched_graphs_per_s": n_graphs / t_batch,
            "plain_h_cliques_per_s": mu / t_plain, "batched_h_cliques_per_s": mu / t_batch,
            "batched_edges_per_s": m / t_batch, "speedup": t_plain / t_batch,
            "peel_rounds_batched": max(r["peel_rounds"] for r in res), "generation_s": t_gen}


def serve_leg(n_requests: int, seed: int):
    """The server under load: requests drawn 95 % from the batched mixture and
    5 % from R-MAT scale 20 (a = 0.57, b = c = 0.19), h in {2, 3, 4}, ops 70 %
    CoreApp, 20 % core decomposition, 10 % CoreExact, on every graph kind.
    Pass 1 submits everything at once (saturation throughput); pass 2 submits
    with Poisson arrivals at half that rate and records each request's
    latency.  Plain = the same requests as sequential single-graph calls.  A
    request the library refuses (an exact step whose network would not fit)
    is counted apart, not as served."""
    import concurrent.futures as cf
    import numpy as np
    import torch
    from paper_1906_00341_amd import dsd, synth
    rng = np.random.default_rng(seed)
    specs = synth.batch_specs(count=8192, seed=seed + 1)
    n_rmat = max(1, n_requests // 20)
    rmat_graph = synth.rmat(scale=20, edge_factor=16, seed=seed)
    small = _batch_graphs([specs[i] for i in range(n_requests)])
    reqs = []
    for i in range(n_requests):
        u = rng.random()
        op = "app" if u < 0.7 else ("core" if u < 0.9 else "exact")
        if i < n_rmat:
            reqs.append((rmat_graph, int(rng.integers(2, 5)), op))
        else:
            reqs.append((small[i], specs[i]["h"], op))
    order = rng.permutation(n_requests)
    reqs = [reqs[i] for i in order]
    calls = {"app": dsd.core_app, "core": dsd.clique_core, "exact": dsd.core_exact}

    def build():
        return [dsd.build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda()) for (n, s, d), _, _ in reqs]

    handles = build()
    torch.cuda.synchronize()
    refused_plain = 0
    t0 = time.perf_counter()
    for g, (_, h, op) in zip(handles, reqs):
        try:
            calls[op](g, h)
        except dsd.DsdError as e:
            if e.status != -5:
                raise
            refused_plain += 1
    t_plain = time.perf_counter() - t0
    say(f"serve leg: {n_requests} sequential plain calls {t_plain:.2f} s")
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
        refused = sum(1 for _, r in outs if r["status"] == -5)
        for g in hs:
            g.free()
        served = [lat[i] for i, (_, r) in enumerate(outs) if r["status"] == 0]
        return total, served, refused

    t_sat, _, refused = run(None)
    say(f"serve leg: saturation pass {t_sat:.2f} s")
    served_n = n_requests - refused
    qps_sat = served_n / t_sat
    t_half, lat, _ = run(0.5 * n_requests / t_sat)
    say(f"serve leg: half-rate pass {t_half:.2f} s")
    srv.close()
    lat_ms = np.sort(np.asarray(lat)) * 1000.0
    return {"requests": n_requests, "rmat20_requests": n_rmat, "mix": "70% app / 20% core / 10% exact",
            "workers": int(os.environ.get("DSD_SERVER_WORKERS", "4")),
            "refused": refused, "refused_plain": refused_plain,
            "plain_qps": (n_requests - refused_plain) / t_plain, "served_qps_saturation": qps_sat,
            "overlap_speedup": (t_plain / t_sat), "offered_qps": 0.5 * n_requests / t_sat,
            "served_qps_at_offered": served_n / t_half,
            "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99))}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat22_h4", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--legs", default="chung_lu_1e6:5,rmat22_h5:1:0",
                    help="further workloads as name:steps[:warmup], comma-separated ('' for none); "
                         "a leg with warmup 0 also skips the step with per-launch kernel timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-graphs", type=int, default=8192,
                    help="graphs of the batched mixture in the batched-vs-plain leg (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=192,
                    help="requests in the serving leg (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path is not sharded "
              f"across GPUs", file=sys.stderr)
        return 2
    head = run_workload(args.workload, args.seed, args.steps, args.warmup)
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "h-cliques/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": head["config"],
        "stages_ms": head["stages_ms"],
        "kernel_rates": head["kernel_rates"],
        "roofline": head["roofline"],
        "roofline_other": head["roofline_other"],
    }
    legs = {}
    for spec in [x for x in args.legs.split(",") if x]:
        parts = spec.split(":")
        name = parts[0]
        k = int(parts[1]) if len(parts) > 1 and parts[1] else 1
        wu = int(parts[2]) if len(parts) > 2 and parts[2] else 1
        r = run_workload(name, args.seed, k, wu, instrument=wu > 0)
        legs[name] = {"value": r["value"], "unit": "h-cliques/s", "ms_per_step": r["ms_per_step"],
                      "steps": k, "warmup": wu, "config": r["config"], "stages_ms": r["stages_ms"],
                      "kernel_rates": r["kernel_rates"], "roofline": r["roofline"]}
    if legs:
        out["legs"] = legs
    if args.batch_graphs > 0:
        out["batch"] = batch_leg(args.batch_graphs, 7)
    if args.serve_requests > 0:
        out["serve"] = serve_leg(args.serve_requests, 5)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload, args.seed)
    out["paper_figures"] = PAPER_FIGURES
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
