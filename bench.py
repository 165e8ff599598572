#!/usr/bin/env python3
"""Benchmark of the GDI annealing path on one MI355X.

One step = one full anneal of the workload (all sweeps of the schedule, every
colour phase, in one persistent launch, plus the initial-state and output
kernels) on synthetic input already resident in HBM. Prints one JSON line.

Default workload: random geometric graph, n = 1,000,000 points in the unit
square, mean degree 8, unit int32 weights, 2000 sweeps with geometric T from
3.0 to 0.05, A = B = 1.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin-updates/s + HBM GB/s; cut @ fixed wall time: plain vs batched/learned"
HBM_PEAK_GBS = 8000.0


def halo_source_hash() -> str:
    """SHA-256 (16 hex digits) of the halo sweep's sources: its kernel file and the shared
    device helpers it includes. Counter figures stand only for the source they were taken on."""
    import hashlib

    h = hashlib.sha256()
    for name in ("gdi_halo.hip", "gdi_device.h"):
        with open(os.path.join(ROOT, "paper_1908_00210_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_bytes_per_sweep(path: str, workload: str):
    """HBM bytes per sweep of the halo sweep on a workload from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), or None when
    there is none for this workload or it was taken on another source of the kernel."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        tj = json.load(f)
    if tj.get("kernel_source_sha256_16") != halo_source_hash():
        return None
    w = tj.get("workloads", {}).get(workload)
    return None if w is None else float(w["hbm_bytes_per_sweep"])


def progress(msg: str):
    """One line per finished stage on stderr (stdout carries only the JSON result line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes_per_sweep(n: int, nnz: int) -> int:
    """row_ptr (4(n+1)) + CSR column and weight (8 nnz) + spin read and write (2n)."""
    return 4 * (n + 1) + 8 * nnz + 2 * n


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def cpu_baseline(g, temps, seed, sweeps_all, sweeps_one, reps=3):
    """The C oracle on the first sweeps of the same workload, timed over its sweep loop
    only (colouring, thresholds and the initial cut excluded): all host threads and one
    thread, median of reps runs each."""
    import numpy as np

    import oracle

    med = {}
    for label, threads, k in (("all", 0, sweeps_all), ("one", 1, sweeps_one)):
        ts = [oracle.anneal(g, temps[:k], seed, n_threads=threads)["sweep_s"] for _ in range(reps)]
        med[label] = (k, float(np.median(ts)))
    (k, t), (k1, t1) = med["all"], med["one"]
    return {"value": g.n * k / t, "unit": "spin-updates/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"first {k} of the {temps.size} sweeps of the same workload (n={g.n}), C oracle with "
                      f"OpenMP over each colour class, sweep loop timed, median of {reps}: {t:.2f} s",
            "cpu_model": cpu_model(), "median_of": reps,
            "one_thread": {"value": g.n * k1 / t1, "sweeps": k1, "median_s": t1}}


def gpu_runs(ann, temps, seed, out_ptr, reps):
    """Device time (ms) of reps anneals of the whole schedule after one warm-up."""
    ann.anneal_dev(temps, seed, out_ptr)
    ann.result()
    ms = []
    for _ in range(reps):
        ann.anneal_dev(temps, seed, out_ptr)
        ms.append(ann.result().sweep_ms)
    return ms


def cut_timing(ann, torch, d_spins, n: int, nnz: int, reps: int = 20) -> dict:
    """gdi_cut from scratch on resident spins through the allocation-free entry point (the
    spins gathered into the annealer's order, k_reduce, the final sum), called reps times
    between two events on the handle's stream with no host synchronisation in between.
    Algorithmic bytes per call: the gather's original ids, input and output spins
    (4n + 2n), then row pointers 4(n+1), CSR entries 8 nnz and spins n (neighbour spins
    are gathers from cache and not counted; the class padding is left out)."""
    d_out = torch.zeros(3, dtype=torch.int64, device="cuda:0")
    for _ in range(3):
        ann.cut_dev_noalloc(d_spins, d_out.data_ptr())
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        ann.cut_dev_noalloc(d_spins, d_out.data_ptr())
    e1.record(s)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    b = 6 * n + 4 * (n + 1) + 8 * nnz + n
    return {"kernel": "k_reduce", "us_per_call": us, "bytes_per_call": b, "algorithmic_gbs": b / us / 1e3,
            "frac": b / us / 1e3 / HBM_PEAK_GBS, "calls": reps}


def form_paper_rule(gdi, g, seed, metropolis_ms: float) -> dict:
    """The paper's acceptance rule (argmin, then a random flip with probability P_f(t);
    P_f geometric 0.2 -> 0.001) on the headline graph, next to the Metropolis schedule's
    kernel time: the rule changes the decision, not the sweep's cost."""
    import numpy as np

    import gdi_synth as gs

    S = 2000
    pf = gs.geometric_temps(0.2, 0.001, S)
    with gdi.Annealer(g) as a:
        a.anneal(pf[:10], seed, acceptance=gdi.ACCEPT_PAPER)
        ms, cuts, Ms = [], [], []
        for rep in range(2):
            r = a.anneal(pf, seed + rep, acceptance=gdi.ACCEPT_PAPER)
            ms.append(r["result"]["sweep_ms"])
            cuts.append(int(r["cut"]))
            Ms.append(int(r["M"]))
    return {"sweeps": S, "p_f": [0.2, 0.001], "mean_kernel_ms": float(np.mean(ms)), "metropolis_kernel_ms": metropolis_ms,
            "cuts": cuts, "M": Ms, "spin_updates_per_s": g.n * S / (float(np.mean(ms)) / 1e3)}


def layout_variants(gdi, g, temps, seed, torch, reps=3):
    """The same 1M-node anneal with the unit-weight form switched off (the packed entries'
    11-bit weights summed as general weights) and with the uncompressed layout (int32
    column + int32 weight per entry, spins gathered from global memory, fenced grid
    sweep). Same results; device time of the sweep launch, median of reps."""
    import numpy as np

    out = {}
    d_out = torch.empty(g.n, dtype=torch.int8, device="cuda:0")
    bpl = algorithmic_bytes_per_sweep(g.n, g.nnz) * temps.size
    for name, tune in (("packed_general_weights", dict(general_weights=1)),
                       ("uncompressed_int32_col_weight", dict(scope=gdi.SCOPE_GRID_FENCED))):
        with gdi.Annealer(g) as a:
            a.set_stream(torch.cuda.current_stream().cuda_stream)
            a.tune(**tune)
            ms = float(np.median(gpu_runs(a, temps, seed, d_out.data_ptr(), reps)))
            r = a.result()
        out[name] = {"kernel_ms": ms, "algorithmic_gbs": bpl / (ms / 1e3) / 1e9,
                     "spin_updates_per_s": g.n * temps.size / (ms / 1e3), "scope": int(r.scope),
                     "M": int(r.magnetization), "cut": int(r.cut_weighted)}
    return out


def config_runs(gdi, gs, torch, seed, names, reps=5):
    """Configurations measured beside the headline: device time of the whole schedule
    (median of reps), the oracle's sweep loop on the full schedule for the small ones
    (all host threads), and whether the GPU's final state equals the oracle's."""
    import numpy as np

    import oracle

    out = {}
    for name in names:
        g, T = gs.workload(name)
        d_out = torch.empty(g.n, dtype=torch.int8, device="cuda:0")
        with gdi.Annealer(g) as a:
            a.set_stream(torch.cuda.current_stream().cuda_stream)
            ms = float(np.median(gpu_runs(a, T, seed, d_out.data_ptr(), reps)))
            r = a.result()
            cw, ce, m = a.cut_dev(d_out.data_ptr())
            cut_row = cut_timing(a, torch, d_out.data_ptr(), g.n, g.nnz) if g.n > 100_000 else None
        kern_s = ms / 1e3
        row = {"n": g.n, "nnz": g.nnz, "sweeps": int(T.size), "scope": int(r.scope), "grid": int(r.grid),
               "colours": int(r.n_colours), "kernel_ms": ms, "sweeps_per_s": T.size / kern_s,
               "spin_updates_per_s": g.n * T.size / kern_s,
               "algorithmic_gbs": algorithmic_bytes_per_sweep(g.n, g.nnz) * T.size / kern_s / 1e9,
               "M": int(m), "cut_weighted": int(cw), "cut_edges": int(ce)}
        if cut_row is not None:
            row["cut"] = cut_row
        cb = counter_bytes_per_sweep(os.path.join(ROOT, "profiles", "traffic.json"), name)
        if cb is not None and r.scope == gdi.SCOPE_GRID:
            row["hbm_gbs_counters"] = cb * T.size / kern_s / 1e9
        if g.n <= 100_000:
            ref = oracle.anneal(g, T, seed)
            row["oracle_sweep_s"] = ref["sweep_s"]
            row["oracle_spin_updates_per_s"] = g.n * T.size / ref["sweep_s"]
            row["oracle_threads"] = oracle.max_threads()
            spins = d_out.cpu().numpy()
            row["bit_exact_vs_oracle"] = bool(np.array_equal(spins, ref["spins"]) and int(m) == ref["M"]
                                              and int(cw) == ref["cut"])
        out[name] = row
    return out


def best_state(Ms, cuts, A=1, B=1):
    """Best final state: lowest weighted cut among |M| <= 2 (energy A M^2 + B cut breaks ties);
    lowest energy if none is balanced."""
    cand = [(c, A * m * m + B * c) for m, c in zip(Ms, cuts) if abs(m) <= 2]
    if cand:
        return min(cand, key=lambda x: (x[0], x[1]))[0]
    return min(A * m * m + B * c for m, c in zip(Ms, cuts))


def forms_batched(gdi, gs, torch, seed):
    """Batched vs plain on one GPU: 256 replicas of the n=2000 ER graph in one launch against
    sequential single-replica anneals in the same wall time; and the throughput of the full
    batched workload (64 uneven graphs + the 256 replicas) in one launch."""
    g, T = gs.workload("er2000")
    out = {}
    with gdi.Annealer(g) as a:
        items = [(a.h, g.n, r) for r in range(256)]
        gdi.anneal_batch(items, T, seed, outputs=False)  # autotunes on first use
        t0 = time.perf_counter()
        res = gdi.anneal_batch(items, T, seed, outputs=False)
        wall_b = time.perf_counter() - t0
        best_b = best_state(res["M"], res["cut"])
        d_out = torch.empty(g.n, dtype=torch.int8, device="cuda:0")
        a.set_stream(torch.cuda.current_stream().cuda_stream)
        a.anneal_dev(T, seed, d_out.data_ptr(), replica=0)
        a.result()
        Ms, cuts = [], []
        t0 = time.perf_counter()
        while not Ms or time.perf_counter() - t0 < wall_b:
            a.anneal_dev(T, seed, d_out.data_ptr(), replica=len(Ms))
            r = a.result()
            Ms.append(r.magnetization)
            cuts.append(r.cut_weighted)
        wall_p = time.perf_counter() - t0
        best_p = best_state(Ms, cuts)
        # how long plain needs on average for the batched best: runs until a cut <= 1.005 x batched best
        out["replicas_256_er2000"] = {
            "sweeps": int(T.size), "batched_wall_ms": wall_b * 1e3, "batched_kernel_ms": res["kernel_ms"],
            "batched_best_cut": int(best_b), "plain_runs_in_same_wall": len(Ms), "plain_wall_ms": wall_p * 1e3,
            "plain_best_cut_in_same_wall": int(best_p),
            "batched_at_least_as_good": bool(best_b <= best_p),
        }
    graphs = gs.batch_mix()
    anns = [gdi.Annealer(x) for x in graphs]
    g2, T2 = gs.workload("er2000")
    a2 = gdi.Annealer(g2)
    items = [(x.h, x.n, 0) for x in anns] + [(a2.h, g2.n, r) for r in range(256)]
    gdi.anneal_batch(items, T2, seed, outputs=False)
    t0 = time.perf_counter()
    res = gdi.anneal_batch(items, T2, seed, outputs=False)
    wall = time.perf_counter() - t0
    updates = sum(i[1] for i in items) * T2.size
    out["full_batch"] = {"instances": len(items), "sum_n": sum(i[1] for i in items), "sweeps": int(T2.size),
                         "wall_ms": wall * 1e3, "kernel_ms": res["kernel_ms"],
                         "spin_updates_per_s": updates / (res["kernel_ms"] / 1e3)}
    for x in anns + [a2]:
        x.close()
    return out


def forms_learned(gdi, gs, torch, seed, k_full=8, replicas=8):
    """Learned frozen-node proposal on one GPU: collect traces from the plain annealer on
    the eight training RGGs, train the network with the library's kernels, then on the
    n=200k evaluation RGG run plain, network and heuristic anneals replica by replica and
    report the wall time each needs to reach a balanced cut within 0.5% of the best plain
    cut over the same number of replicas. The proposals apply from sweep learn_from on
    (0: the whole schedule; S/2: the colder half)."""
    import numpy as np

    out = {}
    S, every, k_label = 2000, 50, k_full - 1
    T = gs.geometric_temps(3.0, 0.05, S)
    graphs = gs.training_graphs()
    snaps = len(range(every - 1, S - k_label, every))
    rows = sum(g.n for g in graphs) * snaps
    dx = torch.zeros(rows * 8, dtype=torch.bfloat16, device="cuda:0")
    dy = torch.zeros(rows, dtype=torch.uint8, device="cuda:0")
    t0 = time.perf_counter()
    off = 0
    for g in graphs:
        with gdi.Annealer(g) as a:
            cnt = a.collect_traces(T, seed, every, k_label, dx.data_ptr() + off * 16, dy.data_ptr() + off, snaps)
        off += cnt * g.n
    torch.cuda.synchronize()
    t_collect = time.perf_counter() - t0
    t0 = time.perf_counter()
    w, losses = gdi.mlp_train(dx.data_ptr(), dy.data_ptr(), off, gdi.mlp_init(seed), epochs=3, batch=4096, lr=2e-3,
                              seed=seed)
    t_train = time.perf_counter() - t0
    progress(f"learned form: traces {t_collect:.1f} s, training {t_train:.1f} s")
    ybar = float(dy[:off].float().mean().item())
    out["training"] = {"graphs": [g.n for g in graphs], "rows": off, "frozen_fraction": ybar,
                       "collect_s": t_collect, "train_s": t_train, "epoch_loss": [float(x) for x in losses],
                       "constant_predictor_loss": float(-(ybar * np.log(ybar) + (1 - ybar) * np.log(1 - ybar)))}
    del dx, dy
    g, Te = gs.workload("rgg200k")
    half = Te.size // 2
    runs = {}
    with gdi.Annealer(g) as a:
        a.anneal(Te[:10], seed)  # warm-up: threshold table, launch choice
        methods = {"plain": lambda r: a.anneal(Te, seed, replica=r)}
        for lf in (0, half):
            for p_skip in (0.9, 0.97):
                methods[f"network_p{p_skip}_from{lf}"] = (
                    lambda r, lf=lf, p_skip=p_skip: a.anneal_learned(
                        Te, seed, k_full, replica=r, skip_mode=gdi.SKIP_MLP, weights=w, skip_threshold=p_skip,
                        learn_from=lf))
            methods[f"heuristic_k{k_full}_from{lf}"] = (
                lambda r, lf=lf: a.anneal_learned(Te, seed, k_full, replica=r, skip_mode=gdi.SKIP_HEURISTIC,
                                                  heuristic_k=k_full, learn_from=lf))
        methods[f"no_proposal_k{k_full}"] = lambda r: a.anneal_learned(Te, seed, k_full, replica=r)
        for name, fn in methods.items():
            ms, Ms, cuts, skip = [], [], [], []
            for r in range(replicas):
                t0 = time.perf_counter()
                res = fn(r)
                ms.append((time.perf_counter() - t0) * 1e3)
                Ms.append(res["M"])
                cuts.append(res["cut"])
                rr = res["result"]
                skip.append(rr.get("node_skips", 0) / max(1, rr.get("node_skips", 0) + rr.get("node_visits", 1)))
            runs[name] = (ms, Ms, cuts, skip)
            progress(f"learned form: {name} x {replicas} replicas, {np.mean(ms):.1f} ms each")
    best_plain = best_state(runs["plain"][1], runs["plain"][2])
    target = best_plain * 1.005 if best_plain >= 0 else best_plain * 0.995
    for name, (ms, Ms, cuts, skip) in runs.items():
        reach = None
        for i, (m, c) in enumerate(zip(Ms, cuts)):
            if abs(m) <= 2 and c <= target:
                reach = float(np.sum(ms[:i + 1]))
                break
        out[name] = {"mean_ms": float(np.mean(ms)), "best_cut": int(best_state(Ms, cuts)),
                     "mean_cut": float(np.mean(cuts)), "balanced": int(sum(abs(m) <= 2 for m in Ms)),
                     "skipped_fraction": float(np.mean(skip)), "ms_to_within_0.5pct_of_plain_best": reach}
    out["eval"] = {"graph": g.name, "n": g.n, "sweeps": int(Te.size), "replicas": replicas, "k_full": k_full,
                   "plain_best_cut": int(best_plain), "target_cut": float(target)}
    return out


def forms_standard(gdi, gs, sweeps=50):
    """GDI vs the standard solver of Alg. 2 (every decision sums all n spins for the
    balance term) on 2-D tori of growing size: same results, time per sweep of each."""
    import numpy as np

    out = []
    T = gs.geometric_temps(3.0, 0.05, sweeps)
    for L in (32, 45, 64, 90, 128, 180):
        g = gs.torus_graph(L, 400 + L, "pm1")
        with gdi.Annealer(g) as a:
            a.anneal(T[:5], 1)
            r_gdi = a.anneal(T, 1)
            a.anneal(T[:5], 1, flags=gdi.FLAG_DENSE_BALANCE)
            r_std = a.anneal(T, 1, flags=gdi.FLAG_DENSE_BALANCE)
        assert np.array_equal(r_gdi["spins"], r_std["spins"])
        out.append({"n": g.n, "sweeps": sweeps, "gdi_ms": r_gdi["result"]["sweep_ms"],
                    "std_ms": r_std["result"]["sweep_ms"],
                    "std_over_gdi": r_std["result"]["sweep_ms"] / r_gdi["result"]["sweep_ms"]})
    return out


def forms_racy(gdi, gs, seed, runs=3):
    """Price of determinism on the 1M-node RGG: the deterministic colour-phase sweep
    against Alg. 3 as printed (asynchronous, per-thread reads of G and one atomic add per
    flip, one persistent launch) with every co-resident workgroup and with 8 workgroups
    (fewer nodes in flight, so more of them see their neighbours' new spins)."""
    import numpy as np

    g, T = gs.workload("rgg1m")
    out = {}
    with gdi.Annealer(g) as a:
        for name, flags, grid in (("deterministic", 0, 0), ("asynchronous", gdi.FLAG_RACY, 0),
                                  ("asynchronous_8wg", gdi.FLAG_RACY, 8)):
            a.tune(grid=grid)
            a.anneal(T[:10], seed, flags=flags)
            ms, cuts, Ms = [], [], []
            for r in range(runs):
                res = a.anneal(T, seed, replica=r, flags=flags)
                ms.append(res["result"]["sweep_ms"])
                cuts.append(res["cut"])
                Ms.append(res["M"])
            out[name] = {"mean_kernel_ms": float(np.mean(ms)), "cuts": [int(c) for c in cuts],
                         "M": [int(m) for m in Ms], "grid": int(res["result"]["grid"])}
    out["random_state_cut"] = int(g.nnz // 4)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rgg1m")
    ap.add_argument("--sweeps", type=int, default=0, help="override the schedule length")
    ap.add_argument("--cpu-sweeps", type=int, default=1000, help="oracle sweeps timed on all host threads")
    ap.add_argument("--cpu-sweeps-one", type=int, default=100, help="oracle sweeps timed on one thread")
    ap.add_argument("--no-configs", action="store_true", help="skip the other configurations and layouts")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the batched / learned comparisons")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    ap.add_argument("--source-hash", action="store_true", help="print the halo sweep's source hash and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (for scaling HBM counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(every instance fits one MI355X; see DESIGN.md for how the path would shard)",
              file=sys.stderr)
        sys.exit(2)

    if args.source_hash:
        print(halo_source_hash())
        return
    import numpy as np
    import torch

    import gdi_synth as gs
    import paper_1908_00210_amd as gdi

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.calibrate_copy, "dispatches": 3}), flush=True)
        return
    spec = gs.WORKLOADS[args.workload]
    g = spec["graph"]()
    S = args.sweeps or spec["sweeps"]
    temps = gs.geometric_temps(spec["t0"], spec["t1"], S)
    seed = 1
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    out = torch.empty(g.n, dtype=torch.int8, device=dev)

    t0 = time.perf_counter()
    ann = gdi.Annealer(g)
    create_s = time.perf_counter() - t0
    ann.set_stream(stream.cuda_stream)
    for _ in range(args.warmup):
        ann.anneal_dev(temps, seed, out.data_ptr())
        ann.result()
    torch.cuda.synchronize()
    sweep_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ann.anneal_dev(temps, seed, out.data_ptr())
        # device time of this step's sweep launch (HIP events on the same stream)
        sweep_ms.append(ann.result().sweep_ms)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    res = ann.result()
    cw, ce, m = ann.cut_dev(out.data_ptr())
    info = ann.info
    # the from-scratch cut (gdi_cut) on the annealed spins, resident on the device
    cut_row = cut_timing(ann, torch, out.data_ptr(), g.n, g.nnz)

    n, nnz = g.n, g.nnz
    updates = n * S
    value = updates * args.steps / elapsed
    kern_s = float(np.mean(sweep_ms)) / 1e3
    bytes_launch = algorithmic_bytes_per_sweep(n, nnz) * S
    achieved = bytes_launch / kern_s / 1e9
    per_sweep = counter_bytes_per_sweep(args.traffic_json, args.workload) if res.scope == gdi.SCOPE_GRID else None
    traffic = per_sweep * S if per_sweep is not None else None
    counter_gbs = traffic / kern_s / 1e9 if traffic is not None else None
    grid_phases = int(info.n_colours)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "spin-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": args.workload, "graph": g.name, "n": n, "nnz": nnz, "sweeps": S,
            "t0": spec["t0"], "t1": spec["t1"], "A": 1, "B": 1, "colours": int(info.n_colours),
            "scope": int(res.scope), "grid": int(res.grid), "block": int(res.block),
            "lanes_per_node": int(res.lanes_per_node), "parallelism": "single-gpu",
        },
        "sweeps_per_s": S * args.steps / elapsed,
        # HBM bytes the counters saw per launch over the kernel's time (null without counters
        # for this kernel source); the algorithmic figure is roofline.achieved
        "hbm_gbs": counter_gbs,
        "algorithmic_gbs": achieved,
        "us_per_phase": kern_s * 1e6 / (S * grid_phases),
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "achieved_counters_gbs": counter_gbs,
            "frac_counters": counter_gbs / HBM_PEAK_GBS if counter_gbs is not None else None,
            "kernel": {gdi.SCOPE_GRID: "k_sweep_halo", gdi.SCOPE_GRID_FENCED: "k_sweep_grid"}.get(res.scope, "k_sweep_wg"),
            "entry_layout": ("packed 32-bit CSR entries (16-bit LDS word, 11-bit weight, 5-bit bit position); "
                             "achieved counts the algorithmic 8 bytes per entry, traffic the bytes the counters saw")
            if res.scope == gdi.SCOPE_GRID else "int32 column + int32 weight per entry",
            "kernel_ms": kern_s * 1e3, "bytes_per_launch": bytes_launch,
        },
        "result": {"M": int(m), "cut_weighted": int(cw), "cut_edges": int(ce),
                   "tracked_cut": int(res.cut_weighted), "create_s": create_s},
        "cut": cut_row,
    }
    ann.close()
    progress(f"{args.workload}: {S} sweeps x {args.steps} steps timed, {line['ms_per_step']:.1f} ms per step")
    if not args.no_configs and args.workload == "rgg1m":
        line["layouts_rgg1m"] = layout_variants(gdi, g, temps, seed, torch)
        progress("layout variants done")
    if not args.no_configs:
        line["configs"] = config_runs(gdi, gs, torch, seed, [w for w in ("er800", "torus100", "rgg8m")
                                                             if w != args.workload])
        progress("configurations done")
    if not args.no_forms:
        line["forms"] = forms_batched(gdi, gs, torch, seed)
        progress("batched form done")
        line["forms"]["learned_rgg200k"] = forms_learned(gdi, gs, torch, seed)
        progress("learned form done")
        line["forms"]["gdi_vs_standard_torus"] = forms_standard(gdi, gs)
        progress("standard solver done")
        line["forms"]["determinism_rgg1m"] = forms_racy(gdi, gs, seed)
        progress("asynchronous form done")
        if args.workload == "rgg1m":
            line["forms"]["paper_rule_rgg1m"] = form_paper_rule(gdi, g, seed, kern_s * 1e3)
            progress("paper acceptance rule done")
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(g, temps, seed, min(args.cpu_sweeps, S), min(args.cpu_sweeps_one, S))
        progress("CPU baseline done")
    print(json.dumps(line), flush=True)
    # every handle is closed by now; leave no device work or library object to process exit
    import gc

    gc.collect()
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
