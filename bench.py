#!/usr/bin/env python3
"""Benchmark: Red-Green-Gray edge classification updates on one MI355X.

Workload (default): the spatial rigid-body roadmap -- 8-sphere robot, 50,000
(position, unit quaternion) nodes, k = 10 nearest-neighbour edges, 20
configurations per edge, 500 box obstacles with sides U[0.2, 1.5] in a 10^3
workspace; each update moves 10% of the boxes by N(0, 0.3) per axis; binary32
tests with a binary64 re-test inside a 1e-5 relative rounding band (relative to
each test's own scale (s + R)(R + L)).

A step is one update: every edge of the roadmap is classified (labels[E] and
the gray list are produced).  Inputs (the roadmap and every obstacle state)
are resident in HBM before timing starts.  The JSON line reports:
  value           edges classified per second, pipelined updates (no events)
  stage_ms_*      per-kernel-stage times from HIP events, a separate pass
  latency_*_us    per-update latency (submit -> labels ready) over a second pass
  graph_*         the same updates launched as captured HIP graphs
  roofline        the classify kernel's algorithmic bytes per launch over its
                  event-timed duration, against 8 TB/s
  cpu_baseline    the FP64 CPU oracle on a bounded sample of the same edges
  validation      full continuous validation of the last update's gray list
                  (rgg_validate_async chained after the update), HIP-event
                  timed, beside the oracle on a sample of the same edges
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--nodes", type=int, default=50000)
    p.add_argument("--cell-size", type=float, default=-1.0)
    p.add_argument("--item-edges", type=int, default=0,
                   help="edges per work item at build (0 = 256); the autotuner may change it")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-edges", type=int, default=300000,
                   help="edges the oracle classifies (capped at the roadmap size)")
    p.add_argument("--cpu-single-edges", type=int, default=20000,
                   help="edges of the one-thread oracle measurement (0 skips it)")
    p.add_argument("--skip-graph", action="store_true")
    p.add_argument("--seed", type=int, default=2)
    p.add_argument("--no-batched", action="store_true",
                   help="skip the batched-planar measurement (64 roadmaps)")
    p.add_argument("--batched-steps", type=int, default=20)
    p.add_argument("--batched-cell-size", type=float, default=0.0)
    p.add_argument("--no-serving", action="store_true",
                   help="skip the serving measurement (16 resident roadmaps, Poisson requests)")
    p.add_argument("--serving-seconds", type=float, default=10.0)
    p.add_argument("--no-tune", action="store_true",
                   help="keep the built work decomposition instead of running the autotuner")
    p.add_argument("--no-other-configs", action="store_true",
                   help="skip the planar (FP64 and FP32) and arm measurements")
    p.add_argument("--no-second-forms", action="store_true",
                   help="skip the oriented-box and spline forms of the approximations")
    p.add_argument("--no-validate", action="store_true",
                   help="skip the full validation of the last update's gray list")
    p.add_argument("--cpu-validate-edges", type=int, default=2000,
                   help="gray edges the oracle validates for the CPU comparison")
    p.add_argument("--only", choices=["arm", "batched"], default=None,
                   help="run one further configuration alone (for profiling): the planar arm on the plain "
                        "path, or the batched planar roadmaps; prints that section as the JSON line")
    p.add_argument("--copy-calibration", action="store_true",
                   help="also run a plain 1 GiB device copy 5 times (reference kernel for "
                        "scaling FETCH_SIZE / WRITE_SIZE counters)")
    return p.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Host cores the CPU legs use: the box gives one GPU's job a 16-core share of
# its host, whatever the CPU count it reports.
CPU_SHARE = 16


def cpu_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(CPU_SHARE, n))


def cpu_host():
    """The host CPU: its model (/proc/cpuinfo), the CPUs the OS reports and
    the ones this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        aff = None
    return {"model": model, "cpus_reported": os.cpu_count(), "cpus_allowed": aff,
            "threads_used": cpu_threads(), "share_per_gpu": CPU_SHARE}


def pair_bytes(r):
    """Algorithmic bytes of one update's balanced pair testing (k_pairs;
    zero unless the roadmap lists pairs) or, in the FP64 mode, of its item
    kernel (k_item64): the classify bytes less the FP32 item kernel's and the
    binary64 pass's."""
    return r.test_bytes - r.item_bytes - r.fp64_bytes


def item_bytes(r, fp64):
    """Algorithmic bytes of one update's item kernel: k_item32 (pair listing
    and the inline pair tests) in the FP32 mode, k_item64 in the FP64 mode."""
    return pair_bytes(r) if fp64 else r.item_bytes


def stages(ms, n, fp64):
    """Milliseconds per update of each stage from rgg_timing_read's sums."""
    n = max(n, 1)
    return {"diff": ms[0] / n, "cells": ms[1] / n, "item_kernel": (ms[3] if fp64 else ms[2]) / n,
            "pair_testing": 0.0 if fp64 else ms[3] / n, "fp64_pass": ms[4] / n, "labels": ms[5] / n}


def item_rooflines(kernel, timed, stage, fp64):
    """The item kernel's roofline (and the pair testing's, when it ran)."""
    out = {"roofline": roofline(kernel, float(np.mean([item_bytes(r, fp64) for r in timed])),
                                stage["item_kernel"])}
    pb = float(np.mean([pair_bytes(r) for r in timed]))
    if not fp64 and pb > 0:
        out["roofline_pairs"] = roofline(kernel.replace("k_item32", "k_pairs"), pb, stage["pair_testing"])
    return out


def roofline(kernel, bytes_per_launch, kernel_ms, note=None):
    """The HBM roofline of one kernel: algorithmic bytes per launch over its
    HIP-event launch time, against 8 TB/s."""
    if not kernel_ms or kernel_ms <= 0:
        return None
    achieved = bytes_per_launch / (kernel_ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "kernel": kernel, "bytes_per_launch": float(bytes_per_launch),
           "kernel_ms": float(kernel_ms)}
    if note:
        out["note"] = note
    return out


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by a plain copy of known size),
    or None when the kernel source changed since those counters were taken."""
    import glob
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    csrc = os.path.join(root, "paper_2603_28674_amd", "csrc")
    h = hashlib.sha256()
    for name in ("kernels.hip", "predicates64.h"):     # the update kernels' device source
        h.update(open(os.path.join(csrc, name), "rb").read())
    sha = h.hexdigest()
    for path in glob.glob(os.path.join(root, "profiles", "*.md")):
        for ln in open(path):
            if ln.startswith("traffic-record:"):
                rec = json.loads(ln.split(":", 1)[1])
                if rec["kernel"] == kernel and rec["source_sha256"] == sha:
                    return (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"]) * 1024.0
    return None


def batched_planar(a):
    """The batched configuration: 64 independent planar rigid-body roadmaps
    (node counts log-uniform in [1e3, 1e5], k = 8, U{20..400} boxes each,
    each update moving U{1..20} of them), FP32 tests + FP64 re-test.  One
    update round updates every roadmap once.  Plain: 64 rgg_update_async
    calls per round on one stream.  Batched: one rgg_batch_launch per round
    (one kernel launch per stage for all 64 roadmaps); batched_graph: the
    same stages as one captured-graph launch.  Every round's edges/s counts
    all edges of all roadmaps."""
    import torch
    from paper_2603_28674_amd import rgg, synth
    K, W = a.batched_steps, 2
    n_rounds = W + 6 * K
    t0 = time.perf_counter()
    ws = synth.batch_of_planar(seed=3, n_updates=n_rounds)
    log(f"[bench] batched: generated {len(ws)} roadmaps, {sum(w.n_edges for w in ws)} edges "
        f"in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    ctx = rgg.rgg_context_create(0)
    t0 = time.perf_counter()
    gs = [rgg.Roadmap.from_workload(ctx, w, precision=rgg.RGG_PREC_FP32_RECHECK,
                                    cell_size=a.batched_cell_size) for w in ws]
    log(f"[bench] batched: built in {time.perf_counter() - t0:.1f}s")
    E_tot = sum(w.n_edges for w in ws)
    bufs = []
    for w in ws:
        states = torch.from_numpy(np.stack([w.absent()] + w.boxes)).to(dev)
        bufs.append((states, torch.zeros(w.n_edges, dtype=torch.uint8, device=dev),
                     torch.zeros(w.n_edges, dtype=torch.int64, device=dev),
                     torch.zeros(rgg.RESULT_BYTES, dtype=torch.uint8, device=dev)))
    stream = torch.cuda.current_stream().cuda_stream

    def reqs(u):
        return [rgg.rgg_update_req(g.h.value, w.n_slots, st[u].data_ptr(), st[u + 1].data_ptr(),
                                   lab.data_ptr(), gr.data_ptr(), w.n_edges, res.data_ptr())
                for w, g, (st, lab, gr, res) in zip(ws, gs, bufs)]

    def plain(u):
        for q in reqs(u):
            rgg.lib().rgg_update_async(C_void(q.rm), C_void(stream), q.m, C_void(q.d_old), C_void(q.d_new),
                                       C_void(q.d_labels), C_void(q.d_gray), q.gray_cap, C_void(q.d_result))

    batch = rgg.rgg_batch_create(ctx, [g.h for g in gs])
    rq = [reqs(u) for u in range(n_rounds)]

    arrs = [(rgg.rgg_update_req * len(q))(*q) for q in rq]

    def batched(u):
        rgg.lib().rgg_batch_launch(batch, arrs[u], C_void(stream))

    def batched_graph(u):
        rgg.lib().rgg_batch_launch_graph(batch, arrs[u], C_void(stream))

    def timed(fn, u):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        host = 0.0
        for _ in range(K):
            h0 = time.perf_counter()
            fn(u)
            host += time.perf_counter() - h0
            u += 1
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return {"edges_per_s": E_tot * K / wall, "ms_per_round": wall / K * 1e3,
                "host_ms_per_round": host / K * 1e3}, u

    u = 0
    for _ in range(W):
        batched(u)
        u += 1
    torch.cuda.synchronize()
    out = {}
    # the built (heuristic) work decomposition, then the autotuned one
    out["batched_heuristic"], u = timed(batched, u)
    tuned = None
    if not a.no_tune:
        # one decomposition for the whole batch, timed on batched updates;
        # the state after rounds 0..u-1 is boxes[u-1], round u moves it to boxes[u]
        t0 = time.perf_counter()
        rep = rgg.rgg_batch_tune(batch, [w.boxes[u - 1] for w in ws], [w.boxes[u] for w in ws], reps=3)
        tuned = {"seconds": time.perf_counter() - t0, "item_edges": rep["item_edges"],
                 "cell_factor": None if not np.isfinite(rep["cell_size"]) else rep["cell_size"],
                 "us_per_round": rep["us_per_update"], "us_before": rep["us_before"],
                 "candidates": [{"item_edges": c["item_edges"],
                                 "cell_factor": None if not np.isfinite(c["cell_size"]) else c["cell_size"],
                                 "us": c["us"]} for c in rep["candidates"]]}
        log(f"[bench] batched: tuned in {tuned['seconds']:.1f}s")
    for name, fn in (("plain", plain), ("batched", batched), ("batched_graph", batched_graph)):
        out[name], u = timed(fn, u)
    lat, round_bytes = [], []
    for _ in range(K):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        batched(u)
        u += 1
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e6)
        round_bytes.append(sum(rgg.result_from_tensor(b[3]).test_bytes for b in bufs))
    ok = all(rgg.result_from_tensor(b[3]).status == 0 for b in bufs)
    # the classify kernels' algorithmic bytes of a round over the whole
    # round's time (every stage): a lower bound for the batched item kernel
    rb = float(np.mean(round_bytes))
    achieved = rb / (out["batched"]["ms_per_round"] * 1e-3) / 1e9
    # the stages' own times, HIP events on the stream between the kernels
    rgg.rgg_batch_timing_enable(batch, True)
    rgg.rgg_batch_timing_read(batch)
    batch_item_bytes = []   # the batched item kernels count their bytes as pair testing
    for _ in range(K):
        batched(u)
        u += 1
        torch.cuda.synchronize()
        batch_item_bytes.append(sum(pair_bytes(rgg.result_from_tensor(b[3])) for b in bufs))
    sms, nt = rgg.rgg_batch_timing_read(batch)
    rgg.rgg_batch_timing_enable(batch, False)
    ok = ok and all(rgg.result_from_tensor(b[3]).status == 0 for b in bufs)
    stage = {"diff": sms[0] / nt, "cells": sms[1] / nt, "item": sms[3] / nt, "fp64_pass": sms[4] / nt,
             "labels": sms[5] / nt}
    final_labels = [b[1].cpu().numpy() for b in bufs]
    cpu = None if a.no_cpu_baseline else batched_cpu_baseline(ws, final_labels, u, a.seed)
    rgg.rgg_batch_destroy(batch)
    for g in gs:
        g.close()
    rgg.rgg_context_destroy(ctx)
    return {
        "workload": "64 planar rigid-body roadmaps (4 disks; nodes log-uniform in [1e3, 1e5], k=8, "
                    "U{20..400} boxes, each update moves U{1..20}), FP32 + FP64 re-test",
        "roadmaps": len(ws), "edges": E_tot, "rounds": K, "cell_size": a.batched_cell_size,
        "autotune": tuned, "batched_heuristic": out["batched_heuristic"],
        "plain": out["plain"], "batched": out["batched"], "batched_graph": out["batched_graph"],
        "speedup_batched_vs_plain": out["batched"]["edges_per_s"] / out["plain"]["edges_per_s"],
        "batched_round_latency_p50_us": float(np.percentile(lat, 50)),
        "batched_round_latency_p99_us": float(np.percentile(lat, 99)),
        "roofline_round": {"bound": "hbm", "bytes_per_round": rb, "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                           "note": "classify bytes of all roadmaps per round over the round's wall time "
                                   "(all stages, pipelined rounds): a lower bound for k_item32_batch"},
        "stage_ms_per_round": stage,
        "roofline": roofline("k_item32_batch<2>", float(np.mean(batch_item_bytes)), stage["item"],
                             "classify bytes of the 64 roadmaps of a round over the batched item kernel's "
                             "HIP-event time"),
        "cpu_baseline": cpu,
        "status_ok": ok,
    }


def batched_cpu_baseline(ws, gpu_final, n_rounds, seed, per_roadmap=400):
    """The FP64 oracle over the batch's whole round sequence on a sample of
    every roadmap's edges (host cores of one GPU's share); also checks the
    GPU's final labels on those edges."""
    import oracle
    rng = np.random.default_rng(seed + 2000)
    threads = cpu_threads()
    tot, dt, match = 0, 0.0, True
    for w, lab in zip(ws, gpu_final):
        idx = np.sort(rng.choice(w.n_edges, size=min(per_roadmap, w.n_edges), replace=False))
        o = oracle.Roadmap(w.robot, w.q, w.edges[idx], w.resolution, w.samples_per_edge, w.n_slots, threads)
        t0 = time.perf_counter()
        prev = w.absent()
        ol = None
        for u in range(n_rounds):
            ol, _ = o.update(prev, w.boxes[u], threads=threads)
            prev = w.boxes[u]
        dt += time.perf_counter() - t0
        tot += len(idx) * n_rounds
        match = match and bool(np.array_equal(ol, lab[idx]))
    return {"value": tot / dt, "unit": "edges/s", "cores": threads, "kind": "oracle",
            "sample": f"{per_roadmap} edges of each of the {len(ws)} roadmaps (all of the smaller ones), "
                      f"{n_rounds} incremental updates each, FP64, {threads} threads",
            "labels_match_gpu_on_sample": match, "host": cpu_host()}


def plain_config(ctx, w, precision, cell_size, K, W, what, do_tune=True, kernel=None, cpu=None, item_edges=0,
                 **forms):
    """A further workload on the plain per-update path (rgg_update_async on
    one stream): pipelined throughput over K updates, the latency of K more,
    one at a time, then K more with the stages timed by HIP events (the
    classify kernel's roofline).  ``w`` must hold at least 1 + W + 3K
    updates.  ``cpu``: edges of the oracle's sample (the CPU baseline), or
    None."""
    import torch
    from paper_2603_28674_amd import rgg
    dev = torch.device("cuda:0")
    g = rgg.Roadmap.from_workload(ctx, w, precision=precision, cell_size=cell_size, item_edges=item_edges, **forms)
    info = g.info()
    E = w.n_edges
    states = torch.from_numpy(np.stack([w.absent()] + w.boxes)).to(dev)
    labels = torch.zeros(E, dtype=torch.uint8, device=dev)
    gray = torch.zeros(E, dtype=torch.int64, device=dev)
    res = torch.zeros((len(w.boxes), rgg.RESULT_BYTES), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream().cuda_stream

    def upd(u):
        g.update_async(stream, states[u], states[u + 1], labels, gray, res[u])

    upd(0)
    torch.cuda.synchronize()
    tuned = tune(g, w.boxes[0], w.boxes[1:9]) if do_tune else None
    info = g.info()
    for u in range(1, 1 + W):
        upd(u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for u in range(1 + W, 1 + W + K):
        upd(u)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = []
    for u in range(1 + W + K, 1 + W + 2 * K):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        upd(u)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e6)
    rgg.rgg_timing_enable(g.h, True)
    rgg.rgg_timing_read(g.h)
    for u in range(1 + W + 2 * K, 1 + W + 3 * K):
        upd(u)
    torch.cuda.synchronize()
    ms, n_timed = rgg.rgg_timing_read(g.h)
    rgg.rgg_timing_enable(g.h, False)
    timed = [rgg.result_from_tensor(res[u]) for u in range(1 + W + 2 * K, 1 + W + 3 * K)]
    results = [rgg.result_from_tensor(res[u]) for u in range(1 + W, 1 + W + 3 * K)]
    final = labels.cpu().numpy()
    g.close()
    stats = {k: float(np.mean([getattr(r, k) for r in results]))
             for k in ("n_changed", "n_pairs", "n_outer_hits", "n_rechecked", "n_gray", "test_bytes")}
    fp64 = precision == rgg.RGG_PREC_FP64
    stage = stages(ms, n_timed, fp64)
    out = {"workload": what, "edges": E, "obstacle_slots": w.n_slots,
           "precision": "fp64" if fp64 else "fp32+fp64 re-test",
           "cell_size": info["cell_size"], "item_edges": info["item_edges"], "autotune": tuned,
           "device_bytes": info["device_bytes"], "updates": K,
           "edges_per_s": E * K / wall, "ms_per_update": wall / K * 1e3,
           "latency_p50_us": float(np.percentile(lat, 50)),
           "latency_p99_us": float(np.percentile(lat, 99)),
           "stage_ms_per_update": stage,
           "per_update": stats, "status_ok": all(r.status == 0 for r in results)}
    if kernel:
        out.update(item_rooflines(kernel, timed, stage, fp64))
    if cpu:
        n_up = 1 + W + 3 * K - 1
        rng = np.random.default_rng(97)
        idx = np.sort(rng.choice(E, size=min(cpu, E), replace=False))
        threads = cpu_threads()
        rate, lab = oracle_rate(w, idx, n_up, threads, **forms)
        out["cpu_baseline"] = {"value": rate, "unit": "edges/s", "cores": threads, "kind": "oracle",
                               "sample": f"{len(idx)} of {E} edges, {n_up} incremental updates, FP64, "
                                         f"{threads} threads",
                               "labels_match_gpu_on_sample": bool(np.array_equal(lab, final[idx])),
                               "host": cpu_host()}
    return out


def other_configs(a):
    """The planar rigid-body roadmap (FP64, and FP32 + re-test beside it) and
    the planar arm, each on the plain path."""
    from paper_2603_28674_amd import rgg, synth
    K, W = a.steps, a.warmup
    ctx = rgg.rgg_context_create(0)
    out = {}
    w = synth.planar_rigid(n_updates=1 + W + 3 * K)
    what = ("planar rigid-body roadmap (4 disks, 2000 nodes, k=10, configurations every 0.05, "
            "50 boxes, 5 moved per update)")
    t = not a.no_tune
    cpu = None if a.no_cpu_baseline else 2000
    out["planar_fp64"] = plain_config(ctx, w, rgg.RGG_PREC_FP64, 0.0, K, W, what, t, "k_item64<2>", cpu)
    out["planar_fp32"] = plain_config(ctx, w, rgg.RGG_PREC_FP32_RECHECK, 0.0, K, W, what, t, "k_item32<2>")
    if not a.no_second_forms:
        # about 100 configurations per edge: the splines replace most copies
        pl = out["planar_fp32"]
        cell = pl["cell_size"] if pl["cell_size"] is not None and np.isfinite(pl["cell_size"]) else -1.0
        out["planar_splines"] = plain_config(ctx, w, rgg.RGG_PREC_FP32_RECHECK, cell, K, W, what + ", spline form",
                                             False, "k_item32<2>", None if a.no_cpu_baseline else 2000,
                                             item_edges=pl["item_edges"], inner_splines=True)
    log("[bench] arm workload")
    w = synth.planar_arm(n_updates=1 + W + 3 * K)
    what = ("planar 7-link arm (3 spheres per link, 100k nodes, k=8, 20 configurations/edge, "
            "300 boxes, 30 moved per update)")
    cpu = None if a.no_cpu_baseline else 20000
    out["arm_fp32"] = plain_config(ctx, w, rgg.RGG_PREC_FP32_RECHECK, 0.0, K, W, what, t, "k_item32<2>", cpu)
    if not a.no_second_forms:
        # the second forms of Sec. 4.2 on the arm, in the decomposition the
        # capsule form was tuned to
        arm = out["arm_fp32"]
        cell = arm["cell_size"] if arm["cell_size"] is not None and np.isfinite(arm["cell_size"]) else -1.0
        cpu = None if a.no_cpu_baseline else 4000
        for name, forms in (("arm_obb", dict(outer_obb=True)),
                            ("arm_obb_splines", dict(outer_obb=True, inner_splines=True))):
            log(f"[bench] {name}")
            out[name] = plain_config(ctx, w, rgg.RGG_PREC_FP32_RECHECK, cell, K, W, what + f", {name[4:]} form",
                                     False, "k_item32<2>", cpu, item_edges=arm["item_edges"], **forms)
    rgg.rgg_context_destroy(ctx)
    return out


def serving(a):
    """The serving configuration: 16 device-resident roadmaps (8 spatial
    rigid-body, 8 planar arm; edge counts log-uniform in [1e4, 5e5]) behind
    the request server (4 streams, batches of up to 64, the box pool sized
    from the free device memory).  Open-loop Poisson arrivals at 100, 1000
    and 10000 requests/s, each moving U{1..50} boxes of a random roadmap.
    Latency is the server's, from submit to completion, split into the wait
    for a launch (queue) and the launch to completion (service); edges/s
    counts the edges of every completed request."""
    import torch
    from paper_2603_28674_amd import rgg, synth
    t0 = time.perf_counter()
    ws = synth.serving_mix(seed=5)
    log(f"[bench] serving: generated {len(ws)} roadmaps, {sum(w.n_edges for w in ws)} edges "
        f"in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    ctx = rgg.rgg_context_create(0)
    t0 = time.perf_counter()
    gs = [rgg.Roadmap.from_workload(ctx, w, precision=rgg.RGG_PREC_FP32_RECHECK, cell_size=0.0) for w in ws]
    log(f"[bench] serving: built in {time.perf_counter() - t0:.1f}s")
    labs = [torch.zeros(w.n_edges, dtype=torch.uint8, device=dev) for w in ws]
    grays = [torch.zeros(w.n_edges, dtype=torch.int64, device=dev) for w in ws]
    for g, w in zip(gs, ws):
        g.update(w.absent(), w.boxes[0], want_labels=False)
    tuned = None
    if not a.no_tune:
        # each roadmap tuned on four moves of 25 boxes (the middle of the
        # requests' 1..50), before the server holds it
        t0 = time.perf_counter()
        trng = np.random.default_rng(a.seed + 78)
        chosen = []
        for g, w in zip(gs, ws):
            sigma = 0.3 if w.robot.kind == synth.SE3 else 2.0
            bs = [synth.move_sequence(trng, w.boxes[0], w.robot.dim, 1, 25, sigma)[1] for _ in range(4)]
            chosen.append(tune(g, w.boxes[0], bs, reps=2))
        tuned = {"seconds": time.perf_counter() - t0,
                 "item_edges": {str(v): sum(r["item_edges"] == v for r in chosen)
                                for v in sorted({r["item_edges"] for r in chosen})},
                 "one_cell": sum(r["cell_size"] is None for r in chosen)}
        log(f"[bench] serving: tuned in {tuned['seconds']:.1f}s")
    vers = [torch.zeros(w.n_edges, dtype=torch.uint8, device=dev) for w in ws]
    srv = rgg.rgg_server_start(ctx, n_streams=4, max_batch=64, pool_bytes=0)
    srv_info = rgg.rgg_server_info(srv)
    rng = np.random.default_rng(a.seed + 77)
    cur = [w.boxes[0] for w in ws]
    levels = []
    ok = True

    def run_rate(rate, validate):
        nonlocal cur, ok
        reqs, cur = synth.serving_requests(rng, ws, rate, a.serving_seconds, start=cur)
        tickets = []
        busy = 0
        t0 = time.perf_counter()
        for (ta, r, old, new) in reqs:
            while time.perf_counter() - t0 < ta:
                pass
            while True:
                try:
                    t = rgg.rgg_server_submit(srv, gs[r].h, old, new, labs[r].data_ptr(), grays[r].data_ptr(),
                                              ws[r].n_edges, validate=validate, d_verdict=vers[r].data_ptr())
                    break
                except rgg.RggError as e:
                    if e.status != rgg.RGG_E_BUSY:
                        raise
                    busy += 1
                    time.sleep(20e-6)
            tickets.append((t, ws[r].n_edges))
        lat, que, svc, bsz, edges = [], [], [], [], 0
        for t, e in tickets:
            done, res, tm = rgg.rgg_server_poll_timing(srv, t, wait=True)
            ok = ok and res.status == 0
            lat.append(tm["latency_us"])
            que.append(tm["queue_us"])
            svc.append(tm["service_us"])
            bsz.append(tm["batch_size"])
            edges += e
        wall = time.perf_counter() - t0
        lat, que, svc, bsz = np.array(lat), np.array(que), np.array(svc), np.array(bsz)
        tail = lat >= np.percentile(lat, 99)
        return {"offered_rate": rate, "requests": len(tickets), "achieved_rate": len(tickets) / wall,
                "edges_per_s": edges / wall, "latency_p50_us": float(np.percentile(lat, 50)),
                "latency_p99_us": float(np.percentile(lat, 99)), "latency_mean_us": float(lat.mean()),
                "queue_p50_us": float(np.percentile(que, 50)), "queue_p99_us": float(np.percentile(que, 99)),
                "service_p50_us": float(np.percentile(svc, 50)), "service_p99_us": float(np.percentile(svc, 99)),
                "batch_size_mean": float(bsz.mean()),
                "slowest_1pct": {"requests": int(tail.sum()), "latency_mean_us": float(lat[tail].mean()),
                                 "queue_mean_us": float(que[tail].mean()),
                                 "service_mean_us": float(svc[tail].mean()),
                                 "batch_size_mean": float(bsz[tail].mean())},
                "busy_retries": busy}

    for rate in (100.0, 1000.0, 10000.0):
        levels.append(run_rate(rate, False))
        log(f"[bench] serving at {rate:.0f}/s: {levels[-1]}")
    # non-lazy requests: each update followed by the full validation of its
    # gray list, the labels rewritten to green / red
    non_lazy = run_rate(1000.0, True)
    log(f"[bench] serving non-lazy at 1000/s: {non_lazy}")
    rgg.rgg_server_stop(srv)
    for g in gs:
        g.close()
    rgg.rgg_context_destroy(ctx)
    return {"workload": "16 resident roadmaps: 8 spatial rigid-body + 8 planar-arm, edges log-uniform in "
                        "[1e4, 5e5]; Poisson requests moving U{1..50} boxes; FP32 + FP64 re-test",
            "roadmaps": len(ws), "edges": int(sum(w.n_edges for w in ws)), "seconds_per_rate": a.serving_seconds,
            "autotune": tuned,
            "server": srv_info, "rates": levels,
            "non_lazy": non_lazy,
            "status_ok": bool(ok)}


def tune(g, a_boxes, b_states, reps=2, full=False):
    """Runs the library's autotuner on the updates a -> b -> a for every b of
    ``b_states`` (a is the roadmap's current state); returns a short summary
    (every candidate when ``full``)."""
    rep = g.tune(a_boxes, b_states, reps=reps)
    out = {"item_edges": rep["item_edges"],
           "cell_size": None if not np.isfinite(rep["cell_size"]) else rep["cell_size"],
           "us_per_update": rep["us_per_update"], "us_before": rep["us_before"]}
    if full:
        out["candidates"] = [{"item_edges": c["item_edges"],
                              "cell_size": None if not np.isfinite(c["cell_size"]) else c["cell_size"],
                              "us": c["us"]} for c in rep["candidates"]]
    return out


def C_void(x):
    import ctypes
    return ctypes.c_void_p(x)


def oracle_rate(w, idx, n_updates, threads, **forms):
    """Edges/s of the FP64 oracle's incremental update over updates
    1..n_updates on the edges idx; returns (rate, final labels)."""
    import oracle
    o = oracle.Roadmap(w.robot, w.q, w.edges[idx], w.resolution, w.samples_per_edge,
                       w.n_slots, threads, **forms)
    o.update(w.absent(), w.boxes[0], threads=threads)
    t0 = time.perf_counter()
    lab = None
    for u in range(1, n_updates + 1):
        lab, _ = o.update(w.boxes[u - 1], w.boxes[u], threads=threads)
    return len(idx) * n_updates / (time.perf_counter() - t0), lab


def cpu_baseline(w, gpu_labels_final, sample_edges, n_updates, seed, single_edges):
    """The FP64 oracle, incremental mode, on a sample of the roadmap's edges
    (every edge by default), over the same obstacle sequence, on one GPU's
    share of the host's cores (16, or fewer if the process may use fewer);
    also checks the GPU's final labels on that sample.  Beside it, the
    oracle on one thread over a smaller sample."""
    rng = np.random.default_rng(seed + 1000)
    E = w.n_edges
    idx = np.sort(rng.choice(E, size=min(sample_edges, E), replace=False))
    threads = cpu_threads()
    rate, lab = oracle_rate(w, idx, n_updates, threads)
    out = {
        "value": rate,
        "unit": "edges/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{len(idx)} of {E} edges, {n_updates} incremental updates, FP64, "
                  f"{threads} threads",
        "labels_match_gpu_on_sample": bool(np.array_equal(lab, gpu_labels_final[idx])),
        "host": cpu_host(),
    }
    if single_edges > 0:
        idx1 = np.sort(rng.choice(E, size=min(single_edges, E), replace=False))
        rate1, _ = oracle_rate(w, idx1, n_updates, 1)
        out["single_thread"] = {"value": rate1, "unit": "edges/s", "cores": 1,
                                "sample": f"{len(idx1)} of {E} edges, {n_updates} incremental "
                                          f"updates, FP64, 1 thread"}
    return out


def copy_bandwidth(torch, dev):
    """HBM bandwidth a plain device-to-device copy of 1 GiB reaches (read +
    write bytes over the HIP-event time of 10 copies)."""
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * src.numel() * 4 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return gbs


def validate_pass(a, torch, rgg, g, w, stream, gray, res_last, last, reps=5):
    """Times rgg_validate_async over the gray list of update `last` (HIP
    events on the update stream) and the oracle on a sample of it."""
    E = w.n_edges
    r = rgg.result_from_tensor(res_last)
    n = int(r.n_gray)
    dev = gray.device
    ver = torch.zeros(max(n, 1), dtype=torch.uint8, device=dev)
    lev = torch.zeros(max(n, 1), dtype=torch.int32, device=dev)
    wit = torch.zeros(max(n, 1), dtype=torch.float64, device=dev)
    rgg.rgg_validate_async(g.h, stream, gray, n, res_last, ver, lev, wit)   # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        rgg.rgg_validate_async(g.h, stream, gray, n, res_last, ver, lev, wit)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    v = ver[:n].cpu().numpy()
    lv = lev[:n].cpu().numpy()
    out = {"gray_edges": n, "ms": ms, "gray_edges_per_s": n / (ms * 1e-3) if ms > 0 else None,
           "free": int(np.sum(v == rgg.RGG_VERDICT_FREE)),
           "collides": int(np.sum(v == rgg.RGG_VERDICT_COLLIDES)),
           "unresolved": int(np.sum(v == rgg.RGG_VERDICT_UNRESOLVED)),
           "level_mean": float(lv.mean()) if n else 0.0, "level_max": int(lv.max(initial=0)),
           "max_level": rgg.RGG_VALIDATE_DEFAULT_LEVELS, "max_active": rgg.RGG_VALIDATE_DEFAULT_ACTIVE,
           "cpu_oracle": None}
    if not a.no_cpu_baseline and n:
        import oracle
        ids = gray[:n].cpu().numpy()
        rng = np.random.default_rng(a.seed)
        sample = np.sort(rng.choice(ids, size=min(n, a.cpu_validate_edges), replace=False))
        threads = cpu_threads()
        o = oracle.Roadmap(w.robot, w.q, w.edges[sample], w.resolution, w.samples_per_edge, w.n_slots, threads)
        o.classify(w.boxes[last])
        t0 = time.perf_counter()
        ov, _, _ = o.validate(np.arange(len(sample)))
        dt = time.perf_counter() - t0
        at = np.searchsorted(ids, sample)
        out["cpu_oracle"] = {"gray_edges_per_s": len(sample) / dt, "cores": threads, "kind": "oracle",
                             "sample": f"{len(sample)} of the {n} gray edges",
                             "verdicts_equal": bool(np.array_equal(ov, v[at]))}
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the update path is not "
              f"sharded across GPUs", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2603_28674_amd import rgg, synth

    if a.only:
        out = {"only": a.only}
        if a.only == "arm":
            a.no_second_forms = True
            K, W = a.steps, a.warmup
            ctx = rgg.rgg_context_create(0)
            w = synth.planar_arm(n_updates=1 + W + 3 * K)
            out["arm_fp32"] = plain_config(ctx, w, rgg.RGG_PREC_FP32_RECHECK, a.cell_size, K, W, "planar arm",
                                           not a.no_tune, "k_item32<2>", None, item_edges=a.item_edges)
        else:
            out["batched_planar"] = batched_planar(a)
        if a.copy_calibration:
            copy_calibration(torch)
        print(json.dumps(out), flush=True)
        return

    K, W = a.steps, a.warmup
    n_updates = W + 5 * K
    log(f"[bench] generating spatial workload: {a.nodes} nodes, {n_updates} updates")
    w = synth.spatial_rigid(seed=a.seed, n_nodes=a.nodes, n_updates=n_updates)
    E, M = w.n_edges, w.n_slots
    dev = torch.device("cuda:0")
    ctx = rgg.rgg_context_create(0)
    log(f"[bench] building roadmap E={E} M={M}")
    g = rgg.Roadmap.from_workload(ctx, w, precision=rgg.RGG_PREC_FP32_RECHECK,
                                  cell_size=a.cell_size, item_edges=a.item_edges)
    info = g.info()
    log(f"[bench] built in {info['build_seconds']:.2f}s, device {info['device_bytes'] / 1e9:.2f} GB, "
        f"grid {info['grid_cells']}")
    states = torch.from_numpy(np.stack([w.absent()] + w.boxes)).to(dev)   # [U+2, M, 6]
    labels = torch.zeros(E, dtype=torch.uint8, device=dev)
    gray = torch.zeros(E, dtype=torch.int64, device=dev)
    res = torch.zeros((n_updates + 2, rgg.RESULT_BYTES), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream().cuda_stream

    def upd(u):   # update u: states[u] -> states[u+1]
        g.update_async(stream, states[u], states[u + 1], labels, gray, res[u])

    upd(0)        # first obstacle set (untimed)
    torch.cuda.synchronize()
    tuned = None
    if not a.no_tune:
        log("[bench] autotuning the work decomposition")
        tuned = tune(g, w.boxes[0], w.boxes[1:9], full=True)
        info = g.info()
    for u in range(1, 1 + W):
        upd(u)
    torch.cuda.synchronize()

    # pass 1: pipelined throughput (the value)
    first = 1 + W
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for u in range(first, first + K):
        upd(u)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    results = [rgg.result_from_tensor(res[u]) for u in range(first, first + K)]
    assert all(r.status == 0 for r in results), "update failed"

    # pass 2: stage times, HIP events recorded on the update stream between
    # the kernels (the events themselves add gaps, so this pass is not the value)
    rgg.rgg_timing_enable(g.h, True)
    rgg.rgg_timing_read(g.h)
    for u in range(first + K, first + 2 * K):
        upd(u)
    torch.cuda.synchronize()
    ms, n_timed = rgg.rgg_timing_read(g.h)
    rgg.rgg_timing_enable(g.h, False)
    results += [rgg.result_from_tensor(res[u]) for u in range(first + K, first + 2 * K)]
    assert all(r.status == 0 for r in results), "update failed"

    # pass 3: latency, one update at a time
    lat = []
    for u in range(first + 2 * K, first + 3 * K):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        upd(u)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e6)
    lat = np.array(lat)

    # pass 3b: the same, with the caches cold: a 1 GiB buffer is rewritten
    # before each update (more than the 256 MB Infinity Cache and the L2s)
    flush = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    lat_cold = []
    rgg.rgg_timing_enable(g.h, True)
    rgg.rgg_timing_read(g.h)
    for u in range(first + 3 * K, first + 4 * K):
        flush.fill_(float(u))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        upd(u)
        torch.cuda.synchronize()
        lat_cold.append((time.perf_counter() - t1) * 1e6)
    ms_cold, n_cold = rgg.rgg_timing_read(g.h)
    rgg.rgg_timing_enable(g.h, False)
    del flush
    lat_cold = np.array(lat_cold)
    results += [rgg.result_from_tensor(res[u]) for u in range(first + 2 * K, first + 4 * K)]
    assert all(r.status == 0 for r in results), "update failed"
    cold_bytes = float(np.mean([item_bytes(r, False) for r in results[3 * K:4 * K]]))
    final_labels = labels.cpu().numpy()
    last = first + 4 * K - 1

    # pass 3d: full validation of the last update's gray list (the non-lazy
    # step after the classification), chained on the device after the
    # update; the oracle validates a sample of the same edges on the host
    validation = None
    if not a.no_validate:
        validation = validate_pass(a, torch, rgg, g, w, stream, gray, res[last], last)

    # pass 3c: the host-buffer entry point (boxes from host memory, labels and
    # gray ids back to host memory), continuing the same sequence: the
    # PCIe-inclusive rate, reported beside the value, never as it
    host_lat = []
    cur_u = first + 4 * K
    n_host = min(K, len(w.boxes) - cur_u)
    for u in range(cur_u, cur_u + n_host):
        t1 = time.perf_counter()
        g.update(w.boxes[u - 1], w.boxes[u])
        host_lat.append((time.perf_counter() - t1) * 1e6)
    host_lat = np.array(host_lat) if host_lat else np.array([0.0])

    # pass 4: the same kind of updates as HIP graphs (one graph per update,
    # instantiated before timing), replaying the sequence from the start
    graph = None
    if not a.skip_graph:
        cell2 = info["cell_size"] if np.isfinite(info["cell_size"]) else -1.0
        g2 = rgg.Roadmap.from_workload(ctx, w, precision=rgg.RGG_PREC_FP32_RECHECK,
                                       cell_size=cell2, item_edges=info["item_edges"])
        lab2 = torch.zeros(E, dtype=torch.uint8, device=dev)
        gray2 = torch.zeros(E, dtype=torch.int64, device=dev)
        res2 = torch.zeros((n_updates + 2, rgg.RESULT_BYTES), dtype=torch.uint8, device=dev)
        gr = []
        for u in range(0, 1 + W + K):
            req = rgg.rgg_update_req(g2.h.value, M, states[u].data_ptr(), states[u + 1].data_ptr(),
                                     lab2.data_ptr(), gray2.data_ptr(), E, res2[u].data_ptr())
            gr.append(rgg.rgg_graph_create(ctx, [req]))
        for u in range(0, 1 + W):
            rgg.rgg_graph_launch(gr[u], stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for u in range(1 + W, 1 + W + K):
            rgg.rgg_graph_launch(gr[u], stream)
        torch.cuda.synchronize()
        gwall = time.perf_counter() - t0
        graph = {"edges_per_s": E * K / gwall, "ms_per_step": gwall / K * 1e3}
        for h in gr:
            rgg.rgg_graph_destroy(h)
        g2.close()

    timed_res = results[K:2 * K]   # the event-timed updates
    st = stages(ms, n_timed, False)
    test_bytes = float(np.mean([item_bytes(r, False) for r in timed_res]))
    stats_tp = {k: float(np.mean([getattr(r, k) for r in results[:K]]))   # the throughput pass
                for k in ("n_pairs", "n_outer_hits", "test_bytes")}
    copy_gbs = copy_bandwidth(torch, dev)
    test_ms = st["item_kernel"]
    achieved = test_bytes / (test_ms * 1e-3) / 1e9
    stats = {k: float(np.mean([getattr(r, k) for r in results]))
             for k in ("n_changed", "n_candidate_edges", "n_pairs", "n_outer_hits", "n_rechecked",
                       "n_cells_visited", "n_gray")}
    line = {
        "metric": "edges classified/sec + p99 update latency, batched vs plain, labels = oracle",
        "value": E * K / wall,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": wall / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "spatial rigid-body roadmap (8 spheres, 50k nodes, k=10, 20 "
                               "configurations/edge, 500 boxes, 50 moved per update), "
                               "FP32 tests + FP64 re-test inside a 1e-5 relative margin band",
                   "nodes": a.nodes, "edges": E, "obstacle_slots": M, "mode": "plain stream",
                   "cell_size": info["cell_size"], "grid_cells": info["grid_cells"],
                   "item_edges": info["item_edges"], "autotune": tuned},
        "latency_p50_us": float(np.percentile(lat, 50)),
        "latency_p99_us": float(np.percentile(lat, 99)),
        "latency_mean_us": float(lat.mean()),
        "latency_cold_p50_us": float(np.percentile(lat_cold, 50)),
        "latency_cold_p99_us": float(np.percentile(lat_cold, 99)),
        "graph": graph,
        "validation": validation,
        "host_buffers": {"edges_per_s": E / (host_lat.mean() * 1e-6), "latency_p50_us": float(np.percentile(host_lat, 50)),
                         "latency_p99_us": float(np.percentile(host_lat, 99)), "updates": int(n_host),
                         "note": "rgg_update: boxes uploaded from host memory, labels and gray ids "
                                 "copied back to host memory; one update at a time"},
        "stage_ms_per_update": st,
        "per_update": stats,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("k_item32<3>"),
                     "kernel": "k_item32<3>", "bytes_per_launch": test_bytes,
                     "kernel_ms": test_ms, "copy_GBps": copy_gbs,
                     "frac_of_copy": achieved / copy_gbs},
        "roofline_cold": roofline("k_item32<3>", cold_bytes, stages(ms_cold, n_cold, False)["item_kernel"],
                                  "the same kernel with the caches flushed before every update (a 1 GiB "
                                  "buffer rewritten: more than the 256 MB Infinity Cache)"),
        "work_rates": {"pairs_per_s": stats_tp["n_pairs"] * K / wall,
                       "outer_hits_per_s": stats_tp["n_outer_hits"] * K / wall,
                       "classify_bytes_per_s": stats_tp["test_bytes"] * K / wall},
        "cpu_baseline": None,
    }
    if not a.no_cpu_baseline:
        log("[bench] cpu baseline (oracle on a sample)")
        line["cpu_baseline"] = cpu_baseline(w, final_labels, a.cpu_sample_edges, last, a.seed,
                                            a.cpu_single_edges)
    g.close()
    if not a.no_second_forms:
        # the second forms of Sec. 4.2 on the same roadmap and updates, in the
        # decomposition the capsule form was tuned to
        cell2 = info["cell_size"] if np.isfinite(info["cell_size"]) else -1.0
        forms_out = {}
        what = line["config"]["workload"]
        cpu = None if a.no_cpu_baseline else 2000
        for name, forms in (("capsules", dict()), ("obb", dict(outer_obb=True)),
                            ("splines", dict(inner_splines=True)),
                            ("obb_splines", dict(outer_obb=True, inner_splines=True))):
            log(f"[bench] spatial, {name} form")
            forms_out[name] = plain_config(ctx, w, rgg.RGG_PREC_FP32_RECHECK, cell2, K, W, what + f", {name} form",
                                           False, "k_item32<3>", cpu, item_edges=info["item_edges"], **forms)
        line["second_forms"] = forms_out
    if not a.no_other_configs:
        log("[bench] planar and arm workloads")
        line["other_workloads"] = other_configs(a)
    if not a.no_batched:
        log("[bench] batched planar roadmaps")
        line["batched_planar"] = batched_planar(a)
    if not a.no_serving:
        log("[bench] serving")
        line["serving"] = serving(a)
    if a.copy_calibration:
        line["copy_calibration_bytes"] = copy_calibration(torch)
    print(json.dumps(line), flush=True)


def copy_calibration(torch):
    """A plain 1 GiB device copy, 5 times, and a 1 GiB fill: the reference
    kernels of known size for scaling FETCH_SIZE / WRITE_SIZE."""
    dev = torch.device("cuda:0")
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    return src.numel() * 4


if __name__ == "__main__":
    main()
