#!/usr/bin/env python3
"""Benchmark of the octree FMM gravity solve on one MI355X.

A step is one whole solve (upward pass, same-level interactions of all
classes, downward pass) of one batch of synthetic input already resident in
HBM.  The headline workload is the uniform level-3 octree (585 sub-grids,
64^3 leaf cells, one n = 1.5 polytrope) in FP64; the JSON line also carries
the mixed-precision form, the binary-star AMR field and the batch of 16
binary-star octrees, the dominant kernel's roofline (timed with HIP events on
the solve's stream) and the CPU oracle timed on this host's cores.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms all|c1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-interactions/sec & % FP64/FP32 peak, FP64 vs mixed vs batched, at stated err"
PEAK_FP64 = 78.6e12      # MI355X FP64 vector, FLOP/s
PEAK_FP32 = 157.3e12     # MI355X FP32 vector (packed), FLOP/s
PEAK_HBM = 8.0e12        # bytes/s

# Arithmetic of one ordered pair in the kernels' formulation (FMA = 2 flop):
FLOP_PAIR_REFINED = 203  # refined target: L0..L3 (order 3) + correction (79 FMA, 35 MUL, 9 ADD, 1 RSQ)
FLOP_PAIR_LEAF_MP = 127  # leaf target, multipole source: L0, L1 + correction (45 FMA, 27 MUL, 9 ADD, 1 RSQ)
FLOP_PAIR_MONO = 6       # leaf <- leaf monopole, lattice kernel tables: 3 FMA


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_flops(st):
    p = st["pairs"]
    return (FLOP_PAIR_REFINED * (p[0] + p[1] + st["pairs_top"]) + FLOP_PAIR_MONO * p[2]
            + FLOP_PAIR_LEAF_MP * p[3])


def parse_shape(spec):
    """'per_class_g5_b3_o1' or 'persistent_g2_b3_o0' -> Plan keyword arguments."""
    kind, rest = spec.split("_g")
    g, b, o = rest.split("_")
    assert kind in ("per_class", "persistent") and b[0] == "b" and o[0] == "o", spec
    return dict(persistent=kind == "persistent", plane_groups=int(g), blocks_per_cu=int(b[1:]),
                overlap=int(o[1:]))


def time_form(fm, torch, trees, rho_np, precision, steps, warmup, use_graph=True, shape=None):
    """Plans with the launch-shape tuner (its timing runs happen in the first,
    untimed solve; no cache file, so every run tunes on its own), or in the
    given shape, then times `steps` graph replays."""
    dev = torch.device("cuda:0")
    rho = torch.tensor(rho_np, dtype=torch.float64, device=dev)
    kw = shape if shape is not None else dict(autotune=True, overlap=2)
    with fm.Plan(trees, precision=precision, use_graph=use_graph, **kw) as plan:
        phi, g = plan.solve(rho)
        shape = plan.launch_shape()
        for _ in range(warmup):
            plan.solve(rho, phi, g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.solve(rho, phi, g)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        st = plan.stats()
    pairs = st["total_pairs"]
    out = {"ms_per_step": dt * 1e3, "pairs_per_step": pairs,
           "cell_interactions_per_s": pairs / dt,
           "paper_convention_gflops": st["paper_flops"] / dt / 1e9,
           "algorithmic_tflops": algorithmic_flops(st) / dt / 1e12,
           "launches_per_step": st["launches"], "n_leaves": st["n_leaves"],
           "n_trees": st["n_trees"], "launch_shape": shape}
    peak = PEAK_FP64 if precision == "fp64" else PEAK_FP32
    out["frac_peak"] = algorithmic_flops(st) / dt / peak
    return out, phi.cpu().numpy(), g.cpu().numpy(), st


def time_paper_model(fm, torch, trees, rho_np, precision, steps, warmup, groups, ref, streams=128):
    """The paper's execution model (Sec. 5.1) on the same work items: eager
    solves with one launch per target sub-grid and class, round-robin over a
    pool of `streams` streams.  `ref` = (phi, g) of the default shape with the
    same plane groups, which it must reproduce bitwise."""
    import numpy as np
    dev = torch.device("cuda:0")
    rho = torch.tensor(rho_np, dtype=torch.float64, device=dev)
    with fm.Plan(trees, precision=precision, plane_groups=groups, launch_streams=streams) as plan:
        phi, g = plan.solve(rho)
        for _ in range(warmup):
            plan.solve(rho, phi, g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.solve(rho, phi, g)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        st = plan.stats()
    same = bool(np.array_equal(phi.cpu().numpy(), ref[0]) and np.array_equal(g.cpu().numpy(), ref[1]))
    return {"ms_per_step": dt * 1e3, "cell_interactions_per_s": st["total_pairs"] / dt,
            "launches_per_step": st["launches"], "streams": streams, "plane_groups": groups,
            "launch": "eager", "bitwise_equal_to_default_shape": same}


def stage_times(fm, torch, trees, rho_np, precision, steps, warmup, shape):
    """Eager solves in the given launch shape, without the overlap's coarse
    branch (so every class is one launch), with HIP events at every stage
    boundary on the solve's stream."""
    dev = torch.device("cuda:0")
    rho = torch.tensor(rho_np, dtype=torch.float64, device=dev)
    with fm.Plan(trees, precision=precision, timing=True, persistent=bool(shape["persistent"]),
                 plane_groups=shape["plane_groups"], blocks_per_cu=shape["blocks_per_cu"],
                 overlap=0) as plan:
        phi, g = plan.solve(rho)
        for _ in range(warmup):
            plan.solve(rho, phi, g)
        torch.cuda.synchronize()
        plan.timings()  # discard warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.solve(rho, phi, g)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        tm = plan.timings()
        st = plan.stats()
    n = tm["solves"]
    return {k: v / n for k, v in tm["ms"].items()}, tm["launches"], wall * 1e3, st


def residuals(np, trees, rho, g):
    """Relative total force and torque |sum| / sum |.| of the leaf accelerations."""
    F_all, T_all = [], []
    off = 0
    for t in trees:
        n = t.n_leaves
        x = t.leaf_cell_centres().reshape(-1, 3) - 0.5
        h = t.leaf_cell_size()
        m = (rho[off:off + n] * (h ** 3)[:, None, None, None]).reshape(-1)
        F = m[:, None] * g[off:off + n].transpose(0, 2, 1).reshape(-1, 3)
        F_all.append(F)
        T_all.append(np.cross(x, F))
        off += n
    res_f = max(float(np.abs(F.sum(0)).max() / np.abs(F).sum(0).max()) for F in F_all)
    res_t = max(float(np.abs(T.sum(0)).max() / np.abs(T).sum(0).max()) for T in T_all)
    return res_f, res_t


def field_err(np, phi, g, pr, gr):
    e = {"phi": float(np.abs(phi - pr).max() / np.abs(pr).max())}
    for a, n in enumerate("xyz"):
        e["g" + n] = float(np.abs(g[:, a] - gr[:, a]).max() / np.abs(gr[:, a]).max())
    return e


def traffic_entry(kernel_name):
    """HBM bytes per solve of the timed stage's launches, from committed
    rocprofv3 counter runs; valid only while the kernel source is unchanged
    (source hash recorded with them)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    src = os.path.join(ROOT, "paper_1908_03121_amd", "csrc", "kernels.hip")
    try:
        with open(path) as f:
            tab = json.load(f)
        with open(src, "rb") as f:
            h = hashlib.sha256(f.read()).hexdigest()
        e = tab.get(kernel_name)
        if e and e.get("kernels_hip_sha256") == h:
            return float(e["bytes_per_solve"])
    except (OSError, ValueError, KeyError):
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # a c1 solve takes about 0.2 ms: 100 steps keep the timed region long
    # enough (about 20 ms) that a short host or clock hiccup does not dominate it
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--forms", default="all", choices=["all", "c1", "c2-stages"],
                    help="c2-stages: only eager, stage-timed c2 FP64 solves in the per-class "
                         "shape (one launch per class), for a kernel trace of the classes' shares")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--profile", action="store_true",
                    help="short run for hardware counters: 3 eager c1 FP64 solves in the launch "
                         "shape --shape (no overlap: one launch per class, as in the timing "
                         "solves), then a 256 MiB device-to-device copy whose byte "
                         "counters calibrate the ones of the solve kernels")
    ap.add_argument("--bpc", type=int, default=0,
                    help="--profile: blocks per CU of the persistent launch (0 = occupancy limit)")
    ap.add_argument("--shape", default="per_class_g2",
                    choices=[f"{k}_g{g}" for k in ("per_class", "persistent") for g in (1, 2, 3, 5)])
    ap.add_argument("--c1-shape", default=None,
                    help="launch shape of the c1 FP64 form instead of the tuner's choice, e.g. "
                         "per_class_g5_b3_o1 or persistent_g2_b3_o0 (a profiled run uses the "
                         "shape an unprofiled run tuned to)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this library runs on exactly one GPU (asked for {args.gpus}); "
              "sharding the octree over several GPUs (by sub-grid ranges, with halo exchanges "
              "per level) is designed but not built.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1908_03121_amd as fm
    from paper_1908_03121_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    fm.lib()
    K, W = args.steps, args.warmup

    if args.profile:
        c1 = wl.c1()
        dev = torch.device("cuda:0")
        rho = torch.tensor(c1.rho, dtype=torch.float64, device=dev)
        pers, groups = args.shape.split("_g")
        with fm.Plan(c1.trees, persistent=pers == "persistent", plane_groups=int(groups), overlap=0,
                     blocks_per_cu=args.bpc) as plan:
            phi, g = plan.solve(rho)
            for _ in range(2):
                plan.solve(rho, phi, g)
            torch.cuda.synchronize()
            st = plan.stats()
        n = 256 * 2 ** 20 // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile": "c1_fp64", "shape": args.shape, "bpc": args.bpc, "solves": 3,
                          "pairs": st["pairs"],
                          "pairs_top": st["pairs_top"], "copy_bytes_each_way": n * 8}), flush=True)
        return

    if args.forms == "c2-stages":
        log("generating c2 (binary-star AMR field)")
        c2 = wl.c2()
        shape = dict(persistent=0, plane_groups=1, blocks_per_cu=0)
        stages, launches, wall, st = stage_times(fm, torch, c2.trees, c2.rho, "fp64", min(K, 10),
                                                 min(W, 3), shape)
        print(json.dumps({"profile": "c2_fp64_stages", "shape": "per_class_g1", "stages_ms": stages,
                          "launches": launches, "eager_ms_per_step": wall, "pairs": st["pairs"],
                          "pairs_top": st["pairs_top"]}), flush=True)
        return

    log("generating c1 (uniform level-3 octree, 64^3 leaf cells)")
    c1 = wl.c1()
    log("c1 fp64 (graph)")
    head, phi64, g64, st64 = time_form(fm, torch, c1.trees, c1.rho, "fp64", K, W,
                                       shape=parse_shape(args.c1_shape) if args.c1_shape else None)
    log(f"  {head['ms_per_step']:.3f} ms/step, {head['cell_interactions_per_s']:.4e} pairs/s")
    shape = head["launch_shape"]
    log(f"c1 fp64 stage timing (eager, HIP events), shape {shape}")
    stages, launches, eager_ms, st_e = stage_times(fm, torch, c1.trees, c1.rho, "fp64", K, W, shape)
    log(f"  stages {stages}")
    p = st_e["pairs"]
    # the timing solves run without the coarse branch, so the roofline
    # kernel's stage is exactly one launch
    if shape["persistent"]:
        kname = f"k_persist<fp64> (every same-level class of every level; {launches['fused']} launch per solve)"
        flops = algorithmic_flops(st_e)
        kms = stages["fused"]
        units = sum(p) + st_e["pairs_top"]
        tkey = f"k_persist_fp64_c1_g{shape['plane_groups']}_bpc{shape['blocks_per_cu']}"
    else:
        kname = (f"k_class<refined-target multipole, fp64> (classes 1+2; {launches['mp_refined']} "
                 "launch per solve, all levels)")
        flops = (p[0] + p[1]) * FLOP_PAIR_REFINED
        kms = stages["mp_refined"]
        units = p[0] + p[1]
        tkey = f"k_class_mp_ref_fp64_c1_g{shape['plane_groups']}"
    achieved = flops / (kms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": traffic_entry(tkey),
                "kernel": kname, "stage_ms": kms, "pairs_per_stage": units,
                "flop_per_pair": {"refined_target": FLOP_PAIR_REFINED, "leaf_multipole": FLOP_PAIR_LEAF_MP,
                                  "leaf_leaf": FLOP_PAIR_MONO}}
    mono_ms = stages["mono"]
    forms = {"c1_fp64": head}
    forms["c1_fp64"]["stages_ms"] = stages
    forms["c1_fp64"]["eager_ms_per_step"] = eager_ms
    if mono_ms > 0 and not shape["persistent"]:
        forms["c1_fp64"]["mono_kernel_tflops"] = p[2] * FLOP_PAIR_MONO / (mono_ms * 1e-3) / 1e12
    forms["c1_fp64"]["residual_force_torque"] = residuals(np, c1.trees, c1.rho, g64)

    log("c1 fp64, the paper's per-sub-grid launch model (128 streams, eager)")
    pm = time_paper_model(fm, torch, c1.trees, c1.rho, "fp64", min(K, 20), min(W, 5), shape["plane_groups"],
                          (phi64, g64))
    pm["default_shape_speedup"] = pm["ms_per_step"] / head["ms_per_step"]
    log(f"  {pm['ms_per_step']:.3f} ms/step, {pm['launches_per_step']} launches")
    forms["c1_fp64_paper_launch_model"] = pm

    log("c1 mixed (graph)")
    mixed, phim, gm, _ = time_form(fm, torch, c1.trees, c1.rho, "mixed", K, W)
    mixed["err_vs_fp64"] = field_err(np, phim, gm, phi64, g64)
    mixed["residual_force_torque"] = residuals(np, c1.trees, c1.rho, gm)
    forms["c1_mixed"] = mixed

    if args.forms == "all":
        log("generating c2 (binary-star AMR field)")
        c2 = wl.c2()
        for prec in ("fp64", "mixed"):
            log(f"c2 {prec}")
            r, p_, g_, _ = time_form(fm, torch, c2.trees, c2.rho, prec, K, W)
            r["residual_force_torque"] = residuals(np, c2.trees, c2.rho, g_)
            if prec == "fp64":
                ref = (p_, g_)
            else:
                r["err_vs_fp64"] = field_err(np, p_, g_, *ref)
            forms["c2_" + prec] = r
            if prec == "fp64":
                log("c2 fp64, the paper's per-sub-grid launch model (128 streams, eager)")
                pm = time_paper_model(fm, torch, c2.trees, c2.rho, "fp64", min(K, 10), min(W, 3),
                                      r["launch_shape"]["plane_groups"], ref)
                pm["default_shape_speedup"] = pm["ms_per_step"] / r["ms_per_step"]
                log(f"  {pm['ms_per_step']:.3f} ms/step, {pm['launches_per_step']} launches")
                forms["c2_fp64_paper_launch_model"] = pm
        log("generating c4 (16 binary-star octrees)")
        c4 = wl.c4()
        for prec in ("fp64", "mixed"):
            log(f"c4 batched {prec}")
            r, p_, g_, _ = time_form(fm, torch, c4.trees, c4.rho, prec, max(3, K // 2), max(1, W // 2))
            r["residual_force_torque"] = residuals(np, c4.trees, c4.rho, g_)
            if prec == "fp64":
                ref = (p_, g_)
            else:
                r["err_vs_fp64"] = field_err(np, p_, g_, *ref)
            forms["c4_batched_" + prec] = r

    cpu = None
    if not args.no_cpu:
        import oracle
        log("cpu baseline: oracle on the full c1 solve")
        t0 = time.perf_counter()
        pr, gr, ost = oracle.solve(c1.trees[0], c1.rho, with_stats=True)
        dt = time.perf_counter() - t0
        pairs = sum(ost["cls"]) + ost["top"]
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cpu = {"value": pairs / dt, "unit": "cell-interactions/s", "cores": threads,
               "kind": "oracle", "sample": "whole c1 solve (upward, same-level, downward), "
               f"{pairs} pairs, {dt:.2f} s wall"}
        forms["c1_fp64"]["err_vs_oracle"] = field_err(np, phi64, g64, pr, gr)
        forms["c1_mixed"]["err_vs_oracle"] = field_err(np, phim, gm, pr, gr)

    out = {
        "metric": METRIC,
        "value": head["cell_interactions_per_s"],
        "unit": "cell-interactions/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "uniform level-3 octree: 585 sub-grids of 8^3 cells, 64^3 leaf "
                               "cells, n=1.5 polytrope r=0.3 + 1e-10 floor",
                   "precision": "fp64", "launch": "hipGraph", "launch_shape": shape,
                   "pairs_per_step": head["pairs_per_step"],
                   "frac_fp64_peak_whole_solve": head["frac_peak"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
