#!/usr/bin/env python3
"""Benchmark of the octree FMM gravity solve on one MI355X.

A step is one whole solve (upward pass, same-level interactions of all
classes, downward pass) of one batch of synthetic input already resident in
HBM.  The headline workload is the largest single-GPU configuration: a batch
of 16 binary-star AMR octrees (30,732 leaf sub-grids, 12.0 G cell pairs) in
one plan, in FP64.  The JSON line also carries the mixed-precision forms, the
uniform level-3 octree and the single binary-star tree, the dominant kernel's
roofline (timed with HIP events on the solve's stream) and the CPU oracle
timed on this host's cores on a bounded sample of the headline batch.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms all|c4]
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
PEAK_FP32_PACKED = 157.3e12  # MI355X FP32 vector with packed FP32 (not used by these kernels)
PEAK_HBM = 8.0e12        # bytes/s

# Arithmetic of one ordered pair in the kernels' formulation (FMA = 2 flop),
# counted in the compiled pair loops:
FLOP_PAIR_REFINED = 196  # refined target: L0..L3 (order 3) + correction (77 FMA, 33 MUL, 8 ADD, 1 RSQ)
FLOP_PAIR_LEAF_MP = 124  # leaf target, multipole source: L0, L1 + correction (45 FMA, 25 MUL, 8 ADD, 1 RSQ)
# leaf <- leaf monopole with lattice kernel tables: per lane and sub-grid
# 8 targets x 744 offsets; phi, the column sum and g_z cost 3 FMA per offset,
# 2 ADD + 3 FMA per +-dz pair of offsets, 2 FMA at dz = 0, plus 2 FMA per
# target and column for g_x, g_y: (8 x 3176 + 100 x 32) / 5952 = 4.8 flop
FLOP_PAIR_MONO = 4.8


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
    # non-packed FP32 (the mixed forms' pair terms) has the same vector peak as
    # FP64 on this chip: 256 CUs x 2.4 GHz x 64 FMA lanes x 2
    out["frac_peak"] = algorithmic_flops(st) / dt / PEAK_FP64
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
                 xcd_queues=bool(shape.get("xcd_queues", 1)),
                 plane_pairs=bool(shape["plane_pairs"]) if "plane_pairs" in shape else None,
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_c4(np, c4, gpu_forms, min_pairs=1.0e9):
    """The CPU oracle (OpenMP over target cells, all of this host's threads)
    on a bounded sample of the headline batch: whole solves of its trees in
    order until min_pairs cell pairs are covered; then one thread on its first
    tree.  The sampled trees also give the GPU forms' error against the
    oracle."""
    import oracle
    import paper_1908_03121_amd as fm
    threads = oracle.set_threads(0)
    off, pairs, wall, used, err = 0, 0, 0.0, [], {}
    for k, t in enumerate(c4.trees):
        n = t.n_leaves
        rho_k = c4.rho[off:off + n]
        t0 = time.perf_counter()
        pr, gr = oracle.solve(t, rho_k)
        wall += time.perf_counter() - t0
        pairs += fm.fmmg_count_pairs([t])["total_pairs"]
        used.append(k)
        for name, (phi, g) in gpu_forms.items():
            e = field_err(np, phi[off:off + n], g[off:off + n], pr, gr)
            worst = err.setdefault(name, {key: 0.0 for key in e})
            for key, v in e.items():
                worst[key] = max(worst[key], v)
        off += n
        if pairs >= min_pairs:
            break
    log(f"  oracle, {threads} threads: trees {used}, {pairs} pairs, {wall:.2f} s")
    t0_tree = c4.trees[0]
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.solve(t0_tree, c4.rho[:t0_tree.n_leaves])
    wall1 = time.perf_counter() - t0
    oracle.set_threads(0)
    pairs1 = fm.fmmg_count_pairs([t0_tree])["total_pairs"]
    log(f"  oracle, 1 thread: tree 0, {pairs1} pairs, {wall1:.2f} s")
    cpu = {"value": pairs / wall, "unit": "cell-interactions/s", "cores": threads, "kind": "oracle",
           "sample": f"whole FP64 solves (upward, same-level, downward) of trees {used} of the 16-tree "
                     f"binary-star batch, {pairs} cell pairs, {wall:.2f} s wall on {threads} OpenMP threads",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "one_thread": {"value": pairs1 / wall1, "unit": "cell-interactions/s", "cores": 1,
                          "sample": f"whole FP64 solve of tree 0 ({t0_tree.n_leaves} leaf sub-grids), "
                                    f"{pairs1} cell pairs, {wall1:.2f} s wall"}}
    return cpu, err, used


def roofline_of(shape, stages, launches, st_e, key_prefix):
    """The dominant kernel of eager timing solves in `shape` (without the
    coarse branch, so it is one launch per solve): the persistent launch of
    every class, or the refined-target class launch."""
    p = st_e["pairs"]
    if shape["persistent"]:
        kname = (f"k_persist<fp64> (every same-level class of every level and tree; "
                 f"{launches['fused']} launch per solve)")
        flops = algorithmic_flops(st_e)
        kms = stages["fused"]
        units = sum(p) + st_e["pairs_top"]
        tkey = f"k_persist_fp64_{key_prefix}_g{shape['plane_groups']}_bpc{shape['blocks_per_cu']}"
    else:
        kname = (f"k_class<refined-target multipole, fp64> (classes 1+2; {launches['mp_refined']} "
                 "launch per solve, all levels)")
        flops = (p[0] + p[1]) * FLOP_PAIR_REFINED
        kms = stages["mp_refined"]
        units = p[0] + p[1]
        tkey = f"k_class_mp_ref_fp64_{key_prefix}_g{shape['plane_groups']}"
    achieved = flops / (kms * 1e-3)
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": traffic_entry(tkey),
            "kernel": kname, "kernel_ms": kms, "algorithmic_gflop_per_launch": flops / 1e9,
            "pairs_per_launch": units,
            "flop_per_pair": {"refined_target": FLOP_PAIR_REFINED, "leaf_multipole": FLOP_PAIR_LEAF_MP,
                              "leaf_leaf": FLOP_PAIR_MONO}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--forms", default="all", choices=["all", "c4", "c2-stages", "c4-stages"],
                    help="c4: the headline batch only; c2-stages / c4-stages: only eager, "
                         "stage-timed FP64 solves in the per-class shape (one launch per class), for "
                         "a kernel trace of the classes' shares")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--profile", default=None, choices=["c1", "c2", "c4"],
                    help="short run for hardware counters: 3 eager FP64 solves of this workload in "
                         "the launch shape --shape (no overlap: one launch per class, or one "
                         "persistent launch, as in the timing solves), then a 256 MiB "
                         "device-to-device copy whose byte counters calibrate the solve kernels'")
    ap.add_argument("--bpc", type=int, default=0,
                    help="--profile: blocks per CU of the persistent launch (0 = occupancy limit)")
    ap.add_argument("--shape", default="per_class_g2",
                    choices=[f"{k}_g{g}" for k in ("per_class", "persistent") for g in (1, 2, 3, 5)])
    ap.add_argument("--head-shape", default=None,
                    help="launch shape of the headline (batch, FP64) instead of the tuner's choice, "
                         "e.g. persistent_g1_b3_o0 or per_class_g2_b3_o1 (a profiled run uses the "
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
    gen = {"c1": wl.c1, "c2": wl.c2, "c4": wl.c4}

    if args.profile:
        work = gen[args.profile]()
        dev = torch.device("cuda:0")
        rho = torch.tensor(work.rho, dtype=torch.float64, device=dev)
        pers, groups = args.shape.split("_g")
        with fm.Plan(work.trees, persistent=pers == "persistent", plane_groups=int(groups), overlap=0,
                     blocks_per_cu=args.bpc, use_graph=False) as plan:
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
        print(json.dumps({"profile": args.profile + "_fp64", "shape": args.shape, "bpc": args.bpc, "solves": 3,
                          "pairs": st["pairs"], "pairs_top": st["pairs_top"],
                          "copy_bytes_each_way": n * 8}), flush=True)
        return

    if args.forms in ("c2-stages", "c4-stages"):
        name = args.forms.split("-")[0]
        log(f"generating {name}")
        work = gen[name]()
        shape = dict(persistent=0, plane_groups=1, blocks_per_cu=0)
        stages, launches, wall, st = stage_times(fm, torch, work.trees, work.rho, "fp64", min(K, 10),
                                                 min(W, 3), shape)
        print(json.dumps({"profile": name + "_fp64_stages", "shape": "per_class_g1", "stages_ms": stages,
                          "launches": launches, "eager_ms_per_step": wall, "pairs": st["pairs"],
                          "pairs_top": st["pairs_top"]}), flush=True)
        return

    forms = {}
    log("generating c4 (16 binary-star octrees)")
    c4 = wl.c4()
    log("c4 batched fp64 (graph)")
    head, phi64, g64, st64 = time_form(fm, torch, c4.trees, c4.rho, "fp64", K, W,
                                       shape=parse_shape(args.head_shape) if args.head_shape else None)
    log(f"  {head['ms_per_step']:.3f} ms/step, {head['cell_interactions_per_s']:.4e} pairs/s")
    shape = head["launch_shape"]
    log(f"c4 fp64 stage timing (eager, HIP events), shape {shape}")
    stages, launches, eager_ms, st_e = stage_times(fm, torch, c4.trees, c4.rho, "fp64", min(K, 20), min(W, 3),
                                                   shape)
    log(f"  stages {stages}")
    roofline = roofline_of(shape, stages, launches, st_e, "c4")
    head["stages_ms"] = stages
    head["eager_ms_per_step"] = eager_ms
    head["residual_force_torque"] = residuals(np, c4.trees, c4.rho, g64)
    forms["c4_batched_fp64"] = head
    c4_sol = {"c4_batched_fp64": (phi64, g64)}

    if args.forms == "all":
        for prec in ("mixed", "mixed_f32"):
            log(f"c4 batched {prec}")
            r, p_, g_, _ = time_form(fm, torch, c4.trees, c4.rho, prec, K, W)
            r["residual_force_torque"] = residuals(np, c4.trees, c4.rho, g_)
            r["err_vs_fp64"] = field_err(np, p_, g_, phi64, g64)
            forms["c4_batched_" + prec] = r
            c4_sol["c4_batched_" + prec] = (p_, g_)
            del p_, g_

        log("generating c1 (uniform level-3 octree, 64^3 leaf cells)")
        c1 = wl.c1()
        c1_sol = {}
        for prec in ("fp64", "mixed", "mixed_f32"):
            log(f"c1 {prec} (graph)")
            r, p_, g_, _ = time_form(fm, torch, c1.trees, c1.rho, prec, max(K, 100), W)
            r["residual_force_torque"] = residuals(np, c1.trees, c1.rho, g_)
            forms["c1_" + prec] = r
            c1_sol[prec] = (p_, g_)
        log("c1 fp64, the paper's per-sub-grid launch model (128 streams, eager)")
        pm = time_paper_model(fm, torch, c1.trees, c1.rho, "fp64", 20, 5,
                              forms["c1_fp64"]["launch_shape"]["plane_groups"], c1_sol["fp64"])
        pm["default_shape_speedup"] = pm["ms_per_step"] / forms["c1_fp64"]["ms_per_step"]
        forms["c1_fp64_paper_launch_model"] = pm
        if not args.no_cpu:
            import oracle
            pr, gr = oracle.solve(c1.trees[0], c1.rho)
            for prec, (p_, g_) in c1_sol.items():
                forms["c1_" + prec]["err_vs_oracle"] = field_err(np, p_, g_, pr, gr)

        log("generating c2 (binary-star AMR field)")
        c2 = wl.c2()
        for prec in ("fp64", "mixed", "mixed_f32"):
            log(f"c2 {prec}")
            r, p_, g_, _ = time_form(fm, torch, c2.trees, c2.rho, prec, max(K, 50), W)
            r["residual_force_torque"] = residuals(np, c2.trees, c2.rho, g_)
            if prec == "fp64":
                ref = (p_, g_)
            else:
                r["err_vs_fp64"] = field_err(np, p_, g_, *ref)
            forms["c2_" + prec] = r
            if prec == "fp64":
                log("c2 fp64, the paper's per-sub-grid launch model (128 streams, eager)")
                pm = time_paper_model(fm, torch, c2.trees, c2.rho, "fp64", 10, 3,
                                      r["launch_shape"]["plane_groups"], ref)
                pm["default_shape_speedup"] = pm["ms_per_step"] / r["ms_per_step"]
                forms["c2_fp64_paper_launch_model"] = pm

    cpu = None
    if not args.no_cpu:
        log("cpu baseline: the oracle on a sample of the c4 batch")
        cpu, err, used = cpu_baseline_c4(np, c4, c4_sol)
        for name, e in err.items():
            forms[name]["err_vs_oracle"] = e
            forms[name]["err_vs_oracle_trees"] = used

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
        "config": {"workload": "batch of 16 binary-star AMR octrees in one plan (30,732 leaf and "
                               "4,388 refined sub-grids of 8^3 cells; mass ratios 0.05-0.5, "
                               "separations 0.3-0.6, deepest levels 4-5; seeds 4000-4015), "
                               "12,038,612,656 cell pairs per solve",
                   "precision": "fp64", "launch": "hipGraph", "launch_shape": shape,
                   "pairs_per_step": head["pairs_per_step"],
                   "frac_fp64_peak_whole_solve": head["frac_peak"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        # context only (other hardware, another workload): the paper's node-level
        # FMM figures (Sec. 6.1 table), GFLOP/s by its nominal convention of 12
        # flop per monopole and 455 per multipole interaction, FP64
        "paper_context": {
            "workload": "V1309 merger model at level 14 (10,928 sub-grids), several time steps",
            "piz_daint_p100_gflops": 973, "piz_daint_p100_frac_fp64_peak": 0.21,
            "best_node_2x_v100_gflops": 5188, "best_node_frac_fp64_peak": 0.37,
            "this_run_paper_convention_gflops": head["paper_convention_gflops"],
        },
        "forms": forms,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
