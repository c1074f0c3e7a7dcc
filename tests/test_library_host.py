"""CPU checks of the product library: it loads, exports every symbol the header
declares, validates trees, and its host planner counts the same pairs that the
oracle evaluates.  No compute call touches a GPU here."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_1908_03121_amd as fm
from paper_1908_03121_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "fmmg.h")).read()
    return sorted(set(re.findall(r"\b(fmmg_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = fm.lib()
    names = header_symbols()
    assert set(names) == set(fm.EXPORTED)
    for n in names:
        assert hasattr(L, n), n
    assert fm.fmmg_version() == 6


def test_default_options():
    o = fm.fmmg_default_options()
    assert o.precision == fm.FMMG_FP64 and o.top_mode == fm.FMMG_TOP_FULL
    assert o.G == 1.0 and o.angular_correction == 1
    assert o.overlap == 1 and o.launch_streams == 0 and o.use_graph == -1 and o.persistent == 0
    assert o.xcd_queues == 1
    assert o.plane_pairs == -1


@pytest.mark.parametrize("bad", [
    {"launch_streams": 129}, {"launch_streams": -1}, {"launch_streams": 4, "timing": 1},
    {"launch_streams": 4, "autotune": 1}, {"overlap": 3}, {"plane_groups": 6}, {"xcd_queues": 2}, {"plane_pairs": 2},
    {"timing": 1, "use_graph": 1}, {"timing": 1, "autotune": 1}, {"blocks_per_cu": -1},
    {"precision": 3},
])
def test_bad_options_are_rejected_before_any_device_call(bad):
    # option checks come first, so they answer the same with or without a GPU
    o = fm.fmmg_default_options()
    for k, v in bad.items():
        setattr(o, k, v)
    with pytest.raises(fm.FmmgError) as e:
        fm.fmmg_plan_create([wl.uniform_tree(1)], o, stream=0)
    assert e.value.status == fm.FMMG_EINVAL


def test_library_does_not_link_the_oracle():
    with open(fm.LIB_PATH, "rb") as f:
        blob = f.read()
    assert b"oracle_" not in blob


@pytest.mark.parametrize("case", ["c0s", "c0f", "c1l2", "amr1", "amr2", "amr3", "c2"])
def test_host_pair_counts_match_oracle(case):
    if case.startswith("c0"):
        W = wl.c0()
        top = case == "c0f"
    elif case == "c1l2":
        W, top = wl.c1(max_level=2), True
    elif case == "c2":
        W, top = wl.c2(), True
    else:
        W, top = wl.small_amr(int(case[-1])), True
    t = W.trees[0]
    st = fm.fmmg_count_pairs([t], fm.FMMG_TOP_FULL if top else fm.FMMG_TOP_STENCIL_ONLY)
    if case == "c2":
        # too large for a full oracle pass here; check the exact-once identity instead
        assert st["n_leaves"] == 3816 and st["n_refined"] == 545
        assert st["pairs"][0] == st["pairs"][3]
        return
    _, _, os_ = oracle.solve(t, W.rho, top_all_pairs=top, with_stats=True)
    assert st["pairs"] == os_["cls"]
    assert st["pairs_top"] == os_["top"]
    assert st["paper_flops"] == 12 * os_["cls"][2] + 455 * (os_["cls"][0] + os_["cls"][1] + os_["cls"][3] + os_["top"])


def test_c1_counts_and_batched_counts_add_up():
    t = wl.c1().trees[0]
    st = fm.fmmg_count_pairs([t])
    assert st["pairs_top"] == 230616
    assert st["pairs"] == [0, 1705080 + 17246904, 176804352, 0]
    st2 = fm.fmmg_count_pairs([t, t])
    assert st2["pairs"] == [2 * v for v in st["pairs"]] and st2["pairs_top"] == 2 * 230616
    assert st2["n_leaves"] == 1024 and st2["n_trees"] == 2


def test_malformed_trees_are_rejected():
    t = wl.uniform_tree(1)
    seven = wl.TreeDesc(t.level[:-1].copy(), t.coord[:-1].copy(), t.origin, t.L0)
    with pytest.raises(fm.FmmgError) as e:
        fm.fmmg_count_pairs([seven])
    assert e.value.status == fm.FMMG_ETREE and "7 of 8 children" in str(e.value)
    orphan = wl.TreeDesc(np.array([1], np.int32), np.array([[0, 0, 0]], np.int32), t.origin, t.L0)
    with pytest.raises(fm.FmmgError) as e:
        fm.fmmg_count_pairs([orphan])
    assert e.value.status == fm.FMMG_ETREE and "parent" in str(e.value)
    dup = wl.TreeDesc(np.array([0, 0], np.int32), np.array([[0, 0, 0], [0, 0, 0]], np.int32), t.origin, t.L0)
    with pytest.raises(fm.FmmgError) as e:
        fm.fmmg_count_pairs([dup])
    assert e.value.status == fm.FMMG_ETREE and "duplicate" in str(e.value)
    neg = wl.TreeDesc(np.array([0], np.int32), np.array([[-1, 0, 0]], np.int32), t.origin, t.L0)
    with pytest.raises(fm.FmmgError) as e:
        fm.fmmg_count_pairs([neg])
    assert e.value.status == fm.FMMG_ETREE
    badL = wl.TreeDesc(t.level, t.coord, t.origin, 0.0)
    with pytest.raises(fm.FmmgError) as e:
        fm.fmmg_count_pairs([badL])
    assert e.value.status == fm.FMMG_EINVAL
    with pytest.raises(fm.FmmgError) as e:
        fm.fmmg_count_pairs([t], top_mode=7)
    assert e.value.status == fm.FMMG_EINVAL


def _plane_visits(usable, sweep, near, far_by_w, near_by_w):
    """Stencil entries the plane items of one target visit in a sweep frame:
    a source plane is visited iff one of the 9 neighbour sub-grids at its
    offset along the sweep axis (z: sweep 0, y: sweep 1, x: sweep 2) is
    usable."""
    axis = (2, 1, 0)[sweep]
    n = 0
    for t in range(8):
        s = 1 - 2 * (t & 1)
        for i in range(10):
            w = t + s * (i - 4)
            side = -1 if w < 0 else (1 if w >= 8 else 0)
            if np.take(usable, side + 1, axis=axis).any():
                n += far_by_w[i] + (near_by_w[i] if near else 0)
    return n


@pytest.mark.parametrize("name", ["c2", "amr3"])
def test_planner_sweep_choice(name):
    """The planner runs a refined target's plane items along the axis (z, y
    or x) whose frame visits the fewest stencil entries, z before y before x
    on a tie; recounted here from the interaction rule and the tree alone."""
    import itertools
    W = wl.c2() if name == "c2" else wl.small_amr(3, max_level=3, p_refine=0.3)
    t = W.trees[0]
    far = np.zeros(10, int)
    near = np.zeros(10, int)
    for d in itertools.product(range(-5, 6), repeat=3):
        if oracle.pair_rule(0, [0, 0, 0], list(d), 0, 1):
            (far if oracle.pair_rule(0, [0, 0, 0], list(d), 0, 0) else near)[d[2] + 4] += 1
    assert far.sum() == 651 and near.sum() == 92
    ref = t.refined_mask()
    key = {(int(l), *map(int, c)): i for i, (l, c) in enumerate(zip(t.level, t.coord))}
    n_y = n_x = 0
    for s in range(t.n_subgrids):
        lv, c = int(t.level[s]), t.coord[s]
        if lv == 0:
            continue                      # the top level has its own all-pairs kernel
        nb = np.full((3, 3, 3), -1)
        for o in itertools.product((-1, 0, 1), repeat=3):
            j = key.get((lv, c[0] + o[0], c[1] + o[1], c[2] + o[2]))
            if j is not None:
                nb[o[0] + 1, o[1] + 1, o[2] + 1] = 1 if ref[j] else 0
        others = nb.copy()
        others[1, 1, 1] = -1
        if not ref[s]:
            continue                      # leaf targets are grouped by parent cell, not by plane
        usable, near_on = nb >= 0, bool((others == 0).any())
        v = [_plane_visits(usable, sw, near_on, far, near) for sw in (0, 1, 2)]
        best = min(range(3), key=lambda k: (v[k], k))
        n_y += best == 1
        n_x += best == 2
    st = fm.fmmg_count_pairs([t])
    print(f"  {name}: {n_y} targets along y, {n_x} along x", flush=True)
    assert st["sweep_y_targets"] == n_y and st["sweep_x_targets"] == n_x and n_y > 0 and n_x > 0


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "exactly one GPU" in r.stderr and r.stdout == ""


def test_bench_c1_shape_spec_parses_to_plan_arguments():
    """--c1-shape names a launch shape as kind, plane groups, blocks per CU and
    overlap; malformed names are rejected."""
    import importlib.util
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    assert bench.parse_shape("per_class_g5_b3_o1") == dict(persistent=False, plane_groups=5,
                                                          blocks_per_cu=3, overlap=1)
    assert bench.parse_shape("persistent_g2_b0_o0") == dict(persistent=True, plane_groups=2,
                                                           blocks_per_cu=0, overlap=0)
    for bad in ("per_class_5_b3_o1", "fused_g1_b1_o0", "per_class_g5_o1_b3"):
        with pytest.raises((AssertionError, ValueError)):
            bench.parse_shape(bad)


def test_noalloc_density_check_refuses_bad_sizes_before_any_device_call():
    """The allocation-free density check validates its size and pointers on the
    host; these calls return FMMG_EINVAL without touching a device."""
    L = fm.lib()
    dummy = ctypes.c_void_p(16)
    for n, rho, out in ((-1, dummy, dummy), (fm.FMMG_NOALLOC_MAX_DENSITIES + 1, dummy, dummy),
                        (8, None, dummy), (8, dummy, None)):
        assert L.fmmg_check_density_noalloc(rho, n, out, None) == fm.FMMG_EINVAL
    assert "maximum" in fm.fmmg_last_error() or "null" in fm.fmmg_last_error()
