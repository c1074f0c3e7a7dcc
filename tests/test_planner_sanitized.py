"""The host planner under AddressSanitizer and UndefinedBehaviorSanitizer.

planner.cpp is pure host code; it is built here with g++ and the sanitizers
(no GPU code is involved) and driven over the uniform, binary-star, forest
and random AMR trees, both top-level modes, and every plane-group count with
and without the coarse-level split.  Any out-of-bounds access, leak or
undefined operation fails the run; the printed pair counts are checked for
the refined/leaf symmetry of the interaction rule (refined<-leaf pairs equal
leaf<-refined pairs) and against the uniform tree's known level totals.
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from paper_1908_03121_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _dump(path, sets):
    with open(path, "wb") as f:
        f.write(struct.pack("<i", len(sets)))
        for name, trees in sets.items():
            f.write(struct.pack("<16s i", name.encode(), len(trees)))
            for t in trees:
                f.write(struct.pack("<i 3d d", t.n_subgrids, *t.origin, t.L0))
                f.write(np.ascontiguousarray(t.level, dtype=np.int32).tobytes())
                f.write(np.ascontiguousarray(t.coord, dtype=np.int32).tobytes())


def test_planner_clean_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined", "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_1908_03121_amd", "csrc"),
           os.path.join(ROOT, "paper_1908_03121_amd", "csrc", "planner.cpp"),
           os.path.join(ROOT, "tests", "planner_sanitize_driver.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr[-2000:]
    sets = {"c0": wl.c0().trees, "c1": wl.c1().trees, "c2": wl.c2().trees,
            "forest": [wl.forest_tree(3)], "uni0": [wl.uniform_tree(0)]}
    for s in range(3):
        sets[f"amr{s}"] = wl.small_amr(s, max_level=3).trees
    dump = str(tmp_path / "trees.bin")
    _dump(dump, sets)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, dump], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-1000:], r.stderr[-3000:])
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    lines = r.stdout.strip().splitlines()
    assert lines[-1] == "done"
    assert lines[-2] == "c4 tables ok", lines[-2]
    rows = {}
    for ln in lines[:-2]:
        name, top_full, *v = ln.split()
        rows[(name, int(top_full))] = [int(x) for x in v]
    assert len(rows) == 2 * len(sets)
    for (name, top_full), (nleaf, nref, c0, c1, c2, c3, top) in rows.items():
        assert c0 == c3, (name, top_full)  # refined<-leaf mirrors leaf<-refined
    # uniform level-3 tree: the leaf level's ordered same-level pairs, and the
    # top level's (the 512 x 511 ordered pairs of level 0 less those closer
    # than 3 cell widths, which its children take over)
    assert rows[("c1", 0)][4] == 176804352 and rows[("c1", 1)][6] == 230616
