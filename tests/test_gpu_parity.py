"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

FP64 bar: per field (phi and each g component), max |gpu - oracle| / max |oracle|
<= 1e-12.  Mixed forms: the stated bounds below (FP32 pair terms), against the
same FP64 oracle, with their force and torque residuals.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1908_03121_amd as fm
from paper_1908_03121_amd import workloads as wl

pytestmark = pytest.mark.gpu
TOL64 = 1e-12
DEV = torch.device("cuda:0")

# Stated bounds of the FP32 forms (per-field error against the FP64 oracle,
# max norm: phi, then every g component; relative total force and torque),
# per workload.  "mixed": FP32 Taylor-coefficient pair terms, the correction
# in FP64; "mixed_f32": the correction in FP32 as well.  FP64: 1e-12 per
# field, force and torque at round-off.
FORM_BOUNDS = {
    # workload: {precision: (phi, g, force, torque)}; mixed-form bounds are
    # about 3x the largest values measured on MI355X (all 16 batch trees for
    # c4; the 3-, 4- and 5-level uniform trees for c1, whose centred sphere
    # makes the torque's denominator sum |x x m g| small; the random AMR trees
    # and the y-sweep forest for amr)
    "c1": {"fp64": (TOL64, TOL64, 1e-15, 1e-13), "mixed": (1e-7, 1.5e-7, 1e-9, 3.5e-7),
           "mixed_f32": (1.5e-7, 2.6e-7, 2e-8, 6.5e-6)},
    "c2": {"fp64": (TOL64, TOL64, 1.5e-13, 1e-14), "mixed": (1.1e-7, 2e-7, 5e-9, 3.5e-9),
           "mixed_f32": (1.8e-7, 3.2e-7, 1.5e-8, 1.2e-8)},
    "c4": {"fp64": (TOL64, TOL64, 3e-13, 1.5e-14), "mixed": (1.4e-7, 2.2e-7, 1e-8, 7e-9),
           "mixed_f32": (1.7e-7, 3.3e-7, 1.8e-8, 7e-8)},
    "amr": {"fp64": (TOL64, TOL64, 1e-13, 1e-13), "mixed": (2.5e-7, 3e-7, 7e-9, 4e-8),
            "mixed_f32": (2.5e-7, 1e-6, 6e-9, 4e-8)},
}


def check_form(workload, precision, errs, force, torque):
    bp, bg, bf, bt = FORM_BOUNDS[workload][precision]
    assert errs[0] < bp and max(errs[1:]) < bg, (workload, precision, errs)
    assert force < bf and torque < bt, (workload, precision, force, torque)


def field_errors(phi, g, pr, gr):
    e = [float(np.abs(phi - pr).max() / np.abs(pr).max())]
    for a in range(3):
        e.append(float(np.abs(g[..., a, :] - gr[..., a, :]).max() / np.abs(gr[..., a, :]).max()))
    return e


def run(trees, rho, **kw):
    print(f"  gpu solve: {len(trees)} tree(s), {rho.shape[0]} leaves, {kw}", flush=True)
    r = torch.tensor(rho, dtype=torch.float64, device=DEV)
    with fm.Plan(trees, **kw) as p:
        phi, g = p.solve(r)
        torch.cuda.synchronize()
        st = p.stats()
        return phi.cpu().numpy(), g.cpu().numpy(), st


def residuals(tree, rho, g, centre=(0.5, 0.5, 0.5)):
    x = tree.leaf_cell_centres().reshape(-1, 3) - np.asarray(centre)
    h = tree.leaf_cell_size()
    m = (rho * (h ** 3)[:, None, None, None]).reshape(-1)
    F = m[:, None] * g.transpose(0, 2, 1).reshape(-1, 3)
    tau = np.cross(x, F)
    return (float(np.abs(F.sum(0)).max() / np.abs(F).sum(0).max()),
            float(np.abs(tau.sum(0)).max() / np.abs(tau).sum(0).max()))


# ---------------------------------------------------------------------------
# FP64 parity
# ---------------------------------------------------------------------------
def test_c0_stencil_neighbourhood_fp64():
    """27 level-0 leaves (24^3 cells) with the parent-near stencil: the
    monopole kernel alone, central sub-grid = 512 x 743 pairs."""
    W = wl.c0()
    t = W.trees[0]
    phi, g, st = run([t], W.rho, top_mode="stencil")
    pr, gr = oracle.solve(t, W.rho, top_all_pairs=False)
    assert max(field_errors(phi, g, pr, gr)) < TOL64
    assert st["pairs"][2] == 7862272
    f, tq = residuals(t, W.rho, g)
    assert f < 1e-13 and tq < 1e-13


def test_c0_forest_all_pairs_fp64():
    W = wl.c0(1)
    t = W.trees[0]
    phi, g, st = run([t], W.rho, top_mode="full")
    pr, gr = oracle.solve(t, W.rho, top_all_pairs=True)
    assert max(field_errors(phi, g, pr, gr)) < TOL64
    assert st["pairs_top"] == 13824 * 13823


SHAPES = {"per_class_g1": dict(plane_groups=1), "per_class_g2": dict(plane_groups=2),
          "persistent_g2": dict(persistent=True, plane_groups=2),
          "persistent_g1": dict(persistent=True, plane_groups=1),
          "per_class_g3": dict(plane_groups=3),
          "persistent_g5": dict(persistent=True, plane_groups=5),
          "persistent_g1_bpc1": dict(persistent=True, plane_groups=1, blocks_per_cu=1),
          "per_class_g2_pairs": dict(plane_groups=2, plane_pairs=True),
          "persistent_g1_pairs": dict(persistent=True, plane_groups=1, plane_pairs=True),
          "persistent_g3_single": dict(persistent=True, plane_groups=3, plane_pairs=False)}


@pytest.mark.parametrize("shape", list(SHAPES))
@pytest.mark.parametrize("seed", [1, 2, 3, 5])
def test_random_amr_fp64(seed, shape):
    """All four classes, coarse-fine boundaries, absent neighbours."""
    W = wl.small_amr(seed)
    t = W.trees[0]
    phi, g, st = run([t], W.rho, **SHAPES[shape])
    pr, gr, ost = oracle.solve(t, W.rho, with_stats=True)
    errs = field_errors(phi, g, pr, gr)
    print("  errors", errs, flush=True)
    assert max(errs) < TOL64
    assert st["pairs"] == ost["cls"] and st["pairs_top"] == ost["top"]
    f, tq = residuals(t, W.rho, g)
    assert f < 1e-13 and tq < 1e-13


@pytest.mark.parametrize("shape", ["per_class_g1", "persistent_g1"])
def test_batch_of_random_amr_trees_fp64(shape):
    """Eight random AMR trees of two and three levels below the root in one
    plan (captured and replayed by default): every cell of every tree
    against the oracle, and every tree's force and torque at round-off."""
    ws = [wl.small_amr(20 + i, max_level=2 + i % 2, p_refine=0.2 + 0.05 * i) for i in range(8)]
    trees = [w.trees[0] for w in ws]
    rho = np.concatenate([w.rho for w in ws])
    phi, g, st = run(trees, rho, **SHAPES[shape])
    off = 0
    for w in ws:
        n = w.n_leaves
        pr, gr = oracle.solve(w.trees[0], w.rho)
        errs = field_errors(phi[off:off + n], g[off:off + n], pr, gr)
        f, tq = residuals(w.trees[0], w.rho, g[off:off + n])
        print(f"  {w.name}: {n} leaves, errors {errs} force {f:.2e} torque {tq:.2e}", flush=True)
        assert max(errs) < TOL64 and f < 1e-13 and tq < 1e-13
        off += n
    assert off == rho.shape[0] and st["n_trees"] == 8


@pytest.mark.parametrize("shape", ["per_class_g2", "persistent_g2"])
def test_random_amr_deeper_fp64(shape):
    W = wl.small_amr(11, max_level=3, p_refine=0.3)
    t = W.trees[0]
    phi, g, _ = run([t], W.rho, **SHAPES[shape])
    pr, gr = oracle.solve(t, W.rho)
    assert max(field_errors(phi, g, pr, gr)) < TOL64


@pytest.mark.parametrize("shape", ["per_class_g1", "persistent_g2"])
def test_stencil_mode_refined_top_level(shape):
    """A refined level-0 forest under the stencil-only top rule (its totals
    are its own terms) with random densities."""
    subs = [(0, x, y, z) for x in range(2) for y in range(2) for z in range(2)]
    subs += [(1, 2 * 0 + a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)]
    t = wl._desc_from_list(subs, (0, 0, 0), 1.0)
    rho = np.random.default_rng(4).lognormal(0, 1, (t.n_leaves, 8, 8, 8))
    phi, g, st = run([t], rho, top_mode="stencil", **SHAPES[shape])
    pr, gr, ost = oracle.solve(t, rho, top_all_pairs=False, with_stats=True)
    assert max(field_errors(phi, g, pr, gr)) < TOL64
    assert st["pairs"] == ost["cls"]


def deep_chain(levels=19, seed=6):
    """One refined sub-grid per level down to the deepest level the interface
    allows (19): 8 children per level, one of them refined further, the path
    wandering between octants; lognormal densities."""
    rng = np.random.default_rng(seed)
    subs, c = [(0, 0, 0, 0)], (0, 0, 0)
    for lv in range(1, levels + 1):
        kids = [(lv, 2 * c[0] + a, 2 * c[1] + b, 2 * c[2] + d) for a in (0, 1) for b in (0, 1) for d in (0, 1)]
        subs += kids
        c = kids[int(rng.integers(0, 8))][1:]
    t = wl._desc_from_list(subs, (0.0, 0.0, 0.0), 1.0)
    return t, rng.lognormal(0.0, 1.0, (t.n_leaves, 8, 8, 8))


@pytest.mark.parametrize("shape", ["per_class_g2", "persistent_g1"])
def test_deep_chain_to_level_19(shape):
    """Twenty levels (cells from 1/8 down to 2^-22 of the domain), so every
    pass runs its longest level chain and the split, top and downward logic
    see many coarse levels."""
    t, rho = deep_chain()
    assert int(t.level.max()) == 19
    for ov in (0, 1):
        phi, g, st = run([t], rho, overlap=ov, **SHAPES[shape])
        pr, gr, ost = oracle.solve(t, rho, with_stats=True)
        errs = field_errors(phi, g, pr, gr)
        print(f"  overlap {ov}: errors {errs}", flush=True)
        assert max(errs) < TOL64
        assert st["pairs"] == ost["cls"] and st["pairs_top"] == ost["top"]


def test_correction_off_matches_uncorrected_oracle():
    W = wl.small_amr(2)
    t = W.trees[0]
    phi, g, _ = run([t], W.rho, angular_correction=False)
    pr, gr = oracle.solve(t, W.rho, correction=False)
    assert max(field_errors(phi, g, pr, gr)) < TOL64
    f, tq = residuals(t, W.rho, g)
    assert tq > 1e-8     # the correction is what removes the torque


def test_gravitational_constant_scales():
    W = wl.small_amr(3)
    t = W.trees[0]
    phi, g, _ = run([t], W.rho, G=6.674e-8)
    pr, gr = oracle.solve(t, W.rho, G=6.674e-8)
    assert max(field_errors(phi, g, pr, gr)) < TOL64


def test_single_leaf_and_single_refined_root():
    t = wl.forest_tree(1, origin=(0, 0, 0))
    rho = np.random.default_rng(0).lognormal(0, 1, (1, 8, 8, 8))
    for mode, top in (("full", True), ("stencil", False)):
        phi, g, _ = run([t], rho, top_mode=mode)
        pr, gr = oracle.solve(t, rho, top_all_pairs=top)
        assert max(field_errors(phi, g, pr, gr)) < TOL64
    t2 = wl.uniform_tree(1)
    rho2 = np.random.default_rng(1).lognormal(0, 1, (8, 8, 8, 8))
    phi, g, _ = run([t2], rho2)
    pr, gr = oracle.solve(t2, rho2)
    assert max(field_errors(phi, g, pr, gr)) < TOL64


@pytest.mark.parametrize("shape", ["per_class_g2", "persistent_g2", "per_class_g3", "persistent_g5"])
def test_c1_full_size_fp64_graph(shape):
    """Uniform level-3 polytrope (64^3 leaf cells), in the launch
    configurations the benchmark may time (captured graph)."""
    W = wl.c1()
    t = W.trees[0]
    phi, g, st = run([t], W.rho, use_graph=True, **SHAPES[shape])
    pr, gr = oracle.solve(t, W.rho)
    errs = field_errors(phi, g, pr, gr)
    print("  c1 errors", errs, flush=True)
    assert max(errs) < TOL64
    assert st["pairs"] == [0, 1705080 + 17246904, 176804352, 0] and st["pairs_top"] == 230616


_CACHE = {}


def cached(key, make):
    """Workloads, oracle solves and GPU solves shared by several tests."""
    if key not in _CACHE:
        _CACHE[key] = make()
    return _CACHE[key]


def c2_workload():
    return cached("c2", wl.c2)


def c2_oracle():
    def make():
        W = c2_workload()
        print("  oracle: binary-star tree (3,816 leaves)", flush=True)
        return oracle.solve(W.trees[0], W.rho)
    return cached("c2_oracle", make)


@pytest.mark.parametrize("shape", ["per_class_g2", "persistent_g2", "persistent_g1"])
def test_c2_full_size_fp64(shape):
    """Binary-star AMR field (3,816 leaves, all four classes, both sweep
    frames): every leaf cell against the oracle."""
    W = c2_workload()
    t = W.trees[0]
    phi, g, st = run([t], W.rho, use_graph=True, **SHAPES[shape])
    pr, gr = c2_oracle()
    errs = field_errors(phi, g, pr, gr)
    print(f"  c2 errors {errs}", flush=True)
    assert max(errs) < TOL64
    assert st["pairs"][0] == st["pairs"][3] > 0
    f, tq = residuals(t, W.rho, g)
    print(f"  c2 residual force {f:.3e} torque {tq:.3e}", flush=True)
    check_form("c2", "fp64", errs, f, tq)


@pytest.mark.parametrize("shape", ["per_class_g2", "persistent_g2"])
def test_batched_trees_equal_each_tree_alone(shape):
    Ws = [wl.small_amr(s) for s in (1, 2, 3)] + [wl.c1(max_level=2)]
    trees = [W.trees[0] for W in Ws]
    rho = np.concatenate([W.rho for W in Ws])
    phi, g, st = run(trees, rho, use_graph=True, **SHAPES[shape])
    off = 0
    for W in Ws:
        n = W.n_leaves
        pr, gr = oracle.solve(W.trees[0], W.rho)
        assert max(field_errors(phi[off:off + n], g[off:off + n], pr, gr)) < TOL64
        off += n
    assert st["n_trees"] == 4


def autotuned_graph_solve(W, precision):
    """The configuration the benchmark times: autotuned launch shape (overlap
    up to 2), graph replays; returns the last replay's result."""
    r = torch.tensor(W.rho, dtype=torch.float64, device=DEV)
    with fm.Plan(W.trees, precision=precision, autotune=True, use_graph=True, overlap=2) as p:
        phi_t, g_t = p.solve(r)
        for _ in range(2):
            p.solve(r, phi_t, g_t)  # replays of the captured graph
        torch.cuda.synchronize()
        sh = p.launch_shape()
        st = p.stats()
    print(f"  {W.name} {precision}: shape {sh}", flush=True)
    return phi_t.cpu().numpy(), g_t.cpu().numpy(), st


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_f32"])
def test_c1_full_size_autotuned_graph(precision):
    """The uniform level-3 field in the benchmark's configuration, every leaf
    cell against the oracle."""
    W = wl.c1()
    t = W.trees[0]
    phi, g, _ = autotuned_graph_solve(W, precision)
    pr, gr = oracle.solve(t, W.rho)
    errs = field_errors(phi, g, pr, gr)
    f, tq = residuals(t, W.rho, g)
    print(f"  errors {errs} force {f:.3e} torque {tq:.3e}", flush=True)
    check_form("c1", precision, errs, f, tq)


def c4_workload():
    return cached("c4", wl.c4)


def c4_solution(precision):
    return cached(("c4", precision), lambda: autotuned_graph_solve(c4_workload(), precision))


@pytest.mark.parametrize("k", range(16))
def test_c4_batch_every_tree_every_cell(k):
    """The 16-tree binary-star batch solved in one plan in the benchmark's
    configuration (autotuned shape, graph replays) in all three precision
    forms; tree k, every leaf cell, against the oracle's solve of that tree
    alone, with its force and torque residuals."""
    W = c4_workload()
    off = sum(t.n_leaves for t in W.trees[:k])
    t = W.trees[k]
    n = t.n_leaves
    rho_k = W.rho[off:off + n]
    sols = {prec: c4_solution(prec) for prec in ("fp64", "mixed", "mixed_f32")}
    assert sols["fp64"][2]["n_trees"] == 16
    print(f"  oracle: tree {k} ({n} leaves)", flush=True)
    pr, gr = oracle.solve(t, rho_k)
    for prec, (phi, g, _) in sols.items():
        errs = field_errors(phi[off:off + n], g[off:off + n], pr, gr)
        f, tq = residuals(t, rho_k, g[off:off + n])
        print(f"  tree {k} {prec}: errors {errs} force {f:.3e} torque {tq:.3e}", flush=True)
        check_form("c4", prec, errs, f, tq)


def test_four_copies_of_the_batch_reproduce_it_bitwise():
    """64 trees in one plan (4 copies of the 16-tree batch, 122,928 leaf
    sub-grids, 4x the benchmark's size) in the persistent shape: every
    copy's potential and acceleration are bitwise those of the 16-tree plan
    (no item's arithmetic depends on another tree or on its position in the
    work list)."""
    W = c4_workload()
    kw = dict(persistent=True, plane_groups=1, blocks_per_cu=3, overlap=0)
    phi1, g1, st1 = run(W.trees, W.rho, **kw)
    rho4 = np.concatenate([W.rho] * 4)
    phi4, g4, st4 = run(W.trees * 4, rho4, **kw)
    n = W.n_leaves
    print(f"  {st4['n_trees']} trees, {st4['n_leaves']} leaves, {sum(st4['pairs']) + st4['pairs_top']} pairs",
          flush=True)
    assert st4["n_trees"] == 64 and st4["n_leaves"] == 4 * n
    assert sum(st4["pairs"]) == 4 * sum(st1["pairs"])
    for c in range(4):
        assert np.array_equal(phi4[c * n:(c + 1) * n], phi1), c
        assert np.array_equal(g4[c * n:(c + 1) * n], g1), c


def test_zero_density_regions():
    """Cells without mass: their centre is their centre of mass and they act
    on nothing; an all-zero field gives exactly zero."""
    W = wl.small_amr(2)
    t = W.trees[0]
    rho = W.rho.copy()
    rho[::2] = 0.0                        # every other leaf empty
    rho[1, :, :, :4] = 0.0                # half of another leaf
    phi, g, _ = run([t], rho)
    pr, gr = oracle.solve(t, rho)
    assert np.isfinite(phi).all() and np.isfinite(g).all()
    assert max(field_errors(phi, g, pr, gr)) < TOL64
    phi0, g0, _ = run([t], np.zeros_like(rho))
    assert not phi0.any() and not g0.any()


@pytest.mark.parametrize("shape", ["per_class_g2", "persistent_g1"])
def test_isolated_point_masses_give_newton_on_the_gpu(shape):
    """At most one massive leaf cell per level-0 cell on the binary-star tree
    (five levels, all four classes, class-4 chunks, both sweep frames): at the
    massive cells the product's field is Newton's sum to round-off, checked
    against the direct sum without going through the FMM oracle."""
    t = c2_workload().trees[0]
    rho = wl.isolated_masses(t, 11)
    li, ci = np.nonzero(rho.reshape(rho.shape[0], 512) > 0)
    print(f"  {li.shape[0]} isolated masses", flush=True)
    assert li.shape[0] > 250
    phi, g, _ = run([t], rho, use_graph=True, **SHAPES[shape])
    pd, gd = oracle.direct_sum_sampled(t, rho, li, ci)
    ep = np.abs(phi[li, ci] - pd).max() / np.abs(pd).max()
    eg = np.abs(g[li, :, ci] - gd).max() / np.abs(gd).max()
    print(f"  errors against Newton: phi {ep:.3e} g {eg:.3e}", flush=True)
    assert ep < TOL64 and eg < TOL64


@pytest.mark.parametrize("shape", ["per_class_g2", "persistent_g2"])
def test_graph_replays_match_eager(shape):
    W = wl.small_amr(5)
    t = W.trees[0]
    r = torch.tensor(W.rho, dtype=torch.float64, device=DEV)
    with fm.Plan([t], **SHAPES[shape]) as pe:
        pe_phi, pe_g = pe.solve(r)
    torch.cuda.synchronize()
    ref_phi, ref_g = pe_phi.clone(), pe_g.clone()
    phi = torch.empty_like(ref_phi)
    g = torch.empty_like(ref_g)
    with fm.Plan([t], use_graph=True, **SHAPES[shape]) as pg:
        for rep in range(4):
            phi.fill_(float("nan"))
            g.fill_(float("nan"))
            x = torch.randn(1000, 1000, device=DEV) @ torch.randn(1000, 1000, device=DEV)  # unrelated eager work
            pg.solve(r, phi, g)
            torch.cuda.synchronize()
            assert torch.equal(phi, ref_phi) and torch.equal(g, ref_g), rep
            del x
        assert pg.stats()["solves"] == 4


def test_graph_recaptures_for_new_buffers_on_a_side_stream():
    """A graph plan used on a non-default stream with two alternating output
    buffers: every solve lands in its own buffers, in stream order."""
    W = wl.small_amr(3)
    t = W.trees[0]
    pr, gr = oracle.solve(t, W.rho)
    r = torch.tensor(W.rho, dtype=torch.float64, device=DEV)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    outs = [(torch.empty((W.n_leaves, 512), dtype=torch.float64, device=DEV),
             torch.empty((W.n_leaves, 3, 512), dtype=torch.float64, device=DEV)) for _ in range(2)]
    with fm.Plan([t], use_graph=True, persistent=True) as p:
        with torch.cuda.stream(s):
            for rep in range(4):
                phi, g = outs[rep % 2]
                phi.fill_(float("nan"))
                g.fill_(float("nan"))
                p.solve(r, phi, g, stream=s)
        s.synchronize()
        assert p.stats()["solves"] == 4
    for phi, g in outs:
        assert max(field_errors(phi.cpu().numpy(), g.cpu().numpy(), pr, gr)) < TOL64


def test_batched_plans_replay_a_graph_by_default():
    """Default options: a batched plan captures its launch sequence on the first
    solve and replays it (the same result as eager launches, bit for bit); a
    one-tree plan and a timed batched plan launch eagerly."""
    a, b = wl.small_amr(2), wl.small_amr(3)
    trees = [a.trees[0], b.trees[0]]
    r = torch.tensor(np.concatenate([a.rho, b.rho]), dtype=torch.float64, device=DEV)
    with fm.Plan(trees, use_graph=False) as pe:
        ref = [x.clone() for x in pe.solve(r)]
        torch.cuda.synchronize()
        assert pe.launch_shape()["use_graph"] == 0
    with fm.Plan(trees) as p:
        assert p.launch_shape()["use_graph"] == 1
        for rep in range(3):
            phi, g = p.solve(r)
            torch.cuda.synchronize()
            assert torch.equal(phi, ref[0]) and torch.equal(g, ref[1]), rep
    with fm.Plan([a.trees[0]]) as p1:
        assert p1.launch_shape()["use_graph"] == 0
    with fm.Plan(trees, timing=True) as pt:
        assert pt.launch_shape()["use_graph"] == 0


@pytest.mark.parametrize("shape", ["per_class_g2", "persistent_g2"])
def test_repeat_solves_are_bitwise_deterministic(shape):
    """Every output is written by one work item in a fixed order, so even the
    dynamically scheduled persistent launch is bitwise reproducible."""
    W = wl.small_amr(2)
    r = torch.tensor(W.rho, dtype=torch.float64, device=DEV)
    with fm.Plan([W.trees[0]], **SHAPES[shape]) as p:
        a = [t.clone() for t in p.solve(r)]
        b = p.solve(r)
        torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


# ---------------------------------------------------------------------------
# mixed precision
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["mixed", "mixed_f32"])
@pytest.mark.parametrize("shape", ["per_class_g2", "persistent_g2"])
def test_mixed_c1_error_bounds(shape, precision):
    W = wl.c1()
    t = W.trees[0]
    phi, g, _ = run([t], W.rho, precision=precision, use_graph=True, **SHAPES[shape])
    pr, gr = oracle.solve(t, W.rho)
    errs = field_errors(phi, g, pr, gr)
    f, tq = residuals(t, W.rho, g)
    print(f"  {precision} c1 errors {errs} force {f:.3e} torque {tq:.3e}", flush=True)
    check_form("c1", precision, errs, f, tq)


@pytest.mark.parametrize("precision", ["mixed", "mixed_f32"])
def test_mixed_c2_against_the_oracle_and_the_truncation_error(precision):
    """Mixed forms on the binary-star field: every leaf cell against the FP64
    oracle within the stated bounds, force and torque residuals, and the
    precision error at most a tenth of the method's own truncation error
    (the oracle against Newton's sum at sampled cells)."""
    W = c2_workload()
    t = W.trees[0]
    pmx, gmx, _ = run([t], W.rho, precision=precision, use_graph=True, persistent=True, plane_groups=1)
    pr, gr = c2_oracle()
    errs = field_errors(pmx, gmx, pr, gr)
    f, tq = residuals(t, W.rho, gmx)
    print(f"  {precision} c2 errors {errs} force {f:.3e} torque {tq:.3e}", flush=True)
    check_form("c2", precision, errs, f, tq)
    rng = np.random.default_rng(7)
    li = rng.integers(0, t.n_leaves, 400).astype(np.int32)
    ci = rng.integers(0, 512, 400).astype(np.int32)
    pd, gd = cached("c2_direct_400", lambda: oracle.direct_sum_sampled(t, W.rho, li, ci))
    n = np.linalg.norm
    trunc_phi = n(pr[li, ci] - pd) / n(pd)
    trunc_g = n(gr[li, :, ci] - gd) / n(gd)
    mix_phi = n(pmx[li, ci] - pr[li, ci]) / n(pd)
    mix_g = n(gmx[li, :, ci] - gr[li, :, ci]) / n(gd)
    print(f"  c2 truncation phi {trunc_phi:.3e} g {trunc_g:.3e}; {precision} phi {mix_phi:.3e} g {mix_g:.3e}",
          flush=True)
    assert mix_phi <= 0.1 * trunc_phi and mix_g <= 0.1 * trunc_g


@pytest.mark.parametrize("precision", ["mixed", "mixed_f32"])
@pytest.mark.parametrize("shape", ["per_class_g2", "persistent_g2", "persistent_g1_pairs"])
def test_mixed_amr_error_bounds(shape, precision):
    W = wl.small_amr(3)
    t = W.trees[0]
    phi, g, _ = run([t], W.rho, precision=precision, **SHAPES[shape])
    pr, gr = oracle.solve(t, W.rho)
    errs = field_errors(phi, g, pr, gr)
    f, tq = residuals(t, W.rho, g)
    print(f"  {precision} amr errors {errs} force {f:.3e} torque {tq:.3e}", flush=True)
    check_form("amr", precision, errs, f, tq)


def flat_forest(seed, axis=1):
    """A 3 x 1 x 3 forest of refined level-0 sub-grids (level 1 is 6 x 2 x 6
    sub-grids, one side in y always absent), a few level-1 sub-grids refined
    once more: refined targets whose sources lie beside them in y, the case
    where plane items run along y, and leaf targets beside refined ones.
    axis = 0: the same with x as the thin axis (1 x 3 x 3, plane items along
    x)."""
    rng = np.random.default_rng(seed)
    n0 = [3, 3, 3]
    n0[axis] = 1
    subs = [(0, x, y, z) for x in range(n0[0]) for y in range(n0[1]) for z in range(n0[2])]
    l1 = [(1, x, y, z) for x in range(2 * n0[0]) for y in range(2 * n0[1]) for z in range(2 * n0[2])]
    subs += l1
    for k in rng.choice(len(l1), 5, replace=False):
        _, x, y, z = l1[k]
        subs += [(2, 2 * x + a, 2 * y + b, 2 * z + c) for a in (0, 1) for b in (0, 1) for c in (0, 1)]
    t = wl._desc_from_list(subs, (0.0, 0.0, 0.0), 1.0)
    return t, rng.lognormal(0.0, 1.0, (t.n_leaves, 8, 8, 8))


@pytest.mark.parametrize("shape", ["per_class_g2", "persistent_g1", "per_class_g3", "persistent_g1_pairs"])
def test_y_sweep_targets_fp64(shape):
    t, rho = flat_forest(7)
    n_y = fm.fmmg_count_pairs([t])["sweep_y_targets"]
    phi, g, st = run([t], rho, **SHAPES[shape])
    pr, gr, ost = oracle.solve(t, rho, with_stats=True)
    errs = field_errors(phi, g, pr, gr)
    f, tq = residuals(t, rho, g, centre=(0.75, 0.0625, 0.75))
    print(f"  {n_y} y-sweep targets, errors {errs}, force {f:.3e} torque {tq:.3e}", flush=True)
    assert n_y >= 3 and st["pairs"][3] > 0
    assert max(errs) < TOL64
    assert st["pairs"] == ost["cls"]
    assert f < 1e-13 and tq < 1e-13


@pytest.mark.parametrize("precision", ["mixed", "mixed_f32"])
def test_y_sweep_targets_mixed(precision):
    t, rho = flat_forest(8)
    phi, g, _ = run([t], rho, precision=precision, persistent=True)
    pr, gr = oracle.solve(t, rho)
    errs = field_errors(phi, g, pr, gr)
    f, tq = residuals(t, rho, g, centre=(0.75, 0.0625, 0.75))
    print(f"  {precision} errors {errs} force {f:.3e} torque {tq:.3e}", flush=True)
    check_form("amr", precision, errs, f, tq)


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_f32"])
def test_plane_pair_and_single_plane_items_against_the_oracle(precision):
    """Refined-target items of both target planes of a parent plane (each
    staged source plane serving 128 targets, two waves per plane) and of one
    plane (four waves): each against the oracle, on a random AMR tree and on
    the forest whose plane items run along y, in one and in three plane
    groups, with the choice reported in the launch shape."""
    cases = [(*wl.small_amr(3).trees, wl.small_amr(3).rho, (0.5, 0.5, 0.5))]
    t, rho = flat_forest(8)
    cases.append((t, rho, (0.75, 0.0625, 0.75)))
    for t, rho, centre in cases:
        pr, gr = oracle.solve(t, rho)
        r = torch.tensor(rho, dtype=torch.float64, device=DEV)
        for groups in (1, 3):
            for pairs in (True, False):
                with fm.Plan([t], precision=precision, persistent=True, plane_groups=groups,
                             plane_pairs=pairs) as p:
                    assert p.launch_shape()["plane_pairs"] == int(pairs)
                    phi, g = p.solve(r)
                    torch.cuda.synchronize()
                errs = field_errors(phi.cpu().numpy(), g.cpu().numpy(), pr, gr)
                f, tq = residuals(t, rho, g.cpu().numpy(), centre=centre)
                print(f"  groups {groups} pairs {pairs}: errors {errs} force {f:.3e} torque {tq:.3e}",
                      flush=True)
                if precision == "fp64":
                    assert max(errs) < TOL64 and f < 1e-13 and tq < 1e-13
                else:
                    check_form("amr", precision, errs, f, tq)


def test_plane_pairs_default_follows_the_item_count():
    """By default refined-target items are paired when the paired items
    number at least 8 per compute unit: on the 16-tree batch, not on the
    uniform level-3 tree."""
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    for W, groups in ((c4_workload(), 1), (wl.c1(), 2)):
        n_ref = sum(int(t.refined_mask().sum()) - int(((t.level == 0) & t.refined_mask()).sum())
                    for t in W.trees)
        with fm.Plan(W.trees, plane_groups=groups) as p:
            got = p.launch_shape()["plane_pairs"]
        print(f"  {W.name}: {n_ref} refined non-top targets, plane_pairs {got}", flush=True)
        assert got == int(n_ref * 4 * groups >= 8 * n_cu)


@pytest.mark.parametrize("shape", ["per_class_g2", "persistent_g1", "persistent_g1_pairs", "persistent_g3_single"])
def test_x_sweep_targets_fp64(shape):
    t, rho = flat_forest(7, axis=0)
    n_x = fm.fmmg_count_pairs([t])["sweep_x_targets"]
    phi, g, st = run([t], rho, **SHAPES[shape])
    pr, gr, ost = oracle.solve(t, rho, with_stats=True)
    errs = field_errors(phi, g, pr, gr)
    f, tq = residuals(t, rho, g, centre=(0.0625, 0.75, 0.75))
    print(f"  {n_x} x-sweep targets, errors {errs}, force {f:.3e} torque {tq:.3e}", flush=True)
    assert n_x >= 3 and st["pairs"][3] > 0
    assert max(errs) < TOL64
    assert st["pairs"] == ost["cls"]
    assert f < 1e-13 and tq < 1e-13


@pytest.mark.parametrize("precision", ["mixed", "mixed_f32"])
def test_x_sweep_targets_mixed(precision):
    t, rho = flat_forest(9, axis=0)
    assert fm.fmmg_count_pairs([t])["sweep_x_targets"] >= 3
    phi, g, _ = run([t], rho, precision=precision, persistent=True, plane_pairs=True)
    pr, gr = oracle.solve(t, rho)
    errs = field_errors(phi, g, pr, gr)
    f, tq = residuals(t, rho, g, centre=(0.0625, 0.75, 0.75))
    print(f"  {precision} errors {errs} force {f:.3e} torque {tq:.3e}", flush=True)
    check_form("amr", precision, errs, f, tq)


# ---------------------------------------------------------------------------
# interface behaviour
# ---------------------------------------------------------------------------
def test_density_check_and_argument_errors():
    W = wl.small_amr(1)
    r = torch.tensor(W.rho, dtype=torch.float64, device=DEV)
    with fm.Plan([W.trees[0]]) as p:
        p.check_density(r)
        bad = r.clone().view(-1, 512)
        bad[3, 100] = -1.0
        with pytest.raises(fm.FmmgError) as e:
            p.check_density(bad)
        assert e.value.status == fm.FMMG_EINVAL and str(3 * 512 + 100) in str(e.value)
        bad[3, 100] = float("nan")
        with pytest.raises(fm.FmmgError):
            p.check_density(bad)
        with pytest.raises(ValueError):
            p.solve(r[:-1].contiguous())
        with pytest.raises(ValueError):
            p.solve(r.float())
        # overlapping buffers are refused before any launch
        n = W.rho.shape[0]
        big = torch.zeros(5 * n * 512, dtype=torch.float64, device=DEV)
        with pytest.raises(fm.FmmgError) as e:
            fm.fmmg_solve(p._h, r, r.view(n, 512), big[:3 * n * 512].view(n, 3, 512))
        assert e.value.status == fm.FMMG_EINVAL and "overlap" in str(e.value)
        with pytest.raises(fm.FmmgError):
            fm.fmmg_solve(p._h, r, big[:n * 512].view(n, 512), big[n * 512 - 8:4 * n * 512 - 8].view(n, 3, 512))
        phi, g = p.solve(r, big[:n * 512].view(n, 512), big[n * 512:4 * n * 512].view(n, 3, 512))
        torch.cuda.synchronize()
        pr, gr = oracle.solve(W.trees[0], W.rho)
        assert max(field_errors(phi.cpu().numpy(), g.cpu().numpy(), pr, gr)) < TOL64


@pytest.mark.parametrize("bpc", [3, 1])
def test_xcd_queues_and_single_list_are_bitwise_equal(bpc):
    """The persistent launch's two item orders (one queue per XCD, or one
    largest-first list) run the same items, each output written by one item
    in a fixed order: bitwise equal results, in a graph and eagerly, on the
    batch of 16 binary-star trees and on one random AMR tree."""
    for W in (c4_workload(), wl.small_amr(5)):
        r = torch.tensor(W.rho, dtype=torch.float64, device=DEV)
        outs = []
        for q in (1, 0):
            for graph in (True, False):
                with fm.Plan(W.trees, persistent=True, plane_groups=1, blocks_per_cu=bpc, xcd_queues=q,
                             use_graph=graph) as p:
                    assert p.launch_shape()["xcd_queues"] == q
                    for _ in range(2):
                        phi, g = p.solve(r)
                    torch.cuda.synchronize()
                    outs.append((phi.clone(), g.clone()))
        print(f"  {W.name}: {len(outs)} runs", flush=True)
        for phi, g in outs[1:]:
            assert torch.equal(phi, outs[0][0]) and torch.equal(g, outs[0][1])


@pytest.mark.parametrize("groups", [1, 3])
def test_persistent_and_class_launches_are_bitwise_equal(groups):
    """The persistent launch (items taken largest first from a counter, all
    classes mixed) and the per-class launches run the same items, each
    writing its own outputs: bitwise equal results, on a tree with every
    class and both sweep frames, and on a batch."""
    t, rho = flat_forest(9)
    a, b = wl.small_amr(5), wl.small_amr(11, max_level=3, p_refine=0.3)
    for trees, r_np in (([t], rho), ([a.trees[0], b.trees[0]], np.concatenate([a.rho, b.rho]))):
        r = torch.tensor(r_np, dtype=torch.float64, device=DEV)
        outs = []
        for kw in (dict(), dict(persistent=True), dict(persistent=True, blocks_per_cu=1)):
            with fm.Plan(trees, plane_groups=groups, **kw) as p:
                outs.append([x.clone() for x in p.solve(r)])
                torch.cuda.synchronize()
        for o in outs[1:]:
            assert torch.equal(o[0], outs[0][0]) and torch.equal(o[1], outs[0][1])


@pytest.mark.parametrize("shape", ["per_class_g2", "persistent_g1"])
def test_overlapped_coarse_branch_equals_one_stream(shape):
    """The coarse levels on the second stream (eager and graph) give bitwise
    the same result as one stream: every output has one writer and a fixed
    summation order, whatever runs concurrently."""
    cases = [wl.c1(), wl.small_amr(1), wl.small_amr(3), wl.c1(max_level=2)]
    forked = 0
    for W in cases:
        t = W.trees[0]
        r = torch.tensor(W.rho, dtype=torch.float64, device=DEV)
        with fm.Plan([t], overlap=False, **SHAPES[shape]) as p1:
            ref = [x.clone() for x in p1.solve(r)]
            torch.cuda.synchronize()
            assert p1.launch_shape()["overlap"] == 0
        for ov, graph in ((1, False), (1, True), (2, False), (2, True)):
            with fm.Plan([t], overlap=ov, use_graph=graph, **SHAPES[shape]) as p2:
                for rep in range(3):
                    out = p2.solve(r)
                    torch.cuda.synchronize()
                    assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1]), (W.name, ov, graph, rep)
                sh = p2.launch_shape()
                print(f"  {W.name}: split level {sh['split_level']}, overlap {sh['overlap']}", flush=True)
                forked += sh["overlap"] > 0
    assert forked >= 4  # the uniform trees split (levels 0-1 coarse)


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_f32"])
def test_per_subgrid_launch_model_equals_class_launches(precision):
    """The paper's execution model (one launch per target sub-grid and class,
    round-robin over a stream pool; Sec. 5.1): against the oracle (1e-12 in
    FP64, the stated bounds in the FP32 forms), and bitwise equal to the class
    launches, which run the same work items, eager and in a graph, for one
    tree, a uniform tree and a batch."""
    a, b, u = wl.small_amr(2), wl.small_amr(3), wl.c1(max_level=2)
    s1 = wl.small_amr(1)
    cases = [([s1.trees[0]], s1.rho, [s1]), ([u.trees[0]], u.rho, [u]),
             ([a.trees[0], b.trees[0]], np.concatenate([a.rho, b.rho]), [a, b])]
    for trees, rho, parts in cases:
        r = torch.tensor(rho, dtype=torch.float64, device=DEV)
        with fm.Plan(trees, precision=precision, plane_groups=2, launch_streams=128) as pm:
            phi, g = pm.solve(r)
            torch.cuda.synchronize()
            phi, g = phi.cpu().numpy(), g.cpu().numpy()
        off = 0
        for W in parts:
            n = W.n_leaves
            pr, gr = oracle.solve(W.trees[0], W.rho)
            errs = field_errors(phi[off:off + n], g[off:off + n], pr, gr)
            f, tq = residuals(W.trees[0], W.rho, g[off:off + n])
            print(f"  launch model {precision} {W.name}: errors {errs} force {f:.3e} torque {tq:.3e}", flush=True)
            check_form("c1" if W.name.startswith("c1") else "amr", precision, errs, f, tq)
            off += n
        r = torch.tensor(rho, dtype=torch.float64, device=DEV)
        with fm.Plan(trees, precision=precision, overlap=0, plane_groups=2) as p1:
            ref = [x.clone() for x in p1.solve(r)]
            torch.cuda.synchronize()
            base_launches = p1.stats()["launches"]
        for ns, graph in ((1, False), (8, False), (128, False), (128, True)):
            with fm.Plan(trees, precision=precision, plane_groups=2, launch_streams=ns, use_graph=graph) as p2:
                for rep in range(2):
                    out = p2.solve(r)
                    torch.cuda.synchronize()
                    assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1]), (len(trees), ns, graph, rep)
                assert p2.launch_shape()["launch_streams"] == ns
                n = p2.stats()["launches"]
        print(f"  {len(trees)} tree(s): {base_launches} class launches, {n} per-sub-grid launches", flush=True)
        assert n > base_launches


def test_autotune_picks_a_shape_and_caches_it(tmp_path):
    W = wl.small_amr(1)
    t = W.trees[0]
    cache = str(tmp_path / "tune.json")
    r = torch.tensor(W.rho, dtype=torch.float64, device=DEV)
    pr, gr = oracle.solve(t, W.rho)
    with fm.Plan([t], autotune=True, tuning_cache=cache, use_graph=True) as p:
        phi, g = p.solve(r)
        torch.cuda.synchronize()
        sh = p.launch_shape()
    assert sh["from_cache"] == 0 and sh["tuned_ms"] > 0
    assert max(field_errors(phi.cpu().numpy(), g.cpu().numpy(), pr, gr)) < TOL64
    import json
    with open(cache) as f:
        tab = json.load(f)
    assert len(tab) == 1
    with fm.Plan([t], autotune=True, tuning_cache=cache, use_graph=True) as p2:
        phi2, g2 = p2.solve(r)
        torch.cuda.synchronize()
        sh2 = p2.launch_shape()
    assert sh2["from_cache"] == 1
    for k in ("persistent", "plane_groups", "blocks_per_cu", "overlap", "split_level", "xcd_queues", "plane_pairs"):
        assert sh2[k] == sh[k]
    assert max(field_errors(phi2.cpu().numpy(), g2.cpu().numpy(), pr, gr)) < TOL64
    # shapes timed as graph replays, or with a larger overlap allowance, are
    # not reused by an eager plan or one that allows less overlap
    for kw in (dict(use_graph=False), dict(use_graph=True, overlap=0)):
        with fm.Plan([t], autotune=True, tuning_cache=cache, **kw) as p3:
            p3.solve(r)
            torch.cuda.synchronize()
            sh3 = p3.launch_shape()
        assert sh3["from_cache"] == 0 and sh3["overlap"] <= kw.get("overlap", 1)
    with open(cache) as f:
        assert len(json.load(f)) == 3


def test_stage_timing_counts_launches():
    W = wl.small_amr(2)
    r = torch.tensor(W.rho, dtype=torch.float64, device=DEV)
    for pers in (False, True):
        with fm.Plan([W.trees[0]], timing=True, persistent=pers) as p:
            for _ in range(3):
                p.solve(r)
            torch.cuda.synchronize()
            tm = p.timings()
        assert tm["solves"] == 3
        assert all(v >= 0 for v in tm["ms"].values())
        if pers:
            assert tm["launches"]["fused"] >= 1 and tm["launches"]["mp_refined"] == 0
        else:
            assert tm["launches"]["mp_refined"] >= 1 and tm["launches"]["fused"] == 0


@pytest.mark.parametrize("shape", ["per_class_g2", "persistent_g2"])
def test_solve_reports_a_bad_density_at_the_next_call(shape):
    """A negative or non-finite density that a solve reads is recorded on the
    device, without synchronising; the next call on the plan returns
    FMMG_EINVAL with the smallest bad flat index and enqueues nothing; the
    report is then taken, and the status query gives the same report.
    Covers parentless leaves (the 27-leaf forest) and leaves under a parent
    (a random AMR tree), eager and captured."""
    cases = [(wl.c0(3), "full"), (wl.small_amr(1), "full")]
    for W, top in cases:
        t = W.trees[0]
        n = W.n_leaves
        pr, gr = oracle.solve(t, W.rho)
        r = torch.tensor(W.rho, dtype=torch.float64, device=DEV)
        for graph in (False, True):
            with fm.Plan([t], use_graph=graph, **SHAPES[shape]) as p:
                phi, g = p.solve(r)
                torch.cuda.synchronize()
                assert p.density_status() == -1
                for val, leaf, cell in ((float("nan"), 3, 100), (-1.0, n - 1, 511), (float("inf"), 0, 0),
                                        (-float("inf"), n // 2, 257)):
                    bad = r.clone().view(n, 512)
                    bad[leaf, cell] = val
                    bad[n - 1, 511] = float("nan")   # a second, larger bad index
                    flat = leaf * 512 + cell
                    print(f"  {W.name} graph={graph} value {val} at {flat}", flush=True)
                    p.solve(bad.view_as(r), phi, g)  # enqueued, reported later
                    torch.cuda.synchronize()
                    with pytest.raises(fm.FmmgError) as e:
                        p.solve(r, phi, g)
                    assert e.value.status == fm.FMMG_EINVAL and f"flat index {flat};" in str(e.value)
                    phi, g = p.solve(r, phi, g)       # the report was taken: this one runs
                    torch.cuda.synchronize()
                    assert max(field_errors(phi.cpu().numpy(), g.cpu().numpy(), pr, gr)) < TOL64
                    assert p.density_status() == -1
                # the status query takes a report as well
                bad = r.clone().view(n, 512)
                bad[1, 2] = -0.5
                p.solve(bad.view_as(r), phi, g)
                torch.cuda.synchronize()
                with pytest.raises(fm.FmmgError) as e:
                    p.density_status()
                assert e.value.status == fm.FMMG_EINVAL and str(512 + 2) in str(e.value)
                assert p.density_status() == -1
                p.solve(r, phi, g)
                torch.cuda.synchronize()
