"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

FP64 bar: per field (phi and each g component), max |gpu - oracle| / max |oracle|
<= 1e-12.  Mixed form: the stated bounds below (FP32 pair terms).
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


@pytest.mark.parametrize("seed", [1, 2, 3, 5])
def test_random_amr_fp64(seed):
    """All four classes, coarse-fine boundaries, absent neighbours."""
    W = wl.small_amr(seed)
    t = W.trees[0]
    phi, g, st = run([t], W.rho)
    pr, gr, ost = oracle.solve(t, W.rho, with_stats=True)
    errs = field_errors(phi, g, pr, gr)
    print("  errors", errs, flush=True)
    assert max(errs) < TOL64
    assert st["pairs"] == ost["cls"] and st["pairs_top"] == ost["top"]
    f, tq = residuals(t, W.rho, g)
    assert f < 1e-13 and tq < 1e-13


def test_random_amr_deeper_fp64():
    W = wl.small_amr(11, max_level=3, p_refine=0.3)
    t = W.trees[0]
    phi, g, _ = run([t], W.rho)
    pr, gr = oracle.solve(t, W.rho)
    assert max(field_errors(phi, g, pr, gr)) < TOL64


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


def test_c1_full_size_fp64_graph():
    """Uniform level-3 polytrope (64^3 leaf cells), in the launch
    configuration that the benchmark times (captured graph)."""
    W = wl.c1()
    t = W.trees[0]
    phi, g, st = run([t], W.rho, use_graph=True)
    pr, gr = oracle.solve(t, W.rho)
    errs = field_errors(phi, g, pr, gr)
    print("  c1 errors", errs, flush=True)
    assert max(errs) < TOL64
    assert st["pairs"] == [0, 1705080 + 17246904, 176804352, 0] and st["pairs_top"] == 230616


def test_c2_full_size_fp64_sampled():
    """Binary-star AMR field (3,816 leaves), sampled against the oracle."""
    W = wl.c2()
    t = W.trees[0]
    phi, g, st = run([t], W.rho, use_graph=True)
    rng = np.random.default_rng(0)
    li = rng.integers(0, t.n_leaves, 1500).astype(np.int32)
    ci = rng.integers(0, 512, 1500).astype(np.int32)
    # include the cells with the largest |g| and the coarse leaves
    big = np.argsort(-np.abs(g).max(1).reshape(-1))[:100]
    coarse = np.nonzero(t.level[t.leaf_indices()] < 5)[0][:50]
    li = np.concatenate([li, (big // 512).astype(np.int32), coarse.astype(np.int32)])
    ci = np.concatenate([ci, (big % 512).astype(np.int32), np.full(coarse.shape, 300, np.int32)])
    ps, gs = oracle.solve_sampled(t, W.rho, li, ci)
    e_phi = np.abs(phi[li, ci] - ps).max() / np.abs(ps).max()
    e_g = np.abs(g[li, :, ci] - gs).max() / np.abs(gs).max()
    print(f"  c2 sampled errors phi {e_phi:.3e} g {e_g:.3e}", flush=True)
    assert e_phi < TOL64 and e_g < TOL64
    f, tq = residuals(t, W.rho, g)
    print(f"  c2 residual force {f:.3e} torque {tq:.3e}", flush=True)
    assert f < 1e-12 and tq < 1e-12


def test_batched_trees_equal_each_tree_alone():
    Ws = [wl.small_amr(s) for s in (1, 2, 3)] + [wl.c1(max_level=2)]
    trees = [W.trees[0] for W in Ws]
    rho = np.concatenate([W.rho for W in Ws])
    phi, g, st = run(trees, rho, use_graph=True)
    off = 0
    for W in Ws:
        n = W.n_leaves
        pr, gr = oracle.solve(W.trees[0], W.rho)
        assert max(field_errors(phi[off:off + n], g[off:off + n], pr, gr)) < TOL64
        off += n
    assert st["n_trees"] == 4


def test_graph_replays_match_eager():
    W = wl.small_amr(5)
    t = W.trees[0]
    r = torch.tensor(W.rho, dtype=torch.float64, device=DEV)
    with fm.Plan([t]) as pe:
        pe_phi, pe_g = pe.solve(r)
    torch.cuda.synchronize()
    ref_phi, ref_g = pe_phi.clone(), pe_g.clone()
    phi = torch.empty_like(ref_phi)
    g = torch.empty_like(ref_g)
    with fm.Plan([t], use_graph=True) as pg:
        for rep in range(4):
            phi.fill_(float("nan"))
            g.fill_(float("nan"))
            x = torch.randn(1000, 1000, device=DEV) @ torch.randn(1000, 1000, device=DEV)  # unrelated eager work
            pg.solve(r, phi, g)
            torch.cuda.synchronize()
            assert torch.equal(phi, ref_phi) and torch.equal(g, ref_g), rep
            del x
        assert pg.stats()["solves"] == 4


def test_repeat_solves_are_bitwise_deterministic():
    W = wl.small_amr(2)
    r = torch.tensor(W.rho, dtype=torch.float64, device=DEV)
    with fm.Plan([W.trees[0]]) as p:
        a = [t.clone() for t in p.solve(r)]
        b = p.solve(r)
        torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


# ---------------------------------------------------------------------------
# mixed precision
# ---------------------------------------------------------------------------
def test_mixed_c1_error_bounds():
    W = wl.c1()
    t = W.trees[0]
    phi, g, _ = run([t], W.rho, precision="mixed", use_graph=True)
    pr, gr = oracle.solve(t, W.rho)
    errs = field_errors(phi, g, pr, gr)
    f, tq = residuals(t, W.rho, g)
    print(f"  mixed c1 errors {errs} force {f:.3e} torque {tq:.3e}", flush=True)
    assert errs[0] < 2e-6 and max(errs[1:]) < 2e-5
    assert f < 1e-6


def test_mixed_amr_error_bounds():
    W = wl.small_amr(3)
    t = W.trees[0]
    phi, g, _ = run([t], W.rho, precision="mixed")
    pr, gr = oracle.solve(t, W.rho)
    errs = field_errors(phi, g, pr, gr)
    f, tq = residuals(t, W.rho, g)
    print(f"  mixed amr errors {errs} force {f:.3e} torque {tq:.3e}", flush=True)
    assert errs[0] < 2e-6 and max(errs[1:]) < 2e-5
    assert f < 1e-6 and tq < 1e-6


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
