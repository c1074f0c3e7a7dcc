"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: numbers the
paper prints (tests/golden/paper_facts.json), closed forms, exact identities,
invariants, and brute force on tiny inputs.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from paper_1908_03121_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def paper_facts():
    with open(os.path.join(GOLDEN, "paper_facts.json")) as f:
        return json.load(f)


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def leaf_masses(tree, rho):
    h = tree.leaf_cell_size()
    return rho * (h ** 3)[:, None, None, None]


def momentum_residuals(tree, rho, g, centre=(0.5, 0.5, 0.5)):
    """|sum m g| / sum |m g| and |sum x x m g| / sum |x x m g| (max over axes)."""
    x = tree.leaf_cell_centres().reshape(-1, 3) - np.asarray(centre)
    m = leaf_masses(tree, rho).reshape(-1)
    F = m[:, None] * g.transpose(0, 2, 1).reshape(-1, 3)
    tau = np.cross(x, F)
    return (float(np.abs(F.sum(0)).max() / np.abs(F).sum(0).max()),
            float(np.abs(tau.sum(0)).max() / np.abs(tau).sum(0).max()))


# ----------------------------------------------------------------------------
# interaction rule and stencil (Sec. 4.3: 1074-element stencil, 549,888/launch)
# ----------------------------------------------------------------------------
def _stencil(parity, far_only=False):
    out = []
    for d in itertools.product(range(-8, 9), repeat=3):
        ca = list(parity)
        cb = [ca[i] + d[i] for i in range(3)]
        # both cells refined: only far pairs; a leaf partner adds the near ones
        if oracle.pair_rule(0, ca, cb, 0, 0 if far_only else 1):
            out.append(d)
    return out


def test_stencil_union_is_papers_1074():
    facts = paper_facts()
    union, far_union = set(), set()
    for p in itertools.product((0, 1), repeat=3):
        s = _stencil(p)
        f = _stencil(p, far_only=True)
        assert len(s) == 743 and len(f) == 651          # per-parity partner counts
        assert max(max(abs(c) for c in d) for d in s) == 5  # reach: 26 neighbours suffice
        union |= set(s)
        far_union |= set(f)
    assert len(union) == facts["stencil_elements"]
    assert len(union) * facts["cells_per_subgrid"] == facts["interactions_per_launch"]
    assert len(far_union) == 982
    assert union == {tuple(-c for c in d) for d in union}    # d -> -d symmetric


def test_rule_is_symmetric_and_excludes_self():
    rng = np.random.default_rng(0)
    for _ in range(2000):
        ca = rng.integers(0, 40, 3)
        cb = ca + rng.integers(-7, 8, 3)
        cb = np.maximum(cb, 0)
        for top in (0, 1):
            for al, bl in itertools.product((0, 1), repeat=2):
                assert oracle.pair_rule(top, ca, cb, al, bl) == oracle.pair_rule(top, cb, ca, bl, al)
        assert oracle.pair_rule(1, ca, ca, 1, 1) == 0


def test_uniform_tree_pair_counts_cover_every_pair_once():
    """C1 (64^3 leaves): per-level ordered pair counts; weighted by the number
    of leaf cells below each side they must add up to N(N-1) exactly."""
    W = wl.c1()
    phi, g, st = oracle.solve(W.trees[0], W.rho, with_stats=True)
    pl = st["per_level"]
    assert pl[:4] == [230616, 1705080, 17246904, 176804352]
    N = 64 ** 3
    assert sum(pl[l] * 64 ** (3 - l) for l in range(4)) == N * (N - 1)
    assert st["top"] == 230616 and st["cls"] == [0, 1705080 + 17246904, 176804352, 0]


def test_pair_coverage_exactly_once_on_amr_trees():
    subs = ([(0, 0, 0, 0)] + [(1, x, y, z) for x in (0, 1) for y in (0, 1) for z in (0, 1)]
            + [(2, 2 + x, y, 2 + z) for x in (0, 1) for y in (0, 1) for z in (0, 1)])
    trees = [wl._desc_from_list(subs, (0, 0, 0), 1.0)]
    trees.append(wl.small_amr(7, max_level=2, p_refine=0.15).trees[0])
    for t in trees:
        if t.n_leaves > 20:
            continue
        cov = oracle.pair_coverage(t)
        assert np.all(np.diag(cov) == 0)
        off = cov + np.eye(cov.shape[0], dtype=np.uint8)
        assert off.min() == 1 and off.max() == 1


# ----------------------------------------------------------------------------
# derivative tensors of 1/r
# ----------------------------------------------------------------------------
def test_dtensors_finite_differences_trace_euler():
    rng = np.random.default_rng(3)
    for _ in range(20):
        R = rng.normal(size=3) * rng.uniform(0.5, 3)
        D = oracle.dtensors(R)
        r = np.linalg.norm(R)
        assert abs(D[0] - 1 / r) < 1e-15 / r
        eps = 1e-5 * r
        for k in range(4):
            # central difference of D^(k) along each axis -> D^(k+1)
            for a in range(3):
                e = np.zeros(3)
                e[a] = eps
                num = (np.asarray(oracle.dtensors(R + e)[k]) - np.asarray(oracle.dtensors(R - e)[k])) / (2 * eps)
                ana = np.take(D[k + 1], a, axis=0)
                assert np.abs(num - ana).max() < 1e-7 * np.abs(D[k + 1]).max()
        for k in range(2, 5):
            T = D[k]
            assert np.abs(np.einsum("ii...->...", T)).max() < 1e-13 * np.abs(T).max()  # harmonic
            for perm in itertools.permutations(range(k)):
                assert np.allclose(T, np.transpose(T, perm), rtol=0, atol=1e-14 * np.abs(T).max())
        for k in range(0, 4):
            # Euler: R . grad D^(k) = -(k+1) D^(k)   (D^(k) homogeneous of degree -(k+1))
            lhs = np.tensordot(R, D[k + 1], axes=(0, 0))
            assert np.abs(lhs + (k + 1) * np.asarray(D[k])).max() < 1e-13 * np.abs(D[k]).max() + 1e-300


# ----------------------------------------------------------------------------
# per-pair expansion (M2L with the n + m <= 3 truncation)
# ----------------------------------------------------------------------------
def _cluster_moments(x, m):
    M = m.sum()
    X = (m[:, None] * x).sum(0) / M
    r = x - X
    return (M, X, np.einsum("a,ai,aj->ij", m, r, r), np.einsum("a,ai,aj,ak->ijk", m, r, r, r))


def test_point_mass_pair_is_exact_newton():
    rng = np.random.default_rng(5)
    xa, xb = rng.normal(size=3), rng.normal(size=3) + 3
    mb = 2.5
    L0, L1, L2, L3, dg = oracle.m2l_pair(1.3, xa, None, mb, xb, None, None, G=0.7)
    R = xa - xb
    r = np.linalg.norm(R)
    assert abs(L0 - (-0.7 * mb / r)) < 1e-15 * abs(L0)
    assert np.abs(-L1 - (-0.7 * mb * R / r ** 3)).max() < 1e-15 * np.abs(L1).max()
    assert np.all(dg == 0)


def test_pair_expansion_convergence_orders():
    """Potential and total force of a cluster pair converge as (a/R)^4, the
    field at points as (a/R)^3: a dropped or mis-signed term breaks the order."""
    rng = np.random.default_rng(1)
    xb, mb = rng.uniform(-.5, .5, (20, 3)), rng.uniform(.5, 1.5, 20)
    xa0, ma = rng.uniform(-.5, .5, (15, 3)), rng.uniform(.5, 1.5, 15)
    errs = []
    for s in (4, 8, 16, 32):
        d = np.array([1.0, 0.7, 0.4]) * s
        MB, XB, M2B, M3B = _cluster_moments(xb, mb)
        MA, XA, M2A, M3A = _cluster_moments(xa0 + d, ma)
        L0, L1, L2, L3, dg = oracle.m2l_pair(MA, XA, M3A, MB, XB, M2B, M3B)
        y = xa0 + d - XA
        P = L0 + y @ L1 + 0.5 * np.einsum("ij,ai,aj->a", L2, y, y) + np.einsum("ijk,ai,aj,ak->a", L3, y, y, y) / 6
        Gm = -(L1 + y @ L2 + 0.5 * np.einsum("ijk,aj,ak->ai", L3, y, y))
        Rab = (xa0 + d)[:, None, :] - xb[None]
        r = np.linalg.norm(Rab, axis=-1)
        Pd = -(mb / r).sum(1)
        Gd = -(mb[None, :, None] * Rab / r[..., None] ** 3).sum(1)
        F = (ma[:, None] * Gm).sum(0) + MA * dg
        Fd = (ma[:, None] * Gd).sum(0)
        errs.append((rel(P, Pd), rel(Gm, Gd), rel(F, Fd)))
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios[:, 0] > 14) and np.all(ratios[:, 0] < 20)   # order 4
    assert np.all(ratios[:, 1] > 7) and np.all(ratios[:, 1] < 10)    # order 3
    assert np.all(ratios[:, 2] > 14) and np.all(ratios[:, 2] < 20)   # order 4


def test_pair_forces_balance_and_torques_cancel_only_with_correction():
    """Angular-momentum conservation of the same-level step (Sec. 4.2/4.3):
    with the correction the two sides' forces are opposite and the total
    torque (orbital + internal from the expansions) vanishes."""
    rng = np.random.default_rng(11)
    for corr, expect_zero in ((1, True), (0, False)):
        xa0, ma = rng.uniform(-.5, .5, (12, 3)), rng.uniform(.5, 1.5, 12)
        xb0, mb = rng.uniform(-.5, .5, (9, 3)), rng.uniform(.5, 1.5, 9)
        xa = xa0 + np.array([2.1, -1.3, 3.2])
        xb = xb0 + np.array([-0.4, 0.8, -0.9])
        A = _cluster_moments(xa, ma)
        B = _cluster_moments(xb, mb)

        def side(T, S, xs, ms):
            L0, L1, L2, L3, dg = oracle.m2l_pair(T[0], T[1], T[3], S[0], S[1], S[2], S[3], correction=corr)
            y = xs - T[1]
            g = -(L1 + y @ L2 + 0.5 * np.einsum("ijk,aj,ak->ai", L3, y, y)) + dg
            f = ms[:, None] * g
            return f.sum(0), np.cross(xs, f).sum(0)
        FA, tA = side(A, B, xa, ma)
        FB, tB = side(B, A, xb, mb)
        scale = np.abs(FA).max()
        assert np.abs(FA + FB).max() < 1e-14 * scale
        torque = np.abs(tA + tB).max() / (np.abs(tA).max() + np.abs(tB).max())
        if expect_zero:
            assert torque < 1e-14
        else:
            assert torque > 1e-8


# ----------------------------------------------------------------------------
# upward and downward passes
# ----------------------------------------------------------------------------
def test_upward_moments_equal_brute_force():
    W = wl.small_amr(2)
    t = W.trees[0]
    m, X, M2, M3 = oracle.upward(t, W.rho)
    xc = t.leaf_cell_centres().reshape(t.n_leaves, 512, 3)
    ml = leaf_masses(t, W.rho).reshape(t.n_leaves, 512)
    leaf_of = {int(s): i for i, s in enumerate(t.leaf_indices())}
    lev, crd = t.level, t.coord
    maxl = lev.max()
    # leaf cells at (level, global coords)
    for s in range(t.n_subgrids):
        if s in leaf_of:
            assert np.allclose(m[s], ml[leaf_of[s]], rtol=1e-15, atol=0)
            assert np.all(M2[s] == 0) and np.all(M3[s] == 0)
            continue
        for q in (0, 77, 300, 511):
            c = crd[s] * 8 + np.array([q >> 6, (q >> 3) & 7, q & 7])
            l = lev[s]
            pts, ms = [], []
            for li, sl in enumerate(t.leaf_indices()):
                L = lev[sl]
                if L < l:
                    continue
                cl = crd[sl] * 8 + np.stack(np.meshgrid(*[np.arange(8)] * 3, indexing="ij"), -1).reshape(512, 3)
                inside = np.all((cl >> (L - l)) == c, axis=1)
                if inside.any():
                    pts.append(xc[li][inside])
                    ms.append(ml[li][inside])
            pts, ms = np.concatenate(pts), np.concatenate(ms)
            Mb, Xb, M2b, M3b = _cluster_moments(pts, ms)
            assert abs(m[s, q] - Mb) <= 1e-13 * Mb
            assert np.abs(X[s, q] - Xb).max() <= 1e-14
            assert np.abs(M2[s, q] - M2b).max() <= 1e-12 * np.abs(M2b).max()
            assert np.abs(M3[s, q] - M3b).max() <= 1e-11 * np.abs(M3b).max()
    assert maxl >= 2


def test_l2l_reexpansion_of_cubic_is_exact():
    rng = np.random.default_rng(4)
    for _ in range(10):
        L0 = rng.normal()
        L1 = rng.normal(size=3)
        A = rng.normal(size=(3, 3))
        L2 = A + A.T
        B = rng.normal(size=(3, 3, 3))
        L3 = sum(np.transpose(B, p) for p in itertools.permutations(range(3)))
        r = rng.normal(size=3)
        o0, o1, o2, o3 = oracle.l2l(L0, L1, L2, L3, r)

        def P(y, c0, c1, c2, c3):
            return c0 + c1 @ y + 0.5 * y @ c2 @ y + np.einsum("ijk,i,j,k", c3, y, y, y) / 6
        for y in rng.normal(size=(5, 3)):
            assert abs(P(y, o0, o1, o2, o3) - P(y + r, L0, L1, L2, L3)) < 1e-12 * (1 + abs(P(y + r, L0, L1, L2, L3)))


# ----------------------------------------------------------------------------
# whole solve
# ----------------------------------------------------------------------------
def test_forest_of_leaves_all_pairs_is_the_direct_sum():
    """A level-0 forest of leaves under the all-pairs top rule evaluates every
    pair of point masses directly: the method reduces to the plain sum."""
    t = wl.forest_tree(2)
    rho = np.random.default_rng(9).lognormal(0, 1, (8, 8, 8, 8))
    phi, g = oracle.solve(t, rho, top_all_pairs=True)
    pd, gd = oracle.direct_sum(t, rho)
    assert rel(phi, pd) < 1e-13 and rel(g, gd) < 1e-13


def test_c0_near_field_equals_direct_sum_over_same_pairs():
    """Central sub-grid of the 3x3x3 forest with the parent-near stencil: its
    512 x 743 = 380,416 point-mass pairs summed directly in numpy."""
    W = wl.c0()
    t = W.trees[0]
    phi, g, st = oracle.solve(t, W.rho, top_all_pairs=False, with_stats=True)
    x = t.leaf_cell_centres().reshape(-1, 3)
    m = leaf_masses(t, W.rho).reshape(-1)
    gc = (t.coord[:, None, :] * 8 + np.stack(np.meshgrid(*[np.arange(8)] * 3, indexing="ij"), -1).reshape(1, 512, 3)).reshape(-1, 3)
    centre = 13
    npairs = 0
    for q in range(0, 512, 7):
        a = centre * 512 + q
        d = gc - gc[a]
        D = (gc // 2) - (gc[a] // 2)
        sel = ((D ** 2).sum(1) <= 8) & np.any(d != 0, axis=1)
        npairs += sel.sum()
        R = x[a] - x[sel]
        r = np.linalg.norm(R, axis=1)
        p = -(m[sel] / r).sum()
        gg = -(m[sel, None] * R / r[:, None] ** 3).sum(0)
        assert sel.sum() == 743
        assert abs(phi[centre, q] - p) < 1e-13 * abs(p)
        assert np.abs(g[centre, :, q] - gg).max() < 1e-13 * np.abs(gg).max()
    assert st["cls"][2] == 7862272


def test_c1_level2_fmm_vs_direct_sum_within_truncation():
    W = wl.c1(max_level=2)
    t = W.trees[0]
    phi, g = oracle.solve(t, W.rho)
    pd, gd = oracle.direct_sum(t, W.rho)
    # measured: phi 2.2e-3, g 1.3e-2 (order-3 expansions at the 1074 stencil)
    assert rel(phi, pd) < 3e-3
    assert max(rel(g[:, a], gd[:, a]) for a in range(3)) < 2e-2
    # the same-level-only (no downward pass) answer is far worse: step 3 matters
    f, tq = momentum_residuals(t, W.rho, g)
    assert f < 1e-13


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_amr_conservation_with_and_without_correction(seed):
    W = wl.small_amr(seed)
    t = W.trees[0]
    phi, g, st = oracle.solve(t, W.rho, with_stats=True)
    assert all(c > 0 for c in st["cls"])          # all four classes occur
    assert st["cls"][0] == st["cls"][3]             # class 1 and 4 pair up
    f, tq = momentum_residuals(t, W.rho, g)
    assert f < 1e-13 and tq < 1e-13
    phi0, g0 = oracle.solve(t, W.rho, correction=False)
    f0, tq0 = momentum_residuals(t, W.rho, g0)
    assert f0 < 1e-13 and tq0 > 1e-7                 # negative control
    pd, gd = oracle.direct_sum(t, W.rho)
    assert rel(phi, pd) < 2e-3


def test_c0_all_targets_symmetric_set_conserves():
    W = wl.c0(1)
    t = W.trees[0]
    phi, g = oracle.solve(t, W.rho, top_all_pairs=False)
    f, tq = momentum_residuals(t, W.rho, g, centre=(0.5, 0.5, 0.5))
    assert f < 1e-13 and tq < 1e-13


def test_mirror_and_permutation_equivariance():
    W = wl.small_amr(3)
    t = W.trees[0]
    phi, g = oracle.solve(t, W.rho)
    n = 2 ** t.level
    # mirror x -> 1 - x: sub-grid s_x -> 2^l - 1 - s_x, cell i -> 7 - i
    cm = t.coord.copy()
    cm[:, 0] = n - 1 - cm[:, 0]
    tm = wl.TreeDesc(t.level.copy(), cm, t.origin, t.L0)
    rho_m = W.rho[:, ::-1, :, :].copy()
    pm, gm = oracle.solve(tm, rho_m)
    P = lambda a: a.reshape(-1, 8, 8, 8)
    assert rel(P(pm)[:, ::-1], P(phi)) < 1e-13
    assert rel(-P(gm[:, 0])[:, ::-1], P(g[:, 0])) < 1e-13
    assert rel(P(gm[:, 1])[:, ::-1], P(g[:, 1])) < 1e-13
    # permutation x <-> y
    cp = t.coord[:, [1, 0, 2]].copy()
    tp = wl.TreeDesc(t.level.copy(), cp, t.origin, t.L0)
    pp, gp = oracle.solve(tp, W.rho.transpose(0, 2, 1, 3).copy())
    assert rel(P(pp).transpose(0, 2, 1, 3), P(phi)) < 1e-13
    assert rel(P(gp[:, 1]).transpose(0, 2, 1, 3), P(g[:, 0])) < 1e-13


def test_uniform_sphere_closed_form():
    """Uniform sphere (volume-fraction weighted cells): phi = -GM(3R^2-r^2)/(2R^3)
    inside, -GM/r outside; the direct sum is checked first so that
    discretisation error is kept apart from expansion error."""
    t = wl.uniform_tree(2)
    x = t.leaf_cell_centres()
    h = t.leaf_cell_size()[0]
    Rs = 0.3
    sub = (np.arange(8) + 0.5) / 8 - 0.5
    frac = np.zeros(x.shape[:-1])
    for ox in sub:
        for oy in sub:
            for oz in sub:
                p = x + h * np.array([ox, oy, oz])
                frac += (((p - 0.5) ** 2).sum(-1) < Rs * Rs)
    rho = frac / 512.0
    M = rho.sum() * h ** 3
    r = np.sqrt(((x - 0.5) ** 2).sum(-1))
    exact = np.where(r < Rs, -M * (3 * Rs ** 2 - r ** 2) / (2 * Rs ** 3), -M / r)
    pd, gd = oracle.direct_sum(t, rho)
    phi, g = oracle.solve(t, rho)
    e_direct = rel(pd.reshape(exact.shape), exact)
    e_fmm = rel(phi.reshape(exact.shape), exact)
    assert e_direct < 1e-2                     # discretisation (self term, O(h) surface)
    assert e_fmm < e_direct + 3e-3            # expansion adds at most its truncation
    assert rel(phi, pd) < 3e-3


def test_sampled_solve_matches_full_solve():
    W = wl.small_amr(1)
    t = W.trees[0]
    phi, g = oracle.solve(t, W.rho)
    rng = np.random.default_rng(0)
    li = rng.integers(0, t.n_leaves, 40).astype(np.int32)
    ci = rng.integers(0, 512, 40).astype(np.int32)
    ps, gs = oracle.solve_sampled(t, W.rho, li, ci)
    assert np.abs(ps - phi[li, ci]).max() < 1e-14 * np.abs(phi).max()
    assert np.abs(gs - g[li, :, ci]).max() < 1e-13 * np.abs(g).max()


def test_thread_count_changes_nothing():
    """Each target cell's sums run in a fixed order on one thread, so the
    solve is bitwise the same on one thread as on all of them (the CPU
    baseline is timed both ways)."""
    W = wl.small_amr(2)
    t = W.trees[0]
    full = oracle.solve(t, W.rho)
    assert oracle.set_threads(1) == 1
    try:
        one = oracle.solve(t, W.rho)
        assert oracle.max_threads() == 1
    finally:
        n = oracle.set_threads(0)
    assert n >= 1 and oracle.max_threads() == n
    assert np.array_equal(one[0], full[0]) and np.array_equal(one[1], full[1])


def test_sampled_direct_sum_matches_full_direct_sum():
    W = wl.small_amr(3)
    t = W.trees[0]
    pd, gd = oracle.direct_sum(t, W.rho)
    rng = np.random.default_rng(1)
    li = rng.integers(0, t.n_leaves, 60).astype(np.int32)
    ci = rng.integers(0, 512, 60).astype(np.int32)
    ps, gs = oracle.direct_sum_sampled(t, W.rho, li, ci)
    assert np.array_equal(ps, pd[li, ci]) and np.array_equal(gs, gd[li, :, ci])
    with pytest.raises(RuntimeError):
        oracle.direct_sum_sampled(t, W.rho, [t.n_leaves], [0])
    with pytest.raises(RuntimeError):
        oracle.direct_sum_sampled(t, W.rho, [0], [512])


def test_c2_fmm_vs_direct_sum_at_sampled_cells():
    """The binary-star AMR field (3,816 leaves over levels 2..5): the order-3
    expansion's error against Newton's sum at 400 sampled leaf cells."""
    W = wl.c2()
    t = W.trees[0]
    rng = np.random.default_rng(5)
    li = rng.integers(0, t.n_leaves, 400).astype(np.int32)
    ci = rng.integers(0, 512, 400).astype(np.int32)
    pf, gf = oracle.solve_sampled(t, W.rho, li, ci)
    pd, gd = oracle.direct_sum_sampled(t, W.rho, li, ci)
    e_phi = np.linalg.norm(pf - pd) / np.linalg.norm(pd)
    e_g = np.linalg.norm(gf - gd) / np.linalg.norm(gd)
    # measured: phi 2.8e-4, g 5.2e-3
    assert e_phi < 1e-3 and e_g < 1e-2
    # without the downward pass the far field is missing: far worse
    assert e_g > 1e-4


def test_c2_truncation_error_interior_and_coarse_fine_boundary_cells():
    """The same field's truncation error reported separately for interior
    leaves (all 26 same-level neighbours are leaves) and coarse-fine boundary
    leaves (a same-level neighbour inside the domain is absent, i.e. coarser,
    or refined): 300 sampled cells each against Newton's sum.  Boundary
    cells, whose near partners across the level change are taken as
    multipoles, carry the larger error."""
    import itertools
    W = wl.c2()
    t = W.trees[0]
    ref = t.refined_mask()
    key = {(int(l), *map(int, c)): i for i, (l, c) in enumerate(zip(t.level, t.coord))}
    bnd = []
    for s in t.leaf_indices():
        lv, c, n = int(t.level[s]), t.coord[s], 1 << int(t.level[s])
        b = False
        for o in itertools.product((-1, 0, 1), repeat=3):
            p = c + np.array(o)
            if o == (0, 0, 0) or (p < 0).any() or (p >= n).any():
                continue
            j = key.get((lv, *map(int, p)))
            b |= j is None or bool(ref[j])
        bnd.append(b)
    bnd = np.array(bnd)
    assert 0 < bnd.sum() < len(bnd)
    rng = np.random.default_rng(11)
    errs = {}
    for name, pool in (("interior", np.nonzero(~bnd)[0]), ("boundary", np.nonzero(bnd)[0])):
        li = rng.choice(pool, 300).astype(np.int32)
        ci = rng.integers(0, 512, 300).astype(np.int32)
        pf, gf = oracle.solve_sampled(t, W.rho, li, ci)
        pd, gd = oracle.direct_sum_sampled(t, W.rho, li, ci)
        errs[name] = (np.linalg.norm(pf - pd) / np.linalg.norm(pd), np.linalg.norm(gf - gd) / np.linalg.norm(gd))
    print(f"  {bnd.sum()} of {len(bnd)} leaves on a coarse-fine boundary; errors {errs}", flush=True)
    # measured: interior phi 6.3e-5, g 1.4e-3; boundary phi 5.6e-4, g 1.0e-2
    assert errs["interior"][0] < 2e-4 and errs["interior"][1] < 4e-3
    assert errs["boundary"][0] < 1.5e-3 and errs["boundary"][1] < 3e-2
    assert errs["boundary"][0] > errs["interior"][0] and errs["boundary"][1] > errs["interior"][1]


@pytest.mark.parametrize("seed,max_level", [(1, 2), (3, 3)])
def test_isolated_point_masses_are_exact_newton(seed, max_level):
    """If every non-leaf cell holds at most one massive leaf cell, each massive
    cell's multipoles about its centre of mass are a bare monopole and every
    downward shift towards a massive cell is by zero: the method then gives
    Newton's field at the massive cells to round-off, through every class and
    level, with or without the correction (whose terms all carry a quadrupole
    or octupole).  A pair counted twice or missed, a wrong sign or G fails
    this at O(1)."""
    t = wl.small_amr(seed, max_level=max_level).trees[0]
    rho = wl.isolated_masses(t, seed)
    sel = rho.reshape(rho.shape[0], 512) > 0
    assert sel.sum() > 250
    phi, g = oracle.solve(t, rho)
    pd, gd = oracle.direct_sum(t, rho)
    gs, gds = g.transpose(0, 2, 1)[sel], gd.transpose(0, 2, 1)[sel]
    assert np.abs(phi[sel] - pd[sel]).max() < 1e-13 * np.abs(pd[sel]).max()
    assert np.abs(gs - gds).max() < 1e-13 * np.abs(gds).max()
    phi0, g0 = oracle.solve(t, rho, correction=False)
    assert np.array_equal(phi0, phi) and np.array_equal(g0, g)
    # the massless cells still carry the truncation error
    assert np.abs(phi[~sel] - pd[~sel]).max() > 1e-4 * np.abs(pd[~sel]).max()


def test_oracle_rejects_malformed_input():
    t = wl.uniform_tree(1)
    rho = np.ones((8, 8, 8, 8))
    bad = wl.TreeDesc(t.level[:-1].copy(), t.coord[:-1].copy(), t.origin, t.L0)  # 7 children
    with pytest.raises(RuntimeError):
        oracle.solve(bad, rho[:7])
    rho2 = rho.copy()
    rho2[0, 0, 0, 0] = -1.0
    with pytest.raises(RuntimeError):
        oracle.solve(t, rho2)
    orphan = wl.TreeDesc(np.array([1], np.int32), np.array([[0, 0, 0]], np.int32), t.origin, t.L0)
    with pytest.raises(RuntimeError):
        oracle.solve(orphan, rho[:1])
