"""Seeded synthetic workloads: octrees of 8x8x8 sub-grids plus leaf-cell densities.

This module only *generates inputs*.  It holds none of the multipole method's
arithmetic, so both the GPU path and the CPU oracle may consume what it makes.

The paper measures on a private binary-star merger state (V1309 Sco, level 14;
Sec. 6, "Results", and the node-level performance table).  That state is not
available, so seeded polytropes stand in for it:

* ``c0``: 27 level-0 leaf sub-grids (a 3x3x3 forest, h = 1/8), lognormal
  densities.  The central sub-grid sees all 26 same-level neighbours, which is
  the per-sub-grid stencil kernel of Sec. 4.3 in isolation.
* ``c1``: a uniform level-3 octree (64^3 leaf cells) holding one n = 1.5
  polytrope of radius 0.3.
* ``c2``: an adaptive octree refined around two n = 1.5 polytropes with mass
  ratio 0.1 and separation 0.4 (binary-star field), +-1 % seeded noise.
* ``c4``: 16 independent binary-star octrees with drawn mass ratios,
  separations and depths (batched form).

Conventions shared with the C-ABI:

* A tree is a list of sub-grids ``(level, sx, sy, sz)``.  A sub-grid at level
  ``l`` covers ``origin + L0 * 2**-l * [s, s+1)``; its cells have size
  ``h = L0 / (8 * 2**l)``.
* A sub-grid is refined iff its 8 children are listed.  Leaf order is the order
  in which leaves appear in the descriptor (concatenated over trees).
* Densities are ``[n_leaf][8][8][8]`` float64 indexed ``[i][j][k]`` (x, y, z)
  with ``k`` fastest.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Sequence

import numpy as np

N_SUB = 8  # cells per sub-grid edge (Sec. 4.2: N = 8 for all runs)


# ----------------------------------------------------------------------------
# data containers
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class TreeDesc:
    level: np.ndarray          # int32 [n]
    coord: np.ndarray          # int32 [n, 3]
    origin: tuple              # (x, y, z) of the level-0 sub-grid (0,0,0) corner
    L0: float                  # edge of a level-0 sub-grid

    @property
    def n_subgrids(self) -> int:
        return int(self.level.shape[0])

    def refined_mask(self) -> np.ndarray:
        lv = self.level.astype(np.int64)
        c = self.coord.astype(np.int64)
        key = (lv << 57) | (c[:, 0] << 38) | (c[:, 1] << 19) | c[:, 2]
        child = ((lv + 1) << 57) | ((2 * c[:, 0]) << 38) | ((2 * c[:, 1]) << 19) | (2 * c[:, 2])
        return np.isin(child, key)

    def leaf_indices(self) -> np.ndarray:
        return np.nonzero(~self.refined_mask())[0].astype(np.int32)

    @property
    def n_leaves(self) -> int:
        return int(self.leaf_indices().shape[0])

    def leaf_cell_centres(self) -> np.ndarray:
        """[n_leaf, 8, 8, 8, 3] centres of the leaf cells, in leaf order."""
        li = self.leaf_indices()
        lev = self.level[li].astype(np.float64)
        h = self.L0 / (N_SUB * 2.0 ** lev)
        ijk = np.arange(N_SUB, dtype=np.float64) + 0.5
        out = np.empty((li.shape[0], N_SUB, N_SUB, N_SUB, 3))
        for a in range(3):
            base = np.asarray(self.origin[a]) + self.coord[li, a] * N_SUB * h
            shape = [1, 1, 1]
            shape[a] = N_SUB
            out[..., a] = base[:, None, None, None] + h[:, None, None, None] * ijk.reshape(shape)
        return out

    def leaf_cell_size(self) -> np.ndarray:
        li = self.leaf_indices()
        return self.L0 / (N_SUB * 2.0 ** self.level[li].astype(np.float64))


@dataclasses.dataclass
class Workload:
    name: str
    trees: List[TreeDesc]
    rho: np.ndarray            # float64 [total_leaves, 8, 8, 8]
    info: dict

    @property
    def n_leaves(self) -> int:
        return int(self.rho.shape[0])


# ----------------------------------------------------------------------------
# Lane-Emden n = 1.5 polytrope (input profile only)
# ----------------------------------------------------------------------------
_LE_CACHE: dict = {}


def lane_emden(n: float = 1.5, dxi: float = 1e-4):
    """Integrate theta'' + 2/xi theta' + theta^n = 0 with classical RK4.

    Returns (xi, theta, xi1, w) where xi1 is the first zero of theta and
    w = xi1^2 |theta'(xi1)| (the mass integral).
    """
    key = (n, dxi)
    if key in _LE_CACHE:
        return _LE_CACHE[key]
    # series start away from the removable singularity at xi = 0
    xi = dxi
    th = 1.0 - xi * xi / 6.0 + n * xi ** 4 / 120.0
    dth = -xi / 3.0 + n * xi ** 3 / 30.0

    def f(x, y, z):
        return z, -(max(y, 0.0) ** n) - 2.0 * z / x

    xs = [0.0, xi]
    ths = [1.0, th]
    while th > 0.0:
        k1y, k1z = f(xi, th, dth)
        k2y, k2z = f(xi + dxi / 2, th + dxi / 2 * k1y, dth + dxi / 2 * k1z)
        k3y, k3z = f(xi + dxi / 2, th + dxi / 2 * k2y, dth + dxi / 2 * k2z)
        k4y, k4z = f(xi + dxi, th + dxi * k3y, dth + dxi * k3z)
        th_new = th + dxi / 6 * (k1y + 2 * k2y + 2 * k3y + k4y)
        dth_new = dth + dxi / 6 * (k1z + 2 * k2z + 2 * k3z + k4z)
        if th_new <= 0.0:
            # linear root between the last two steps
            frac = th / (th - th_new)
            xi1 = xi + frac * dxi
            dth1 = dth + frac * (dth_new - dth)
            xs.append(xi1)
            ths.append(0.0)
            xi, th, dth = xi1, 0.0, dth1
            break
        xi += dxi
        th, dth = th_new, dth_new
        xs.append(xi)
        ths.append(th)
    xs = np.asarray(xs)
    ths = np.asarray(ths)
    out = (xs, ths, float(xi), float(xi * xi * abs(dth)))
    _LE_CACHE[key] = out
    return out


def polytrope(points: np.ndarray, centre, radius: float, rho_c: float) -> np.ndarray:
    """Density of an n = 1.5 polytrope at ``points`` [..., 3]; zero outside.
    theta is interpolated linearly on the uniform RK4 grid."""
    xs, ths, xi1, _ = lane_emden()
    d = points - np.asarray(centre)
    xi = np.sqrt((d * d).sum(-1)) * (xi1 / radius)
    step = xs[2] - xs[1]
    u = xi / step
    i = np.minimum(u.astype(np.int64), xs.shape[0] - 2)
    f = np.clip(u - i, 0.0, 1.0)
    th = ths[i] * (1.0 - f) + ths[i + 1] * f
    th = np.where(xi < xi1, np.maximum(th, 0.0), 0.0)
    return rho_c * th * np.sqrt(th)


def polytrope_rho_c(mass: float, radius: float) -> float:
    """Central density of an n = 1.5 polytrope of given mass and radius."""
    _, _, xi1, w = lane_emden()
    return mass * xi1 ** 3 / (4.0 * math.pi * radius ** 3 * w)


# ----------------------------------------------------------------------------
# tree builders
# ----------------------------------------------------------------------------
def _desc_from_list(subs: Sequence[tuple], origin, L0) -> TreeDesc:
    arr = np.asarray(subs, dtype=np.int32).reshape(-1, 4)
    return TreeDesc(level=np.ascontiguousarray(arr[:, 0]),
                    coord=np.ascontiguousarray(arr[:, 1:4]),
                    origin=tuple(float(o) for o in origin), L0=float(L0))


def uniform_tree(max_level: int, origin=(0.0, 0.0, 0.0), L0: float = 1.0) -> TreeDesc:
    """Complete octree of sub-grids at levels 0..max_level (level by level)."""
    subs = []
    for l in range(max_level + 1):
        n = 2 ** l
        for x in range(n):
            for y in range(n):
                for z in range(n):
                    subs.append((l, x, y, z))
    return _desc_from_list(subs, origin, L0)


def forest_tree(n: int = 3, origin=(-1.0, -1.0, -1.0), L0: float = 1.0) -> TreeDesc:
    """n^3 level-0 leaf sub-grids (a forest with no parents)."""
    subs = [(0, x, y, z) for x in range(n) for y in range(n) for z in range(n)]
    return _desc_from_list(subs, origin, L0)


def _subgrid_cell_centres(level: int, coord, origin, L0) -> np.ndarray:
    h = L0 / (N_SUB * 2.0 ** level)
    ijk = np.arange(N_SUB) + 0.5
    base = np.asarray(origin) + np.asarray(coord) * N_SUB * h
    g = np.stack(np.meshgrid(ijk, ijk, ijk, indexing="ij"), -1)
    return base + h * g


def adaptive_tree(density: Callable[[np.ndarray], np.ndarray], max_level: int,
                  threshold: float, origin=(0.0, 0.0, 0.0), L0: float = 1.0) -> TreeDesc:
    """Refine from a single root: a sub-grid below ``max_level`` is refined iff
    the maximum of ``density`` over its own cell centres exceeds ``threshold``.
    Sub-grids are listed level by level (breadth first, sorted coordinates)."""
    subs = [(0, 0, 0, 0)]
    frontier = np.zeros((1, 3), dtype=np.int64)
    ijk = np.arange(N_SUB) + 0.5
    local = np.stack(np.meshgrid(ijk, ijk, ijk, indexing="ij"), -1).reshape(-1, 3)
    e = np.array([(x, y, z) for x in (0, 1) for y in (0, 1) for z in (0, 1)], dtype=np.int64)
    for l in range(max_level):
        if frontier.shape[0] == 0:
            break
        h = L0 / (N_SUB * 2.0 ** l)
        refine = np.zeros(frontier.shape[0], dtype=bool)
        for b0 in range(0, frontier.shape[0], 4096):
            fb = frontier[b0:b0 + 4096]
            pts = np.asarray(origin) + (fb[:, None, :] * N_SUB + local[None]) * h
            refine[b0:b0 + 4096] = density(pts).max(axis=1) > threshold
        kids = (2 * frontier[refine][:, None, :] + e[None]).reshape(-1, 3)
        order = np.lexsort((kids[:, 2], kids[:, 1], kids[:, 0]))
        kids = kids[order]
        subs.extend((l + 1, int(c[0]), int(c[1]), int(c[2])) for c in kids)
        frontier = kids
    return _desc_from_list(subs, origin, L0)


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------
def c0(seed: int = 0) -> Workload:
    """27 level-0 leaf sub-grids (24^3 cells, h = 1/8), lognormal(0, 1) densities."""
    tree = forest_tree(3)
    rng = np.random.default_rng(seed)
    block = rng.lognormal(0.0, 1.0, (24, 24, 24))
    rho = np.empty((27, 8, 8, 8))
    for i, (sx, sy, sz) in enumerate(tree.coord):
        rho[i] = block[8 * sx:8 * sx + 8, 8 * sy:8 * sy + 8, 8 * sz:8 * sz + 8]
    return Workload("c0", [tree], rho, {"seed": seed, "central_leaf": 13})


def c1(max_level: int = 3, radius: float = 0.3, floor: float = 1e-10) -> Workload:
    """Uniform octree to ``max_level`` (default 3: 64^3 leaf cells) with one
    centred n = 1.5 polytrope (rho_c = 1) plus an additive floor."""
    tree = uniform_tree(max_level)
    x = tree.leaf_cell_centres()
    rho = polytrope(x, (0.5, 0.5, 0.5), radius, 1.0) + floor
    return Workload(f"c1_l{max_level}", [tree], np.ascontiguousarray(rho),
                    {"max_level": max_level, "radius": radius})


def _binary_fields(q: float, a: float, r1: float, r2: float):
    m1, m2 = 1.0, q
    x1 = 0.5 - a * m2 / (m1 + m2)
    x2 = 0.5 + a * m1 / (m1 + m2)
    rc1 = polytrope_rho_c(m1, r1)
    rc2 = polytrope_rho_c(m2, r2)

    def dens(p):
        return (polytrope(p, (x1, 0.5, 0.5), r1, rc1) +
                polytrope(p, (x2, 0.5, 0.5), r2, rc2))
    return dens, max(rc1, rc2), (x1, x2)


def binary_tree(q: float, a: float, r1: float, r2: float, max_level: int,
                refine_frac: float = 1e-4):
    dens, rmax, _ = _binary_fields(q, a, r1, r2)
    return adaptive_tree(dens, max_level, refine_frac * rmax), dens, rmax


def binary_density(tree: TreeDesc, dens, rmax: float, rng: np.random.Generator,
                   noise: float = 0.01, floor_frac: float = 1e-10) -> np.ndarray:
    x = tree.leaf_cell_centres()
    u = rng.uniform(-1.0, 1.0, size=x.shape[:-1])
    return np.ascontiguousarray(dens(x) * (1.0 + noise * u) + floor_frac * rmax)


def binary_star(q: float, a: float, r1: float, r2: float, max_level: int,
                rng: np.random.Generator, noise: float = 0.01,
                refine_frac: float = 1e-4, floor_frac: float = 1e-10):
    tree, dens, rmax = binary_tree(q, a, r1, r2, max_level, refine_frac)
    return tree, binary_density(tree, dens, rmax, rng, noise, floor_frac)


def c2(seed: int = 2, max_level: int = 5, r1: float = 0.25, r2: float = 0.10) -> Workload:
    """Binary-star AMR field: mass ratio 0.1, separation 0.4 along x."""
    rng = np.random.default_rng(seed)
    tree, rho = binary_star(0.1, 0.4, r1, r2, max_level, rng)
    return Workload("c2", [tree], rho, {"seed": seed, "q": 0.1, "a": 0.4,
                                        "r1": r1, "r2": r2, "max_level": max_level})


def eggleton(q: float) -> float:
    """Roche-lobe radius over separation for mass ratio q (Eggleton 1983)."""
    q23 = q ** (2.0 / 3.0)
    return 0.49 * q23 / (0.6 * q23 + math.log(1.0 + q ** (1.0 / 3.0)))


def c4_tree(t: int, base_seed: int = 4, lo: int = 500, hi: int = 8000):
    """One binary-star tree of the batch; parameters are redrawn until the tree
    has lo <= leaves <= hi, then the noise is drawn."""
    rng = np.random.default_rng(base_seed * 1000 + t)
    while True:
        q = float(rng.uniform(0.05, 0.5))
        a = float(rng.uniform(0.3, 0.6))
        r1 = 1.1 * a * eggleton(1.0 / q)
        r2 = 1.1 * a * eggleton(q)
        span = a + r1 + r2
        if span > 0.94:
            s = (0.94 - a) / (r1 + r2)
            r1 *= s
            r2 *= s
        max_level = int(rng.integers(4, 7))
        tree, dens, rmax = binary_tree(q, a, r1, r2, max_level)
        if lo <= tree.n_leaves <= hi:
            rho = binary_density(tree, dens, rmax, rng)
            return tree, rho, dict(q=q, a=a, r1=r1, r2=r2, max_level=max_level)


def c4(n_trees: int = 16, base_seed: int = 4) -> Workload:
    trees, rhos, infos = [], [], []
    for t in range(n_trees):
        tree, rho, info = c4_tree(t, base_seed)
        trees.append(tree)
        rhos.append(rho)
        infos.append(info)
    return Workload("c4", trees, np.ascontiguousarray(np.concatenate(rhos)),
                    {"trees": infos, "base_seed": base_seed})


def small_amr(seed: int, max_level: int = 2, p_refine: float = 0.4) -> Workload:
    """Random small AMR tree (root refined, then each sub-grid refined with
    probability p_refine) with lognormal densities; for brute-force checks."""
    rng = np.random.default_rng(seed)
    subs = [(0, 0, 0, 0)]
    frontier = [(0, (0, 0, 0))]
    while frontier:
        nxt = []
        for (l, c) in frontier:
            if l >= max_level:
                continue
            if l == 0 or rng.uniform() < p_refine:
                for ex in (0, 1):
                    for ey in (0, 1):
                        for ez in (0, 1):
                            nxt.append((l + 1, (2 * c[0] + ex, 2 * c[1] + ey, 2 * c[2] + ez)))
        nxt.sort()
        subs.extend((l, *c) for (l, c) in nxt)
        frontier = nxt
    tree = _desc_from_list(subs, (0.0, 0.0, 0.0), 1.0)
    rho = rng.lognormal(0.0, 1.0, (tree.n_leaves, 8, 8, 8))
    return Workload(f"amr{seed}", [tree], rho, {"seed": seed})


CONFIGS = {"c0": c0, "c1": c1, "c2": c2, "c4": c4}


def isolated_masses(tree: TreeDesc, seed: int, fill: float = 0.6) -> np.ndarray:
    """Densities that are zero except in single leaf cells, at most one per
    cell of the level-0 sub-grid (so every non-leaf cell holds at most one
    massive leaf cell below it): a random ``fill`` fraction of the level-0
    cells gets one, at a random leaf cell inside it, with a lognormal
    density.  Needs a refined root."""
    if tree.level.shape[0] < 2:
        raise ValueError("isolated_masses needs a refined root sub-grid")
    rng = np.random.default_rng(seed)
    x = tree.leaf_cell_centres().reshape(-1, 3)
    root = np.floor((x - np.asarray(tree.origin)) / (tree.L0 / N_SUB)).astype(np.int64)
    key = (root[:, 0] * N_SUB + root[:, 1]) * N_SUB + root[:, 2]
    rho = np.zeros(x.shape[0])
    for k in np.unique(key):
        if rng.uniform() < fill:
            cells = np.nonzero(key == k)[0]
            rho[cells[rng.integers(cells.shape[0])]] = rng.lognormal(0.0, 1.0)
    return rho.reshape(-1, N_SUB, N_SUB, N_SUB)
