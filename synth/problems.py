"""Seeded synthetic problem instances: meshes, element densities, supports, loads.

This module is the single source of inputs for both the CPU oracle and the GPU
path.  It holds none of the solver's arithmetic (no stiffness, no SIMP law, no
multigrid): it only draws densities and lists which degrees of freedom are
supported and loaded, following the test domains of the paper (cantilever,
MBB half-beam, 3D cantilever, a thin-strut lattice standing in for the spaced
grid / bridge domains).  The paper's problems are produced by an optimiser we
do not run, so their density fields are replaced by seeded random fields of the
same shape and contrast.

Numbering conventions shared by every consumer:
  * node (i, j[, k]) has id  i + (nx+1) * (j + (ny+1) * k)
  * dof  = dim * node + component   (components interleaved)
  * element (ex, ey[, ez]) has id  ex + nx * (ey + ny * ez)
so a C-ordered numpy array indexed [ez, ey, ex] flattens to element order.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np
from scipy.ndimage import gaussian_filter, label

VOID = 1e-3


@dataclass
class Problem:
    name: str
    dim: int
    nel: Tuple[int, ...]            # elements per axis (x, y[, z])
    rho: np.ndarray                 # element densities, float64, element order
    fixed: np.ndarray               # constrained dof ids, int64, sorted, unique
    loads: np.ndarray               # (n_rhs, n_dof) float64
    p: float = 3.0
    E0: float = 1.0
    Emin: float = 1e-9
    nu: float = 0.3
    h: float = 1.0
    opts: Dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(np.prod([n + 1 for n in self.nel]))

    @property
    def n_dof(self) -> int:
        return self.dim * self.n_nodes

    @property
    def n_el(self) -> int:
        return int(np.prod(self.nel))


# --------------------------------------------------------------------------- ids
def node_id(nel, *ijk) -> np.ndarray:
    nx1 = nel[0] + 1
    ny1 = nel[1] + 1
    i = np.asarray(ijk[0], dtype=np.int64)
    j = np.asarray(ijk[1], dtype=np.int64)
    k = np.asarray(ijk[2], dtype=np.int64) if len(ijk) > 2 else 0
    return i + nx1 * (j + ny1 * k)


def _dofs(nel, dim, nodes, comps) -> np.ndarray:
    nodes = np.atleast_1d(np.asarray(nodes, dtype=np.int64))
    comps = np.atleast_1d(np.asarray(comps, dtype=np.int64))
    return (dim * nodes[:, None] + comps[None, :]).ravel()


def _uniq(a) -> np.ndarray:
    return np.unique(np.asarray(a, dtype=np.int64))


# ----------------------------------------------------------------- density fields
def smoothed_field(shape_zyx, seed: int, sigma: float = 4.0) -> np.ndarray:
    """Gaussian-smoothed i.i.d. N(0,1) noise on the element grid (reflecting edges)."""
    g = np.random.default_rng(seed).standard_normal(shape_zyx)
    return gaussian_filter(g, sigma=sigma, mode="reflect", truncate=4.0)


def minmax_density(field: np.ndarray, lo: float = VOID) -> np.ndarray:
    f = (field - field.min()) / (field.max() - field.min())
    return lo + (1.0 - lo) * f


def threshold_density(field: np.ndarray, lo: float = VOID) -> np.ndarray:
    return np.where(field >= 0.0, 1.0, lo)


def _zyx(nel):
    return tuple(reversed(nel))


def solid_ball(rho_zyx: np.ndarray, center_xyz, radius: float) -> None:
    """Set elements whose centre lies within `radius` of a point to solid (in place)."""
    grids = np.meshgrid(*[np.arange(s) + 0.5 for s in rho_zyx.shape], indexing="ij")
    c = list(reversed(center_xyz))
    d2 = sum((g - cc) ** 2 for g, cc in zip(grids, c))
    rho_zyx[d2 <= radius * radius] = 1.0


# ------------------------------------------------------------- supports / loads
def clamp_x0(nel, dim) -> np.ndarray:
    """All dofs of every node on the face x = 0."""
    ranges = [np.arange(n + 1) for n in nel[1:]]
    grid = np.meshgrid(*ranges, indexing="ij")
    nodes = node_id(nel, 0, *[g.ravel() for g in grid])
    return _uniq(_dofs(nel, dim, nodes, range(dim)))


def edge_line_load(nel, y_node: int, total: float = -1.0) -> np.ndarray:
    """3D: total force in -y spread over the nodes (nx, y_node, k), k = 0..nz,
    with trapezoid weights (end nodes carry half)."""
    nx, ny, nz = nel
    f = np.zeros(3 * np.prod([n + 1 for n in nel]))
    k = np.arange(nz + 1)
    w = np.full(nz + 1, 1.0 / nz)
    w[0] = w[-1] = 0.5 / nz
    nodes = node_id(nel, nx, y_node, k)
    f[3 * nodes + 1] = total * w
    return f


# ------------------------------------------------------------------- problems
def mbb_2d(uniform: bool = True, seed: int = 1, nel=(60, 20)) -> Problem:
    """MBB half-beam: x-symmetry on the left edge, roller at the bottom-right
    node, unit downward point load at the top-left node."""
    nx, ny = nel
    n_dof = 2 * (nx + 1) * (ny + 1)
    left = node_id(nel, 0, np.arange(ny + 1))
    fixed = _uniq(np.concatenate([2 * left, [2 * node_id(nel, nx, 0) + 1]]))
    f = np.zeros((1, n_dof))
    f[0, 2 * node_id(nel, 0, ny) + 1] = -1.0
    if uniform:
        rho = np.full(nx * ny, 0.5)
    else:
        rho = np.random.default_rng(seed).uniform(0.0, 1.0, size=nx * ny)
    return Problem("mbb", 2, (nx, ny), rho, fixed, f, p=3.0, E0=1.0, Emin=1e-9, nu=0.3,
                   opts=dict(n_levels=3, omega=0.6, nu_pre=2, nu_post=2, rtol=1e-8))


def cantilever_2d(nel=(1024, 512), seed: int = 2, n_levels: int = 7, chord: float = 0.06) -> Problem:
    """2D cantilever: left edge clamped, unit downward load at the middle of the
    right edge.  Density: smoothed noise thresholded at 0 to {1e-3, 1}, joined
    to solid top and bottom chords and a solid right-edge band (each `chord` of
    the height thick, so the load sits on material), after which every solid
    piece not connected through element edges to the clamped edge is set to
    void: like an optimised design, no material floats in the void."""
    nx, ny = nel
    solid = smoothed_field(_zyx(nel), seed) >= 0.0
    c = max(1, int(round(chord * ny)))
    solid[:c, :] = True
    solid[ny - c:, :] = True
    solid[:, nx - c:] = True
    lab, _ = label(solid)
    anchored = np.unique(lab[:, 0])
    solid = np.isin(lab, anchored[anchored > 0])
    rho = np.where(solid, 1.0, VOID)
    f = np.zeros((1, 2 * (nx + 1) * (ny + 1)))
    f[0, 2 * node_id(nel, nx, ny // 2) + 1] = -1.0
    return Problem("cantilever2d", 2, (nx, ny), rho.ravel(), clamp_x0(nel, 2), f,
                   opts=dict(n_levels=n_levels, omega=0.5, nu_pre=1, nu_post=1, rtol=1e-8))


def cantilever_3d(nel=(192, 96, 96), seed: int = 3, n_levels: int = 6) -> Problem:
    """3D cantilever (2:1:1): face x = 0 clamped, total unit downward load along
    the bottom edge (y = 0) of the opposite face.  Density: smoothed noise
    rescaled to [1e-3, 1]."""
    rho = minmax_density(smoothed_field(_zyx(nel), seed))
    f = edge_line_load(nel, 0)[None, :]
    return Problem("cantilever3d", 3, tuple(nel), rho.ravel(), clamp_x0(nel, 3), f,
                   opts=dict(n_levels=n_levels, omega=0.5, nu_pre=1, nu_post=1, rtol=1e-8))


def _strut_positions(rng, n: int, lo: int = 8, hi: int = 24) -> Tuple[List[int], List[int]]:
    """Positions 0, then cumulative spacings drawn from U{lo..hi}, always ending
    with a strut flush with the far edge; each strut 1 or 2 elements wide."""
    pos = [0]
    p = 0
    while True:
        p += int(rng.integers(lo, hi + 1))
        if p > n - 2 - lo // 2:
            break
        pos.append(p)
    widths = [int(w) for w in rng.integers(1, 3, size=len(pos) + 1)]
    pos.append(n - widths[-1])
    return pos, widths


def strut_lattice(nel, seed: int = 4, deck: float = 0.05) -> np.ndarray:
    """Axis-aligned lattice of 1-2 element struts at rho = 1 in rho = 1e-3 void,
    with a solid deck over the top `deck` fraction of the height (y is up).
    Returns densities in [ez, ey, ex] layout."""
    nx, ny, nz = nel
    rng = np.random.default_rng(seed)
    px, wx = _strut_positions(rng, nx)
    py, wy = _strut_positions(rng, ny)
    pz, wz = _strut_positions(rng, nz)
    mx = np.zeros(nx, bool)
    my = np.zeros(ny, bool)
    mz = np.zeros(nz, bool)
    for p, w in zip(px, wx):
        mx[p:p + w] = True
    for p, w in zip(py, wy):
        my[p:p + w] = True
    for p, w in zip(pz, wz):
        mz[p:p + w] = True
    Z, Y, X = np.meshgrid(mz, my, mx, indexing="ij")
    # an element is solid if it lies on a strut along some axis: two of its
    # three coordinates fall on strut positions
    solid = (Y & Z) | (X & Z) | (X & Y)
    top = ny - int(np.ceil(deck * ny))
    solid[:, top:, :] = True
    return np.where(solid, 1.0, VOID)


def bridge_3d(nel=(256, 128, 128), seed: int = 4) -> Problem:
    """3D bridge: the four bottom corner nodes pinned (all dofs), uniform unit
    downward pressure on the top face y = ny as consistent bilinear nodal
    forces, thin-strut lattice density."""
    nx, ny, nz = nel
    corners = node_id(nel, np.array([0, nx, 0, nx]), 0, np.array([0, 0, nz, nz]))
    fixed = _uniq(_dofs(nel, 3, corners, range(3)))
    wx = np.ones(nx + 1)
    wx[[0, -1]] = 0.5
    wz = np.ones(nz + 1)
    wz[[0, -1]] = 0.5
    W = np.outer(wz, wx) / (nx * nz)            # [k, i], sums to 1
    K, I = np.meshgrid(np.arange(nz + 1), np.arange(nx + 1), indexing="ij")
    nodes = node_id(nel, I.ravel(), ny, K.ravel())
    f = np.zeros((1, 3 * (nx + 1) * (ny + 1) * (nz + 1)))
    f[0, 3 * nodes + 1] = -W.ravel()
    rho = strut_lattice(nel, seed)
    return Problem("bridge3d", 3, tuple(nel), rho.ravel(), fixed, f,
                   opts=dict(n_levels=0, n_geometric=3, max_coarse=1000, omega=0.5,
                             nu_pre=1, nu_post=1, rtol=1e-8))


# -------------------------------------------------------------- served stream
SERVED_SIZES = [(2, (128, 64)), (2, (512, 256)), (3, (48, 48, 48)), (3, (96, 48, 48))]


def served_loads(nel, dim, n_rhs: int) -> np.ndarray:
    """Load case k (1..n_rhs): unit downward point (2D) or line (3D) load on the
    far face x = nx at height round(ny * k / (n_rhs + 1))."""
    n_dof = dim * int(np.prod([n + 1 for n in nel]))
    F = np.zeros((n_rhs, n_dof))
    for k in range(1, n_rhs + 1):
        y = int(round(nel[1] * k / (n_rhs + 1)))
        if dim == 2:
            F[k - 1, 2 * node_id(nel, nel[0], y) + 1] = -1.0
        else:
            F[k - 1] = edge_line_load(nel, y)
    return F


def served_request(rid: int, base_seed: int = 5) -> Problem:
    rng = np.random.default_rng([base_seed, rid])
    dim, nel = SERVED_SIZES[int(rng.integers(len(SERVED_SIZES)))]
    n_rhs = int(rng.integers(1, 5))
    rho = minmax_density(smoothed_field(_zyx(nel), base_seed + rid))
    return Problem(f"served{rid}", dim, nel, rho.ravel(), clamp_x0(nel, dim),
                   served_loads(nel, dim, n_rhs),
                   opts=dict(n_levels=0, max_coarse=1000, omega=0.5, nu_pre=1, nu_post=1,
                             rtol=1e-6))


def density_update(rho: np.ndarray, nel, seed: int, step: int, amp: float = 0.05) -> np.ndarray:
    """One synthetic design update: rho + amp * smoothed noise, clipped to [1e-3, 1]."""
    g = smoothed_field(_zyx(nel), seed * 1000003 + step)
    return np.clip(rho + amp * g.ravel(), VOID, 1.0)


def design_sequence(rho0: np.ndarray, nel, seed: int, amp: float = 0.05):
    """Callable t -> densities of design t: rho0, then successive seeded updates."""
    cache = [np.asarray(rho0, dtype=np.float64)]

    def densities(t: int) -> np.ndarray:
        while len(cache) <= t:
            cache.append(density_update(cache[-1], nel, seed=seed, step=len(cache), amp=amp))
        return cache[t]

    return densities


def poisson_arrivals(n: int, rate_per_s: float, seed: int = 5) -> np.ndarray:
    """Arrival times (s) of n requests of a Poisson process."""
    rng = np.random.default_rng([seed, 999])
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


# ------------------------------------------------------------- test vectors
def seeded_vector(n: int, seed: int, fixed=None) -> np.ndarray:
    """n standard-normal values from default_rng(seed), zero on the `fixed`
    dofs if given: the input vectors of the sampled parity cases."""
    v = np.random.default_rng(seed).standard_normal(n)
    if fixed is not None:
        v[np.asarray(fixed, dtype=np.int64)] = 0.0
    return v


# ------------------------------------------------------------- small cases
def small_case(dim: int, nel, seed: int = 11, contrast: bool = True,
               support: str = "clamp", n_rhs: int = 1) -> Problem:
    """Small seeded case for parity tests: clamped (or corner-pinned) domain,
    smoothed density in [1e-3, 1] (or uniform 1), n_rhs far-face loads."""
    if contrast:
        rho = minmax_density(smoothed_field(_zyx(nel), seed, sigma=1.5)).ravel()
    else:
        rho = np.ones(int(np.prod(nel)))
    if support == "clamp":
        fixed = clamp_x0(nel, dim)
    else:
        if dim == 2:
            fixed = _uniq([2 * node_id(nel, 0, 0), 2 * node_id(nel, 0, 0) + 1,
                           2 * node_id(nel, nel[0], 0) + 1])
        else:
            c = node_id(nel, np.array([0, nel[0], 0, nel[0]]), 0,
                        np.array([0, 0, nel[2], nel[2]]))
            fixed = _uniq(_dofs(nel, 3, c, range(3)))
    F = served_loads(nel, dim, n_rhs)
    return Problem(f"small{dim}d", dim, tuple(nel), rho, fixed, F)


def grid_2d(sx: int = 16, sy: int = 256, nel=(520, 520), width: int = 8) -> Problem:
    """2D varying-spaced grid (Sec. 4.3): a square of nel elements, all dofs of
    the bottom nodes fixed, a uniform downward load of total 1 on the top edge
    (consistent nodal forces, end nodes half), density 1 in beams and columns
    `width` elements wide and VOID elsewhere.  Columns start at x = 0, sx, 2 sx,
    ... with one flush with the right edge; beams end at the top edge and repeat
    every sy elements downwards.  No random numbers are involved."""
    nx, ny = nel
    rho = np.full((ny, nx), VOID)
    for x0 in list(range(0, nx - width + 1, sx)) + [nx - width]:
        rho[:, x0:x0 + width] = 1.0
    for y1 in range(ny, width - 1, -sy):
        rho[y1 - width:y1, :] = 1.0
    bottom = node_id(nel, np.arange(nx + 1), 0)
    fixed = _uniq(_dofs(nel, 2, bottom, range(2)))
    w = np.full(nx + 1, 1.0 / nx)
    w[[0, -1]] *= 0.5
    F = np.zeros((1, 2 * (nx + 1) * (ny + 1)))
    F[0, 2 * node_id(nel, np.arange(nx + 1), ny) + 1] = -w
    return Problem(f"grid2d_{sx}_{sy}", 2, tuple(nel), rho.ravel(), fixed, F)


def column_2d(nel=(256, 1024), seed: int = 6, flange: float = 0.125, band: float = 0.02,
              uniform: bool = False) -> Problem:
    """2D column for the stability problem (Sec. 2, Sec. 4 column example):
    all dofs of the bottom nodes fixed, a uniform downward (compressive) load
    of total 1 on the top edge (consistent nodal forces, end nodes half).
    Density: two solid flanges (`flange` of the width each) and solid bottom
    and top bands (`band` of the height) joined by a web of smoothed noise
    thresholded to {1e-3, 1}; web pieces not connected to the bottom are void.
    `uniform` gives density 1 everywhere (a prismatic column)."""
    nx, ny = nel
    if uniform:
        rho = np.ones((ny, nx))
    else:
        solid = smoothed_field(_zyx(nel), seed) >= 0.0
        f = max(1, int(round(flange * nx)))
        b = max(1, int(round(band * ny)))
        solid[:, :f] = True
        solid[:, nx - f:] = True
        solid[:b, :] = True
        solid[ny - b:, :] = True
        lab, _ = label(solid)
        anchored = np.unique(lab[0, :])
        solid = np.isin(lab, anchored[anchored > 0])
        rho = np.where(solid, 1.0, VOID)
    bottom = node_id(nel, np.arange(nx + 1), 0)
    fixed = _uniq(_dofs(nel, 2, bottom, range(2)))
    w = np.full(nx + 1, 1.0 / nx)
    w[[0, -1]] *= 0.5
    F = np.zeros((1, 2 * (nx + 1) * (ny + 1)))
    F[0, 2 * node_id(nel, np.arange(nx + 1), ny) + 1] = -w
    return Problem("column2d", 2, tuple(nel), rho.ravel(), fixed, F,
                   opts=dict(n_levels=5, omega=0.5, nu_pre=1, nu_post=1, rtol=1e-8))


CONFIGS = {
    "mbb_uniform": lambda: mbb_2d(True),
    "mbb_random": lambda: mbb_2d(False),
    "mbb_random": lambda: mbb_2d(False),
    "cantilever2d": cantilever_2d,
    "cantilever3d": cantilever_3d,
    "bridge3d": bridge_3d,
    "grid2d": grid_2d,
    "column2d": column_2d,
}


def get(name: str) -> Problem:
    return CONFIGS[name]()
