"""Oracle, part 5: the linear density filter (CPU, FP64).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Sec. 2 writes the filtered densities as rho = S alpha with a filtering matrix
S (the linear density filter it cites); Sec. 4 sets the radius to 1.5 element
sizes.  Definition used here: element centres c_e on the unit grid,
H[e, i] = max(0, r - |c_e - c_i|) over all pairs of elements of the grid, and
S = diag(1 / sum_i H[e, i]) H, so every row of S sums to one.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def element_centres(nel) -> np.ndarray:
    """(n_el, dim) centres in element order, x fastest."""
    axes = [np.arange(n) + 0.5 for n in nel]
    grids = np.meshgrid(*axes[::-1], indexing="ij")       # slowest axis first
    return np.stack([g.ravel() for g in grids[::-1]], axis=1)


def cone_weights(nel, r: float) -> sp.csr_matrix:
    """H with H[e, i] = max(0, r - |c_e - c_i|), by offsets up to ceil(r) - 1."""
    dim = len(nel)
    c = element_centres(nel)
    n = c.shape[0]
    idx = np.arange(n).reshape(nel[::-1])                  # [z][y][x] or [y][x]
    R = int(np.ceil(r)) - 1
    rows, cols, vals = [], [], []
    rng = range(-R, R + 1)
    offsets = [(dx, dy, dz) for dz in (rng if dim == 3 else [0]) for dy in rng for dx in rng]
    for dx, dy, dz in offsets:
        h = r - np.sqrt(dx * dx + dy * dy + dz * dz)
        if h <= 0:
            continue
        src = idx
        # pairs (e, e + offset) that both lie in the grid
        sl_e, sl_i = [], []
        for d, n_ax in zip((dz, dy, dx)[-dim:] if dim == 3 else (dy, dx), nel[::-1]):
            sl_e.append(slice(max(0, -d), n_ax - max(0, d)))
            sl_i.append(slice(max(0, d), n_ax - max(0, -d)))
        e = src[tuple(sl_e)].ravel()
        i = src[tuple(sl_i)].ravel()
        rows.append(e)
        cols.append(i)
        vals.append(np.full(e.size, h))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def filter_matrix(nel, r: float) -> sp.csr_matrix:
    """S = diag(1 / row sums of H) H."""
    H = cone_weights(nel, r)
    w = np.asarray(H.sum(axis=1)).ravel()
    return sp.diags(1.0 / w) @ H


def apply(nel, r: float, x: np.ndarray, transpose: bool = False) -> np.ndarray:
    S = filter_matrix(nel, r)
    return (S.T @ x) if transpose else (S @ x)


def apply_rows(nel, r: float, x: np.ndarray, rows, transpose: bool = False) -> np.ndarray:
    """Selected entries of S x (or S^T x), each from the definition alone:
    for S x, out_e = sum_i H[e, i] x_i / sum_i H[e, i]; for S^T x,
    out_i = sum_e H[e, i] x_e / sum_j H[e, j] (H is symmetric).  For spot checks
    on grids too large for the whole matrix."""
    dim = len(nel)
    R = int(np.ceil(r)) - 1
    rng = range(-R, R + 1)
    offs = [(dx, dy, dz) for dz in (rng if dim == 3 else [0]) for dy in rng for dx in rng]

    def coords(e):
        i = e % nel[0]
        j = (e // nel[0]) % nel[1]
        k = e // (nel[0] * nel[1]) if dim == 3 else 0
        return i, j, k

    def index(i, j, k):
        return (k * nel[1] + j) * nel[0] + i if dim == 3 else j * nel[0] + i

    def neighbours(e):
        i, j, k = coords(e)
        for dx, dy, dz in offs:
            h = r - np.sqrt(dx * dx + dy * dy + dz * dz)
            ii, jj, kk = i + dx, j + dy, k + dz
            inside = 0 <= ii < nel[0] and 0 <= jj < nel[1] and (dim == 2 or 0 <= kk < nel[2])
            if h > 0 and inside:
                yield index(ii, jj, kk), h

    def wsum(e):
        return sum(h for _, h in neighbours(e))

    out = []
    for e in rows:
        if transpose:
            out.append(sum(h * x[q] / wsum(q) for q, h in neighbours(e)))
        else:
            out.append(sum(h * x[q] for q, h in neighbours(e)) / wsum(e))
    return np.array(out)
