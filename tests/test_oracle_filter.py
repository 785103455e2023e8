"""Pins of the oracle's density filter (Sec. 2 filtering matrix, Sec. 4 radius
1.5): brute force over element pairs, closed-form interior weights, row sums,
radius below one element, and the transpose by the inner-product identity."""
import itertools
import math

import numpy as np
import pytest

from oracle import filter as flt


def _brute(nel, r):
    dim = len(nel)
    cells = list(itertools.product(*[range(n) for n in nel[::-1]]))   # slowest axis first
    n = len(cells)
    H = np.zeros((n, n))
    for a, ca in enumerate(cells):
        for b, cb in enumerate(cells):
            d = math.sqrt(sum((x - y) ** 2 for x, y in zip(ca, cb)))
            H[a, b] = max(0.0, r - d)
    return H / H.sum(axis=1, keepdims=True)


@pytest.mark.parametrize("nel,r", [((4, 3), 1.5), ((5, 4), 2.5), ((3, 3, 2), 1.5), ((4, 3, 3), 2.2)])
def test_matches_brute_force(nel, r):
    S = flt.filter_matrix(nel, r).toarray()
    assert np.allclose(S, _brute(nel, r), rtol=0, atol=1e-15)


def test_interior_weights_closed_form_2d_and_3d():
    r = 1.5
    d1, d2 = r - 1.0, r - math.sqrt(2.0)          # face and edge neighbours; corners (sqrt 3) are out
    S2 = flt.filter_matrix((5, 5), r)
    row = S2.getrow(12).toarray().ravel()         # centre element of 5x5
    w2 = r + 4 * d1 + 4 * d2
    assert math.isclose(row[12], r / w2, rel_tol=1e-15)
    assert math.isclose(row[11], d1 / w2, rel_tol=1e-15) and math.isclose(row[6], d2 / w2, rel_tol=1e-15)
    assert np.count_nonzero(row) == 9
    S3 = flt.filter_matrix((5, 5, 5), r)
    row = S3.getrow(62).toarray().ravel()         # centre element of 5x5x5
    w3 = r + 6 * d1 + 12 * d2
    assert math.isclose(row[62], r / w3, rel_tol=1e-15)
    assert np.count_nonzero(row) == 19


def test_rows_sum_to_one_and_small_radius_is_identity():
    for nel in [(7, 3), (4, 5, 3)]:
        S = flt.filter_matrix(nel, 1.5)
        assert np.allclose(np.asarray(S.sum(axis=1)).ravel(), 1.0, rtol=0, atol=1e-15)
        x = np.random.default_rng(0).random(S.shape[0])
        assert np.array_equal(flt.apply(nel, 1.0, x), x)         # no neighbour closer than 1
        assert np.array_equal(flt.apply(nel, 0.7, x), x)


def test_transpose_by_inner_products():
    nel, r = (6, 5, 4), 1.5
    rng = np.random.default_rng(1)
    a, b = rng.random(120), rng.random(120)
    lhs = flt.apply(nel, r, a) @ b
    rhs = a @ flt.apply(nel, r, b, transpose=True)
    assert math.isclose(lhs, rhs, rel_tol=1e-13)


@pytest.mark.parametrize("transpose", [False, True])
def test_row_spot_checks_equal_the_matrix(transpose):
    nel, r = (7, 5, 4), 1.5
    x = np.random.default_rng(2).random(140)
    full = flt.apply(nel, r, x, transpose=transpose)
    rows = [0, 6, 34, 69, 70, 139]
    assert np.allclose(flt.apply_rows(nel, r, x, rows, transpose=transpose), full[rows], rtol=1e-14, atol=0)
