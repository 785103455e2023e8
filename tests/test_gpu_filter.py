"""The density filter kernel (tm_density_filter) against the oracle: whole
grids with ragged sizes, several radii, S and S^T; at the 3D cantilever size,
spot rows from the definition."""
import numpy as np
import pytest

from oracle import filter as flt

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("nel", [(37, 11), (64, 32), (13, 9, 7), (24, 16, 10)])
@pytest.mark.parametrize("r", [0.8, 1.5, 2.5, 3.7])
@pytest.mark.parametrize("transpose", [False, True])
def test_filter_matches_oracle(nel, r, transpose):
    from paper_2001_01655_amd import density_filter
    print(f"filter {nel} r={r} transpose={transpose}", flush=True)
    x = np.random.default_rng(len(nel) * 100 + int(10 * r)).random(int(np.prod(nel)))
    y = density_filter(nel, torch.tensor(x, device="cuda"), r, transpose).cpu().numpy()
    ref = flt.apply(nel, r, x, transpose=transpose)
    assert _rel(y, ref) <= 1e-14
    if r < 1.0:        # no other centre within the radius: x itself, up to the two roundings of (h x) / h
        assert _rel(y, x) <= 5e-16


@pytest.mark.parametrize("transpose", [False, True])
def test_filter_full_size_spot_rows(transpose):
    from paper_2001_01655_amd import density_filter
    nel, r = (192, 96, 96), 1.5
    n = int(np.prod(nel))
    x = np.random.default_rng(7).random(n)
    y = density_filter(nel, torch.tensor(x, device="cuda"), r, transpose).cpu().numpy()
    rows = np.unique(np.concatenate([[0, nel[0] - 1, n - 1, n // 2],
                                     np.random.default_rng(8).integers(0, n, 300)]))
    ref = flt.apply_rows(nel, r, x, rows, transpose=transpose)
    assert np.max(np.abs(y[rows] - ref) / np.abs(ref)) <= 1e-14
    # a constant field is a fixed point of S (rows of S sum to one)
    ones = density_filter(nel, torch.ones(n, dtype=torch.float64, device="cuda"), r).cpu().numpy()
    assert np.max(np.abs(ones - 1.0)) <= 1e-15
