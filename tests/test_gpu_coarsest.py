"""The coarsest solve multiplies by an explicit FP64 inverse, formed once at
setup from the Cholesky factor of the coarsest operator (Sec. 3.2 factorises
that operator once per hierarchy).  Its error against triangular solves with
the same factorisation, measured on the coarsest operators of the full-size
hierarchies (stiffness contrast 1e9), against the forward-error bound of
either method (a multiple of n eps cond(A))."""
import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = {
    "cantilever2d": (lambda: synth.get("cantilever2d"), dict(n_levels=7)),
    "grid2d": (lambda: synth.get("grid2d"), dict(n_levels=5)),
    "cantilever3d": (lambda: synth.get("cantilever3d"), dict(n_levels=6)),
    "bridge3d": (lambda: synth.get("bridge3d"), dict(n_geometric=3, max_coarse=1000)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_coarse_inverse_against_triangular_solves(name):
    from paper_2001_01655_amd import Hierarchy
    make, opts = CASES[name]
    p = make()
    print(f"coarsest inverse {name}", flush=True)
    H = Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, **opts)
    lc = H.num_levels() - 1
    rp, ci, v = H.export_csr(lc)
    n = rp.size - 1
    A = sp.csr_matrix((v, ci, rp), shape=(n, n)).toarray()
    Ainv = H.export_coarse_inverse()
    H.close()
    cond = float(np.linalg.cond(A))
    fac = sl.cho_factor(A, lower=True)
    B = np.random.default_rng(17).standard_normal((n, 4))
    Xc = sl.cho_solve(fac, B)
    Xi = Ainv @ B
    err = float(np.max(np.linalg.norm(Xi - Xc, axis=0) / np.linalg.norm(Xc, axis=0)))
    bound = 10.0 * n * np.finfo(float).eps * cond
    sym = float(np.linalg.norm(Ainv - Ainv.T) / np.linalg.norm(Ainv))
    print(f"  n={n} cond={cond:.2e} err={err:.2e} (bound {bound:.2e}) asym={sym:.1e}", flush=True)
    assert err <= bound
    assert sym <= 1e3 * np.finfo(float).eps * cond
