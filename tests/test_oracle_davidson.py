"""Pins of the oracle's generalized Davidson solver (Algorithm 2): the leading
eigenvalues of the pencil (K_sigma~, K~) against a dense generalized symmetric
eigensolver, B-orthonormal Ritz vectors with small residuals, the same answer
with forced restarts, and the non-converged and argument paths."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import buckling, davidson, fem, mg
from synth import problems as P


def _setup(p, levels):
    KE = fem.element_stiffness(p.dim, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = mg.build_geometric(p.nel, E, KE, p.fixed, levels)
    K = H.A[0]
    u = mg.dense_solve(K, p.loads[0])
    Ks = buckling.stress_stiffness(p.nel, u, p.rho, p.p, p.E0, p.nu, p.fixed)
    return H, K, Ks


def _dense_top(K, Ks, fixed, nev):
    free = fem.free_mask(K.shape[0], fixed) > 0
    lam = sla.eigh(Ks.toarray()[np.ix_(free, free)], K.toarray()[np.ix_(free, free)], eigvals_only=True)
    return lam[::-1][:nev]


def _start(n, k, fixed, seed=0):
    V0 = np.random.default_rng(seed).standard_normal((n, k))
    V0[fixed] = 0.0
    return V0


@pytest.mark.parametrize("case", ["column", "small3d"])
def test_leading_eigenvalues_match_dense_solver(case):
    if case == "column":
        p, levels = P.column_2d(nel=(8, 32), seed=2), 3
    else:
        p = P.small_case(3, (4, 4, 6), seed=5)
        levels = 2
    H, K, Ks = _setup(p, levels)
    nev = 6
    res = davidson.generalized_davidson(lambda v: Ks @ v, lambda v: K @ v, lambda r: mg.vcycle(H, r),
                                        _start(K.shape[0], 10, p.fixed), nev=nev, j_min=10, j_max=25)
    assert res.converged and res.n_conv == nev
    want = _dense_top(K, Ks, p.fixed, nev)
    assert np.allclose(res.theta, want, rtol=1e-8, atol=0)
    Phi = res.Phi
    assert np.allclose(Phi.T @ (K @ Phi), np.eye(nev), atol=1e-10)
    # a pair stops at relative residual 1e-6 or when its eigenvalue changes by
    # less than 1e-13 (relative) between iterations; with voids (E = 1e-9 K
    # entries) the second test fires first, at residuals near 1e-5
    for i in range(nev):
        r = Ks @ Phi[:, i] - res.theta[i] * (K @ Phi[:, i])
        assert np.linalg.norm(r) <= 1e-4 * abs(res.theta[i]) * np.linalg.norm(K @ Phi[:, i])


def test_forced_restarts_reach_the_same_eigenvalues():
    p = P.column_2d(nel=(8, 32), seed=3)
    H, K, Ks = _setup(p, 3)
    a = davidson.generalized_davidson(lambda v: Ks @ v, lambda v: K @ v, lambda r: mg.vcycle(H, r),
                                      _start(K.shape[0], 4, p.fixed), nev=3, j_min=4, j_max=6)
    assert a.converged
    assert np.allclose(a.theta, _dense_top(K, Ks, p.fixed, 3), rtol=1e-8, atol=0)
    assert a.iters > 6          # several restarts happened


def test_iteration_limit_reports_not_converged():
    p = P.column_2d(nel=(8, 32), seed=2)
    H, K, Ks = _setup(p, 3)
    res = davidson.generalized_davidson(lambda v: Ks @ v, lambda v: K @ v, lambda r: mg.vcycle(H, r),
                                        _start(K.shape[0], 10, p.fixed), nev=6, max_iters=2)
    assert not res.converged and res.iters == 2 and res.n_conv < 6


def test_arguments_and_dependent_start():
    n = 10
    A = np.diag(np.arange(1.0, n + 1))
    f = lambda v: A @ v
    with pytest.raises(ValueError):
        davidson.generalized_davidson(f, f, f, np.ones((n, 2)), nev=3, j_min=3, j_max=5)
    V0 = np.ones((n, 2))
    with pytest.raises(ValueError):
        davidson.generalized_davidson(f, lambda v: v, f, V0, nev=1, j_min=2, j_max=4)


def test_standard_problem_with_exact_inverse_preconditioner():
    """B = I, A diagonal: the eigenvalues are the diagonal; with M = I (plain
    residual expansion, i.e. Lanczos-like growth) the top three are found."""
    n = 40
    d = np.linspace(1.0, 10.0, n)
    d[-1], d[-2], d[-3] = 30.0, 20.0, 15.0
    res = davidson.generalized_davidson(lambda v: d * v, lambda v: v.copy(), lambda r: r.copy(),
                                        np.random.default_rng(1).standard_normal((n, 4)),
                                        nev=3, j_min=5, j_max=12, max_iters=200)
    assert res.converged
    assert np.allclose(res.theta, [30.0, 20.0, 15.0], rtol=1e-10)


def test_zero_pencil_converges_without_expansion():
    """A = 0 (no stress, e.g. u = 0): every Ritz value is 0 with a zero
    residual, so all pairs converge before the first expansion."""
    n = 30
    B = np.diag(np.linspace(1.0, 2.0, n))
    res = davidson.generalized_davidson(lambda v: np.zeros_like(v), lambda v: B @ v, lambda r: r.copy(),
                                        np.random.default_rng(0).standard_normal((n, 10)), nev=6)
    assert res.converged and res.iters == 0 and np.all(res.theta == 0.0)
