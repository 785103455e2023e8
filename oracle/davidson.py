"""Oracle, part 7: the generalized Davidson eigensolver (CPU, FP64).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Follows Algorithm 2 of the paper (Sec. 3, eigenvalue solvers) for the pencil
A x = theta B x with B symmetric positive definite (here A = K_sigma~,
B = K~ and the preconditioner M = one multigrid V-cycle for K~): a search
space V is grown by one preconditioned residual per iteration, the Ritz pair
of interest is taken from the Rayleigh-Ritz projection onto V, and V is cut
back to the leading Ritz vectors when it reaches j_max.  Sec. 4 uses
j_min = 10, j_max = 25, six eigenvalues, and stops a pair when its relative
residual is below 1e-6 or its eigenvalue changes by less than 1e-13
(relative) between consecutive iterations.

Readings (the paper leaves them open):
  * Gram-Schmidt works in the B inner product, so V^T B V = I and the
    projected problem is the standard symmetric H = V^T A V; classical
    Gram-Schmidt with one repetition when the B-norm drops below 1/sqrt(2)
    of its value before the projection (the Daniel-Gragg-Kaufman-Stewart
    test), the norm after the projection taken from Pythagoras
    (||z||_B^2 - ||c||^2); a vector whose B-norm after the projection is
    below 1e-10 of the original is a breakdown;
  * the target is the largest Ritz value not yet converged: pairs converge
    in descending order and stay in V (no hard deflation), the (k+1)-th is
    targeted once the first k have converged;
  * relative residual = ||A q - theta B q||_2 / (|theta| ||B q||_2);
    the stagnation test compares theta with the same target's Ritz value of
    the previous iteration (not after the target has moved on);
  * when the target converges, the next target is tested in the same
    iteration, before the space is expanded;
  * the restart (j = j_max) keeps the j_min leading Ritz vectors, and the
    projected matrix becomes diag(theta_1..theta_jmin);
  * the iteration count is the number of expansions (preconditioner calls);
  * the initial vectors are the caller's, taken in order and B-orthonormalised
    with the same Gram-Schmidt; a dependent one is an error.
The returned vectors are the Ritz vectors of the first nev Ritz values, so
Phi^T B Phi = I.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List

import numpy as np

ETA = 1.0 / np.sqrt(2.0)
BREAKDOWN = 1e-10


@dataclass
class GDResult:
    theta: np.ndarray            # nev Ritz values, descending
    Phi: np.ndarray              # (n, nev) Ritz vectors, B-orthonormal
    iters: int                   # expansions
    n_conv: int
    converged: bool
    history: List[tuple] = field(default_factory=list)   # (iteration, target, theta, relres)


def b_orthonormalize(V: np.ndarray, j: int, z: np.ndarray, apply_B: Callable):
    """B-orthonormalise z against the first j columns of V (CGS with one
    conditional repetition).  Returns the unit vector, or None on breakdown."""
    w = apply_B(z)
    zz0 = float(z @ w)
    if not zz0 > 0.0:
        return None
    zz = zz0
    for _ in range(2):
        c = V[:, :j].T @ w
        beta2 = zz - float(c @ c)
        z = z - V[:, :j] @ c
        if beta2 > ETA * ETA * zz:
            break
        w = apply_B(z)
        zz = float(z @ w)
    if not beta2 > (BREAKDOWN ** 2) * zz0:
        return None
    return z / np.sqrt(beta2)


def generalized_davidson(apply_A: Callable, apply_B: Callable, precond: Callable, V0: np.ndarray,
                         nev: int = 6, j_min: int = 10, j_max: int = 25, tol: float = 1e-6,
                         stag_tol: float = 1e-13, max_iters: int = 1000) -> GDResult:
    n = V0.shape[0]
    if not (1 <= nev < j_min < j_max) or V0.shape[1] < 1 or V0.shape[1] > j_max:
        raise ValueError("need 1 <= nev < j_min < j_max and 1 <= initial vectors <= j_max")
    V = np.zeros((n, j_max))
    H = np.zeros((j_max, j_max))
    j = 0

    def append(z):
        nonlocal j
        v = b_orthonormalize(V, j, z, apply_B)
        if v is None:
            return False
        V[:, j] = v
        Av = apply_A(v)
        hcol = V[:, :j + 1].T @ Av
        H[:j + 1, j] = hcol
        H[j, :j + 1] = hcol
        j += 1
        return True

    for i in range(V0.shape[1]):
        if not append(V0[:, i].astype(np.float64)):
            raise ValueError("initial vectors are dependent in the B inner product")

    k = 0                       # converged pairs
    it = 0
    prev_theta = None           # the target's Ritz value in the previous iteration
    hist = []
    while True:
        theta, Y = np.linalg.eigh(H[:j, :j])
        order = np.argsort(theta)[::-1]
        theta, Y = theta[order], Y[:, order]
        while k < nev:
            q = V[:, :j] @ Y[:, k]
            Aq, Bq = apply_A(q), apply_B(q)
            r = Aq - theta[k] * Bq
            den = abs(theta[k]) * np.linalg.norm(Bq)
            rel = np.linalg.norm(r) / den if den > 0.0 else (0.0 if not r.any() else np.inf)
            hist.append((it, k, float(theta[k]), float(rel)))
            stag = prev_theta is not None and abs(theta[k] - prev_theta) < stag_tol * abs(theta[k])
            if rel < tol or stag:
                k += 1
                prev_theta = None
                continue
            break
        if k == nev or it >= max_iters:
            break
        prev_theta = float(theta[k])
        if j == j_max:
            V[:, :j_min] = V[:, :j] @ Y[:, :j_min]
            H[:, :] = 0.0
            H[np.arange(j_min), np.arange(j_min)] = theta[:j_min]
            j = j_min
        z = precond(r)
        it += 1
        if not append(z):
            raise FloatingPointError("search space breakdown: the correction lies in the search space")
    theta, Y = np.linalg.eigh(H[:j, :j])
    order = np.argsort(theta)[::-1]
    theta, Y = theta[order], Y[:, order]
    Phi = V[:, :j] @ Y[:, :nev]
    return GDResult(theta[:nev].copy(), Phi, it, k, k == nev, hist)
