"""The tensor-product form of the trilinear cube's KE that the fine operators
(and the optional level-1 form) apply, restated in numpy and checked against
the oracle's element stiffness and assembled operators (CPU only).

Sum / difference modes of an element's corner values (bit k of the mode
index set: difference along axis k): KE = F^T C F per pair of components with
C nonzero only where component d's input mode m feeds component c's output
mode m (c = d, m != 0) or m with bits c and d flipped (c != d, bits c and d of
m differ).  Level 1 of an even grid is the sum over its fine sub-elements of
P_k^T (E_k M_k KE M_k) P_k (Sec. 3.2's Galerkin product with the supports M)."""
import itertools

import numpy as np
import pytest

import synth
from oracle import fem, mg


def _loc(lx, ly, lz):
    # the oracle's corner order: bottom face counter-clockwise, then the top face
    return 4 * lz + ((2 if lx else 3) if ly else (1 if lx else 0))


def _modes_matrix():
    F = np.zeros((8, 8))
    for m in range(8):
        for lx, ly, lz in itertools.product((0, 1), repeat=3):
            w = 1.0
            for k, l in enumerate((lx, ly, lz)):
                if (m >> k) & 1:
                    w *= 1.0 if l else -1.0
            F[m, _loc(lx, ly, lz)] = w
    return F


def _coupled(c, d, mo, mi):
    if c == d:
        return mo == mi and mi != 0
    return ((mi >> c) & 1) != ((mi >> d) & 1) and mo == mi ^ (1 << c) ^ (1 << d)


@pytest.mark.parametrize("nu", [0.0, 0.3, 0.45])
def test_ke_in_modes_has_45_couplings(nu):
    KE = fem.element_stiffness(3, nu)
    F = _modes_matrix()
    amax = np.abs(KE).max()
    K2 = np.zeros_like(KE)
    n_on = 0
    for c in range(3):
        for d in range(3):
            C = F @ KE[c::3, d::3] @ F.T / 64.0
            for mo in range(8):
                for mi in range(8):
                    if _coupled(c, d, mo, mi):
                        n_on += 1
                    else:
                        assert abs(C[mo, mi]) <= 1e-13 * amax
            K2[c::3, d::3] = F.T @ C @ F
    assert n_on == 45
    assert np.abs(K2 - KE).max() <= 1e-14 * amax


def test_half_element_interpolation_in_modes():
    """Per axis, the trilinear interpolation to the lower / upper half maps
    (sigma, delta) to (sigma -+ delta / 2, delta / 2), and its transpose maps
    output modes back as (sigma, (delta -+ sigma) / 2)."""
    F1 = np.array([[1.0, 1.0], [-1.0, 1.0]])            # rows: sigma, delta
    halves = {0: np.array([[1.0, 0.0], [0.5, 0.5]]), 1: np.array([[0.5, 0.5], [0.0, 1.0]])}
    for h, P in halves.items():
        s = 1.0 if h else -1.0
        T = F1 @ P @ np.linalg.inv(F1)                   # input modes of the half from the whole's
        np.testing.assert_allclose(T, [[1.0, s / 2], [0.0, 0.5]], atol=1e-15)
        Tt = np.linalg.inv(F1.T) @ P.T @ F1.T            # output modes of the whole from the half's
        np.testing.assert_allclose(Tt, [[1.0, 0.0], [s / 2, 0.5]], atol=1e-15)


@pytest.mark.parametrize("nel,support", [((8, 6, 4), "clamp"), ((6, 4, 8), "corner")])
def test_level1_is_the_sum_over_fine_sub_elements(nel, support):
    p = synth.small_case(3, nel, seed=21, support=support)
    KE = fem.element_stiffness(3, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = mg.build_geometric(p.nel, E, KE, p.fixed, 2)
    nx, ny, nz = nel
    cx, cy, cz = nx // 2, ny // 2, nz // 2
    NXc, NYc = cx + 1, cy + 1
    x = np.random.default_rng(5).standard_normal(H.A[1].shape[0])
    free = fem.free_mask((nx + 1) * (ny + 1) * (nz + 1) * 3, p.fixed)
    Eg = E.reshape(nz, ny, nx)
    half = {0: np.array([[1.0, 0.0], [0.5, 0.5]]), 1: np.array([[0.5, 0.5], [0.0, 1.0]])}
    y = np.zeros_like(x)
    for kz, ky, kx in itertools.product(range(cz), range(cy), range(cx)):
        uc = np.zeros((3, 2, 2, 2))
        cn = {}
        for lz, ly, lx in itertools.product((0, 1), repeat=3):
            cn[lz, ly, lx] = ((kz + lz) * NYc + (ky + ly)) * NXc + (kx + lx)
            uc[:, lz, ly, lx] = x[3 * cn[lz, ly, lx]:3 * cn[lz, ly, lx] + 3]
        yc = np.zeros((3, 2, 2, 2))
        for hz, hy, hx in itertools.product((0, 1), repeat=3):
            ex, ey, ez = 2 * kx + hx, 2 * ky + hy, 2 * kz + hz
            uf = np.einsum('ai,bj,ck,dijk->dabc', half[hz], half[hy], half[hx], uc)
            ue, mk = np.zeros(24), np.zeros(24)
            for lz, ly, lx in itertools.product((0, 1), repeat=3):
                f = ((ez + lz) * (ny + 1) + (ey + ly)) * (nx + 1) + (ex + lx)
                a = _loc(lx, ly, lz)
                ue[3 * a:3 * a + 3] = uf[:, lz, ly, lx]
                mk[3 * a:3 * a + 3] = free[3 * f:3 * f + 3]
            fe = Eg[ez, ey, ex] * (mk * (KE @ (mk * ue)))
            yf = np.zeros((3, 2, 2, 2))
            for lz, ly, lx in itertools.product((0, 1), repeat=3):
                a = _loc(lx, ly, lz)
                yf[:, lz, ly, lx] = fe[3 * a:3 * a + 3]
            yc += np.einsum('ai,bj,ck,dabc->dijk', half[hz], half[hy], half[hx], yf)
        for key, node in cn.items():
            y[3 * node:3 * node + 3] += yc[(slice(None),) + key]
    ref = H.A[1] @ x
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
