"""Compliance sensitivity on the GPU against the oracle's formula, on the same
displacements (element by element), for one and several load cases, and the
homogeneity identity at full configuration size."""
import numpy as np
import pytest

import synth
from oracle import fem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _bound(nel, rho, p, KE, U):
    """Rounding bound of the element quadratic forms: (ND^2 + 2) eps times the
    absolute-value form sum |u_r| |KE_rs| |u_s| (cancellation in near-rigid
    elements makes the form itself much smaller than its terms)."""
    nd = KE.shape[0]
    return (nd * nd + 2) * np.finfo(float).eps * np.abs(
        fem.compliance_sensitivity(nel, rho, p.p, p.E0, p.Emin, np.abs(KE), np.abs(U)))


@pytest.mark.parametrize("dim,nel,L,n_rhs", [(2, (40, 24), 3, 1), (3, (12, 8, 8), 3, 2), (3, (10, 6, 4), 2, 3)])
def test_sensitivity_vs_oracle(dim, nel, L, n_rhs):
    from paper_2001_01655_amd import Hierarchy
    print(f"sensitivity {nel} rhs={n_rhs}", flush=True)
    p = synth.small_case(dim, nel, seed=41, n_rhs=n_rhs)
    H = Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, n_levels=L)
    r = H.solve(torch.tensor(p.loads, device="cuda"), rtol=1e-10)
    dc = H.compliance_sensitivity(r.u).cpu().numpy()
    U = r.u.cpu().numpy().reshape(n_rhs, -1)
    KE = fem.element_stiffness(dim, p.nu)
    ref = fem.compliance_sensitivity(p.nel, p.rho, p.p, p.E0, p.Emin, KE, U)
    assert np.all(np.abs(dc - ref) <= _bound(p.nel, p.rho, p, KE, U))
    # the densities follow tm_update_density
    rho2 = synth.density_update(p.rho, p.nel, seed=41, step=1)
    H.update_density(torch.tensor(rho2, device="cuda"))
    dc2 = H.compliance_sensitivity(r.u).cpu().numpy()
    ref2 = fem.compliance_sensitivity(p.nel, rho2, p.p, p.E0, p.Emin, KE, U)
    assert np.all(np.abs(dc2 - ref2) <= _bound(p.nel, rho2, p, KE, U))
    H.close()


@pytest.mark.parametrize("dim,nel,L,n_rhs", [(2, (40, 24), 3, 2), (3, (12, 8, 8), 3, 1)])
def test_sensitivity_end_to_end(dim, nel, L, n_rhs):
    """From the loads to dc on both sides: the oracle's own displacements
    (a sparse direct solve of its assembled K~) and its formula, against the
    GPU's solve at rtol 1e-10 and its sensitivity kernel.  The difference is
    that of the two solutions, carried to first order by 2 |u_e| |KE| |du_e|:
    bounded here by 1e-7 of the largest |dc_e|."""
    import scipy.sparse.linalg as spl
    from paper_2001_01655_amd import Hierarchy
    print(f"sensitivity end to end {nel} rhs={n_rhs}", flush=True)
    p = synth.small_case(dim, nel, seed=43, n_rhs=n_rhs)
    KE = fem.element_stiffness(dim, p.nu)
    K = fem.apply_dirichlet(fem.assemble(p.nel, fem.simp(p.rho, p.p, p.E0, p.Emin), KE), p.fixed).tocsc()
    F = p.loads.copy()
    F[:, p.fixed] = 0.0
    U_ref = np.stack([spl.spsolve(K, F[k]) for k in range(n_rhs)])
    ref = fem.compliance_sensitivity(p.nel, p.rho, p.p, p.E0, p.Emin, KE, U_ref)
    H = Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, n_levels=L)
    r = H.solve(torch.tensor(p.loads, device="cuda"), rtol=1e-10)
    dc = H.compliance_sensitivity(r.u).cpu().numpy()
    H.close()
    err = float(np.max(np.abs(dc - ref)) / np.max(np.abs(ref)))
    print(f"  max |dc - dc_oracle| / max |dc_oracle| = {err:.2e}", flush=True)
    assert err <= 1e-7


def test_sensitivity_full_size_homogeneity():
    """3D cantilever at full size: sum_e rho_e dc_e = -p c up to the Emin part,
    which the oracle's element sum evaluates exactly on the GPU solution."""
    from paper_2001_01655_amd import Hierarchy
    p = synth.get("cantilever3d")
    H = Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, n_levels=6)
    r = H.solve(torch.tensor(p.loads[0], device="cuda"), rtol=1e-10)
    dc = H.compliance_sensitivity(r.u).cpu().numpy()
    u = r.u.cpu().numpy()
    # c = u^T K u = sum_e E_e q_e and rho_e dc_e = -p (E_e - Emin) q_e, so
    # sum rho dc = -p (c - Emin sum_e q_e), q_e = u_e^T KE u_e
    KE = fem.element_stiffness(3, p.nu)
    q = -fem.compliance_sensitivity(p.nel, np.ones_like(p.rho), 1.0, 1.0, 0.0, KE, u)
    c = r.compliance[0]
    lhs = float(p.rho @ dc)
    rhs = -p.p * (c - p.Emin * q.sum())
    print(f"  sum rho dc = {lhs:.12e}, -p (c - Emin sum q) = {rhs:.12e}", flush=True)
    assert abs(lhs - rhs) <= 1e-7 * abs(rhs)
    H.close()
