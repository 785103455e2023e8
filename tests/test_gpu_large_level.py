"""GPU parity of the large-level coarse operator against the oracle, at sizes
whose first coarse level is big enough to take that kernel by the library's own
choice (at least 256 workgroups of nodes: 65,281 nodes or more).

Cases (the configurations' recipes at a size the oracle builds in seconds):
  * 3D cantilever 128x64x64, 5 levels: level 1 has 65x33x33 = 70,785 nodes;
  * 2D cantilever 1024x512, 7 levels: level 1 has 513x257 = 131,841 nodes.
Each compares, element by element, the Galerkin operators of every coarse
level (pattern bit-exact, values), the level operators applied in FP64 and
FP32, and one V-cycle (Algorithm 1) with block-Jacobi 1/1 and Chebyshev 2/2
smoothing, in FP64 and FP32.  The oracle hierarchy is built once per case."""
import numpy as np
import pytest

import synth
from oracle import fem, mg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LARGE_NODES = 255 * 256 + 1        # first level size that fills 256 workgroups of 256 nodes


def _say(msg):
    print(msg, flush=True)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


CASES = {
    "3d_128x64x64": (lambda: synth.cantilever_3d(nel=(128, 64, 64)), 5),
    "2d_1024x512": (lambda: synth.cantilever_2d(nel=(1024, 512)), 7),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    make, L = CASES[request.param]
    p = make()
    _say(f"oracle hierarchy {request.param} ({p.n_dof} dofs, {L} levels)")
    KE = fem.element_stiffness(p.dim, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = mg.build_geometric(p.nel, E, KE, p.fixed, L)
    n1 = H.A[1].shape[0] // p.dim
    assert n1 >= LARGE_NODES, "level 1 must be large enough for the large-level kernel"
    yield request.param, p, L, H


def _gpu(p, L, **kw):
    from paper_2001_01655_amd import Hierarchy
    return Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, n_levels=L, **kw)


@pytest.mark.parametrize("kern", [0, 1], ids=["by_size", "large_everywhere"])
def test_coarse_operators(case, kern):
    """Every coarse level's CSR (pattern bit-exact, values <= 1e-12) and the
    stored operator applied to a seeded vector in FP64 (<= 1e-13) and FP32
    (<= 2e-6 against the FP64 product of the rounded input)."""
    name, p, L, H = case
    _say(f"coarse operators {name} stencil_kernel={kern}")
    G = _gpu(p, L, stencil_kernel=kern)
    for l in range(1, L):
        A = H.A[l]
        rp, ci, v = G.export_csr(l)
        assert np.array_equal(rp, A.indptr) and np.array_equal(ci, A.indices), f"pattern level {l}"
        assert _rel(v, A.data) <= 1e-12, f"values level {l}"
        x = synth.seeded_vector(A.shape[0], 300 + l)
        y = G.apply(l, torch.tensor(x, device="cuda"), fp=64).cpu().numpy()
        e64 = _rel(y, A @ x)
        x32 = x.astype(np.float32)
        y32 = G.apply(l, torch.tensor(x32, device="cuda"), fp=32).cpu().numpy()
        e32 = _rel(y32.astype(np.float64), A @ x32.astype(np.float64))
        _say(f"  level {l}: {A.shape[0]} rows, {A.nnz} nnz, apply err fp64 {e64:.1e} fp32 {e32:.1e}")
        assert e64 <= 1e-13 and e32 <= 2e-6, f"apply level {l}"
    G.close()


@pytest.mark.parametrize("smoother", ["jacobi", "chebyshev"])
def test_vcycle(case, smoother):
    """One V-cycle from zero on a seeded masked right-hand side: FP64 against
    the oracle's V-cycle (<= 1e-9; the coarsest solve multiplies by an explicit
    inverse), FP32 within FP32 accuracy (<= 1e-3)."""
    name, p, L, H = case
    _say(f"vcycle {name} {smoother}")
    if smoother == "jacobi":
        Ho, kw = H, {}
    else:
        Ho = mg.finish(H.A, H.P, H.bs, H.omega, 2, 2, kinds=H.kinds, smoother="chebyshev", fixed=p.fixed)
        kw = dict(smoother=2, nu_pre=2, nu_post=2)
    b = synth.seeded_vector(p.n_dof, 310, p.fixed)
    ref = mg.vcycle(Ho, b)
    G = _gpu(p, L, vcycle_fp=64, **kw)
    z = G.vcycle(torch.tensor(b, device="cuda"), fp=64).cpu().numpy()
    z32 = G.vcycle(torch.tensor(b, device="cuda", dtype=torch.float32), fp=32).cpu().numpy()
    e64, e32 = _rel(z, ref), _rel(z32.astype(np.float64), ref)
    _say(f"  err fp64 {e64:.1e} fp32 {e32:.1e}")
    assert e64 <= 1e-9 and e32 <= 1e-3
    G.close()
