"""The seeded generators are deterministic and produce the stated shapes."""
import hashlib

import numpy as np

import synth


def _digest(p):
    h = hashlib.sha256()
    for a in (p.rho, p.fixed, p.loads):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_same_seed_same_bytes():
    for make in (lambda: synth.mbb_2d(False), lambda: synth.cantilever_2d((64, 32)),
                 lambda: synth.cantilever_3d((16, 8, 8)), lambda: synth.bridge_3d((32, 16, 16)),
                 lambda: synth.served_request(3)):
        assert _digest(make()) == _digest(make())


def test_shapes_and_ranges():
    p = synth.cantilever_3d((16, 8, 8))
    assert p.rho.shape == (16 * 8 * 8,) and p.rho.min() == 1e-3 and p.rho.max() == 1.0
    assert p.loads.shape == (1, p.n_dof) and abs(p.loads.sum() + 1.0) < 1e-14
    b = synth.bridge_3d((32, 16, 16))
    assert set(np.unique(b.rho)) == {1e-3, 1.0}
    assert len(b.fixed) == 12 and abs(b.loads.sum() + 1.0) < 1e-14
    s = synth.served_request(7)
    assert 1 <= s.loads.shape[0] <= 4
    t = synth.poisson_arrivals(50, 10.0)
    assert np.all(np.diff(t) > 0)


def test_cantilever_2d_solid_is_anchored():
    from scipy.ndimage import label
    p = synth.cantilever_2d((128, 64))
    nx, ny = p.nel
    solid = (p.rho == 1.0).reshape(ny, nx)
    lab, n = label(solid)
    assert n == 1 and solid[:, 0].any()
    # the element under the load node is solid and the field is not all solid
    assert solid[ny // 2, nx - 1] and 0.3 < solid.mean() < 0.9


def test_grid_recipe():
    """Varying-spaced grid (Sec. 4.3): 8-element features at the given
    spacings, bottom nodes fixed, unit total load on the top edge."""
    import synth
    p = synth.grid_2d(16, 64, nel=(520, 520))
    rho = p.rho.reshape(520, 520)
    assert set(np.unique(rho)) == {synth.problems.VOID, 1.0}
    assert np.all(rho[:, 0:8] == 1.0) and np.all(rho[:, 512:520] == 1.0)    # first and last column
    assert np.all(rho[512:520, :] == 1.0)                                     # top beam
    assert np.all(rho[:, 8:16][100:110] == synth.problems.VOID)               # between two columns, between beams
    assert len(p.fixed) == 2 * 521 and np.isclose(p.loads[0].sum(), -1.0)
