"""Pins of the oracle's automated hybrid (second hybrid of Sec. 4.4): the
policy's level counts and, for every design, the solution against a dense
Cholesky solve (the preconditioner changes, the answer does not)."""
import numpy as np
import pytest

import synth
from oracle import adaptive, fem, mg

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")

NEL = (8, 4, 4)


def _stream(n=4, seed=51):
    p = synth.small_case(3, NEL, seed=seed)
    rhos = [p.rho]
    for t in range(1, n):
        rhos.append(synth.density_update(rhos[-1], p.nel, seed=seed, step=t))
    return p, rhos


def _dense(p, rho):
    KE = fem.element_stiffness(3, p.nu)
    E = fem.simp(rho, p.p, p.E0, p.Emin)
    A = fem.apply_dirichlet(fem.assemble(p.nel, E, KE), p.fixed)
    f = p.loads[0].copy()
    f[p.fixed] = 0.0
    return mg.dense_solve(A, f)


def test_threshold_never_reached_keeps_the_geometric_hierarchy():
    p, rhos = _stream(3)
    steps = adaptive.adaptive_stream(p.nel, rhos, p.fixed, p.loads[0], n_start=3, threshold=10 ** 6,
                                     max_coarse=100)
    assert [s.n_geometric for s in steps] == [3, 3, 3]
    assert [s.levels for s in steps] == [3, 3, 3]          # 36 dofs at the bottom: no aggregation
    for s, rho in zip(steps, rhos):
        ud = _dense(p, rho)
        assert np.linalg.norm(s.u - ud) <= 1e-7 * np.linalg.norm(ud)


def test_every_solve_over_the_threshold_drops_one_geometric_level_down_to_two():
    p, rhos = _stream(4)
    steps = adaptive.adaptive_stream(p.nel, rhos, p.fixed, p.loads[0], n_start=3, threshold=1,
                                     max_coarse=100)
    assert all(s.iters > 1 for s in steps)
    assert [s.n_geometric for s in steps] == [3, 2, 2, 2]
    # with two geometric levels the last one (135 dofs) is over the coarse limit,
    # so smoothed aggregation adds a level below it
    assert steps[0].levels == 3 and all(s.levels == 3 for s in steps[1:])
    for s, rho in zip(steps, rhos):
        ud = _dense(p, rho)
        assert np.linalg.norm(s.u - ud) <= 1e-7 * np.linalg.norm(ud)


def test_floor_of_geometric_levels_holds():
    p, rhos = _stream(2)
    steps = adaptive.adaptive_stream(p.nel, rhos, p.fixed, p.loads[0], n_start=3, threshold=1,
                                     max_coarse=100, min_geometric=3)
    assert [s.n_geometric for s in steps] == [3, 3]        # the floor holds
