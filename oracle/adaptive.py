"""Oracle, part 4: the automated GMG->AMG hybrid over a design stream (CPU,
FP64).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Follows the second hybrid of Sec. 4.4 (3D cantilever): the hierarchy starts
with a number of geometric levels, and every time the linear solver needs more
than a threshold of iterations (200 in the paper) one geometric level is
given up for algebraic (smoothed-aggregation) coarsening, until two geometric
levels remain; the coarse-size limit (1000 dofs) holds throughout.

Reading (the paper does not fix it): the decision taken after the solve of
design t applies from design t+1 on, since the hierarchy of design t is the one
the solve just used.  Iteration counts of the PCG come from mg.mg_pcg.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import fem, mg, sa


@dataclass
class StreamStep:
    n_geometric: int        # geometric levels (fine grid included) used for this design
    levels: int             # all levels of the hierarchy
    iters: int              # PCG iterations to rtol
    u: np.ndarray


def hierarchy(nel, E, KE, fixed, n_geometric: int, max_coarse: int, **kw) -> mg.Hierarchy:
    """n_geometric geometric levels, then smoothed aggregation while the last
    level has at least max_coarse dofs (none if it is already smaller)."""
    return sa.build_hybrid(nel, E, KE, fixed, n_geometric, max_coarse=max_coarse, **kw)


def adaptive_stream(nel, rhos, fixed, f, *, n_start: int = 6, threshold: int = 200, min_geometric: int = 2,
                    max_coarse: int = 1000, rtol: float = 1e-8, p: float = 3.0, E0: float = 1.0,
                    Emin: float = 1e-9, nu: float = 0.3, **kw) -> list[StreamStep]:
    """Solve K(rho_t) u = f for each design of the stream with the automated
    hybrid; returns what each design used and needed."""
    KE = fem.element_stiffness(len(nel), nu)
    G = n_start
    out = []
    for rho in rhos:
        E = fem.simp(rho, p, E0, Emin)
        H = hierarchy(nel, E, KE, fixed, G, max_coarse, **kw)
        r = mg.mg_pcg(H, f, rtol)
        out.append(StreamStep(G, len(H.A), r.iters, r.u))
        if r.iters > threshold and G > min_geometric:
            G -= 1
    return out
