"""Assembly with the velocity at the quadrature points (``hdg_assemble_q``):
for an affine field it equals the vertex-velocity assembly; for a field that
is not affine (``SwirlFlow``) it matches the oracle, which evaluates the
velocity at its quadrature points, while the vertex interpolant does not.

Tolerances as in the other assembly parity tests: scaled matrix and
right-hand side 1e-12 relative to the largest entry; solution at tol 1e-12
within 1e-10."""
import numpy as np
import pytest

from oracle import air as oair
from oracle.drivers import setup_problem, air_fgmres_solve
from gpu_cases import case, gpu_system, to_scipy, rel_sparse_diff
from workloads import square_tri_mesh, slab_prism_tet_mesh
from workloads.problems import SwirlFlow

pytestmark = pytest.mark.gpu


def _scaled(g):
    e = g.export()
    return to_scipy(e["rowptr"], e["col"], e["val"], g.n), e["hhat"].cpu().numpy()


@pytest.mark.parametrize("name", ["c1", "slab", "kuhn_nu4"])
def test_points_equal_vertices_for_affine_fields(name):
    print("case", name, flush=True)
    v, c, prob, p = case(name)
    A1, h1 = _scaled(gpu_system(v, c, prob, p))
    A2, h2 = _scaled(gpu_system(v, c, prob, p, at_points=True))
    assert rel_sparse_diff(A2, A1) <= 1e-13
    assert np.abs(h2 - h1).max() <= 1e-13 * np.abs(h1).max()


@pytest.mark.parametrize("d, p", [(1, 1), (1, 2), (2, 1), (2, 2)])
def test_non_affine_velocity_matches_oracle(d, p):
    from paper_2010_11130_amd import Hierarchy
    print("case swirl d", d, "p", p, flush=True)
    prob = SwirlFlow(d, 1e-3)
    v, c = square_tri_mesh(8) if d == 1 else slab_prism_tet_mesh(6, 1.0 / 8)
    o = setup_problem(v, c, prob, p)
    gq = gpu_system(v, c, prob, p, at_points=True)
    Aq, hq = _scaled(gq)
    assert rel_sparse_diff(Aq, o.Shat) <= 1e-12
    assert np.abs(hq - o.Hhat).max() <= 1e-12 * np.abs(o.Hhat).max()
    # the vertex interpolant of this field assembles a different operator
    Av, _ = _scaled(gpu_system(v, c, prob, p))
    assert rel_sparse_diff(Av, o.Shat) > 1e-6
    x, info = Hierarchy(gq, max_coarse=40).solve(tol=1e-12)
    xo, _ = air_fgmres_solve(o, tol=1e-12, hier=oair.setup(o.Shat, max_coarse=40))
    assert info["converged"]
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
