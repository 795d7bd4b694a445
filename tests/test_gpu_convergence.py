"""Order of convergence of the HIP path on the C1 problem (1+1D, manufactured
u = sin 2 pi (x - t) e^-t, nu = 1e-4): the space-time L2 error of u_h
reconstructed on the GPU from the GPU solution, on the meshes 8^2 ... 128^2,
falls at the rate p + 1 of the HDG method (Section 4.1).  The error is
evaluated with the oracle's quadrature from the GPU's element values; the
FP32 cycle gives the same errors to FP64 accuracy (its solution agrees with
the FP64 one to 1e-8 at tol 1e-12)."""
import numpy as np
import pytest
import torch

from oracle.drivers import setup_problem
from oracle.hdg import l2_error
from gpu_cases import gpu_system
from workloads import square_tri_mesh
from workloads.problems import C1Advection1D

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("p, sizes", [(1, (8, 16, 32, 64, 128)), (2, (8, 16, 32, 64))])
def test_c1_convergence_order_on_gpu(p, sizes):
    from paper_2010_11130_amd import Hierarchy
    prob = C1Advection1D(1e-4)
    errs, errs32 = [], []
    for n in sizes:
        print("case c1 n", n, "p", p, flush=True)
        v, c = square_tri_mesh(n)
        g = gpu_system(v, c, prob, p)
        H = Hierarchy(g, fp32_cycle=1)
        x, info = H.solve(tol=1e-12)
        x32, info32 = H.solve(tol=1e-12, precision=1)
        assert info["converged"] and info32["converged"]
        assert torch.linalg.norm(x32 - x).item() <= 1e-8 * torch.linalg.norm(x).item()
        o = setup_problem(v, c, prob, p)
        errs.append(l2_error(o, g.reconstruct(x).cpu().numpy(), prob.u))
        errs32.append(l2_error(o, g.reconstruct(x32).cpu().numpy(), prob.u))
    errs, errs32 = np.array(errs), np.array(errs32)
    rates = np.log2(errs[:-1] / errs[1:])
    print("errors", errs, "rates", rates, flush=True)
    assert np.all(np.abs(rates - (p + 1)) < 0.25), rates
    assert np.allclose(errs32, errs, rtol=1e-6)
