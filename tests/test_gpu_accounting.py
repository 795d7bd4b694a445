"""The algorithmic bytes the library reports for its level-0 relaxation
sweeps: these figures are the numerators of the roofline entry of the
measurement.  They are recounted here from the exported level-0 matrix and
its C/F splitting.  The count for a sweep over the rows X: each value of the
off-diagonal blocks of X once (the diagonal blocks, identities after the
facet-block scaling, are not stored in the facet-block layout), one int32
column index per off-diagonal block, one int64 offset per block row, one
int32 per row of the X list, x once, b on X and the updates of X written
(twice on the second F sweep, which also fills the cycle's output)."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_cases import case, gpu_system
from workloads import slab_prism_tet_mesh
from workloads.problems import slab_hill

pytestmark = pytest.mark.gpu


def _block_size(D, p):
    return p + 1 if D == 2 else (p + 1) * (p + 2) // 2


def _expected(lv, b):
    rp = lv["rowptr"].cpu().numpy()
    cf = lv["cf"].cpu().numpy()
    n = lv["n"]
    # a scaled row holds its diagonal entry (1) and its off-diagonal blocks
    off = np.diff(rp) - 1
    assert np.all(off % b == 0)
    nob = off // b
    # the scalar rows of one block row share its block pattern
    assert np.all(nob.reshape(-1, b) == nob[::b, None])
    off_blocks = int(nob[::b].sum())
    F = cf == 0
    nF, nC = int(F.sum()), int((~F).sum())
    vF = int(off[F].sum())
    vC = int(off[~F].sum())
    common = off_blocks * 4 + (n // b + 1) * 8 + n * 8
    f_first = vF * 8 + common + nF * 4 + nF * 2 * 8
    f_second = vF * 8 + common + nF * 4 + nF * 3 * 8
    c_sweep = vC * 8 + common + nC * 4 + nC * 2 * 8
    return f_first + f_second, c_sweep


def _profiled_cycle(H, n):
    from paper_2010_11130_amd import lib
    r = torch.as_tensor(np.random.default_rng(2).standard_normal(n), device="cuda")
    lib().ah_profile_reset()
    lib().ah_profile_enable(1)
    H.vcycle(r)
    torch.cuda.synchronize()
    lib().ah_profile_enable(0)
    out = {}
    for tag in ("relax0_f", "relax0_c"):
        k, ms, by = C.c_int64(), C.c_double(), C.c_double()
        lib().ah_profile_read(tag.encode(), C.byref(k), C.byref(ms), C.byref(by))
        out[tag] = (k.value, by.value)
    lib().ah_profile_reset()
    return out


def _check(g, D, p):
    from paper_2010_11130_amd import Hierarchy
    H = Hierarchy(g)
    lv = H.level(0)
    f_pair, c_sweep = _expected(lv, _block_size(D, p))
    got = _profiled_cycle(H, lv["n"])
    assert got["relax0_f"] == (2, float(f_pair))
    assert got["relax0_c"] == (1, float(c_sweep))
    return f_pair / 2


@pytest.mark.parametrize("name", ["slab", "kuhn_nu4", "c1"])
def test_level0_sweep_bytes(name):
    print("case", name, flush=True)
    v, c, prob, p = case(name)
    _check(gpu_system(v, c, prob, p), v.shape[1], p)


def test_level0_sweep_bytes_c2_slab():
    """The full-size slab (64 x 64 quads, one time step of 1/64, p = 2): the
    per-launch figure of the F sweep that the measurement divides by."""
    print("case c2 slab", flush=True)
    v, c = slab_prism_tet_mesh(64, 1.0 / 64)
    per_launch = _check(gpu_system(v, c, slab_hill(1e-4), 2), 3, 2)
    assert per_launch == 75182792.0
