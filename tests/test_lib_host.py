"""The C-ABI library loads, exports every declared symbol, and its host-side
logic (quadrature rules, mesh topology, argument validation) agrees with the
oracle.  No device work is launched here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle.quad import simplex_rule
from oracle.hdg import Mesh as OMesh
from workloads import square_tri_mesh, slab_prism_tet_mesh, kuhn_cube_mesh, boundary_kinds

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2010_11130_amd._lib import lib, LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.fail("libairhdg.so not built: run __graft_entry__.build()")
    return lib()


def _declared():
    txt = open(os.path.join(ROOT, "include", "airhdg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b(?:ah_status|void|const char\*)\s+(\w+)\s*\(", txt))
    return sorted(names)


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(L, n), n


def test_binding_covers_header():
    from paper_2010_11130_amd._lib import SIGNATURES
    assert set(_declared()) == set(SIGNATURES)


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_quadrature_rule_matches_oracle(L, dim, n):
    from paper_2010_11130_amd.api import quad_rule
    xi, w = quad_rule(dim, n)
    xo, wo = simplex_rule(dim, n)
    assert np.abs(xi - xo).max() < 1e-14
    assert np.abs(w - wo).max() < 1e-15


@pytest.mark.parametrize("mesh", ["tri", "slab", "kuhn"])
def test_mesh_topology_matches_oracle(L, mesh):
    from paper_2010_11130_amd.api import Mesh
    if mesh == "tri":
        v, c = square_tri_mesh(5)
    elif mesh == "slab":
        v, c = slab_prism_tet_mesh(4, 0.25)
    else:
        v, c = kuhn_cube_mesh(3)
    m = Mesh(v, c)
    o = OMesh(v, c)
    fv, fe = m.facets()
    assert m.nf == o.nf
    assert np.array_equal(fv, o.facet_vert)
    # each facet's adjacent cells contain it
    for f in range(0, m.nf, 7):
        for e in fe[f]:
            if e >= 0:
                assert f in o.elem_facet[e]
    assert np.array_equal(np.sort(m.boundary_facets()), np.nonzero(o.is_boundary)[0])
    kinds = boundary_kinds(o.vert, o.facet_vert, o.is_boundary)
    m.set_bc(kinds)


def test_mesh_errors(L):
    from paper_2010_11130_amd.api import Mesh
    from paper_2010_11130_amd._lib import AirHdgError, AH_ESINGULAR, AH_EINVAL
    v = np.array([[0, 0], [1, 0], [2, 0.0]])
    with pytest.raises(AirHdgError) as e:
        Mesh(v, np.array([[0, 1, 2]]))
    assert e.value.status == AH_ESINGULAR
    with pytest.raises(AirHdgError) as e:
        Mesh(v, np.array([[0, 1, 7]]))
    assert e.value.status == AH_EINVAL
    v, c = square_tri_mesh(2)
    m = Mesh(v, c)
    bad = np.zeros(m.nf, dtype=np.int8)          # boundary facets left untagged
    with pytest.raises(AirHdgError) as e:
        m.set_bc(bad)
    assert e.value.status == AH_EINVAL


def test_sizes(L):
    from paper_2010_11130_amd.api import sizes
    assert sizes(2, 1) == (9, 3, 3, 2)
    assert sizes(3, 2) == (64, 16, 10, 6)
    assert sizes(3, 1) == (27, 9, 4, 3)


def test_set_allocator_needs_both_callbacks(L):
    from paper_2010_11130_amd._lib import ALLOC_FN, FREE_FN, AH_EINVAL, AH_OK
    keep = ALLOC_FN(lambda ctx, n, s: None)
    assert L.ah_set_allocator(keep, FREE_FN(), None) == AH_EINVAL
    assert b"both" in L.ah_last_error()
    assert L.ah_set_allocator(ALLOC_FN(), FREE_FN(), None) == AH_OK
