"""The library's RT numbering of unstructured hexahedral meshes (host code,
no GPU) against the oracle's (Section 3.2, Algorithm 1: element-to-dof index
arrays with orientation signs): the same global dof and the same sign for
every local dof of every element, on a structured mesh renumbered and turned
element by element, and on an O-grid mesh whose central corners join three
elements in the cross-section; and the element-array errors."""
import numpy as np
import pytest

from oracle import unstructured as un
from paper_2304_12387_amd import inputs


def lib():
    from paper_2304_12387_amd import hdivsp
    return hdivsp


def _compare(V, el, p):
    m = un.HexMesh(V, el, p)
    nu, l2g = lib().host_unstructured_map(V.shape[0], el, p)
    assert nu == m.n_u
    g = np.where(l2g < 0, ~l2g, l2g)
    s = np.where(l2g < 0, -1, 1)
    assert np.array_equal(g, m.l2g)
    assert np.array_equal(s, m.sgn.astype(int))
    return m


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_numbering_of_a_scrambled_structured_mesh(p):
    V = inputs.jittered_vertices(3, 2, 2, 0.1, 7)
    Vv, el = inputs.from_structured(3, 2, 2, V)
    V2, el2, _ = inputs.scramble(Vv, el, 11 + p)
    m = _compare(V2, el2, p)
    assert (m.sgn < 0).any()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_numbering_of_an_o_grid_mesh(p):
    V, el = inputs.o_grid(2, 1, 2, seed=3)
    _compare(V, el, p)


def test_element_array_errors():
    h = lib()
    V, el = inputs.o_grid(2, 1, 1, seed=3)
    bad = el.copy()
    bad[0, 0] = V.shape[0]                     # vertex number out of range
    with pytest.raises(h.HdError):
        h.host_unstructured_map(V.shape[0], bad, 2)
    rep = el.copy()
    rep[0, 1] = rep[0, 0]                      # a face with a repeated vertex
    with pytest.raises(h.HdError):
        h.host_unstructured_map(V.shape[0], rep, 2)
    three = np.concatenate([el, el[:1]])       # the first element twice: faces shared by 3+ elements
    with pytest.raises(h.HdError):
        h.host_unstructured_map(V.shape[0], three, 2)
