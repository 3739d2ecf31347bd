"""Incomplete (carved) octrees (paper Sec. 4: traversals visit only the
octants that exist; Sec. 5.4: the 1 x 8 x 1 Rayleigh-Taylor column), host
side and oracle pins (CPU).

* The library's carved mesh equals the oracle's, leaf for leaf, node for
  node, including hanging nodes and their parents, for a 2D column and the
  3D 1 x 8 x 1 column refined around the Rayleigh-Taylor interface.
* Oracle pins: every leaf lies inside the box and the leaves tile it
  (their volumes sum to the box volume); 2:1 balance by brute force; a box
  equal to the whole cube gives the uncarved mesh; the walls are exactly the
  nodes on the box faces; the pressure operator of a carved mesh with
  hanging nodes is symmetric, has the constants in its null space and passes
  the patch test (A x = 0 at every node off the box faces for a linear x).
* Bad carvings are refused (carve level above min_level, extent beyond the
  cube).
"""
import numpy as np
import pytest

import chns_inputs as ci
from oracle import chns, fem, mesh as om

from .test_host_mesh import _compare


def _rt_pred(width):
    return lambda lev, lo, hi: ci.rt_slab_meets(lo[1], hi[1], width)


def _lib_rt(dim, lmin, lmax, width, carve, extent):
    from paper_2107_05123_amd import Mesh
    side = 1 << lmax
    ext = tuple(extent) + (0,) * (3 - len(extent))

    def refine(anchor, level):
        size = side >> level
        return ci.rt_slab_meets(anchor[1] / side, (anchor[1] + size) / side, width)
    return Mesh(dim=dim, min_level=lmin, max_level=lmax, rule="callback", refine=refine, carve_level=carve,
                extent=ext)


def _box(carve, extent):
    return [e / (1 << carve) for e in extent]


CASES = [(2, 2, 6, 0.6, 2, (1, 4)), (3, 3, 6, 0.5, 3, ci.RT_EXTENT), (3, 3, 5, 1.0, 3, (2, 8, 1))]


@pytest.mark.parametrize("dim,lmin,lmax,width,carve,extent", CASES)
def test_carved_mesh_matches_oracle(dim, lmin, lmax, width, carve, extent):
    lib = _lib_rt(dim, lmin, lmax, width, carve, extent)
    orc = om.from_predicate(dim, lmin, lmax, _rt_pred(width), _box(carve, extent))
    _compare(lib, orc)
    s = lib.summary()
    assert not s["uniform"] and s["n_hanging"] > 0
    assert s["box"] == [e << (lmax - carve) for e in extent]


@pytest.mark.parametrize("dim,lmin,lmax,width,carve,extent", CASES)
def test_oracle_carved_mesh_pins(dim, lmin, lmax, width, carve, extent):
    orc = om.from_predicate(dim, lmin, lmax, _rt_pred(width), _box(carve, extent))
    box = orc.box
    size = orc.size()
    assert np.all(orc.anchor + size[:, None] <= box[None, :])
    assert (size.astype(float) ** dim).sum() == np.prod(box.astype(float))
    assert om.is_balanced(orc.level, orc.anchor, orc.max_level)
    el = chns.Elems(orc)
    c = orc.indep_coords()
    on_face = np.any((c == 0) | (c == box[None, :]), axis=1)
    assert np.array_equal(el.wall(), on_face)
    x = c / orc.side
    phi = ci.phi_rt(x, cn=0.2)
    A = fem.pp_matrix(orc, phi, 1.0, 0.74)
    assert abs(A - A.T).max() <= 1e-14 * abs(A).max()
    assert np.abs(A @ np.ones(orc.n_indep)).max() <= 1e-13 * abs(A).max()
    K = fem.stiffness_matrix(orc)
    lin = c @ np.array([0.3, -1.1, 0.7][:dim])
    assert np.abs((K @ lin)[~on_face]).max() <= 1e-11 * np.abs(lin).max()


def test_full_box_equals_uncarved_mesh():
    a = om.from_predicate(3, 2, 4, _rt_pred(1.0), [1.0, 1.0, 1.0])
    b = om.from_predicate(3, 2, 4, _rt_pred(1.0))
    assert np.array_equal(a.level, b.level) and np.array_equal(a.anchor, b.anchor)
    assert np.array_equal(a.nodes, b.nodes)


def test_bad_carvings_are_refused():
    from paper_2107_05123_amd import Mesh
    from paper_2107_05123_amd._lib import ChnsError
    with pytest.raises(ChnsError):
        Mesh(dim=3, min_level=2, max_level=4, rule="uniform", carve_level=3, extent=(1, 8, 1))
    with pytest.raises(ChnsError):
        Mesh(dim=3, min_level=3, max_level=4, rule="uniform", carve_level=3, extent=(1, 9, 1))
    with pytest.raises(ChnsError):
        Mesh(dim=2, min_level=3, max_level=4, rule="uniform", carve_level=2, extent=(0, 4))
