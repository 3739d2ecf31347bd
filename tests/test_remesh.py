"""Remeshing by the phase field and intergrid transfer (host logic, no GPU).

Oracle pins (independent of the oracle's own arithmetic):
* Q1 reproduces linear fields, so transferring a linear field onto any mesh
  gives the linear field at the new nodes (leaf location, shape functions and
  hanging-node values all enter);
* transfer onto the same mesh is the identity (copy);
* refining everywhere and coming back is the identity (injection undoes
  interpolation at the coarse nodes);
* every leaf of a remeshed mesh whose half-open box holds an old node with
  |phi| <= thr is at max_level (the refinement criterion itself).
Library against oracle: the remeshed leaves are identical; the library's
transfer matrix reproduces the oracle's point values to 1e-14.
"""
import numpy as np
import pytest

import chns_inputs as ci
from oracle import mesh as om
from oracle import remesh as orm

from ._pairs import Pair

THR = 0.95


def _bubble(pair, cn, centre):
    x = pair.x_unit
    c = np.asarray(centre[:pair.dim])
    r = 0.15
    d = np.sqrt(((x - c[None, :]) ** 2).sum(axis=1)) - r
    return np.tanh(d / (np.sqrt(2.0) * cn))


def _leaf_set(level, anchor):
    return {(int(l),) + tuple(int(v) for v in a) for l, a in zip(level, anchor)}


def _oracle_values_on(orc_mesh, lib_mesh, v_orc_new, side):
    """Oracle vector on `orc_mesh` reordered to `lib_mesh` node order."""
    perm = om.node_index_map(lib_mesh.node_coords(), orc_mesh.indep_coords(), side)
    return v_orc_new[perm]


CASES = [(2, 3, 7, 0.02), (3, 2, 5, 0.04)]


@pytest.mark.parametrize("dim,lmin,lmax,cn", CASES)
def test_oracle_transfer_pins(dim, lmin, lmax, cn):
    old = om.sphere_band(dim, lmin, lmax, (0.5, 0.3, 0.5)[:dim], 0.15, 0.05)
    x = old.indep_coords() / float(old.side)
    phi = np.tanh((np.sqrt(((x - np.array([0.5, 0.36, 0.5])[:dim]) ** 2).sum(1)) - 0.15) / (np.sqrt(2) * cn))
    new = orm.remesh(old, phi, lmin, THR)
    # linear fields are reproduced exactly (to rounding)
    a = np.array([0.3, -0.7, 1.1])[:dim]
    lin_old = x @ a + 0.25
    lin_new = orm.transfer(old, new, lin_old)
    xn = new.indep_coords() / float(new.side)
    assert np.abs(lin_new - (xn @ a + 0.25)).max() <= 1e-14
    # copy onto the same mesh
    v = np.asarray(ci.normal_vector(4, old.n_indep))
    assert np.array_equal(orm.transfer(old, old, v), v)
    # refine everywhere and back: identity
    fine = om.uniform(dim, lmax)
    back = orm.transfer(fine, old, orm.transfer(old, fine, v))
    assert np.abs(back - v).max() <= 1e-15 * np.abs(v).max()
    # refinement criterion: leaves holding an old node with |phi| <= thr are finest
    vals = orm.old_node_values(old, phi)
    size = new.size()
    for lev, anc, s in zip(new.level, new.anchor, size):
        inside = np.all((old.nodes >= anc) & (old.nodes < anc + s), axis=1)
        if np.any(np.abs(vals[inside]) <= THR):
            assert lev == lmax


@pytest.mark.parametrize("dim,lmin,lmax,cn", CASES)
def test_library_remesh_and_transfer_match_oracle(dim, lmin, lmax, cn):
    from paper_2107_05123_amd import Transfer
    pair = Pair("band", dim, lmin, lmax, band=0.05)
    side = 1 << lmax
    # the interface moved up by 0.06: remesh around the new position
    phi = _bubble(pair, cn, (0.5, 0.36, 0.5))
    new_lib = pair.lib.remesh(phi, lmin, THR)
    new_orc = orm.remesh(pair.orc, pair.to_orc(phi), lmin, THR)
    lev_l, anc_l = new_lib.leaves()
    assert _leaf_set(lev_l, anc_l) == _leaf_set(new_orc.level, new_orc.anchor)
    print(f"{dim}d: {pair.lib.n_elems} -> {new_lib.n_elems} leaves, {new_lib.n_nodes} nodes", flush=True)
    # transfer matrix against the oracle's point values, several fields
    t = Transfer(pair.lib, new_lib)
    assert (t.rows, t.cols) == (new_lib.n_nodes, pair.lib.n_nodes)
    ptr, col, val = t.matrix()
    import scipy.sparse as sp
    P = sp.csr_matrix((val, col, ptr), shape=(t.rows, t.cols))
    for v in (phi, np.asarray(ci.normal_vector(5, pair.lib.n_nodes))):
        got = P @ v
        ref = _oracle_values_on(new_orc, new_lib, orm.transfer(pair.orc, new_orc, pair.to_orc(v)), side)
        assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
    # every row sums to one (partition of unity) and weights lie in [0, 1]
    assert np.abs(np.asarray(P.sum(axis=1)).ravel() - 1.0).max() <= 1e-15
    assert val.min() >= 0.0 and val.max() <= 1.0


def test_remesh_rejects_bad_arguments():
    from paper_2107_05123_amd import Mesh, Transfer
    from paper_2107_05123_amd import _lib as L
    m = Mesh(dim=2, min_level=2, max_level=4, rule="uniform")
    phi = np.zeros(m.n_nodes)
    with pytest.raises(L.ChnsError) as e:
        m.remesh(phi, 5, THR)  # min_level above max_level
    assert e.value.code == L.EINVAL
    other = Mesh(dim=2, min_level=3, max_level=3, rule="uniform")
    with pytest.raises(L.ChnsError) as e:
        Transfer(m, other)  # different max_level
    assert e.value.code == L.EINVAL
