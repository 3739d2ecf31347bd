"""Pins for the oracle's octree mesh (CPU only).

Each expected value below is derived by hand from the geometry (counts of
hanging nodes on a once-refined octant) or is an invariant that any correct
hanging-node interpolation must satisfy (reproduction of constants and linear
fields), so a mistake in the oracle's enumeration shows up here.
"""
import itertools

import numpy as np
import pytest

from oracle import mesh as om


def _refine_one(dim):
    # level-1 tree with the octant at the origin refined once more
    lev, anc = [], []
    for bits in itertools.product((0, 1), repeat=dim):
        a = np.array(bits) * 2
        if not any(bits):
            for b2 in itertools.product((0, 1), repeat=dim):
                lev.append(2)
                anc.append(np.array(b2))
        else:
            lev.append(1)
            anc.append(a)
    return om.from_leaves(dim, 2, lev, anc)


def test_uniform_counts():
    m = om.uniform(3, 2)
    assert m.n_elems == 64
    assert m.n_indep == 125
    assert not m.hanging.any()
    m2 = om.uniform(2, 3)
    assert m2.n_elems == 64 and m2.n_indep == 81


def test_refined_octant_3d_hanging_count():
    # refined octant [0,1/2]^3 inside the level-1 tree: its three interior faces
    # carry 3 face-centre hanging nodes (4 parents) and 9 edge-midpoint hanging
    # nodes (2 parents); the 3 edges through the origin lie on two domain faces
    # and are not hanging.  Independent nodes: 27 coarse + 7 fine = 34.
    m = _refine_one(3)
    assert m.n_elems == 7 + 8
    assert m.nodes.shape[0] == 46
    assert int(m.hanging.sum()) == 12
    assert m.n_indep == 34
    npar = np.diff(m.P.indptr)[m.hanging]
    assert sorted(npar.tolist()) == [2] * 9 + [4] * 3
    w = m.P.data.reshape(-1)
    assert set(np.round(w, 12).tolist()) <= {1.0, 0.5, 0.25}


def test_refined_quad_2d_hanging_count():
    m = _refine_one(2)
    assert int(m.hanging.sum()) == 2
    assert m.n_indep == 12


def test_constraints_reproduce_linear_fields():
    m = om.sphere_band(3, 2, 5, (0.5, 0.3, 0.5), 0.15, 0.03)
    assert m.hanging.any()
    x = m.nodes.astype(np.float64) / m.side
    for coef in ([1.0, 0, 0, 0], [0.3, -1.0, 2.0, 0.5]):
        lin = coef[0] + x @ np.array(coef[1:])
        assert np.allclose(m.P @ lin[m.indep], lin, atol=1e-14, rtol=0)


def test_balance_brute_force():
    # deep refinement around a point close to the edge of a level-1 quadrant puts
    # level-6 leaves next to the unrefined level-1 neighbour across x = 1/2
    p = np.array([0.49, 0.3])

    def pred(lev, lo, hi):
        return bool(np.all((lo <= p) & (p <= hi)))

    lev, anc = om.refine_top_down(2, 1, 6, pred)
    assert not om.is_balanced(lev, anc, 6)
    lev_b, anc_b = om.balance_2to1(lev, anc, 6)
    assert om.is_balanced(lev_b, anc_b, 6)
    # balancing only refines: covered volume is unchanged
    side = 1 << 6
    vol = ((side >> lev_b) ** 2).sum()
    assert vol == side * side


def test_band_mesh_is_balanced_and_parents_independent():
    m = om.sphere_band(3, 2, 5, (0.5, 0.3, 0.5), 0.15, 0.03)
    assert om.is_balanced(m.level, m.anchor, m.max_level)
    par_cols = m.P[m.hanging].indices
    # every parent column maps to an independent node (P is square on indep rows)
    assert np.all(par_cols < m.n_indep)
    assert m.level.min() == 2 and m.level.max() == 5


def test_shell_predicate_exact_cases():
    c = np.array([0.5, 0.5, 0.5])
    # box containing the centre but entirely inside the inner radius
    assert not om.box_meets_shell(np.array([0.45] * 3), np.array([0.55] * 3), c, 0.2, 0.3)
    # box straddling the shell
    assert om.box_meets_shell(np.array([0.7, 0.45, 0.45]), np.array([0.8, 0.55, 0.55]), c, 0.2, 0.3)
    # box outside the outer radius
    assert not om.box_meets_shell(np.array([0.9] * 3), np.array([1.0] * 3), c, 0.2, 0.3)
