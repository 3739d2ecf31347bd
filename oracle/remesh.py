"""Oracle remeshing by the phase field and intergrid transfer of nodal fields.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import or call
this module; it checks the library's host-side remeshing and its GPU transfer
against a plain, slow, independently written FP64 implementation.

* Remeshing (the paper refines the interface region |phi| <= 0.95 and
  coarsens away from it as the interface moves, its scaling section; octree
  construction is top-down refinement by a predicate, Sec. 4.2): an octant is
  refined to max_level while the old nodal phase values that lie in its
  half-open box [a, a + s)^d span a range meeting [-thr, thr]; every leaf is
  at least min_level deep; then 2:1 balance.  Old values at hanging nodes are
  their interpolated values (the old mesh's constraint).
* Transfer (the paper's traversal-based intergrid transfer, Sec. 4: copy on
  leaves common to both meshes, evaluation of the old shape functions at the
  child nodes of refined leaves, projection to the parent of coarsened ones):
  every new node takes the value of the old Q1 field at its position.  For a
  coarsened leaf the new corners are old nodes, so the projection reads the
  old nodal values there (injection); we take that reading of "project".
  Evaluated here by testing every old leaf for the point (closed box) and
  summing its corner values times the trilinear shape functions.
"""
from __future__ import annotations

import numpy as np

from . import fem, mesh


def old_node_values(old: mesh.OracleMesh, phi_indep: np.ndarray) -> np.ndarray:
    """Values at every distinct leaf corner of the old mesh (hanging ones
    interpolated)."""
    return fem.all_node_values(old, np.asarray(phi_indep, dtype=np.float64))


def remesh(old: mesh.OracleMesh, phi_indep: np.ndarray, min_level: int, thr: float) -> mesh.OracleMesh:
    vals = old_node_values(old, phi_indep)
    coords = old.nodes
    side = old.side

    def pred(lev, lo, hi):
        a = np.rint(lo * side).astype(np.int64)
        s = side >> lev
        inside = np.all((coords >= a[None, :]) & (coords < a[None, :] + s), axis=1)
        if not inside.any():
            return False
        v = vals[inside]
        return bool(v.max() >= -thr and v.min() <= thr)

    return mesh.from_predicate(old.dim, min_level, old.max_level, pred)


def transfer(old: mesh.OracleMesh, new: mesh.OracleMesh, v_indep: np.ndarray) -> np.ndarray:
    """Old Q1 field (independent nodal values) evaluated at the new mesh's
    independent nodes."""
    if old.dim != new.dim or old.max_level != new.max_level:
        raise ValueError("meshes must share dimension and max_level")
    va = old_node_values(old, v_indep)
    pts = new.indep_coords().astype(np.int64)
    out = np.full(pts.shape[0], np.nan)
    done = np.zeros(pts.shape[0], dtype=bool)
    bits = fem.corner_bits(old.dim)
    size = old.size()
    for e in range(old.n_elems):
        a = old.anchor[e]
        s = size[e]
        inside = ~done & np.all((pts >= a[None, :]) & (pts <= a[None, :] + s), axis=1)
        if not inside.any():
            continue
        xi = (pts[inside] - a[None, :]) / float(s)
        val = np.zeros(xi.shape[0])
        for c in range(1 << old.dim):
            w = np.prod(np.where(bits[c][None, :] == 1, xi, 1.0 - xi), axis=1)
            val += w * va[old.elem_nodes[e, c]]
        out[inside] = val
        done |= inside
    if not done.all():
        raise ValueError("new node outside the old mesh")
    return out
