"""Oracle octree mesh: refinement, 2:1 vertex balance, nodes, hanging constraints.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import or call
this package; it exists so that the GPU path can be checked against a plain,
slow, independently written FP64 implementation.

What is built here follows the paper's octree section (Sec. 4):
* top-down refinement of the unit cube by a user predicate on the octant
  (Sec. 4.2), starting at the root;
* 2:1 balance between neighbouring leaves (Sec. 4.2); we read "neighbouring"
  as sharing at least a vertex;
* independent nodes = leaf corners that are not hanging; a corner is hanging
  when it lies on the boundary of a touching coarser leaf without being one of
  that leaf's corners (Sec. 4.3), and its value is interpolated from that
  leaf's trilinear field (Fig. 1 caption: hanging values come from the
  immediate parent).  The interpolation weights are the coarse leaf's Q1 shape
  functions evaluated at the hanging point.

Coordinates are integers in units of 2^-max_level, so every comparison is
exact.  Everything is brute force: point location by testing every level.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


def _encode(ijk: np.ndarray, side: int) -> np.ndarray:
    """Injective int64 key of integer points with coordinates in [0, side]."""
    ijk = np.asarray(ijk, dtype=np.int64)
    key = np.zeros(ijk.shape[0], dtype=np.int64)
    for d in range(ijk.shape[1] - 1, -1, -1):
        key = key * (side + 1) + ijk[:, d]
    return key


@dataclass
class OracleMesh:
    dim: int
    max_level: int
    level: np.ndarray                 # (E,) leaf levels
    anchor: np.ndarray                # (E, dim) integer lower corners
    nodes: np.ndarray = None          # (N_all, dim) every distinct leaf corner
    elem_nodes: np.ndarray = None     # (E, 2^dim) indices into `nodes`
    hanging: np.ndarray = None        # (N_all,) bool
    indep: np.ndarray = None          # (N_ind,) indices into `nodes` of independent nodes
    P: sp.csr_matrix = None           # (N_all, N_ind) hanging interpolation
    extra: dict = field(default_factory=dict)
    box_hi: np.ndarray = None         # (dim,) domain box in units of 2^-max_level; None: whole cube

    @property
    def n_elems(self) -> int:
        return int(self.level.shape[0])

    @property
    def n_indep(self) -> int:
        return int(self.indep.shape[0])

    @property
    def side(self) -> int:
        return 1 << self.max_level

    def size(self) -> np.ndarray:
        """Integer edge length of every leaf."""
        return (1 << (self.max_level - self.level)).astype(np.int64)

    def indep_coords(self) -> np.ndarray:
        return self.nodes[self.indep]

    @property
    def box(self) -> np.ndarray:
        """Upper corner of the domain box (integer units of 2^-max_level)."""
        return np.full(self.dim, self.side, dtype=np.int64) if self.box_hi is None else self.box_hi


# ---------------------------------------------------------------- refinement
def box_meets_shell(lo: np.ndarray, hi: np.ndarray, centre, r_in: float, r_out: float) -> bool:
    """True if the closed box [lo, hi] meets {x : r_in <= |x - c| <= r_out}."""
    dmin2 = 0.0
    dmax2 = 0.0
    for d in range(len(lo)):
        c = centre[d]
        nearest = min(max(c, lo[d]), hi[d])
        dmin2 += (nearest - c) * (nearest - c)
        far = max(abs(lo[d] - c), abs(hi[d] - c))
        dmax2 += far * far
    if dmin2 > r_out * r_out:
        return False
    if r_in > 0.0 and dmax2 < r_in * r_in:
        return False
    return True


def refine_top_down(dim: int, min_level: int, max_level: int, predicate=None, box=None):
    """Leaves of the tree refined to min_level everywhere and, where the
    predicate(level, lo, hi) holds, further down to max_level.  box: the
    domain of an incomplete (carved) octree in unit coordinates, a union of
    octants no finer than min_level; octants whose lower corner lies outside
    it do not exist (paper Sec. 4: traversals visit only existing octants)."""
    side = 1 << max_level
    out_level, out_anchor = [], []
    stack = [(0, (0,) * dim)]
    while stack:
        lev, anc = stack.pop()
        size = side >> lev
        if box is not None and lev >= min_level and any(a / side >= b for a, b in zip(anc, box)):
            continue
        refine = lev < min_level
        if not refine and lev < max_level and predicate is not None:
            lo = np.array(anc, dtype=np.float64) / side
            hi = (np.array(anc, dtype=np.float64) + size) / side
            refine = bool(predicate(lev, lo, hi))
        if refine:
            half = size // 2
            for bits in itertools.product((0, 1), repeat=dim):
                stack.append((lev + 1, tuple(a + b * half for a, b in zip(anc, bits))))
        else:
            out_level.append(lev)
            out_anchor.append(anc)
    return np.array(out_level, dtype=np.int64), np.array(out_anchor, dtype=np.int64).reshape(-1, dim)


class _Locator:
    """Find the leaf that contains points given in doubled coordinates."""

    def __init__(self, level, anchor, max_level):
        self.max_level = max_level
        self.dim = anchor.shape[1]
        self.side2 = 2 << max_level  # doubled side
        self.by_level = {}
        for lev in np.unique(level):
            idx = np.nonzero(level == lev)[0]
            keys = _encode(2 * anchor[idx], self.side2)
            order = np.argsort(keys)
            self.by_level[int(lev)] = (keys[order], idx[order])

    def locate(self, p2: np.ndarray) -> np.ndarray:
        """Leaf index containing each doubled point (strictly inside the domain)."""
        res = np.full(p2.shape[0], -1, dtype=np.int64)
        for lev, (keys, idx) in self.by_level.items():
            s2 = 2 << (self.max_level - lev)
            anc2 = (p2 // s2) * s2
            k = _encode(anc2, self.side2)
            pos = np.searchsorted(keys, k)
            pos = np.minimum(pos, keys.shape[0] - 1)
            hit = keys[pos] == k
            res[hit] = idx[pos[hit]]
        return res


def balance_2to1(level, anchor, max_level, box_hi=None):
    """Vertex 2:1 balance by repeated refinement of too-coarse neighbours
    (neighbours only inside the domain box, integer units)."""
    dim = anchor.shape[1]
    side = 1 << max_level
    hi2 = 2 * (np.full(dim, side) if box_hi is None else np.asarray(box_hi))
    dirs = np.array([d for d in itertools.product((-1, 0, 1), repeat=dim) if any(d)], dtype=np.int64)
    while True:
        loc = _Locator(level, anchor, max_level)
        size = (1 << (max_level - level)).astype(np.int64)
        marked = np.zeros(level.shape[0], dtype=bool)
        for d in dirs:
            # centre of the same-size neighbour in direction d, doubled coordinates
            c2 = 2 * anchor + (2 * d[None, :] + 1) * size[:, None]
            inside = np.all((c2 > 0) & (c2 < hi2[None, :]), axis=1)
            src = np.nonzero(inside)[0]
            nb = loc.locate(c2[src])
            too_coarse = level[nb] < level[src] - 1
            marked[nb[too_coarse]] = True
        if not marked.any():
            return level, anchor
        keep = ~marked
        new_level = [level[keep]]
        new_anchor = [anchor[keep]]
        half = (size[marked] // 2)[:, None]
        for bits in itertools.product((0, 1), repeat=dim):
            new_level.append(level[marked] + 1)
            new_anchor.append(anchor[marked] + np.array(bits)[None, :] * half)
        level = np.concatenate(new_level)
        anchor = np.concatenate(new_anchor)


def is_balanced(level, anchor, max_level) -> bool:
    """Brute-force check: every pair of touching leaves differs by <= 1 level."""
    n = level.shape[0]
    size = (1 << (max_level - level)).astype(np.int64)
    lo = anchor
    hi = anchor + size[:, None]
    for i in range(n):
        touch = np.all((lo <= hi[i][None, :]) & (hi >= lo[i][None, :]), axis=1)
        if np.any(np.abs(level[touch] - level[i]) > 1):
            return False
    return True


# ------------------------------------------------------------- node numbering
def enumerate_nodes(mesh: OracleMesh) -> OracleMesh:
    dim, L = mesh.dim, mesh.max_level
    side = 1 << L
    size = mesh.size()
    # corner a has bit d = (a >> d) & 1, i.e. x varies fastest
    corners = np.array([[(a >> d) & 1 for d in range(dim)] for a in range(1 << dim)], dtype=np.int64)
    allc = mesh.anchor[:, None, :] + corners[None, :, :] * size[:, None, None]  # (E, 2^d, dim)
    flat = allc.reshape(-1, dim)
    keys = _encode(flat, side)
    ukeys, first, inv = np.unique(keys, return_index=True, return_inverse=True)
    nodes = flat[first]
    mesh.nodes = nodes
    mesh.elem_nodes = inv.reshape(mesh.n_elems, 1 << dim)

    # hanging detection: look at the 2^dim points diagonally around each node
    loc = _Locator(mesh.level, mesh.anchor, L)
    n_all = nodes.shape[0]
    hang_leaf = np.full(n_all, -1, dtype=np.int64)
    hi2 = 2 * mesh.box
    for o in itertools.product((-1, 1), repeat=dim):
        p2 = 2 * nodes + np.array(o)[None, :]
        inside = np.all((p2 > 0) & (p2 < hi2[None, :]), axis=1)
        src = np.nonzero(inside)[0]
        leaf = loc.locate(p2[src])
        rel = nodes[src] - mesh.anchor[leaf]
        s = size[leaf][:, None]
        at_corner = np.all((rel == 0) | (rel == s), axis=1)
        hang_leaf[src[~at_corner]] = leaf[~at_corner]
    hanging = hang_leaf >= 0
    mesh.hanging = hanging
    mesh.indep = np.nonzero(~hanging)[0]
    ind_of = np.full(n_all, -1, dtype=np.int64)
    ind_of[mesh.indep] = np.arange(mesh.indep.shape[0])

    rows, cols, vals = [], [], []
    rows.append(mesh.indep)
    cols.append(np.arange(mesh.indep.shape[0]))
    vals.append(np.ones(mesh.indep.shape[0]))
    hidx = np.nonzero(hanging)[0]
    if hidx.size:
        leaf = hang_leaf[hidx]
        s = size[leaf].astype(np.float64)
        xi = (nodes[hidx] - mesh.anchor[leaf]) / s[:, None]          # in [0,1]^dim
        for a in range(1 << dim):
            bits = corners[a]
            w = np.prod(np.where(bits[None, :] == 1, xi, 1.0 - xi), axis=1)
            par = mesh.elem_nodes[leaf, a]
            nz = w > 0
            if np.any(hanging[par[nz]]):
                raise RuntimeError("constraint parent is itself hanging: mesh not 2:1 balanced")
            rows.append(hidx[nz])
            cols.append(ind_of[par[nz]])
            vals.append(w[nz])
    mesh.P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                           shape=(n_all, mesh.indep.shape[0]))
    return mesh


# ------------------------------------------------------------------ builders
def uniform(dim: int, level: int) -> OracleMesh:
    n = 1 << level
    grids = np.meshgrid(*([np.arange(n, dtype=np.int64)] * dim), indexing="ij")
    anchor = np.stack([g.ravel() for g in grids], axis=1)
    lev = np.full(anchor.shape[0], level, dtype=np.int64)
    m = OracleMesh(dim=dim, max_level=level, level=lev, anchor=anchor)
    return enumerate_nodes(m)


def from_predicate(dim: int, min_level: int, max_level: int, predicate, box=None) -> OracleMesh:
    """box: optional carved domain [0, box[d]] (unit coordinates, a union of
    octants no finer than min_level)."""
    lev, anc = refine_top_down(dim, min_level, max_level, predicate, box)
    box_hi = None if box is None else np.array([round(b * (1 << max_level)) for b in box], dtype=np.int64)
    lev, anc = balance_2to1(lev, anc, max_level, box_hi)
    m = OracleMesh(dim=dim, max_level=max_level, level=lev, anchor=anc, box_hi=box_hi)
    return enumerate_nodes(m)


def sphere_band(dim: int, min_level: int, max_level: int, centre, radius: float, band: float,
                box=None) -> OracleMesh:
    """Refine to max_level every octant meeting radius-band <= |x-c| <= radius+band."""
    c = np.asarray(centre, dtype=np.float64)[:dim]

    def pred(lev, lo, hi):
        return box_meets_shell(lo, hi, c, radius - band, radius + band)

    return from_predicate(dim, min_level, max_level, pred, box)


def carved_uniform(dim: int, level: int, box) -> OracleMesh:
    """Every leaf at `level` inside the box (an incomplete octree)."""
    return from_predicate(dim, level, level, None, box)


def from_leaves(dim: int, max_level: int, level, anchor) -> OracleMesh:
    m = OracleMesh(dim=dim, max_level=max_level, level=np.asarray(level, dtype=np.int64),
                   anchor=np.asarray(anchor, dtype=np.int64).reshape(-1, dim))
    return enumerate_nodes(m)


def node_index_map(coords_a: np.ndarray, coords_b: np.ndarray, side: int) -> np.ndarray:
    """perm such that coords_b[perm] == coords_a (exact integer matching)."""
    ka = _encode(coords_a, side)
    kb = _encode(coords_b, side)
    order = np.argsort(kb)
    pos = np.searchsorted(kb[order], ka)
    perm = order[np.minimum(pos, kb.shape[0] - 1)]
    if not np.array_equal(kb[perm], ka):
        raise ValueError("node sets differ")
    return perm
