"""Matched (library mesh, oracle mesh) pairs for parity tests.

Both sides build their own mesh from the same spec; nodes are matched by
exact integer coordinates.  Inputs come from chns_inputs only.
"""
from __future__ import annotations

import numpy as np

import chns_inputs as ci
from oracle import mesh as om


class Pair:
    def __init__(self, kind, dim, lmin, lmax, centre=(0.5, 0.3, 0.5), radius=0.15, band=0.03, brick_max=0):
        from paper_2107_05123_amd import Mesh
        self.kind, self.dim = kind, dim
        c = tuple(centre[:dim])
        if kind == "uniform":
            self.lib = Mesh(dim=dim, min_level=lmax, max_level=lmax, rule="uniform", brick_max=brick_max)
            self.orc = om.uniform(dim, lmax)
        elif kind == "band":
            self.lib = Mesh(dim=dim, min_level=lmin, max_level=lmax, rule="sphere_band", centres=[c],
                            radii=[radius], band=band, brick_max=brick_max)
            self.orc = om.sphere_band(dim, lmin, lmax, c, radius, band)
        else:
            raise ValueError(kind)
        self.max_level = lmax
        side = 1 << lmax
        self.lib_coords = self.lib.node_coords()
        # perm: oracle vector -> library order (lib[i] = orc[perm[i]])
        self.perm = om.node_index_map(self.lib_coords, self.orc.indep_coords(), side)
        self.x_unit = ci.unit_coords(self.lib_coords, lmax)

    def to_lib(self, v_orc):
        return v_orc[self.perm]

    def to_orc(self, v_lib):
        out = np.empty_like(v_lib)
        out[self.perm] = v_lib
        return out

    def phi(self, kind="drops", seed=0, cn=0.01):
        if kind == "drops":
            c, r = ci.drops(seed, dim=self.dim)
            return ci.phi_drops(self.x_unit, c, r, cn)
        if kind == "bubble":
            return ci.phi_bubble(self.x_unit, cn=cn)
        if kind == "drop2d":
            return ci.phi_drop2d(self.x_unit, cn=cn)
        raise ValueError(kind)
