"""MI355X-native matrix-free hot path of the projection-based semi-implicit
Cahn-Hilliard Navier-Stokes solver on adaptive octrees.

Thin Python binding over libchns (include/chns.h): argument marshalling only.
Every step of the hot path runs in the library's HIP kernels; PyTorch provides
device memory and the current stream.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib as L
from ._lib import ChnsError  # noqa: F401

__all__ = ["Mesh", "Context", "ChnsError", "octree_build"]

# pressure solve modes: FP64, FP64 refinement around FP32 CG restarted at
# every step, or continuing its search direction across the steps
_MODES = {"fp64": L.MODE_FP64, "mixed": L.MODE_MIXED_IR, "mixed_ru": L.MODE_MIXED_RU}


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_ptr(t, dtype, numel=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


class Mesh:
    """A 2:1-balanced octree on the unit cube (or square) with its independent
    nodes, hanging constraints and brick decomposition (built on the host)."""

    def __init__(self, dim=3, min_level=0, max_level=5, rule="uniform", centres=None, radii=None,
                 band=0.0, refine=None, brick_max=0, carve_level=0, extent=(0, 0, 0)):
        lib = L.lib()
        spec = L.MeshSpec()
        spec.dim, spec.min_level, spec.max_level = dim, min_level, max_level
        rules = {"uniform": L.RULE_UNIFORM, "sphere_band": L.RULE_SPHERE_BAND,
                 "multi_sphere_band": L.RULE_MULTI_SPHERE_BAND, "callback": L.RULE_CALLBACK}
        spec.rule = rules[rule]
        self._keep = []
        if centres is not None:
            c = np.ascontiguousarray(np.asarray(centres, dtype=np.float64).reshape(-1, dim))
            r = np.ascontiguousarray(np.asarray(radii, dtype=np.float64).reshape(-1))
            self._keep += [c, r]
            spec.n_spheres = r.shape[0]
            spec.centres = c.ctypes.data_as(C.POINTER(C.c_double))
            spec.radii = r.ctypes.data_as(C.POINTER(C.c_double))
        spec.band = band
        spec.brick_max = int(brick_max)
        spec.carve_level = int(carve_level)
        for d, e in enumerate(tuple(extent)[:3]):
            spec.extent[d] = int(e)
        if refine is not None:
            def _cb(anchor, level, user):
                return int(bool(refine([anchor[i] for i in range(3)], level)))
            cb = L.REFINE_CB(_cb)
            self._keep.append(cb)
            spec.refine = cb
        else:
            spec.refine = L.REFINE_CB()
        h = C.c_void_p()
        L.check(lib.chns_octree_build(C.byref(spec), C.byref(h)))
        self._h = h
        self._destroy = L.lib().chns_mesh_destroy
        self.dim = dim
        self.info = self._info()

    def _info(self):
        info = L.MeshInfo()
        L.check(L.lib().chns_mesh_info_get(self._h, C.byref(info)))
        return info

    @classmethod
    def _wrap(cls, h, dim):
        m = cls.__new__(cls)
        m._keep = []
        m._h = h
        m._destroy = L.lib().chns_mesh_destroy
        m.dim = dim
        m.info = m._info()
        return m

    def remesh(self, phi, min_level, threshold=0.95, brick_max=0) -> "Mesh":
        """New mesh refined to max_level where the nodal phase field (host
        array in this mesh's vector order) meets |phi| <= threshold."""
        p = np.ascontiguousarray(np.asarray(phi, dtype=np.float64).reshape(-1))
        if p.shape[0] != self.n_nodes:
            raise ValueError("phi must have one value per node")
        h = C.c_void_p()
        L.check(L.lib().chns_mesh_remesh(self._h, p.ctypes.data_as(C.c_void_p), int(min_level), float(threshold),
                                         int(brick_max), C.byref(h)))
        return Mesh._wrap(h, self.dim)

    @property
    def n_nodes(self) -> int:
        return int(self.info.n_nodes)

    @property
    def n_elems(self) -> int:
        return int(self.info.n_elems)

    @property
    def max_level(self) -> int:
        return int(self.info.max_level)

    def node_coords(self) -> np.ndarray:
        out = np.empty((self.n_nodes, self.dim), dtype=np.int64)
        L.check(L.lib().chns_mesh_node_coords(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def leaves(self):
        lev = np.empty(self.n_elems, dtype=np.int32)
        anc = np.empty((self.n_elems, self.dim), dtype=np.int64)
        L.check(L.lib().chns_mesh_leaves(self._h, lev.ctypes.data_as(C.c_void_p), anc.ctypes.data_as(C.c_void_p)))
        return lev, anc

    def hanging(self):
        n = int(self.info.n_hanging)
        coords = np.empty((n, self.dim), dtype=np.int64)
        par = np.empty((n, 4), dtype=np.int32)
        if n:
            L.check(L.lib().chns_mesh_hanging(self._h, coords.ctypes.data_as(C.c_void_p),
                                              par.ctypes.data_as(C.c_void_p)))
        return coords, par

    def summary(self) -> dict:
        i = self.info
        return {"dim": i.dim, "max_level": i.max_level, "uniform": bool(i.uniform), "n_elems": i.n_elems,
                "n_nodes": i.n_nodes, "n_hanging": i.n_hanging, "n_bricks": list(i.n_bricks),
                "elems_in_bricks": list(i.elems_in_bricks), "n_slots": i.n_slots, "n_shared": i.n_shared,
                "n_colors": i.n_colors, "level_counts": {l: c for l, c in enumerate(i.level_counts) if c},
                "box": list(i.box)[:self.dim]}

    def __del__(self):
        # only attributes of the object itself: module globals may already be
        # gone when this runs at interpreter shutdown
        h = getattr(self, "_h", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and h.value and destroy is not None:
            destroy(h)
            h.value = None


def octree_build(**kw) -> Mesh:
    return Mesh(**kw)


class Transfer:
    """Intergrid transfer of nodal fields from one mesh to another (same
    dimension and max_level): each node of `dst` takes the Q1 field of `src`
    at its position."""

    def __init__(self, src: Mesh, dst: Mesh):
        h = C.c_void_p()
        L.check(L.lib().chns_transfer_create(src._h, dst._h, C.byref(h)))
        self._h = h
        self._destroy = L.lib().chns_transfer_destroy
        r, c, z = C.c_int64(), C.c_int64(), C.c_int64()
        L.check(L.lib().chns_transfer_info(h, C.byref(r), C.byref(c), C.byref(z)))
        self.rows, self.cols, self.nnz = r.value, c.value, z.value

    def matrix(self):
        """(ptr, col, val) of the CSR on the host."""
        ptr = np.empty(self.rows + 1, dtype=np.int32)
        col = np.empty(max(self.nnz, 1), dtype=np.int32)
        val = np.empty(max(self.nnz, 1), dtype=np.float64)
        L.check(L.lib().chns_transfer_matrix(self._h, ptr.ctypes.data_as(C.c_void_p),
                                             col.ctypes.data_as(C.c_void_p), val.ctypes.data_as(C.c_void_p)))
        return ptr, col[:self.nnz], val[:self.nnz]

    def apply(self, x, n_fields=1, y=None, stream=None):
        import torch
        if y is None:
            y = torch.empty(n_fields * self.rows, dtype=torch.float64, device=x.device)
        L.check(L.lib().chns_transfer_apply(self._h, int(n_fields), _dev_ptr(x, torch.float64, n_fields * self.cols),
                                            _dev_ptr(y, torch.float64, n_fields * self.rows), _stream_ptr(stream)))
        return y

    def __del__(self):
        h = getattr(self, "_h", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and h.value and destroy is not None:
            destroy(h)
            h.value = None


@dataclass
class SolveStats:
    iterations: int
    outer_iterations: int
    rel_residual: float
    ms_setup: float
    ms_solve: float
    fallback: int
    status: int


class Context:
    """Device state for one mesh and parameter set (uploads the mesh to the
    current device)."""

    PRESSURE, MOMENTUM, CH_JACOBIAN, MASS_RHO, MASS, MOMENTUM_SCALAR = (
        L.OP_PRESSURE, L.OP_MOMENTUM, L.OP_CH_JACOBIAN, L.OP_MASS_RHO, L.OP_MASS, L.OP_MOMENTUM_SCALAR)

    def __init__(self, mesh: Mesh, Re=100.0, We=1.0, Cn=0.01, Pe=0.0, Fr=1.0, rho_plus=1.0, rho_minus=1.0,
                 eta_plus=1.0, eta_minus=1.0, dt=1e-3, C_I=6.0, gravity_axis=1):
        self.mesh = mesh
        p = L.Params(Re, We, Cn, Pe, Fr, rho_plus, rho_minus, eta_plus, eta_minus, dt, C_I, gravity_axis)
        self.params = p
        h = C.c_void_p()
        L.check(L.lib().chns_context_create(mesh._h, C.byref(p), C.byref(h)))
        self._h = h
        self._destroy = L.lib().chns_context_destroy
        self.n = mesh.n_nodes
        self.dim = mesh.dim

    def fields(self, op: int) -> int:
        return {L.OP_PRESSURE: 1, L.OP_MASS: 1, L.OP_MASS_RHO: self.dim, L.OP_MOMENTUM: self.dim,
                L.OP_CH_JACOBIAN: 2, L.OP_MOMENTUM_SCALAR: 1}[op]

    def set_phase_field(self, phi, phi_prev=None, stream=None):
        import torch
        pp = _dev_ptr(phi_prev, torch.float64, self.n) if phi_prev is not None else C.c_void_p()
        L.check(L.lib().chns_set_phase_field(self._h, _dev_ptr(phi, torch.float64, self.n), pp,
                                             _stream_ptr(stream)))

    def apply(self, op, x, y=None, prec=None, stream=None):
        import torch
        dt = x.dtype
        if prec is None:
            prec = L.FP64 if dt == torch.float64 else L.FP32
        want = torch.float64 if prec == L.FP64 else torch.float32
        nf = self.fields(op)
        if y is None:
            y = torch.empty(nf * self.n, dtype=want, device=x.device)
        L.check(L.lib().chns_apply_operator(self._h, op, prec, _dev_ptr(x, want, nf * self.n),
                                            _dev_ptr(y, want, nf * self.n), _stream_ptr(stream)))
        return y

    def diagonal(self, op, prec=L.FP64, stream=None):
        import torch
        want = torch.float64 if prec == L.FP64 else torch.float32
        d = torch.empty(self.fields(op) * self.n, dtype=want, device="cuda")
        L.check(L.lib().chns_operator_diagonal(self._h, op, prec, _dev_ptr(d, want), _stream_ptr(stream)))
        return d

    def solve_pressure(self, b, x=None, rtol=1e-8, max_it=20000, pc="jacobi", mode="fp64", inner_rtol=None,
                       check_every=16, max_outer=30, graphs=True, learned_every=0, stream=None,
                       raise_on_noconv=True):
        import torch
        if x is None:
            x = torch.zeros_like(b)
        if inner_rtol is None:
            inner_rtol = 1e-2 if mode == "mixed_ru" else 1e-4
        o = L.SolveOpts(rtol, max_it, {"jacobi": L.PC_JACOBI, "gmg": L.PC_GMG, "learned": L.PC_LEARNED,
                                       "none": L.PC_NONE}[pc],
                        _MODES[mode], inner_rtol, check_every, max_outer, 0 if graphs else 1, int(learned_every))
        st = L.SolveStats()
        rc = L.lib().chns_solve_pressure(self._h, _dev_ptr(b, torch.float64, self.n),
                                         _dev_ptr(x, torch.float64, self.n), C.byref(o), C.byref(st),
                                         _stream_ptr(stream))
        L.check(rc, allow=() if raise_on_noconv else (L.ENOCONV,))
        return x, SolveStats(st.iterations, st.outer_iterations, st.rel_residual, st.ms_setup, st.ms_solve,
                             st.fallback, rc)

    # ------------------------------------------------ CHNS forms and stepping
    def _ptrs(self, fields, lens):
        import torch
        arr = (C.c_void_p * len(fields))()
        for k, (f, nl) in enumerate(zip(fields, lens)):
            arr[k] = _dev_ptr(f, torch.float64, nl * self.n).value
        return arr

    def set_coefficients(self, op, fields, stream=None):
        """MOMENTUM: (phi~, mu~, u^); CH_JACOBIAN: (phi^{k+1}, phi^k, u~)."""
        arr = self._ptrs(fields, (1, 1, self.dim))
        L.check(L.lib().chns_set_coefficients(self._h, op, arr, _stream_ptr(stream)))

    FORM_LENS = {L.FORM_CH_RESIDUAL: ("2", 1, 1, "d"), L.FORM_VP_RHS: (1, 1, "d", "d", 1),
                 L.FORM_PP_RHS: (1, 1, "d", "d", 1, "d"), L.FORM_VU_RHS: (1, 1, "d", "d", 1, "d", 1),
                 L.FORM_ENERGY: (1, "d")}
    FORM_OUT = {L.FORM_CH_RESIDUAL: "2", L.FORM_VP_RHS: "d", L.FORM_PP_RHS: 1, L.FORM_VU_RHS: "d",
                L.FORM_ENERGY: 1}

    def _len(self, code):
        return {"2": 2, "d": self.dim}.get(code, code)

    def assemble(self, form, fields, out=None, stream=None):
        import torch
        lens = [self._len(c) for c in self.FORM_LENS[form]]
        if len(fields) != len(lens):
            raise ValueError(f"form {form} takes {len(lens)} fields")
        arr = self._ptrs(fields, lens)
        no = self._len(self.FORM_OUT[form]) * self.n
        if out is None:
            out = torch.empty(no, dtype=torch.float64, device=fields[0].device)
        L.check(L.lib().chns_assemble(self._h, form, arr, _dev_ptr(out, torch.float64, no), _stream_ptr(stream)))
        return out

    def initial_mu(self, phi, mu=None, stream=None):
        import torch
        if mu is None:
            mu = torch.empty_like(phi)
        L.check(L.lib().chns_initial_mu(self._h, _dev_ptr(phi, torch.float64, self.n),
                                        _dev_ptr(mu, torch.float64, self.n), _stream_ptr(stream)))
        return mu

    def advance_step(self, state: dict, blocks=2, newton_rtol=1e-8, newton_atol=1e-12, max_newton=20,
                     lin_rtol=1e-8, max_it=5000, restart=64, pp_pc="jacobi", pp_mode="fp64", graphs=True,
                     ch_pc="block", vp_pc="jacobi", forcing=None, stream=None):
        """state: dict of device FP64 tensors u, u_prev (dim*n), p, phi, mu (n), updated in place;
        forcing: optional (f_v (dim*n), f_phi (n), f_mu (n)) device tensors (None entries allowed),
        nodal body forces at the step's mid time."""
        import torch
        d = self.dim * self.n
        fv, fp, fm = forcing if forcing is not None else (None, None, None)
        fptr = lambda t, k: _dev_ptr(t, torch.float64, k) if t is not None else C.c_void_p()
        st = L.State(_dev_ptr(state["u"], torch.float64, d), _dev_ptr(state["u_prev"], torch.float64, d),
                     _dev_ptr(state["p"], torch.float64, self.n), _dev_ptr(state["phi"], torch.float64, self.n),
                     _dev_ptr(state["mu"], torch.float64, self.n))
        o = L.StepOpts(blocks, newton_rtol, newton_atol, max_newton, lin_rtol, max_it, restart,
                       {"jacobi": L.PC_JACOBI, "gmg": L.PC_GMG}[pp_pc],
                       _MODES[pp_mode], 0 if graphs else 1,
                       {"block": L.CH_PC_BLOCK_JACOBI, "schur": L.CH_PC_SCHUR_GMG}[ch_pc],
                       {"jacobi": L.VP_PC_JACOBI, "gmg": L.VP_PC_GMG}[vp_pc],
                       fptr(fv, d), fptr(fp, self.n), fptr(fm, self.n))
        ss = L.StepStats()
        L.check(L.lib().chns_advance_step(self._h, C.byref(st), C.byref(o), C.byref(ss), _stream_ptr(stream)))
        return {"newton": list(ss.newton_iterations)[:blocks], "ch_iterations": ss.ch_iterations,
                "vp_iterations": ss.vp_iterations, "pp_iterations": ss.pp_iterations,
                "vu_iterations": ss.vu_iterations, "ch_residual": ss.ch_residual, "mass": ss.mass,
                "energy": ss.energy, "ms": ss.ms}

    # ------------------------------------------------ learned preconditioner
    def pc_init(self, seed=0, out_scale=1.0, omega=0.0, stream=None):
        L.check(L.lib().chns_pc_init(self._h, int(seed), float(out_scale), float(omega), _stream_ptr(stream)))

    def pc_load(self, blob: bytes, stream=None):
        buf = C.create_string_buffer(bytes(blob), len(blob))
        L.check(L.lib().chns_pc_load(self._h, buf, len(blob), _stream_ptr(stream)))

    def pc_save(self) -> bytes:
        n = C.c_size_t()
        L.check(L.lib().chns_pc_save(self._h, None, 0, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        L.check(L.lib().chns_pc_save(self._h, buf, n.value, C.byref(n)))
        return buf.raw[:n.value]

    def pc_param_count(self) -> int:
        n = C.c_size_t()
        L.check(L.lib().chns_pc_param_count(self._h, C.byref(n)))
        return n.value

    def pc_gradients(self) -> np.ndarray:
        n = self.pc_param_count()
        g = np.empty(n, dtype=np.float32)
        L.check(L.lib().chns_pc_gradients(self._h, g.ctypes.data_as(C.c_void_p), n))
        return g

    def pc_forward(self, phi, r, origin=(0, 0, 0), flip=0, crop=16, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(crop ** 3, dtype=torch.float32, device=phi.device)
        org = (C.c_int32 * 3)(*[int(v) for v in origin])
        L.check(L.lib().chns_pc_forward(self._h, _dev_ptr(phi, torch.float64, self.n),
                                        _dev_ptr(r, torch.float64, self.n), org, int(flip), int(crop),
                                        _dev_ptr(out, torch.float32, crop ** 3), _stream_ptr(stream)))
        return out

    def pc_train_step(self, phis, rs, es, origins=None, crop=8, flips=None, lr=1e-3, objective="crop_mse",
                      stream=None) -> float:
        import torch
        k = len(rs)
        if origins is None:
            origins = [(0, 0, 0)] * k
        P = (C.c_void_p * k)(*[_dev_ptr(t, torch.float64, self.n).value for t in phis])
        R = (C.c_void_p * k)(*[_dev_ptr(t, torch.float64, self.n).value for t in rs])
        E = (C.c_void_p * k)(*[_dev_ptr(t, torch.float64, self.n).value for t in es])
        O = (C.c_int32 * (3 * k))(*[int(v) for o in origins for v in o])
        F = (C.c_int32 * k)(*([int(f) for f in flips] if flips is not None else [0] * k))
        b = L.PcBatch(k, C.cast(P, C.POINTER(C.c_void_p)), C.cast(R, C.POINTER(C.c_void_p)),
                      C.cast(E, C.POINTER(C.c_void_p)), O, F, int(crop),
                      {"crop_mse": 0, "anorm": 1}[objective])
        loss = C.c_float()
        L.check(L.lib().chns_pc_train_step(self._h, C.byref(b), float(lr), C.byref(loss), _stream_ptr(stream)))
        return loss.value

    def profile(self, enable=True):
        L.check(L.lib().chns_profile_enable(self._h, int(enable)))

    def profile_reset(self):
        L.check(L.lib().chns_profile_reset(self._h))

    def profile_read(self, tag):
        ms = C.c_double()
        n = C.c_int64()
        L.check(L.lib().chns_profile_read(self._h, tag.encode(), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def __del__(self):
        # only attributes of the object itself: module globals may already be
        # gone when this runs at interpreter shutdown
        h = getattr(self, "_h", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and h.value and destroy is not None:
            destroy(h)
            h.value = None
