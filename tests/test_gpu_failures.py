"""Failure handling forced from the host (every kernel still exits normally).

* A NaN in the phase field: the pull back would silently map it to a pure
  phase, so chns_set_phase_field flags it and chns_solve_pressure returns
  CHNS_EINVAL at once, with its statistics filled (0 iterations, residual
  NaN) and x untouched; a NaN in the right-hand side likewise.  The context
  works again after a valid phase field.
* A learned preconditioner whose output is zero (output scale K = 0): flexible
  CG breaks down at r_0 (r.z = 0); the solve ends that iteration at x_0 and
  continues with Jacobi-PCG (fallback flag set), reaching 1e-8 measured with
  the oracle's matrix.
* A time step whose Newton iteration cannot converge (one Newton iteration
  allowed, an unreachable tolerance): CHNS_ENOCONV, the state untouched, and
  the context's phase field marked unset (a pressure solve is then
  CHNS_ESTATE until chns_set_phase_field); a NaN in the state's phase field
  is CHNS_ENOCONV from the first residual, without iterating.
"""
import ctypes as C
import math

import numpy as np
import pytest

import chns_inputs as ci
from oracle import fem

from ._pairs import Pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RHO_P, RHO_M = 1.0, 1e-3


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _raw_solve(ctx, b, x, pc):
    from paper_2107_05123_amd import _lib as L
    o = L.SolveOpts(1e-8, 2000, pc, L.MODE_FP64, 1e-4, 16, 30, 0, 0)
    st = L.SolveStats()
    st.iterations, st.rel_residual = -1, -1.0
    rc = L.lib().chns_solve_pressure(ctx._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), C.byref(o),
                                     C.byref(st), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, st


def test_nan_in_phase_field_or_rhs_is_einval_with_stats():
    from paper_2107_05123_amd import Context
    from paper_2107_05123_amd import _lib as L
    pair = Pair("band", 3, 2, 5, band=0.03)
    n = pair.lib.n_nodes
    phi = pair.phi("bubble", cn=0.02)
    ctx = Context(pair.lib, rho_plus=RHO_P, rho_minus=RHO_M)
    bad = phi.copy()
    bad[n // 2] = np.nan
    ctx.set_phase_field(_dev(bad))
    amps, waves = ci.rhs_modes(1)
    f = _dev(ci.rhs_field(pair.x_unit, amps, waves))
    b = ctx.apply(ctx.MASS, f)
    for pc in (L.PC_JACOBI, L.PC_GMG):
        x = torch.full((n,), 7.0, dtype=torch.float64, device="cuda")
        rc, st = _raw_solve(ctx, b, x, pc)
        assert rc == L.EINVAL, rc
        assert b"NaN" in L.lib().chns_last_error()
        assert st.iterations == 0 and math.isnan(st.rel_residual)
        assert float((x - 7.0).abs().max()) == 0.0
    # a valid phase field makes the context usable again
    ctx.set_phase_field(_dev(phi))
    A = fem.pp_matrix(pair.orc, pair.to_orc(phi), RHO_P, RHO_M)
    xs, st = ctx.solve_pressure(b, rtol=1e-8)
    bo = pair.to_orc(b.cpu().numpy())
    bo -= bo.mean()
    assert np.linalg.norm(bo - A @ pair.to_orc(xs.cpu().numpy())) <= 1.05e-8 * np.linalg.norm(bo)
    bnan = b.clone()
    bnan[3] = float("nan")
    rc, st = _raw_solve(ctx, bnan, torch.zeros_like(b), L.PC_JACOBI)
    assert rc == L.EINVAL and st.iterations == 0 and math.isnan(st.rel_residual)


def test_zero_output_network_falls_back_to_jacobi():
    from paper_2107_05123_amd import Context, Mesh
    m = Mesh(dim=3, min_level=4, max_level=4, rule="uniform")
    from oracle import mesh as om
    orc = om.uniform(3, 4)
    coords = m.node_coords()
    perm = om.node_index_map(coords, orc.indep_coords(), 1 << 4)
    x_unit = ci.unit_coords(coords, 4)
    c, r = ci.drops(0)
    phi = ci.phi_drops(x_unit, c, r, 0.05)
    ctx = Context(m, rho_plus=RHO_P, rho_minus=RHO_M)
    ctx.set_phase_field(_dev(phi))
    ctx.pc_init(seed=1, out_scale=0.0)
    amps, waves = ci.rhs_modes(1)
    b = ctx.apply(ctx.MASS, _dev(ci.rhs_field(x_unit, amps, waves)))
    phi_o = np.empty_like(phi)
    phi_o[perm] = phi
    A = fem.pp_matrix(orc, phi_o, RHO_P, RHO_M)
    for every in (0, 8):
        x, st = ctx.solve_pressure(b, rtol=1e-8, pc="learned", learned_every=every)
        print(f"learned_every={every}: iterations {st.iterations} fallback {st.fallback} "
              f"residual {st.rel_residual:.3e}", flush=True)
        assert st.fallback == 1
        xo = np.empty(m.n_nodes)
        xo[perm] = x.cpu().numpy()
        bo = np.empty(m.n_nodes)
        bo[perm] = b.cpu().numpy()
        bo -= bo.mean()
        assert np.linalg.norm(bo - A @ xo) <= 1.05e-8 * np.linalg.norm(bo)


def test_failed_step_leaves_state_and_unsets_phase_field():
    from paper_2107_05123_amd import Context
    from paper_2107_05123_amd import _lib as L
    pair = Pair("uniform", 2, 5, 5)
    n = pair.lib.n_nodes
    kw = dict(Re=100.0, We=1.0, Cn=0.04, Fr=1.0, rho_plus=1.0, rho_minus=0.1, eta_plus=1.0, eta_minus=0.1, dt=1e-3)
    ctx = Context(pair.lib, **kw)
    phi0 = _dev(pair.phi("drop2d", cn=0.04))
    mu0 = ctx.initial_mu(phi0)
    z = torch.zeros(2 * n, dtype=torch.float64, device="cuda")
    state = {"u": z.clone(), "u_prev": z.clone(), "p": torch.zeros(n, dtype=torch.float64, device="cuda"),
             "phi": phi0.clone(), "mu": mu0.clone()}
    before = {k: v.clone() for k, v in state.items()}
    ctx.set_phase_field(phi0)
    for ch_pc in ("block", "schur"):
        with pytest.raises(L.ChnsError) as e:
            ctx.advance_step(state, max_newton=1, newton_rtol=1e-30, newton_atol=0.0, ch_pc=ch_pc, pp_pc="gmg")
        assert e.value.code == L.ENOCONV
        for k in state:
            assert torch.equal(state[k], before[k]), k
        b = ctx.apply(ctx.MASS, phi0)
        with pytest.raises(L.ChnsError) as e:
            ctx.solve_pressure(b)
        assert e.value.code == L.ESTATE
        ctx.set_phase_field(phi0)
        x, st = ctx.solve_pressure(b, rtol=1e-8, pc="gmg")
        assert st.rel_residual <= 1e-8
    # NaN in the state: the first residual is not finite
    state["phi"][5] = float("nan")
    with pytest.raises(L.ChnsError) as e:
        ctx.advance_step(state)
    assert e.value.code == L.ENOCONV
    assert b"not finite" in L.lib().chns_last_error()
    # a good state steps normally afterwards
    state = {k: v.clone() for k, v in before.items()}
    s = ctx.advance_step(state, lin_rtol=1e-10)
    assert s["newton"][0] >= 1
