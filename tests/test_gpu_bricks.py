"""GPU parity on the brick classes that the large meshes run on, with the
rising-bubble physics (density ratio 1000, viscosity ratio 100, Re 35,
We 10, Fr 1, dt 5e-4; paper Sec. 5, rising-bubble benchmark parameters lifted
to 3D).

The library groups leaves into aligned bricks of 8^d, 4^d, 2^d leaves or
single leaves; the brick edge is chosen automatically, and the small meshes
of the other parity tests only reach the smaller classes.  Here every mesh is
built with the largest edge allowed (brick_max = 8), so that
* the 3D uniform level-4 mesh runs the structured (table-free) 8^3 bricks,
  whose node layers stream through an LDS ring;
* the 3D band mesh (levels 3-6) has table bricks of all four classes and
  hanging nodes, so the ring with node tables and the interior-node direct
  write of 8^3 bricks run next to the small classes;
* the 2D meshes have 8^2 bricks (structured on the uniform mesh, with node
  tables on the band mesh).

Bars: every matrix-free form (pressure apply and diagonal in FP64, the FP32
pressure apply, mass with density, CH residual, CH Jacobian apply and
diagonal, VMS momentum apply and diagonal, scalar momentum operator, the
three right-hand sides, energy) agrees with the oracle's assembled result to
1e-12 relative (2-norm and max-norm); the FP32 pressure, CH Jacobian and
momentum applies to 2e-5 of the largest entry.  Steps with the
rising-bubble physics match the oracle's steps to 1e-6 in every field (the
oracle solves exactly; the GPU's Krylov solves stop at 1e-11), and the mass
drift of the GPU steps is reported and bounded.
"""
import numpy as np
import pytest

from oracle import chns, fem

from ._pairs import Pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (id, kind, dim, lmin, lmax, radius, band, Cn, brick classes that must be present)
CASES = [
    ("uniform3d_l4", "uniform", 3, 4, 4, 0.15, 0.03, 0.04, (0,)),
    ("band3d_l3-6", "band", 3, 3, 6, 0.15, 0.06, 0.03, (0, 1, 2, 3)),
    ("uniform2d_l6", "uniform", 2, 6, 6, 0.15, 0.02, 0.02, (0,)),
    ("band2d_l4-8", "band", 2, 4, 8, 0.15, 0.05, 0.01, (0, 1, 2, 3)),
]


def _bubble_params(cn):
    return dict(Re=35.0, We=10.0, Cn=cn, Fr=1.0, rho_plus=1.0, rho_minus=1e-3, eta_plus=1.0, eta_minus=1e-2,
                dt=5e-4)


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _close(y, ref, tol=1e-12):
    r2 = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    rinf = np.abs(y - ref).max() / np.abs(ref).max()
    assert r2 <= tol and rinf <= tol, (r2, rinf)


def _fp32_close(y32, refs, tol=2e-5):
    """FP32 apply (FP32 fields and arithmetic) against the FP64 oracle: every
    entry within tol of the largest entry of its field."""
    y32 = y32.cpu().numpy().astype(np.float64).reshape(len(refs), -1)
    for f, ref in enumerate(refs):
        err = np.abs(y32[f] - ref).max() / np.abs(ref).max()
        print(f"fp32 field {f}: {err:.2e}", flush=True)
        assert err <= tol, (f, err)


class Case:
    def __init__(self, spec):
        name, kind, dim, lmin, lmax, radius, band, cn, classes = spec
        from paper_2107_05123_amd import Context
        self.pair = Pair(kind, dim, lmin, lmax, radius=radius, band=band, brick_max=8)
        info = self.pair.lib.summary()
        print(f"case {name}: n={info['n_nodes']} hanging={info['n_hanging']} bricks={info['n_bricks']} "
              f"leaves in bricks={info['elems_in_bricks']}", flush=True)
        for k in classes:
            assert info["n_bricks"][k] > 0, (name, info["n_bricks"])
        self.dim = dim
        self.n = self.pair.lib.n_nodes
        self.prm_kw = _bubble_params(cn)
        self.prm = chns.Params(**self.prm_kw)
        self.ctx = Context(self.pair.lib, **self.prm_kw)
        self.el = chns.Elems(self.pair.orc)
        rng = np.random.default_rng(11)
        n = self.n
        self.phi0 = self.pair.phi("bubble", cn=cn)
        self.phi1 = self.phi0 + 0.05 * rng.standard_normal(n)
        self.mu0 = 0.1 * rng.standard_normal(n)
        self.mu1 = self.mu0 + 0.05 * rng.standard_normal(n)
        self.u = 0.3 * rng.standard_normal((dim, n))
        self.uprev = 0.3 * rng.standard_normal((dim, n))
        self.v = 0.3 * rng.standard_normal((dim, n))
        self.p = rng.standard_normal(n)
        self.pnew = rng.standard_normal(n)

    def o(self, v):
        v = np.asarray(v)
        return np.stack([self.pair.to_orc(c) for c in v]) if v.ndim == 2 else self.pair.to_orc(v)

    def lib(self, v):
        v = np.asarray(v)
        return np.stack([self.pair.to_lib(c) for c in v]) if v.ndim == 2 else self.pair.to_lib(v)

    def qpstate(self, phit, mut, uhat):
        return chns.QPState(self.el, self.prm, self.o(phit), self.o(mut), self.o(uhat), self.o(self.u),
                            self.o(self.p))


@pytest.fixture(scope="module", params=CASES, ids=lambda c: c[0])
def case(request):
    return Case(request.param)


def test_pressure_apply_diagonal_and_rho_mass_match_oracle(case):
    c = case
    m = c.pair.orc
    c.ctx.set_phase_field(_dev(c.phi0))
    A = fem.pp_matrix(m, c.o(c.phi0), c.prm.rho_plus, c.prm.rho_minus)
    x = np.random.default_rng(5).standard_normal(c.n)
    ref = c.lib(A @ c.o(x))
    _close(c.ctx.apply(c.ctx.PRESSURE, _dev(x)).cpu().numpy(), ref)
    y32 = c.ctx.apply(c.ctx.PRESSURE, _dev(x, torch.float32)).cpu().numpy().astype(np.float64)
    assert np.abs(y32 - ref).max() <= 2e-5 * np.abs(ref).max()
    _close(c.ctx.diagonal(c.ctx.PRESSURE).cpu().numpy(), c.lib(A.diagonal()))
    # rho-weighted mass with identity wall rows (velocity update operator)
    S = c.qpstate(c.phi0, c.mu0, c.u)
    M = chns.rho_mass_walls(c.el, c.prm, S)
    v = np.random.default_rng(6).standard_normal((c.dim, c.n))
    y = c.ctx.apply(c.ctx.MASS_RHO, _dev(v.reshape(-1))).cpu().numpy().reshape(c.dim, -1)
    for i in range(c.dim):
        _close(y[i], c.lib(M @ c.o(v[i])))


def test_ch_residual_jacobian_and_diagonal_match_oracle(case):
    from paper_2107_05123_amd import _lib as L
    c = case
    ut = 0.5 * (c.u + c.v)
    X = np.concatenate([c.phi1, c.mu1])
    r = c.ctx.assemble(L.FORM_CH_RESIDUAL, [_dev(X), _dev(c.phi0), _dev(c.mu0), _dev(ut.reshape(-1))])
    r = r.cpu().numpy().reshape(2, -1)
    Rp, Rm = chns.ch_residual(c.el, c.prm, c.o(c.phi1), c.o(c.mu1), c.o(c.phi0), c.o(c.mu0), c.o(ut))
    _close(r[0], c.lib(Rp))
    _close(r[1], c.lib(Rm))
    c.ctx.set_coefficients(c.ctx.CH_JACOBIAN, [_dev(c.phi1), _dev(c.phi0), _dev(ut.reshape(-1))])
    d = np.random.default_rng(3).standard_normal((2, c.n))
    y = c.ctx.apply(c.ctx.CH_JACOBIAN, _dev(d.reshape(-1))).cpu().numpy().reshape(2, -1)
    J = chns.ch_jacobian(c.el, c.prm, c.o(c.phi1), c.o(c.phi0), c.o(ut))
    ref = (J @ np.concatenate([c.o(d[0]), c.o(d[1])])).reshape(2, -1)
    _close(y[0], c.lib(ref[0]))
    _close(y[1], c.lib(ref[1]))
    _fp32_close(c.ctx.apply(c.ctx.CH_JACOBIAN, _dev(d.reshape(-1), torch.float32)), [c.lib(r) for r in ref])
    dg = c.ctx.diagonal(c.ctx.CH_JACOBIAN).cpu().numpy().reshape(2, -1)
    dref = J.diagonal().reshape(2, -1)
    _close(dg[0], c.lib(dref[0]))
    _close(dg[1], c.lib(dref[1]))


def test_momentum_apply_diagonal_and_scalar_operator_match_oracle(case):
    c = case
    phit, mut = 0.5 * (c.phi1 + c.phi0), 0.5 * (c.mu1 + c.mu0)
    uhat = 1.5 * c.u - 0.5 * c.uprev
    c.ctx.set_coefficients(c.ctx.MOMENTUM, [_dev(phit), _dev(mut), _dev(uhat.reshape(-1))])
    y = c.ctx.apply(c.ctx.MOMENTUM, _dev(c.v.reshape(-1))).cpu().numpy().reshape(c.dim, -1)
    A = chns.vp_matrix(c.el, c.prm, c.qpstate(phit, mut, uhat))
    refs = [c.lib(A @ c.o(c.v[i])) for i in range(c.dim)]
    for i in range(c.dim):
        _close(y[i], refs[i])
    _fp32_close(c.ctx.apply(c.ctx.MOMENTUM, _dev(c.v.reshape(-1), torch.float32)), refs)
    dg = c.ctx.diagonal(c.ctx.MOMENTUM).cpu().numpy().reshape(c.dim, -1)
    for i in range(c.dim):
        _close(dg[i], c.lib(A.diagonal()))
    m = c.pair.orc
    c.ctx.set_phase_field(_dev(c.phi0))
    x = np.random.default_rng(8).standard_normal(c.n)
    qp = fem.qp_values(m, c.o(c.phi0))
    ref = fem.mass_matrix(m, c.prm.rho(qp)) / c.prm.dt + fem.stiffness_matrix(m, c.prm.eta(qp)) / (2 * c.prm.Re)
    _close(c.ctx.apply(c.ctx.MOMENTUM_SCALAR, _dev(x)).cpu().numpy(), c.lib(ref @ c.o(x)))


def test_right_hand_sides_and_energy_match_oracle(case):
    from paper_2107_05123_amd import _lib as L
    c = case
    phit, mut = 0.5 * (c.phi1 + c.phi0), 0.5 * (c.mu1 + c.mu0)
    uhat = 1.5 * c.u - 0.5 * c.uprev
    S = c.qpstate(phit, mut, uhat)
    base = [_dev(phit), _dev(mut), _dev(uhat.reshape(-1)), _dev(c.u.reshape(-1)), _dev(c.p)]
    vp = c.ctx.assemble(L.FORM_VP_RHS, base).cpu().numpy().reshape(c.dim, -1)
    ref = chns.vp_rhs(c.el, c.prm, S, c.o(c.u), c.o(c.p), c.o(phit))
    for i in range(c.dim):
        _close(vp[i], c.lib(ref[i]))
    pp = c.ctx.assemble(L.FORM_PP_RHS, base + [_dev(c.v.reshape(-1))]).cpu().numpy()
    _close(pp, c.lib(chns.pp_rhs(c.el, c.prm, S, c.o(c.v), c.o(c.p))))
    vu = c.ctx.assemble(L.FORM_VU_RHS, base + [_dev(c.v.reshape(-1)), _dev(c.pnew)]).cpu().numpy()
    vu = vu.reshape(c.dim, -1)
    ref = chns.vu_rhs(c.el, c.prm, S, c.o(c.v), c.o(c.pnew), c.o(c.p))
    for i in range(c.dim):
        _close(vu[i], c.lib(ref[i]))
    e = c.ctx.assemble(L.FORM_ENERGY, [_dev(c.phi1), _dev(c.u.reshape(-1))]).sum().item()
    st = chns.State(u=c.o(c.u), u_prev=c.o(c.u), p=c.o(c.p), phi=c.o(c.phi1), mu=c.o(c.mu1))
    eref = chns.energy(c.el, c.prm, st)
    assert abs(e - eref) <= 1e-12 * abs(eref), (e, eref)


# Steps with the rising-bubble physics.  The 3D band mesh is left out: the
# oracle's sparse LU needs minutes per step there.
@pytest.mark.parametrize("idx,nsteps", [(0, 2), (3, 3)], ids=["uniform3d_l4", "band2d_l4-8"])
def test_bubble_physics_steps_match_oracle(idx, nsteps):
    c = Case(CASES[idx])
    mu0 = c.ctx.initial_mu(_dev(c.phi0))
    z = np.zeros((c.dim, c.n))
    state = {"u": _dev(z.reshape(-1)), "u_prev": _dev(z.reshape(-1)), "p": _dev(np.zeros(c.n)),
             "phi": _dev(c.phi0), "mu": mu0}
    stats = [c.ctx.advance_step(state, lin_rtol=1e-11, ch_pc="schur", pp_pc="gmg", vp_pc="gmg")
             for _ in range(nsteps)]
    st = chns.initial_state(c.el, c.prm, c.o(c.phi0))
    m0 = chns.mass(c.el, st.phi)
    for s in stats:
        st, info = chns.step(c.el, c.prm, st)
        print(f"gpu newton {s['newton']} ch {s['ch_iterations']} vp {s['vp_iterations']} pp {s['pp_iterations']} "
              f"vu {s['vu_iterations']} mass drift {s['mass'] - m0:.3e}; oracle newton {info['newton']}",
              flush=True)
        assert abs(s["mass"] - m0) <= 1e-10 * abs(m0)
    got = {k: v.cpu().numpy() for k, v in state.items()}
    for name, ref in (("phi", st.phi), ("mu", st.mu), ("p", st.p)):
        err = np.linalg.norm(c.o(got[name]) - ref) / np.linalg.norm(ref)
        print(f"{name}: relative difference {err:.2e}", flush=True)
        assert err <= 1e-6, (name, err)
    u = c.o(got["u"].reshape(c.dim, -1))
    err = np.linalg.norm(u - st.u) / np.linalg.norm(st.u)
    print(f"u: relative difference {err:.2e}", flush=True)
    assert err <= 1e-6, ("u", err)
    e = chns.energy(c.el, c.prm, st)
    assert abs(stats[-1]["energy"] - e) <= 1e-8 * abs(e)
