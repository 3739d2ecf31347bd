"""GPU parity on incomplete (carved) octrees: the paper's Rayleigh-Taylor
column (Sec. 5.4: a 1 x 8 x 1 box, here the part x, z < 1/8 of the unit
root cube at carve level 3) and a 2D column, refined around the
Rayleigh-Taylor interface, with hanging nodes.

Bars: the pressure apply (FP64 1e-12, FP32 2e-5) and its diagonal, the CH
residual and Jacobian, the momentum apply and the three right-hand sides
agree with the oracle's assembled forms on the carved mesh (walls on the box
faces); Jacobi- and multigrid-preconditioned pressure solves reach 1e-8
measured with the oracle's matrix (the multigrid hierarchy stops at the
carve level, whose octants tile the box); projection steps with
Rayleigh-Taylor physics (Atwood number 0.15: density ratio 1/0.74, equal
kinematic viscosities, heavy fluid on top) match the oracle's steps to 1e-6
and conserve mass.
"""
import numpy as np
import pytest

import chns_inputs as ci
from oracle import chns, fem, mesh as om

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (id, dim, lmin, lmax, slab half width (physical), carve level, extent, brick_max)
CASES = [
    ("col2d_l2-7", 2, 2, 7, 0.4, 2, (1, 4), 0),
    ("col2d_l2-7_b8", 2, 2, 7, 0.4, 2, (1, 4), 8),
    ("rt3d_l3-7", 3, 3, 7, 0.3, 3, ci.RT_EXTENT, 0),
    ("rt3d_l3-7_b8", 3, 3, 7, 0.3, 3, ci.RT_EXTENT, 8),
]
RT = dict(Re=1000.0, We=1000.0, Cn=0.02, Fr=1.0, rho_plus=1.0, rho_minus=0.74, eta_plus=1.0, eta_minus=0.74,
          dt=1e-3)


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _close(y, ref, tol=1e-12):
    r2 = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    rinf = np.abs(y - ref).max() / np.abs(ref).max()
    assert r2 <= tol and rinf <= tol, (r2, rinf)


class CarvedCase:
    def __init__(self, spec):
        from paper_2107_05123_amd import Context, Mesh
        name, dim, lmin, lmax, width, carve, extent, bmax = spec
        side = 1 << lmax

        def refine(anchor, level):
            size = side >> level
            return ci.rt_slab_meets(anchor[1] / side, (anchor[1] + size) / side, width)
        ext = tuple(extent) + (0,) * (3 - len(extent))
        self.lib = Mesh(dim=dim, min_level=lmin, max_level=lmax, rule="callback", refine=refine, carve_level=carve,
                        extent=ext, brick_max=bmax)
        self.orc = om.from_predicate(dim, lmin, lmax, lambda lev, lo, hi: ci.rt_slab_meets(lo[1], hi[1], width),
                                     [e / (1 << carve) for e in extent])
        s = self.lib.summary()
        print(f"{name}: n={s['n_nodes']} hanging={s['n_hanging']} bricks={s['n_bricks']} box={s['box']}",
              flush=True)
        self.dim, self.n = dim, self.lib.n_nodes
        coords = self.lib.node_coords()
        self.perm = om.node_index_map(coords, self.orc.indep_coords(), side)
        self.x = ci.unit_coords(coords, lmax)
        self.prm = chns.Params(**RT)
        self.ctx = Context(self.lib, **RT)
        self.el = chns.Elems(self.orc)
        self.phi = ci.phi_rt(self.x, cn=8 * RT["Cn"])

    def o(self, v):
        v = np.asarray(v)
        if v.ndim == 2:
            return np.stack([self.o(c) for c in v])
        out = np.empty_like(v)
        out[self.perm] = v
        return out

    def lib_order(self, v):
        return np.asarray(v)[self.perm]


@pytest.fixture(scope="module", params=CASES, ids=lambda c: c[0])
def case(request):
    return CarvedCase(request.param)


def test_pressure_apply_and_solves_on_carved_mesh(case):
    c = case
    c.ctx.set_phase_field(_dev(c.phi))
    A = fem.pp_matrix(c.orc, c.o(c.phi), RT["rho_plus"], RT["rho_minus"])
    x = ci.normal_vector(4, c.n)
    ref = c.lib_order(A @ c.o(x))
    _close(c.ctx.apply(c.ctx.PRESSURE, _dev(x)).cpu().numpy(), ref)
    y32 = c.ctx.apply(c.ctx.PRESSURE, _dev(x, torch.float32)).cpu().numpy().astype(np.float64)
    assert np.abs(y32 - ref).max() <= 2e-5 * np.abs(ref).max()
    _close(c.ctx.diagonal(c.ctx.PRESSURE).cpu().numpy(), c.lib_order(A.diagonal()))
    amps, waves = ci.rhs_modes(1, dim=c.dim)
    b = c.ctx.apply(c.ctx.MASS, _dev(ci.rhs_field(c.x, amps, waves)))
    bo = c.o(b.cpu().numpy())
    bo -= bo.mean()
    for pc in ("jacobi", "gmg"):
        xs, st = c.ctx.solve_pressure(b, rtol=1e-8, pc=pc)
        rel = np.linalg.norm(bo - A @ c.o(xs.cpu().numpy())) / np.linalg.norm(bo)
        print(f"{pc}: {st.iterations} iterations, oracle residual {rel:.2e}", flush=True)
        assert rel <= 1.05e-8


def test_chns_forms_on_carved_mesh(case):
    from paper_2107_05123_amd import _lib as L
    c = case
    rng = np.random.default_rng(9)
    n, dim = c.n, c.dim
    phi0 = c.phi
    phi1 = phi0 + 0.05 * rng.standard_normal(n)
    mu0, mu1 = 0.1 * rng.standard_normal(n), 0.1 * rng.standard_normal(n)
    u, uprev, v = (0.3 * rng.standard_normal((dim, n)) for _ in range(3))
    p, pnew = rng.standard_normal(n), rng.standard_normal(n)
    ut = 0.5 * (u + v)
    r = c.ctx.assemble(L.FORM_CH_RESIDUAL, [_dev(np.concatenate([phi1, mu1])), _dev(phi0), _dev(mu0),
                                            _dev(ut.reshape(-1))]).cpu().numpy().reshape(2, -1)
    Rp, Rm = chns.ch_residual(c.el, c.prm, c.o(phi1), c.o(mu1), c.o(phi0), c.o(mu0), c.o(ut))
    _close(r[0], c.lib_order(Rp))
    _close(r[1], c.lib_order(Rm))
    c.ctx.set_coefficients(c.ctx.CH_JACOBIAN, [_dev(phi1), _dev(phi0), _dev(ut.reshape(-1))])
    d = rng.standard_normal((2, n))
    y = c.ctx.apply(c.ctx.CH_JACOBIAN, _dev(d.reshape(-1))).cpu().numpy().reshape(2, -1)
    ref = (chns.ch_jacobian(c.el, c.prm, c.o(phi1), c.o(phi0), c.o(ut)) @ np.concatenate([c.o(d[0]), c.o(d[1])]))
    ref = ref.reshape(2, -1)
    _close(y[0], c.lib_order(ref[0]))
    _close(y[1], c.lib_order(ref[1]))
    phit, mut, uhat = 0.5 * (phi1 + phi0), 0.5 * (mu1 + mu0), 1.5 * u - 0.5 * uprev
    c.ctx.set_coefficients(c.ctx.MOMENTUM, [_dev(phit), _dev(mut), _dev(uhat.reshape(-1))])
    S = chns.QPState(c.el, c.prm, c.o(phit), c.o(mut), c.o(uhat), c.o(u), c.o(p))
    A = chns.vp_matrix(c.el, c.prm, S)
    y = c.ctx.apply(c.ctx.MOMENTUM, _dev(v.reshape(-1))).cpu().numpy().reshape(dim, -1)
    for i in range(dim):
        _close(y[i], c.lib_order(A @ c.o(v[i])))
    base = [_dev(phit), _dev(mut), _dev(uhat.reshape(-1)), _dev(u.reshape(-1)), _dev(p)]
    vp = c.ctx.assemble(L.FORM_VP_RHS, base).cpu().numpy().reshape(dim, -1)
    for i, b in enumerate(chns.vp_rhs(c.el, c.prm, S, c.o(u), c.o(p), c.o(phit))):
        _close(vp[i], c.lib_order(b))
    pp = c.ctx.assemble(L.FORM_PP_RHS, base + [_dev(v.reshape(-1))]).cpu().numpy()
    _close(pp, c.lib_order(chns.pp_rhs(c.el, c.prm, S, c.o(v), c.o(p))))
    vu = c.ctx.assemble(L.FORM_VU_RHS, base + [_dev(v.reshape(-1)), _dev(pnew)]).cpu().numpy().reshape(dim, -1)
    for i, b in enumerate(chns.vu_rhs(c.el, c.prm, S, c.o(v), c.o(pnew), c.o(p))):
        _close(vu[i], c.lib_order(b))


@pytest.mark.parametrize("idx,nsteps", [(0, 3), (2, 2)], ids=["col2d", "rt3d"])
def test_rayleigh_taylor_steps_on_carved_mesh_match_oracle(idx, nsteps):
    c = CarvedCase(CASES[idx])
    mu0 = c.ctx.initial_mu(_dev(c.phi))
    z = np.zeros((c.dim, c.n))
    state = {"u": _dev(z.reshape(-1)), "u_prev": _dev(z.reshape(-1)), "p": _dev(np.zeros(c.n)),
             "phi": _dev(c.phi), "mu": mu0}
    stats = [c.ctx.advance_step(state, lin_rtol=1e-11, ch_pc="schur", pp_pc="gmg", vp_pc="gmg")
             for _ in range(nsteps)]
    st = chns.initial_state(c.el, c.prm, c.o(c.phi))
    m0 = chns.mass(c.el, st.phi)
    for s in stats:
        st, info = chns.step(c.el, c.prm, st)
        print(f"gpu {s}; oracle newton {info['newton']}", flush=True)
        assert abs(s["mass"] - m0) <= 1e-10 * abs(m0)
    got = {k: v.cpu().numpy() for k, v in state.items()}
    for name, ref in (("phi", st.phi), ("mu", st.mu), ("p", st.p)):
        err = np.linalg.norm(c.o(got[name]) - ref) / np.linalg.norm(ref)
        print(f"{name}: {err:.2e}", flush=True)
        assert err <= 1e-6, (name, err)
    u = c.o(got["u"].reshape(c.dim, -1))
    err = np.linalg.norm(u - st.u) / np.linalg.norm(st.u)
    print(f"u: {err:.2e}", flush=True)
    assert err <= 1e-6
