"""Pins for the oracle's Cahn-Hilliard / VMS momentum / projection step (CPU).

Independent pins: Newton Jacobian against central differences of the
residual; discrete mass conservation (testing the CH equation with q = 1,
Prop. 1); the flat tanh profile is an equilibrium of the continuous
chemical-potential equation, so the discrete mu of that profile vanishes at
second order (a wrong sign or factor on psi' or on the Cn^2 term leaves an
O(1) mu); advection moves a drop along the velocity; with u^ = J = 0 the
VMS operator reduces to (1/dt) M_rho + (1/2Re) K_eta assembled through the
independent routines of oracle/fem.py; tau_m closed form; full steps
conserve mass, do not increase the total energy, and the projection
reduces the divergence; a static drop carries the Young-Laplace pressure
jump.
"""
import numpy as np
import pytest

import chns_inputs as ci
from oracle import chns, fem, mesh as om


def _setup(level=4, cn=0.05, **kw):
    m = om.uniform(2, level)
    el = chns.Elems(m)
    prm = chns.Params(Cn=cn, **kw)
    x = m.indep_coords() / m.side
    return m, el, prm, x


def test_ch_jacobian_matches_central_differences():
    m, el, prm, x = _setup(level=3, cn=0.1, dt=1e-2)
    rng = np.random.default_rng(0)
    n = m.n_indep
    phi0 = np.tanh((0.3 - np.linalg.norm(x - 0.5, axis=1)) / (np.sqrt(2) * 0.1))
    mu0 = rng.standard_normal(n) * 0.1
    ut = rng.standard_normal((2, n))
    phi1 = phi0 + 0.1 * rng.standard_normal(n)
    mu1 = mu0 + 0.1 * rng.standard_normal(n)
    J = chns.ch_jacobian(el, prm, phi1, phi0, ut)
    d = rng.standard_normal(2 * n)
    eps = 1e-4
    Rp = np.concatenate(chns.ch_residual(el, prm, phi1 + eps * d[:n], mu1 + eps * d[n:], phi0, mu0, ut))
    Rm = np.concatenate(chns.ch_residual(el, prm, phi1 - eps * d[:n], mu1 - eps * d[n:], phi0, mu0, ut))
    fd = (Rp - Rm) / (2 * eps)
    assert np.linalg.norm(J @ d - fd) <= 1e-8 * np.linalg.norm(fd)


def test_ch_mass_conservation_of_residual():
    m, el, prm, x = _setup(level=4, cn=0.05)
    rng = np.random.default_rng(1)
    n = m.n_indep
    phi0, phi1 = rng.standard_normal(n), rng.standard_normal(n)
    mu0, mu1 = rng.standard_normal(n), rng.standard_normal(n)
    ut = rng.standard_normal((2, n))
    Rphi, _ = chns.ch_residual(el, prm, phi1, mu1, phi0, mu0, ut)
    # q = 1 kills every gradient term
    assert abs(Rphi.sum() - (chns.mass(el, phi1) - chns.mass(el, phi0)) / prm.dt) < 1e-9 * np.abs(Rphi).sum()


def test_flat_tanh_profile_has_second_order_small_mu():
    # Cn small enough that the profile meets the no-flux walls to ~1e-8
    errs = []
    for level in (5, 6, 7):
        m, el, prm, x = _setup(level=level, cn=0.04)
        phi = np.tanh((x[:, 0] - 0.5) / (np.sqrt(2) * prm.Cn))
        mu = chns.initial_mu(el, prm, phi)
        errs.append(np.sqrt(chns.mass(el, mu ** 2)))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 2e-3 and min(rates) > 1.7, (errs, rates)
    # a flipped Cn^2 sign would give mu ~ 2 psi'(phi), of order one
    m, el, prm, x = _setup(level=7, cn=0.04)
    phi = np.tanh((x[:, 0] - 0.5) / (np.sqrt(2) * prm.Cn))
    assert np.sqrt(chns.mass(el, (2 * chns.dpsi(phi)) ** 2)) > 100 * errs[-1]


def test_advection_moves_drop_along_velocity_and_conserves_mass():
    m, el, prm, x = _setup(level=5, cn=0.04, dt=2e-3)
    n = m.n_indep
    phi = ci.phi_drop2d(x, centre=(0.4, 0.5), radius=0.15, cn=prm.Cn)
    mu = chns.initial_mu(el, prm, phi)
    # divergence-free shear flow u = (sin^2(pi y), 0), equal to 1 at the drop
    # centre; the centroid is taken away from the walls at x = 0 and x = 1
    ut = np.zeros((2, n))
    ut[0] = np.sin(np.pi * x[:, 1]) ** 2

    def centroid(p):
        w = el.detJ[:, None]
        xq = el.val(x[:, 0])
        window = (xq > 0.15) & (xq < 0.85)
        heavy = el.val(0.5 * (p + 1.0)) * window
        return (w * heavy * xq).sum() / (w * heavy).sum()

    c0, m0 = centroid(phi), chns.mass(el, phi)
    for _ in range(5):
        phi, mu, nit, hist = chns.ch_solve(el, prm, phi, mu, ut, rtol=1e-12, atol=1e-13)
    assert centroid(phi) - c0 == pytest.approx(5 * prm.dt, rel=0.35)
    assert abs(chns.mass(el, phi) - m0) < 1e-12


def test_vp_reduces_to_mass_plus_viscous_when_uhat_and_J_vanish():
    m, el, prm, x = _setup(level=4, cn=0.05, rho_minus=0.1, eta_minus=0.01)
    n = m.n_indep
    phit = ci.phi_drop2d(x, cn=prm.Cn)
    mut = np.zeros(n)
    z = np.zeros((2, n))
    S = chns.QPState(el, prm, phit, mut, z, z, np.zeros(n))
    A = chns.vp_matrix(el, prm, S).toarray()
    rq = prm.rho(fem.qp_values(m, phit))
    eq = prm.eta(fem.qp_values(m, phit))
    ref = (fem.mass_matrix(m, rq) / prm.dt + fem.stiffness_matrix(m, eq) / (2 * prm.Re)).toarray()
    wall = el.wall()
    ref[wall, :] = 0.0
    ref[:, wall] = 0.0
    ref[wall, wall] = 1.0
    assert np.abs(A - ref).max() <= 1e-12 * np.abs(ref).max()
    # tau_m closed form (u^ = J = 0)
    h = 1.0 / (1 << 4)
    tau = (4 / prm.dt ** 2 + prm.C_I * 2 * (2 / h) ** 4 * (eq / (rq * prm.Re)) ** 2) ** -0.5
    assert np.allclose(S.tau, tau, rtol=1e-14, atol=0)


def test_steps_conserve_mass_and_do_not_raise_energy():
    m, el, prm, x = _setup(level=4, cn=0.04, dt=1e-3, Re=100.0, rho_minus=0.1, eta_minus=0.1)
    phi0 = ci.phi_drop2d(x, cn=prm.Cn)
    st = chns.initial_state(el, prm, phi0)
    m0 = chns.mass(el, st.phi)
    e = [chns.energy(el, prm, st)]
    for _ in range(4):
        st, info = chns.step(el, prm, st)
        e.append(chns.energy(el, prm, st))
        assert abs(chns.mass(el, st.phi) - m0) <= 1e-12 * abs(m0) + 1e-13
        assert max(info["newton"]) <= 3
    assert all(e[k + 1] <= e[k] + 1e-12 * abs(e[0]) for k in range(len(e) - 1)), e
    assert e[-1] < e[0]
    # the drop is heavy and falls: the velocity points down near its centre
    c = np.argmin(np.linalg.norm(x - 0.5, axis=1))
    assert st.u[1][c] < 0


def test_projection_reduces_divergence():
    m, el, prm, x = _setup(level=4, cn=0.04, dt=1e-3)
    phi0 = ci.phi_drop2d(x, cn=prm.Cn)
    st = chns.initial_state(el, prm, phi0)
    uhat = 1.5 * st.u - 0.5 * st.u_prev
    phi1, mu1, *_ = chns.ch_solve(el, prm, st.phi, st.mu, st.u)
    phit, mut = 0.5 * (phi1 + st.phi), 0.5 * (mu1 + st.mu)
    S = chns.QPState(el, prm, phit, mut, uhat, st.u, st.p)
    import scipy.sparse.linalg as spla
    A = chns.vp_matrix(el, prm, S).tocsc()
    v = np.stack([spla.spsolve(A, b) for b in chns.vp_rhs(el, prm, S, st.u, st.p, phit)])
    p = chns.solve_singular(chns.pp_matrix_rhot(el, prm, S), chns.pp_rhs(el, prm, S, v, st.p))
    M = chns.rho_mass_walls(el, prm, S).tocsc()
    u = np.stack([spla.spsolve(M, b) for b in chns.vu_rhs(el, prm, S, v, p, st.p)])

    def div_norm(w):
        d = sum(el.grad(w[i])[..., i] for i in range(2))
        return np.sqrt((el.detJ[:, None] * d ** 2).sum())

    assert div_norm(u) < 0.5 * div_norm(v)


def test_static_drop_pressure_jump_follows_laplace_law():
    # Young-Laplace: for the equilibrium profile the capillary term
    # (Cn/We) d_j(d_i phi d_j phi) integrates across a circular interface of
    # radius R to a pressure jump (Cn/We)(1/R) int phi'^2 dr = 2 sqrt(2)/(3 We R).
    # The scheme's momentum equation sees the average of p^k and p^{k+1}
    # (the velocity update carries dt/2 grad(p^{k+1} - p^k)), so the average
    # of consecutive pressures is compared.  A flipped or mis-scaled capillary
    # term, or a wrong factor in the pressure / update chain, fails this.
    m, el, prm, x = _setup(level=6, cn=0.04, Re=1.0, We=1.0, Fr=1e12, rho_minus=1.0, eta_minus=1.0, dt=1e-3)
    R = 0.25
    st = chns.initial_state(el, prm, ci.phi_drop2d(x, radius=R, cn=prm.Cn))
    c = np.argmin(np.linalg.norm(x - 0.5, axis=1))
    far = np.argmin(np.linalg.norm(x - 0.05, axis=1))
    laplace = 2.0 * np.sqrt(2.0) / (3.0 * prm.We * R)
    p_prev = st.p.copy()
    for _ in range(2):
        st, _info = chns.step(el, prm, st)
        avg = 0.5 * (st.p + p_prev)
        assert avg[c] - avg[far] == pytest.approx(laplace, rel=0.05)
        p_prev = st.p.copy()
    assert np.abs(st.u).max() < 0.01
