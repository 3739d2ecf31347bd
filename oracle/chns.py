"""Oracle for the CHNS time step: Cahn-Hilliard residual and Newton Jacobian,
VMS velocity prediction, pressure Poisson right-hand side, velocity update and
the two-block projection step, all as assembled FP64 sparse systems solved
with sparse LU.

TEST INFRASTRUCTURE ONLY (see oracle/mesh.py).

Equations (paper Sec. 2-3):
* mixture laws rho(phi) = alpha phi + beta, eta(phi) = gamma phi + xi, with
  the pull back phi* (remark on the pull back) in rho and eta only;
* psi(phi) = (phi^2 - 1)^2 / 4, psi' = phi^3 - phi, psi'' = 3 phi^2 - 1;
* time averages: phi~ = (phi^{k+1} + phi^k)/2, mu~ likewise, u~ = (u^k + u^{k+1})/2,
  u^ = (3 u^k - u^{k-1})/2 (read as second-order extrapolation);
* discrete Cahn-Hilliard (Def. 6, diffusion sign of Def. 1):
    R_phi(q) = (q, (phi1 - phi0)/dt) - (grad q, u~ phi~) + 1/(Pe Cn) (grad q, grad mu~)
    R_mu(q)  = -(q, mu~) + (q, psi'(phi~)) + Cn^2 (grad q, grad phi~)
* VMS velocity prediction (Def. 3) with the residual-based fine scales
  rho~ v^f = -tau_m R_m and the VMS parameter tau_m of Sec. 3.1;
* VMS pressure Poisson (Def. 4) including the boxed stabilisation term, and
  the VMS velocity update (Def. 5); the pressure absorbs 1/We (text after
  Def. 1);
* block iteration CH -> VP -> PP -> VU, done twice per step (flowchart).

Readings where the paper is silent or garbled (kept identical on the GPU):
* Gauss points: 2 per direction; every coefficient and every nonlinear
  function (psi', psi'', rho, eta, tau_m) is evaluated at the Gauss points
  from the interpolated nodal fields;
* J in the momentum equation is (rho- - rho+)/(2 rho+ Cn) grad mu~ (the
  chemical potential of the current block, m = 1);
* G = (2/h)^2 I for the cube leaves, so v.G v = (2/h)^2 |v|^2 and
  G:G = d (2/h)^4; C_I = 6;
* inside R_m, Q1 functions have no pure second derivatives: the viscous
  term reduces to grad eta~ . grad v (grad eta~ = gamma grad phi~ where
  |phi~| < 1, else 0) and the capillary divergence to
  sum_{j != i} d_i d_j phi~ d_j phi~;
* velocities are zero on the walls (identity rows); phi and mu have natural
  boundary conditions; gravity is -e_y with Fr.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem
from .mesh import OracleMesh


@dataclass
class Params:
    Re: float = 100.0
    We: float = 1.0
    Cn: float = 0.02
    Pe: float = 0.0          # <= 0: 1/Pe = 3 Cn^2
    Fr: float = 1.0
    rho_plus: float = 1.0
    rho_minus: float = 0.1
    eta_plus: float = 1.0
    eta_minus: float = 0.1
    dt: float = 1e-3
    C_I: float = 6.0
    gravity_axis: int = 1

    @property
    def pe(self):
        return self.Pe if self.Pe > 0 else 1.0 / (3.0 * self.Cn ** 2)

    def rho(self, phi):
        a, b = fem.rho_coeffs(self.rho_plus, self.rho_minus)
        return a * fem.pull_back(phi) + b

    def eta_coeffs(self):
        g = (self.eta_plus - self.eta_minus) / (2.0 * self.eta_plus)
        x = (self.eta_plus + self.eta_minus) / (2.0 * self.eta_plus)
        return g, x

    def eta(self, phi):
        g, x = self.eta_coeffs()
        return g * fem.pull_back(phi) + x

    @property
    def cJ(self):
        return (self.rho_minus - self.rho_plus) / (2.0 * self.rho_plus * self.Cn)


def psi(p):
    return 0.25 * (p * p - 1.0) ** 2


def dpsi(p):
    return p ** 3 - p


def d2psi(p):
    return 3.0 * p * p - 1.0


class Elems:
    """Per-element Gauss-point tabulation on an oracle mesh."""

    def __init__(self, mesh: OracleMesh):
        self.m = mesh
        self.dim = mesh.dim
        self.N, self.dNr = fem.tabulate(mesh.dim)          # (nq, nc), (nq, nc, d)
        self.h = fem.elem_h(mesh)
        self.detJ = (self.h / 2.0) ** mesh.dim              # (E,)
        gs = 2.0 / self.h
        self.dN = self.dNr[None, :, :, :] * gs[:, None, None, None]   # (E, nq, nc, d)
        # mixed second derivatives d_i d_j N_a (i != j) at the Gauss points
        bits = fem.corner_bits(mesh.dim)
        xi_a = 2.0 * bits - 1.0
        xi_q = (2.0 * bits - 1.0) / np.sqrt(3.0)
        nq = nc = 1 << mesh.dim
        H = np.zeros((nq, nc, mesh.dim, mesh.dim))
        for q in range(nq):
            for a in range(nc):
                for i in range(mesh.dim):
                    for j in range(mesh.dim):
                        if i == j:
                            continue
                        f = 1.0
                        for k in range(mesh.dim):
                            if k in (i, j):
                                f *= xi_a[a, k] / 2.0
                            else:
                                f *= (1.0 + xi_a[a, k] * xi_q[q, k]) / 2.0
                        H[q, a, i, j] = f
        self.HN = H[None] * (gs ** 2)[:, None, None, None, None]       # (E, nq, nc, d, d)

    def loc(self, v):
        return (self.m.P @ v)[self.m.elem_nodes]

    def val(self, v):
        return self.loc(v) @ self.N.T

    def grad(self, v):
        return np.einsum("ea,eqad->eqd", self.loc(v), self.dN)

    def hess(self, v):
        return np.einsum("ea,eqaij->eqij", self.loc(v), self.HN)

    def assemble(self, Ke):
        return fem.assemble(self.m, Ke)

    def load(self, Fe):
        """P^T of element vectors (E, nc)."""
        n_all = self.m.nodes.shape[0]
        b = np.zeros(n_all)
        np.add.at(b, self.m.elem_nodes, Fe)
        return self.m.P.T @ b

    def wall(self):
        c = self.m.indep_coords()
        return np.any((c == 0) | (c == self.m.box[None, :]), axis=1)


# ----------------------------------------------------------------- Cahn-Hilliard
def ch_residual(el: Elems, prm: Params, phi1, mu1, phi0, mu0, ut, f_phi=None, f_mu=None):
    """(R_phi, R_mu) of the discrete CH system; ut: (d, n) advecting velocity.

    Optional body forces (nodal values at the step's mid time, manufactured
    solutions): R_phi -= (q, f_phi), R_mu += (q, f_mu)."""
    pt = 0.5 * (phi1 + phi0)
    mt = 0.5 * (mu1 + mu0)
    w = el.detJ[:, None]
    N = el.N
    dphi_dt = el.val(phi1 - phi0) / prm.dt
    ptq = el.val(pt)
    utq = np.stack([el.val(ut[d]) for d in range(el.dim)], axis=-1)        # (E, nq, d)
    gmt = el.grad(mt)
    gpt = el.grad(pt)
    Rphi = (np.einsum("eq,qa->ea", w * dphi_dt, N)
            - np.einsum("eqad,eqd->ea", el.dN, w[..., None] * utq * ptq[..., None])
            + np.einsum("eqad,eqd->ea", el.dN, w[..., None] * gmt) / (prm.pe * prm.Cn))
    Rmu = (np.einsum("eq,qa->ea", w * (dpsi(ptq) - el.val(mt)), N)
           + prm.Cn ** 2 * np.einsum("eqad,eqd->ea", el.dN, w[..., None] * gpt))
    if f_phi is not None:
        Rphi = Rphi - np.einsum("eq,qa->ea", w * el.val(f_phi), N)
    if f_mu is not None:
        Rmu = Rmu + np.einsum("eq,qa->ea", w * el.val(f_mu), N)
    return el.load(Rphi), el.load(Rmu)


def ch_jacobian(el: Elems, prm: Params, phi1, phi0, ut):
    """Jacobian of (R_phi, R_mu) w.r.t. (phi1, mu1) as a 2x2 block sparse matrix."""
    pt = 0.5 * (phi1 + phi0)
    w = el.detJ[:, None]
    N = el.N
    ptq = el.val(pt)
    utq = np.stack([el.val(ut[d]) for d in range(el.dim)], axis=-1)
    MM = np.einsum("eq,qa,qb->eab", w, N, N)
    KK = np.einsum("eq,eqad,eqbd->eab", w, el.dN, el.dN)
    adv = np.einsum("eq,eqad,eqd,qb->eab", w, el.dN, utq, N)
    MP = np.einsum("eq,qa,qb->eab", w * d2psi(ptq), N, N)
    Jpp = el.assemble(MM / prm.dt - 0.5 * adv)
    Jpm = el.assemble(KK / (2.0 * prm.pe * prm.Cn))
    Jmp = el.assemble(0.5 * MP + 0.5 * prm.Cn ** 2 * KK)
    Jmm = el.assemble(-0.5 * MM)
    return sp.bmat([[Jpp, Jpm], [Jmp, Jmm]]).tocsr()


def ch_solve(el: Elems, prm: Params, phi0, mu0, ut, phi_guess=None, mu_guess=None, rtol=1e-8, atol=1e-12,
             max_newton=20, f_phi=None, f_mu=None):
    """Newton iteration x <- x - J^{-1} R until |R| <= max(rtol |R0|, atol)."""
    n = phi0.shape[0]
    phi = (phi0 if phi_guess is None else phi_guess).copy()
    mu = (mu0 if mu_guess is None else mu_guess).copy()
    Rp, Rm = ch_residual(el, prm, phi, mu, phi0, mu0, ut, f_phi, f_mu)
    r0 = np.linalg.norm(np.concatenate([Rp, Rm]))
    hist = [r0]
    it = 0
    while hist[-1] > max(rtol * r0, atol) and it < max_newton:
        J = ch_jacobian(el, prm, phi, phi0, ut)
        d = spla.spsolve(J.tocsc(), -np.concatenate([Rp, Rm]))
        phi = phi + d[:n]
        mu = mu + d[n:]
        Rp, Rm = ch_residual(el, prm, phi, mu, phi0, mu0, ut, f_phi, f_mu)
        hist.append(np.linalg.norm(np.concatenate([Rp, Rm])))
        it += 1
    return phi, mu, it, hist


def initial_mu(el: Elems, prm: Params, phi0):
    """L2 projection: (q, mu0) = (q, psi'(phi0)) + Cn^2 (grad q, grad phi0)."""
    w = el.detJ[:, None]
    M = el.assemble(np.einsum("eq,qa,qb->eab", w, el.N, el.N))
    rhs = el.load(np.einsum("eq,qa->ea", w * dpsi(el.val(phi0)), el.N)
                  + prm.Cn ** 2 * np.einsum("eqad,eqd->ea", el.dN, w[..., None] * el.grad(phi0)))
    return spla.spsolve(M.tocsc(), rhs)


# ------------------------------------------------------------ VMS momentum
class QPState:
    """Gauss-point coefficients shared by the velocity prediction, the
    pressure right-hand side and the velocity update."""

    def __init__(self, el: Elems, prm: Params, phit, mut, uhat, uk, pk, f_v=None):
        """f_v: optional body force (d, n) at the step's mid time; it is the
        known right-hand side of the momentum equation, so it enters R_m
        with a minus sign (and the velocity-prediction right-hand side)."""
        d = el.dim
        self.fvq = None if f_v is None else [el.val(f_v[i]) for i in range(d)]
        self.ptq = el.val(phit)
        self.rho = prm.rho(self.ptq)
        self.eta = prm.eta(self.ptq)
        g, _ = prm.eta_coeffs()
        self.gphi = el.grad(phit)
        inside = (np.abs(self.ptq) < 1.0)[..., None]
        self.geta = g * self.gphi * inside
        self.uh = np.stack([el.val(uhat[i]) for i in range(d)], axis=-1)      # (E, nq, d)
        self.J = prm.cJ * el.grad(mut)
        gs2 = (2.0 / el.h) ** 2
        arg = (4.0 / prm.dt ** 2 + gs2[:, None] * (self.uh ** 2).sum(-1)
               + gs2[:, None] * (self.uh * self.J).sum(-1) / (self.rho * prm.pe)
               + prm.C_I * d * (gs2 ** 2)[:, None] * (self.eta / (self.rho * prm.Re)) ** 2)
        self.tau = 1.0 / np.sqrt(arg)
        # stabilisation test functions s_a = 1/2 u^.grad N_a + 1/(2 Pe rho) J.grad N_a
        self.s = (0.5 * np.einsum("eqd,eqad->eqa", self.uh, el.dN)
                  + np.einsum("eqd,eqad->eqa", self.J, el.dN) / (2.0 * prm.pe * self.rho[..., None]))
        # known parts of R_m for each component i (u = u^k, p = p^k)
        H = el.hess(phit)
        self.Rk = []
        for i in range(d):
            ui = el.val(uk[i])
            gui = el.grad(uk[i])
            kort = sum(H[..., i, j] * self.gphi[..., j] for j in range(d) if j != i)
            gp = el.grad(pk)[..., i]
            grav = -1.0 if i == prm.gravity_axis else 0.0
            rk = (-self.rho * ui / prm.dt
                  + 0.5 * self.rho * (self.uh * gui).sum(-1)
                  + (self.J * gui).sum(-1) / (2.0 * prm.pe)
                  - (self.geta * gui).sum(-1) / (2.0 * prm.Re)
                  + prm.Cn / prm.We * kort + gp - self.rho * grav / prm.Fr)
            if self.fvq is not None:
                rk = rk - self.fvq[i]
            self.Rk.append(rk)

    def rlin_of(self, el, prm, v):
        """R_lin(v) at the Gauss points for a nodal field v."""
        vq = el.val(v)
        gv = el.grad(v)
        return (self.rho * vq / prm.dt + 0.5 * self.rho * (self.uh * gv).sum(-1)
                + (self.J * gv).sum(-1) / (2.0 * prm.pe) - (self.geta * gv).sum(-1) / (2.0 * prm.Re))


def vp_matrix(el: Elems, prm: Params, S: QPState):
    """Velocity-prediction operator of one component (identical for all)
    with identity rows and zero columns on the walls."""
    w = el.detJ[:, None]
    N = el.N
    dN = el.dN
    rho, eta, uh, J, tau = S.rho, S.eta, S.uh, S.J, S.tau
    gal = (np.einsum("eq,qa,qb->eab", w * rho / prm.dt, N, N)
           + 0.5 * np.einsum("eq,qa,eqd,eqbd->eab", w * rho, N, uh, dN)
           + np.einsum("eq,qa,eqd,eqbd->eab", w, N, J, dN) / (2.0 * prm.pe)
           + np.einsum("eq,eqad,eqbd->eab", w * eta, dN, dN) / (2.0 * prm.Re))
    rlin = (rho[..., None] * N[None] / prm.dt + 0.5 * rho[..., None] * np.einsum("eqd,eqbd->eqb", uh, dN)
            + np.einsum("eqd,eqbd->eqb", J, dN) / (2.0 * prm.pe)
            - np.einsum("eqd,eqbd->eqb", S.geta, dN) / (2.0 * prm.Re))
    stab = np.einsum("eq,eqa,eqb->eab", w * tau, S.s, rlin)
    A = el.assemble(gal + stab).tolil()
    wall = np.nonzero(el.wall())[0]
    A[wall, :] = 0.0
    A[:, wall] = 0.0
    for i in wall:
        A[i, i] = 1.0
    return A.tocsr()


def vp_rhs(el: Elems, prm: Params, S: QPState, uk, pk, phit):
    """Right-hand sides of the velocity prediction, one per component."""
    w = el.detJ[:, None]
    N = el.N
    d = el.dim
    wall = el.wall()
    out = []
    for i in range(d):
        ui = el.val(uk[i])
        gui = el.grad(uk[i])
        gp = el.grad(pk)[..., i]
        grav = -1.0 if i == prm.gravity_axis else 0.0
        f_N = (S.rho * ui / prm.dt - 0.5 * S.rho * (S.uh * gui).sum(-1) - (S.J * gui).sum(-1) / (2.0 * prm.pe)
               - gp + S.rho * grav / prm.Fr)
        if S.fvq is not None:
            f_N = f_N + S.fvq[i]
        b = (np.einsum("eq,qa->ea", w * f_N, N)
             - np.einsum("eqad,eqd->ea", el.dN, w[..., None] * S.eta[..., None] * gui) / (2.0 * prm.Re)
             + prm.Cn / prm.We * np.einsum("eqad,eqd->ea", el.dN,
                                           w[..., None] * S.gphi[..., i:i + 1] * S.gphi)
             - np.einsum("eq,eqa->ea", w * S.tau * S.Rk[i], S.s))
        bi = el.load(b)
        bi[wall] = 0.0
        out.append(bi)
    return out


def pp_rhs(el: Elems, prm: Params, S: QPState, v, pk):
    """-(2/dt)(q, div v) - (2/dt)(grad q, tau R_m / rho) + (grad q, grad p^k / rho)."""
    w = el.detJ[:, None]
    d = el.dim
    div = sum(el.grad(v[i])[..., i] for i in range(d))
    tR = np.stack([S.tau * (S.rlin_of(el, prm, v[i]) + S.Rk[i]) for i in range(d)], axis=-1)  # (E, nq, d)
    gp = el.grad(pk)
    b = (-(2.0 / prm.dt) * np.einsum("eq,qa->ea", w * div, el.N)
         - (2.0 / prm.dt) * np.einsum("eqad,eqd->ea", el.dN, w[..., None] * tR / S.rho[..., None])
         + np.einsum("eqad,eqd->ea", el.dN, w[..., None] * gp / S.rho[..., None]))
    return el.load(b)


def vu_rhs(el: Elems, prm: Params, S: QPState, v, p_new, pk):
    """(w, rho v_i) - (w, tau R_m,i) - (dt/2)(w, d_i (p^{k+1} - p^k)), walls zero."""
    w = el.detJ[:, None]
    d = el.dim
    wall = el.wall()
    gdp = el.grad(p_new - pk)
    out = []
    for i in range(d):
        f = (S.rho * el.val(v[i]) - S.tau * (S.rlin_of(el, prm, v[i]) + S.Rk[i]) - 0.5 * prm.dt * gdp[..., i])
        bi = el.load(np.einsum("eq,qa->ea", w * f, el.N))
        bi[wall] = 0.0
        out.append(bi)
    return out


def rho_mass_walls(el: Elems, prm: Params, S: QPState):
    w = el.detJ[:, None]
    M = el.assemble(np.einsum("eq,qa,qb->eab", w * S.rho, el.N, el.N)).tolil()
    wall = np.nonzero(el.wall())[0]
    M[wall, :] = 0.0
    M[:, wall] = 0.0
    for i in wall:
        M[i, i] = 1.0
    return M.tocsr()


def pp_matrix_rhot(el: Elems, prm: Params, S: QPState):
    w = el.detJ[:, None]
    return el.assemble(np.einsum("eq,eqad,eqbd->eab", w / S.rho, el.dN, el.dN))


# ------------------------------------------------------------------ time step
@dataclass
class State:
    u: np.ndarray       # (d, n) u^k
    u_prev: np.ndarray  # (d, n) u^{k-1}
    p: np.ndarray       # (n,)
    phi: np.ndarray
    mu: np.ndarray


def initial_state(el: Elems, prm: Params, phi0):
    n = phi0.shape[0]
    z = np.zeros((el.dim, n))
    return State(u=z.copy(), u_prev=z.copy(), p=np.zeros(n), phi=phi0.copy(), mu=initial_mu(el, prm, phi0))


def solve_singular(A, b):
    """Pure-Neumann pressure system: b projected to 1^T b = 0, solution mean-free."""
    n = A.shape[0]
    b = b - b.mean()
    one = np.ones((n, 1))
    Ab = sp.bmat([[A, sp.csr_matrix(one)], [sp.csr_matrix(one.T), None]]).tocsc()
    x = spla.spsolve(Ab, np.concatenate([b, [0.0]]))[:n]
    return x - x.mean()


def step(el: Elems, prm: Params, st: State, blocks=2, forcing=None):
    """One projection time step: `blocks` passes of CH -> VP -> PP -> VU.

    forcing: optional body forces (f_v (d, n), f_phi, f_mu), nodal values at
    the step's mid time t^k + dt/2 (the time the scheme's averages are
    centred on), used by manufactured solutions."""
    d = el.dim
    f_v, f_phi, f_mu = forcing if forcing is not None else (None, None, None)
    uhat = 1.5 * st.u - 0.5 * st.u_prev
    u_new = st.u.copy()
    phi1, mu1 = st.phi.copy(), st.mu.copy()
    p_new = st.p.copy()
    info = {"newton": []}
    for _ in range(blocks):
        ut = 0.5 * (st.u + u_new)
        phi1, mu1, nit, hist = ch_solve(el, prm, st.phi, st.mu, ut, phi1, mu1, f_phi=f_phi, f_mu=f_mu)
        info["newton"].append(nit)
        phit = 0.5 * (phi1 + st.phi)
        mut = 0.5 * (mu1 + st.mu)
        S = QPState(el, prm, phit, mut, uhat, st.u, st.p, f_v)
        A = vp_matrix(el, prm, S).tocsc()
        v = np.stack([spla.spsolve(A, b) for b in vp_rhs(el, prm, S, st.u, st.p, phit)])
        p_new = solve_singular(pp_matrix_rhot(el, prm, S), pp_rhs(el, prm, S, v, st.p))
        M = rho_mass_walls(el, prm, S).tocsc()
        u_new = np.stack([spla.spsolve(M, b) for b in vu_rhs(el, prm, S, v, p_new, st.p)])
    new = State(u=u_new, u_prev=st.u.copy(), p=p_new, phi=phi1, mu=mu1)
    return new, info


def mass(el: Elems, phi):
    return float((el.detJ[:, None] * el.val(phi)).sum())


def energy(el: Elems, prm: Params, st: State):
    """E = int 1/2 rho |u|^2 + 1/(Cn We) int (psi + Cn^2/2 |grad phi|^2) + 1/Fr int rho y."""
    w = el.detJ[:, None]
    rho = prm.rho(el.val(st.phi))
    ke = 0.5 * (w * rho * sum(el.val(st.u[i]) ** 2 for i in range(el.dim))).sum()
    gp = el.grad(st.phi)
    fe = (w * (psi(el.val(st.phi)) + 0.5 * prm.Cn ** 2 * (gp ** 2).sum(-1))).sum() / (prm.Cn * prm.We)
    y = el.val(el.m.indep_coords()[:, prm.gravity_axis].astype(float) / el.m.side)
    pe = (w * rho * y).sum() / prm.Fr
    return float(ke + fe + pe)
