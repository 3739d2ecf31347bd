"""Manufactured solution of the 2D CHNS system and its body forces (inputs
shared by the oracle and the GPU path).

The paper's manufactured-solution study (Sec. 5.1) takes a solenoidal
velocity, a pressure and phase field / chemical potential that are periodic
in time,

    v   = (pi sin^2(pi x) sin(2 pi y), -pi sin(2 pi x) sin^2(pi y)) sin t,
    p   = cos(pi x) sin(pi y) sin t,
    phi = mu = cos(pi x) cos(pi y) sin t,

substitutes them into the continuous equations (Sec. 2, with 1/We absorbed
into the pressure and mobility 1) and uses what is left over as body forces:

    f_v,i = rho (d_t v_i + v . grad v_i) + J . grad v_i / Pe
            + (Cn/We) d_j(d_i phi d_j phi) + d_i p - d_j(eta d_j v_i) / Re
            - rho g_i / Fr,                                   J = cJ grad mu
    f_phi = d_t phi + div(v phi) - lap(mu) / (Pe Cn),
    f_mu  = mu - psi'(phi) + Cn^2 lap(phi),

so that the manufactured fields solve the forced system exactly.  The
velocity vanishes on the walls and phi, mu have zero normal derivative there,
as the scheme's boundary conditions require.  Fields are sums of products of
sines, so every derivative is exact (a derivative shifts a phase by pi/2).

This module evaluates the prescribed fields and the continuous equations at
given points; it holds none of the discretisation (no shape functions,
quadrature, time stepping or solver).  Parameters follow the paper's study:
Re 10, We 1, Cn 1, Pe 3, Fr 1, density ratio rho-/rho+ = 0.85; the viscosity
ratio is not stated and is taken equal to the density ratio, so that the
variable-viscosity terms take part.
"""
from __future__ import annotations

import numpy as np

PI = np.pi
PARAMS = dict(Re=10.0, We=1.0, Cn=1.0, Pe=3.0, Fr=1.0, rho_plus=1.0, rho_minus=0.85, eta_plus=1.0,
              eta_minus=0.85, C_I=6.0, gravity_axis=1)


class SinField:
    """sum_k c_k prod_d sin(w_kd x_d + s_kd) in 2D."""

    def __init__(self, terms):
        self.terms = [(float(c), np.asarray(w, float), np.asarray(s, float)) for c, w, s in terms]

    def __call__(self, x):
        out = np.zeros(x.shape[0])
        for c, w, s in self.terms:
            out += c * np.prod(np.sin(x * w[None, :] + s[None, :]), axis=1)
        return out

    def d(self, k):
        e = np.eye(2)[k]
        return SinField([(c * w[k], w, s + e * PI / 2) for c, w, s in self.terms])

    def grad(self, x):
        return np.stack([self.d(0)(x), self.d(1)(x)], axis=1)

    def lap(self, x):
        return self.d(0).d(0)(x) + self.d(1).d(1)(x)


H = PI / 2  # phase of a cosine / a constant factor
# spatial parts (the time factor is sin t): sin^2(pi x) = 1/2 - cos(2 pi x)/2
V1 = SinField([(PI / 2, [0, 2 * PI], [H, 0]), (-PI / 2, [2 * PI, 2 * PI], [H, 0])])
V2 = SinField([(-PI / 2, [2 * PI, 0], [0, H]), (PI / 2, [2 * PI, 2 * PI], [0, H])])
P = SinField([(1.0, [PI, PI], [H, 0])])
PHI = SinField([(1.0, [PI, PI], [H, H])])
MU = PHI


def fields(x, t):
    """Manufactured (v (2, n), p, phi, mu) at points x (n, 2) and time t."""
    s = np.sin(t)
    return np.stack([V1(x), V2(x)]) * s, P(x) * s, PHI(x) * s, MU(x) * s


def forcing(x, t, prm=PARAMS):
    """Body forces (f_v (2, n), f_phi, f_mu) at points x and time t."""
    s, c = np.sin(t), np.cos(t)
    a, b = prm["rho_plus"], prm["rho_minus"]
    alpha, beta = (a - b) / (2 * a), (a + b) / (2 * a)
    ea, eb = prm["eta_plus"], prm["eta_minus"]
    gam, xi = (ea - eb) / (2 * ea), (ea + eb) / (2 * ea)
    Re, We, Cn, Pe, Fr = prm["Re"], prm["We"], prm["Cn"], prm["Pe"], prm["Fr"]
    cJ = (b - a) / (2 * a * Cn)
    V = [V1, V2]
    v = np.stack([f(x) for f in V]) * s
    phi = PHI(x) * s
    gphi = PHI.grad(x) * s
    lphi = PHI.lap(x) * s
    mu = MU(x) * s
    gmu = MU.grad(x) * s
    rho = alpha * phi + beta            # |phi| <= 1: the pull back is the identity
    eta = gam * phi + xi
    geta = gam * gphi
    J = cJ * gmu
    fv = []
    for i in range(2):
        dv_dt = V[i](x) * c
        gv = V[i].grad(x) * s
        lv = V[i].lap(x) * s
        kort = sum(PHI.d(i).d(j)(x) * s * gphi[:, j] for j in range(2)) + gphi[:, i] * lphi
        grav = -1.0 if i == prm["gravity_axis"] else 0.0
        fv.append(rho * (dv_dt + (v.T * gv).sum(1)) + (J * gv).sum(1) / Pe + Cn / We * kort
                  + P.d(i)(x) * s - ((geta * gv).sum(1) + eta * lv) / Re - rho * grav / Fr)
    div_v = V[0].d(0)(x) * s + V[1].d(1)(x) * s
    fphi = PHI(x) * c + (v.T * gphi).sum(1) + phi * div_v - MU.lap(x) * s / (Pe * Cn)
    fmu = mu - (phi ** 3 - phi) + Cn ** 2 * lphi
    return np.stack(fv), fphi, fmu
