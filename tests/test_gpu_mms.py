"""Manufactured solutions for the whole scheme on the GPU (paper Sec. 5.1).

* Forced steps (body forces through chns_step_opts) match the oracle's
  forced steps to 1e-6 in every field, on a uniform and an adaptive mesh.
* Spatial convergence at a fixed small time step (levels 5-8, 32^2 to 256^2
  quads): every field converges at second order to the manufactured solution
  (L2 errors measured with the library's mass matrix).
* Temporal convergence on the paper's 512^2 mesh to t = 1 with 8, 16, 32
  steps: the phase field at second order (the chemical potential too until
  it meets the spatial error of the mesh), the pressure at least at first
  order (the scheme carries the pressure of the previous step), the velocity
  error falling until it meets the spatial error of the mesh (the paper's
  velocity rate likewise tapers off).
"""
import numpy as np
import pytest

import mms_inputs as mi
from oracle import chns

from ._pairs import Pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# parity runs solve to 1e-11; the convergence studies to 1e-10 (far below the
# discretisation errors; on the 512^2 mesh 1e-11 is at the FP64 rounding floor
# of the pressure system)
STEP = dict(lin_rtol=1e-11, ch_pc="schur", pp_pc="gmg", vp_pc="gmg")
STUDY = dict(STEP, lin_rtol=1e-10)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _gpu_run(mesh, ctx, x, nsteps, T, **kw):
    n = mesh.n_nodes
    z = torch.zeros(2 * n, dtype=torch.float64, device="cuda")
    st = {"u": z.clone(), "u_prev": z.clone(), "p": z[:n].clone(), "phi": z[:n].clone(), "mu": z[:n].clone()}
    dt = T / nsteps
    for k in range(nsteps):
        fv, fphi, fmu = mi.forcing(x, (k + 0.5) * dt)
        s = ctx.advance_step(st, forcing=(_dev(fv.reshape(-1)), _dev(fphi), _dev(fmu)), **kw)
    return st, s


def _errors(ctx, st, x, T):
    v, p, phi, mu = mi.fields(x, T)
    n = x.shape[0]

    def l2(e):
        e = _dev(e)
        return float(torch.dot(e, ctx.apply(ctx.MASS, e))) ** 0.5
    u = st["u"].cpu().numpy().reshape(2, n)
    return {"v": np.hypot(l2(u[0] - v[0]), l2(u[1] - v[1])), "p": l2(st["p"].cpu().numpy() - p),
            "phi": l2(st["phi"].cpu().numpy() - phi), "mu": l2(st["mu"].cpu().numpy() - mu)}


@pytest.mark.parametrize("kind,lmin,lmax", [("uniform", 5, 5), ("band", 3, 6)])
def test_forced_steps_match_oracle(kind, lmin, lmax):
    from paper_2107_05123_amd import Context
    pair = Pair(kind, 2, lmin, lmax, centre=(0.5, 0.5), radius=0.3, band=0.05)
    T, nsteps = 0.25, 8
    prm = chns.Params(dt=T / nsteps, **mi.PARAMS)
    ctx = Context(pair.lib, dt=T / nsteps, **mi.PARAMS)
    x = pair.x_unit
    print(f"{kind} {lmin}-{lmax}: n={pair.lib.n_nodes} hanging={pair.lib.info.n_hanging}", flush=True)
    st, _ = _gpu_run(pair.lib, ctx, x, nsteps, T, **STEP)
    el = chns.Elems(pair.orc)
    xo = pair.orc.indep_coords() / pair.orc.side
    n = pair.lib.n_nodes
    z = np.zeros((2, n))
    ost = chns.State(u=z.copy(), u_prev=z.copy(), p=np.zeros(n), phi=np.zeros(n), mu=np.zeros(n))
    for k in range(nsteps):
        ost, _ = chns.step(el, prm, ost, forcing=mi.forcing(xo, (k + 0.5) * prm.dt))
    got = {k: v.cpu().numpy() for k, v in st.items()}
    for name, ref in (("phi", ost.phi), ("mu", ost.mu), ("p", ost.p)):
        err = np.linalg.norm(pair.to_orc(got[name]) - ref) / np.linalg.norm(ref)
        print(f"{name}: {err:.2e}", flush=True)
        assert err <= 1e-6, (name, err)
    u = got["u"].reshape(2, n)
    uo = np.stack([pair.to_orc(u[0]), pair.to_orc(u[1])])
    err = np.linalg.norm(uo - ost.u) / np.linalg.norm(ost.u)
    print(f"u: {err:.2e}", flush=True)
    assert err <= 1e-6


def _uniform(level, dt):
    from paper_2107_05123_amd import Context, Mesh
    import chns_inputs as ci
    m = Mesh(dim=2, min_level=level, max_level=level, rule="uniform")
    return m, Context(m, dt=dt, **mi.PARAMS), ci.unit_coords(m.node_coords(), level)


def test_manufactured_solution_converges_at_second_order_in_space():
    T, nsteps = 0.25, 64
    errs = []
    for level in (5, 6, 7, 8):
        m, ctx, x = _uniform(level, T / nsteps)
        st, s = _gpu_run(m, ctx, x, nsteps, T, **STUDY)
        errs.append(_errors(ctx, st, x, T))
        print(level, {k: "%.3e" % v for k, v in errs[-1].items()}, flush=True)
    for k in ("phi", "mu", "v", "p"):
        e = [x[k] for x in errs]
        rates = [np.log2(e[i] / e[i + 1]) for i in range(3)]
        print(k, ["%.2f" % r for r in rates], flush=True)
        assert rates[-1] > 1.8, (k, e, rates)


def test_manufactured_solution_converges_in_time():
    T = 1.0
    errs = []
    for nsteps in (8, 16, 32):
        m, ctx, x = _uniform(9, T / nsteps)
        st, s = _gpu_run(m, ctx, x, nsteps, T, **STUDY)
        errs.append(_errors(ctx, st, x, T))
        print(nsteps, {k: "%.3e" % v for k, v in errs[-1].items()}, flush=True)
    for k, floor in (("phi", (1.8, 1.8)), ("mu", (1.8, 1.2)), ("p", (0.9, 0.9))):
        e = [x[k] for x in errs]
        rates = [np.log2(e[i] / e[i + 1]) for i in range(2)]
        print(k, ["%.2f" % r for r in rates], flush=True)
        assert rates[0] > floor[0] and rates[1] > floor[1], (k, e, rates)
    e = [x["v"] for x in errs]
    assert e[1] < 0.5 * e[0], e
