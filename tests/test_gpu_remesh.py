"""GPU parity of the intergrid transfer and of time stepping across a remesh.

* The device transfer (chns_transfer_apply, one and several fields) against
  the oracle's point evaluation of the old Q1 field at the new nodes: 1e-14
  of max|ref| per field.
* One projection step on the old mesh, a remesh around a moved interface (a
  seeded indicator field, the same on both sides, so both build the same
  mesh), the state carried over by each side's own transfer, one more step on
  the new mesh with a new context: every field within 1e-6 of the oracle,
  which runs the same sequence (steps at the solves' 1e-11, as in the other
  step tests).
"""
import numpy as np
import pytest

from oracle import chns
from oracle import mesh as om
from oracle import remesh as orm

from ._pairs import Pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

THR = 0.95
PRM = dict(Re=100.0, We=1.0, Cn=0.02, Fr=1.0, rho_plus=1.0, rho_minus=0.1, eta_plus=1.0, eta_minus=0.1, dt=1e-3)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _moved_bubble(x_unit, dim, cn, dy):
    c = np.array([0.5, 0.3 + dy, 0.5])[:dim]
    d = np.sqrt(((x_unit - c[None, :]) ** 2).sum(axis=1)) - 0.15
    return np.tanh(d / (np.sqrt(2.0) * cn))


CASES = [(2, 3, 7), (3, 2, 5)]


@pytest.mark.parametrize("dim,lmin,lmax", CASES)
def test_device_transfer_matches_oracle(dim, lmin, lmax):
    from paper_2107_05123_amd import Transfer
    pair = Pair("band", dim, lmin, lmax, band=0.05)
    ind = _moved_bubble(pair.x_unit, dim, 0.02, 0.06)
    new = pair.lib.remesh(ind, lmin, THR)
    new_orc = orm.remesh(pair.orc, pair.to_orc(ind), lmin, THR)
    perm = om.node_index_map(new.node_coords(), new_orc.indep_coords(), 1 << lmax)
    t = Transfer(pair.lib, new)
    rng = np.random.default_rng(11)
    v = rng.standard_normal((3, pair.lib.n_nodes))
    for nf in (1, 3):
        y = t.apply(_dev(v[:nf].reshape(-1)), n_fields=nf).cpu().numpy().reshape(nf, -1)
        for f in range(nf):
            ref = orm.transfer(pair.orc, new_orc, pair.to_orc(v[f]))[perm]
            assert np.abs(y[f] - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("dim,lmin,lmax", CASES)
def test_steps_across_a_remesh_match_oracle(dim, lmin, lmax):
    from paper_2107_05123_amd import Context, Transfer
    pair = Pair("band", dim, lmin, lmax, band=0.05)
    prm = chns.Params(**PRM)
    phi0 = pair.phi("bubble", cn=PRM["Cn"])
    n = pair.lib.n_nodes
    # GPU: one step on the old mesh
    ctx = Context(pair.lib, **PRM)
    z = np.zeros(dim * n)
    st = {"u": _dev(z), "u_prev": _dev(z), "p": _dev(np.zeros(n)), "phi": _dev(phi0)}
    st["mu"] = ctx.initial_mu(st["phi"])
    ctx.advance_step(st, lin_rtol=1e-11)
    # oracle: the same step
    el = chns.Elems(pair.orc)
    ost = chns.step(el, prm, chns.initial_state(el, prm, pair.to_orc(phi0)))[0]
    # remesh both sides around a moved interface (same seeded indicator)
    ind = _moved_bubble(pair.x_unit, dim, PRM["Cn"], 0.05)
    new = pair.lib.remesh(ind, lmin, THR)
    new_orc = orm.remesh(pair.orc, pair.to_orc(ind), lmin, THR)
    m = new.n_nodes
    print(f"{dim}d remesh: {pair.lib.n_elems} -> {new.n_elems} leaves, {n} -> {m} nodes", flush=True)
    t = Transfer(pair.lib, new)
    nst = {"u": t.apply(st["u"], n_fields=dim), "u_prev": t.apply(st["u_prev"], n_fields=dim),
           "p": t.apply(st["p"]), "phi": t.apply(st["phi"]), "mu": t.apply(st["mu"])}
    ctx2 = Context(new, **PRM)
    ctx2.advance_step(nst, lin_rtol=1e-11)
    tr = lambda v: orm.transfer(pair.orc, new_orc, v)
    ost2 = chns.State(u=np.stack([tr(c) for c in ost.u]), u_prev=np.stack([tr(c) for c in ost.u_prev]),
                      p=tr(ost.p), phi=tr(ost.phi), mu=tr(ost.mu))
    ost2 = chns.step(chns.Elems(new_orc), prm, ost2)[0]
    perm = om.node_index_map(new.node_coords(), new_orc.indep_coords(), 1 << lmax)
    got = {k: v.cpu().numpy() for k, v in nst.items()}
    for name in ("phi", "mu", "p"):
        ref = getattr(ost2, name)[perm]
        err = np.linalg.norm(got[name] - ref) / np.linalg.norm(ref)
        print(f"{name}: {err:.3e}", flush=True)
        assert err <= 1e-6, name
    u = got["u"].reshape(dim, m)
    uref = ost2.u[:, perm]
    err = np.linalg.norm(u - uref) / np.linalg.norm(uref)
    print(f"u: {err:.3e}", flush=True)
    assert err <= 1e-6
