"""GPU edge cases through the C ABI.

* The smallest meshes and ragged brick classes: uniform level 1 in 2D and 3D
  (2^d single-leaf bricks), level-2 uniform, small band meshes made of single
  leaves with hanging nodes, and a levels 3-7 band mesh whose leaves fall
  into 4^3, 2^3 and single-leaf bricks (8^3 bricks: the uniform full-size
  tests): the FP64 apply matches the oracle's assembled matrix to 1e-12, FP32
  to 2e-5; the zero vector maps to zero exactly and constants to zero within
  rounding.
* Error behaviour: an operator or a solve before set_phase_field is
  CHNS_ESTATE; aliasing x and y, an unknown precision and multigrid on a
  level-1 mesh (no coarser level) are CHNS_EINVAL; all leave the context
  usable.
* Solves: a zero right-hand side returns x = 0 after zero iterations; a solve
  stopped by max_it is CHNS_ENOCONV with the statistics filled and the last
  iterate in x, whose true residual (oracle matrix) is the reported one.
"""
import ctypes as C

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


def _ctx(pair):
    from paper_2107_05123_amd import Context
    return Context(pair.lib, rho_plus=RHO_P, rho_minus=RHO_M)


SMALL = [
    ("uniform", 2, 1, 1, 0.0),
    ("uniform", 3, 1, 1, 0.0),
    ("uniform", 3, 2, 2, 0.0),
    ("band", 2, 1, 5, 0.05),
    ("band", 3, 1, 4, 0.08),
    ("band", 3, 3, 7, 0.05),
]


@pytest.mark.parametrize("kind,dim,lmin,lmax,band", SMALL, ids=lambda v: str(v))
def test_small_and_ragged_meshes_match_oracle(kind, dim, lmin, lmax, band):
    pair = Pair(kind, dim, lmin, lmax, band=band if band else 0.03)
    info = pair.lib.summary()
    print(f"{kind} {dim}d {lmin}-{lmax}: n={pair.lib.n_nodes} hanging={info['n_hanging']} "
          f"bricks={info['n_bricks']}", flush=True)
    phi = pair.phi("bubble", cn=0.05)
    A = fem.pp_matrix(pair.orc, pair.to_orc(phi), RHO_P, RHO_M)
    ctx = _ctx(pair)
    ctx.set_phase_field(_dev(phi))
    x = ci.normal_vector(3, pair.lib.n_nodes)
    ref = pair.to_lib(A @ pair.to_orc(x))
    y = ctx.apply(ctx.PRESSURE, _dev(x)).cpu().numpy()
    scale = np.abs(ref).max()
    assert np.abs(y - ref).max() <= 1e-12 * scale
    y32 = ctx.apply(ctx.PRESSURE, _dev(x, torch.float32)).cpu().numpy().astype(np.float64)
    assert np.abs(y32 - ref).max() <= 2e-5 * scale
    n = pair.lib.n_nodes
    assert float(ctx.apply(ctx.PRESSURE, torch.zeros(n, dtype=torch.float64, device="cuda")).abs().max()) == 0.0
    ones = ctx.apply(ctx.PRESSURE, torch.ones(n, dtype=torch.float64, device="cuda")).cpu().numpy()
    assert np.abs(ones).max() <= 1e-13 * scale


def test_error_codes_and_recovery():
    from paper_2107_05123_amd import _lib as L
    from paper_2107_05123_amd import Context, Mesh
    mesh = Mesh(dim=3, min_level=2, max_level=2, rule="uniform")
    ctx = Context(mesh, rho_plus=RHO_P, rho_minus=RHO_M)
    n = mesh.n_nodes
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    with pytest.raises(L.ChnsError) as e:
        ctx.apply(ctx.PRESSURE, x)
    assert e.value.code == L.ESTATE
    with pytest.raises(L.ChnsError) as e:
        ctx.solve_pressure(x)
    assert e.value.code == L.ESTATE
    ctx.set_phase_field(torch.zeros(n, dtype=torch.float64, device="cuda"))
    with pytest.raises(L.ChnsError) as e:
        ctx.apply(ctx.PRESSURE, x, x)
    assert e.value.code == L.EINVAL
    y = torch.empty_like(x)
    rc = L.lib().chns_apply_operator(ctx._h, ctx.PRESSURE, 7, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                     C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == L.EINVAL
    assert b"prec" in L.lib().chns_last_error()
    b = ctx.apply(ctx.MASS, _dev(ci.normal_vector(1, n)))
    m1 = Mesh(dim=3, min_level=1, max_level=1, rule="uniform")
    c1 = Context(m1, rho_plus=RHO_P, rho_minus=RHO_M)
    c1.set_phase_field(torch.zeros(m1.n_nodes, dtype=torch.float64, device="cuda"))
    b1 = c1.apply(c1.MASS, _dev(ci.normal_vector(1, m1.n_nodes)))
    with pytest.raises(L.ChnsError) as e:
        c1.solve_pressure(b1, pc="gmg")  # level 1: no coarser level to build
    assert e.value.code == L.EINVAL
    # the contexts still work after every error
    xs, st = ctx.solve_pressure(b, rtol=1e-8, pc="gmg")
    assert st.rel_residual <= 1e-8
    xs, st = c1.solve_pressure(b1, rtol=1e-8)
    assert st.rel_residual <= 1e-8


def test_zero_rhs_and_iteration_limit():
    from paper_2107_05123_amd import _lib as L
    pair = Pair("band", 3, 2, 5, band=0.03)
    phi = pair.phi("bubble", cn=0.02)
    A = fem.pp_matrix(pair.orc, pair.to_orc(phi), RHO_P, RHO_M)
    ctx = _ctx(pair)
    ctx.set_phase_field(_dev(phi))
    n = pair.lib.n_nodes
    zero = torch.zeros(n, dtype=torch.float64, device="cuda")
    for pc in ("jacobi", "gmg"):
        x, st = ctx.solve_pressure(zero, pc=pc)
        assert st.iterations == 0 and st.rel_residual == 0.0
        assert float(x.abs().max()) == 0.0
    amps, waves = ci.rhs_modes(1)
    b = ctx.apply(ctx.MASS, _dev(ci.rhs_field(pair.x_unit, amps, waves)))
    x, st = ctx.solve_pressure(b, rtol=1e-8, max_it=5, raise_on_noconv=False)
    assert st.status == L.ENOCONV and st.iterations == 5
    bo = pair.to_orc(b.cpu().numpy())
    bo = bo - bo.mean()
    rel = np.linalg.norm(bo - A @ pair.to_orc(x.cpu().numpy())) / np.linalg.norm(bo)
    print(f"after 5 iterations: reported {st.rel_residual:.6e}, oracle {rel:.6e}", flush=True)
    assert 1e-8 < rel < 1.0
    assert abs(rel - st.rel_residual) <= 1e-10 * rel
    with pytest.raises(L.ChnsError) as e:
        ctx.solve_pressure(b, rtol=1e-8, max_it=5)
    assert e.value.code == L.ENOCONV
