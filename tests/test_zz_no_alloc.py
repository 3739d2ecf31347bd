"""The allocation-free apply (chns_apply_operator_noalloc), called through the
C ABI, against chns_apply_operator on the same inputs: the same kernels with
the slot partial sums in the library's static per-GPU scratch, so the result
is bitwise the same.  Two calls in a row, the second on a smaller mesh (the
scratch keeps the first call's contents, which the second overwrites), for
the pressure operator in FP64 and FP32 and for the Cahn-Hilliard Jacobian;
a mesh that needs more scratch than the array holds is refused with
CHNS_EINVAL and the context stays usable.
"""
import ctypes as C

import numpy as np
import pytest

import chns_inputs as ci

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _noalloc(ctx, op, prec, x, y):
    from paper_2107_05123_amd import _lib as L
    return L.lib().chns_apply_operator_noalloc(ctx._h, op, prec, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                               C.c_void_p(torch.cuda.current_stream().cuda_stream))


def _setup(spec, seed):
    from paper_2107_05123_amd import Context, Mesh
    m = Mesh(**spec)
    ctx = Context(m, Re=35.0, We=10.0, Cn=0.04, rho_plus=1.0, rho_minus=1e-3, eta_plus=1.0, eta_minus=1e-2, dt=5e-4)
    x_unit = ci.unit_coords(m.node_coords(), m.max_level)
    phi = ci.phi_bubble(x_unit, cn=0.04)
    ctx.set_phase_field(_dev(phi))
    rng = np.random.default_rng(seed)
    n = m.n_nodes
    ut = 0.3 * rng.standard_normal(m.dim * n)
    ctx.set_coefficients(ctx.CH_JACOBIAN, [_dev(phi + 0.05 * rng.standard_normal(n)), _dev(phi), _dev(ut)])
    print(f"mesh {spec}: n={n} slots={m.info.n_slots}", flush=True)
    return m, ctx, rng


def _check_ops(ctx, n, rng):
    from paper_2107_05123_amd import _lib as L
    for op, nf in ((ctx.PRESSURE, 1), (ctx.CH_JACOBIAN, 2)):
        x = _dev(rng.standard_normal(nf * n))
        ref = ctx.apply(op, x)
        y = torch.full_like(ref, float("nan"))
        assert _noalloc(ctx, op, L.FP64, x, y) == L.OK, L.lib().chns_last_error()
        torch.cuda.synchronize()
        assert torch.equal(y, ref), float((y - ref).abs().max())
    x32 = _dev(rng.standard_normal(n), torch.float32)
    ref32 = ctx.apply(ctx.PRESSURE, x32)
    y32 = torch.full_like(ref32, float("nan"))
    assert _noalloc(ctx, ctx.PRESSURE, L.FP32, x32, y32) == L.OK, L.lib().chns_last_error()
    torch.cuda.synchronize()
    assert torch.equal(y32, ref32)


def test_noalloc_apply_matches_apply_on_two_calls_in_a_row():
    big = dict(dim=3, min_level=3, max_level=6, rule="sphere_band", centres=[(0.5, 0.3, 0.5)], radii=[0.15],
               band=0.06, brick_max=8)
    small = dict(dim=3, min_level=3, max_level=3, rule="uniform")
    m1, c1, r1 = _setup(big, 1)
    _check_ops(c1, m1.n_nodes, r1)
    m2, c2, r2 = _setup(small, 2)
    assert m2.info.n_slots < m1.info.n_slots
    _check_ops(c2, m2.n_nodes, r2)


def test_noalloc_apply_refuses_meshes_beyond_the_scratch():
    from paper_2107_05123_amd import _lib as L
    # 64^3 single-leaf bricks: 2.1 M slots; the three FP64 momentum fields
    # need 50 MB
    m, ctx, rng = _setup(dict(dim=3, min_level=6, max_level=6, rule="uniform", brick_max=1), 3)
    n = m.n_nodes
    phi = ci.phi_bubble(ci.unit_coords(m.node_coords(), m.max_level), cn=0.04)
    ctx.set_coefficients(ctx.MOMENTUM, [_dev(phi), _dev(0.1 * rng.standard_normal(n)),
                                        _dev(0.3 * rng.standard_normal(3 * n))])
    x = _dev(rng.standard_normal(3 * n))
    y = torch.zeros_like(x)
    assert _noalloc(ctx, ctx.MOMENTUM, L.FP64, x, y) == L.EINVAL
    assert b"scratch" in L.lib().chns_last_error()
    assert float(y.abs().max()) == 0.0
    # one FP64 field fits
    x1 = _dev(rng.standard_normal(n))
    y1 = torch.empty_like(x1)
    assert _noalloc(ctx, ctx.PRESSURE, L.FP64, x1, y1) == L.OK
    torch.cuda.synchronize()
    assert torch.equal(y1, ctx.apply(ctx.PRESSURE, x1))
