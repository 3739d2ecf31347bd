"""Pins for the oracle's pressure-Poisson and mass operators (CPU only).

Independent pins: textbook closed forms of Q1 element matrices, the textbook
assembled Laplacian stencils (equal densities), a hand-derived entry with a
Gauss-point coefficient, invariants (symmetry, constant null space, positive
semi-definiteness, patch test across hanging nodes) and second-order
convergence for a manufactured variable-coefficient Poisson problem.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem, krylov, mesh as om


def _unit_elem_mesh(dim, level=0):
    return om.uniform(dim, level)


def test_q1_stiffness_closed_form_3d():
    m = om.uniform(3, 1)  # h = 1/2
    K = fem.pp_element_matrices(m, np.zeros(m.n_indep), 1.0, 1.0)[0]
    h = 0.5
    bits = fem.corner_bits(3)
    for a in range(8):
        for b in range(8):
            nd = int(np.abs(bits[a] - bits[b]).sum())
            expect = {0: h / 3, 1: 0.0, 2: -h / 12, 3: -h / 12}[nd]
            assert abs(K[a, b] - expect) < 1e-15


def test_q1_stiffness_closed_form_2d():
    m = om.uniform(2, 2)
    K = fem.pp_element_matrices(m, np.zeros(m.n_indep), 1.0, 1.0)[0]
    bits = fem.corner_bits(2)
    for a in range(4):
        for b in range(4):
            nd = int(np.abs(bits[a] - bits[b]).sum())
            expect = {0: 2 / 3, 1: -1 / 6, 2: -1 / 3}[nd]
            assert abs(K[a, b] - expect) < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_q1_mass_closed_form(dim):
    m = om.uniform(dim, 2)
    M = fem.mass_matrix(m).toarray()
    # one element's matrix: tensor product of (h/6)[[2,1],[1,2]]
    h = 0.25
    mono = om.uniform(dim, 0)
    M0 = fem.mass_matrix(mono).toarray()
    bits = fem.corner_bits(dim)
    node_of = {tuple(c): i for i, c in enumerate(mono.indep_coords())}
    for a in range(1 << dim):
        for b in range(1 << dim):
            expect = np.prod([(1.0 / 6.0) * (2.0 if bits[a][d] == bits[b][d] else 1.0) for d in range(dim)])
            ia, ib = node_of[tuple(bits[a])], node_of[tuple(bits[b])]
            assert abs(M0[ia, ib] - expect) < 1e-15
    assert abs(M.sum() - 1.0) < 1e-13  # integrates 1 over the unit domain


def test_assembled_interior_stencils_equal_density():
    for dim, lev in ((2, 3), (3, 3)):
        m = om.uniform(dim, lev)
        A = fem.pp_matrix(m, np.zeros(m.n_indep), 1.0, 1.0).toarray()
        h = 1.0 / (1 << lev)
        coords = m.indep_coords()
        centre = np.full(dim, 1 << (lev - 1))
        i = int(np.nonzero(np.all(coords == centre, axis=1))[0][0])
        for j in range(m.n_indep):
            off = np.abs(coords[j] - centre)
            if off.max() > 1:
                assert A[i, j] == 0.0
                continue
            nd = int(off.sum())
            if dim == 2:
                expect = {0: 8 / 3, 1: -1 / 3, 2: -1 / 3}[nd]
            else:
                expect = {0: 8 * h / 3, 1: 0.0, 2: -h / 6, 3: -h / 12}[nd]
            assert abs(A[i, j] - expect) < 1e-14, (dim, off, A[i, j], expect)


def test_gauss_point_coefficient_hand_entry_2d():
    # one bilinear quad with h = 2 (xi = x - 1 on [0,2]) is not representable on the
    # unit domain, so use h = 1 and rescale: in 2D the stiffness is scale-free.
    m = om.uniform(2, 0)
    rp, rm = 1.0, 0.1
    alpha, beta = fem.rho_coeffs(rp, rm)
    coords = m.indep_coords().astype(float)
    phi = -0.8 + 1.2 * coords[:, 0]           # varies along x only, within [-1, 1]
    K = fem.pp_element_matrices(m, phi, rp, rm)[0]
    s = 1.0 / np.sqrt(3.0)
    xq = np.array([(1 - s) / 2, (1 + s) / 2])   # Gauss abscissae in [0,1]
    cm, cp = 1.0 / (alpha * (-0.8 + 1.2 * xq) + beta)
    # |grad N_0|^2 at (xi, eta) = ((1-eta)^2 + (1-xi)^2)/16 on [-1,1]^2; sum over eta of
    # (1-eta)^2 is 8/3; corner 0 sits at xi = -1 so xi = -s pairs with c(-s) = cm
    k00 = (cm * (8 / 3 + 2 * (1 + s) ** 2) + cp * (8 / 3 + 2 * (1 - s) ** 2)) / 16
    assert abs(K[0, 0] - k00) < 1e-15


def test_clamp_only_enters_density():
    m = om.uniform(3, 1)
    rp, rm = 1.0, 1e-3
    big = np.full(m.n_indep, 3.0)            # pulled back to +1 -> rho = 1
    A = fem.pp_matrix(m, big, rp, rm).toarray()
    A1 = fem.pp_matrix(m, np.ones(m.n_indep), rp, rm).toarray()
    # interpolating phi = 1 can round to 1 - ulp, so compare to rounding
    assert np.allclose(A, A1, rtol=0, atol=1e-15 * np.abs(A1).max())
    low = np.full(m.n_indep, -5.0)           # pulled back to -1 -> rho = beta - alpha = rm
    Al = fem.pp_matrix(m, low, rp, rm).toarray()
    alpha, beta = fem.rho_coeffs(rp, rm)
    assert abs((beta - alpha) - rm) < 1e-16
    ref = A1 * (alpha + beta) / (beta - alpha)
    assert np.allclose(Al, ref, rtol=0, atol=1e-14 * np.abs(ref).max())


def _band_mesh():
    return om.sphere_band(3, 2, 5, (0.5, 0.3, 0.5), 0.15, 0.03)


def test_invariants_adaptive_variable_coefficient():
    m = _band_mesh()
    x = m.indep_coords() / m.side
    phi = np.tanh((np.linalg.norm(x - np.array([0.5, 0.3, 0.5]), axis=1) - 0.15) / (np.sqrt(2) * 0.03))
    A = fem.pp_matrix(m, phi, 1.0, 1e-3)
    assert abs(A - A.T).max() <= 1e-15 * abs(A).max()
    assert np.abs(A @ np.ones(m.n_indep)).max() <= 1e-12 * abs(A).max()
    ev = spla.eigsh(A, k=3, which="SA", return_eigenvectors=False, tol=1e-10)
    assert ev.min() > -1e-10


def test_patch_test_across_hanging_nodes():
    m = _band_mesh()
    A = fem.pp_matrix(m, np.zeros(m.n_indep), 1.0, 1.0)
    c = m.indep_coords().astype(float) / m.side
    lin = 0.7 * c[:, 0] - 1.3 * c[:, 1] + 0.4 * c[:, 2] + 2.0
    y = A @ lin
    interior = np.all((m.indep_coords() > 0) & (m.indep_coords() < m.side), axis=1)
    assert np.abs(y[interior]).max() < 1e-13
    assert np.abs(y[~interior]).max() > 1e-3   # boundary rows carry the flux


# ------------------------------------------------------------ manufactured solution
def _mms_case(level):
    """-div(c grad p) = f with p = cos(pi x)cos(pi y)cos(pi z), c = 1/rho(phi(x))."""
    rp, rm = 1.0, 0.1
    alpha, beta = fem.rho_coeffs(rp, rm)
    ctr = np.array([0.5, 0.5, 0.5])
    r0, eps = 0.3, 0.15

    def phi(x):
        d = np.linalg.norm(x - ctr, axis=-1)
        return np.tanh((r0 - d) / eps)

    def grad_phi(x):
        d = np.linalg.norm(x - ctr, axis=-1)
        t = np.tanh((r0 - d) / eps)
        return ((1 - t ** 2) * (-1.0 / eps) / d)[..., None] * (x - ctr)

    def p_exact(x):
        return np.prod(np.cos(np.pi * x), axis=-1)

    def grad_p(x):
        cx, cy, cz = np.cos(np.pi * x[..., 0]), np.cos(np.pi * x[..., 1]), np.cos(np.pi * x[..., 2])
        sx, sy, sz = np.sin(np.pi * x[..., 0]), np.sin(np.pi * x[..., 1]), np.sin(np.pi * x[..., 2])
        return -np.pi * np.stack([sx * cy * cz, cx * sy * cz, cx * cy * sz], axis=-1)

    def f(x):
        rho = alpha * phi(x) + beta
        c = 1.0 / rho
        grad_c = (-alpha / rho ** 2)[..., None] * grad_phi(x)
        lap_p = -3 * np.pi ** 2 * p_exact(x)
        return -(c * lap_p + (grad_c * grad_p(x)).sum(-1))

    m = om.uniform(3, level)
    xn = m.indep_coords() / m.side
    A = fem.pp_matrix(m, phi(xn), rp, rm)
    # load vector with a 3-point Gauss rule per direction (independent of the
    # operator's 2-point rule)
    g, w = np.polynomial.legendre.leggauss(3)
    h = 1.0 / (1 << level)
    b = np.zeros(m.nodes.shape[0])
    err_terms = []
    anchors = m.anchor.astype(float) * h
    bits = fem.corner_bits(3)
    for i, gi in enumerate(g):
        for j, gj in enumerate(g):
            for k, gk in enumerate(g):
                xi = np.array([gi, gj, gk])
                wq = w[i] * w[j] * w[k] * (h / 2) ** 3
                xq = anchors + (xi + 1) / 2 * h
                Nq = np.prod((1 + (2 * bits - 1) * xi[None, :]) / 2, axis=1)   # (8,)
                fq = f(xq)
                np.add.at(b, m.elem_nodes, wq * fq[:, None] * Nq[None, :])
    b = m.P.T @ b
    p_h, it, hist = krylov.pcg(A, b, rtol=1e-12, M_inv_diag=1.0 / A.diagonal(), singular=True)
    # remove the discrete mean in the L2 sense and measure the L2 error with 3-pt Gauss
    M = fem.mass_matrix(m)
    one = np.ones(m.n_indep)
    p_h = p_h - (one @ (M @ p_h)) / (one @ (M @ one))
    err2 = 0.0
    pa = m.P @ p_h
    for i, gi in enumerate(g):
        for j, gj in enumerate(g):
            for k, gk in enumerate(g):
                xi = np.array([gi, gj, gk])
                wq = w[i] * w[j] * w[k] * (h / 2) ** 3
                xq = anchors + (xi + 1) / 2 * h
                Nq = np.prod((1 + (2 * bits - 1) * xi[None, :]) / 2, axis=1)
                ph_q = pa[m.elem_nodes] @ Nq
                err2 += (wq * (ph_q - p_exact(xq)) ** 2).sum()
    return np.sqrt(err2)


@pytest.mark.slow
def test_poisson_mms_second_order():
    errs = [_mms_case(l) for l in (2, 3, 4, 5)]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert rates[-1] > 1.85 and rates[-2] > 1.8, (errs, rates)
