"""Oracle Q1 finite elements: element matrices and assembled sparse operators.

TEST INFRASTRUCTURE ONLY (see oracle/mesh.py).

Discretisation (paper Sec. 3.1, remark on element order: r = 1, i.e.
bilinear quads / trilinear hexes):
* reference element [-1,1]^d, corner a with coordinate bits b_d in {0,1}
  (bit d of a), reference coordinate xi_{a,d} = 2 b_d - 1;
* N_a(xi) = prod_d (1 + xi_{a,d} xi_d) / 2;
* leaves are axis-aligned cubes of side h = 2^-level, so grad_x = (2/h) grad_xi
  and det J = (h/2)^d;
* quadrature: 2-point Gauss per direction (xi_q in {-1/sqrt3, +1/sqrt3}^d,
  unit weights); the paper does not state the rule.

Operators assembled here, each as y = P^T (sum_e S_e^T K_e S_e) P x with P the
hanging-node interpolation of oracle/mesh.py:
* pressure Poisson (Sec. 3, Def. 2 and the VMS pressure Poisson definition):
  a(q, p) = sum_q w detJ c_q grad N . grad N with c_q = 1/rho(phi*_q), where
  phi_q is the interpolated phase field at the Gauss point, phi* its clamp to
  [-1, 1] (remark on the pull back) and rho(phi) = alpha phi + beta (Sec. 2).
* mass and rho-weighted mass (velocity update, Def. 2 / VMS velocity update).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mesh import OracleMesh

GAUSS = 1.0 / np.sqrt(3.0)


def corner_bits(dim: int) -> np.ndarray:
    return np.array([[(a >> d) & 1 for d in range(dim)] for a in range(1 << dim)], dtype=np.int64)


def tabulate(dim: int):
    """N[q, a] and dN[q, a, d] (reference gradient) at the 2^d Gauss points."""
    bits = corner_bits(dim)
    xi_a = 2.0 * bits - 1.0                      # (2^d, d)
    xi_q = (2.0 * bits - 1.0) * GAUSS            # (2^d, d) Gauss points, same ordering
    nq = 1 << dim
    N = np.ones((nq, nq))
    dN = np.ones((nq, nq, dim))
    for q in range(nq):
        for a in range(nq):
            f = (1.0 + xi_a[a] * xi_q[q]) / 2.0   # per-direction factors
            N[q, a] = np.prod(f)
            for d in range(dim):
                g = f.copy()
                g[d] = xi_a[a, d] / 2.0
                dN[q, a, d] = np.prod(g)
    return N, dN


def rho_coeffs(rho_plus: float, rho_minus: float):
    """alpha, beta of rho(phi) = alpha phi + beta (Sec. 2, normalised by rho_plus)."""
    alpha = (rho_plus - rho_minus) / (2.0 * rho_plus)
    beta = (rho_plus + rho_minus) / (2.0 * rho_plus)
    return alpha, beta


def pull_back(phi: np.ndarray) -> np.ndarray:
    """phi* of the pull-back remark: phi if |phi| <= 1 else sign(phi)."""
    return np.where(np.abs(phi) <= 1.0, phi, np.sign(phi))


def elem_h(mesh: OracleMesh) -> np.ndarray:
    return 1.0 / (2.0 ** mesh.level.astype(np.float64))


def all_node_values(mesh: OracleMesh, v_indep: np.ndarray) -> np.ndarray:
    """Values at every leaf corner, hanging ones interpolated (P v)."""
    return mesh.P @ v_indep


def qp_values(mesh: OracleMesh, v_indep: np.ndarray, elems=None) -> np.ndarray:
    """Interpolated field at the Gauss points of each element: (E, 2^d)."""
    N, _ = tabulate(mesh.dim)
    va = all_node_values(mesh, v_indep)
    en = mesh.elem_nodes if elems is None else mesh.elem_nodes[elems]
    return va[en] @ N.T


def assemble(mesh: OracleMesh, Ke: np.ndarray, elems=None) -> sp.csr_matrix:
    """P^T (sum_e S_e^T K_e S_e) P from element matrices Ke (E, 2^d, 2^d)."""
    en = mesh.elem_nodes if elems is None else mesh.elem_nodes[elems]
    nloc = en.shape[1]
    rows = np.repeat(en, nloc, axis=1).ravel()
    cols = np.tile(en, (1, nloc)).ravel()
    n_all = mesh.nodes.shape[0]
    K = sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(n_all, n_all)).tocsr()
    P = mesh.P
    return (P.T @ K @ P).tocsr()


def pp_element_matrices(mesh: OracleMesh, phi_indep: np.ndarray, rho_plus: float, rho_minus: float,
                        elems=None) -> np.ndarray:
    """Variable-coefficient stiffness K_e[a,b] = sum_q detJ c_q grad N_a . grad N_b."""
    dim = mesh.dim
    _, dN = tabulate(dim)
    alpha, beta = rho_coeffs(rho_plus, rho_minus)
    phiq = qp_values(mesh, phi_indep, elems)
    c = 1.0 / (alpha * pull_back(phiq) + beta)              # (E, nq)
    h = elem_h(mesh) if elems is None else elem_h(mesh)[elems]
    scale = (h / 2.0) ** dim * (2.0 / h) ** 2               # detJ * (2/h)^2
    S = np.einsum("qad,qbd->qab", dN, dN)                    # (nq, nloc, nloc)
    return np.einsum("e,eq,qab->eab", scale, c, S)


def pp_matrix(mesh: OracleMesh, phi_indep: np.ndarray, rho_plus: float, rho_minus: float) -> sp.csr_matrix:
    return assemble(mesh, pp_element_matrices(mesh, phi_indep, rho_plus, rho_minus))


def stiffness_matrix(mesh: OracleMesh, coef_q: np.ndarray = None) -> sp.csr_matrix:
    """sum_e sum_q detJ k_q grad N . grad N with k_q given per element and Gauss point (default 1)."""
    dim = mesh.dim
    _, dN = tabulate(dim)
    h = elem_h(mesh)
    scale = (h / 2.0) ** dim * (2.0 / h) ** 2
    if coef_q is None:
        coef_q = np.ones((mesh.n_elems, 1 << dim))
    S = np.einsum("qad,qbd->qab", dN, dN)
    return assemble(mesh, np.einsum("e,eq,qab->eab", scale, coef_q, S))


def mass_matrix(mesh: OracleMesh, coef_q: np.ndarray = None) -> sp.csr_matrix:
    """sum_e sum_q detJ k_q N_a N_b (k = 1 by default)."""
    dim = mesh.dim
    N, _ = tabulate(dim)
    h = elem_h(mesh)
    detj = (h / 2.0) ** dim
    if coef_q is None:
        coef_q = np.ones((mesh.n_elems, 1 << dim))
    S = np.einsum("qa,qb->qab", N, N)
    return assemble(mesh, np.einsum("e,eq,qab->eab", detj, coef_q, S))


def rho_mass_matrix(mesh: OracleMesh, phi_indep: np.ndarray, rho_plus: float, rho_minus: float) -> sp.csr_matrix:
    """Mass matrix weighted by rho(phi*) at the Gauss points (velocity update)."""
    alpha, beta = rho_coeffs(rho_plus, rho_minus)
    rq = alpha * pull_back(qp_values(mesh, phi_indep)) + beta
    return mass_matrix(mesh, rq)
