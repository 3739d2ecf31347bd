"""Oracle Krylov solvers in FP64: Jacobi-preconditioned CG and restarted GMRES.

TEST INFRASTRUCTURE ONLY (see oracle/mesh.py).

The paper solves every linear system with PETSc Krylov methods (appendix on
solver options: CG for the velocity update, GMRES variants for the others).
These are the textbook algorithms, written plainly; the stopping rule is the
unpreconditioned relative residual |b - A x|_2 / |b|_2 <= rtol from x0.
"""
from __future__ import annotations

import numpy as np


def pcg(A, b, rtol=1e-8, max_it=100000, M_inv_diag=None, x0=None, singular=False):
    """Preconditioned CG; returns (x, iterations, relative residual history).

    If singular is set the system is the pure-Neumann Poisson problem: b is
    projected to 1^T b = 0 and the result is shifted to 1^T x = 0.
    """
    b = np.array(b, dtype=np.float64)
    if singular:
        b = b - b.mean()
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    dinv = np.ones(n) if M_inv_diag is None else M_inv_diag
    r = b - A @ x
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, [0.0]
    hist = [np.linalg.norm(r) / bnorm]
    z = dinv * r
    p = z.copy()
    rz = r @ z
    it = 0
    while hist[-1] > rtol and it < max_it:
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
        hist.append(np.linalg.norm(r) / bnorm)
    if singular:
        x -= x.mean()
    return x, it, hist


def gmres(A, b, rtol=1e-8, restart=50, max_it=10000, x0=None, M_inv_diag=None):
    """Right-preconditioned restarted GMRES (Arnoldi with modified Gram-Schmidt,
    least-squares solve of the small Hessenberg system)."""
    b = np.array(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    dinv = np.ones(n) if M_inv_diag is None else M_inv_diag
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, [0.0]
    r = b - A @ x
    hist = [np.linalg.norm(r) / bnorm]
    it = 0
    while hist[-1] > rtol and it < max_it:
        beta = np.linalg.norm(r)
        V = np.zeros((restart + 1, n))
        H = np.zeros((restart + 1, restart))
        V[0] = r / beta
        k_done = 0
        for k in range(restart):
            w = A @ (dinv * V[k])
            for j in range(k + 1):
                H[j, k] = w @ V[j]
                w = w - H[j, k] * V[j]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] > 0:
                V[k + 1] = w / H[k + 1, k]
            k_done = k + 1
            it += 1
            e1 = np.zeros(k + 2)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(H[: k + 2, : k + 1], e1, rcond=None)
            res = np.linalg.norm(H[: k + 2, : k + 1] @ y - e1) / bnorm
            if res <= rtol or H[k + 1, k] == 0 or it >= max_it:
                break
        e1 = np.zeros(k_done + 1)
        e1[0] = beta
        y, *_ = np.linalg.lstsq(H[: k_done + 1, :k_done], e1, rcond=None)
        x = x + dinv * (V[:k_done].T @ y)
        r = b - A @ x
        hist.append(np.linalg.norm(r) / bnorm)
    return x, it, hist
