"""Oracle Krylov solver in FP64: Jacobi-preconditioned CG.

TEST INFRASTRUCTURE ONLY (see oracle/mesh.py).

The paper solves every linear system with PETSc Krylov methods (appendix on
solver options: CG for the velocity update, GMRES variants for the others).
This is the textbook algorithm, written plainly; the stopping rule is the
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
