"""Krylov iterations preconditioned by the RS-S factorization (test
infrastructure).

Sec. 5 uses the factorization as a preconditioner: conjugate gradients for the
first-kind Laplace system (real symmetric positive definite) and GMRES for the
complex symmetric, indefinite Lippmann-Schwinger system, counting iterations
n_it until the relative residual ||A x - b|| / ||b|| reaches 1e-12
(Tab. t:notations).  Both are the textbook methods (Saad, Iterative Methods
for Sparse Linear Systems, Alg. 9.1 preconditioned CG and Alg. 9.5 right
preconditioned GMRES) for one right-hand side; the products with A come from
a callable (here the exact FFT product), the preconditioner M^{-1} is the
factorization's solve (Sec. 2.6).
"""
from __future__ import annotations

import numpy as np


def pcg(matvec, precond, b, tol: float = 1e-12, maxit: int = 200):
    """Preconditioned CG.  Returns (x, iterations, history of relres)."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b)
    r = b.copy()
    z = precond(r)
    p = z.copy()
    rz = np.vdot(r, z)
    nb = np.linalg.norm(b)
    hist = [1.0]
    it = 0
    while it < maxit:
        Ap = matvec(p)
        alpha = rz / np.vdot(p, Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        it += 1
        rel = np.linalg.norm(r) / nb
        hist.append(rel)
        if rel <= tol:
            break
        z = precond(r)
        rz_new = np.vdot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, hist


def _gmres_cycle(matvec, precond, r0, nb, tol, m):
    """One GMRES cycle of at most m steps from the residual r0: returns the
    correction M^{-1} u, the steps taken and the estimated relres after each."""
    beta = np.linalg.norm(r0)
    V = [r0 / beta]
    H = np.zeros((m + 1, m), dtype=np.complex128)
    cs = np.zeros(m, dtype=np.complex128)
    sn = np.zeros(m, dtype=np.complex128)
    g = np.zeros(m + 1, dtype=np.complex128)
    g[0] = beta
    hist = []
    k = 0
    for k in range(m):
        w = matvec(precond(V[k]))
        for i in range(k + 1):
            H[i, k] = np.vdot(V[i], w)
            w = w - H[i, k] * V[i]
        H[k + 1, k] = np.linalg.norm(w)
        V.append(w / H[k + 1, k] if H[k + 1, k] != 0 else w)
        # rotations G_i = [[conj(c_i), conj(s_i)], [-s_i, c_i]] (unitary)
        for i in range(k):
            t = np.conj(cs[i]) * H[i, k] + np.conj(sn[i]) * H[i + 1, k]
            H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
            H[i, k] = t
        a, c = H[k, k], H[k + 1, k]
        den = np.sqrt(abs(a) ** 2 + abs(c) ** 2)
        cs[k] = a / den if den else 1.0
        sn[k] = c / den if den else 0.0
        H[k, k] = den
        H[k + 1, k] = 0.0
        g[k + 1] = -sn[k] * g[k]
        g[k] = np.conj(cs[k]) * g[k]
        hist.append(abs(g[k + 1]) / nb)
        if hist[-1] <= tol:
            break
    steps = k + 1
    y = np.linalg.solve(np.triu(H[:steps, :steps]), g[:steps])
    u = sum(y[i] * V[i] for i in range(steps))
    return precond(u), steps, hist


def gmres(matvec, precond, b, tol: float = 1e-12, maxit: int = 200, restart: int = 0):
    """Right-preconditioned GMRES: A M^{-1} u = b, x = M^{-1} u, Arnoldi by
    modified Gram-Schmidt, the least-squares problem by Givens rotations.
    restart m > 0: GMRES(m) (Saad Alg. 6.11), each cycle of at most m steps
    restarting from the true residual b - A x (Tab. t:h2 counts GMRES(20)
    iterations without a preconditioner); 0: no restart.  maxit bounds the
    total steps.  Returns (x, iterations, history of relres)."""
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    r = b.copy()
    hist = [1.0]
    it = 0
    while it < maxit:
        m = min(restart if restart > 0 else maxit, maxit - it)
        dx, steps, h = _gmres_cycle(matvec, precond, r, nb, tol, m)
        x = x + dx
        it += steps
        hist.extend(h)
        r = b - matvec(x)
        if np.linalg.norm(r) <= tol * nb:
            break
    return x, it, hist
