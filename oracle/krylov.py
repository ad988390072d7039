"""Krylov solvers for the global trace system (Sec. 4.2).  Test
infrastructure (oracle).

Readings (the paper takes these from PETSc defaults and does not print them):
  * "iterative classical Gram-Schmidt" = two classical Gram-Schmidt passes;
  * outer solver: right-preconditioned FGMRES(restart) whose preconditioner
    is an inner GMRES with a fixed number of steps, zero initial guess, left
    preconditioned by the inverse of the face-block-diagonal A_uhat-uhat;
  * convergence: true residual ||b - A x||_2 <= max(rtol ||b||_2, atol).
The small Hessenberg least-squares problems are solved with numpy.linalg.lstsq
(the GPU path uses Givens rotations; both give the minimiser).
"""
import numpy as np


def _cgs2(V, w, j):
    h = V[:j + 1] @ w
    w = w - V[:j + 1].T @ h
    h2 = V[:j + 1] @ w
    w = w - V[:j + 1].T @ h2
    return h + h2, w


def gmres_left_fixed(A, Minv, v, steps):
    """`steps` Arnoldi steps of GMRES on Minv A z = Minv v from z = 0."""
    r0 = Minv(v)
    beta = np.linalg.norm(r0)
    n = v.size
    if beta == 0.0:
        return np.zeros(n)
    V = np.zeros((steps + 1, n))
    H = np.zeros((steps + 1, steps))
    V[0] = r0 / beta
    k = steps
    for j in range(steps):
        w = Minv(A(V[j]))
        h, w = _cgs2(V, w, j)
        H[:j + 1, j] = h
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] == 0.0:
            k = j + 1
            break
        V[j + 1] = w / H[j + 1, j]
    e1 = np.zeros(k + 1); e1[0] = beta
    y = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)[0]
    return V[:k].T @ y


def fgmres(A, b, x0=None, precond=None, restart=30, rtol=1e-8, atol=0.0, max_outer=200):
    """Right-preconditioned flexible GMRES with CGS2.  Returns (x, info) with
    info = dict(its, res0, res, converged)."""
    n = b.size
    x = np.zeros(n) if x0 is None else x0.copy()
    P = precond if precond is not None else (lambda v: v)
    r = b - A(x)
    res0 = np.linalg.norm(b)
    tol = max(rtol * res0, atol)
    res = np.linalg.norm(r)
    its = 0
    while res > tol and its < max_outer:
        beta = res
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        V[0] = r / beta
        k = 0
        for j in range(restart):
            Z[j] = P(V[j])
            w = A(Z[j])
            h, w = _cgs2(V, w, j)
            H[:j + 1, j] = h
            H[j + 1, j] = np.linalg.norm(w)
            its += 1
            k = j + 1
            e1 = np.zeros(k + 1); e1[0] = beta
            y = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)[0]
            est = np.linalg.norm(e1 - H[:k + 1, :k] @ y)
            if H[j + 1, j] == 0.0 or est <= tol or its >= max_outer:
                break
            V[j + 1] = w / H[j + 1, j]
        x = x + Z[:k].T @ y
        r = b - A(x)
        res = np.linalg.norm(r)
    return x, dict(its=its, res0=res0, res=res, converged=bool(res <= tol))
