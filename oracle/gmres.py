"""Restarted GMRES (Saad and Schultz 1986) on the final system (section V eq. finalsystem).

The paper names GMRES and nothing more of its setup; the readings here: x0 = 0,
modified Gram-Schmidt Arnoldi, Givens rotations for the least-squares update, and
convergence judged on the true residual ||b - A x|| / ||b|| recomputed in FP64 at
every restart; every right-hand side is solved independently.  Unpreconditioned by
default; with `precond` (a callable applying P) it is right preconditioned (Saad,
Iterative Methods for Sparse Linear Systems, 2nd ed., sec. 9.3.2): the Krylov space
is built from v -> A P v, the iterate is updated by x += P (V y), and the residual
that stops it is still b - A x of the unpreconditioned system.
"""
from __future__ import annotations

import numpy as np


def gmres(matvec, b: np.ndarray, restart: int = 50, tol: float = 1e-6, max_iters: int = 1000,
          x0: np.ndarray | None = None, precond=None):
    """Solve A x = b for one vector.  Returns (x, info) with iters, restarts, relres, history."""
    P = (lambda v: v) if precond is None else precond
    n = b.shape[0]
    x = np.zeros(n, dtype=np.complex128) if x0 is None else x0.astype(np.complex128).copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, {"iters": 0, "restarts": 0, "relres": 0.0, "converged": True, "history": []}
    iters = 0
    restarts = 0
    history = []
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    while True:
        relres = beta / bnorm
        history.append(relres)
        if relres <= tol or iters >= max_iters:
            return x, {"iters": iters, "restarts": restarts, "relres": relres,
                       "converged": relres <= tol, "history": history}
        V = np.zeros((restart + 1, n), dtype=np.complex128)
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart, dtype=np.complex128)
        sn = np.zeros(restart, dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        j_used = 0
        for j in range(restart):
            w = matvec(P(V[j]))
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            # apply the previous rotations, then the one that zeroes H[j+1, j];
            # rotation i maps (p, q) to (conj(c) p + conj(s) q, -s p + c q)
            for i in range(j):
                p, q = H[i, j], H[i + 1, j]
                H[i, j] = np.conj(cs[i]) * p + np.conj(sn[i]) * q
                H[i + 1, j] = -sn[i] * p + cs[i] * q
            a, c = H[j, j], H[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(c) ** 2)
            cs[j] = a / den if den != 0 else 1.0
            sn[j] = c / den if den != 0 else 0.0
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = np.conj(cs[j]) * g[j]
            iters += 1
            j_used = j + 1
            if abs(g[j + 1]) / bnorm <= tol or iters >= max_iters:
                break
        y = np.linalg.solve(np.triu(H[:j_used, :j_used]), g[:j_used])
        x = x + P(V[:j_used].T @ y)
        restarts += 1
        r = b - matvec(x)
        beta = np.linalg.norm(r)
