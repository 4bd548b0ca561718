"""Oracle: solvers for Z I = V and its preconditioned form, eq. (4) and eq. (precon). Test infrastructure only.

* ``lu_solve``: the exact solution Z^{-1} b by dense LU (numpy/LAPACK).
* ``fgmres``: right-preconditioned flexible GMRES(m) in complex FP64 (Saad's FGMRES):
  Arnoldi with modified Gram-Schmidt on w = Z (P v_j), Givens rotations on the
  Hessenberg matrix, x += [P v_1 ... P v_j] y after each cycle, and a true residual
  ||b - Z x|| / ||b|| checked before stopping.  x0 = 0.  Right preconditioning makes
  the stopping test the unpreconditioned residual chi_sol.  The paper's solver is
  TFQMR with left preconditioning; GMRES replaces it here (reading).
"""
from __future__ import annotations

import numpy as np


def lu_solve(Z: np.ndarray, b: np.ndarray) -> np.ndarray:
    return np.linalg.solve(Z, b)


def fgmres(A, b: np.ndarray, M=None, tol: float = 1e-6, restart: int = 20, max_iter: int = 3000):
    """Solve A x = b for one column b; A and M map (N,) -> (N,).

    Returns (x, iterations, converged, history) where history holds the estimated
    relative residual after every Arnoldi step.
    """
    b = np.asarray(b, dtype=np.complex128)
    n = b.shape[0]
    M = M if M is not None else (lambda v: v)
    bnorm = np.linalg.norm(b)
    x = np.zeros(n, dtype=np.complex128)
    if bnorm == 0.0:
        return x, 0, True, []
    r = b.copy()
    beta = bnorm
    it = 0
    hist = []
    converged = False
    while it < max_iter:
        m = restart
        V = np.zeros((m + 1, n), dtype=np.complex128)
        Zs = np.zeros((m, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        j_end = 0
        for j in range(m):
            Zs[j] = M(V[j])
            w = A(Zs[j])
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):  # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + np.conj(cs[i]) * H[i + 1, j]
                H[i, j] = t
            a, c = H[j, j], H[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(c) ** 2)
            if den == 0:
                cs[j], sn[j] = 1.0, 0.0
            else:
                cs[j] = a / den
                sn[j] = c / den
            # rotation [c s; -conj(s) conj(c)] applied to (a, c) gives (den, 0)
            cs[j], sn[j] = np.conj(cs[j]), np.conj(sn[j])
            H[j, j] = cs[j] * a + sn[j] * c
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_end = j + 1
            est = abs(g[j + 1]) / bnorm
            hist.append(est)
            if est <= tol or it >= max_iter:
                break
        y = np.linalg.solve(np.triu(H[:j_end, :j_end]), g[:j_end])
        x = x + Zs[:j_end].T @ y
        r = b - A(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol:
            converged = True
            break
    return x, it, converged, hist
