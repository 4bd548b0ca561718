"""Oracle: interpolative decomposition, eq. (ID) of Section III-A. Test infrastructure only.

M (m x n) ~ M(:, J) V with |J| = r skeleton columns and V (r x n) the interpolation
matrix, truncated so that ||M - M(:, J) V||_F <= chi ||M||_F (the paper asks for
O(chi) in the Frobenius norm).

Steps: column-pivoted QR, M P = Q R (LAPACK geqp3 through scipy, a library
primitive).  Keeping the first r pivots leaves the residual
M(:, P[r:]) - M(:, P[:r]) R11^{-1} R12 = Q(:, r:) R22, whose Frobenius norm is
||R22||_F; r is the smallest rank with ||R22||_F <= chi ||M||_F.  Then
V(:, P[:r]) = I and V(:, P[r:]) = R11^{-1} R12.  An all-zero M gives r = 0.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def interp_decomp(M: np.ndarray, chi: float):
    """Return (J, V): skeleton column indices (r,) and interpolation matrix (r, n)."""
    M = np.asarray(M, dtype=np.complex128)
    m, n = M.shape
    total = np.linalg.norm(M)
    if n == 0 or m == 0 or total == 0.0:
        return np.zeros(0, dtype=np.int64), np.zeros((0, n), dtype=np.complex128)
    R, P = sla.qr(M, mode="r", pivoting=True)
    k = min(m, n)
    R = R[:k]
    # tail[r] = ||R[r:, r:]||_F.  R is upper trapezoidal, so row i >= r of R[r:, r:]
    # is R[i, i:], and the squared norms accumulate row by row from the bottom.
    tail = np.zeros(k + 1)
    for r in range(k - 1, -1, -1):
        tail[r] = np.sqrt(tail[r + 1] ** 2 + np.sum(np.abs(R[r, r:]) ** 2))
    r = next(rr for rr in range(k + 1) if tail[rr] <= chi * total)
    J = P[:r].astype(np.int64)
    V = np.zeros((r, n), dtype=np.complex128)
    if r > 0:
        V[:, P[:r]] = np.eye(r)
        if r < n:
            V[:, P[r:]] = sla.solve_triangular(R[:r, :r], R[:r, r:])
    return J, V
