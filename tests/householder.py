"""From-scratch Householder QR with column pivoting (complex), a textbook
routine used to pin the oracle on tiny inputs.

Column pivoting in the Businger-Golub form: at step k the column of largest
trailing norm ||A[k:, j]|| (recomputed from scratch each step, no downdating)
is swapped into position k, then a Householder reflector zeroes A[k+1:, k].
S Pi = Q R with |R_kk| non-increasing; by Corollary 5.6 and Theorem 4.3 of
the paper, the greedy error after k vectors is |R_kk| and each column's
residual is the norm of its trailing subcolumn of R.

Pure numpy, small inputs only.
"""
from __future__ import annotations

import numpy as np


def householder_qrcp(S_rows: np.ndarray):
    """S_rows: (M, N) array whose row j is column s_j.
    Returns (perm, R) with S[:, perm] = Q R, R of shape (N, M) upper
    trapezoidal (trailing rows below min(N, M) are zero)."""
    A = np.array(S_rows, dtype=np.complex128).T.copy()  # N x M
    N, M = A.shape
    perm = np.arange(M)
    for k in range(min(N, M)):
        norms = np.array([np.sqrt(np.sum(np.abs(A[k:, j]) ** 2)) for j in range(k, M)])
        p = k + int(np.argmax(norms))
        if p != k:
            A[:, [k, p]] = A[:, [p, k]]
            perm[[k, p]] = perm[[p, k]]
        x = A[k:, k].copy()
        xn = np.sqrt(np.sum(np.abs(x) ** 2))
        if xn == 0.0:
            continue
        phase = x[0] / abs(x[0]) if x[0] != 0 else 1.0
        alpha = -phase * xn
        v = x.copy()
        v[0] -= alpha
        vn = np.sqrt(np.sum(np.abs(v) ** 2))
        if vn == 0.0:
            continue
        v /= vn
        # H = I - 2 v v^H applied to the trailing block
        A[k:, k:] -= 2.0 * np.outer(v, v.conj() @ A[k:, k:])
        A[k + 1:, k] = 0.0
    return perm, np.triu(A)
