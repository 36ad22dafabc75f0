"""Oracle for the reconstruction algorithm (Alg. 4, Sec. 5.2.2; Theorem 5.8).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.

Alg. 4 runs the greedy (MGS with column pivoting) until |R(j,j)| < tau1,
giving S ~ Q_j R(1:j, :).  Then it takes the SVD R(1:j, :) = V Sigma W^H,
picks k from the singular values against tau2, and returns X_k = Q_j V(:, 1:k).
In complex arithmetic, ^T becomes ^H.

The rows of R(1:j, :) are R(i, l) = q_i^H s_{pi(l)}.  Since q_i is orthogonal
to q_1..q_{i-1}, the projection of the residual equals the projection of the
snapshot itself, so R(1:j, :) = Q_j^H S Pi.  Its singular values and left
singular vectors are therefore those of C = Q_j^H S, with columns in S's own
order.  The oracle uses C.

Readings (the algorithm's own statement is loose):
- Dimensions: X_k = Q_j V(:, 1:k) is N x k.  The printed form multiplies Q_k
  by the k x k block V(1:k, 1:k), which does not match Theorem 5.8.
- Selecting k: sigma_{k+1} < tau2 < sigma_k is read as k = #{i : sigma_i >= tau2}.
  Then ||S - X_k X_k^H S||_2 = sigma_{k+1} < tau2 whenever k < j, the same
  strict test the greedy's stopping rule makes.

The SVD is the library's (numpy / LAPACK), used as one step.
"""
from __future__ import annotations

import numpy as np

from . import greedy, project


def from_coefficients(E, C, tau2: float) -> dict:
    """Steps 5-7 of Alg. 4 given the basis E (j, N) and C = E^H S (j, M).

    Returns dict with:
    - X: (k, N), row i = x_{i+1};
    - sigma: (j,), non-increasing;
    - V: (j, j), the left singular vectors as columns;
    - k.
    """
    E = np.asarray(E, dtype=np.complex128)
    C = np.asarray(C, dtype=np.complex128)
    j = E.shape[0]
    if j == 0:
        return dict(X=np.zeros((0, E.shape[1]), dtype=np.complex128), sigma=np.zeros(0), V=np.zeros((0, 0)), k=0)
    V, sigma, _ = np.linalg.svd(C, full_matrices=False)
    k = int(np.count_nonzero(sigma >= tau2))
    X = V[:, :k].T @ E  # X_k = Q_j V(:, 1:k), stored as rows
    return dict(X=X, sigma=sigma, V=V, k=k)


def reconstruct(S, tau1: float, tau2: float, kmax: int | None = None) -> dict:
    """The whole of Alg. 4 on the snapshot matrix S (M, N): greedy to tau1,
    C = E^H S, then from_coefficients.  Also returns the greedy's record."""
    S = np.asarray(S, dtype=np.complex128)
    M, N = S.shape
    g = greedy(S, tau1, min(N, M) if kmax is None else kmax)
    C = project(g["E"], S)
    out = from_coefficients(g["E"], C, tau2)
    out["greedy"] = g
    out["C"] = C
    return out
