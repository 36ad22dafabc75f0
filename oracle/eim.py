"""Oracle for empirical-interpolation (EI) nodes of a reduced basis (Sec. 6.1).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.

The paper selects EI nodes with the fast algorithm of Antil, Field, Nochetto
and Tiglio (2013), which is not reproduced in the paper.  This file follows
the standard definition of the empirical interpolation method on a discrete
basis (Maday, Nguyen, Patera & Pau 2009; the discrete form of Chaturantabut
& Sorensen 2010), which that algorithm computes.

For the basis e_1..e_k (rows of E), the interpolant of f at nodes p_1..p_m
is I_m[f] = sum_l c_l e_l.  The coefficients solve B_m c = f(p), where
B_m[l, i] = e_i(p_l).

- Node 1 is the argmax over n of |e_1(n)|.
- Node j is the argmax over n of |e_j(n) - I_{j-1}[e_j](n)|, the point where
  the interpolant of the next basis vector through the earlier nodes is worst.

Ties go to the lowest index.  |.| is the complex modulus, in FP64.  The
solve is the library's (numpy / LAPACK), used as one step.
"""
from __future__ import annotations

import numpy as np


def nodes(E, force=None) -> dict:
    """EI nodes of the basis E (k, N).

    force: optional node sequence to replay.  At step j the node is force[j]
    instead of the argmax; both are recorded.

    Returns dict with:
    - nodes: (k,) int64;
    - B: (k, k), B[l, i] = e_i(p_l);
    - pick: (k, 2), |r_j| at the node taken and max_n |r_j(n)|;
    - resid: (k, N), the residuals r_j = e_j - I_{j-1}[e_j].
    """
    E = np.asarray(E, dtype=np.complex128)
    k, N = E.shape
    p = np.zeros(k, dtype=np.int64)
    pick = np.zeros((k, 2))
    resid = np.zeros((k, N), dtype=np.complex128)
    for j in range(k):
        if j == 0:
            r = E[0].copy()
        else:
            Bj = E[:j, p[:j]].T
            c = np.linalg.solve(Bj, E[j, p[:j]])
            r = E[j] - c @ E[:j]
        a = np.abs(r)
        best = int(np.argmax(a))  # first index of the maximum
        pj = best if force is None else int(force[j])
        p[j] = pj
        pick[j] = (a[pj], a[best])
        resid[j] = r
    return dict(nodes=p, B=E[:, p].T.copy(), pick=pick, resid=resid)


def interpolate(E, p, F) -> np.ndarray:
    """Empirical interpolant of each row of F (M, N) on basis E through nodes p:
    I[f] = E^T (B^{-1} f(p)), returned as (M, N)."""
    E = np.asarray(E, dtype=np.complex128)
    F = np.asarray(F, dtype=np.complex128)
    B = E[:, p].T
    coef = np.linalg.solve(B, F[:, p].T)  # (k, M)
    return coef.T @ E


def interpolation_errors(E, p, F) -> np.ndarray:
    """||f - I[f]||_2 for each row of F (out-of-sample validation of the
    empirical interpolant)."""
    F = np.asarray(F, dtype=np.complex128)
    return np.linalg.norm(F - interpolate(E, p, F), axis=1)
