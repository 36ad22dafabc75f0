"""Pins of the oracle's widening steps: greedy continuation from a given
basis (enrichment), out-of-sample validation residuals, the reconstruction
algorithm (Alg. 4) and empirical-interpolation nodes.

Each function is checked against something other than the oracle itself:
- closed forms (Kahan, diagonal and triangular-permutation inputs, unitary
  constructions);
- a textbook Householder QRCP;
- LAPACK's SVD of S (a different matrix from the one the oracle
  decomposes);
- LAPACK's LU with partial pivoting;
- the theorems of Sec. 5.

CPU only.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle
import rb_inputs as ri
from householder import householder_qrcp
from oracle import eim, reconstruct as rc

U = 2.0 ** -53


# --------------------------------------------------------------------------
# greedy continued from a given basis
# --------------------------------------------------------------------------

@pytest.mark.parametrize("k1", [1, 4, 9])
def test_resume_kahan_closed_form(k1):
    """Kahan's matrix with column scaling (1-delta)^j.  span(s_0..s_{k-1}) =
    span(coordinate vectors 0..k-1), and every trailing norm after k rows is
    sin(theta)^k.  Started from the first k1 coordinate vectors, the greedy
    continues with pivots k1, k1+1, ... and err_k = (sin theta (1-delta))^k."""
    n, theta, delta = 14, 1.2, 0.01
    S = ri.kahan(n, theta, delta)
    E0 = np.eye(n, dtype=np.complex128)[:k1]
    r = oracle.greedy(S, 0.0, n, E0=E0)
    assert r["k0"] == k1 and r["k"] == n
    np.testing.assert_array_equal(r["piv"], np.arange(k1, n))
    want = (math.sin(theta) * (1 - delta)) ** np.arange(k1, n)
    np.testing.assert_allclose(r["err"][:n - k1], want, rtol=1e-12)
    np.testing.assert_allclose(r["rho"], want, rtol=1e-12)
    np.testing.assert_array_equal(r["E"][:k1], E0)


@pytest.mark.parametrize("seed,k1", [(41, 3), (42, 8), (43, 12)])
def test_resume_continues_householder_qrcp(seed, k1):
    """Started from an orthonormal basis of the first k1 QRCP pivot columns
    (LAPACK QR of those columns), the greedy continues along the Householder
    QRCP: pivots perm[k1:], errors |R_kk| for k >= k1."""
    S = ri.gaussian(seed, 24, 20)
    perm, R = householder_qrcp(S)
    Q, _ = np.linalg.qr(S[perm[:k1]].T)
    r = oracle.greedy(S, 0.0, 20, E0=Q.T)
    kk = min(S.shape)
    np.testing.assert_array_equal(r["piv"], perm[k1:kk])
    diag = np.abs(np.diag(R))[:kk]
    np.testing.assert_allclose(r["err"][:kk - k1], diag[k1:], rtol=1e-10)
    np.testing.assert_allclose(r["rho"], diag[k1:kk], rtol=1e-10)
    Ek = r["E"]
    assert np.linalg.norm(Ek.conj() @ Ek.T - np.eye(r["k"]), 2) < 1e-13


def test_resume_stops_at_once_when_below_tol():
    """A starting basis that already approximates every column: no vector is
    added and err[k0] is the largest residual."""
    S = ri.low_rank(44, 30, 20, 4)
    Q, _ = np.linalg.qr(S.T)
    Q = Q[:, :4]
    r = oracle.greedy(S, 1e-8, 20, E0=Q.T)
    assert r["k"] == 4 and r["status"] == "OK" and r["piv"].size == 0
    assert r["err"][0] < 1e-12


# --------------------------------------------------------------------------
# out-of-sample validation residuals and enrichment
# --------------------------------------------------------------------------

def test_residual_norms_closed_form():
    """E = first k columns of a unitary U and V = U [A; B]: the residual of
    column j against span(E) is exactly ||B[:, j]||."""
    N, k, M = 30, 7, 25
    Uu = ri.unitary(45, N)
    rng = np.random.default_rng(46)
    A = rng.standard_normal((k, M)) + 1j * rng.standard_normal((k, M))
    B = (rng.standard_normal((N - k, M)) + 1j * rng.standard_normal((N - k, M))) * np.logspace(0, -9, M)
    V = (Uu @ np.vstack([A, B])).T
    got = oracle.residual_norms(Uu[:, :k].T, V)
    want = np.linalg.norm(B, axis=0)
    np.testing.assert_allclose(got, want, rtol=1e-6, atol=64 * U * np.linalg.norm(V, axis=1).max())


def test_enrich_certifies_validation_set():
    """After one enrichment every validation column's residual, computed
    here with numpy (V - (V E^H) E), is below tol.  The added pivots are
    among the columns that failed.  The basis stays orthonormal."""
    N, flo, fhi = 256, 20.0, 512.0
    P = ri.chirp_params(1805, 400, 40, 60, 1, 4)
    S = oracle.chirp(P, N, flo, fhi)
    tol = 1e-8
    g = oracle.greedy(S, tol, 200)
    V = oracle.chirp(ri.chirp_params(1806, 600, 40, 60, 1, 4), N, flo, fhi)
    e = oracle.enrich(g["E"], V, tol, 200)
    assert e["fail"].size > 0 and e["k"] > g["k"]
    assert set(e["piv"].tolist()) <= set(e["fail"].tolist())
    E = e["E"]
    R = V - (V @ E.conj().T) @ E
    assert np.linalg.norm(R, axis=1).max() < tol
    assert np.linalg.norm(E.conj() @ E.T - np.eye(e["k"]), 2) < 1e-13
    # the validation residuals against the old basis agree with numpy's
    R0 = V - (V @ g["E"].conj().T) @ g["E"]
    np.testing.assert_allclose(e["resid"], np.linalg.norm(R0, axis=1), rtol=1e-6, atol=1e-13)


# --------------------------------------------------------------------------
# reconstruction (Alg. 4)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("rank", [3, 6])
def test_reconstruct_low_rank_matches_svd_of_s(rank):
    """Theorem 5.8 (ordinary rank k): for S of rank r the greedy stops at
    j = r.  The singular values of R(1:j, :) are those of S, from LAPACK's
    SVD of S itself.  ||S - X_i X_i^H S||_2 = sigma_{i+1} for every i < r,
    and X_i spans S's leading left singular subspace."""
    S = ri.low_rank(50 + rank, 40, 30, rank)
    Ssv = np.linalg.svd(S.T, compute_uv=False)
    out = rc.reconstruct(S, 1e-10 * Ssv[0], 0.0)
    assert out["greedy"]["k"] == rank and out["k"] == rank
    np.testing.assert_allclose(out["sigma"], Ssv[:rank], rtol=1e-12)
    Us, _, _ = np.linalg.svd(S.T)
    for i in range(1, rank):
        Xi = rc.from_coefficients(out["greedy"]["E"], out["C"], out["sigma"][i - 1])["X"]
        assert Xi.shape[0] == i
        resid = S.T - Xi.T @ (Xi.conj() @ S.T)
        assert abs(np.linalg.norm(resid, 2) - Ssv[i]) <= 1e-12 * Ssv[0]
        P1 = Xi.T @ Xi.conj()
        P2 = Us[:, :i] @ Us[:, :i].conj().T
        assert np.linalg.norm(P1 - P2, 2) < 1e-10


def test_reconstruct_diagonal_closed_form():
    """Diagonal S: the singular values are |d| sorted, and X_k holds the
    coordinate vectors of the k largest |d| (up to phase)."""
    d = np.array([0.3, 2.0, -1.5, 0.7, 1e-3, 5.0, 0.02j, 1.1])
    S = ri.diagonal(d)
    out = rc.reconstruct(S, 0.0, 0.5)
    srt = np.sort(np.abs(d))[::-1]
    np.testing.assert_allclose(out["sigma"], srt, rtol=1e-15)
    assert out["k"] == int(np.count_nonzero(srt >= 0.5))
    order = np.argsort(-np.abs(d), kind="stable")
    for i in range(out["k"]):
        x = out["X"][i]
        assert abs(abs(x[order[i]]) - 1.0) < 1e-15
        assert np.linalg.norm(np.delete(x, order[i])) < 1e-15


def test_reconstruct_weyl_and_error_on_chirps():
    """General S: S = Q_j C + D with D = S - Q_j Q_j^H S, so by Weyl
    |sigma_i(C) - sigma_i(S)| <= ||D||_2.  The reconstruction error
    ||S - X_k X_k^H S||_2 is at most sigma_{k+1}(C) + ||D||_2.  Both sides
    come from LAPACK SVDs of different matrices."""
    P = ri.chirp_params(1805, 80, 40, 60, 1, 4)
    S = oracle.chirp(P, 128, 20.0, 512.0)
    out = rc.reconstruct(S, 1e-6, 1e-3)
    E, j = out["greedy"]["E"], out["greedy"]["k"]
    D = S.T - E.T @ (E.conj() @ S.T)
    dn = np.linalg.norm(D, 2)
    Ssv = np.linalg.svd(S.T, compute_uv=False)
    assert np.max(np.abs(out["sigma"] - Ssv[:j])) <= dn * (1 + 1e-9) + 1e-13
    k = out["k"]
    assert 0 < k < j
    X = out["X"]
    err = np.linalg.norm(S.T - X.T @ (X.conj() @ S.T), 2)
    assert err <= out["sigma"][k] + dn + 1e-12
    assert out["sigma"][k] < 1e-3 <= out["sigma"][k - 1]
    assert np.linalg.norm(X.conj() @ X.T - np.eye(k), 2) < 1e-13


# --------------------------------------------------------------------------
# empirical-interpolation nodes
# --------------------------------------------------------------------------

def test_eim_triangular_permutation_closed_form():
    """e_j = delta_{pi_j} + sum_{i<j} a_ji delta_{pi_i}: the interpolant
    through the earlier nodes removes the earlier terms, so r_j = delta_{pi_j}
    and the nodes are pi."""
    rng = np.random.default_rng(60)
    N, k = 50, 9
    pi = rng.permutation(N)[:k]
    E = np.zeros((k, N), dtype=np.complex128)
    for j in range(k):
        E[j, pi[j]] = 1.0
        for i in range(j):
            E[j, pi[i]] = 0.9 * (rng.standard_normal() + 1j * rng.standard_normal())
    out = eim.nodes(E)
    np.testing.assert_array_equal(out["nodes"], pi)
    for j in range(k):
        want = np.zeros(N)
        want[pi[j]] = 1.0
        np.testing.assert_allclose(np.abs(out["resid"][j]), want, atol=64 * U * k)


@pytest.mark.parametrize("seed", [61, 62, 63])
def test_eim_equals_lu_partial_pivoting(seed):
    """For a real basis the EI residual of e_j through the earlier nodes is
    column j of the Schur complement in Gaussian elimination, so the nodes
    are the pivot rows of LAPACK's LU with partial pivoting of E^T."""
    rng = np.random.default_rng(seed)
    N, k = 80, 12
    E = rng.standard_normal((k, N))
    lu, piv = scipy.linalg.lu_factor(E.T)
    perm = np.arange(N)
    for i, p in enumerate(piv):
        perm[i], perm[p] = perm[p], perm[i]
    out = eim.nodes(E.astype(np.complex128))
    np.testing.assert_array_equal(out["nodes"], perm[:k])
    # the pivots of the elimination are the residuals at the nodes
    np.testing.assert_allclose(np.abs(np.diag(lu)[:k]), out["pick"][:, 1], rtol=1e-10)


def test_eim_interpolation_property():
    """The interpolant reproduces every basis vector and anything in their
    span.  r_j vanishes at the earlier nodes.  B is the basis sampled at the
    nodes."""
    P = ri.chirp_params(1805, 60, 40, 60, 1, 4)
    S = oracle.chirp(P, 200, 20.0, 512.0)
    g = oracle.greedy(S, 1e-6, 60)
    E = g["E"]
    out = eim.nodes(E)
    p = out["nodes"]
    assert len(set(p.tolist())) == len(p)
    np.testing.assert_array_equal(out["B"], E[:, p].T)
    for j in range(1, len(p)):
        assert np.max(np.abs(out["resid"][j][p[:j]])) < 1e-12
    np.testing.assert_allclose(eim.interpolate(E, p, E), E, atol=1e-10)
    rng = np.random.default_rng(64)
    F = (rng.standard_normal((5, len(p))) + 1j * rng.standard_normal((5, len(p)))) @ E
    assert eim.interpolation_errors(E, p, F).max() < 1e-9
