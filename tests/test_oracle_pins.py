"""Pins of the CPU oracle against facts fixed by the paper and by mathematics
(not against itself): a textbook Householder QRCP, LAPACK's geqp3, closed
forms (Kahan, diagonal, rank-k), theorems of Secs. 4-5, invariances and
generator properties.  CPU only."""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle
import rb_inputs as ri
from householder import householder_qrcp

U = 2.0 ** -53


def _inputs():
    return {
        "gauss_24x16": ri.gaussian(11, 24, 16),
        "gauss_16x24": ri.gaussian(12, 16, 24),
        "graded_40x30": ri.graded(13, 40, 30, 0.85),
        "real_20x20": ri.gaussian(14, 20, 20, real=True),
        # unit-norm chirps tie at step 0; distinct column scales remove the tie
        "chirp_64x48": oracle.chirp(ri.chirp_params(1805, 48, 40, 60, 1, 4), 64, 20.0, 512.0)
        * np.linspace(1.0, 0.9, 48)[:, None],
    }


@pytest.mark.parametrize("name", list(_inputs().keys()))
def test_greedy_equals_householder_qrcp(name):
    """Proposition 5.3 + Corollary 5.6: greedy pivots = QRCP pivots and the
    greedy error after k vectors equals |R_kk| (both forms of the oracle)."""
    S = _inputs()[name]
    M, N = S.shape
    perm, R = householder_qrcp(S)
    kk = min(N, M)
    diag = np.abs(np.diag(R))[:kk]
    for mode in ("explicit", "pythag"):
        r = oracle.greedy(S, 0.0, kk, mode=mode)
        k = r["k"]
        # the Pythagorean form is compared while the error is well above its
        # rounding floor (Eq. (6.3) cancels)
        upto = k if mode == "explicit" else int(np.sum(diag > 1e-6 * diag[0]))
        upto = min(upto, k)
        np.testing.assert_array_equal(r["piv"][:upto], perm[:upto])
        scale = diag[0]
        if mode == "explicit":
            np.testing.assert_allclose(r["err"][:upto], diag[:upto], rtol=1e-10, atol=64 * U * scale * kk)
        else:
            # Eq. (6.3) gives err^2 to an absolute error of order k u max||s||^2
            np.testing.assert_allclose(r["err"][:upto] ** 2, diag[:upto] ** 2, rtol=1e-10,
                                       atol=64 * U * scale ** 2 * kk)
        np.testing.assert_allclose(r["rho"][:upto], diag[:upto], rtol=1e-10, atol=64 * U * scale * kk)


@pytest.mark.parametrize("name", ["gauss_24x16", "graded_40x30", "chirp_64x48"])
def test_every_column_residual_is_trailing_subcolumn(name):
    """Theorem 4.3: ||s_i - Q_k Q_k^H s_i|| = ||R[k:, pos(i)]|| for every
    column i and every k."""
    S = _inputs()[name]
    M, N = S.shape
    perm, R = householder_qrcp(S)
    r = oracle.greedy(S, 0.0, min(N, M))
    pos = np.empty(M, dtype=int)
    pos[perm] = np.arange(M)
    scale = np.abs(R[0, 0])
    for k in range(0, r["k"] + 1, max(1, r["k"] // 6)):
        res = oracle.residual_norms(r["E"][:k], S)
        trail = np.array([np.linalg.norm(R[k:, pos[i]]) for i in range(M)])
        np.testing.assert_allclose(res, trail, rtol=1e-9, atol=256 * U * scale * (k + 1))
        # greedy error = max residual (Corollary 5.6)
        assert abs(r["err"][k] - res.max()) <= 1e-9 * res.max() + 256 * U * scale * (k + 1)


def test_lapack_geqp3_crosscheck():
    """Library cross-check: LAPACK's column-pivoted QR on a well-conditioned
    input selects the same pivots with the same |R_kk|."""
    S = ri.gaussian(21, 30, 20)
    Q, R, P = scipy.linalg.qr(S.T, pivoting=True, mode="economic")
    r = oracle.greedy(S, 0.0, 20)
    np.testing.assert_array_equal(r["piv"], P[: r["k"]])
    np.testing.assert_allclose(r["rho"], np.abs(np.diag(R)), rtol=1e-11)


@pytest.mark.parametrize("theta,delta,n", [(1.2, 1e-3, 12), (0.3, 1e-2, 10), (1.45, 1e-4, 16)])
def test_kahan_closed_form(theta, delta, n):
    """Kahan's matrix (Sec. 1): every column has unit norm before scaling and
    every trailing norm after k steps is sin(theta)^k, so with the (1-delta)^j
    scaling the pivots are 0, 1, 2, ... and err_k = (sin theta (1-delta))^k."""
    S = ri.kahan(n, theta, delta)
    r = oracle.greedy(S, 0.0, n)
    np.testing.assert_array_equal(r["piv"], np.arange(n))
    want = (math.sin(theta) * (1 - delta)) ** np.arange(n)
    np.testing.assert_allclose(r["err"][:n], want, rtol=1e-12)
    np.testing.assert_allclose(r["rho"], want, rtol=1e-12)


def test_diagonal_sorted():
    """Diagonal S: the errors are |d| sorted decreasingly, pivots follow."""
    d = np.array([0.3, 2.0, -1.5, 0.7, 1e-3, 5.0, 0.02j, 1.1])
    S = ri.diagonal(d)
    r = oracle.greedy(S, 1e-12, 8)
    order = np.argsort(-np.abs(d), kind="stable")
    np.testing.assert_array_equal(r["piv"], order)
    np.testing.assert_allclose(r["err"][:8], np.abs(d)[order], rtol=1e-15)
    assert r["err"][8] == 0.0


@pytest.mark.parametrize("mode", ["explicit", "pythag"])
@pytest.mark.parametrize("rank", [1, 3, 7])
def test_rank_k_terminates_at_k(mode, rank):
    """A rank-k input (ordinary rank, Def. 2.2) stops with exactly k vectors
    at tol 1e-10 (explicit form: residual at rounding level)."""
    S = ri.low_rank(31 + rank, 40, 25, rank)
    r = oracle.greedy(S, 1e-10 * np.sqrt(oracle.sqnorms(S).max()), 25, mode=mode)
    assert r["k"] == rank
    if mode == "explicit":
        assert r["status"] == "OK"
        assert r["err"][rank] < 1e-13 * r["err"][0]


@pytest.mark.parametrize("mode", ["explicit", "pythag"])
def test_orthogonality(mode):
    """Sec. 6.1.2 (Hoffmann's bound kappa eps sqrt(k)): ||E^H E - I|| small."""
    w = ri.WORKLOADS["chirp_small_c128"]
    S = oracle.chirp(w.params(M=400), 500, w.flo, w.fhi)
    r = oracle.greedy(S, 1e-6, 200, mode=mode)
    E = r["E"]
    G = E.conj() @ E.T
    dev = np.linalg.norm(G - np.eye(r["k"]), 2)
    assert r["k"] > 10
    assert dev <= 10 * 2 * U * math.sqrt(r["k"]) * 10, dev


def test_monotone_errors_and_triangular_coefficients():
    """Proposition 5.3 (R(1,1) >= R(2,2) >= ...) and S Pi = Q R: the
    coefficients restricted to pivot columns are upper triangular with
    |R_ii| = rho_i."""
    S = ri.graded(41, 50, 40, 0.9)
    r = oracle.greedy(S, 0.0, 40, want_coeffs=True)
    k = r["k"]
    assert np.all(np.diff(r["err"][:k]) <= 1e-14 * r["err"][0])
    Cp = r["C"][:, r["piv"]]
    below = np.tril(Cp, -1)
    assert np.max(np.abs(below)) <= 1e-13 * r["err"][0]
    np.testing.assert_allclose(np.abs(np.diag(Cp)), r["rho"], rtol=1e-12)


def test_invariances():
    """Row-unitary invariance (Lemma 3.1), column phases, global scaling and
    column permutation change pivots/errors only in the predicted way."""
    S = ri.gaussian(51, 20, 15)
    base = oracle.greedy(S, 0.0, 15)
    Uq = ri.unitary(52, 20)
    S_u = (Uq @ S.T).T
    ph = np.exp(1j * np.linspace(0, 5, 15))
    perm = np.random.default_rng(53).permutation(15)
    alpha = 3.5
    ru = oracle.greedy(S_u, 0.0, 15)
    rp = oracle.greedy(S * ph[:, None], 0.0, 15)
    ra = oracle.greedy(alpha * S, 0.0, 15)
    rq = oracle.greedy(S[perm], 0.0, 15)
    for r in (ru, rp, ra):
        np.testing.assert_array_equal(r["piv"], base["piv"])
    np.testing.assert_allclose(ru["err"], base["err"], rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(rp["err"], base["err"], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(ra["err"], alpha * base["err"], rtol=1e-13, atol=1e-13)
    np.testing.assert_array_equal(perm[rq["piv"]], base["piv"])
    np.testing.assert_allclose(rq["err"], base["err"], rtol=1e-12, atol=1e-13)


def test_svd_relations():
    """Remark 4.2 / Theorem 4.1 (sigma_{k+1} <= ||R22||_2 and
    e_max <= e_2) and the product formula of Corollary 5.7 in its corrected
    form: prod_{i<=k+1} sigma_i(S_{k+1}) = prod_{i<=k+1} |R_ii|, where S_{k+1}
    holds the first k+1 pivot columns."""
    S = ri.gaussian(61, 25, 18)
    r = oracle.greedy(S, 0.0, 18)
    sig = np.linalg.svd(S.T, compute_uv=False)
    for k in range(1, 17):
        res = oracle.residual_norms(r["E"][:k], S)
        Rk = (S.T - r["E"][:k].T @ (r["E"][:k].conj() @ S.T))
        r22 = np.linalg.norm(Rk, 2)
        assert sig[k] <= r22 * (1 + 1e-12)
        assert res.max() <= r22 * (1 + 1e-12)
        Sk = S[r["piv"][: k + 1]].T
        ls = np.sum(np.log(np.linalg.svd(Sk, compute_uv=False)))
        assert abs(ls - np.sum(np.log(r["rho"][: k + 1]))) < 1e-10 * (k + 1)


def test_replay_reproduces_free_run():
    S = ri.gaussian(71, 30, 30)
    a = oracle.greedy(S, 1e-8, 30)
    b = oracle.greedy(S, 1e-8, 30, force=a["piv"])
    np.testing.assert_array_equal(a["piv"], b["piv"])
    np.testing.assert_array_equal(a["err"], b["err"])
    np.testing.assert_array_equal(b["pick"][:, 0], b["pick"][:, 1])
    # forcing a different first pivot is recorded as a loss against the max
    f = a["piv"].copy()
    f[0] = a["piv"][1]
    c = oracle.greedy(S, 1e-8, 30, force=f[:1])
    assert c["piv"][0] == f[0]
    assert c["pick"][0, 0] < c["pick"][0, 1]


def test_edge_cases():
    # max ||s|| < tol: no vector (Alg. 2 reading)
    S = 1e-12 * ri.gaussian(81, 5, 4)
    r = oracle.greedy(S, 1e-6, 4)
    assert r["k"] == 0 and r["status"] == "OK"
    # kmax clamps to min(N, M); single column; single row
    r = oracle.greedy(ri.gaussian(82, 3, 10), 0.0, 100)
    assert r["k"] == 3
    r = oracle.greedy(ri.gaussian(83, 7, 1), 0.0, 5)
    assert r["k"] == 1 and r["err"][1] == 0.0
    r = oracle.greedy(ri.gaussian(84, 1, 6), 0.0, 5)
    assert r["k"] == 1
    # zero matrix
    r = oracle.greedy(np.zeros((4, 6), dtype=np.complex128), 1e-10, 4)
    assert r["k"] == 0
    # non-finite input is rejected
    S = ri.gaussian(85, 4, 4)
    S[2, 1] = np.nan
    with pytest.raises(RuntimeError):
        oracle.greedy(S, 0.0, 4)


def test_sqnorm_exact():
    """The accumulated norm is the exact sum rounded once: compare with
    exact rational arithmetic."""
    from fractions import Fraction
    rng = np.random.default_rng(91)
    for _ in range(5):
        x = rng.standard_normal(300) * np.exp(rng.uniform(-5, 5, 300)) + 1j * rng.standard_normal(300)
        exact = sum(Fraction(float(v.real)) ** 2 + Fraction(float(v.imag)) ** 2 for v in x)
        assert oracle.sqnorm(x) == float(exact)


# --------------------------- generator pins ---------------------------

def test_splitmix64_reference_values():
    """Published SplitMix64 reference outputs for state seed 1234567."""
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    got = ri.splitmix64(1234567, np.arange(5, dtype=np.uint64))
    assert [int(v) for v in got] == want


def test_chirp_amplitude_norm_and_phase():
    """Generator: unit-L2 columns; |h(f)| proportional to f^(-7/6); the phase
    equals the chirp-mass form of the 0PN term plus the 1PN correction."""
    P = np.array([[45.0, 2.5], [20.0, 1.0], [60.0, 4.0]])
    N, flo, fhi = 257, 20.0, 512.0
    S = oracle.chirp(P, N, flo, fhi)
    f = flo + np.arange(N) * (fhi - flo) / (N - 1)
    np.testing.assert_allclose(np.linalg.norm(S, axis=1), 1.0, rtol=1e-14)
    for j in range(3):
        a = np.abs(S[j])
        np.testing.assert_allclose(a / a[0], (f / f[0]) ** (-7.0 / 6.0), rtol=1e-13)
        Mt, q = P[j]
        eta = q / (1 + q) ** 2
        Tsun = 4.925490947641267e-6
        mchirp = eta ** 0.6 * Mt * Tsun
        # 0PN: 3/128 (pi Mc f)^(-5/3); 1PN: times (3715/756 + 55 eta/9) (pi M f)^(2/3)
        x = (np.pi * Mt * Tsun * f) ** (2.0 / 3.0)
        psi = -np.pi / 4 + 3.0 / 128.0 * (np.pi * mchirp * f) ** (-5.0 / 3.0) * (1 + (3715 / 756 + 55 * eta / 9) * x)
        # compare exp(-i psi) with the normalised column's phase
        ph = S[j] / a
        np.testing.assert_allclose(ph, np.exp(-1j * psi), atol=2e-11 * np.abs(psi).max())


def test_chirp_params_ranges():
    w = ri.WORKLOADS["chirp_10k_409600_c128"]
    P = w.params(M=10000)
    assert P[:, 0].min() >= w.mlo and P[:, 0].max() < w.mhi
    assert P[:, 1].min() >= w.qlo and P[:, 1].max() < w.qhi
    # counter-based: a slice equals the corresponding rows of the whole
    np.testing.assert_array_equal(w.params(M=100, start=500), P[500:600])


def test_small_chirp_workload_reaches_tol():
    """The small chirp workload is resolved by the explicit oracle to
    tol 1e-10 well before kmax, with orthonormal basis."""
    w = ri.WORKLOADS["chirp_small_c128"]
    S = oracle.chirp(w.params(), w.N, w.flo, w.fhi)
    r = oracle.greedy(S, w.tol, w.kmax)
    assert r["status"] == "OK" and 20 < r["k"] < 100
    assert r["err"][-1] < w.tol <= r["err"][-2]
    E = r["E"]
    assert np.linalg.norm(E.conj() @ E.T - np.eye(r["k"]), 2) < 1e-13
