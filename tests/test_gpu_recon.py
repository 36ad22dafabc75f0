"""GPU parity of the reconstruction algorithm (Alg. 4, Theorem 5.8):
rb_reconstruct_z against the oracle (LAPACK SVD of the same coefficients)
and against closed forms.

Inputs (basis and coefficients) come from the oracle's greedy and
projection on the host and are uploaded; the oracle never sees a GPU value.

Tolerances (u = 2^-53, j basis vectors):
- singular values: |d sigma_i| <= 64 sqrt(j) u sigma_1.  This is the
  absolute accuracy of an SVD of C; the refinement step reaches it also for
  coefficient rows that are not graded.
- X_k: the projector onto span(X_k) within 64 sqrt(j) u sigma_1 / gap_k +
  1e-12 of the oracle's, with gap_k = sigma_k - sigma_{k+1};
  orthonormality within 1e-13.
"""
import numpy as np
import pytest
import torch

import oracle
import rb_inputs as ri
from oracle import reconstruct as rc

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _run(rb, E, C, tau2, want_v=False):
    """E (j, N) and C (j, M) host arrays -> GPU reconstruction."""
    return rb.reconstruct(_dev(E), _dev(C.T), tau2, want_v=want_v)


def _compare(got, ref, j):
    s1 = ref["sigma"][0]
    tol_s = 64 * np.sqrt(j) * U * s1
    assert np.all(np.abs(got["sigma"] - ref["sigma"]) <= tol_s), np.max(np.abs(got["sigma"] - ref["sigma"]))
    assert got["k"] == ref["k"]
    k = got["k"]
    if k == 0:
        return
    X = got["X"].cpu().numpy()
    assert np.linalg.norm(X.conj() @ X.T - np.eye(k), 2) <= 1e-13
    gap = ref["sigma"][k - 1] - (ref["sigma"][k] if k < j else 0.0)
    Pg = X.T @ X.conj()
    Pr = ref["X"].T @ ref["X"].conj()
    assert np.linalg.norm(Pg - Pr, 2) <= tol_s / gap + 1e-12


def test_reconstruct_chirp_parity(rb):
    """The small chirp family: greedy to 1e-10 (j = 46), tau2 = 1e-6."""
    w = ri.WORKLOADS["chirp_small_c128"]
    S = oracle.chirp(w.params(), w.N, w.flo, w.fhi)
    g = oracle.greedy(S, w.tol, w.kmax)
    C = oracle.project(g["E"], S)
    ref = rc.from_coefficients(g["E"], C, 1e-6)
    got = _run(rb, g["E"], C, 1e-6)
    _compare(got, ref, g["k"])
    # Theorem 5.8 (S is Q_j C up to the greedy residual D):
    # ||S - X_k X_k^H S||_2 <= sigma_{k+1} + ||D||_2
    X = got["X"].cpu().numpy()
    D = S.T - g["E"].T @ C
    err = np.linalg.norm(S.T - X.T @ (X.conj() @ S.T), 2)
    assert err <= ref["sigma"][got["k"]] + np.linalg.norm(D, 2) + 1e-12


def test_reconstruct_low_rank_matches_svd_of_s(rb):
    """Rank-6 S: the greedy stops at j = 6 and the singular values are those
    of S itself (LAPACK's SVD of S, a different matrix)."""
    S = ri.low_rank(80, 200, 150, 6)
    sv = np.linalg.svd(S.T, compute_uv=False)
    g = oracle.greedy(S, 1e-10 * sv[0], 150)
    assert g["k"] == 6
    C = oracle.project(g["E"], S)
    got = _run(rb, g["E"], C, 0.0)
    assert got["k"] == 6
    np.testing.assert_allclose(got["sigma"], sv[:6], rtol=0, atol=64 * np.sqrt(6) * U * sv[0])


def test_reconstruct_rows_not_graded(rb):
    """Coefficients premultiplied by a random unitary (same singular values,
    rows no longer graded): the refinement step keeps the small singular
    values to the absolute accuracy of an SVD (a Gram matrix alone loses
    them: its error is about sqrt(u) sigma_1 there)."""
    w = ri.WORKLOADS["chirp_small_c128"]
    S = oracle.chirp(w.params(), w.N, w.flo, w.fhi)
    g = oracle.greedy(S, w.tol, w.kmax)
    Q = ri.unitary(81, g["k"])
    C = Q @ oracle.project(g["E"], S)
    E = (Q.conj() @ g["E"])  # E C is unchanged: E' = Q^* E keeps E'^T C' = E^T C
    ref = rc.from_coefficients(E, C, 1e-6)
    got = _run(rb, E, C, 1e-6)
    _compare(got, ref, g["k"])


def test_reconstruct_multi_tile(rb):
    """j = 300 (ten 32-row Gram tiles, ragged last tile; larger than the LDS
    Jacobi takes, so the global-memory solve) on a graded
    Gaussian 400 x 600 input; several thresholds."""
    S = ri.graded(82, 400, 600, 0.99)
    g = oracle.greedy(S, 0.0, 300)
    C = oracle.project(g["E"], S)
    for tau2 in (0.0, 1e-2, 1.0):
        ref = rc.from_coefficients(g["E"], C, tau2)
        got = _run(rb, g["E"], C, tau2)
        _compare(got, ref, 300)


def test_reconstruct_diagonal_closed_form(rb):
    """Diagonal S: sigma = |d| sorted, X_k = the coordinate vectors of the
    k largest |d| up to phase."""
    d = np.array([0.3, 2.0, -1.5, 0.7, 1e-3, 5.0, 0.02j, 1.1])
    S = ri.diagonal(d)
    g = oracle.greedy(S, 0.0, 8)
    C = oracle.project(g["E"], S)
    got = _run(rb, g["E"], C, 0.5)
    srt = np.sort(np.abs(d))[::-1]
    np.testing.assert_allclose(got["sigma"], srt, rtol=1e-14)
    assert got["k"] == 5
    X = got["X"].cpu().numpy()
    order = np.argsort(-np.abs(d), kind="stable")
    for i in range(5):
        assert abs(abs(X[i, order[i]]) - 1.0) < 1e-14


def test_reconstruct_edges(rb):
    """j = 1; fewer columns than basis vectors; tau2 above sigma_1 (k = 0);
    the singular vectors returned with V."""
    S = ri.gaussian(83, 50, 1)
    g = oracle.greedy(S, 0.0, 1)
    C = oracle.project(g["E"], S)
    got = _run(rb, g["E"], C, 0.0, want_v=True)
    assert got["k"] == 1 and abs(got["sigma"][0] - np.linalg.norm(S)) <= 1e-13 * np.linalg.norm(S)
    S = ri.gaussian(84, 40, 30)
    g = oracle.greedy(S, 0.0, 30)
    C = oracle.project(g["E"], S)[:, :7]  # 30 x 7: rank 7
    ref = rc.from_coefficients(g["E"], C, 1e-8)
    got = _run(rb, g["E"], C, 1e-8, want_v=True)
    assert got["k"] == ref["k"] == 7
    assert np.all(got["sigma"][7:] <= 64 * np.sqrt(30) * U * ref["sigma"][0])
    V = got["V"].cpu().numpy()
    assert np.linalg.norm(V.conj().T @ V - np.eye(30), 2) <= 1e-13
    got = _run(rb, g["E"], C, 1e9)
    assert got["k"] == 0 and got["X"].shape[0] == 0


def test_reconstruct_caller_workspace(rb):
    """A caller workspace gives the same bits as the library's own, on two
    calls in a row sharing it (the second smaller); an undersized one is
    refused with RB_ENOMEM."""
    w = ri.WORKLOADS["chirp_small_c128"]
    S = oracle.chirp(w.params(), w.N, w.flo, w.fhi)
    g = oracle.greedy(S, w.tol, w.kmax)
    C = oracle.project(g["E"], S)
    E, Ct = _dev(g["E"]), _dev(C.T)
    j, M = E.shape[0], Ct.shape[0]
    ws = torch.empty(rb.reconstruct_workspace_bytes(j, M), dtype=torch.uint8, device="cuda")
    ws.fill_(0xFF)
    for jj in (j, j - 7):
        ref = rb.reconstruct(E[:jj].contiguous(), Ct[:, :jj].contiguous(), 1e-6, want_v=True)
        got = rb.reconstruct(E[:jj].contiguous(), Ct[:, :jj].contiguous(), 1e-6, want_v=True, ws=ws)
        assert got["k"] == ref["k"]
        assert np.array_equal(got["sigma"], ref["sigma"])
        assert torch.equal(got["X"], ref["X"]) and torch.equal(got["V"], ref["V"])
    small = torch.empty(rb.reconstruct_workspace_bytes(j, M) - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(rb.RBError):
        rb.reconstruct(E, Ct, 1e-6, ws=small)
    # ws == NULL: the library allocates its own, same bits
    import ctypes
    X = torch.empty((j, N := E.shape[1]), dtype=torch.complex128, device="cuda")
    sig = np.zeros(j)
    kk = ctypes.c_int64()
    rc = rb.load().rb_reconstruct_z(ctypes.c_void_p(E.data_ptr()), N, j, N, ctypes.c_void_p(Ct.data_ptr()), M, j,
                                    1e-6, ctypes.c_void_p(X.data_ptr()), N, sig.ctypes.data_as(ctypes.c_void_p),
                                    None, ctypes.byref(kk), None, 0, None)
    torch.cuda.synchronize()
    ref = rb.reconstruct(E, Ct, 1e-6)
    assert rc == 0 and kk.value == ref["k"]
    assert np.array_equal(sig, ref["sigma"]) and torch.equal(X[:kk.value], ref["X"])
