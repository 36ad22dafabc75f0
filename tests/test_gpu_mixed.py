"""Mixed precision (complex64 storage, FP32 sweep, FP64 confirmation and
basis) against the FP64 oracle on the same seeded chirp inputs.

What is compared (the FP64 method and the mixed method pick pivots from
different rounding of the same columns, so their pivot sequences are not
expected to coincide; every unit-norm column ties at step 0):
  - the mixed sweep's c_j / est_j / top-8 against the oracle's definitions
    evaluated on the same complex64 values (FP32 products: |dc| <=
    8 u32 sqrt(N) ||e|| ||s||);
  - the oracle replayed along the mixed pivots: every reported error and
    pivot residual is the oracle's explicit residual of that pivot
    (|d| <= 1e-10 rel + generator rounding 1e-11); each pivot's residual is
    at least 0.9 of the oracle's maximum (a weak-greedy step at worst);
  - the final basis: the oracle's explicit max residual over all FP64
    columns is < tol (equal error), ||E^H E - I|| <= 2e-13, and the basis
    size is within 2 of the FP64 oracle's.
"""
import numpy as np
import pytest
import torch

import oracle
import rb_inputs as ri

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _small(M=None, N=None):
    w = ri.WORKLOADS["chirp_small_c128"]
    M = M or w.M
    N = N or w.N
    P = w.params(M=M)
    S64 = oracle.chirp(P, N, w.flo, w.fhi)
    return w, P, S64


@pytest.mark.parametrize("N,M", [(1000, 2000), (777, 1234), (1, 9), (513, 1)])
def test_sweep_c_matches_oracle(rb, N, M):
    S = ri.gaussian(100 + N, N, M).astype(np.complex64)
    e = ri.gaussian(101, N, 1)[0]
    e = (e / np.linalg.norm(e)).astype(np.complex64)
    S64 = S.astype(np.complex128)
    e64 = e.astype(np.complex128)
    rng = np.random.default_rng(102)
    acc0 = rng.uniform(0, 0.5, M)
    mask = (rng.uniform(size=M) < 0.2).astype(np.uint8)
    nrm = oracle.sqnorms(S64)
    c_ref = oracle.project(e64[None, :], S64)[0]
    acc_ref = acc0 + np.abs(c_ref) ** 2
    est_ref = np.where(mask == 0, nrm - acc_ref, -np.inf)
    acc = _dev(acc0)
    c = torch.zeros(M, dtype=torch.complex128, device="cuda")
    est, J = rb.sweep_c(_dev(S), _dev(e), _dev(nrm), acc, _dev(mask), c)
    scale = np.sqrt(nrm)
    dc = np.abs(c.cpu().numpy() - c_ref)
    assert np.all(dc <= 8 * U32 * np.sqrt(N) * scale + 1e-30)
    bound = 2 * 8 * U32 * np.sqrt(N) * scale * (np.abs(c_ref) + scale)
    assert np.all(np.abs(acc.cpu().numpy() - acc_ref) <= bound + 1e-14)
    order = np.lexsort((np.arange(M), -est_ref))
    nvalid = int(np.sum(mask == 0))
    want = order[: min(8, nvalid)]
    got = J[J >= 0]
    assert len(got) == len(want)
    # the 8 nominated are the oracle's 8 up to near-ties within the FP32 bound
    thr = est_ref[want[-1]] - 2 * bound.max()
    assert np.all(est_ref[got] >= thr)
    assert np.all(np.diff(est[: len(got)]) <= 0)
    np.testing.assert_allclose(est[: len(got)], est_ref[got], atol=2 * bound.max() + 1e-14)


def _mixed_vs_oracle(rb, w, P, S64, tol, **opts):
    S32 = S64.astype(np.complex64)
    g = rb.greedy_c(_dev(S32), tol, w.kmax, _dev(P), w.flo, w.fhi, **opts)
    k = g["k"]
    E = g["E"].cpu().numpy()
    # replay the FP64 oracle along the mixed pivots
    ref = oracle.greedy(S64, 0.0, k, force=g["piv"])
    assert ref["k"] == k
    np.testing.assert_array_equal(ref["piv"], g["piv"])
    res_ref = np.sqrt(np.maximum(ref["pick"][:, 0], 0))
    mx_ref = np.sqrt(np.maximum(ref["pick"][:, 1], 0))
    assert np.all(np.abs(g["rho"] - res_ref) <= 1e-10 * res_ref + 1e-11)
    assert np.all(res_ref >= 0.9 * mx_ref - 1e-11), np.min(res_ref / np.maximum(mx_ref, 1e-300))
    np.testing.assert_allclose(g["err"][:k], g["rho"], rtol=0, atol=0)
    # equal error: the basis approximates every FP64 column to tol
    res_all = oracle.residual_norms(E, S64)
    mask = np.ones(S64.shape[0], bool)
    mask[g["piv"]] = False
    if g["status"] == "OK":
        assert res_all[mask].max() < tol * (1 + 1e-6) + 1e-12, res_all[mask].max()
    assert np.linalg.norm(E.conj() @ E.T - np.eye(k), 2) <= 2e-13
    return g, ref


@pytest.mark.parametrize("tol", [1e-10, 1e-5])
def test_greedy_c_small_chirp(rb, tol):
    w, P, S64 = _small()
    g, _ = _mixed_vs_oracle(rb, w, P, S64, tol)
    free = oracle.greedy(S64, tol, w.kmax)
    assert g["status"] == "OK"
    assert abs(g["k"] - free["k"]) <= 2, (g["k"], free["k"])


@pytest.mark.parametrize("opts", [dict(certify=0), dict(certify=1), dict(anchor_max=4), dict(theta32=1e-2), dict(regen_chunk=77)])
def test_greedy_c_options(rb, opts):
    w, P, S64 = _small(M=900, N=700)
    g, _ = _mixed_vs_oracle(rb, w, P, S64, 1e-10, **opts)
    assert g["stats"]["anchors"] >= 1


def test_greedy_c_inplace_and_W(rb):
    w, P, S64 = _small(M=600, N=500)
    S32 = _dev(S64.astype(np.complex64))
    a = rb.greedy_c(S32.clone(), 1e-10, 200, _dev(P), w.flo, w.fhi)
    b = rb.greedy_c(S32, 1e-10, 200, _dev(P), w.flo, w.fhi, W=torch.empty_like(S32))
    X = S32.clone()
    c = rb.greedy_c(X, 1e-10, 200, _dev(P), w.flo, w.fhi, W=X)
    for r in (b, c):
        np.testing.assert_array_equal(r["piv"], a["piv"])
        np.testing.assert_array_equal(r["err"], a["err"])


def test_greedy_c_edge_cases(rb):
    w, P, S64 = _small(M=50, N=40)
    S32 = _dev(S64.astype(np.complex64))
    g = rb.greedy_c(S32, 2.0, 10, _dev(P), w.flo, w.fhi)   # max ||s|| = 1 < tol
    assert g["k"] == 0 and g["status"] == "OK"
    g = rb.greedy_c(S32, 0.0, 100, _dev(P), w.flo, w.fhi)  # kmax clamps to N
    assert g["k"] <= 40
    with pytest.raises(rb.RBError):
        rb.greedy_c(S32, 1e-10, 10, _dev(P), w.flo, w.fhi, theta32=2.0)
