"""The greedy's C-ABI contract on the GPU: a caller workspace, the
breakdown and non-finite statuses, and the per-step timing record.

- With ws (rb_greedy_z_workspace / rb_greedy_c_workspace bytes) the greedy
  runs the same kernels in the same order as with its own allocation, so
  every output is bit-identical.
- Hoffmann's criterion (Sec. 6.1.2): a pass that shrinks ||v|| by kappa or
  more asks for another one.  On Kahan's matrix (column norms 1, pivot k's
  residual s^k (1 - delta)^k with s = sin theta, Sec. 1) the first pass at
  step k shrinks the stored column by exactly s^k, so with nu_max = 1 the
  first step with s^k <= 1/2 must stop with RB_EBREAKDOWN, the steps before
  it being the closed-form ones.
- Non-finite values: S with an Inf (found by the exact initial norms) and a
  regenerator whose parameters are NaN (found at the first confirmation)
  both give RB_ENONFINITE.
"""
import numpy as np
import pytest
import torch

import oracle
import rb_inputs as ri

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _same(g1, g2):
    assert g1["k"] == g2["k"] and g1["status"] == g2["status"]
    for key in ("piv", "err", "rho", "nu"):
        np.testing.assert_array_equal(g1[key], g2[key])
    assert torch.equal(g1["E"], g2["E"])


@pytest.mark.parametrize("anchor_max", [128, 8])
def test_fp64_workspace_matches_own_allocation(rb, anchor_max):
    w = ri.WORKLOADS["chirp_small_c128"]
    S_host = oracle.chirp(w.params(), w.N, w.flo, w.fhi)
    S = _dev(S_host)
    g0 = rb.greedy(S, w.tol, w.kmax, W=torch.empty_like(S), anchor_max=anchor_max)
    ws = rb.workspace(w.N, w.M, w.kmax, anchor_max=anchor_max)
    ws.fill_(0xAB)  # the contents on entry must not matter
    g1 = rb.greedy(S, w.tol, w.kmax, W=torch.empty_like(S), ws=ws, anchor_max=anchor_max)
    _same(g0, g1)
    assert g1["k"] > 30 and g1["status"] == "OK"
    # too small a workspace is refused before any device work
    with pytest.raises(rb.RBError) as ei:
        rb.greedy(S, w.tol, w.kmax, W=torch.empty_like(S), ws=ws[:-256], anchor_max=anchor_max)
    assert ei.value.code == -2


def test_resume_with_workspace(rb):
    w = ri.WORKLOADS["chirp_small_c128"]
    S_host = oracle.chirp(w.params(M=900), 700, w.flo, w.fhi)
    S = _dev(S_host)
    g = rb.greedy(S, w.tol, w.kmax)
    E0 = g["E"][:10].contiguous()
    r0 = rb.greedy(S, w.tol, w.kmax, E0=E0, W=torch.empty_like(S))
    ws = rb.workspace(700, 900, w.kmax)
    r1 = rb.greedy(S, w.tol, w.kmax, E0=E0, W=torch.empty_like(S), ws=ws)
    _same(r0, r1)


def test_mixed_workspace_matches_own_allocation(rb):
    w = ri.WORKLOADS["chirp_small_c128"]
    P = _dev(w.params())
    S32 = rb.chirp_fill(P, w.N, w.flo, w.fhi, dtype=torch.complex64)
    g0 = rb.greedy_c(S32, w.tol, w.kmax, P, w.flo, w.fhi, W=torch.empty_like(S32))
    ws = rb.workspace(w.N, w.M, w.kmax, mixed=True)
    ws.fill_(0x5C)
    g1 = rb.greedy_c(S32, w.tol, w.kmax, P, w.flo, w.fhi, W=torch.empty_like(S32), ws=ws)
    _same(g0, g1)
    assert g1["stats"]["regen_anchors"] == g0["stats"]["regen_anchors"]


def test_breakdown_kahan_nu_max_1(rb):
    theta, delta, n = 1.3, 1e-3, 80
    s = np.sin(theta)
    kb = int(np.argmax(s ** np.arange(n) <= 0.5))  # first step whose pass shrinks by >= 2
    assert s ** (kb - 1) > 0.51 and s ** kb < 0.499  # clear of the threshold
    S = _dev(ri.kahan(n, theta, delta))
    g = rb.greedy(S, 0.0, n, nu_max=1, check=False)
    assert g["status"] == "EBREAKDOWN" and g["k"] == kb
    np.testing.assert_array_equal(g["piv"], np.arange(kb))
    np.testing.assert_allclose(g["rho"], (s * (1 - delta)) ** np.arange(kb), rtol=1e-12)
    # the default nu_max settles every vector: a second pass from step kb on
    g4 = rb.greedy(S, 0.0, n)
    assert g4["status"] != "EBREAKDOWN" and g4["k"] == n
    assert np.all(g4["nu"][1:kb] == 1) and np.all(g4["nu"][kb:] >= 2)
    with pytest.raises(rb.RBError) as ei:
        rb.greedy(S, 0.0, n, nu_max=1)
    assert ei.value.code == -5


def test_breakdown_mixed_nu_max_1(rb):
    """Mixed precision: the first pass of a regenerated candidate shrinks it
    from ||s|| = 1 to its residual rho, so with nu_max = 1 the first chosen
    candidate with rho <= 1/2 stops the greedy."""
    w = ri.WORKLOADS["chirp_small_c128"]
    P = _dev(w.params())
    S32 = rb.chirp_fill(P, w.N, w.flo, w.fhi, dtype=torch.complex64)
    g = rb.greedy_c(S32, w.tol, w.kmax, P, w.flo, w.fhi, nu_max=1, check=False)
    assert g["status"] == "EBREAKDOWN"
    k = g["k"]
    assert np.all(g["rho"][1:] > 0.5) and 0 < k < w.kmax
    E = g["E"].cpu().numpy()
    # one classical pass per vector while rho > 1/2 keeps E orthonormal to
    # about u / (1/2)
    assert np.linalg.norm(E.conj() @ E.T - np.eye(k), 2) <= 1e-13


def test_nonfinite_input_and_regenerated_candidate(rb):
    S_host = ri.gaussian(7, 64, 40)
    S_host[5, 3] = np.inf
    with pytest.raises(rb.RBError) as ei:
        rb.greedy(_dev(S_host), 1e-10, 20)
    assert ei.value.code == -4
    w = ri.WORKLOADS["chirp_small_c128"]
    P = _dev(w.params(M=300))
    S32 = rb.chirp_fill(P, 500, w.flo, w.fhi, dtype=torch.complex64)
    Pnan = torch.full_like(P, float("nan"))
    g = rb.greedy_c(S32, w.tol, 50, Pnan, w.flo, w.fhi, check=False)
    assert g["status"] == "ENONFINITE" and g["k"] == 0


def test_step_trace(rb):
    """Per-step device times add up to the totals of the same call."""
    w = ri.WORKLOADS["chirp_small_c128"]
    S = _dev(oracle.chirp(w.params(), w.N, w.flo, w.fhi))
    g = rb.greedy(S, w.tol, w.kmax, trace=True)
    t, st = g["step_ms"], g["stats"]
    assert t.shape == (g["k"] + 1, 3) and np.all(t >= 0)
    # the sweep slot holds a plain sweep, a fused pass (re-anchoring and
    # sweep) or the estimate update of a step taken from a prediction
    sweep_ms = st["ms_sweep"] + st["ms_fused"] + st["ms_apply"]
    assert abs(t[:, 1].sum() - sweep_ms) <= 1e-6 * sweep_ms + 1e-9
    assert abs(t[:, 0].sum() - st["ms_gs"]) <= 1e-6 * st["ms_gs"] + 1e-9
    assert t[:, 2].sum() <= st["ms_anchor"] + 1e-9  # the initial norms are not a step's
    assert np.count_nonzero(t[:, 1]) == st["sweeps"] + st["fused"] + st["look_steps"] == g["k"]
    # a step taken from a prediction has no orthogonalisation of its own
    assert np.count_nonzero(t[:, 0]) == g["k"] - st["look_steps"]
    assert st["ms_look"] > 0 and st["look_gs"] >= st["look_steps"]
    P = _dev(w.params())
    S32 = rb.chirp_fill(P, w.N, w.flo, w.fhi, dtype=torch.complex64)
    gc = rb.greedy_c(S32, w.tol, w.kmax, P, w.flo, w.fhi, trace=True)
    tc, stc = gc["step_ms"], gc["stats"]
    sweep_c_ms = stc["ms_sweep"] + stc["ms_apply"]
    assert abs(tc[:, 1].sum() - sweep_c_ms) <= 1e-6 * sweep_c_ms + 1e-9
    assert abs(tc[:, 0].sum() - stc["ms_gs"]) <= 1e-6 * stc["ms_gs"] + 1e-9
    assert np.count_nonzero(tc[:, 1]) == stc["sweeps"] + stc["look_steps"] == gc["k"]
