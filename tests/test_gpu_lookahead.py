"""Pivot lookahead of the FP64 greedy: a sweep that also carries predicted
vectors, and steps taken from those predictions without a sweep of their
own, must leave every output bit-identical to the greedy without lookahead
(the predicted coefficients and estimates are formed with the sweep's own
arithmetic and the predicted vectors by the same orthogonalisation code).

Cases: the small chirp workload at every depth, short candidate lists
(many wrong predictions), a narrow coefficient panel (predictions cut at
the panel's end, written re-anchorings), a continuation from a given basis,
Gaussian columns, and Kahan's matrix stopped by the breakdown test."""
import numpy as np
import pytest
import torch

import oracle
import rb_inputs as ri

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _same(g0, g1):
    assert g0["k"] == g1["k"] and g0["status"] == g1["status"]
    for key in ("piv", "err", "rho", "nu"):
        np.testing.assert_array_equal(g0[key], g1[key], err_msg=key)
    assert torch.equal(g0["E"], g1["E"])


@pytest.fixture(scope="module")
def chirp_small():
    w = ri.WORKLOADS["chirp_small_c128"]
    return w, _dev(oracle.chirp(w.params(), w.N, w.flo, w.fhi))


@pytest.mark.parametrize("depth", [1, 2, 3, 4, 5])
def test_lookahead_bit_identical(rb, chirp_small, depth):
    w, S = chirp_small
    g0 = rb.greedy(S, w.tol, w.kmax, lookahead=0)
    g1 = rb.greedy(S, w.tol, w.kmax, lookahead=depth)
    _same(g0, g1)
    st = g1["stats"]
    assert g0["stats"]["look_steps"] == 0 and g0["stats"]["look_gs"] == 0
    assert st["look_steps"] > 0 and st["look_sweeps"] > 0
    # every basis vector has exactly one sweep, fused pass or prediction
    assert st["sweeps"] + st["fused"] + st["look_steps"] == g1["k"]
    assert st["look_steps"] <= depth * st["look_sweeps"]


@pytest.mark.parametrize("look_k", [1, 3, 8192])
def test_lookahead_list_lengths(rb, chirp_small, look_k):
    w, S = chirp_small
    g0 = rb.greedy(S, w.tol, w.kmax, lookahead=0)
    g1 = rb.greedy(S, w.tol, w.kmax, lookahead=5, look_k=look_k)
    _same(g0, g1)


def test_lookahead_narrow_panel_and_theta(rb, chirp_small):
    """anchor_max = 6: predictions stop at the panel's end and written
    re-anchorings come every few steps; theta = 1e-3 adds norms-only and
    fused re-anchorings."""
    w, S = chirp_small
    for kw in (dict(anchor_max=6), dict(theta=1e-3), dict(anchor_max=6, theta=1e-3, fuse=0)):
        g0 = rb.greedy(S, w.tol, w.kmax, W=torch.empty_like(S), lookahead=0, **kw)
        g1 = rb.greedy(S, w.tol, w.kmax, W=torch.empty_like(S), lookahead=5, **kw)
        _same(g0, g1)
        assert g1["stats"]["anchors"] == g0["stats"]["anchors"]


def test_lookahead_resume(rb):
    w = ri.WORKLOADS["chirp_small_c128"]
    S = _dev(oracle.chirp(w.params(M=900), 700, w.flo, w.fhi))
    E0 = rb.greedy(S, w.tol, w.kmax)["E"][:12].contiguous()
    g0 = rb.greedy(S, w.tol, w.kmax, E0=E0, W=torch.empty_like(S), lookahead=0)
    g1 = rb.greedy(S, w.tol, w.kmax, E0=E0, W=torch.empty_like(S), lookahead=3)
    _same(g0, g1)
    assert g1["stats"]["look_steps"] > 0


def test_lookahead_gaussian_and_kmax(rb):
    """Gaussian columns (flat spectrum: many wrong predictions) up to kmax,
    with kmax cutting a prediction chain."""
    S = _dev(ri.gaussian(3, 500, 700))
    for kmax in (37, 120):
        g0 = rb.greedy(S, 0.0, kmax, lookahead=0)
        g1 = rb.greedy(S, 0.0, kmax, lookahead=5)
        _same(g0, g1)
        assert g1["k"] == kmax


def test_lookahead_two_pass_predictions_rank_and_graded(rb, chirp_small):
    """A predicted pivot's orthogonalisation queues only two passes (one
    that would need more is not accepted and its step runs its own).  Runs
    into the numerical rank (exactly low-rank inputs, tol 0), a strongly
    graded matrix and kappa squeezed towards 1 on full-rank columns stay
    bit-identical to no lookahead, rank detection included.  (On these
    inputs every orthogonalisation settles within two passes: a second pass
    changes ||v|| only at second order.)"""
    w, S = chirp_small
    cases = [(_dev(ri.low_rank(31 + r, 400, 600, r)), 0.0, r + 12, {}) for r in (10, 40)]
    cases.append((_dev(ri.graded(7, 300, 500, 0.7)), 0.0, 200, {}))
    cases += [(S, w.tol, w.kmax, dict(kappa=1.0 + 2.0 ** -52))]
    for Sx, tol, kmax, kw in cases:
        g0 = rb.greedy(Sx, tol, kmax, check=False, lookahead=0, **kw)
        g1 = rb.greedy(Sx, tol, kmax, check=False, lookahead=5, **kw)
        _same(g0, g1)
        assert g0["k"] == 0 or int(np.max(g0["nu"][:g0["k"]])) <= 2


def test_lookahead_breakdown(rb):
    theta, delta, n = 1.3, 1e-3, 80
    S = _dev(ri.kahan(n, theta, delta))
    g0 = rb.greedy(S, 0.0, n, nu_max=1, check=False, lookahead=0)
    g1 = rb.greedy(S, 0.0, n, nu_max=1, check=False, lookahead=5)
    assert g1["status"] == "EBREAKDOWN"
    _same(g0, g1)


def test_lookahead_many_columns(rb):
    """600,000 columns (37,500 groups of 16): the candidate list is selected
    from the maxima of pairs of groups; still bit-identical."""
    w = ri.WORKLOADS["chirp_10k_409600_c128"]
    P = _dev(w.params(M=600_000))
    S = rb.chirp_fill(P, 64, w.flo, w.fhi)
    g0 = rb.greedy(S, 1e-9, 64, lookahead=0)
    g1 = rb.greedy(S, 1e-9, 64)
    _same(g0, g1)
    assert g1["k"] > 20 and g1["stats"]["look_steps"] > 0


@pytest.mark.parametrize("look", [3, 5])
def test_mixed_lookahead_ragged_columns(rb, look):
    """A column count that is not a multiple of a workgroup's 16 columns
    (1,995 of the small chirp family) with depths whose sweeps spread the
    16 columns over eight waves of two: bit-identical to no lookahead."""
    w = ri.WORKLOADS["chirp_small_c128"]
    P = _dev(w.params(M=1995))
    S32 = rb.chirp_fill(P, w.N, w.flo, w.fhi, dtype=torch.complex64)
    g0 = rb.greedy_c(S32, w.tol, w.kmax, P, w.flo, w.fhi, W=torch.empty_like(S32), lookahead32=0)
    g1 = rb.greedy_c(S32, w.tol, w.kmax, P, w.flo, w.fhi, W=torch.empty_like(S32), lookahead32=look)
    _same(g0, g1)
    assert g1["stats"]["look_steps"] > 0 and g1["k"] > 20


@pytest.mark.parametrize("kw", [dict(), dict(lookahead32=1), dict(lookahead32=5), dict(anchor_max=6, lookahead32=4),
                                dict(lookahead32=2, look_k=3)])
def test_mixed_lookahead_bit_identical(rb, kw):
    """The mixed greedy: a step is taken from a prediction when the top-8
    set of the complex64 estimates equals the predicted one; pivots, errors,
    residuals, passes, status and basis are bit-identical to the mixed
    greedy without lookahead (deflating and exact re-anchorings included)."""
    w = ri.WORKLOADS["chirp_small_c128"]
    P = _dev(w.params())
    S32 = rb.chirp_fill(P, w.N, w.flo, w.fhi, dtype=torch.complex64)
    g0 = rb.greedy_c(S32, w.tol, w.kmax, P, w.flo, w.fhi, W=torch.empty_like(S32), lookahead32=0,
                     **{a: b for a, b in kw.items() if a not in ("lookahead32", "look_k")})
    g1 = rb.greedy_c(S32, w.tol, w.kmax, P, w.flo, w.fhi, W=torch.empty_like(S32), **kw)
    _same(g0, g1)
    for key in ("anchors", "regen_anchors", "misses"):
        assert g0["stats"][key] == g1["stats"][key], key
    st = g1["stats"]
    assert g0["stats"]["look_steps"] == 0
    if kw.get("look_k", 4096) > 3:
        assert st["look_steps"] > 0
    assert st["sweeps"] + st["look_steps"] == g1["k"]
