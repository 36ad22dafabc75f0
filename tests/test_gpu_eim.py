"""GPU parity of empirical-interpolation nodes and interpolant validation
(rb_eim_z, rb_eim_errors_z) against closed forms, LAPACK's LU with partial
pivoting, and the oracle (the standard EIM definition with LAPACK solves).

Bases come from the oracle's greedy or from closed-form constructions and
are uploaded; the oracle never sees a GPU value except the node sequence it
is asked to replay.

Tolerances: a node must lie in the near-tie window of the oracle's own
maximum, |r(p_gpu)| >= max |r| (1 - 1e-9).  The elimination form and the
oracle's solve differ by rounding times the conditioning of the
interpolation matrix, so peaks and interpolation errors are compared to
1e-8 relative plus 1e-12 absolute.
"""
import numpy as np
import pytest
import scipy.linalg
import torch

import oracle
import rb_inputs as ri
from oracle import eim as oeim

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_eim_triangular_permutation_closed_form(rb):
    """e_j = delta_{pi_j} + sum_{i<j} a_ji delta_{pi_i}: nodes = pi, every
    peak = 1."""
    rng = np.random.default_rng(90)
    N, k = 700, 60
    pi = rng.permutation(N)[:k]
    E = np.zeros((k, N), dtype=np.complex128)
    for j in range(k):
        E[j, pi[j]] = 1.0
        for i in range(j):
            E[j, pi[i]] = 0.9 * (rng.standard_normal() + 1j * rng.standard_normal())
    out = rb.eim(_dev(E))
    assert out["status"] == "OK" and out["k"] == k
    np.testing.assert_array_equal(out["nodes"], pi)
    np.testing.assert_allclose(out["peak"], 1.0, atol=1e-12)


@pytest.mark.parametrize("seed,N,k", [(91, 300, 30), (92, 1000, 129), (93, 64, 64)])
def test_eim_equals_lu_partial_pivoting(rb, seed, N, k):
    """Real basis: the nodes are the pivot rows of LAPACK's LU with partial
    pivoting of E^T and the peaks are |U_jj|."""
    rng = np.random.default_rng(seed)
    E = rng.standard_normal((k, N))
    lu, piv = scipy.linalg.lu_factor(E.T)
    perm = np.arange(N)
    for i, p in enumerate(piv):
        perm[i], perm[p] = perm[p], perm[i]
    out = rb.eim(_dev(E.astype(np.complex128)))
    np.testing.assert_array_equal(out["nodes"], perm[:k])
    np.testing.assert_allclose(out["peak"], np.abs(np.diag(lu)[:k]), rtol=1e-10)


def test_eim_chirp_parity_and_interpolant(rb):
    """The small chirp family's basis (oracle greedy, 46 vectors).
    - The nodes replay in the oracle; peaks and normalised residuals agree.
    - The interpolant reproduces the basis.
    - Its errors on 2,000 held-out chirps agree with the oracle's LAPACK
      solve."""
    w = ri.WORKLOADS["chirp_small_c128"]
    S = oracle.chirp(w.params(), w.N, w.flo, w.fhi)
    E = oracle.greedy(S, w.tol, w.kmax)["E"]
    k = E.shape[0]
    out = rb.eim(_dev(E))
    assert out["status"] == "OK"
    ref = oeim.nodes(E, force=out["nodes"])
    mine, mx = ref["pick"][:, 0], ref["pick"][:, 1]
    assert np.all(mine >= mx * (1 - 1e-9))
    free = oeim.nodes(E)
    np.testing.assert_array_equal(free["nodes"], out["nodes"])
    np.testing.assert_allclose(out["peak"], mine, rtol=1e-8, atol=1e-12)
    R = out["R"].cpu().numpy()
    Rref = ref["resid"] / ref["resid"][np.arange(k), out["nodes"]][:, None]
    assert np.max(np.abs(R - Rref)) <= 1e-8 * np.max(np.abs(Rref))
    np.testing.assert_allclose(out["Tinv"].cpu().numpy() @ np.tril(R[:, out["nodes"]].T), np.eye(k), atol=1e-10)
    # the interpolant reproduces the basis
    eb = rb.eim_errors(out, _dev(E)).cpu().numpy()
    assert eb.max() <= 1e-12
    V = oracle.chirp(w.params(seed=ri.HELDOUT_SEED), w.N, w.flo, w.fhi)
    got = rb.eim_errors(out, _dev(V)).cpu().numpy()
    want = oeim.interpolation_errors(E, out["nodes"], V)
    assert np.all(np.abs(got - want) <= 1e-8 * want + 1e-12), np.max(np.abs(got - want) / (want + 1e-12))


def test_eim_dependent_basis(rb):
    """A basis whose fourth vector repeats the second: r_3 = 0, status RANK
    with k_out = 3."""
    E = ri.gaussian(94, 200, 6)
    E[3] = E[1]
    out = rb.eim(_dev(E))
    assert out["status"] == "RANK" and out["k"] == 3
    np.testing.assert_array_equal(out["nodes"][:3], oeim.nodes(E[:3])["nodes"])
