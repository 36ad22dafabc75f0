"""GPU parity of the HIP path against the CPU oracle on the same seeded
inputs (the oracle never sees a value produced by the HIP path as input).

Tolerances (derived from the arithmetic):
  u = 2^-53,  A = max_j ||s_j||^2,  phi_k = 16 (k+1) u sqrt(A)
  resolution of Eq. (6.3) between anchorings: the estimated squared residual
  carries an absolute error <= 16 (anchor_max+1) u A_w and is trusted only
  while est >= theta A_w, so its relative error is <= 16 (am+1) u / theta.
  err_k:   |d err| <= err_ref (1e-10 + 8 (am+1) u / theta) + phi_k
  pivots:  replayed in the oracle; the GPU's pivot must be within the
           near-tie window of the oracle's max squared residual:
           w_k = max_ref (2e-9 + 16 (am+1) u / theta) + 2 sqrt(max_ref) phi_k
  basis:   ||d e_k|| <= 1e-10 + 64 (k+1) u sqrt(A) / rho_k
"""
import numpy as np
import pytest
import torch

import oracle
import rb_inputs as ri

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _gpu_greedy_and_replay(rb, S_host, tol, kmax, **opts):
    S = _dev(S_host)
    g = rb.greedy(S, tol, kmax, **opts)
    ref = oracle.greedy(S_host, tol, kmax, force=g["piv"])
    return g, ref


def _check_replay(g, ref, S_host, theta=None, am=128):
    """theta: the resolution threshold the greedy ran with (None: the
    library default)."""
    if theta is None:
        import paper_1805_06124_amd as rbm
        theta = rbm.default_opts().theta
    k = g["k"]
    A = float(oracle.sqnorms(S_host).max())
    res = 16 * (am + 1) * U / theta
    # the oracle followed the same pivots to the same length (checked before
    # its per-step records are indexed)
    assert ref["k"] == k, (ref["k"], k, g["status"], ref["status"])
    # every forced pivot is within the near-tie window of the oracle's max
    for i in range(k):
        mine, mx = ref["pick"][i]
        phi = 16 * (i + 1) * U * np.sqrt(A)
        w = mx * (2e-9 + res) + 2 * np.sqrt(max(mx, 0.0)) * phi
        assert mine >= mx - w, (i, mine, mx, w)
    np.testing.assert_array_equal(ref["piv"], g["piv"])
    phis = 16 * (np.arange(k + 1) + 1) * U * np.sqrt(A)
    tol_err = ref["err"] * (1e-10 + res / 2) + phis
    assert np.all(np.abs(g["err"] - ref["err"]) <= tol_err), np.max(np.abs(g["err"] - ref["err"]) - tol_err)
    tol_rho = ref["rho"] * 1e-10 + phis[:k]
    assert np.all(np.abs(g["rho"] - ref["rho"]) <= tol_rho)
    E = g["E"].cpu().numpy()
    dE = np.linalg.norm(E - ref["E"], axis=1)
    tol_e = 1e-10 + 64 * (np.arange(k) + 1) * U * np.sqrt(A) / np.maximum(ref["rho"], 1e-300)
    assert np.all(dE <= tol_e), (np.argmax(dE - tol_e), dE.max())
    if k:
        G = E.conj() @ E.T
        assert np.linalg.norm(G - np.eye(k), 2) <= 2e-13


def test_colnorms_bit_exact(rb):
    """Exact column norms: the same bits as the oracle's."""
    for (N, M, seed) in [(1000, 2000, 1), (777, 129, 2), (1, 5, 3), (4099, 17, 4)]:
        S_host = ri.gaussian(seed, N, M) * np.exp(np.random.default_rng(seed).uniform(-3, 3, M))[:, None]
        nrm = rb.colnorms(_dev(S_host)).cpu().numpy()
        np.testing.assert_array_equal(nrm, oracle.sqnorms(S_host))
    w = ri.WORKLOADS["chirp_small_c128"]
    S_host = oracle.chirp(w.params(), w.N, w.flo, w.fhi)
    np.testing.assert_array_equal(rb.colnorms(_dev(S_host)).cpu().numpy(), oracle.sqnorms(S_host))


def test_colnorms_nonfinite(rb):
    S_host = ri.gaussian(5, 64, 10)
    S_host[3, 7] = np.inf
    with pytest.raises(rb.RBError) as ei:
        rb.colnorms(_dev(S_host))
    assert ei.value.code == -4


@pytest.mark.parametrize("N,M", [(1000, 2000), (777, 1234), (1, 7), (300, 1), (4096, 33)])
def test_sweep_matches_oracle(rb, N, M):
    """One fused sweep: c_j, acc_j and est_j against the oracle's definitions
    on ragged shapes (several tiles plus a tail in both dimensions)."""
    S_host = ri.gaussian(10 + N, N, M)
    e_host = ri.gaussian(11, N, 1)[0]
    e_host /= np.linalg.norm(e_host)
    rng = np.random.default_rng(12)
    acc0 = rng.uniform(0, 0.5, M)
    mask = (rng.uniform(size=M) < 0.1).astype(np.uint8)
    if mask.all():
        mask[0] = 0
    nrm = oracle.sqnorms(S_host)
    c_ref = oracle.project(e_host[None, :], S_host)[0]
    acc_ref = acc0 + (c_ref.real ** 2 + c_ref.imag ** 2)
    est_ref = nrm - acc_ref
    acc = _dev(acc0)
    c = torch.zeros(M, dtype=torch.complex128, device="cuda")
    est, J = rb.sweep(_dev(S_host), _dev(e_host), _dev(nrm), acc, _dev(mask), c)
    cg = c.cpu().numpy()
    scale = np.sqrt(nrm) * np.linalg.norm(e_host)
    assert np.all(np.abs(cg - c_ref) <= 16 * U * np.sqrt(N) * scale + 1e-300)
    np.testing.assert_allclose(acc.cpu().numpy(), acc_ref, rtol=1e-13, atol=64 * U * nrm.max() * np.sqrt(N))
    est_m = np.where(mask == 0, est_ref, -np.inf)
    jr = int(np.argmax(est_m))
    # pivot: exact unless the runner-up is within rounding of the max
    if J != jr:
        assert est_m[J] >= est_m[jr] - 1e-12 * abs(est_m[jr]) - 64 * U * nrm.max() * np.sqrt(N)
    assert abs(est - est_m[jr]) <= 1e-12 * abs(est_m[jr]) + 64 * U * nrm.max() * np.sqrt(N)


def test_sweep_all_masked(rb):
    S_host = ri.gaussian(20, 50, 9)
    e_host = np.zeros(50, dtype=np.complex128)
    e_host[0] = 1
    est, J = rb.sweep(_dev(S_host), _dev(e_host), _dev(oracle.sqnorms(S_host)),
                      torch.zeros(9, dtype=torch.float64, device="cuda"),
                      torch.ones(9, dtype=torch.uint8, device="cuda"))
    assert J == -1 and est == -np.inf


def test_chirp_fill_matches_oracle(rb):
    """Device generator vs the oracle's: the two evaluate the same formula
    with different libm/ocml, so agree to the phase's rounding
    (|Psi| u, Psi up to ~1.4e3 rad)."""
    for key in ("chirp_small_c128", "chirp_10k_409600_c128", "chirp_10k_1638400_c64"):
        w = ri.WORKLOADS[key]
        P = w.params(M=257, start=1000)
        ref = oracle.chirp(P, w.N, w.flo, w.fhi)
        got = rb.chirp_fill(_dev(P), w.N, w.flo, w.fhi).cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 2e-12 * np.max(np.abs(ref))
        np.testing.assert_allclose(np.linalg.norm(got, axis=1), 1.0, rtol=1e-14)
        got32 = rb.chirp_fill(_dev(P), w.N, w.flo, w.fhi, dtype=torch.complex64).cpu().numpy()
        assert np.max(np.abs(got32 - ref)) <= 2 ** -24 * np.max(np.abs(ref)) * 1.01 + 2e-12


def test_greedy_small_chirp_workload(rb):
    """The small chirp workload (1,000 x 2,000, tol 1e-10): replay parity,
    free-run pivots, termination at the oracle's k."""
    w = ri.WORKLOADS["chirp_small_c128"]
    S_host = oracle.chirp(w.params(), w.N, w.flo, w.fhi)
    g, ref = _gpu_greedy_and_replay(rb, S_host, w.tol, w.kmax)
    _check_replay(g, ref, S_host)
    free = oracle.greedy(S_host, w.tol, w.kmax)
    assert g["k"] == free["k"] and g["status"] == "OK"
    assert g["err"][-1] < w.tol
    np.testing.assert_array_equal(g["piv"], free["piv"])


@pytest.mark.parametrize("case", ["gauss", "graded", "kahan", "rank5", "diag", "wide", "real"])
def test_greedy_structured_inputs(rb, case):
    if case == "gauss":
        S_host, tol, kmax = ri.gaussian(30, 300, 200), 1e-10, 200
    elif case == "graded":
        S_host, tol, kmax = ri.graded(31, 257, 300, 0.97), 1e-8, 300
    elif case == "kahan":
        S_host, tol, kmax = ri.kahan(80, 1.3, 1e-3), 0.0, 80
    elif case == "rank5":
        S_host, tol, kmax = ri.low_rank(32, 513, 700, 5), 1e-10, 50
    elif case == "diag":
        S_host, tol, kmax = ri.diagonal(np.linspace(3, 0.1, 40)), 0.05, 40
    elif case == "wide":
        S_host, tol, kmax = ri.gaussian(33, 20, 500), 0.0, 500
    else:
        S_host, tol, kmax = ri.gaussian(34, 100, 90, real=True), 1e-12, 90
    g, ref = _gpu_greedy_and_replay(rb, S_host, tol, kmax)
    _check_replay(g, ref, S_host)
    if case == "kahan":
        s = np.sin(1.3) * (1 - 1e-3)
        np.testing.assert_array_equal(g["piv"], np.arange(80))
        np.testing.assert_allclose(g["err"][:80], s ** np.arange(80), rtol=1e-10)
    if case == "rank5":
        assert g["k"] == 5
    if case == "wide":
        assert g["k"] == 20


def test_greedy_tol_squared_reading(rb):
    """tol = 1e-5 (the squared-error reading of 1e-10) on the small workload."""
    w = ri.WORKLOADS["chirp_small_c128"]
    S_host = oracle.chirp(w.params(), w.N, w.flo, w.fhi)
    g, ref = _gpu_greedy_and_replay(rb, S_host, 1e-5, w.kmax)
    _check_replay(g, ref, S_host)
    assert g["err"][-1] < 1e-5 <= g["err"][-2]


@pytest.mark.parametrize("mode", ["W", "inplace", "own"])
def test_greedy_working_matrix_modes(rb, mode):
    w = ri.WORKLOADS["chirp_small_c128"]
    S_host = oracle.chirp(w.params(M=700), 600, w.flo, w.fhi)
    S = _dev(S_host)
    if mode == "W":
        g = rb.greedy(S, 1e-10, 200, W=torch.empty_like(S))
    elif mode == "inplace":
        g = rb.greedy(S, 1e-10, 200, W=S)
    else:
        g = rb.greedy(S, 1e-10, 200)
    ref = oracle.greedy(S_host, 1e-10, 200, force=g["piv"])
    _check_replay(g, ref, S_host)
    assert g["stats"]["anchors"] >= 1


def test_greedy_theta_1e3(rb):
    """The coarser threshold theta = 1e-3 (more re-anchorings) with its
    tighter resolution bound."""
    w = ri.WORKLOADS["chirp_small_c128"]
    S_host = oracle.chirp(w.params(M=900), 800, w.flo, w.fhi)
    g, ref = _gpu_greedy_and_replay(rb, S_host, 1e-10, 200, theta=1e-3)
    _check_replay(g, ref, S_host, theta=1e-3)


def test_greedy_anchor_options(rb):
    """A small panel and a tight theta force many re-anchorings; results stay
    within the same bounds."""
    w = ri.WORKLOADS["chirp_small_c128"]
    S_host = oracle.chirp(w.params(M=900), 800, w.flo, w.fhi)
    g, ref = _gpu_greedy_and_replay(rb, S_host, 1e-10, 200, anchor_max=4, theta=0.1)
    _check_replay(g, ref, S_host, theta=0.1, am=4)
    assert g["stats"]["anchors"] > g["k"] // 4 - 1


def test_greedy_edge_cases(rb):
    # max ||s|| < tol -> no vector
    g = rb.greedy(_dev(1e-12 * ri.gaussian(40, 10, 10)), 1e-6, 5)
    assert g["k"] == 0 and g["status"] == "OK"
    # kmax = 0
    g = rb.greedy(_dev(ri.gaussian(41, 10, 10)), 1e-6, 0)
    assert g["k"] == 0 and g["status"] == "KMAX"
    # one column / one row
    S1 = ri.gaussian(42, 33, 1)
    g = rb.greedy(_dev(S1), 0.0, 3)
    assert g["k"] == 1 and g["err"][1] == 0.0 and g["piv"][0] == 0
    g = rb.greedy(_dev(ri.gaussian(43, 1, 9)), 0.0, 3)
    assert g["k"] == 1
    # zero matrix
    g = rb.greedy(torch.zeros((6, 8), dtype=torch.complex128, device="cuda"), 1e-10, 4)
    assert g["k"] == 0
    # exact rank deficiency with tol = 0: stops by rank, not by kmax
    g = rb.greedy(_dev(ri.low_rank(44, 50, 40, 3)), 0.0, 40)
    assert g["k"] == 3 and g["status"] == "RANK"
    # non-finite input
    S = ri.gaussian(45, 10, 10)
    S[1, 1] = np.nan
    with pytest.raises(rb.RBError):
        rb.greedy(_dev(S), 1e-6, 5)


def test_greedy_deterministic(rb):
    w = ri.WORKLOADS["chirp_small_c128"]
    S = _dev(oracle.chirp(w.params(), w.N, w.flo, w.fhi))
    a = rb.greedy(S, w.tol, w.kmax)
    b = rb.greedy(S, w.tol, w.kmax)
    np.testing.assert_array_equal(a["piv"], b["piv"])
    np.testing.assert_array_equal(a["err"], b["err"])
    assert torch.equal(a["E"], b["E"])


@pytest.mark.parametrize("N,k,M", [(1000, 47, 2000), (777, 65, 1234), (64, 1, 1), (4, 130, 3), (10000, 3, 100),
                                   (300, 161, 517), (300, 190, 700), (257, 224, 65), (300, 250, 129),
                                   (300, 450, 70)])
def test_project_matches_oracle(rb, N, k, M):
    """Every block height (32 to 224 basis vectors) and several passes over
    S for k > 224, with ragged tails in rows, columns and basis vectors."""
    E_host = ri.gaussian(50 + k, N, k)
    S_host = ri.gaussian(51 + M, N, M)
    C = rb.project(_dev(E_host), _dev(S_host)).cpu().numpy()  # (M, k)
    ref = oracle.project(E_host, S_host)                      # (k, M)
    scale = np.linalg.norm(E_host, axis=1)[None, :] * np.linalg.norm(S_host, axis=1)[:, None]
    assert np.all(np.abs(C - ref.T) <= 16 * U * np.sqrt(N) * scale)


def test_chirp_params_bit_exact(rb):
    """The device parameter generator (SplitMix64 counters, step-by-step
    rounded affine maps) returns the same bits as the shared seeded
    generator, including a large counter offset."""
    cases = [(1805, 409600, 0, (20.0, 60.0, 1.0, 4.0)), (1806, 1000, 12345, (40.0, 60.0, 1.0, 4.0)),
             (7, 3, 2 ** 33, (20.0, 80.0, 1.0, 8.0))]
    for seed, M, start, rng in cases:
        got = rb.chirp_params(seed, M, *rng, start=start).cpu().numpy()
        want = ri.chirp_params(seed, M, *rng, start=start)
        np.testing.assert_array_equal(got, want)


def test_stream_read_sums(rb):
    """The plain streaming read visits every element once: its partial sums
    add up to the sum of the buffer (exactly representable values)."""
    x = torch.arange(1, 2 * 1000003 + 1, dtype=torch.float64, device="cuda").view(-1, 2)
    x = torch.view_as_complex(x.contiguous())
    part = torch.zeros(64, dtype=torch.float64, device="cuda")
    rb.stream_read(x, part)
    n = 2 * 1000003
    assert part.sum().item() == n * (n + 1) / 2
