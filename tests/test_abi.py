"""The C ABI of librb.so: it loads, exports every entry point include/rb.h
declares, and validates arguments on the host before any device work.
CPU only (no call here reaches a GPU)."""
import ctypes
import os
import re

import pytest

import paper_1805_06124_amd as rbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rb.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rb_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(rbm.LIB_PATH):
        pytest.skip("librb.so not built")
    return rbm.load_library()


def test_header_declares_expected_entry_points():
    d = _declared()
    for name in ("rb_greedy_z", "rb_sweep_z", "rb_colnorms_z", "rb_project_z", "rb_chirp_fill",
                 "rb_default_opts", "rb_strerror", "rb_last_error"):
        assert name in d


def test_every_declared_symbol_is_exported(L):
    for name in _declared():
        assert hasattr(L, name), name
    assert set(rbm.EXPORTS) <= set(_declared())


def test_default_opts_and_strerror(L):
    o = rbm.Opts()
    L.rb_default_opts(ctypes.byref(o))
    assert o.kappa == 2.0 and o.nu_max == 4 and o.nu_min == 1 and o.anchor_max == 128
    assert 0 < o.theta < 1
    assert b"invalid" in L.rb_strerror(-1)
    assert b"kmax" in L.rb_strerror(1)
    assert b"Gram-Schmidt" in L.rb_strerror(-5)
    assert b"eigen" in L.rb_strerror(-6)
    assert o.step_ms is None


def _greedy_args(N=10, M=10, ldS=10, kmax=3, tol=1e-10, S=1, E=1, ldE=10, piv=True):
    import numpy as np
    P = ctypes.c_void_p
    piv_a = np.zeros(4, dtype=np.int64)
    err = np.zeros(5)
    rho = np.zeros(4)
    k = ctypes.c_int64(-7)
    return [P(S) if S else None, N, M, ldS, tol, kmax, None, 0, P(E) if E else None, ldE,
            piv_a.ctypes.data_as(P) if piv else None, err.ctypes.data_as(P), rho.ctypes.data_as(P), None,
            ctypes.byref(k), None, 0, None, None, None], k


@pytest.mark.parametrize("bad", [dict(N=0), dict(M=-1), dict(ldS=5), dict(kmax=-1), dict(tol=-1.0),
                                 dict(tol=float("nan")), dict(S=0), dict(E=0), dict(ldE=3), dict(piv=False)])
def test_greedy_rejects_bad_arguments_on_host(L, bad):
    args, k = _greedy_args(**bad)
    assert L.rb_greedy_z(*args) == -1
    assert k.value == -7  # nothing written
    assert L.rb_last_error()


def test_other_entry_points_reject_bad_arguments(L):
    P = ctypes.c_void_p
    d = ctypes.c_double()
    j = ctypes.c_int64()
    assert L.rb_colnorms_z(None, 4, 4, 4, P(1), None) == -1
    assert L.rb_colnorms_z(P(1), 4, 4, 3, P(1), None) == -1
    assert L.rb_sweep_z(P(1), 4, 4, 4, None, P(1), P(1), None, None, 1, ctypes.byref(d), ctypes.byref(j), None) == -1
    assert L.rb_project_z(P(1), 4, 2, 4, P(1), 4, 4, P(1), 1, None) == -1  # ldC < k
    assert L.rb_chirp_fill(P(1), 4, 0.0, 10.0, 8, 0, P(1), 8, None) == -1  # flo must be > 0
    assert L.rb_chirp_fill(P(1), 4, 20.0, 10.0, 8, 0, P(1), 8, None) == -1  # fhi < flo
    assert L.rb_chirp_fill(P(1), 4, 20.0, 30.0, 8, 2, P(1), 8, None) == -1  # dtype


def test_bad_options_rejected(L):
    o = rbm.Opts()
    L.rb_default_opts(ctypes.byref(o))
    o.kappa = 1.0
    args, k = _greedy_args()
    args[17] = ctypes.byref(o)
    assert L.rb_greedy_z(*args) == -1


def test_product_package_does_not_import_oracle():
    import ast
    pkg = os.path.join(ROOT, "paper_1805_06124_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                tree = ast.parse(open(os.path.join(dirpath, f)).read())
                for node in ast.walk(tree):
                    if isinstance(node, ast.Import):
                        assert all(not a.name.startswith("oracle") for a in node.names)
                    if isinstance(node, ast.ImportFrom):
                        assert not (node.module or "").startswith("oracle")
            if f.endswith((".hip", ".h", ".cpp")):
                assert "oracle" not in open(os.path.join(dirpath, f)).read().lower()


def test_workspace_sizes(L):
    """The size queries: positive for valid sizes, 0 for invalid ones, and
    they grow with the coefficient panel (anchor_max x M complex128) and, for
    the mixed greedy, hold the regeneration chunk and its coefficients."""
    o = rbm.Opts()
    L.rb_default_opts(ctypes.byref(o))
    z = L.rb_greedy_z_workspace(1000, 2000, 200, None)
    assert z == L.rb_greedy_z_workspace(1000, 2000, 200, ctypes.byref(o))
    assert z >= 16 * 128 * 2000 + 25 * 2000
    assert L.rb_greedy_z_workspace(1000, 4000, 200, None) > z
    o.anchor_max = 16
    assert L.rb_greedy_z_workspace(1000, 2000, 200, ctypes.byref(o)) < z - 16 * 100 * 2000
    assert L.rb_greedy_z_workspace(0, 2000, 200, None) == 0
    assert L.rb_greedy_z_workspace(1000, 2000, -1, None) == 0
    o.anchor_max = 0
    assert L.rb_greedy_z_workspace(1000, 2000, 200, ctypes.byref(o)) == 0
    # the pivot lookahead: depth 0..5, a list of 1..8192 columns (24 bytes
    # each: the record and its running sum) only when the depth is nonzero
    L.rb_default_opts(ctypes.byref(o))
    assert (o.lookahead, o.look_k, o.lookahead32) == (5, 4096, -1)
    for look, k_list, ok in ((0, 0, True), (5, 1, True), (5, 8192, True), (6, 2048, False), (-1, 2048, False),
                             (3, 0, False), (3, 8193, False)):
        o.lookahead, o.look_k = look, k_list
        assert (L.rb_greedy_z_workspace(1000, 2000, 200, ctypes.byref(o)) > 0) == ok, (look, k_list)
    o.lookahead, o.look_k = 0, 2048
    z0 = L.rb_greedy_z_workspace(1000, 2000, 200, ctypes.byref(o))
    o.lookahead = 1
    assert L.rb_greedy_z_workspace(1000, 2000, 200, ctypes.byref(o)) >= z0 + 24 * 2048
    c = L.rb_greedy_c_workspace(1000, 2000, 200, None)
    chunk = 2000  # regen_chunk (32768) clamped to M
    assert c >= z + 16 * chunk * (1000 + 200)
    assert L.rb_greedy_c_workspace(1000, 0, 200, None) == 0


def _ws_args(ws, nbytes, W=1):
    args, k = _greedy_args()
    args[6] = ctypes.c_void_p(W) if W else None  # W
    args[7] = 10
    args[15] = ctypes.c_void_p(ws) if ws else None
    args[16] = nbytes
    return args, k


def test_greedy_workspace_contract_on_host(L):
    """With a caller workspace: too small -> RB_ENOMEM, missing W or a
    misaligned workspace -> RB_EINVAL, all before any device work (the
    pointers here are not device memory)."""
    need = L.rb_greedy_z_workspace(10, 10, 3, None)
    args, k = _ws_args(4096, need - 1)
    assert L.rb_greedy_z(*args) == -2
    assert k.value == -7 and b"needed" in L.rb_last_error()
    args, k = _ws_args(4096, need, W=0)
    assert L.rb_greedy_z(*args) == -1
    args, k = _ws_args(4100, need)
    assert L.rb_greedy_z(*args) == -1
    # the mixed greedy: same contract with its own size
    needc = L.rb_greedy_c_workspace(10, 10, 3, None)
    assert needc > need
    P = ctypes.c_void_p
    import numpy as np
    piv, err, rho = np.zeros(4, dtype=np.int64), np.zeros(5), np.zeros(4)
    kk = ctypes.c_int64(-7)
    rc = L.rb_greedy_c(P(1), 10, 10, 10, 1e-10, 3, P(1), None, P(1), 10, P(1), 10, piv.ctypes.data_as(P),
                       err.ctypes.data_as(P), rho.ctypes.data_as(P), None, ctypes.byref(kk), P(4096), needc - 1,
                       None, None, None)
    assert rc == -2 and kk.value == -7


def test_reconstruct_workspace_contract_on_host(L):
    """rb_reconstruct_z_workspace grows with j and M and rejects sizes the
    routine rejects; with a caller workspace, too small -> RB_ENOMEM and
    misaligned -> RB_EINVAL, before any device work (the pointers here are
    not device memory)."""
    z = L.rb_reconstruct_z_workspace(141, 409600)
    assert z >= 16 * (141 * 409600 + 5 * 141 * 141)
    assert L.rb_reconstruct_z_workspace(141, 409601) > z
    assert L.rb_reconstruct_z_workspace(140, 409600) < z
    # j > 141: the global-memory Jacobi, no rotation log
    assert L.rb_reconstruct_z_workspace(142, 409600) < z
    for j, M in ((0, 10), (2049, 10), (5, 0), (-1, 10)):
        assert L.rb_reconstruct_z_workspace(j, M) == 0, (j, M)
    assert L.rb_reconstruct_z_workspace(2048, 10) > 0
    import numpy as np
    P = ctypes.c_void_p
    need = L.rb_reconstruct_z_workspace(3, 10)
    sigma = np.zeros(3)

    def call(ws, nbytes, j=3):
        k = ctypes.c_int64(-7)
        rc = L.rb_reconstruct_z(P(1), 8, j, 8, P(1), 10, 3, 0.0, P(1), 8, sigma.ctypes.data_as(P), None,
                                ctypes.byref(k), P(ws) if ws else None, nbytes, None)
        return rc, k.value

    assert call(4096, need - 1) == (-2, -7)
    assert b"needed" in L.rb_last_error()
    assert call(4096 + 16, need) == (-1, -7)
    assert call(4096, need, j=0) == (-1, -7)
