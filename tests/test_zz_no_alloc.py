"""rb_greedy_z_noalloc through the C ABI against rb_greedy_z on the same
inputs: two calls in a row on one device (the second on a smaller matrix,
so the fixed workspace holds the first call's data when the second starts),
and a request larger than the fixed workspace (refused with RB_ENOMEM before
any device work).  Both entry points run the same kernels in the same order
on the same inputs, so every output must be bit-identical."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_1805_06124_amd as rbm
import rb_inputs as ri

pytestmark = pytest.mark.gpu


def _call(L, fn, S, tol, kmax, W, E, *extra):
    M, N = S.shape
    kcap = min(kmax, N, M)
    P = ctypes.c_void_p
    piv = np.full(kcap, -1, dtype=np.int64)
    err = np.full(kcap + 1, -1.0)
    rho = np.full(kcap, -1.0)
    nu = np.zeros(kcap, dtype=np.int32)
    k = ctypes.c_int64(-7)
    rc = getattr(L, fn)(P(S.data_ptr()), N, M, S.stride(0), tol, kmax, P(W.data_ptr()), W.stride(0),
                        P(E.data_ptr()), E.stride(0), piv.ctypes.data_as(P), err.ctypes.data_as(P),
                        rho.ctypes.data_as(P), nu.ctypes.data_as(P), ctypes.byref(k), *extra, None, None,
                        P(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    kk = k.value
    return rc, kk, piv[:kk], err[:kk + 1], rho[:kk], nu[:kk], E[:kk].clone()


def _case(rb, L, N, M, seed):
    w = ri.WORKLOADS["chirp_small_c128"]
    S_host = oracle.chirp(w.params(M=M, seed=seed), N, w.flo, w.fhi)
    S = torch.from_numpy(S_host).cuda()
    kmax = 200
    kcap = min(kmax, N, M)
    E1 = torch.full((kcap, N), float("nan"), dtype=torch.complex128, device="cuda")
    E2 = torch.full((kcap, N), float("nan"), dtype=torch.complex128, device="cuda")
    ref = _call(L, "rb_greedy_z", S, 1e-10, kmax, torch.empty_like(S), E1, None, 0)
    got = _call(L, "rb_greedy_z_noalloc", S, 1e-10, kmax, torch.empty_like(S), E2)
    assert ref[0] == 0 and got[0] == 0, (ref[0], got[0], L.rb_last_error())
    assert got[1] == ref[1] and got[1] > 20
    for a, b in zip(ref[2:6], got[2:6]):
        np.testing.assert_array_equal(a, b)
    assert torch.equal(ref[6], got[6])
    return got[1]


def test_noalloc_matches_rb_greedy_z_twice(rb):
    L = rb.load()
    k1 = _case(rb, L, 1000, 2000, 1805)
    k2 = _case(rb, L, 600, 700, 4242)  # smaller: the array still holds call 1's data
    assert k1 > 0 and k2 > 0


def test_noalloc_refuses_oversize(rb):
    L = rb.load()
    need = L.rb_greedy_z_workspace(16, 40000, 16, None)
    assert need > rbm.NOALLOC_SCRATCH_BYTES
    P = ctypes.c_void_p
    piv, err, rho = np.zeros(16, dtype=np.int64), np.zeros(17), np.zeros(16)
    k = ctypes.c_int64(-7)
    # pointers are never dereferenced: the size check comes first
    rc = L.rb_greedy_z_noalloc(P(256), 16, 40000, 16, 1e-10, 16, P(256), 16, P(256), 16, piv.ctypes.data_as(P),
                               err.ctypes.data_as(P), rho.ctypes.data_as(P), None, ctypes.byref(k), None, None, None)
    assert rc == -2 and k.value == -7 and b"exceeds" in L.rb_last_error()
    # the same columns fit with a shorter coefficient panel
    o = rbm.default_opts(anchor_max=16)
    assert L.rb_greedy_z_workspace(16, 40000, 16, ctypes.byref(o)) <= rbm.NOALLOC_SCRATCH_BYTES
