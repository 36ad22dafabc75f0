"""CPU FP64 oracle for the reduced-basis greedy (arXiv 1805.06124).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The product
library (``paper_1805_06124_amd``) never imports it, and it never imports the
product: the two share no code.  The only module both sides use is
``rb_inputs`` (seeded parameter generators, none of the method's arithmetic).

The arithmetic lives in ``rb_oracle.c`` (plain C99, FP64, compiled with gcc by
``oracle/build.py``); this module is argument marshalling through ctypes, plus
the FP64 MLP of ``oracle/mlp.py``.

Array conventions: a complex N x M snapshot matrix is passed as a C-contiguous
numpy ``complex128`` array of shape ``(M, N)`` (row j = column s_j), which is
exactly the column-major N x M layout the C code reads.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# RB_ORACLE_SANITIZE=1 selects a build with AddressSanitizer and
# UndefinedBehaviorSanitizer (the interpreter must then preload libasan and
# libubsan; see tests/test_oracle_sanitized.py)
SANITIZE = os.environ.get("RB_ORACLE_SANITIZE", "") == "1"
LIB_PATH = os.path.join(_HERE, "liboracle_san.so" if SANITIZE else "liboracle.so")
SRC_PATH = os.path.join(_HERE, "rb_oracle.c")

STATUS = {0: "OK", 1: "KMAX", 2: "RANK", -1: "EINVAL", -2: "ENOMEM", -4: "ENONFINITE", -6: "EREPLAY"}


def build(force: bool = False) -> str:
    """Compile rb_oracle.c with gcc into liboracle.so (OpenMP on)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-o", tmp, SRC_PATH, "-lm"]
        if SANITIZE:
            cmd[1:2] = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        L.oracle_sqnorm.restype = D
        L.oracle_sqnorm.argtypes = [P, I64]
        L.oracle_sqnorms.restype = None
        L.oracle_sqnorms.argtypes = [P, I64, I64, I64, P]
        L.oracle_chirp.restype = None
        L.oracle_chirp.argtypes = [P, I64, D, D, I64, P, I64]
        for name in ("oracle_greedy_explicit", "oracle_greedy_pythag"):
            f = getattr(L, name)
            f.restype = ctypes.c_int
            f.argtypes = [P, I64, I64, I64, D, I64, D, ctypes.c_int, P, I64,
                          P, P, P, P, P, P, P, P]
        L.oracle_greedy_resume.restype = ctypes.c_int
        L.oracle_greedy_resume.argtypes = [P, I64, I64, I64, D, I64, D, ctypes.c_int, P, I64, I64,
                                           P, P, P, P, P, P, P, P]
        L.oracle_project.restype = None
        L.oracle_project.argtypes = [P, I64, I64, I64, P, I64, I64, P, I64]
        L.oracle_residual_norms.restype = None
        L.oracle_residual_norms.argtypes = [P, I64, I64, I64, P, I64, I64, P]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_threads.restype = None
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _cmat(S) -> np.ndarray:
    S = np.ascontiguousarray(S, dtype=np.complex128)
    if S.ndim != 2:
        raise ValueError("snapshot matrix must be 2-D (M, N)")
    return S


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def sqnorm(x) -> float:
    """||x||^2 accumulated exactly and rounded once."""
    x = np.ascontiguousarray(x, dtype=np.complex128).ravel()
    return float(lib().oracle_sqnorm(_ptr(x), x.size))


def sqnorms(S) -> np.ndarray:
    S = _cmat(S)
    M, N = S.shape
    out = np.empty(M, dtype=np.float64)
    lib().oracle_sqnorms(_ptr(S), N, M, N, _ptr(out))
    return out


def chirp(params, N: int, flo: float, fhi: float) -> np.ndarray:
    """Unit-norm chirp snapshots, shape (M, N) complex128; params (M, 2) = (Mtot [M_sun], q)."""
    params = np.ascontiguousarray(params, dtype=np.float64).reshape(-1, 2)
    M = params.shape[0]
    out = np.empty((M, N), dtype=np.complex128)
    lib().oracle_chirp(_ptr(params), M, float(flo), float(fhi), int(N), _ptr(out), int(N))
    return out


def greedy(S, tol: float, kmax: int, mode: str = "explicit", force=None, kappa: float = 2.0,
           nu_max: int = 4, want_coeffs: bool = False, E0=None) -> dict:
    """Run the oracle greedy.

    mode "explicit": Alg. 2 form (residual matrix), the reference definition.
    mode "pythag"  : pivot search by the Eq. (6.3) update (the paper's code).
    force          : optional pivot sequence to replay (forced-pivot mode);
                     with E0 it lists the pivots of the new steps only.
    E0             : optional (k0, N) orthonormal basis to continue from
                     (explicit mode only); kmax counts all k vectors.
    Returns dict(E (k, N), piv (k - k0,), err (k - k0 + 1,), rho, nu,
    pick (k - k0, 2), C (k, M) or None, k, k0, status); err[i] is the
    greedy error with k0 + i vectors.
    """
    S = _cmat(S)
    M, N = S.shape
    k0 = 0
    if E0 is not None:
        if mode != "explicit":
            raise ValueError("a starting basis needs the explicit mode")
        E0 = _cmat(E0)
        if E0.shape[1] != N:
            raise ValueError("E0 and S row counts differ")
        k0 = E0.shape[0]
    kcap = max(0, min(int(kmax), N, k0 + M))
    if kcap < k0:
        raise ValueError("kmax is below the starting basis size")
    E = np.zeros((max(kcap, 1), N), dtype=np.complex128)
    if k0:
        E[:k0] = E0
    piv = np.full(max(kcap, 1), -1, dtype=np.int64)
    err = np.zeros(kcap + 1, dtype=np.float64)
    rho = np.zeros(max(kcap, 1), dtype=np.float64)
    nu = np.zeros(max(kcap, 1), dtype=np.int32)
    pick = np.zeros((max(kcap, 1), 2), dtype=np.float64)
    C = np.zeros((M, max(kcap, 1)), dtype=np.complex128) if want_coeffs else None
    kout = np.zeros(1, dtype=np.int64)
    if force is not None:
        force = np.ascontiguousarray(force, dtype=np.int64)
        nforce = force.size
    else:
        nforce = 0
    fp = _ptr(force) if force is not None else None
    if k0:
        st = lib().oracle_greedy_resume(_ptr(S), N, M, N, float(tol), int(kmax), float(kappa), int(nu_max),
                                        fp, nforce, k0, _ptr(E), _ptr(piv), _ptr(err), _ptr(rho), _ptr(nu),
                                        _ptr(pick), _ptr(C) if C is not None else None, _ptr(kout))
    else:
        fn = {"explicit": lib().oracle_greedy_explicit, "pythag": lib().oracle_greedy_pythag}[mode]
        st = fn(_ptr(S), N, M, N, float(tol), int(kmax), float(kappa), int(nu_max), fp, nforce,
                _ptr(E), _ptr(piv), _ptr(err), _ptr(rho), _ptr(nu), _ptr(pick),
                _ptr(C) if C is not None else None, _ptr(kout))
    if st < 0:
        raise RuntimeError("oracle greedy failed: %s" % STATUS.get(st, st))
    k = int(kout[0])
    return dict(E=E[:k].copy(), piv=piv[k0:k].copy(), err=err[k0:k + 1].copy(), rho=rho[k0:k].copy(),
                nu=nu[k0:k].copy(), pick=pick[k0:k].copy(),
                C=(C[:, :k].T.copy() if C is not None else None), k=k, k0=k0, status=STATUS[st])


def project(E, S) -> np.ndarray:
    """C = E^H S as an array of shape (k, M) (row i = coefficients on e_i)."""
    E = _cmat(E)
    S = _cmat(S)
    k, N = E.shape
    M = S.shape[0]
    if S.shape[1] != N:
        raise ValueError("E and S row counts differ")
    Ct = np.empty((M, max(k, 1)), dtype=np.complex128)
    lib().oracle_project(_ptr(E), N, k, N, _ptr(S), M, N, _ptr(Ct), max(k, 1))
    return Ct[:, :k].T.copy()


def residual_norms(E, S) -> np.ndarray:
    """||s_j - E E^H s_j||_2 for every column, computed explicitly."""
    E = _cmat(E) if len(E) else np.zeros((0, np.asarray(S).shape[1]), dtype=np.complex128)
    S = _cmat(S)
    k, N = E.shape
    M = S.shape[0]
    out = np.empty(M, dtype=np.float64)
    lib().oracle_residual_norms(_ptr(E) if k else None, N, k, N, _ptr(S), M, N, _ptr(out))
    return out


def enrich(E, V, tol: float, kmax: int, kappa: float = 2.0, nu_max: int = 4, force=None) -> dict:
    """Out-of-sample validation of the basis E (k0, N) on the columns V (Mv, N),
    then one enrichment (Sec. 6.1): the columns whose explicit residual is
    >= tol, in index order, continue the greedy from E.

    Residuals shrink as the basis grows, so after the enrichment every column
    of V, failing or not, is below tol (unless kmax stopped it first).

    Returns dict with:
    - resid: (Mv,), the residuals against E;
    - fail: indices into V;
    - E: (k, N);
    - piv: pivots as indices into V;
    - err, rho, nu;
    - k, k0, status.
    """
    E = _cmat(E)
    V = _cmat(V)
    r = residual_norms(E, V)
    fail = np.nonzero(r >= tol)[0]
    k0 = E.shape[0]
    if fail.size == 0:
        return dict(resid=r, fail=fail, E=E.copy(), piv=np.zeros(0, np.int64), err=np.zeros(0),
                    rho=np.zeros(0), nu=np.zeros(0, np.int32), k=k0, k0=k0, status="OK")
    f = None
    if force is not None:
        pos = {int(c): i for i, c in enumerate(fail)}
        f = np.array([pos[int(c)] for c in force], dtype=np.int64)
    g = greedy(V[fail], tol, kmax, kappa=kappa, nu_max=nu_max, E0=E, force=f)
    return dict(resid=r, fail=fail, E=g["E"], piv=fail[g["piv"]], err=g["err"], rho=g["rho"], nu=g["nu"],
                pick=g["pick"], k=g["k"], k0=k0, status=g["status"])
