"""MI355X (gfx950) reduced-basis greedy: Python binding of librb.so.

The arithmetic runs in the HIP library declared by ``include/rb.h``; this
module only marshals torch tensors (device memory, streams) into the C ABI
through ctypes.  There is no CPU fallback: ``load()`` raises if the library
or a GPU is missing.

Layout: a complex snapshot matrix S with N rows and M columns is a torch
tensor of shape (M, N) (row j = column s_j), complex128 or complex64, on the
GPU, with unit stride along N (the C side's column-major N x M, ld =
S.stride(0)).
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librb.so")

STATUS = {0: "OK", 1: "KMAX", 2: "RANK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENONFINITE",
          -5: "EBREAKDOWN", -6: "ENOCONV"}


class RBError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__("%s failed: %s (%d) %s" % (fn, STATUS.get(code, "?"), code, msg))
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_double), ("nu_max", ctypes.c_int32), ("nu_min", ctypes.c_int32),
                ("theta", ctypes.c_double), ("anchor_max", ctypes.c_int32), ("collect_stats", ctypes.c_int32),
                ("theta32", ctypes.c_double), ("regen_chunk", ctypes.c_int32), ("certify", ctypes.c_int32),
                ("step_ms", ctypes.c_void_p), ("fuse", ctypes.c_int32), ("lookahead", ctypes.c_int32),
                ("look_k", ctypes.c_int32), ("lookahead32", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("anchors", ctypes.c_int64), ("gs_passes", ctypes.c_int64),
                ("ms_sweep", ctypes.c_double), ("ms_gs", ctypes.c_double), ("ms_anchor", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("regen_anchors", ctypes.c_int64), ("misses", ctypes.c_int64),
                ("fused", ctypes.c_int64), ("ms_fused", ctypes.c_double), ("look_sweeps", ctypes.c_int64),
                ("look_steps", ctypes.c_int64), ("look_gs", ctypes.c_int64), ("ms_look", ctypes.c_double),
                ("ms_apply", ctypes.c_double), ("ms_look_sweep", ctypes.c_double),
                ("look_vectors", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ChirpCtx(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p), ("flo", ctypes.c_double), ("fhi", ctypes.c_double),
                ("N", ctypes.c_int64), ("table", ctypes.c_void_p)]


EXPORTS = ["rb_default_opts", "rb_strerror", "rb_last_error", "rb_colnorms_z", "rb_sweep_z", "rb_greedy_z",
           "rb_sweep_c", "rb_greedy_c", "rb_chirp_table", "rb_chirp_regen", "rb_project_z", "rb_chirp_fill",
           "rb_mlp_param_count", "rb_mlp_workspace_bytes", "rb_mlp_forward", "rb_mlp_loss", "rb_mlp_backward",
           "rb_mlp_adam", "rb_mlp_gather", "rb_coef_targets", "rb_coef_relerr", "rb_greedy_resume_z",
           "rb_residual_norms_z", "rb_enrich_z", "rb_reconstruct_z", "rb_reconstruct_z_workspace", "rb_eim_z",
           "rb_eim_errors_z",
           "rb_chirp_params", "rb_stream_read", "rb_greedy_z_workspace", "rb_greedy_c_workspace",
           "rb_greedy_z_noalloc", "rb_mlp_phase_features", "rb_mlp_train", "rb_mlp_train_workspace_bytes"]

_lib = None


def lib_path() -> str:
    return LIB_PATH


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load librb.so and declare the C signatures (no GPU work)."""
    if not os.path.exists(path):
        raise RuntimeError("librb.so not built (%s); run paper_1805_06124_amd.build.build()" % path)
    L = ctypes.CDLL(path)
    P, I64, D, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int32
    L.rb_default_opts.restype = None
    L.rb_default_opts.argtypes = [ctypes.POINTER(Opts)]
    L.rb_strerror.restype = ctypes.c_char_p
    L.rb_strerror.argtypes = [ctypes.c_int]
    L.rb_last_error.restype = ctypes.c_char_p
    L.rb_last_error.argtypes = []
    L.rb_colnorms_z.restype = ctypes.c_int
    L.rb_colnorms_z.argtypes = [P, I64, I64, I64, P, P]
    L.rb_sweep_z.restype = ctypes.c_int
    L.rb_sweep_z.argtypes = [P, I64, I64, I64, P, P, P, P, P, I64, ctypes.POINTER(D), ctypes.POINTER(I64), P]
    L.rb_greedy_z.restype = ctypes.c_int
    SZ = ctypes.c_size_t
    L.rb_greedy_z.argtypes = [P, I64, I64, I64, D, I64, P, I64, P, I64, P, P, P, P, ctypes.POINTER(I64), P, SZ,
                              ctypes.POINTER(Opts), ctypes.POINTER(Stats), P]
    L.rb_greedy_z_noalloc.restype = ctypes.c_int
    L.rb_greedy_z_noalloc.argtypes = [P, I64, I64, I64, D, I64, P, I64, P, I64, P, P, P, P, ctypes.POINTER(I64),
                                      ctypes.POINTER(Opts), ctypes.POINTER(Stats), P]
    L.rb_greedy_z_workspace.restype = SZ
    L.rb_greedy_z_workspace.argtypes = [I64, I64, I64, ctypes.POINTER(Opts)]
    L.rb_greedy_c_workspace.restype = SZ
    L.rb_greedy_c_workspace.argtypes = [I64, I64, I64, ctypes.POINTER(Opts)]
    L.rb_greedy_resume_z.restype = ctypes.c_int
    L.rb_greedy_resume_z.argtypes = [P, I64, I64, I64, D, I64, P, I64, P, I64, I64, P, P, P, P, ctypes.POINTER(I64),
                                     P, SZ, ctypes.POINTER(Opts), ctypes.POINTER(Stats), P]
    L.rb_residual_norms_z.restype = ctypes.c_int
    L.rb_residual_norms_z.argtypes = [P, I64, I64, I64, P, I64, I64, P, P]
    L.rb_enrich_z.restype = ctypes.c_int
    L.rb_enrich_z.argtypes = [P, P, I64, I64, I64, D, I64, P, I64, I64, P, P, P, P, ctypes.POINTER(I64), P, P, P,
                              ctypes.POINTER(Opts), ctypes.POINTER(Stats), P]
    L.rb_reconstruct_z.restype = ctypes.c_int
    L.rb_reconstruct_z.argtypes = [P, I64, I64, I64, P, I64, I64, D, P, I64, P, P, ctypes.POINTER(I64), P,
                                   ctypes.c_size_t, P]
    L.rb_reconstruct_z_workspace.restype = ctypes.c_size_t
    L.rb_reconstruct_z_workspace.argtypes = [I64, I64]
    L.rb_eim_z.restype = ctypes.c_int
    L.rb_eim_z.argtypes = [P, I64, I64, I64, P, P, P, P, ctypes.POINTER(I64), P]
    L.rb_eim_errors_z.restype = ctypes.c_int
    L.rb_eim_errors_z.argtypes = [P, I64, I64, I64, P, P, P, I64, I64, P, P]
    L.rb_chirp_params.restype = ctypes.c_int
    L.rb_chirp_params.argtypes = [ctypes.c_uint64, I64, I64, D, D, D, D, P, P]
    L.rb_stream_read.restype = ctypes.c_int
    L.rb_stream_read.argtypes = [P, ctypes.c_size_t, P, I64, P]
    L.rb_sweep_c.restype = ctypes.c_int
    L.rb_sweep_c.argtypes = [P, I64, I64, I64, P, P, P, P, P, I64, P, P, P]
    L.rb_greedy_c.restype = ctypes.c_int
    L.rb_greedy_c.argtypes = [P, I64, I64, I64, D, I64, P, P, P, I64, P, I64, P, P, P, P, ctypes.POINTER(I64), P,
                              SZ, ctypes.POINTER(Opts), ctypes.POINTER(Stats), P]
    L.rb_chirp_table.restype = ctypes.c_int
    L.rb_chirp_table.argtypes = [D, D, I64, P, P]
    L.rb_chirp_regen.restype = ctypes.c_int
    L.rb_chirp_regen.argtypes = [P, P, I64, P, I64, P]
    L.rb_project_z.restype = ctypes.c_int
    L.rb_project_z.argtypes = [P, I64, I64, I64, P, I64, I64, P, I64, P]
    L.rb_chirp_fill.restype = ctypes.c_int
    L.rb_chirp_fill.argtypes = [P, I64, D, D, I64, ctypes.c_int, P, I64, P]
    C_INT, F = ctypes.c_int, ctypes.c_float
    L.rb_mlp_param_count.restype = I64
    L.rb_mlp_param_count.argtypes = [C_INT, C_INT, C_INT]
    L.rb_mlp_workspace_bytes.restype = ctypes.c_size_t
    L.rb_mlp_workspace_bytes.argtypes = [I64, C_INT, C_INT, C_INT]
    L.rb_mlp_forward.restype = C_INT
    L.rb_mlp_forward.argtypes = [P, P, C_INT, C_INT, C_INT, P, I64, P, P, P]
    L.rb_mlp_loss.restype = C_INT
    L.rb_mlp_loss.argtypes = [P, P, I64, C_INT, P, P, P, C_INT, C_INT, P]
    L.rb_mlp_backward.restype = C_INT
    L.rb_mlp_backward.argtypes = [P, P, C_INT, C_INT, C_INT, P, I64, P, P, P, P]
    L.rb_mlp_adam.restype = C_INT
    L.rb_mlp_adam.argtypes = [P, P, P, P, P, I64, F, F, F, F, I64, P]
    L.rb_mlp_gather.restype = C_INT
    L.rb_mlp_gather.argtypes = [P, P, P, I64, C_INT, P, P, P, P]
    L.rb_mlp_phase_features.restype = C_INT
    L.rb_mlp_phase_features.argtypes = [P, P, P, I64, C_INT, P, P, I64, P, P, P, P]
    L.rb_mlp_train_workspace_bytes.restype = ctypes.c_size_t
    L.rb_mlp_train_workspace_bytes.argtypes = [I64, C_INT, C_INT, C_INT]
    L.rb_mlp_train.restype = C_INT
    L.rb_mlp_train.argtypes = [P, P, P, P, C_INT, C_INT, C_INT, P, P, P, I64, I64, I64, P, F, F, F, P, P, I64, P,
                               P, P, ctypes.c_size_t, P]
    L.rb_coef_targets.restype = C_INT
    L.rb_coef_targets.argtypes = [P, I64, I64, C_INT, P, P]
    L.rb_coef_relerr.restype = C_INT
    L.rb_coef_relerr.argtypes = [P, P, I64, I64, C_INT, P, P]
    return L


def load() -> ctypes.CDLL:
    """The library, loaded once; requires a GPU (no CPU fallback)."""
    global _lib
    if _lib is None:
        if not torch.cuda.is_available():
            raise RuntimeError("paper_1805_06124_amd needs a ROCm GPU; none is visible")
        _lib = load_library()
    return _lib


def _check(fn: str, rc: int, ok=(0,)):
    if rc not in ok:
        raise RBError(fn, rc, load().rb_last_error().decode())
    return rc


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _mat(S: torch.Tensor, dtype) -> tuple:
    if not S.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if S.dtype != dtype:
        raise TypeError("expected %s, got %s" % (dtype, S.dtype))
    if S.dim() != 2 or S.stride(1) != 1 or S.stride(0) < S.shape[1]:
        raise ValueError("expected a (M, N) tensor with unit stride along N")
    M, N = S.shape
    return M, N, S.stride(0)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def default_opts(**kw) -> Opts:
    o = Opts()
    load().rb_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k) or k == "step_ms":
            raise TypeError("unknown option %r" % k)
        setattr(o, k, v)
    return o


def workspace_bytes(N: int, M: int, kmax: int, mixed: bool = False, **opts) -> int:
    """Device workspace (bytes) of greedy (mixed=False) or greedy_c for these
    sizes and options (rb_greedy_z_workspace / rb_greedy_c_workspace)."""
    o = default_opts(**opts)
    f = load().rb_greedy_c_workspace if mixed else load().rb_greedy_z_workspace
    n = f(int(N), int(M), int(kmax), ctypes.byref(o))
    if n == 0:
        raise ValueError("invalid sizes or options")
    return int(n)


def workspace(N: int, M: int, kmax: int, mixed: bool = False, device="cuda", **opts) -> torch.Tensor:
    """A uint8 device tensor sized for greedy/greedy_c (pass it as ws=)."""
    return torch.empty(workspace_bytes(N, M, kmax, mixed, **opts), dtype=torch.uint8, device=device)


def _ws(ws):
    if ws is None:
        return None, 0
    if not ws.is_cuda or ws.dtype != torch.uint8 or not ws.is_contiguous():
        raise ValueError("ws must be a contiguous uint8 GPU tensor")
    return _ptr(ws), ws.numel()


def _trace(o: Opts, kcap: int, trace: bool):
    """Per-step timing buffer (3 doubles per basis position) hooked into the
    options when trace is set."""
    import numpy as np
    if not trace:
        return None
    buf = np.zeros(3 * (kcap + 1), dtype=np.float64)
    o.collect_stats = 1
    o.step_ms = buf.ctypes.data_as(ctypes.c_void_p).value
    return buf


def colnorms(S: torch.Tensor, stream=None) -> torch.Tensor:
    """Exact ||s_j||^2 for every column (double-double, rounded once)."""
    M, N, ld = _mat(S, torch.complex128)
    out = torch.empty(M, dtype=torch.float64, device=S.device)
    _check("rb_colnorms_z", load().rb_colnorms_z(_ptr(S), N, M, ld, _ptr(out), _stream(stream)))
    return out


def sweep(S: torch.Tensor, e: torch.Tensor, nrm: torch.Tensor, acc: torch.Tensor, mask: torch.Tensor | None = None,
          c_out: torch.Tensor | None = None, stream=None):
    """One fused Eq. (6.3) sweep; updates acc in place, writes c_j into c_out
    (complex128[M]) if given.  Returns (est_max, J)."""
    M, N, ld = _mat(S, torch.complex128)
    if e.dtype != torch.complex128 or e.numel() != N or not e.is_contiguous():
        raise ValueError("e must be a contiguous complex128 vector of length N")
    for t, n in ((nrm, "nrm"), (acc, "acc")):
        if t.dtype != torch.float64 or t.numel() != M or not t.is_contiguous():
            raise ValueError("%s must be contiguous float64[M]" % n)
    if mask is not None and (mask.dtype != torch.uint8 or mask.numel() != M):
        raise ValueError("mask must be uint8[M]")
    if c_out is not None and (c_out.dtype != torch.complex128 or c_out.numel() < M):
        raise ValueError("c_out must be complex128[M]")
    est = ctypes.c_double()
    J = ctypes.c_int64()
    _check("rb_sweep_z", load().rb_sweep_z(_ptr(S), N, M, ld, _ptr(e), _ptr(nrm), _ptr(acc), _ptr(mask),
                                           _ptr(c_out), 1, ctypes.byref(est), ctypes.byref(J), _stream(stream)))
    return est.value, J.value


def greedy(S: torch.Tensor, tol: float, kmax: int, W: torch.Tensor | None = None, stream=None,
           E0: torch.Tensor | None = None, ws: torch.Tensor | None = None, trace: bool = False,
           check: bool = True, **opts) -> dict:
    """RB-greedy (Alg. 3) over complex128 S.  W: optional (M, N) working matrix
    for re-anchoring (may be S itself: S is then overwritten).  E0: optional
    (k0, N) orthonormal basis to continue from (rb_greedy_resume_z); kmax
    then counts all vectors.  ws: optional workspace (workspace()); the call
    then allocates nothing (W required).  trace: per-step device times
    (step_ms, (k, 3): orthogonalisation, sweep, re-anchoring).  check=False
    returns error statuses in the dict instead of raising.  Returns dict
    with E (k, N) complex128 on the GPU, piv, err, rho, nu (numpy; the
    k - k0 new steps, err from k0 to k), k, k0, status and stats."""
    import numpy as np
    M, N, ld = _mat(S, torch.complex128)
    k0 = 0
    if E0 is not None:
        k0, N0, _ = _mat(E0, torch.complex128)
        if N0 != N:
            raise ValueError("E0 and S row counts differ")
    kcap = max(0, min(int(kmax), N, k0 + M))
    if kcap < k0:
        raise ValueError("kmax is below the starting basis size")
    E = torch.empty((max(kcap, 1), N), dtype=torch.complex128, device=S.device)
    if k0:
        E[:k0].copy_(E0)
    piv = np.zeros(max(kcap, 1), dtype=np.int64)
    err = np.zeros(kcap + 1, dtype=np.float64)
    rho = np.zeros(max(kcap, 1), dtype=np.float64)
    nu = np.zeros(max(kcap, 1), dtype=np.int32)
    kout = ctypes.c_int64(k0)
    o = default_opts(**opts)
    tr = _trace(o, kcap, trace)
    st = Stats()
    if W is not None:
        Mw, Nw, ldW = _mat(W, torch.complex128)
        if (Mw, Nw) != (M, N):
            raise ValueError("W must have the shape of S")
    else:
        ldW = N
    wp, wn = _ws(ws)
    hp = [a.ctypes.data_as(ctypes.c_void_p) for a in (piv, err, rho, nu)]
    ok = (0, 1, 2) if check else tuple(STATUS)
    if k0:
        rc = load().rb_greedy_resume_z(_ptr(S), N, M, ld, float(tol), int(kmax), _ptr(W), ldW, _ptr(E), N, k0,
                                       *hp, ctypes.byref(kout), wp, wn, ctypes.byref(o), ctypes.byref(st),
                                       _stream(stream))
        _check("rb_greedy_resume_z", rc, ok=ok)
    else:
        rc = load().rb_greedy_z(_ptr(S), N, M, ld, float(tol), int(kmax), _ptr(W), ldW, _ptr(E), N, *hp,
                                ctypes.byref(kout), wp, wn, ctypes.byref(o), ctypes.byref(st), _stream(stream))
        _check("rb_greedy_z", rc, ok=ok)
    k = kout.value
    out = dict(E=E[:k], piv=piv[k0:k].copy(), err=err[k0:k + 1].copy(), rho=rho[k0:k].copy(),
               nu=nu[k0:k].copy(), k=k, k0=k0, status=STATUS[rc], stats=st.as_dict())
    if tr is not None:
        out["step_ms"] = tr.reshape(-1, 3)[k0:k + 1].copy()
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20  # RB_NOALLOC_SCRATCH_BYTES


def greedy_noalloc(S: torch.Tensor, tol: float, kmax: int, W: torch.Tensor, E: torch.Tensor, stream=None,
                   **opts) -> dict:
    """rb_greedy_z_noalloc: the FP64 greedy with the library's fixed device
    workspace (no allocation inside the call).  W (working matrix, may be S)
    and E ((>= min(kmax, N, M), N) complex128 basis buffer) are the
    caller's.  Returns as greedy() (no timings)."""
    import numpy as np
    M, N, ld = _mat(S, torch.complex128)
    Mw, Nw, ldW = _mat(W, torch.complex128)
    kE, NE, ldE = _mat(E, torch.complex128)
    kcap = max(0, min(int(kmax), N, M))
    if (Mw, Nw) != (M, N) or NE != N or kE < max(kcap, 1):
        raise ValueError("W must have the shape of S and E room for min(kmax, N, M) vectors")
    piv = np.zeros(max(kcap, 1), dtype=np.int64)
    err = np.zeros(kcap + 1, dtype=np.float64)
    rho = np.zeros(max(kcap, 1), dtype=np.float64)
    nu = np.zeros(max(kcap, 1), dtype=np.int32)
    kout = ctypes.c_int64()
    o = default_opts(**opts)
    st = Stats()
    hp = [a.ctypes.data_as(ctypes.c_void_p) for a in (piv, err, rho, nu)]
    rc = load().rb_greedy_z_noalloc(_ptr(S), N, M, ld, float(tol), int(kmax), _ptr(W), ldW, _ptr(E), ldE, *hp,
                                    ctypes.byref(kout), ctypes.byref(o), ctypes.byref(st), _stream(stream))
    _check("rb_greedy_z_noalloc", rc, ok=(0, 1, 2))
    k = kout.value
    return dict(E=E[:k], piv=piv[:k].copy(), err=err[:k + 1].copy(), rho=rho[:k].copy(), nu=nu[:k].copy(), k=k,
                status=STATUS[rc], stats=st.as_dict())


def residual_norms(E: torch.Tensor, V: torch.Tensor, stream=None) -> torch.Tensor:
    """Out-of-sample validation: ||v_j - E E^H v_j||_2 for every row v_j of
    V (M, N) against the orthonormal rows of E (k, N); float64 (M,) on the GPU."""
    M, N, ldV = _mat(V, torch.complex128)
    if E is None or E.shape[0] == 0:
        k, ldE, Ep = 0, N, None
    else:
        k, NE, ldE = _mat(E, torch.complex128)
        if NE != N:
            raise ValueError("E and V row counts differ")
        Ep = _ptr(E)
    out = torch.empty(M, dtype=torch.float64, device=V.device)
    _check("rb_residual_norms_z", load().rb_residual_norms_z(Ep, N, k, ldE, _ptr(V), M, ldV, _ptr(out),
                                                             _stream(stream)))
    return out


def enrich(E: torch.Tensor, params: torch.Tensor, flo: float, fhi: float, tol: float, kmax: int, Mv: int,
           rounds: int = 1, want_resid: bool = False, stream=None, **opts) -> dict:
    """Validation and iterative enrichment of the basis E (k_in, N) on the
    chirp family with parameters `params` ((rounds * Mv, 2) float64 on the
    GPU): round r validates rows r*Mv .. r*Mv + Mv - 1 and continues the
    greedy on the failing ones.  Returns dict with E (k, N), piv (family
    indices of the added vectors), err (k_in .. k), rho, nu, n_fail,
    resid_max (per round), resid ((rounds*Mv,) on the GPU or None), k,
    k_in, status, stats."""
    import numpy as np
    k_in, N, _ = _mat(E, torch.complex128)
    if (not params.is_cuda or params.dtype != torch.float64 or params.numel() != 2 * Mv * rounds
            or not params.is_contiguous()):
        raise ValueError("params must be a contiguous float64 GPU tensor of shape (rounds * Mv, 2)")
    kcap = max(k_in, min(int(kmax), N))
    Eb = torch.empty((max(kcap, 1), N), dtype=torch.complex128, device=E.device)
    Eb[:k_in].copy_(E)
    piv = np.zeros(max(kcap, 1), dtype=np.int64)
    err = np.zeros(kcap + 1, dtype=np.float64)
    rho = np.zeros(max(kcap, 1), dtype=np.float64)
    nu = np.zeros(max(kcap, 1), dtype=np.int32)
    n_fail = np.zeros(rounds, dtype=np.int64)
    rmax = np.zeros(rounds, dtype=np.float64)
    resid = torch.empty(rounds * Mv, dtype=torch.float64, device=E.device) if want_resid else None
    kout = ctypes.c_int64()
    o = default_opts(**opts)
    st = Stats()
    L = load()
    table = torch.empty(3 * N, dtype=torch.float64, device=E.device)
    _check("rb_chirp_table", L.rb_chirp_table(float(flo), float(fhi), N, _ptr(table), _stream(stream)))
    ctx = ChirpCtx(params.data_ptr(), float(flo), float(fhi), N, table.data_ptr())
    fn = ctypes.cast(L.rb_chirp_regen, ctypes.c_void_p)
    hp = [a.ctypes.data_as(ctypes.c_void_p) for a in (piv, err, rho, nu)]
    rc = L.rb_enrich_z(fn, ctypes.cast(ctypes.pointer(ctx), ctypes.c_void_p), N, int(Mv), int(rounds), float(tol),
                       int(kmax), _ptr(Eb), N, k_in, *hp, ctypes.byref(kout), n_fail.ctypes.data_as(ctypes.c_void_p),
                       rmax.ctypes.data_as(ctypes.c_void_p), _ptr(resid), ctypes.byref(o), ctypes.byref(st),
                       _stream(stream))
    _check("rb_enrich_z", rc, ok=(0, 1, 2))
    k = kout.value
    return dict(E=Eb[:k], piv=piv[k_in:k].copy(), err=err[k_in:k + 1].copy(), rho=rho[k_in:k].copy(),
                nu=nu[k_in:k].copy(), n_fail=n_fail, resid_max=rmax, resid=resid, k=k, k_in=k_in,
                status=STATUS[rc], stats=st.as_dict())


def sweep_c(S32: torch.Tensor, e32: torch.Tensor, nrm: torch.Tensor, acc: torch.Tensor,
            mask: torch.Tensor | None = None, c_out: torch.Tensor | None = None, stream=None):
    """One mixed-precision sweep (complex64 S32, complex64 e32); updates acc in
    place, writes c_j (complex128) into c_out if given.  Returns the 8 best
    (est, J) as two numpy arrays (J = -1 for unused slots)."""
    import numpy as np
    M, N, ld = _mat(S32, torch.complex64)
    if e32.dtype != torch.complex64 or e32.numel() != N or not e32.is_contiguous():
        raise ValueError("e32 must be a contiguous complex64 vector of length N")
    for t, n in ((nrm, "nrm"), (acc, "acc")):
        if t.dtype != torch.float64 or t.numel() != M or not t.is_contiguous():
            raise ValueError("%s must be contiguous float64[M]" % n)
    if mask is not None and (mask.dtype != torch.uint8 or mask.numel() != M):
        raise ValueError("mask must be uint8[M]")
    if c_out is not None and (c_out.dtype != torch.complex128 or c_out.numel() < M):
        raise ValueError("c_out must be complex128[M]")
    est = np.zeros(8)
    J = np.zeros(8, dtype=np.int64)
    _check("rb_sweep_c", load().rb_sweep_c(_ptr(S32), N, M, ld, _ptr(e32), _ptr(nrm), _ptr(acc), _ptr(mask),
                                           _ptr(c_out), 1, est.ctypes.data_as(ctypes.c_void_p),
                                           J.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
    return est, J


def greedy_c(S32: torch.Tensor, tol: float, kmax: int, params: torch.Tensor, flo: float, fhi: float,
             W: torch.Tensor | None = None, stream=None, ws: torch.Tensor | None = None, trace: bool = False,
             check: bool = True, **opts) -> dict:
    """Mixed-precision RB-greedy over complex64 S32 (basis in FP64).  Columns
    are regenerated in FP64 by the built-in chirp regenerator from `params`
    ((M, 2) float64 on the GPU: Mtot in solar masses, q) on [flo, fhi].
    W: optional (M, N) complex64 working matrix (may be S32 itself).  ws,
    trace, check: as greedy (ws from workspace(..., mixed=True))."""
    import numpy as np
    M, N, ld = _mat(S32, torch.complex64)
    if not params.is_cuda or params.dtype != torch.float64 or params.numel() != 2 * M or not params.is_contiguous():
        raise ValueError("params must be a contiguous float64 GPU tensor of shape (M, 2)")
    kcap = max(0, min(int(kmax), N, M))
    E = torch.empty((max(kcap, 1), N), dtype=torch.complex128, device=S32.device)
    piv = np.zeros(max(kcap, 1), dtype=np.int64)
    err = np.zeros(kcap + 1, dtype=np.float64)
    rho = np.zeros(max(kcap, 1), dtype=np.float64)
    nu = np.zeros(max(kcap, 1), dtype=np.int32)
    kout = ctypes.c_int64()
    o = default_opts(**opts)
    tr = _trace(o, kcap, trace)
    st = Stats()
    if W is not None:
        Mw, Nw, ldW = _mat(W, torch.complex64)
        if (Mw, Nw) != (M, N):
            raise ValueError("W must have the shape of S32")
    else:
        ldW = N
    L = load()
    table = torch.empty(3 * N, dtype=torch.float64, device=S32.device)
    _check("rb_chirp_table", L.rb_chirp_table(float(flo), float(fhi), N, _ptr(table), _stream(stream)))
    ctx = ChirpCtx(params.data_ptr(), float(flo), float(fhi), N, table.data_ptr())
    fn = ctypes.cast(L.rb_chirp_regen, ctypes.c_void_p)
    rc = L.rb_greedy_c(_ptr(S32), N, M, ld, float(tol), int(kmax), fn, ctypes.cast(ctypes.pointer(ctx), ctypes.c_void_p),
                       _ptr(W), ldW, _ptr(E), N, piv.ctypes.data_as(ctypes.c_void_p),
                       err.ctypes.data_as(ctypes.c_void_p), rho.ctypes.data_as(ctypes.c_void_p),
                       nu.ctypes.data_as(ctypes.c_void_p), ctypes.byref(kout), *_ws(ws), ctypes.byref(o),
                       ctypes.byref(st), _stream(stream))
    _check("rb_greedy_c", rc, ok=(0, 1, 2) if check else tuple(STATUS))
    k = kout.value
    out = dict(E=E[:k], piv=piv[:k].copy(), err=err[:k + 1].copy(), rho=rho[:k].copy(), nu=nu[:k].copy(), k=k,
               status=STATUS[rc], stats=st.as_dict())
    if tr is not None:
        out["step_ms"] = tr.reshape(-1, 3)[:k + 1].copy()
    return out


def project(E: torch.Tensor, S: torch.Tensor, stream=None) -> torch.Tensor:
    """C = E^H S on FP64 matrix cores.  E: (k, N), S: (M, N) complex128.
    Returns a (M, k) tensor whose row j holds the coefficients of s_j."""
    k, N, ldE = _mat(E, torch.complex128)
    M, N2, ldS = _mat(S, torch.complex128)
    if N != N2:
        raise ValueError("E and S row counts differ")
    C = torch.empty((M, k), dtype=torch.complex128, device=S.device)
    _check("rb_project_z", load().rb_project_z(_ptr(E), N, k, ldE, _ptr(S), M, ldS, _ptr(C), k, _stream(stream)))
    return C


def reconstruct_workspace_bytes(j: int, M: int) -> int:
    """Device workspace bytes of reconstruct() for j basis vectors and M
    coefficient columns (0 if the sizes are rejected)."""
    return int(load().rb_reconstruct_z_workspace(int(j), int(M)))


def reconstruct(E: torch.Tensor, C: torch.Tensor, tau2: float, want_v: bool = False, stream=None,
                ws: torch.Tensor | None = None) -> dict:
    """Alg. 4 from the greedy basis E (j, N) and its coefficients C = E^H S
    as returned by project() ((M, j): row m holds the coefficients of s_m).
    ws: optional uint8 GPU workspace of reconstruct_workspace_bytes(j, M)
    bytes; by default one is taken from torch's allocator (so repeated calls
    reuse its cached memory).  Returns dict with X ((k, N) complex128 on the
    GPU, row i = x_{i+1}), sigma (numpy (j,), non-increasing), k, and V
    ((j, j) on the GPU, column i = left singular vector i of C) if want_v."""
    import numpy as np
    j, N, ldE = _mat(E, torch.complex128)
    M, j2, ldC = _mat(C, torch.complex128)
    if j2 != j:
        raise ValueError("C must have one coefficient per basis vector")
    X = torch.empty((j, N), dtype=torch.complex128, device=E.device)
    V = torch.empty((j, j), dtype=torch.complex128, device=E.device) if want_v else None
    if ws is None:
        nbytes = reconstruct_workspace_bytes(j, M)
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=E.device)
    ptr, nws = _ws(ws)
    sigma = np.zeros(j)
    kout = ctypes.c_int64()
    _check("rb_reconstruct_z", load().rb_reconstruct_z(_ptr(E), N, j, ldE, _ptr(C), M, ldC, float(tau2), _ptr(X),
                                                       N, sigma.ctypes.data_as(ctypes.c_void_p), _ptr(V),
                                                       ctypes.byref(kout), ptr, nws, _stream(stream)))
    k = kout.value
    # V was written column-major j x j: the tensor's row i is column i
    return dict(X=X[:k], sigma=sigma, k=k, V=(V.T if V is not None else None))


def eim(E: torch.Tensor, stream=None) -> dict:
    """Empirical-interpolation nodes of the basis E (k, N).  Returns dict
    with nodes (numpy int64 (k,)), peak (numpy (k,), |r_j(p_j)|), R ((k, N)
    on the GPU: row j = r_j / r_j(p_j)), Tinv ((k, k) on the GPU, matrix
    form) and the interpolant's pieces for eim_errors, k, status."""
    import numpy as np
    k, N, ldE = _mat(E, torch.complex128)
    nodes = np.zeros(k, dtype=np.int64)
    peak = np.zeros(k)
    R = torch.empty((k, N), dtype=torch.complex128, device=E.device)
    Tcm = torch.empty((k, k), dtype=torch.complex128, device=E.device)  # column-major k x k
    kout = ctypes.c_int64()
    rc = load().rb_eim_z(_ptr(E), N, k, ldE, nodes.ctypes.data_as(ctypes.c_void_p),
                         peak.ctypes.data_as(ctypes.c_void_p), _ptr(R), _ptr(Tcm), ctypes.byref(kout),
                         _stream(stream))
    _check("rb_eim_z", rc, ok=(0, 2))
    return dict(nodes=nodes, peak=peak, R=R, Tinv=Tcm.T, _Tcm=Tcm, k=kout.value, status=STATUS[rc])


def eim_errors(ei: dict, V: torch.Tensor, stream=None) -> torch.Tensor:
    """||v - I[v]||_2 for every row v of V (M, N), with the interpolant of
    eim() (ei); float64 (M,) on the GPU."""
    R, Tcm = ei["R"], ei["_Tcm"]
    k, N, ldR = _mat(R, torch.complex128)
    M, N2, ldV = _mat(V, torch.complex128)
    if N2 != N:
        raise ValueError("V and the basis row counts differ")
    nodes = torch.from_numpy(ei["nodes"]).to(V.device)
    out = torch.empty(M, dtype=torch.float64, device=V.device)
    _check("rb_eim_errors_z", load().rb_eim_errors_z(_ptr(R), N, k, ldR, _ptr(Tcm), _ptr(nodes), _ptr(V), M, ldV,
                                                     _ptr(out), _stream(stream)))
    return out


def chirp_params(seed: int, M: int, mlo: float, mhi: float, qlo: float, qhi: float, start: int = 0,
                 device="cuda", stream=None) -> torch.Tensor:
    """(M, 2) float64 GPU tensor of chirp parameters (Mtot, q) for columns
    start .. start + M - 1 from the seed (SplitMix64 counters)."""
    out = torch.empty((M, 2), dtype=torch.float64, device=device)
    _check("rb_chirp_params", load().rb_chirp_params(int(seed) & (2 ** 64 - 1), int(start), int(M), float(mlo),
                                                     float(mhi), float(qlo), float(qhi), _ptr(out),
                                                     _stream(stream)))
    return out


def stream_read(t: torch.Tensor, partial: torch.Tensor, stream=None) -> None:
    """Read the whole of tensor t once (plain streaming read, partial sums
    into the float64 tensor `partial`, one per workgroup)."""
    if not t.is_cuda or not t.is_contiguous() or partial.dtype != torch.float64 or not partial.is_cuda:
        raise ValueError("stream_read needs a contiguous GPU tensor and a float64 GPU partial buffer")
    nbytes = t.numel() * t.element_size()
    _check("rb_stream_read", load().rb_stream_read(_ptr(t), nbytes - nbytes % 16, _ptr(partial), partial.numel(),
                                                   _stream(stream)))


def chirp_fill(params: torch.Tensor, N: int, flo: float, fhi: float, dtype=torch.complex128,
               out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Unit-norm chirp snapshots on the GPU; params (M, 2) float64 (Mtot in
    solar masses, q) on the GPU.  Returns (M, N) complex128 or complex64."""
    if not params.is_cuda or params.dtype != torch.float64 or not params.is_contiguous():
        raise ValueError("params must be a contiguous float64 GPU tensor of shape (M, 2)")
    M = params.numel() // 2
    code = {torch.complex128: 0, torch.complex64: 1}[dtype]
    if out is None:
        out = torch.empty((M, N), dtype=dtype, device=params.device)
    Mo, No, ld = _mat(out, dtype)
    if (Mo, No) != (M, N):
        raise ValueError("out has the wrong shape")
    _check("rb_chirp_fill", load().rb_chirp_fill(_ptr(params), M, float(flo), float(fhi), int(N), code, _ptr(out),
                                                 ld, _stream(stream)))
    return out
