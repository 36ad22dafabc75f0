"""Learned coefficient surrogate on the GPU: an MLP from the snapshot
parameters to [Re c; Im c], the projection coefficients c = E^H s of a
snapshot on the greedy basis, trained on the method's own output (the
projection of the training snapshots) with the library's BF16 matrix-core
forward/backward kernels and Adam.  The plain projection of the regenerated
snapshot checks each prediction and replaces it when its relative error
exceeds a threshold.

Inputs: either the mapped parameters (Mtot, q) alone, or those plus the
snapshot's phase factors at the empirical-interpolation nodes of the basis
(phase_features()).  On the chirp family the coefficients oscillate far too
fast in (Mtot, q) for a network to follow from the parameters alone, while
they are a linear map of the phase factors at the nodes (every snapshot has
the same amplitude there).

Everything numeric runs in librb.so (rb_mlp_*, rb_coef_*, rb_chirp_fill,
rb_project_z); this module allocates device buffers and sequences the calls.
"""
from __future__ import annotations

import ctypes
import math
import time

import numpy as np
import torch

from . import _check, _ptr, _stream, load, chirp_fill, project


def phase_features(E: torch.Tensor, flo: float, fhi: float) -> dict:
    """Inputs that carry the snapshot phase: the empirical-interpolation
    nodes of the basis E (k, N) (rb_eim_z) and the chirp row table of the
    grid.  din = 2 + 2k."""
    from . import eim
    ei = eim(E)
    N = E.shape[1]
    table = torch.empty(3 * N, dtype=torch.float64, device=E.device)
    _check("rb_chirp_table", load().rb_chirp_table(float(flo), float(fhi), N, _ptr(table), _stream()))
    rows = torch.from_numpy(np.ascontiguousarray(ei["nodes"][:ei["k"]], dtype=np.int64)).to(E.device)
    return {"rows": rows, "table": table, "din": 2 + 2 * int(rows.numel())}


class Surrogate:
    def __init__(self, k: int, init: np.ndarray, ranges, hidden: int = 256, batch: int = 4096, din: int = 2,
                 device="cuda", features: dict | None = None):
        """features: None (inputs = mapped (Mtot, q), din = 2) or the dict of
        phase_features() (din = 2 + 2 * number of nodes)."""
        L = load()
        self.features = features
        if features is not None:
            din = features["din"]
        self.din, self.hidden, self.dout, self.batch = din, hidden, 2 * k, batch
        self.k = k
        n = L.rb_mlp_param_count(din, hidden, self.dout)
        if n <= 0 or init.size != n:
            raise ValueError("initial parameter vector has the wrong length")
        self.n = n
        self.dev = torch.device(device)
        self.p32 = torch.from_numpy(np.ascontiguousarray(init, dtype=np.float32)).to(self.dev)
        self.p16 = torch.zeros(n, dtype=torch.int16, device=self.dev)
        self.grad = torch.zeros(n, dtype=torch.float32, device=self.dev)
        self.m = torch.zeros(n, dtype=torch.float32, device=self.dev)
        self.v = torch.zeros(n, dtype=torch.float32, device=self.dev)
        self.ranges = (ctypes.c_double * 4)(*[float(x) for x in ranges])
        self._ws = {}
        self.step = 0
        # BF16 copy of the initial weights: one Adam step with lr 0 and zero
        # gradient leaves p32 unchanged and writes p16
        _check("rb_mlp_adam", L.rb_mlp_adam(_ptr(self.p32), _ptr(self.p16), _ptr(self.grad), _ptr(self.m),
                                            _ptr(self.v), n, 0.0, 0.9, 0.999, 1e-8, 1, _stream()))

    def workspace(self, batch: int) -> torch.Tensor:
        if batch not in self._ws:
            nb = load().rb_mlp_workspace_bytes(batch, self.din, self.hidden, self.dout)
            self._ws[batch] = torch.empty(nb, dtype=torch.uint8, device=self.dev)
        return self._ws[batch]

    # -- primitives -------------------------------------------------------
    def forward(self, X: torch.Tensor, Y: torch.Tensor | None = None) -> torch.Tensor:
        B = X.shape[0]
        if Y is None:
            Y = torch.empty((B, self.dout), dtype=torch.float32, device=self.dev)
        _check("rb_mlp_forward", load().rb_mlp_forward(_ptr(self.p32), _ptr(self.p16), self.din, self.hidden,
                                                       self.dout, _ptr(X), B, _ptr(Y), _ptr(self.workspace(B)),
                                                       _stream()))
        return Y

    def loss_backward(self, X: torch.Tensor, Y: torch.Tensor, T: torch.Tensor, loss: torch.Tensor):
        B = X.shape[0]
        ws = self.workspace(B)
        L = load()
        _check("rb_mlp_loss", L.rb_mlp_loss(_ptr(Y), _ptr(T), B, self.dout, None, _ptr(loss), _ptr(ws), self.din,
                                            self.hidden, _stream()))
        _check("rb_mlp_backward", L.rb_mlp_backward(_ptr(self.p32), _ptr(self.p16), self.din, self.hidden,
                                                    self.dout, _ptr(X), B, None, _ptr(self.grad), _ptr(ws),
                                                    _stream()))

    def adam(self, lr: float, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        _check("rb_mlp_adam", load().rb_mlp_adam(_ptr(self.p32), _ptr(self.p16), _ptr(self.grad), _ptr(self.m),
                                                 _ptr(self.v), self.n, lr, b1, b2, eps, self.step, _stream()))

    def gather(self, params: torch.Tensor, targets: torch.Tensor | None, idx: torch.Tensor, X, T):
        if self.features is not None:
            f = self.features
            _check("rb_mlp_phase_features", load().rb_mlp_phase_features(
                _ptr(params), _ptr(targets), _ptr(idx), idx.numel(), self.dout, self.ranges, _ptr(f["rows"]),
                f["rows"].numel(), _ptr(f["table"]), _ptr(X), _ptr(T), _stream()))
            return
        _check("rb_mlp_gather", load().rb_mlp_gather(_ptr(params), _ptr(targets), _ptr(idx), idx.numel(),
                                                     self.dout, self.ranges, _ptr(X), _ptr(T), _stream()))

    # -- training -----------------------------------------------------------
    def train_steps(self, params: torch.Tensor, targets: torch.Tensor, idx: torch.Tensor, lr, loss=None):
        """len(lr) Adam steps in one rb_mlp_train call: step s on the samples
        idx[s] (device int64 (steps, batch)) with learning rate lr[s]; loss
        (device float32 (steps,), optional) receives each step's loss."""
        steps, B = idx.shape
        lr = np.ascontiguousarray(lr, dtype=np.float32)
        assert lr.shape == (steps,) and idx.is_contiguous()
        L = load()
        key = ("train", B)
        if key not in self._ws:
            nb = L.rb_mlp_train_workspace_bytes(B, self.din, self.hidden, self.dout)
            self._ws[key] = torch.empty(nb, dtype=torch.uint8, device=self.dev)
        ws = self._ws[key]
        f = self.features
        _check("rb_mlp_train", L.rb_mlp_train(
            _ptr(self.p32), _ptr(self.p16), _ptr(self.m), _ptr(self.v), self.din, self.hidden, self.dout,
            _ptr(params), _ptr(targets), _ptr(idx), B, steps, self.step, lr.ctypes.data_as(ctypes.c_void_p),
            0.9, 0.999, 1e-8, self.ranges, _ptr(f["rows"]) if f is not None else None,
            f["rows"].numel() if f is not None else 0, _ptr(f["table"]) if f is not None else None,
            _ptr(loss), _ptr(ws), ws.numel(), _stream()))
        self.step += steps

    def train(self, params: torch.Tensor, targets: torch.Tensor, steps: int, index_fn, lr0: float = 1e-3,
              log_every: int = 0, log=None) -> list:
        """Adam with cosine-decayed learning rate.  index_fn(start, count)
        returns a (count, batch) int64 numpy array of sample indices.

        The steps run in chunks of 500 (one rb_mlp_train call each).  The
        host draws the next chunk's indices and reads the previous chunk's
        losses while the device trains on the current one: indices go up and
        losses come back through pinned double buffers, so the stream never
        waits for the host."""
        hist = []
        chunk = 500
        starts = list(range(0, steps, chunk))
        counts = [min(chunk, steps - s) for s in starts]
        B = self.batch
        h_idx = [torch.empty((chunk, B), dtype=torch.int64, pin_memory=True) for _ in range(2)]
        d_idx = [torch.empty((chunk, B), dtype=torch.int64, device=self.dev) for _ in range(2)]
        d_loss = [torch.zeros(chunk, dtype=torch.float32, device=self.dev) for _ in range(2)]
        h_loss = [torch.zeros(chunk, dtype=torch.float32, pin_memory=True) for _ in range(2)]
        ev_idx = [torch.cuda.Event() for _ in range(2)]
        ev_loss = [torch.cuda.Event() for _ in range(2)]
        for e in ev_idx:
            e.record()

        def logged(i):
            s = starts[i]
            return [j for j in range(counts[i]) if log_every and ((s + j) % log_every == 0 or s + j == steps - 1)]

        def fill(i):
            b = i % 2
            a = index_fn(starts[i], counts[i])
            assert a.shape == (counts[i], B), "index_fn must return (count, batch) indices"
            ev_idx[b].synchronize()  # the upload that last read this buffer has ended
            h_idx[b].numpy()[:counts[i]] = a

        def drain(i):
            b = i % 2
            js = logged(i)
            if not js:
                return
            ev_loss[b].synchronize()
            lv = h_loss[b].numpy()
            for j in js:
                hist.append((starts[i] + j, float(lv[j])))
                if log:
                    log("surrogate step %d loss %.3e" % (starts[i] + j, float(lv[j])))

        if starts:
            fill(0)
        for i, (s, c) in enumerate(zip(starts, counts)):
            b = i % 2
            d_idx[b][:c].copy_(h_idx[b][:c], non_blocking=True)
            ev_idx[b].record()
            lr = 0.5 * lr0 * (1.0 + np.cos(np.pi * (s + np.arange(c)) / steps))
            self.train_steps(params, targets, d_idx[b][:c], lr, d_loss[b])
            if logged(i):
                h_loss[b][:c].copy_(d_loss[b][:c], non_blocking=True)
                ev_loss[b].record()
            if i + 1 < len(starts):
                fill(i + 1)
            if i >= 1:
                drain(i - 1)
        if starts:
            drain(len(starts) - 1)
        return hist

    def predict(self, params: torch.Tensor, chunk: int = 65536) -> torch.Tensor:
        """FP32 [Re c; Im c] for every parameter row."""
        M = params.shape[0]
        out = torch.empty((M, self.dout), dtype=torch.float32, device=self.dev)
        for c0 in range(0, M, chunk):
            mc = min(chunk, M - c0)
            idx = torch.arange(c0, c0 + mc, dtype=torch.int64, device=self.dev)
            X = torch.empty((mc, self.din), dtype=torch.float32, device=self.dev)
            self.gather(params, None, idx, X, None)
            self.forward(X, out[c0:c0 + mc])
        return out


def coef_targets(C: torch.Tensor) -> torch.Tensor:
    """(M, k) complex128 coefficients -> (M, 2k) FP32 [Re; Im] targets."""
    M, k = C.shape
    T = torch.empty((M, 2 * k), dtype=torch.float32, device=C.device)
    _check("rb_coef_targets", load().rb_coef_targets(_ptr(C), C.stride(0), M, k, _ptr(T), _stream()))
    return T


def coef_relerr(Yh: torch.Tensor, C: torch.Tensor) -> torch.Tensor:
    M, k = C.shape
    out = torch.empty(M, dtype=torch.float64, device=C.device)
    _check("rb_coef_relerr", load().rb_coef_relerr(_ptr(Yh), _ptr(C), C.stride(0), M, k, _ptr(out), _stream()))
    return out


def evaluate(sur: Surrogate, E: torch.Tensor, params: torch.Tensor, N: int, flo: float, fhi: float,
             chunk: int = 16384, thresholds=(1e-2, 1e-3, 1e-4, 1e-5, 1e-6)) -> dict:
    """Held-out evaluation: per chunk, regenerate the snapshots (FP64), project
    them on E (the reference), predict with the surrogate, and compare.  Returns
    the error distribution, fallback rates and both throughputs."""
    M = params.shape[0]
    errs = torch.empty(M, dtype=torch.float64, device=params.device)
    t_proj = 0.0
    t_sur = 0.0
    # warm both paths at the chunk size (buffer allocation is not timed)
    p = params[:min(chunk, M)].contiguous()
    sur.predict(p)
    project(E, chirp_fill(p, N, flo, fhi))
    for c0 in range(0, M, chunk):
        mc = min(chunk, M - c0)
        p = params[c0:c0 + mc].contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S = chirp_fill(p, N, flo, fhi)
        C = project(E, S)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        Yh = sur.predict(p)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        errs[c0:c0 + mc] = coef_relerr(Yh, C)
        t_proj += t1 - t0
        t_sur += t2 - t1
        del S, C, Yh
    e = errs.cpu().numpy()
    sur_rate, proj_rate = M / t_sur, M / t_proj
    fb = {("%.0e" % t): float(np.mean(e > t)) for t in thresholds}
    # every sample is predicted; those above the threshold are also
    # regenerated and projected: time per sample 1/sur + f/proj
    eff = {key: 1.0 / (1.0 / sur_rate + f / proj_rate) for key, f in fb.items()}
    return {
        "n": int(M),
        "relerr_median": float(np.median(e)), "relerr_p90": float(np.percentile(e, 90)),
        "relerr_max": float(e.max()), "relerr_min": float(e.min()),
        "fallback_rate": fb,
        "surrogate_evals_per_s": sur_rate, "projections_per_s": proj_rate,
        "effective_evals_per_s": eff,
        "effective_gain": {key: v / proj_rate for key, v in eff.items()},
        "errors": e,
    }
