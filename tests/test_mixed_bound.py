"""The rounding bound behind the mixed greedy's certification (the
complex64 sweep's coefficients), checked against an emulation of the
sweep's own FP32 summation: per lane and 512-row tile, the 8 complex
values of rows base + 128 u + 2 lane + p (u < 4, p < 2) are summed in
FP32 in that order with the FP32 copy of the basis vector, the tile sums
added in FP64, the tail rows (lane + 64 t) summed in FP32 likewise.

Bounds (u32 = 2^-24, ||e|| = 1):
  |c~ - c| <= 25 u32 ||x||                       (one coefficient)
  | sum |c~_i|^2 - sum |c_i|^2 | <= 51 sqrt(m) u32 ||x||^2   (m of them)
Inputs include columns phase-aligned with e, so that every partial sum
grows in one direction."""
import numpy as np


U32 = 2.0 ** -24
F32 = np.float32


def _sweep32(e64, x32):
    """c~ = e^H x as the complex64 sweep forms it (no fused multiply-add:
    every product and sum rounded, one of the orders the bound covers)."""
    e32 = e64.astype(np.complex64)
    ex, ey = e32.real.astype(F32), e32.imag.astype(F32)
    sx, sy = x32.real.astype(F32), x32.imag.astype(F32)
    pr = (ex * sx).astype(F32) + (ey * sy).astype(F32)
    pi = (ex * sy).astype(F32) - (ey * sx).astype(F32)
    N = x32.size
    nfull = (N // 512) * 512
    tot = 0.0 + 0.0j
    for part in (pr, pi):
        # row t*512 + 128 u + 2 l + p -> (tile, lane, 8 values in (u, p) order)
        v = part[:nfull].reshape(-1, 4, 64, 2).transpose(0, 2, 1, 3).reshape(-1, 64, 8)
        acc = np.zeros(v.shape[:2], dtype=F32)
        for q in range(8):
            acc = (acc + v[:, :, q]).astype(F32)
        lane = acc.astype(np.float64).sum(axis=0)
        tail = part[nfull:]
        tacc = np.zeros(64, dtype=F32)
        for t0 in range(0, tail.size, 64):
            blk = np.zeros(64, dtype=F32)
            blk[:min(64, tail.size - t0)] = tail[t0:t0 + 64]
            tacc = (tacc + blk).astype(F32)
        s = float(lane.sum() + tacc.astype(np.float64).sum())
        tot = tot + (s if part is pr else 1j * s)
    return tot


def _unit(rng, N):
    v = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    return v / np.linalg.norm(v)


def test_coefficient_bound():
    rng = np.random.default_rng(101)
    for N in (10000, 1000, 777):
        for trial in range(6):
            e = _unit(rng, N)
            if trial % 2 == 0:
                x = (rng.standard_normal(N) + 1j * rng.standard_normal(N)) * (10.0 ** rng.uniform(-3, 3))
            else:  # phase-aligned with e: every term of e^H x positive
                x = np.abs(rng.standard_normal(N)) * np.exp(1j * np.angle(e)) * 1e2
            x32 = x.astype(np.complex64)
            x64 = x32.astype(np.complex128)  # the stored column is the reference
            c = np.vdot(e, x64)
            got = _sweep32(e, x32)
            assert abs(got - c) <= 25 * U32 * np.linalg.norm(x64), (N, trial, abs(got - c) / np.linalg.norm(x64) / U32)


def test_accumulated_estimate_bound():
    rng = np.random.default_rng(102)
    N, m = 4096, 24
    Q, _ = np.linalg.qr(rng.standard_normal((N, m)) + 1j * rng.standard_normal((N, m)))
    for trial in range(3):
        x = Q @ (rng.standard_normal(m) + 1j * rng.standard_normal(m)) + 1e-3 * _unit(rng, N)
        x32 = x.astype(np.complex64)
        x64 = x32.astype(np.complex128)
        exact = sum(abs(np.vdot(Q[:, i], x64)) ** 2 for i in range(m))
        approx = sum(abs(_sweep32(Q[:, i], x32)) ** 2 for i in range(m))
        assert abs(approx - exact) <= 51 * np.sqrt(m) * U32 * np.linalg.norm(x64) ** 2
