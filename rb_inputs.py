"""Seeded synthetic inputs shared by the product's tests/benchmark and the oracle.

This module generates *inputs only* and holds none of the greedy's arithmetic:
chirp-family parameter draws (SplitMix64 counters), the workload definitions
(matrix shapes, frequency bands, parameter ranges, tolerances) and a few
structured test matrices (Gaussian, low-rank products, Kahan, diagonal).

Workloads stand in for the paper's IMRPhenomPv2 snapshot matrices (Sec. 6.1.1,
N = 10,000 rows): each column is a leading-1PN frequency-domain chirp at
parameters (Mtot, q) drawn here; the waveform itself is evaluated by each side
on its own (the oracle in C, the product on the GPU).

SplitMix64 (Steele, Lea & Flood 2014): for counter i the state is
seed + (i + 1) * 0x9E3779B97F4A7C15 (mod 2^64), followed by the published
finaliser (xor-shift 30, multiply 0xBF58476D1CE4E5B9, xor-shift 27, multiply
0x94D049BB133111EB, xor-shift 31).  A uniform double in [0, 1) is
(z >> 11) * 2^-53.  Column j takes Mtot from counter 2j and q from 2j + 1.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """SplitMix64 outputs for the given counters (uint64 array)."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (c + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, counters: np.ndarray) -> np.ndarray:
    z = splitmix64(seed, counters)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def chirp_params(seed: int, M: int, mlo: float, mhi: float, qlo: float, qhi: float,
                 start: int = 0) -> np.ndarray:
    """(M, 2) float64 array of (total mass in solar masses, mass ratio q) for
    columns start .. start+M-1."""
    j = np.arange(start, start + M, dtype=np.uint64)
    u_m = uniform01(seed, 2 * j)
    u_q = uniform01(seed, 2 * j + np.uint64(1))
    out = np.empty((M, 2), dtype=np.float64)
    out[:, 0] = mlo + (mhi - mlo) * u_m
    out[:, 1] = qlo + (qhi - qlo) * u_q
    return out


@dataclass(frozen=True)
class Workload:
    name: str
    N: int            # rows (frequency samples)
    M: int            # columns (snapshots)
    flo: float        # Hz
    fhi: float        # Hz
    mlo: float        # total mass range, solar masses
    mhi: float
    qlo: float        # mass-ratio range
    qhi: float
    tol: float
    kmax: int
    dtype: str        # "c128" or "c64" storage
    seed: int = 1805

    def params(self, M: int | None = None, start: int = 0, seed: int | None = None) -> np.ndarray:
        return chirp_params(self.seed if seed is None else seed, self.M if M is None else M,
                            self.mlo, self.mhi, self.qlo, self.qhi, start=start)

    @property
    def bytes_per_elem(self) -> int:
        return 16 if self.dtype == "c128" else 8


# Snapshot families (the small case the oracle finishes in seconds, one GPU's
# share of the paper's largest matrix, its complex64 form, the larger complex64
# family, and a family for held-out surrogate evaluation).
WORKLOADS = {
    "chirp_small_c128": Workload("chirp_small_c128", 1000, 2000, 20.0, 512.0, 40.0, 60.0, 1.0, 4.0,
                                 1e-10, 200, "c128"),
    "chirp_10k_409600_c128": Workload("chirp_10k_409600_c128", 10000, 409600, 20.0, 1024.0, 20.0, 60.0,
                                      1.0, 4.0, 1e-10, 1500, "c128"),
    "chirp_10k_409600_c64": Workload("chirp_10k_409600_c64", 10000, 409600, 20.0, 1024.0, 20.0, 60.0,
                                     1.0, 4.0, 1e-10, 1500, "c64"),
    "chirp_10k_1638400_c64": Workload("chirp_10k_1638400_c64", 10000, 1638400, 20.0, 1024.0, 20.0, 80.0,
                                      1.0, 8.0, 1e-10, 3000, "c64"),
}
HELDOUT_SEED = 1806


# ---------------------------------------------------------------------------
# Structured test matrices; all returned as (M, N) complex128 arrays whose row
# j is snapshot column s_j (column-major N x M).
# ---------------------------------------------------------------------------

def gaussian(seed: int, N: int, M: int, real: bool = False) -> np.ndarray:
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((M, N))
    if not real:
        A = A + 1j * rng.standard_normal((M, N))
    return np.ascontiguousarray(A, dtype=np.complex128)


def low_rank(seed: int, N: int, M: int, rank: int) -> np.ndarray:
    """S = A B with A (N x rank) and B (rank x M) complex Gaussian."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((N, rank)) + 1j * rng.standard_normal((N, rank))
    B = rng.standard_normal((rank, M)) + 1j * rng.standard_normal((rank, M))
    return np.ascontiguousarray((A @ B).T, dtype=np.complex128)


def graded(seed: int, N: int, M: int, decay: float) -> np.ndarray:
    """Gaussian columns scaled by decay**j (a wide spread of column norms)."""
    S = gaussian(seed, N, M)
    return np.ascontiguousarray(S * (decay ** np.arange(M))[:, None])


def kahan(n: int, theta: float, delta: float = 0.0) -> np.ndarray:
    """Kahan's matrix K = diag(1, s, .., s^(n-1)) (I - c U), c = cos theta,
    s = sin theta, U strictly upper triangular ones; column j additionally
    scaled by (1 - delta)^j.  Returned as (n, n) complex128 rows = columns."""
    c, s = np.cos(theta), np.sin(theta)
    K = np.triu(-c * np.ones((n, n)), 1) + np.eye(n)
    K = (s ** np.arange(n))[:, None] * K
    K = K * ((1.0 - delta) ** np.arange(n))[None, :]
    return np.ascontiguousarray(K.T, dtype=np.complex128)


def diagonal(values) -> np.ndarray:
    d = np.asarray(values, dtype=np.complex128)
    return np.ascontiguousarray(np.diag(d).T)


def unitary(seed: int, n: int) -> np.ndarray:
    """Haar-ish random unitary (QR of a complex Gaussian with phase fix)."""
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    ph = np.diag(R) / np.abs(np.diag(R))
    return Q * ph[None, :]


# ---------------------------------------------------------------------------
# Seeded draws of the learned surrogate (the network's initial weights and
# its minibatch order); the training arithmetic is elsewhere.
# ---------------------------------------------------------------------------

def mlp_layout(din: int, hidden: int, dout: int) -> dict:
    """Offsets of W1, b1, W2, b2, W3, b3, W4, b4 (row-major [in][out]) in the
    flat parameter vector, and the total length."""
    off = {}
    o = 0
    for name, n in (("W1", din * hidden), ("b1", hidden), ("W2", hidden * hidden), ("b2", hidden),
                    ("W3", hidden * hidden), ("b3", hidden), ("W4", hidden * dout), ("b4", dout)):
        off[name] = (o, n)
        o += n
    off["total"] = o
    return off


def mlp_init(seed: int, din: int, hidden: int, dout: int) -> np.ndarray:
    """Glorot-uniform weights, zero biases, as a flat float32 vector."""
    rng = np.random.default_rng(seed)
    lay = mlp_layout(din, hidden, dout)
    p = np.zeros(lay["total"], dtype=np.float32)
    shapes = {"W1": (din, hidden), "W2": (hidden, hidden), "W3": (hidden, hidden), "W4": (hidden, dout)}
    for name, (fi, fo) in shapes.items():
        o, n = lay[name]
        lim = np.sqrt(6.0 / (fi + fo))
        p[o:o + n] = rng.uniform(-lim, lim, n).astype(np.float32)
    return p


def batch_indices(seed: int, M: int, batch: int, steps: int, start_step: int = 0) -> np.ndarray:
    """Minibatch sample indices for steps start_step .. start_step+steps-1:
    each epoch is a fresh permutation of range(M) (epoch e from seed + e);
    shape (steps, batch) int64."""
    out = np.empty((steps, batch), dtype=np.int64)
    per_epoch = max(1, M // batch)
    for s in range(steps):
        g = start_step + s
        e, r = divmod(g, per_epoch)
        perm = _perm_cache(seed, e, M)
        if batch <= M:
            out[s] = perm[r * batch:(r + 1) * batch]
        else:
            out[s] = np.resize(perm, batch)
    return out


_PERM = {}


def _perm_cache(seed: int, e: int, M: int) -> np.ndarray:
    key = (seed, e, M)
    if key not in _PERM:
        if len(_PERM) > 4:
            _PERM.clear()
        _PERM[key] = np.random.default_rng(seed + e).permutation(M)
    return _PERM[key]
