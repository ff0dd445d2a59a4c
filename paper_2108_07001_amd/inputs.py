"""Seeded synthetic workloads for the demapping / information-rate path.

This module only draws inputs: constellation points, bit labels, transmitted
indices, unit-variance noise and SNR grids (and, for the serving mix, a job
stream). It holds none of the method's arithmetic (no symbol energies of the
demapper, noise variances, distances or likelihoods; the only energies computed
here are the normalisations that define the constellations) and is the one
piece shared by the test oracle and the GPU path.

The paper names its multidimensional formats only in its acronym list
(4D-64PRS, 8D-2048PRS, PM-QPSK, a 3-core coupled-core multi-core fibre); their
point sets are not given, so stand-ins of the same sizes are drawn here:

* ``pmqpsk``      PM-QPSK as a 4-D set, M = 16: coordinate d of the point with
                  label l is (1 - 2 * bit_d(l)) / sqrt(2) (Gray per dimension).
* ``psk8x8``      8-PSK x 8-PSK, M = 64, D = 4: phases 2 pi k / 8, point
                  p = 8 a + b = (cos a, sin a, cos b, sin b) / sqrt(2) (unit
                  average energy), labels a seeded permutation of 0..63.
* ``gauss8d2048`` M = 2048 points i.i.d. N(0, I_8), scaled to unit average
                  energy, natural-binary labels (label j = j).
* ``gauss12d4096`` M = 4096 points i.i.d. N(0, I_12) (3 cores x 2
                  polarisations x I/Q), unit average energy, seeded-permuted
                  labels.

* ``qam4`` ... ``qam64`` the paper's own 1 GBaud formats, 2-D M-QAM with
                  M = 4, 8, 16, 32, 64 (D = 2): a product of Gray-labelled PAM
                  levels per dimension, 2^ceil(m/2) levels in-phase and
                  2^floor(m/2) in quadrature (square for M = 4, 16, 64,
                  rectangular 4 x 2 and 8 x 4 for 8- and 32-QAM, whose
                  geometry the paper does not give), label = (I label <<
                  floor(m/2)) | Q label, unit average energy. One buffer of
                  the paper's receiver holds 2^22 ADC samples at 4 samples per
                  symbol, i.e. 2^20 symbols; the workload is one such buffer.

Seeds: ``SeedSequence(cfg_seed).spawn(3)`` gives the (constellation + labels,
transmitted index, noise) generators. Noise is drawn in FP64 and rounded once
to FP32 (``pmqpsk`` keeps FP64). Every draw is a prefix of the full-size one,
so a workload with a smaller N is the leading part of the full workload.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

CONFIGS = {
    "pmqpsk": dict(seed=1, M=16, D=4, N=100_000, snr_db=[0.0, 5.0, 10.0, 15.0, 20.0],
                   noise="f64", desc="PM-QPSK as 4-D M=16, FP64 method"),
    "psk8x8": dict(seed=2, M=64, D=4, N=1_000_000, snr_db=[float(s) for s in range(-2, 19)],
                   noise="f32", desc="8-PSK x 8-PSK 4-D M=64, 21 SNR points"),
    "gauss8d2048": dict(seed=3, M=2048, D=8, N=4_000_000,
                        snr_db=[float(s) for s in range(4, 25, 2)], noise="f32",
                        desc="Gaussian 8-D M=2048, natural labels, 11 SNR points"),
    "gauss12d4096": dict(seed=5, M=4096, D=12, N=16_000_000,
                         snr_db=[0.5 * i for i in range(41)], noise="f32",
                         desc="Gaussian 12-D M=4096, permuted labels, 41-point sweep"),
}
for _m in range(2, 7):
    CONFIGS[f"qam{1 << _m}"] = dict(seed=10 + _m, M=1 << _m, D=2, N=1 << 20, snr_db=[18.0],
                                    noise="f32", desc=f"{1 << _m}-QAM (2-D), one 2^20-symbol buffer")

# Serving mix: Poisson arrivals of demap + AIR jobs.
SERVING = dict(seed=4, rate_hz=2000.0, jobs=20_000, M_choices=(16, 64, 256, 2048),
               D_for_M={16: 2, 64: 4, 256: 4, 2048: 8}, N_log10=(3.0, 6.0),
               snr_db=(0.0, 25.0), pool_per_M=8)


@dataclasses.dataclass
class Workload:
    name: str
    X: np.ndarray          # M x D float64, row-major
    labels: np.ndarray     # M uint32, bijection onto 0..M-1
    tx: np.ndarray         # N uint32, transmitted index into X
    z: np.ndarray          # N x D unit-variance noise (float32, or float64)
    snr_db: np.ndarray     # S float64

    @property
    def M(self) -> int:
        return self.X.shape[0]

    @property
    def D(self) -> int:
        return self.X.shape[1]

    @property
    def N(self) -> int:
        return self.tx.shape[0]

    @property
    def m(self) -> int:
        return int(round(math.log2(self.M)))


def _rngs(seed: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(3)]


def pm_qpsk() -> tuple:
    """PM-QPSK as a 4-D, 16-point set with Gray-per-dimension labels."""
    lab = np.arange(16, dtype=np.uint32)
    X = np.empty((16, 4))
    for l in range(16):
        for d in range(4):
            X[l, d] = (1.0 - 2.0 * ((l >> d) & 1)) / math.sqrt(2.0)
    return X, lab


def psk8_x_psk8(rng: np.random.Generator) -> tuple:
    """8-PSK x 8-PSK product set (unit average energy) with seeded-permuted labels."""
    th = 2.0 * math.pi * np.arange(8) / 8.0
    X = np.empty((64, 4))
    for a in range(8):
        for b in range(8):
            X[8 * a + b] = [math.cos(th[a]), math.sin(th[a]), math.cos(th[b]), math.sin(th[b])]
    X /= math.sqrt(2.0)
    labels = rng.permutation(64).astype(np.uint32)
    return X, labels


def gaussian(rng: np.random.Generator, M: int, D: int, permuted: bool) -> tuple:
    """M points i.i.d. N(0, I_D), scaled to unit average energy; natural or permuted labels."""
    X = rng.standard_normal((M, D))
    X = X / math.sqrt(np.mean(np.sum(X * X, axis=1)))
    labels = rng.permutation(M).astype(np.uint32) if permuted else np.arange(M, dtype=np.uint32)
    return X, labels


def _gray(n: int) -> int:
    return n ^ (n >> 1)


def qam(M: int) -> tuple:
    """2-D M-QAM as a product of Gray-labelled PAM levels (unit average energy)."""
    m = int(round(math.log2(M)))
    mi, mq = (m + 1) // 2, m // 2
    li, lq = 1 << mi, 1 << mq
    X = np.empty((M, 2))
    labels = np.empty(M, dtype=np.uint32)
    for a in range(li):
        for b in range(lq):
            j = a * lq + b
            X[j] = [2 * a - (li - 1), 2 * b - (lq - 1)]
            labels[j] = (_gray(a) << mq) | _gray(b)
    X /= math.sqrt(np.mean(np.sum(X * X, axis=1)))
    return X, labels


def constellation(name: str):
    """(X, labels) of a named workload (drawn from its constellation generator)."""
    cfg = CONFIGS[name]
    rc, _, _ = _rngs(cfg["seed"])
    if name == "pmqpsk":
        return pm_qpsk()
    if name == "psk8x8":
        return psk8_x_psk8(rc)
    if name == "gauss8d2048":
        return gaussian(rc, 2048, 8, permuted=False)
    if name == "gauss12d4096":
        return gaussian(rc, 4096, 12, permuted=True)
    if name.startswith("qam"):
        return qam(int(name[3:]))
    raise KeyError(name)


def noise(rng: np.random.Generator, N: int, D: int, f64: bool, chunk: int = 1 << 20) -> np.ndarray:
    """N x D unit normal noise, drawn in FP64 in row chunks and rounded once to FP32."""
    out = np.empty((N, D), dtype=np.float64 if f64 else np.float32)
    for lo in range(0, N, chunk):
        hi = min(N, lo + chunk)
        out[lo:hi] = rng.standard_normal((hi - lo, D))
    return out


def make(name: str, N: Optional[int] = None, snr_db=None) -> Workload:
    """The named workload, optionally cut to its first N samples or another SNR grid."""
    cfg = CONFIGS[name]
    X, labels = constellation(name)
    _, rt, rn = _rngs(cfg["seed"])
    n = cfg["N"] if N is None else int(N)
    tx = rt.integers(0, X.shape[0], size=n, dtype=np.int64).astype(np.uint32)
    z = noise(rn, n, X.shape[1], f64=(cfg["noise"] == "f64"))
    snr = np.asarray(cfg["snr_db"] if snr_db is None else snr_db, dtype=np.float64)
    return Workload(name, X, labels, tx, z, np.atleast_1d(snr))


def random_constellation(seed: int, M: int, D: int, permuted: bool = True) -> tuple:
    """A seeded Gaussian constellation of any size (for edge-case tests)."""
    return gaussian(np.random.default_rng(seed), M, D, permuted)


def random_block(seed: int, M: int, N: int, D: int, f64: bool = False) -> tuple:
    """Seeded (tx, z): N uniform indices into M points and N x D unit noise."""
    r = np.random.default_rng(seed)
    tx = r.integers(0, M, size=N, dtype=np.int64).astype(np.uint32)
    return tx, noise(r, N, D, f64)


# ---- serving mix ----------------------------------------------------------

@dataclasses.dataclass
class Job:
    arrival_s: float
    M: int
    D: int
    N: int
    snr_db: float
    const_id: int          # index into the pool of constellations for this M
    seed: int              # seed of this job's (tx, z)


def serving_pool(M: int):
    """The resident pool of seeded constellations for one M of the serving mix."""
    D = SERVING["D_for_M"][M]
    rc, _, _ = _rngs(SERVING["seed"] * 1000 + M)
    return [gaussian(rc, M, D, permuted=True) for _ in range(SERVING["pool_per_M"])]


def serving_jobs(n_jobs: Optional[int] = None) -> list:
    """Poisson job stream of the serving mix (arrival times in seconds)."""
    r = np.random.default_rng(SERVING["seed"])
    n = SERVING["jobs"] if n_jobs is None else int(n_jobs)
    gaps = r.exponential(1.0 / SERVING["rate_hz"], size=n)
    t = np.cumsum(gaps)
    Ms = r.choice(np.asarray(SERVING["M_choices"]), size=n)
    lo, hi = SERVING["N_log10"]
    Ns = np.round(10.0 ** r.uniform(lo, hi, size=n)).astype(np.int64)
    snr = r.uniform(*SERVING["snr_db"], size=n)
    cid = r.integers(0, SERVING["pool_per_M"], size=n)
    seeds = r.integers(0, 2**31 - 1, size=n)
    return [Job(float(t[i]), int(Ms[i]), SERVING["D_for_M"][int(Ms[i])], int(Ns[i]),
                float(snr[i]), int(cid[i]), int(seeds[i])) for i in range(n)]
