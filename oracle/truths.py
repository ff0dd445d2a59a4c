"""Closed-form and quadrature truths for the oracle's pins (test infrastructure).

* Binary antipodal input {+a, -a} over real AWGN with per-dimension noise
  variance sigma^2, s = a^2 / sigma^2 (the textbook BPSK capacity with
  equiprobable inputs):

      C_BPSK(s) = 1 - E_z[ log2(1 + exp(-2 s - 2 sqrt(s) z)) ],  z ~ N(0, 1).

  Any product of independent binary antipodal coordinates (PM-QPSK as a 4-D
  set with the Gray-per-dimension labelling) factorises, so its MI and its GMI
  both equal (number of coordinates) x C_BPSK. With the SNR reading
  snr = Es / (D sigma^2), every coordinate of PM-QPSK has s = snr.

* The same input with a receiver whose Gaussian metric assumes the noise
  variance sigma_a^2 instead of sigma^2 (mismatched decoding): by symmetry the
  transmitted point can be fixed to +a, and

      MI_aux = 1 - E_z[ log2(1 + exp(-2 a (a + sigma z) / sigma_a^2)) ],

  which is at most C_BPSK, with equality at sigma_a = sigma.

* Mutual information of 8-PSK (radius r, uniform input) over 2-D real AWGN by
  a Gauss-Hermite product rule; by rotational symmetry the transmitted point
  can be fixed to the first one.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate


def c_bpsk(snr: float) -> float:
    """Equiprobable BPSK MI in bits at s = a^2/sigma^2 (linear), adaptive quadrature."""
    s = float(snr)
    rs = math.sqrt(s)

    def f(z):
        x = -2.0 * s - 2.0 * rs * z
        # log2(1 + e^x) without overflow
        l1p = x + math.log1p(math.exp(-x)) if x > 0 else math.log1p(math.exp(x))
        return math.exp(-0.5 * z * z) / math.sqrt(2 * math.pi) * l1p / math.log(2.0)

    # the integrand has its knee at z = -sqrt(s)
    pts = sorted({-rs, 0.0})
    val, _ = integrate.quad(f, -np.inf, pts[0], limit=400, epsabs=1e-14, epsrel=1e-13)
    for lo, hi in zip(pts, pts[1:] + [np.inf]):
        v, _ = integrate.quad(f, lo, hi, limit=400, epsabs=1e-14, epsrel=1e-13)
        val += v
    return 1.0 - val


def c_bpsk_gauss_hermite(snr: float, n: int = 160) -> float:
    """Same quantity by an n-node Gauss-Hermite rule (an independent check)."""
    s = float(snr)
    xg, wg = np.polynomial.hermite.hermgauss(n)
    z = math.sqrt(2.0) * xg
    x = -2.0 * s - 2.0 * math.sqrt(s) * z
    l1p = np.where(x > 0, x + np.log1p(np.exp(-np.abs(x))), np.log1p(np.exp(np.minimum(x, 0))))
    return 1.0 - float(np.sum(wg * l1p) / math.sqrt(math.pi) / math.log(2.0))


def c_bpsk_aux(a: float, sigma2: float, sigma2_aux: float) -> float:
    """Binary antipodal {+a, -a} rate (bits) under a Gaussian metric of
    variance sigma2_aux when the true noise variance is sigma2, by adaptive
    quadrature over z ~ N(0, 1)."""
    sig = math.sqrt(sigma2)
    g = 2.0 * a / sigma2_aux

    def f(z):
        x = -g * (a + sig * z)
        l1p = x + math.log1p(math.exp(-x)) if x > 0 else math.log1p(math.exp(x))
        return math.exp(-0.5 * z * z) / math.sqrt(2 * math.pi) * l1p / math.log(2.0)

    knee = -a / sig
    val = 0.0
    for lo, hi in ((-np.inf, knee), (knee, 0.0 if knee < 0 else knee + 1.0), (0.0 if knee < 0 else knee + 1.0, np.inf)):
        v, _ = integrate.quad(f, lo, hi, limit=400, epsabs=1e-14, epsrel=1e-13)
        val += v
    return 1.0 - val


def mi_8psk(snr: float, radius: float = 1.0 / math.sqrt(2.0), n: int = 96) -> float:
    """MI (bits) of uniform 8-PSK over 2-D real AWGN with snr = Es / (2 sigma^2)."""
    es = radius * radius
    sigma2 = es / (2.0 * snr)
    sigma = math.sqrt(sigma2)
    th = 2 * math.pi * np.arange(8) / 8
    pts = radius * np.stack([np.cos(th), np.sin(th)], axis=1)
    xg, wg = np.polynomial.hermite.hermgauss(n)
    z1, z2 = np.meshgrid(math.sqrt(2.0) * xg, math.sqrt(2.0) * xg, indexing="ij")
    w = np.outer(wg, wg) / math.pi
    y1 = pts[0, 0] + sigma * z1
    y2 = pts[0, 1] + sigma * z2
    a = -((y1[..., None] - pts[:, 0]) ** 2 + (y2[..., None] - pts[:, 1]) ** 2) / (2 * sigma2)
    a0 = a[..., 0]
    amax = a.max(axis=-1)
    lse = amax + np.log(np.exp(a - amax[..., None]).sum(axis=-1))
    u = (lse - a0) / math.log(2.0)
    return 3.0 - float(np.sum(w * u))
