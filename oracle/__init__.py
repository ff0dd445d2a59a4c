"""FP64 CPU oracle for soft demapping and Monte-Carlo MI/GMI (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It wraps ``liboracle.so`` (built from
``oracle.c`` with gcc) through ctypes and shares nothing with the GPU library.

The quantities follow the standard definitions of the mutual information of a
uniform discrete input over real AWGN, the bit-wise generalised mutual
information under bit-metric decoding, and per-bit log-likelihood ratios; the
paper lists these only among its acronyms (MI, GMI, LLR, BMD, AIR, AWGN), so
the readings R1-R6 stated at the top of ``oracle.c`` apply.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(verbose: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (gcc, OpenMP, portable -O3)."""
    cmd = ["gcc", "-O3", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    up = ctypes.POINTER(ctypes.c_uint32)
    fp = ctypes.POINTER(ctypes.c_float)
    lib.oracle_bits.argtypes = [up, ctypes.c_int, ctypes.c_int]
    lib.oracle_bits.restype = ctypes.c_int
    lib.oracle_es.argtypes = [dp, ctypes.c_int, ctypes.c_int]
    lib.oracle_es.restype = ctypes.c_double
    lib.oracle_sigma2.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double]
    lib.oracle_sigma2.restype = ctypes.c_double
    lib.oracle_eval.argtypes = [dp, up, ctypes.c_int, ctypes.c_int, dp, up, ctypes.c_int64,
                                ctypes.c_double, dp, dp, dp, dp]
    lib.oracle_eval.restype = ctypes.c_int
    lib.oracle_sweep.argtypes = [dp, up, ctypes.c_int, ctypes.c_int, up, fp, dp, ctypes.c_int64,
                                 dp, ctypes.c_int, dp, dp, dp, dp]
    lib.oracle_sweep.restype = ctypes.c_int
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = ctypes.c_int
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.oracle_hd.argtypes = [dp, up, ctypes.c_int, ctypes.c_int, fp, up, ctypes.c_int64, up, u64p]
    lib.oracle_hd.restype = ctypes.c_int
    lib.oracle_hd_sweep.argtypes = [dp, up, ctypes.c_int, ctypes.c_int, up, fp, ctypes.c_int64, dp,
                                    ctypes.c_int, up, u64p]
    lib.oracle_hd_sweep.restype = ctypes.c_int
    lib.oracle_eval_maxlog.argtypes = lib.oracle_eval.argtypes
    lib.oracle_eval_maxlog.restype = ctypes.c_int
    lib.oracle_eval_aux.argtypes = lib.oracle_eval.argtypes
    lib.oracle_eval_aux.restype = ctypes.c_int
    lib.oracle_noise_var.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp, up, ctypes.c_int64, dp]
    lib.oracle_noise_var.restype = ctypes.c_int
    lib.oracle_q_db.argtypes = [ctypes.c_double]
    lib.oracle_q_db.restype = ctypes.c_double
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_ngmi.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp]
    lib.oracle_ngmi.restype = ctypes.c_int
    lib.oracle_hd_rates.argtypes = [u64p, ctypes.c_int, ctypes.c_int64, ctypes.c_int, dp]
    lib.oracle_hd_rates.restype = ctypes.c_int
    lib.oracle_fec_net.argtypes = [dp, ctypes.c_int64, ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int,
                                   ctypes.c_double, i32p, dp, i32p]
    lib.oracle_fec_net.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class OracleError(RuntimeError):
    pass


def _const(X, labels):
    X = np.ascontiguousarray(X, dtype=np.float64)
    labels = np.ascontiguousarray(labels, dtype=np.uint32)
    if X.ndim != 2 or labels.shape != (X.shape[0],):
        raise OracleError("X must be M x D and labels length M")
    return X, labels


def bits(labels, M: int, D: int) -> int:
    """m = log2 M, or -1 if the constellation shape or labelling is invalid."""
    labels = np.ascontiguousarray(labels, dtype=np.uint32)
    return _load().oracle_bits(_ptr(labels, ctypes.c_uint32), M, D)


def es(X) -> float:
    """Average symbol energy (1/M) sum_j |x_j|^2."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    return _load().oracle_es(_ptr(X, ctypes.c_double), X.shape[0], X.shape[1])


def sigma2(X, snr_db: float) -> float:
    """Noise variance per real dimension: Es / (D * 10^(snr_db/10))."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    return _load().oracle_sigma2(es(X), X.shape[1], float(snr_db))


def evaluate(X, labels, Y, snr_db: float, tx=None, llr: bool = True, per_sample: bool = False):
    """Demap the block Y (N x D) at one SNR.

    Returns a dict with ``stats`` = [MI, GMI, SE_MI, SE_GMI] (bits; needs tx),
    ``llr`` (N x m, nats) and, with per_sample, ``u`` and ``v`` (bits).
    """
    return _evaluate("oracle_eval", X, labels, Y, snr_db, tx, llr, per_sample)


def evaluate_aux(X, labels, Y, sigma2_aux: float, tx=None, llr: bool = True,
                 per_sample: bool = False):
    """As evaluate, with the receiver's Gaussian metric of noise variance
    sigma2_aux per real dimension (auxiliary channel, reading R10 of oracle.c)."""
    return _evaluate("oracle_eval_aux", X, labels, Y, sigma2_aux, tx, llr, per_sample)


def evaluate_maxlog(X, labels, Y, snr_db: float, tx=None, llr: bool = True,
                    per_sample: bool = False):
    """Max-log demapping of Y at one SNR (readings R13, R14 of oracle.c):
    ``llr`` (N x m, nats), ``stats`` = [NaN, GMI, NaN, SE_GMI] with tx, and
    with per_sample ``v`` (``u`` is NaN)."""
    return _evaluate("oracle_eval_maxlog", X, labels, Y, snr_db, tx, llr, per_sample)


def sweep_maxlog(X, labels, tx, Z, snr_db, llr: bool = True):
    """Max-log over an SNR sweep: y = x_t + sigma_s z formed in FP64 from Z as
    in sweep (reading R6). Returns ``stats`` (S x 4) and ``llr`` (S x N x m)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    snr = np.atleast_1d(np.asarray(snr_db, dtype=np.float64))
    xt = X[np.asarray(tx, dtype=np.int64)]
    st, L = [], []
    for s in snr:
        r = evaluate_maxlog(X, labels, xt + math.sqrt(sigma2(X, s)) * Z, s, tx=tx, llr=llr)
        st.append(r["stats"])
        if llr:
            L.append(r["llr"])
    out = {"stats": np.array(st)}
    if llr:
        out["llr"] = np.array(L)
    return out


def noise_var(X, Y, tx):
    """Noise variance estimates with known transmitted points (reading R11):
    D per-dimension values, then the isotropic one."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    txa = np.ascontiguousarray(tx, dtype=np.uint32)
    M, D = X.shape
    if Y.ndim != 2 or Y.shape != (txa.shape[0], D):
        raise OracleError("Y must be N x D with N = len(tx)")
    out = np.empty(D + 1)
    rc = _load().oracle_noise_var(_ptr(X, ctypes.c_double), M, D, _ptr(Y, ctypes.c_double),
                                  _ptr(txa, ctypes.c_uint32), Y.shape[0], _ptr(out, ctypes.c_double))
    if rc != 0:
        raise OracleError(f"oracle_noise_var failed with code {rc}")
    return out


def ngmi(gmi: float, m: int) -> float:
    """Normalised GMI, 1 - (H(X) - GMI) / m with H(X) = m (reading R12)."""
    return float(ngmi_table(np.array([[np.nan, gmi, np.nan, np.nan]]), m)[0, 0])


def ngmi_table(stats, m: int):
    """NGMI and its standard error (S x 2) of S points of MI/GMI statistics
    (S x 4: MI, GMI, SE_MI, SE_GMI), reading R12."""
    st = np.ascontiguousarray(np.asarray(stats, dtype=np.float64).reshape(-1, 4))
    out = np.empty((st.shape[0], 2))
    rc = _load().oracle_ngmi(_ptr(st, ctypes.c_double), st.shape[0], int(m), _ptr(out, ctypes.c_double))
    if rc != 0:
        raise OracleError(f"oracle_ngmi failed with code {rc}")
    return out


def hd_rates(counts, N: int, m: int):
    """BER, SER and Q-factor in dB (S x 3) of S points of hard-decision error
    counts (S x 2: symbol errors, bit errors) over N symbols (readings R8, R9)."""
    c = np.ascontiguousarray(np.asarray(counts, dtype=np.uint64).reshape(-1, 2))
    out = np.empty((c.shape[0], 3))
    rc = _load().oracle_hd_rates(_ptr(c, ctypes.c_uint64), c.shape[0], int(N), int(m), _ptr(out, ctypes.c_double))
    if rc != 0:
        raise OracleError(f"oracle_hd_rates failed with code {rc}")
    return out


def fec_net(ber, m: int, overhead, threshold, symbol_rate: float = 1.0):
    """HD-FEC pass/fail (S x F), net rate (S) and the index of the code that
    gives it (S, -1: none) for S bit error rates and F codes of the given
    overheads (fractions) and threshold BERs (readings R15, R16)."""
    b = np.ascontiguousarray(np.atleast_1d(np.asarray(ber, dtype=np.float64)))
    oh = np.ascontiguousarray(np.atleast_1d(np.asarray(overhead, dtype=np.float64)))
    th = np.ascontiguousarray(np.atleast_1d(np.asarray(threshold, dtype=np.float64)))
    if oh.shape != th.shape:
        raise OracleError("overhead and threshold must have the same length")
    S, F = b.shape[0], oh.shape[0]
    pas = np.empty((S, F), dtype=np.int32)
    net = np.empty(S)
    best = np.empty(S, dtype=np.int32)
    rc = _load().oracle_fec_net(_ptr(b, ctypes.c_double), 1, S, int(m), _ptr(oh, ctypes.c_double),
                                _ptr(th, ctypes.c_double), F, float(symbol_rate), _ptr(pas, ctypes.c_int32),
                                _ptr(net, ctypes.c_double), _ptr(best, ctypes.c_int32))
    if rc != 0:
        raise OracleError(f"oracle_fec_net failed with code {rc}")
    return {"pass": pas.astype(bool), "net": net, "best": best}


def _evaluate(fn, X, labels, Y, noise, tx, llr, per_sample):
    X, labels = _const(X, labels)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    M, D = X.shape
    if Y.ndim != 2 or Y.shape[1] != D:
        raise OracleError("Y must be N x D")
    N = Y.shape[0]
    m = bits(labels, M, D)
    if m < 0:
        raise OracleError("invalid constellation")
    out = {}
    txa = None if tx is None else np.ascontiguousarray(tx, dtype=np.uint32)
    stats = np.full(4, np.nan) if txa is not None else None
    L = np.empty((N, m)) if llr else None
    u = np.empty(N) if (per_sample and txa is not None) else None
    v = np.empty(N) if (per_sample and txa is not None) else None
    rc = getattr(_load(), fn)(_ptr(X, ctypes.c_double), _ptr(labels, ctypes.c_uint32), M, D,
                              _ptr(Y, ctypes.c_double), _ptr(txa, ctypes.c_uint32), N,
                              float(noise), _ptr(stats, ctypes.c_double), _ptr(L, ctypes.c_double),
                              _ptr(u, ctypes.c_double), _ptr(v, ctypes.c_double))
    if rc != 0:
        raise OracleError(f"{fn} failed with code {rc}")
    if stats is not None:
        out["stats"] = stats
    if L is not None:
        out["llr"] = L
    if u is not None:
        out["u"], out["v"] = u, v
    return out


def sweep(X, labels, tx, Z, snr_db, llr: bool = True, per_sample: bool = False):
    """SNR sweep with y = x_t + sigma_s z in FP64 from the caller's noise Z.

    Z may be float32 (promoted exactly) or float64. Returns ``stats`` (S x 4),
    ``llr`` (S x N x m) and, with per_sample, ``u`` and ``v`` (S x N).
    """
    X, labels = _const(X, labels)
    M, D = X.shape
    txa = np.ascontiguousarray(tx, dtype=np.uint32)
    Z = np.asarray(Z)
    if Z.ndim != 2 or Z.shape[1] != D or Z.shape[0] != txa.shape[0]:
        raise OracleError("Z must be N x D with N = len(tx)")
    z32 = np.ascontiguousarray(Z) if Z.dtype == np.float32 else None
    z64 = None if z32 is not None else np.ascontiguousarray(Z, dtype=np.float64)
    snr = np.ascontiguousarray(np.atleast_1d(snr_db), dtype=np.float64)
    S, N = snr.shape[0], txa.shape[0]
    m = bits(labels, M, D)
    if m < 0:
        raise OracleError("invalid constellation")
    stats = np.full((S, 4), np.nan)
    L = np.empty((S, N, m)) if llr else None
    u = np.empty((S, N)) if per_sample else None
    v = np.empty((S, N)) if per_sample else None
    rc = _load().oracle_sweep(_ptr(X, ctypes.c_double), _ptr(labels, ctypes.c_uint32), M, D,
                              _ptr(txa, ctypes.c_uint32), _ptr(z32, ctypes.c_float),
                              _ptr(z64, ctypes.c_double), N, _ptr(snr, ctypes.c_double), S,
                              _ptr(stats, ctypes.c_double), _ptr(L, ctypes.c_double),
                              _ptr(u, ctypes.c_double), _ptr(v, ctypes.c_double))
    if rc != 0:
        raise OracleError(f"oracle_sweep failed with code {rc}")
    out = {"stats": stats}
    if L is not None:
        out["llr"] = L
    if u is not None:
        out["u"], out["v"] = u, v
    return out


def threads() -> int:
    """OpenMP threads the oracle library uses."""
    return _load().oracle_threads()


def hard_decisions(X, labels, Y, tx=None):
    """Nearest-point decisions of an FP32 block Y (readings R7, R8 of oracle.c).

    Returns ``decided`` (N X rows) and, with tx, ``counts`` = [symbol errors,
    bit errors]."""
    X, labels = _const(X, labels)
    M, D = X.shape
    Y = np.ascontiguousarray(Y, dtype=np.float32)
    if Y.ndim != 2 or Y.shape[1] != D:
        raise OracleError("Y must be N x D")
    N = Y.shape[0]
    txa = None if tx is None else np.ascontiguousarray(tx, dtype=np.uint32)
    dec = np.empty(N, dtype=np.uint32)
    counts = np.zeros(2, dtype=np.uint64) if txa is not None else None
    rc = _load().oracle_hd(_ptr(X, ctypes.c_double), _ptr(labels, ctypes.c_uint32), M, D,
                           _ptr(Y, ctypes.c_float), _ptr(txa, ctypes.c_uint32), N,
                           _ptr(dec, ctypes.c_uint32), _ptr(counts, ctypes.c_uint64))
    if rc != 0:
        raise OracleError(f"oracle_hd failed with code {rc}")
    out = {"decided": dec}
    if counts is not None:
        out["counts"] = counts
    return out


def hard_decisions_sweep(X, labels, tx, Z, snr_db, decided: bool = False):
    """Hard decisions of the SNR sweep (y = fmaf(sigma_f, z, x_t) in FP32).

    Returns ``counts`` (S x 2: symbol errors, bit errors) and optionally
    ``decided`` (S x N)."""
    X, labels = _const(X, labels)
    M, D = X.shape
    txa = np.ascontiguousarray(tx, dtype=np.uint32)
    Z = np.ascontiguousarray(Z, dtype=np.float32)
    if Z.ndim != 2 or Z.shape != (txa.shape[0], D):
        raise OracleError("Z must be N x D with N = len(tx)")
    snr = np.ascontiguousarray(np.atleast_1d(snr_db), dtype=np.float64)
    S, N = snr.shape[0], txa.shape[0]
    counts = np.zeros((S, 2), dtype=np.uint64)
    dec = np.empty((S, N), dtype=np.uint32) if decided else None
    rc = _load().oracle_hd_sweep(_ptr(X, ctypes.c_double), _ptr(labels, ctypes.c_uint32), M, D,
                                 _ptr(txa, ctypes.c_uint32), _ptr(Z, ctypes.c_float), N,
                                 _ptr(snr, ctypes.c_double), S, _ptr(dec, ctypes.c_uint32),
                                 _ptr(counts, ctypes.c_uint64))
    if rc != 0:
        raise OracleError(f"oracle_hd_sweep failed with code {rc}")
    out = {"counts": counts}
    if dec is not None:
        out["decided"] = dec
    return out


def q_factor_db(ber: float) -> float:
    """Q-factor in dB from a bit error rate (reading R9 of oracle.c)."""
    return _load().oracle_q_db(float(ber))
