"""Thin ctypes binding of libair (C ABI in include/air.h).

Argument marshalling only: torch tensors supply device memory and the HIP
stream; every step of the computation runs in the library's HIP kernels.
There is no CPU fallback: if libair.so is missing or fails to load, every
entry point raises.
"""
from __future__ import annotations

import ctypes
import os
import sys
import weakref
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libair.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "air.h")

AIR_OK, AIR_E_INVAL, AIR_E_UNSUPPORTED, AIR_E_NOMEM, AIR_E_DEVICE, AIR_E_BUSY, AIR_E_RANGE = \
    0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "AIR_OK", -1: "AIR_E_INVAL", -2: "AIR_E_UNSUPPORTED", -3: "AIR_E_NOMEM",
                -4: "AIR_E_DEVICE", -5: "AIR_E_BUSY", -6: "AIR_E_RANGE"}
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp16x3": 3}

_lib = None


class AirJob(ctypes.Structure):
    """air_job of include/air.h."""
    _fields_ = [("c", ctypes.c_void_p), ("in_", ctypes.c_void_p), ("tx", ctypes.c_void_p),
                ("N", ctypes.c_int64), ("snr_db", ctypes.c_double), ("noise_in", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("llr", ctypes.c_void_p),
                ("t_arrival_ns", ctypes.c_uint64), ("tag", ctypes.c_uint64)]


class AirResult(ctypes.Structure):
    """air_result of include/air.h."""
    _fields_ = [("id", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("mi", ctypes.c_double), ("gmi", ctypes.c_double),
                ("se_mi", ctypes.c_double), ("se_gmi", ctypes.c_double),
                ("recomputed", ctypes.c_uint64), ("t_arrival_ns", ctypes.c_uint64),
                ("t_admit_ns", ctypes.c_uint64), ("t_launch_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64), ("footprint", ctypes.c_uint64)]


class AirServerInfo(ctypes.Structure):
    """air_server_info of include/air.h."""
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("in_use", ctypes.c_uint64),
                ("peak_in_use", ctypes.c_uint64), ("budget", ctypes.c_uint64),
                ("max_batch", ctypes.c_int32), ("queued", ctypes.c_int32)]


class AirRoofs(ctypes.Structure):
    """air_roofs of include/air.h."""
    _fields_ = [("exp_per_s", ctypes.c_double), ("explog_per_s", ctypes.c_double),
                ("fma_per_s", ctypes.c_double), ("exp_fma_ratio", ctypes.c_double * 3),
                ("mfma_f16_flops", ctypes.c_double), ("mfma_bf16_flops", ctypes.c_double),
                ("copy_bytes_per_s", ctypes.c_double)]


class AirError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load() -> ctypes.CDLL:
    """Load libair.so (built in-tree by paper_2108_07001_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2108_07001_amd.build` "
                           "(there is no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    pvp = ctypes.POINTER(ctypes.c_void_p)
    lib.air_create.argtypes = [pvp, ci, vp]
    lib.air_create.restype = ci
    lib.air_destroy.argtypes = [vp]
    lib.air_destroy.restype = None
    lib.air_set_stream.argtypes = [vp, vp]
    lib.air_set_stream.restype = ci
    lib.air_last_error.argtypes = [vp]
    lib.air_last_error.restype = ctypes.c_char_p
    lib.air_sync.argtypes = [vp]
    lib.air_sync.restype = ci
    lib.air_const_create.argtypes = [vp, vp, vp, ci, ci, pvp]
    lib.air_const_create.restype = ci
    lib.air_const_destroy.argtypes = [vp]
    lib.air_const_destroy.restype = None
    lib.air_const_bits.argtypes = [vp]
    lib.air_const_bits.restype = ci
    lib.air_llr.argtypes = [vp, vp, vp, i64, dbl, ci, vp]
    lib.air_llr.restype = ci
    lib.air_mi_gmi.argtypes = [vp, vp, vp, vp, i64, dbl, ci, vp, vp]
    lib.air_mi_gmi.restype = ci
    lib.air_sweep.argtypes = [vp, vp, vp, vp, i64, vp, ci, ci, vp, vp]
    lib.air_sweep.restype = ci
    lib.air_sweep_noalloc.argtypes = [vp, vp, vp, vp, i64, vp, ci, ci, vp, vp]
    lib.air_sweep_noalloc.restype = ci
    lib.air_last_recomputed.argtypes = [vp]
    lib.air_last_recomputed.restype = i64
    lib.air_last_exact.argtypes = [vp]
    lib.air_last_exact.restype = i64
    lib.air_set_timing.argtypes = [vp, ci]
    lib.air_set_timing.restype = ci
    lib.air_kernel_time.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
    lib.air_kernel_time.restype = ci
    lib.air_measure_roofs.argtypes = [vp, ctypes.POINTER(AirRoofs)]
    lib.air_measure_roofs.restype = ci
    lib.air_llr_maxlog.argtypes = [vp, vp, vp, i64, dbl, ci, vp]
    lib.air_llr_maxlog.restype = ci
    lib.air_gmi_maxlog.argtypes = [vp, vp, vp, vp, i64, dbl, ci, vp, vp]
    lib.air_gmi_maxlog.restype = ci
    lib.air_sweep_maxlog.argtypes = [vp, vp, vp, vp, i64, vp, ci, ci, vp, vp]
    lib.air_sweep_maxlog.restype = ci
    lib.air_llr_aux.argtypes = [vp, vp, vp, i64, dbl, ci, vp]
    lib.air_llr_aux.restype = ci
    lib.air_mi_gmi_aux.argtypes = [vp, vp, vp, vp, i64, dbl, ci, vp, vp]
    lib.air_mi_gmi_aux.restype = ci
    lib.air_noise_var.argtypes = [vp, vp, vp, vp, i64, ci, vp]
    lib.air_noise_var.restype = ci
    lib.air_pipe_create.argtypes = [vp, vp, i64, ci, ci, ctypes.POINTER(ctypes.c_void_p)]
    lib.air_pipe_create.restype = ci
    lib.air_pipe_push.argtypes = [vp, vp, i64, dbl, vp]
    lib.air_pipe_push.restype = ci
    lib.air_pipe_wait.argtypes = [vp]
    lib.air_pipe_wait.restype = ci
    lib.air_pipe_destroy.argtypes = [vp]
    lib.air_pipe_destroy.restype = None
    lib.air_hard_decide.argtypes = [vp, vp, vp, vp, i64, vp, vp]
    lib.air_hard_decide.restype = ci
    lib.air_hard_sweep.argtypes = [vp, vp, vp, vp, i64, vp, ci, vp, vp]
    lib.air_hard_sweep.restype = ci
    lib.air_q_factor_db.argtypes = [dbl]
    lib.air_q_factor_db.restype = dbl
    lib.air_server_create.argtypes = [vp, ctypes.c_size_t, ci, pvp]
    lib.air_server_create.restype = ci
    lib.air_server_submit.argtypes = [vp, ctypes.POINTER(AirJob), ctypes.POINTER(ctypes.c_uint64)]
    lib.air_server_submit.restype = ci
    lib.air_server_poll.argtypes = [vp, ctypes.POINTER(AirResult), ci]
    lib.air_server_poll.restype = ci
    lib.air_server_drain.argtypes = [vp, ci]
    lib.air_server_drain.restype = ci
    lib.air_server_query.argtypes = [vp, ctypes.POINTER(AirServerInfo)]
    lib.air_server_query.restype = ci
    lib.air_server_last_error.argtypes = [vp]
    lib.air_server_last_error.restype = ctypes.c_char_p
    lib.air_server_destroy.argtypes = [vp]
    lib.air_server_destroy.restype = ci
    lib.air_aux_rates.argtypes = [vp, vp, vp, vp, i64, ci, vp, vp]
    lib.air_aux_rates.restype = ci
    lib.air_ngmi.argtypes = [vp, ci, ci, vp]
    lib.air_ngmi.restype = ci
    lib.air_hd_rates.argtypes = [vp, ci, i64, ci, vp]
    lib.air_hd_rates.restype = ci
    lib.air_fec_net.argtypes = [vp, i64, ci, ci, vp, vp, ci, dbl, vp, vp, vp]
    lib.air_fec_net.restype = ci
    _lib = lib
    return lib


def header_functions() -> list:
    """Names of the functions declared in include/air.h."""
    import re
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(air_[a-z_0-9]+)\s*\(", txt)))


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(device: int):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Const:
    """A constellation resident on the device (air_const_create)."""

    def __init__(self, ctx: "Context", X, labels):
        X = np.ascontiguousarray(X, dtype=np.float64)
        lab = np.ascontiguousarray(labels, dtype=np.uint32)
        if X.ndim != 2 or lab.shape != (X.shape[0],):
            raise AirError(AIR_E_INVAL, "X must be M x D and labels of length M")
        self.ctx = ctx
        self.M, self.D = X.shape
        h = ctypes.c_void_p()
        st = ctx.lib.air_const_create(ctx.h, X.ctypes.data, lab.ctypes.data, self.M, self.D,
                                      ctypes.byref(h))
        ctx.check(st)
        self.h = h
        self.m = ctx.lib.air_const_bits(h)
        ctx._consts.add(self)

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.air_const_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # never call into the HIP runtime while the interpreter tears down
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Context:
    """An air_ctx on one device, issuing work on a torch stream."""

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None):
        self.lib = load()
        self.device = int(device)
        h = ctypes.c_void_p()
        sh = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream_handle(self.device)
        st = self.lib.air_create(ctypes.byref(h), self.device, sh)
        if st != AIR_OK:
            raise AirError(st, "air_create failed")
        self.h = h
        self.torch_device = torch.device("cuda", self.device)
        self._consts = weakref.WeakSet()
        self._servers = weakref.WeakSet()

    # -- plumbing -----------------------------------------------------------
    def check(self, st: int):
        if st != AIR_OK:
            raise AirError(st, self.lib.air_last_error(self.h).decode())

    def set_stream(self, stream: torch.cuda.Stream):
        self.check(self.lib.air_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)))

    def sync(self):
        self.check(self.lib.air_sync(self.h))

    def last_recomputed(self) -> int:
        return int(self.lib.air_last_recomputed(self.h))

    def last_exact(self) -> int:
        return int(self.lib.air_last_exact(self.h))

    def set_timing(self, enable: bool):
        self.check(self.lib.air_set_timing(self.h, 1 if enable else 0))

    def kernel_time(self):
        """(total ms, launches) of the demapping kernels timed since the last read."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self.check(self.lib.air_kernel_time(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def measure_roofs(self) -> dict:
        """air_measure_roofs: measured rates of the units bounding the path."""
        r = AirRoofs()
        self.check(self.lib.air_measure_roofs(self.h, ctypes.byref(r)))
        return {"exp_per_s": r.exp_per_s, "explog_per_s": r.explog_per_s, "fma_per_s": r.fma_per_s,
                "exp_fma_ratio": {"K1": r.exp_fma_ratio[0], "K2": r.exp_fma_ratio[1],
                                  "K4": r.exp_fma_ratio[2]},
                "mfma_f16_flops": r.mfma_f16_flops, "mfma_bf16_flops": r.mfma_bf16_flops,
                "copy_bytes_per_s": r.copy_bytes_per_s}

    def close(self):
        if getattr(self, "h", None):
            for sv in list(self._servers):
                sv.close()
            for c in list(self._consts):
                c.close()
            self.lib.air_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def const(self, X, labels) -> Const:
        return Const(self, X, labels)

    def server(self, budget_bytes: int, max_inflight: int = 256) -> "Server":
        sv = Server(self, budget_bytes, max_inflight)
        self._servers.add(sv)
        return sv

    def pipe(self, c: Const, max_symbols: int, depth: int = 3, prec: str = "fp32") -> "Pipe":
        pp = Pipe(self, c, max_symbols, depth, prec)
        self._servers.add(pp)          # closed with the context, before its constellations
        return pp

    def _dtype(self, prec: str):
        return torch.float64 if prec == "fp64" else torch.float32

    def _check_block(self, t: torch.Tensor, c: Const, prec: str, name: str):
        if not isinstance(t, torch.Tensor) or t.device != self.torch_device:
            raise AirError(AIR_E_INVAL, f"{name} must be a tensor on {self.torch_device}")
        if t.dtype != self._dtype(prec) or t.dim() != 2 or t.shape[1] != c.D or not t.is_contiguous():
            raise AirError(AIR_E_INVAL, f"{name} must be a contiguous N x {c.D} {self._dtype(prec)} tensor")

    def _check_tx(self, tx: torch.Tensor, N: int):
        if (not isinstance(tx, torch.Tensor) or tx.device != self.torch_device or
                tx.dtype not in (torch.int32, torch.uint32) or tx.shape != (N,) or not tx.is_contiguous()):
            raise AirError(AIR_E_INVAL, f"tx must be a contiguous int32/uint32 tensor of length {N}")

    # -- entry points (air_llr, air_mi_gmi, air_sweep) -----------------------
    def llr(self, c: Const, Y: torch.Tensor, snr_db: float, prec: str = "fp32",
            out: Optional[torch.Tensor] = None) -> torch.Tensor:
        self._check_block(Y, c, prec, "Y")
        N = Y.shape[0]
        if out is None:
            out = torch.empty((N, c.m), dtype=self._dtype(prec), device=self.torch_device)
        elif out.shape != (N, c.m) or out.dtype != self._dtype(prec) or not out.is_contiguous():
            raise AirError(AIR_E_INVAL, "out has the wrong shape or dtype")
        self.check(self.lib.air_llr(self.h, c.h, _ptr(Y), N, float(snr_db), PREC[prec], _ptr(out)))
        return out

    def mi_gmi(self, c: Const, Y: torch.Tensor, tx: torch.Tensor, snr_db: float,
               prec: str = "fp32", llr: bool = False):
        self._check_block(Y, c, prec, "Y")
        N = Y.shape[0]
        self._check_tx(tx, N)
        stats = torch.empty(4, dtype=torch.float64, device=self.torch_device)
        L = torch.empty((N, c.m), dtype=self._dtype(prec), device=self.torch_device) if llr else None
        self.check(self.lib.air_mi_gmi(self.h, c.h, _ptr(Y), _ptr(tx), N, float(snr_db),
                                       PREC[prec], _ptr(stats), _ptr(L)))
        return stats, L

    # -- auxiliary-channel rates (air_noise_var, air_llr_aux, air_mi_gmi_aux) --
    def noise_var(self, c: Const, Y: torch.Tensor, tx: torch.Tensor, prec: str = "fp32"):
        """Noise variance estimates with known tx: D per-dimension values, then
        the isotropic one (float64 tensor of D + 1, on the device)."""
        self._check_block(Y, c, prec, "Y")
        N = Y.shape[0]
        self._check_tx(tx, N)
        var = torch.empty(c.D + 1, dtype=torch.float64, device=self.torch_device)
        self.check(self.lib.air_noise_var(self.h, c.h, _ptr(Y), _ptr(tx), N, PREC[prec], _ptr(var)))
        return var

    def llr_aux(self, c: Const, Y: torch.Tensor, sigma2_aux: float, prec: str = "fp32",
                out: Optional[torch.Tensor] = None):
        """LLRs with the receiver's Gaussian metric of variance sigma2_aux."""
        self._check_block(Y, c, prec, "Y")
        N = Y.shape[0]
        if out is None:
            out = torch.empty((N, c.m), dtype=self._dtype(prec), device=self.torch_device)
        self.check(self.lib.air_llr_aux(self.h, c.h, _ptr(Y), N, float(sigma2_aux), PREC[prec],
                                        _ptr(out)))
        return out

    def mi_gmi_aux(self, c: Const, Y: torch.Tensor, tx: torch.Tensor, sigma2_aux: float,
                   prec: str = "fp32", llr: bool = False):
        """MI, GMI (+ SEs) of the mismatched receiver with metric variance sigma2_aux."""
        self._check_block(Y, c, prec, "Y")
        N = Y.shape[0]
        self._check_tx(tx, N)
        stats = torch.empty(4, dtype=torch.float64, device=self.torch_device)
        L = torch.empty((N, c.m), dtype=self._dtype(prec), device=self.torch_device) if llr else None
        self.check(self.lib.air_mi_gmi_aux(self.h, c.h, _ptr(Y), _ptr(tx), N, float(sigma2_aux),
                                           PREC[prec], _ptr(stats), _ptr(L)))
        return stats, L

    def aux_rates(self, c: Const, Y: torch.Tensor, tx: torch.Tensor, prec: str = "fp32"):
        """air_aux_rates: the isotropic noise-variance estimate from (Y, tx), then
        the rates of the receiver that demaps with it and their NGMI (synchronises).
        Returns a dict with sigma2, the per-dimension variances, MI, GMI, their
        SEs, NGMI and its SE."""
        self._check_block(Y, c, prec, "Y")
        N = Y.shape[0]
        self._check_tx(tx, N)
        var = np.empty(c.D + 1)
        rates = np.empty(7)
        self.check(self.lib.air_aux_rates(self.h, c.h, _ptr(Y), _ptr(tx), N, PREC[prec],
                                          var.ctypes.data, rates.ctypes.data))
        keys = ["sigma2", "mi", "gmi", "se_mi", "se_gmi", "ngmi", "se_ngmi"]
        out = {k: float(v) for k, v in zip(keys, rates)}
        out["var"] = var[:-1]
        return out

    def hard_decide(self, c: Const, Y: torch.Tensor, tx: Optional[torch.Tensor] = None,
                    decided: bool = True):
        """Nearest-point decisions of a float32 block (air_hard_decide).
        Returns (decided X rows or None, counts [symbol errors, bit errors] or None)."""
        self._check_block(Y, c, "fp32", "Y")
        N = Y.shape[0]
        if tx is not None:
            self._check_tx(tx, N)
        dec = torch.empty(N, dtype=torch.int32, device=self.torch_device) if decided else None
        counts = torch.empty(2, dtype=torch.int64, device=self.torch_device) if tx is not None else None
        self.check(self.lib.air_hard_decide(self.h, c.h, _ptr(Y), _ptr(tx), N, _ptr(dec), _ptr(counts)))
        return dec, counts

    def hard_sweep(self, c: Const, tx: torch.Tensor, Z: torch.Tensor, snr_db: Sequence[float],
                   decided: bool = False):
        """Decisions over an SNR sweep (air_hard_sweep). Returns (counts S x 2,
        decided S x N or None)."""
        self._check_block(Z, c, "fp32", "Z")
        N = Z.shape[0]
        self._check_tx(tx, N)
        snr = np.ascontiguousarray(np.atleast_1d(np.asarray(snr_db, dtype=np.float64)))
        S = snr.shape[0]
        counts = torch.empty((S, 2), dtype=torch.int64, device=self.torch_device)
        dec = torch.empty((S, N), dtype=torch.int32, device=self.torch_device) if decided else None
        self.check(self.lib.air_hard_sweep(self.h, c.h, _ptr(tx), _ptr(Z), N, snr.ctypes.data, S,
                                           _ptr(counts), _ptr(dec)))
        return counts, dec

    # -- max-log form (air_llr_maxlog, air_gmi_maxlog, air_sweep_maxlog) -------
    def llr_maxlog(self, c: Const, Y: torch.Tensor, snr_db: float, prec: str = "fp32",
                   out: Optional[torch.Tensor] = None) -> torch.Tensor:
        self._check_block(Y, c, prec, "Y")
        N = Y.shape[0]
        if out is None:
            out = torch.empty((N, c.m), dtype=self._dtype(prec), device=self.torch_device)
        elif out.shape != (N, c.m) or out.dtype != self._dtype(prec) or not out.is_contiguous():
            raise AirError(AIR_E_INVAL, "out has the wrong shape or dtype")
        self.check(self.lib.air_llr_maxlog(self.h, c.h, _ptr(Y), N, float(snr_db), PREC[prec], _ptr(out)))
        return out

    def gmi_maxlog(self, c: Const, Y: torch.Tensor, tx: torch.Tensor, snr_db: float,
                   prec: str = "fp32", llr: bool = False):
        """[NaN, GMI, NaN, SE_GMI] of the max-log receiver, and optionally its LLRs."""
        self._check_block(Y, c, prec, "Y")
        N = Y.shape[0]
        self._check_tx(tx, N)
        stats = torch.empty(4, dtype=torch.float64, device=self.torch_device)
        L = torch.empty((N, c.m), dtype=self._dtype(prec), device=self.torch_device) if llr else None
        self.check(self.lib.air_gmi_maxlog(self.h, c.h, _ptr(Y), _ptr(tx), N, float(snr_db),
                                           PREC[prec], _ptr(stats), _ptr(L)))
        return stats, L

    def sweep_maxlog(self, c: Const, tx: torch.Tensor, Z: torch.Tensor, snr_db: Sequence[float],
                     prec: str = "fp32", llr: bool = False, stats_out: Optional[torch.Tensor] = None,
                     llr_out: Optional[torch.Tensor] = None):
        return self.sweep(c, tx, Z, snr_db, prec, llr, stats_out, llr_out, _fn="air_sweep_maxlog")

    def sweep(self, c: Const, tx: torch.Tensor, Z: torch.Tensor, snr_db: Sequence[float],
              prec: str = "fp32", llr: bool = False, stats_out: Optional[torch.Tensor] = None,
              llr_out: Optional[torch.Tensor] = None, _fn: str = "air_sweep"):
        self._check_block(Z, c, prec, "Z")
        N = Z.shape[0]
        self._check_tx(tx, N)
        snr = np.ascontiguousarray(np.atleast_1d(np.asarray(snr_db, dtype=np.float64)))
        S = snr.shape[0]
        stats = stats_out if stats_out is not None else torch.empty(
            (S, 4), dtype=torch.float64, device=self.torch_device)
        if stats.shape != (S, 4) or stats.dtype != torch.float64:
            raise AirError(AIR_E_INVAL, "stats_out must be S x 4 float64")
        L = llr_out
        if L is None and llr:
            L = torch.empty((S, N, c.m), dtype=self._dtype(prec), device=self.torch_device)
        if L is not None and (L.shape != (S, N, c.m) or L.dtype != self._dtype(prec)):
            raise AirError(AIR_E_INVAL, "llr_out has the wrong shape or dtype")
        self.check(getattr(self.lib, _fn)(self.h, c.h, _ptr(tx), _ptr(Z), N, snr.ctypes.data, S,
                                          PREC[prec], _ptr(stats), _ptr(L)))
        return stats, L

    def sweep_noalloc(self, c: Const, tx: torch.Tensor, Z: torch.Tensor, snr_db: Sequence[float],
                      prec: str = "fp32", stats_out: torch.Tensor = None, llr_out: torch.Tensor = None):
        """air_sweep_noalloc: as sweep, with caller-allocated outputs (the call
        allocates no device memory)."""
        if stats_out is None:
            raise AirError(AIR_E_INVAL, "sweep_noalloc needs stats_out")
        return self.sweep(c, tx, Z, snr_db, prec=prec, stats_out=stats_out, llr_out=llr_out,
                          _fn="air_sweep_noalloc")


def _buffer(x, dtype, shape, name: str, device: torch.device):
    """Address of a job buffer: a contiguous tensor (on the server's device or on
    the host) or a C-contiguous numpy array, of the given dtype and shape."""
    if isinstance(x, torch.Tensor):
        ok_dev = x.device == device or x.device.type == "cpu"
        if not ok_dev or x.dtype != dtype or tuple(x.shape) != shape or not x.is_contiguous():
            raise AirError(AIR_E_INVAL, f"{name} must be a contiguous {dtype} tensor of shape {shape} "
                                        f"on {device} or the host")
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        npd = {torch.float32: np.float32, torch.int32: np.int32}[dtype]
        if x.dtype not in (npd, np.uint32 if npd is np.int32 else npd) or x.shape != shape \
                or not x.flags.c_contiguous:
            raise AirError(AIR_E_INVAL, f"{name} must be a C-contiguous {npd.__name__} array of shape {shape}")
        return x.ctypes.data
    raise AirError(AIR_E_INVAL, f"{name} must be a tensor or numpy array")


class Pipe:
    """Per-buffer streaming from host memory (air_pipe_*): push() host buffers
    of received symbols, wait() for their LLRs in host buffers. Buffers are
    kept referenced here until wait() returns."""

    def __init__(self, ctx: Context, c: Const, max_symbols: int, depth: int = 3, prec: str = "fp32"):
        self.ctx = ctx
        self.lib = ctx.lib
        self.c = c
        self.prec = prec
        self.max_symbols = int(max_symbols)
        h = ctypes.c_void_p()
        ctx.check(self.lib.air_pipe_create(ctx.h, c.h, self.max_symbols, int(depth), PREC[prec],
                                           ctypes.byref(h)))
        self.h = h
        self._held = []

    def _host(self, x, shape, name):
        dt = np.float64 if self.prec == "fp64" else np.float32
        tdt = torch.float64 if self.prec == "fp64" else torch.float32
        if isinstance(x, torch.Tensor):
            if x.device.type != "cpu" or x.dtype != tdt or tuple(x.shape) != shape or not x.is_contiguous():
                raise AirError(AIR_E_INVAL, f"{name} must be a contiguous host {dt.__name__} tensor {shape}")
            return x.data_ptr()
        if not isinstance(x, np.ndarray) or x.dtype != dt or x.shape != shape or not x.flags.c_contiguous:
            raise AirError(AIR_E_INVAL, f"{name} must be a C-contiguous {dt.__name__} array {shape}")
        return x.ctypes.data

    def push(self, Y, snr_db: float, llr):
        """Queue one buffer: Y (N x D) and llr (N x m), host tensors (pinned or
        not) or numpy arrays of the pipe's precision."""
        N = int(Y.shape[0])
        yp = self._host(Y, (N, self.c.D), "Y")
        lp = self._host(llr, (N, self.c.m), "llr")
        self.ctx.check(self.lib.air_pipe_push(self.h, ctypes.c_void_p(yp), N, float(snr_db),
                                              ctypes.c_void_p(lp)))
        self._held.append((Y, llr))

    def wait(self):
        st = self.lib.air_pipe_wait(self.h)
        self._held.clear()
        self.ctx.check(st)

    def close(self):
        if getattr(self, "h", None):
            self.lib.air_pipe_destroy(self.h)
            self.h = None
            self._held.clear()

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The serving loop (air_server_*): jobs are queued with submit() and their
    results collected with poll() / results(). Buffers handed to a job are kept
    referenced here until its result has been polled."""

    def __init__(self, ctx: Context, budget_bytes: int, max_inflight: int = 256):
        self.ctx = ctx
        self.lib = ctx.lib
        h = ctypes.c_void_p()
        ctx.check(self.lib.air_server_create(ctx.h, int(budget_bytes), int(max_inflight), ctypes.byref(h)))
        self.h = h
        self._held = {}

    def check(self, st: int):
        if st != AIR_OK:
            raise AirError(st, self.lib.air_server_last_error(self.h).decode())

    def submit(self, c: Const, inp, snr_db: float, tx=None, prec: str = "fp16x3",
               noise: bool = False, llr=None, t_arrival_ns: int = 0, tag: int = 0) -> int:
        """Queue a job. inp: N x D float32 received points (or unit noise with
        noise=True); tx: N int32 indices or None; llr: N x m float32 output or None.
        Each may be a tensor on the device or on the host, or a numpy array."""
        N = int(inp.shape[0])
        j = AirJob()
        j.c = c.h.value
        j.in_ = _buffer(inp, torch.float32, (N, c.D), "inp", self.ctx.torch_device)
        j.tx = None if tx is None else _buffer(tx, torch.int32, (N,), "tx", self.ctx.torch_device)
        j.N = N
        j.snr_db = float(snr_db)
        j.noise_in = 1 if noise else 0
        j.prec = PREC[prec]
        j.llr = None if llr is None else _buffer(llr, torch.float32, (N, c.m), "llr", self.ctx.torch_device)
        j.t_arrival_ns = int(t_arrival_ns)
        j.tag = int(tag)
        jid = ctypes.c_uint64()
        self.check(self.lib.air_server_submit(self.h, ctypes.byref(j), ctypes.byref(jid)))
        self._held[jid.value] = (c, inp, tx, llr)
        return jid.value

    def poll(self, max_results: int = 256) -> list:
        """Finished results (dicts), at most max_results; never blocks."""
        buf = (AirResult * max_results)()
        n = self.lib.air_server_poll(self.h, buf, max_results)
        if n < 0:
            raise AirError(n, "air_server_poll failed")
        out = []
        for r in buf[:n]:
            d = {k: getattr(r, k) for k, _ in AirResult._fields_ if k != "pad"}
            self._held.pop(r.id, None)
            out.append(d)
        return out

    def drain(self, timeout_ms: int = -1):
        st = self.lib.air_server_drain(self.h, int(timeout_ms))
        if st != AIR_OK:
            raise AirError(st, "air_server_drain")

    def results(self, timeout_ms: int = -1) -> list:
        """Drain, then every result not yet polled."""
        self.drain(timeout_ms)
        out = []
        while True:
            part = self.poll(1024)
            out += part
            if len(part) < 1024:
                return out

    def info(self) -> dict:
        inf = AirServerInfo()
        self.check(self.lib.air_server_query(self.h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in AirServerInfo._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.lib.air_server_destroy(self.h)
            self.h = None
            self._held.clear()

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def q_factor_db(ber: float) -> float:
    """Q-factor in dB from a bit error rate (air_q_factor_db)."""
    return float(load().air_q_factor_db(float(ber)))


# Flat aliases with the C names.
def air_create(device: int = 0, stream: Optional[torch.cuda.Stream] = None) -> Context:
    return Context(device, stream)


def air_const_create(ctx: Context, X, labels) -> Const:
    return ctx.const(X, labels)


def _check_host(st: int, what: str):
    if st != AIR_OK:
        raise AirError(st, what)


def ngmi_table(stats, m: int) -> np.ndarray:
    """air_ngmi: NGMI and its SE (S x 2) of S points of statistics (S x 4)."""
    st = np.ascontiguousarray(np.asarray(stats, dtype=np.float64).reshape(-1, 4))
    out = np.empty((st.shape[0], 2))
    _check_host(load().air_ngmi(st.ctypes.data, st.shape[0], int(m), out.ctypes.data), "air_ngmi")
    return out


def ngmi(gmi: float, m: int) -> float:
    """NGMI of one GMI value (air_ngmi)."""
    return float(ngmi_table([[np.nan, gmi, np.nan, np.nan]], m)[0, 0])


def hd_rates(counts, N: int, m: int) -> np.ndarray:
    """air_hd_rates: BER, SER, Q_dB (S x 3) of S points of error counts (S x 2)."""
    c = np.ascontiguousarray(np.asarray(counts, dtype=np.uint64).reshape(-1, 2))
    out = np.empty((c.shape[0], 3))
    _check_host(load().air_hd_rates(c.ctypes.data, c.shape[0], int(N), int(m), out.ctypes.data),
                "air_hd_rates")
    return out


def fec_net(ber, m: int, overhead, threshold, symbol_rate: float = 1.0) -> dict:
    """air_fec_net: HD-FEC pass/fail (S x F), net rate (S) and the code giving it
    (S, -1 for none) for S BERs and F codes (overheads and threshold BERs)."""
    b = np.ascontiguousarray(np.atleast_1d(np.asarray(ber, dtype=np.float64)))
    oh = np.ascontiguousarray(np.atleast_1d(np.asarray(overhead, dtype=np.float64)))
    th = np.ascontiguousarray(np.atleast_1d(np.asarray(threshold, dtype=np.float64)))
    if oh.shape != th.shape:
        raise AirError(AIR_E_INVAL, "overhead and threshold must have the same length")
    S, F = b.shape[0], oh.shape[0]
    pas = np.empty((S, F), dtype=np.int32)
    net = np.empty(S)
    code = np.empty(S, dtype=np.int32)
    _check_host(load().air_fec_net(b.ctypes.data, 1, S, int(m), oh.ctypes.data, th.ctypes.data, F,
                                   float(symbol_rate), pas.ctypes.data, net.ctypes.data, code.ctypes.data),
                "air_fec_net")
    return {"pass": pas.astype(bool), "net": net, "code": code}


def air_llr(ctx: Context, c: Const, Y, snr_db, prec="fp32", out=None):
    return ctx.llr(c, Y, snr_db, prec, out)


def air_mi_gmi(ctx: Context, c: Const, Y, tx, snr_db, prec="fp32", llr=False):
    return ctx.mi_gmi(c, Y, tx, snr_db, prec, llr)


def air_sweep(ctx: Context, c: Const, tx, Z, snr_db, prec="fp32", llr=False):
    return ctx.sweep(c, tx, Z, snr_db, prec, llr)
