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
    lib.air_last_recomputed.argtypes = [vp]
    lib.air_last_recomputed.restype = i64
    lib.air_set_timing.argtypes = [vp, ci]
    lib.air_set_timing.restype = ci
    lib.air_kernel_time.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
    lib.air_kernel_time.restype = ci
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

    def __del__(self):
        # never call into the HIP runtime while the interpreter tears down
        if sys.is_finalizing():
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

    def set_timing(self, enable: bool):
        self.check(self.lib.air_set_timing(self.h, 1 if enable else 0))

    def kernel_time(self):
        """(total ms, launches) of the demapping kernels timed since the last read."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self.check(self.lib.air_kernel_time(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "h", None):
            for c in list(self._consts):
                c.close()
            self.lib.air_destroy(self.h)
            self.h = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def const(self, X, labels) -> Const:
        return Const(self, X, labels)

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

    def sweep(self, c: Const, tx: torch.Tensor, Z: torch.Tensor, snr_db: Sequence[float],
              prec: str = "fp32", llr: bool = False, stats_out: Optional[torch.Tensor] = None,
              llr_out: Optional[torch.Tensor] = None):
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
        self.check(self.lib.air_sweep(self.h, c.h, _ptr(tx), _ptr(Z), N, snr.ctypes.data, S,
                                      PREC[prec], _ptr(stats), _ptr(L)))
        return stats, L


# Flat aliases with the C names.
def air_create(device: int = 0, stream: Optional[torch.cuda.Stream] = None) -> Context:
    return Context(device, stream)


def air_const_create(ctx: Context, X, labels) -> Const:
    return ctx.const(X, labels)


def air_llr(ctx: Context, c: Const, Y, snr_db, prec="fp32", out=None):
    return ctx.llr(c, Y, snr_db, prec, out)


def air_mi_gmi(ctx: Context, c: Const, Y, tx, snr_db, prec="fp32", llr=False):
    return ctx.mi_gmi(c, Y, tx, snr_db, prec, llr)


def air_sweep(ctx: Context, c: Const, tx, Z, snr_db, prec="fp32", llr=False):
    return ctx.sweep(c, tx, Z, snr_db, prec, llr)
