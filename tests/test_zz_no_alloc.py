"""air_sweep_noalloc (the sweep for callers that cannot allocate device
memory) against air_sweep, through the C ABI: two calls in a row, the second
with a smaller input, in every precision; LLRs bit for bit, statistics to
FP64 rounding (a launch may hold fewer SNR points, which changes only the
order of the per-block FP64 sums). Sizes beyond the scratch are refused
before any kernel runs."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2108_07001_amd import air, inputs
from tests.helpers import to_dev, tx_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = air.Context(0)
    yield c
    c.close()


def _both(ctx, c, w, prec):
    z = to_dev(w.z, torch.float64 if prec == "fp64" else torch.float32)
    tx = tx_dev(w.tx)
    S = len(w.snr_db)
    dt = torch.float64 if prec == "fp64" else torch.float32
    ref, Lr = ctx.sweep(c, tx, z, w.snr_db, prec=prec, llr=True)
    st = torch.empty((S, 4), dtype=torch.float64, device=ctx.torch_device)
    L = torch.empty((S, w.N, c.m), dtype=dt, device=ctx.torch_device)
    ctx.sweep_noalloc(c, tx, z, w.snr_db, prec=prec, stats_out=st, llr_out=L)
    ctx.sync()
    return ref.cpu().numpy(), Lr.cpu().numpy(), st.cpu().numpy(), L.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp16x3", "bf16x3", "fp32", "fp64"])
def test_noalloc_matches_sweep_twice_then_smaller(ctx, prec):
    big = inputs.make("psk8x8", N=1_000_000, snr_db=np.linspace(-2.0, 40.0, 22))
    small = inputs.make("psk8x8", N=3_000 + 17, snr_db=[30.0, 5.0, 45.0])
    c = ctx.const(big.X, big.labels)
    for w in (big, small):
        if prec == "fp64":
            w = inputs.Workload(w.name, w.X, w.labels, w.tx, w.z.astype(np.float64), w.snr_db)
        ref, Lr, st, L = _both(ctx, c, w, prec)
        print(f"{prec} N={w.N} S={len(w.snr_db)}: max |dstats| {np.abs(st - ref).max():.2e}")
        assert np.array_equal(L, Lr)
        np.testing.assert_allclose(st, ref, rtol=1e-12, atol=1e-12)
    c.close()


def test_noalloc_large_set_second_tier(ctx):
    w = inputs.make("gauss8d2048", N=200_000, snr_db=[14.0, 24.0, 4.0])
    c = ctx.const(w.X, w.labels)
    for n in (w.N, 5_000):
        wn = inputs.Workload(w.name, w.X, w.labels, w.tx[:n].copy(), np.ascontiguousarray(w.z[:n]), w.snr_db)
        ref, Lr, st, L = _both(ctx, c, wn, "fp16x3")
        assert ctx.last_recomputed() > 0
        assert np.array_equal(L, Lr)
        np.testing.assert_allclose(st, ref, rtol=1e-12, atol=1e-12)
    c.close()


def test_noalloc_refuses_sizes_beyond_its_scratch(ctx):
    w = inputs.make("psk8x8", N=1000, snr_db=[10.0])
    c = ctx.const(w.X, w.labels)
    z = to_dev(w.z)
    tx = tx_dev(w.tx)
    st = torch.empty((1, 4), dtype=torch.float64, device=ctx.torch_device)
    snr = np.array([10.0])
    # a claimed N far beyond the buffers: refused by the size check before any launch
    r = ctx.lib.air_sweep_noalloc(ctx.h, c.h, ctypes.c_void_p(tx.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                  ctypes.c_int64(50_000_000), snr.ctypes.data, 1, air.PREC["fp16x3"],
                                  ctypes.c_void_p(st.data_ptr()), None)
    assert r == air.AIR_E_INVAL
    assert b"air_sweep_noalloc" in ctx.lib.air_last_error(ctx.h)
    # the context still works
    s2 = torch.empty((1, 4), dtype=torch.float64, device=ctx.torch_device)
    ctx.sweep_noalloc(c, tx, z, snr, prec="fp16x3", stats_out=s2)
    ref, _ = ctx.sweep(c, tx, z, snr, prec="fp16x3")
    ctx.sync()
    np.testing.assert_allclose(s2.cpu().numpy(), ref.cpu().numpy(), rtol=1e-12, atol=1e-12)
    c.close()
