"""GPU parity of the vector-ALU kernels (AIR_FP64, AIR_FP32) against the FP64 oracle.

All calls go through the C ABI (libair.so via the ctypes binding); inputs are
the seeded workloads, outputs are compared element by element.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2108_07001_amd import air, inputs
from tests.helpers import FP64_TOL, assert_llr, assert_stats, llr_err, to_dev, tx_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = air.Context(0)
    yield c
    c.close()


def _sweep(ctx, w, prec, llr=True):
    c = ctx.const(w.X, w.labels)
    zt = to_dev(w.z, torch.float64 if prec == "fp64" else torch.float32)
    stats, L = ctx.sweep(c, tx_dev(w.tx), zt, w.snr_db, prec=prec, llr=llr)
    ctx.sync()
    return stats.cpu().numpy(), (L.cpu().numpy() if L is not None else None), c


def test_fp64_pmqpsk_full_sweep_matches_oracle(ctx):
    w = inputs.make("pmqpsk")                      # N = 1e5, 5 SNR points, FP64 noise
    stats, L, _ = _sweep(ctx, w, "fp64")
    ref = oracle.sweep(w.X, w.labels, w.tx, w.z, w.snr_db)
    np.testing.assert_allclose(stats[:, :2], ref["stats"][:, :2], rtol=0, atol=FP64_TOL)
    np.testing.assert_allclose(stats[:, 2:], ref["stats"][:, 2:], rtol=1e-7, atol=1e-12)
    assert llr_err(L, ref["llr"]) <= FP64_TOL


def test_fp32_psk8x8_sweep_matches_oracle(ctx):
    w = inputs.make("psk8x8", N=60_000)
    stats, L, _ = _sweep(ctx, w, "fp32")
    ref = oracle.sweep(w.X, w.labels, w.tx, w.z, w.snr_db)
    assert_stats(stats, ref["stats"])
    assert_llr(L, ref["llr"])


def test_fp32_gauss8d2048_mi_gmi_given_block(ctx):
    w = inputs.make("gauss8d2048", N=3000)
    c = ctx.const(w.X, w.labels)
    for snr in [4.0, 14.0, 24.0]:
        es = np.mean(np.sum(w.X ** 2, axis=1))
        Y = (w.X[w.tx] + math.sqrt(es / (8 * 10 ** (snr / 10))) * w.z).astype(np.float32)
        stats, L = ctx.mi_gmi(c, to_dev(Y), tx_dev(w.tx), snr, prec="fp32", llr=True)
        ctx.sync()
        ref = oracle.evaluate(w.X, w.labels, Y.astype(np.float64), snr, tx=w.tx)
        assert_stats(stats.cpu().numpy(), ref["stats"])
        assert_llr(L.cpu().numpy(), ref["llr"])


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_llr_only(ctx, prec):
    X, lab = inputs.random_constellation(8, 256, 4)
    rng = np.random.default_rng(3)
    Y = rng.normal(size=(1000, 4)) * 0.6
    dt = np.float64 if prec == "fp64" else np.float32
    c = ctx.const(X, lab)
    L = ctx.llr(c, to_dev(Y.astype(dt)), 9.0, prec=prec)
    ctx.sync()
    ref = oracle.evaluate(X, lab, Y.astype(dt).astype(np.float64), 9.0)
    if prec == "fp64":
        assert llr_err(L.cpu().numpy(), ref["llr"]) <= FP64_TOL
    else:
        assert_llr(L.cpu().numpy(), ref["llr"])


@pytest.mark.parametrize("M,D,N", [(2, 1, 1), (4, 2, 257), (8, 3, 1000), (16, 16, 333),
                                   (32, 5, 700), (4096, 12, 300)])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_shapes_and_ragged_tails(ctx, M, D, N, prec):
    X, lab = inputs.random_constellation(M + D, M, D)
    tx, z = inputs.random_block(N + M, M, N, D, f64=(prec == "fp64"))
    w = inputs.Workload("t", X, lab, tx, z, np.array([-3.0, 7.0, 19.0]))
    stats, L, _ = _sweep(ctx, w, prec)
    ref = oracle.sweep(X, lab, tx, z, w.snr_db)
    if prec == "fp64":
        np.testing.assert_allclose(stats[:, :2], ref["stats"][:, :2], atol=FP64_TOL, rtol=0)
        assert llr_err(L, ref["llr"]) <= FP64_TOL
    else:
        assert_stats(stats, ref["stats"], se_rel=2e-2)
        assert_llr(L, ref["llr"])
    if N == 1:
        assert np.isnan(stats[:, 2:]).all()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_huge_llrs_take_the_exact_path(ctx, prec):
    # binary antipodal at 45 dB: |L| = |2y/sigma^2| reaches ~1e5 nats
    X = np.array([[1.0], [-1.0]])
    lab = np.array([0, 1], dtype=np.uint32)
    tx, z = inputs.random_block(1, 2, 2000, 1, f64=(prec == "fp64"))
    w = inputs.Workload("t", X, lab, tx, z, np.array([45.0, 0.0]))
    stats, L, _ = _sweep(ctx, w, prec)
    ref = oracle.sweep(X, lab, tx, z, w.snr_db)
    # FP32: the fast path's log2 sums carry ~1e-5 nat of absolute rounding
    assert llr_err(L, ref["llr"]) <= (FP64_TOL if prec == "fp64" else 1e-4)
    if prec == "fp32":
        assert ctx.last_recomputed() > 0


def test_high_snr_limit_and_far_received_points(ctx):
    X, lab = inputs.random_constellation(5, 64, 4)
    rng = np.random.default_rng(5)
    tx = rng.integers(0, 64, 500).astype(np.uint32)
    Y = X[tx] + 1e-4 * rng.normal(size=(500, 4))
    Y[:10] += 40.0          # far from every point: the total itself is starved at 30 dB
    c = ctx.const(X, lab)
    stats, L = ctx.mi_gmi(c, to_dev(Y.astype(np.float32)), tx_dev(tx), 30.0, prec="fp32", llr=True)
    ctx.sync()
    ref = oracle.evaluate(X, lab, Y.astype(np.float32).astype(np.float64), 30.0, tx=tx)
    assert_llr(L.cpu().numpy(), ref["llr"])
    # the outliers carry per-sample MI terms of ~6e5 bits, kept in FP32 per sample
    big = np.abs(ref["stats"][:2]).max()
    assert_stats(stats.cpu().numpy(), ref["stats"], tol=1e-4 + 1e-6 * big)


def test_deterministic(ctx):
    w = inputs.make("psk8x8", N=20_000)
    a, La, _ = _sweep(ctx, w, "fp32")
    b, Lb, _ = _sweep(ctx, w, "fp32")
    assert np.array_equal(a, b, equal_nan=True) and np.array_equal(La, Lb)


def test_invalid_tx_sets_range_error(ctx):
    w = inputs.make("psk8x8", N=1000, snr_db=[5.0])
    tx = w.tx.astype(np.int32).copy()
    tx[17] = 64
    c = ctx.const(w.X, w.labels)
    stats, L = ctx.sweep(c, tx_dev(tx), to_dev(w.z), w.snr_db, prec="fp32", llr=True)
    with pytest.raises(air.AirError) as e:
        ctx.sync()
    assert e.value.status == air.AIR_E_RANGE
    assert np.isnan(stats.cpu().numpy()).all()
    assert np.isnan(L.cpu().numpy()[0, 17]).all()
    ctx.sync()          # the error was cleared


def test_argument_errors(ctx):
    X, lab = inputs.pm_qpsk()
    with pytest.raises(air.AirError):
        ctx.const(X, np.zeros(16, dtype=np.uint32))           # labels not a bijection
    with pytest.raises(air.AirError):
        ctx.const(np.zeros((12, 2)), np.arange(12))            # M not a power of two
    c = ctx.const(X, lab)
    lib = ctx.lib
    host = np.zeros((4, 4), dtype=np.float32)
    out = torch.empty((4, 4), device="cuda")
    import ctypes
    st = lib.air_llr(ctx.h, c.h, ctypes.c_void_p(host.ctypes.data), 4, 0.0, 1,
                     ctypes.c_void_p(out.data_ptr()))
    assert st == air.AIR_E_INVAL                                # host pointer rejected
    st = lib.air_llr(ctx.h, c.h, ctypes.c_void_p(out.data_ptr()), 0, 0.0, 1,
                     ctypes.c_void_p(out.data_ptr()))
    assert st == air.AIR_E_INVAL                                # N = 0
    st = lib.air_llr(ctx.h, c.h, ctypes.c_void_p(out.data_ptr()), 4, 0.0, 7,
                     ctypes.c_void_p(out.data_ptr()))
    assert st == air.AIR_E_INVAL                                # unknown precision


def test_many_snr_points_span_launches(ctx):
    w = inputs.make("psk8x8", N=2000, snr_db=np.linspace(-5, 20, 70))
    stats, L, _ = _sweep(ctx, w, "fp32")
    ref = oracle.sweep(w.X, w.labels, w.tx, w.z, w.snr_db)
    assert_stats(stats, ref["stats"], se_rel=2e-2)
    assert_llr(L, ref["llr"])


def test_fp32_second_tier_frame64_window(ctx):
    """8-D, M = 2048 at 16..24 dB: |LLR| of several hundred nats, beyond the
    FP32 frame; those items are finished by the FP32 vector kernel's second
    tier in the FP64 frame (few or none need the exact path)."""
    w = inputs.make("gauss8d2048", N=3000 + 37, snr_db=[16.0, 20.0, 24.0])
    stats, L, _ = _sweep(ctx, w, "fp32")
    rec, exact = ctx.last_recomputed(), ctx.last_exact()
    ref = oracle.sweep(w.X, w.labels, w.tx, w.z, w.snr_db)
    print(f"second tier {rec} of {w.N * 3} items, exact path {exact}, max |L| {np.abs(ref['llr']).max():.0f}")
    assert_stats(stats, ref["stats"])
    assert_llr(L, ref["llr"])
    assert rec > 0 and exact < rec


@pytest.mark.parametrize("M,D,N", [(2, 1, 1), (8, 2, 65), (64, 4, 1000 + 37), (256, 3, 257)])
def test_fp32_second_tier_shapes_and_launches(ctx, M, D, N):
    """Second-tier items in ragged tails, at every group size (M < 16 too) and
    over 70 SNR points up to 45 dB (two launches, each with its own lists)."""
    X, lab = inputs.random_constellation(M + D, M, D)
    tx, z = inputs.random_block(N + M, M, N, D)
    w = inputs.Workload("t", X, lab, tx, z, np.linspace(-5.0, 45.0, 70))
    stats, L, _ = _sweep(ctx, w, "fp32")
    rec = ctx.last_recomputed()
    ref = oracle.sweep(X, lab, tx, z, w.snr_db)
    assert_stats(stats, ref["stats"], se_rel=2e-2)
    assert_llr(L, ref["llr"])
    assert rec > 0


def test_fp32_second_tier_counts_and_results_repeat(ctx):
    """The second tier's lists and counts start clean on every call: results
    and counts repeat bit for bit across calls of different sizes and SNRs."""
    hi = inputs.make("psk8x8", N=20_000, snr_db=[30.0, 40.0])
    lo = inputs.make("psk8x8", N=5_000, snr_db=[-2.0])
    c = ctx.const(hi.X, hi.labels)

    def run(wl):
        st, L = ctx.sweep(c, tx_dev(wl.tx), to_dev(wl.z), wl.snr_db, prec="fp32", llr=True)
        ctx.sync()
        return st.cpu().numpy(), L.cpu().numpy(), ctx.last_recomputed(), ctx.last_exact()

    a = run(hi)
    assert a[2] > 0
    b = run(lo)
    assert b[2] == 0 and b[3] == 0
    for _ in range(2):
        a2 = run(hi)
        assert np.array_equal(a2[0], a[0]) and np.array_equal(a2[1], a[1]) and a2[2:] == a[2:]
        b2 = run(lo)
        assert np.array_equal(b2[0], b[0]) and b2[2:] == b[2:]
    ref = oracle.sweep(hi.X, hi.labels, hi.tx, hi.z, hi.snr_db)
    assert_stats(a[0], ref["stats"])
    assert_llr(a[1], ref["llr"])
