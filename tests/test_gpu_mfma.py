"""GPU parity of the matrix-core kernels (AIR_FP16X3, AIR_BF16X3) against the FP64 oracle."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2108_07001_amd import air, inputs
from tests.helpers import assert_llr, assert_stats, llr_err, to_dev, tx_dev

pytestmark = pytest.mark.gpu

PRECS = ["fp16x3", "bf16x3"]
# Both split forms are held to the contract: |dL| <= 1e-3 max(|L|, 1 nat).
LLR_BAR = {"fp16x3": 1e-3, "bf16x3": 1e-3}


@pytest.fixture(scope="module")
def ctx():
    c = air.Context(0)
    yield c
    c.close()


def _sweep(ctx, w, prec, llr=True):
    c = ctx.const(w.X, w.labels)
    stats, L = ctx.sweep(c, tx_dev(w.tx), to_dev(w.z, torch.float32), w.snr_db, prec=prec, llr=llr)
    ctx.sync()
    return stats.cpu().numpy(), (L.cpu().numpy() if L is not None else None)


def _report(name, st, L, ref):
    dmi = np.abs(st[:, :2] - ref["stats"][:, :2]).max()
    print(f"{name}: max|dMI,dGMI| {dmi:.2e}  LLR rel {llr_err(L, ref['llr']):.2e}")


@pytest.mark.parametrize("prec", PRECS)
def test_psk8x8_sweep(ctx, prec):
    w = inputs.make("psk8x8", N=60_000)
    st, L = _sweep(ctx, w, prec)
    ref = oracle.sweep(w.X, w.labels, w.tx, w.z, w.snr_db)
    _report(f"psk8x8 {prec}", st, L, ref)
    assert_stats(st, ref["stats"])
    assert_llr(L, ref["llr"], LLR_BAR[prec])


@pytest.mark.parametrize("prec", PRECS)
def test_gauss8d2048_sweep(ctx, prec):
    w = inputs.make("gauss8d2048", N=2500)
    st, L = _sweep(ctx, w, prec)
    ref = oracle.sweep(w.X, w.labels, w.tx, w.z, w.snr_db)
    _report(f"gauss8d2048 {prec}", st, L, ref)
    assert_stats(st, ref["stats"], se_rel=2e-2)
    assert_llr(L, ref["llr"], LLR_BAR[prec])


@pytest.mark.parametrize("prec", PRECS)
def test_gauss12d4096_sweep(ctx, prec):
    w = inputs.make("gauss12d4096", N=400)
    st, L = _sweep(ctx, w, prec)
    ref = oracle.sweep(w.X, w.labels, w.tx, w.z, w.snr_db)
    _report(f"gauss12d4096 {prec}", st, L, ref)
    assert_stats(st, ref["stats"], se_rel=2e-2)
    assert_llr(L, ref["llr"], LLR_BAR[prec])


@pytest.mark.parametrize("M,D,N", [(16, 2, 333), (32, 4, 1000), (64, 1, 97), (128, 5, 515),
                                   (256, 4, 2049), (512, 9, 300), (1024, 16, 257), (16, 15, 70)])
@pytest.mark.parametrize("prec", PRECS)
def test_shapes(ctx, M, D, N, prec):
    X, lab = inputs.random_constellation(M * 7 + D, M, D)
    tx, z = inputs.random_block(N + M, M, N, D)
    w = inputs.Workload("t", X, lab, tx, z, np.array([-4.0, 3.0, 11.0, 22.0]))
    st, L = _sweep(ctx, w, prec)
    ref = oracle.sweep(X, lab, tx, z, w.snr_db)
    _report(f"M{M} D{D} N{N} {prec}", st, L, ref)
    assert_stats(st, ref["stats"], se_rel=2e-2)
    assert_llr(L, ref["llr"], LLR_BAR[prec])


@pytest.mark.parametrize("prec", PRECS)
def test_given_block_and_llr_only(ctx, prec):
    w = inputs.make("gauss8d2048", N=1500)
    c = ctx.const(w.X, w.labels)
    snr = 12.0
    es = np.mean(np.sum(w.X ** 2, axis=1))
    Y = (w.X[w.tx] + math.sqrt(es / (8 * 10 ** (snr / 10))) * w.z).astype(np.float32)
    stats, L = ctx.mi_gmi(c, to_dev(Y), tx_dev(w.tx), snr, prec=prec, llr=True)
    L2 = ctx.llr(c, to_dev(Y), snr, prec=prec)
    ctx.sync()
    ref = oracle.evaluate(w.X, w.labels, Y.astype(np.float64), snr, tx=w.tx)
    assert_stats(stats.cpu().numpy(), ref["stats"])
    assert_llr(L.cpu().numpy(), ref["llr"], LLR_BAR[prec])
    assert np.array_equal(L.cpu().numpy(), L2.cpu().numpy())


def test_small_sets_run_the_vector_kernel(ctx):
    X, lab = inputs.random_constellation(2, 8, 3)
    tx, z = inputs.random_block(3, 8, 500, 3)
    w = inputs.Workload("t", X, lab, tx, z, np.array([5.0]))
    a, La = _sweep(ctx, w, "fp16x3")
    b, Lb = _sweep(ctx, w, "fp32")
    assert np.array_equal(La, Lb) and np.allclose(a, b, equal_nan=True, rtol=0, atol=0)


def test_extreme_snr_takes_exact_path(ctx):
    X, lab = inputs.random_constellation(5, 64, 4)
    tx, z = inputs.random_block(6, 64, 700, 4)
    w = inputs.Workload("t", X, lab, tx, z, np.array([60.0, 45.0]))
    st, L = _sweep(ctx, w, "fp16x3")
    ref = oracle.sweep(X, lab, tx, z, w.snr_db)
    np.testing.assert_allclose(st[:, :2], 6.0, atol=1e-9)
    assert_llr(L, ref["llr"], LLR_BAR["fp16x3"])
    assert ctx.last_recomputed() > 0


@pytest.mark.parametrize("prec", PRECS)
def test_many_snr_points_span_launches(ctx, prec):
    # 70 SNR points: two launches of at most 64 points each; N = 40 000 gives a
    # first tier of 157 blocks (628 waves: three partial groups of 256 in the
    # second tier's collection); the high points send many samples there
    w = inputs.make("psk8x8", N=40_000, snr_db=np.linspace(-4.0, 31.0, 70))
    st, L = _sweep(ctx, w, prec)
    ref = oracle.sweep(w.X, w.labels, w.tx, w.z, w.snr_db)
    _report(f"psk8x8 70 points {prec}", st, L, ref)
    assert ctx.last_recomputed() > 0
    assert_stats(st, ref["stats"], se_rel=2e-2)
    assert_llr(L, ref["llr"], LLR_BAR[prec])


@pytest.mark.parametrize("prec", PRECS)
def test_deterministic(ctx, prec):
    w = inputs.make("psk8x8", N=20_000)
    a, La = _sweep(ctx, w, prec)
    b, Lb = _sweep(ctx, w, prec)
    assert np.array_equal(a, b, equal_nan=True) and np.array_equal(La, Lb)


def test_invalid_tx(ctx):
    w = inputs.make("psk8x8", N=1000, snr_db=[5.0])
    tx = w.tx.astype(np.int32).copy()
    tx[999] = 1 << 20
    c = ctx.const(w.X, w.labels)
    stats, L = ctx.sweep(c, tx_dev(tx), to_dev(w.z), w.snr_db, prec="fp16x3", llr=True)
    with pytest.raises(air.AirError) as e:
        ctx.sync()
    assert e.value.status == air.AIR_E_RANGE
    assert np.isnan(stats.cpu().numpy()).all()
    Lh = L.cpu().numpy()
    assert np.isnan(Lh[0, 999]).all() and np.isfinite(Lh[0, :999]).all()


@pytest.mark.parametrize("prec", PRECS)
def test_direct_rounds_at_high_snr(ctx, prec):
    # 8-D, M = 2048 at 24 dB: ~98 % of the samples have a bit side below the
    # first tier's FP32 frame, so after one mostly flagged round every wave
    # lists its later rounds for the second tier as they are. N = 1e6 gives
    # each of the 6144 waves two or three rounds. Sampled LLRs (taken from
    # all over the block, most from those later rounds) against the oracle,
    # and a bad transmitted index in a late round: NaN LLRs for that sample
    # only, and the range error.
    w = inputs.make("gauss8d2048", N=1_000_000, snr_db=[24.0])
    c = ctx.const(w.X, w.labels)
    z = to_dev(w.z)
    st, L = ctx.sweep(c, tx_dev(w.tx), z, w.snr_db, prec=prec, llr=True)
    ctx.sync()
    assert ctx.last_recomputed() >= 0.97 * w.N
    idx = np.sort(np.random.default_rng(3).choice(w.N, size=120, replace=False))
    got = L[:, torch.from_numpy(idx).to(L.device), :].cpu().numpy()
    ref = oracle.sweep(w.X, w.labels, w.tx[idx], w.z[idx], w.snr_db)
    assert_llr(got, ref["llr"], LLR_BAR[prec])
    assert np.isfinite(st.cpu().numpy()).all()
    tx = w.tx.astype(np.int32).copy()
    bad = w.N - 1                          # the last pair: a wave's later round
    tx[bad] = 1 << 20
    st2, L2 = ctx.sweep(c, tx_dev(tx), z, w.snr_db, prec=prec, llr=True)
    with pytest.raises(air.AirError) as e:
        ctx.sync()
    assert e.value.status == air.AIR_E_RANGE
    Lh = L2[0, bad - 2:].cpu().numpy()
    assert np.isnan(Lh[2]).all() and np.isfinite(Lh[:2]).all()
    c.close()


@pytest.mark.parametrize("prec", PRECS + ["fp32"])
def test_mi_gmi_without_llrs(ctx, prec):
    # Without LLRs only the total and the transmitted point's bit sides have
    # to stay inside the first tier's frame: at 16..24 dB on 8-D, M = 2048
    # most flagged items have only far sides starved, and they no longer go
    # to the second tier. MI/GMI still match the oracle.
    w = inputs.make("gauss8d2048", N=3000 + 37, snr_db=[16.0, 20.0, 24.0])
    c = ctx.const(w.X, w.labels)
    tx, z = tx_dev(w.tx), to_dev(w.z)
    st_l, _ = ctx.sweep(c, tx, z, w.snr_db, prec=prec, llr=True)
    ctx.sync()
    rec_l = ctx.last_recomputed()
    st, L = ctx.sweep(c, tx, z, w.snr_db, prec=prec)
    ctx.sync()
    rec = ctx.last_recomputed()
    assert L is None
    ref = oracle.sweep(w.X, w.labels, w.tx, w.z, w.snr_db, llr=False)
    print(f"{prec}: second tier {rec} items without LLRs, {rec_l} with")
    assert_stats(st.cpu().numpy(), ref["stats"], se_rel=2e-2)
    assert_stats(st_l.cpu().numpy(), ref["stats"], se_rel=2e-2)
    assert rec_l > 1000 and rec * 10 < rec_l
    c.close()


def test_call_words_start_clean(ctx):
    # the per-call words (tx-range error, second-tier counts) are zeroed by
    # the previous call's last kernel: counts and errors never carry over
    w = inputs.make("psk8x8", N=20_000, snr_db=[30.0])
    low = inputs.make("psk8x8", N=20_000, snr_db=[-2.0])
    c = ctx.const(w.X, w.labels)
    z = to_dev(w.z)

    def run(wl, tx, sync=True):
        # LLRs on: at 30 dB their far bit sides send items to the second tier
        st, _ = ctx.sweep(c, tx_dev(tx), z, wl.snr_db, prec="fp16x3", llr=True)
        if sync:
            ctx.sync()
        return st.cpu().numpy(), ctx.last_recomputed(), ctx.last_exact()

    a = run(w, w.tx)
    assert a[1] > 0
    b = run(low, low.tx)
    assert b[1] == 0 and b[2] == 0
    a2 = run(w, w.tx)
    assert a2[1:] == a[1:] and np.array_equal(a2[0], a[0])
    bad = w.tx.astype(np.int32).copy()
    bad[7] = 1 << 20
    st, _ = ctx.sweep(c, tx_dev(bad), z, w.snr_db, prec="fp16x3", llr=True)
    with pytest.raises(air.AirError):
        ctx.sync()
    assert np.isnan(st.cpu().numpy()).all()
    # the call after the failed one: its own words start at zero again
    for _ in range(3):
        b2 = run(low, low.tx)
        assert np.array_equal(b2[0], b[0]) and b2[1] == 0 and b2[2] == 0
        a3 = run(w, w.tx)
        assert np.array_equal(a3[0], a[0]) and a3[1:] == a[1:]


def test_set_stream_orders_the_workspace(ctx):
    # switching streams waits for the work issued on the old one, which the
    # next call's reuse of the workspace relies on
    w = inputs.make("psk8x8", N=50_000, snr_db=np.linspace(0.0, 20.0, 9))
    c = ctx.const(w.X, w.labels)
    tx, z = tx_dev(w.tx), to_dev(w.z)
    ref, _ = ctx.sweep(c, tx, z, w.snr_db, prec="fp16x3")
    ctx.sync()
    ref = ref.cpu().numpy()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    try:
        for k in range(4):
            ctx.set_stream(s1 if k % 2 == 0 else s2)
            st, _ = ctx.sweep(c, tx, z, w.snr_db, prec="fp16x3")
            outs.append(st)
        ctx.sync()
    finally:
        ctx.set_stream(torch.cuda.default_stream())
    torch.cuda.synchronize()
    for st in outs:
        assert np.array_equal(st.cpu().numpy(), ref, equal_nan=True)
