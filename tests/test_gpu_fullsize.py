"""GPU parity at the full workload sizes, in the launch configuration bench.py
times (one air_sweep over all samples and SNR points).

8-PSK^2 is checked element by element against the FP64 oracle on the whole
workload. For the two large Gaussian sets the oracle cannot run on the whole
workload within a test, so
(a) MI/GMI are compared with statistics the oracle wrote beforehand
    (tests/golden/make_golden.py): the whole 8-D, M = 2048 sweep (4e6 samples,
    11 SNR points) and the 12-D, M = 4096 sweep on its first 2^20 samples at
    all 41 SNR points, each SNR point to 1e-4 bit;
(b) the LLRs of a random sample of received points are checked one by one
    against the oracle run on exactly those points;
(c) the full-size MI/GMI must equal the sample-weighted combination of two
    calls on the halves of the block (the sums are additive; it catches lost
    or doubled tiles, lists and partial sums). A sample's products are the
    same in both calls, but which tier finishes it can differ: a wave of the
    large sets' first tier hands its later rounds at an SNR point to the
    second tier once a round has mostly been flagged, and the rounds a wave
    sees depend on the block size. The two tiers agree to FP32 rounding
    (~1e-7 bit per sample), so the combination is held to 1e-7 bit; a lost
    or doubled tile of 32 samples moves the mean by ~1e-5."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2108_07001_amd import air, inputs
from tests.helpers import assert_llr, assert_stats, to_dev, tx_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = air.Context(0)
    yield c
    c.close()


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def psk8x8_ref():
    w = inputs.make("psk8x8")
    return w, oracle.sweep(w.X, w.labels, w.tx, w.z, w.snr_db)


@pytest.mark.parametrize("prec", ["fp16x3", "bf16x3"])
def test_psk8x8_full_size_elementwise(ctx, psk8x8_ref, prec):
    w, ref = psk8x8_ref
    c = ctx.const(w.X, w.labels)
    st, L = ctx.sweep(c, tx_dev(w.tx), to_dev(w.z, torch.float32), w.snr_db, prec=prec, llr=True)
    ctx.sync()
    assert_stats(st.cpu().numpy(), ref["stats"])
    assert_llr(L.cpu().numpy(), ref["llr"])
    c.close()


@pytest.mark.parametrize("case", ["gauss8d2048_full", "gauss12d4096_prefix"])
@pytest.mark.parametrize("prec", ["fp16x3", "bf16x3", "fp32"])
def test_large_sets_against_stored_oracle_stats(ctx, case, prec):
    g = json.load(open(os.path.join(GOLDEN, case + ".json")))
    w = inputs.make(g["workload"], N=g["N"])
    assert [float(s) for s in w.snr_db] == g["snr_db"]
    c = ctx.const(w.X, w.labels)
    st, _ = ctx.sweep(c, tx_dev(w.tx), to_dev(w.z, torch.float32), w.snr_db, prec=prec)
    ctx.sync()
    st = st.cpu().numpy()
    ref = np.asarray(g["stats"])
    d = np.abs(st[:, :2] - ref[:, :2])
    print(f"{case} {prec}: N={w.N} S={len(w.snr_db)} max|dMI| {d[:, 0].max():.2e} "
          f"max|dGMI| {d[:, 1].max():.2e} bit, recomputed {ctx.last_recomputed()}")
    assert_stats(st, ref, se_rel=1e-2)
    c.close()


def _halves_consistent(ctx, c, w, st_full, prec):
    """Full-size MI/GMI against the N-weighted mean of the two halves' values."""
    N = w.N
    h = N // 2
    parts = []
    for lo, hi in ((0, h), (h, N)):
        # with LLRs, as the full call: which bit sides must stay inside the
        # first tier's frame depends on whether LLRs are written
        st, L = ctx.sweep(c, tx_dev(w.tx[lo:hi]), to_dev(np.ascontiguousarray(w.z[lo:hi]), torch.float32),
                          w.snr_db, prec=prec, llr=True)
        parts.append((hi - lo, st.cpu().numpy()))
        del L
        torch.cuda.empty_cache()
    comb = sum(n * s[:, :2] for n, s in parts) / N
    np.testing.assert_allclose(st_full[:, :2], comb, rtol=0, atol=1e-7)


@pytest.mark.parametrize("prec", ["fp16x3", "bf16x3"])
@pytest.mark.parametrize("name,nsample", [("gauss8d2048", 400), ("gauss12d4096", 150)])
def test_large_sets_full_size_sampled(ctx, name, nsample, prec):
    w = inputs.make(name)
    c = ctx.const(w.X, w.labels)
    tx = tx_dev(w.tx)
    z = to_dev(w.z, torch.float32)
    st, L = ctx.sweep(c, tx, z, w.snr_db, prec=prec, llr=True)
    ctx.sync()
    st = st.cpu().numpy()
    idx = np.sort(np.random.default_rng(17).choice(w.N, size=nsample, replace=False))
    got = L[:, torch.from_numpy(idx).to(L.device), :].cpu().numpy()
    del L
    torch.cuda.empty_cache()
    ref = oracle.sweep(w.X, w.labels, w.tx[idx], w.z[idx], w.snr_db)
    print(f"{name} {prec}: {nsample} sampled points x {len(w.snr_db)} SNR, "
          f"MI {st[0, 0]:.4f}..{st[-1, 0]:.4f} bit, recomputed {ctx.last_recomputed()}")
    assert_llr(got, ref["llr"])
    assert np.isfinite(st).all()
    _halves_consistent(ctx, c, w, st, prec)
    c.close()


def test_psk8x8_full_size_maxlog_and_hard_decisions(ctx):
    """The max-log sweep and the hard-decision sweep at the full workload
    size, against the oracle's forms on the whole workload."""
    w = inputs.make("psk8x8")
    c = ctx.const(w.X, w.labels)
    txd, zd = tx_dev(w.tx), to_dev(w.z, torch.float32)
    st, L = ctx.sweep_maxlog(c, txd, zd, w.snr_db, prec="fp16x3", llr=True)
    counts, _ = ctx.hard_sweep(c, txd, zd, w.snr_db)
    ctx.sync()
    ref = oracle.sweep_maxlog(w.X, w.labels, w.tx, w.z, w.snr_db)
    st = st.cpu().numpy()
    assert np.isnan(st[:, 0]).all()
    assert np.max(np.abs(st[:, 1] - ref["stats"][:, 1])) <= 1e-4
    assert_llr(L.cpu().numpy(), ref["llr"])
    del L
    torch.cuda.empty_cache()
    hd = oracle.hard_decisions_sweep(w.X, w.labels, w.tx, w.z.astype(np.float32), w.snr_db)
    np.testing.assert_array_equal(counts.cpu().numpy().astype(np.uint64), hd["counts"])
    c.close()
