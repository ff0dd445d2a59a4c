"""GPU auxiliary-channel rates (air_noise_var, air_llr_aux, air_mi_gmi_aux)
against the oracle on the same seeded inputs."""
import math

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


def _block(seed, M, D, N, snr_db):
    X, lab = inputs.random_constellation(seed, M, D)
    tx, z = inputs.random_block(seed + 1, M, N, D)
    s2 = oracle.sigma2(X, snr_db)
    Y = (X[tx] + math.sqrt(s2) * z.astype(np.float64)).astype(np.float32)
    return X, lab, tx, Y, s2


@pytest.mark.parametrize("M,D,N", [(2, 1, 1), (16, 4, 1000), (64, 3, 4097), (256, 16, 333), (4096, 12, 20_001)])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noise_var_matches_oracle(ctx, M, D, N, prec):
    X, lab, tx, Y, s2 = _block(M * 7 + D, M, D, N, 9.0)
    Yp = Y.astype(np.float64) if prec == "fp64" else Y
    c = ctx.const(X, lab)
    v = ctx.noise_var(c, to_dev(Yp), tx_dev(tx), prec)
    v2 = ctx.noise_var(c, to_dev(Yp), tx_dev(tx), prec)
    ctx.sync()
    ref = oracle.noise_var(X, Y.astype(np.float64), tx)
    np.testing.assert_allclose(v.cpu().numpy(), ref, rtol=1e-12, atol=0)
    assert torch.equal(v, v2)                       # fixed-order sums: identical bits
    c.close()


@pytest.mark.parametrize("name,N,prec", [("psk8x8", 20_000, "fp16x3"), ("psk8x8", 3001, "fp32"),
                                         ("gauss8d2048", 2000, "fp16x3"), ("pmqpsk", 5000, "fp64")])
@pytest.mark.parametrize("ratio", [0.7, 1.0, 1.6])
def test_mi_gmi_aux_matches_oracle(ctx, name, N, prec, ratio):
    w = inputs.make(name, N=N)
    snr_db = float(w.snr_db[len(w.snr_db) // 2])
    s2 = oracle.sigma2(w.X, snr_db)
    dt = np.float64 if prec == "fp64" else np.float32
    Y = (w.X[w.tx] + math.sqrt(s2) * w.z.astype(np.float64)).astype(dt)
    c = ctx.const(w.X, w.labels)
    st, L = ctx.mi_gmi_aux(c, to_dev(Y), tx_dev(w.tx), ratio * s2, prec, llr=True)
    L2 = ctx.llr_aux(c, to_dev(Y), ratio * s2, prec)
    ctx.sync()
    ref = oracle.evaluate_aux(w.X, w.labels, Y.astype(np.float64), ratio * s2, tx=w.tx)
    tol = 1e-11 if prec == "fp64" else None
    assert_stats(st.cpu().numpy()[None], ref["stats"][None], **({"tol": tol} if tol else {}))
    assert_llr(L.cpu().numpy(), ref["llr"], **({"rel": tol} if tol else {}))
    assert torch.equal(L, L2)
    c.close()


def test_aux_at_true_variance_equals_snr_call(ctx):
    w = inputs.make("psk8x8", N=10_000)
    snr_db = 6.0
    s2 = oracle.sigma2(w.X, snr_db)
    Y = (w.X[w.tx] + math.sqrt(s2) * w.z.astype(np.float64)).astype(np.float32)
    c = ctx.const(w.X, w.labels)
    a, _ = ctx.mi_gmi(c, to_dev(Y), tx_dev(w.tx), snr_db, "fp16x3")
    b, _ = ctx.mi_gmi_aux(c, to_dev(Y), tx_dev(w.tx), s2, "fp16x3")
    ctx.sync()
    np.testing.assert_allclose(a.cpu().numpy(), b.cpu().numpy(), rtol=0, atol=1e-12)
    c.close()


def test_aux_rates_end_to_end(ctx):
    w = inputs.make("psk8x8", N=50_000)
    snr_db = 8.0
    s2 = oracle.sigma2(w.X, snr_db)
    Y = (w.X[w.tx] + math.sqrt(s2) * w.z.astype(np.float64)).astype(np.float32)
    c = ctx.const(w.X, w.labels)
    r = ctx.aux_rates(c, to_dev(Y), tx_dev(w.tx), "fp16x3")
    ref_var = oracle.noise_var(w.X, Y.astype(np.float64), w.tx)
    assert r["sigma2"] == pytest.approx(ref_var[-1], rel=1e-12)
    ref = oracle.evaluate_aux(w.X, w.labels, Y.astype(np.float64), ref_var[-1], tx=w.tx, llr=False)
    assert abs(r["mi"] - ref["stats"][0]) <= 1e-4 and abs(r["gmi"] - ref["stats"][1]) <= 1e-4
    assert r["ngmi"] == pytest.approx(oracle.ngmi(ref["stats"][1], 6), abs=2e-5)
    np.testing.assert_allclose(r["var"], ref_var[:-1], rtol=1e-12)
    assert r["se_ngmi"] == pytest.approx(r["se_gmi"] / 6, rel=1e-15)
    assert abs(r["se_gmi"] - ref["stats"][3]) <= 1e-2 * ref["stats"][3] + 1e-6
    c.close()


def test_aux_rates_range_error(ctx):
    X, lab, tx, Y, s2 = _block(92, 16, 2, 100, 5.0)
    c = ctx.const(X, lab)
    badtx = tx.astype(np.int64).copy()
    badtx[7] = 99
    with pytest.raises(air.AirError) as e:
        ctx.aux_rates(c, to_dev(Y), tx_dev(badtx), "fp32")
    assert e.value.status == air.AIR_E_RANGE
    # the context stays usable
    r = ctx.aux_rates(c, to_dev(Y), tx_dev(tx), "fp32")
    assert r["sigma2"] == pytest.approx(oracle.noise_var(X, Y.astype(np.float64), tx)[-1], rel=1e-12)
    c.close()


def test_aux_errors(ctx):
    X, lab, tx, Y, s2 = _block(91, 16, 2, 100, 5.0)
    c = ctx.const(X, lab)
    for bad in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(air.AirError) as e:
            ctx.llr_aux(c, to_dev(Y), bad)
        assert e.value.status == air.AIR_E_INVAL
    badtx = tx.astype(np.int64).copy()
    badtx[3] = 16
    v = ctx.noise_var(c, to_dev(Y), tx_dev(badtx))
    with pytest.raises(air.AirError) as e:
        ctx.sync()
    assert e.value.status == air.AIR_E_RANGE
    assert np.isnan(v.cpu().numpy()).all()
    c.close()
