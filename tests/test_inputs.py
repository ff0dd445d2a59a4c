"""Seeded workload generator: shapes, determinism, prefix property, labellings."""
import math

import numpy as np
import pytest

from paper_2108_07001_amd import inputs


@pytest.mark.parametrize("name", ["pmqpsk", "psk8x8", "gauss8d2048", "gauss12d4096"])
def test_shapes_and_labels(name):
    cfg = inputs.CONFIGS[name]
    w = inputs.make(name, N=1000)
    assert w.X.shape == (cfg["M"], cfg["D"]) and w.X.dtype == np.float64
    assert sorted(w.labels.tolist()) == list(range(cfg["M"]))
    assert w.tx.dtype == np.uint32 and w.tx.max() < cfg["M"]
    assert w.z.shape == (1000, cfg["D"])
    assert w.z.dtype == (np.float64 if cfg["noise"] == "f64" else np.float32)
    assert list(w.snr_db) == cfg["snr_db"]
    # every stand-in has unit average energy except PM-QPSK (+-1/sqrt2 per dim)
    es = np.mean(np.sum(w.X ** 2, axis=1))
    assert es == pytest.approx(2.0 if name == "pmqpsk" else 1.0, rel=1e-12)


def test_prefix_and_determinism():
    a = inputs.make("psk8x8", N=5000)
    b = inputs.make("psk8x8", N=1234)
    np.testing.assert_array_equal(a.tx[:1234], b.tx)
    np.testing.assert_array_equal(a.z[:1234], b.z)
    c = inputs.make("psk8x8", N=1234)
    np.testing.assert_array_equal(b.z, c.z)
    # chunked drawing equals one draw
    r1, r2 = np.random.default_rng(3), np.random.default_rng(3)
    np.testing.assert_array_equal(inputs.noise(r1, 3000, 3, False, chunk=700),
                                  inputs.noise(r2, 3000, 3, False, chunk=1 << 20))


def test_named_constellations():
    X, lab = inputs.pm_qpsk()
    for l in range(16):
        for d in range(4):
            assert X[l, d] == pytest.approx((1 - 2 * ((l >> d) & 1)) / math.sqrt(2))
    X, lab = inputs.constellation("psk8x8")
    assert np.allclose(np.sum(X[:, :2] ** 2, axis=1), 0.5)
    X, lab = inputs.constellation("gauss8d2048")
    assert (lab == np.arange(2048)).all()
    X, lab = inputs.constellation("gauss12d4096")
    assert not (lab == np.arange(4096)).all()


def test_serving_stream():
    jobs = inputs.serving_jobs(500)
    t = np.array([j.arrival_s for j in jobs])
    assert (np.diff(t) > 0).all()
    assert 0.15 < t[-1] < 0.35                    # 500 jobs at 2000/s
    for j in jobs:
        assert j.M in (16, 64, 256, 2048) and j.D == inputs.SERVING["D_for_M"][j.M]
        assert 1000 <= j.N <= 1_000_000 and 0.0 <= j.snr_db <= 25.0
    pool = inputs.serving_pool(64)
    assert len(pool) == 8 and pool[0][0].shape == (64, 4)
