"""Per-SNR summaries computed by libair on the host (air_ngmi, air_hd_rates,
air_fec_net) against the oracle's own implementation of the same readings.
These calls are host arithmetic on host arrays, so they run without a GPU."""
import math

import numpy as np
import pytest

import oracle
from paper_2108_07001_amd import air


def test_ngmi_table_matches_oracle():
    rng = np.random.default_rng(5)
    for m in (1, 2, 6, 11, 12):
        st = np.column_stack([rng.uniform(0, m, 9), rng.uniform(-0.01, m, 9),
                              rng.uniform(0, 1e-2, 9), rng.uniform(0, 1e-2, 9)])
        st[3, 3] = np.nan                       # a saturated point's SE
        got, ref = air.ngmi_table(st, m), oracle.ngmi_table(st, m)
        np.testing.assert_allclose(got, ref, rtol=1e-15, atol=1e-15)
        assert np.isnan(got[3, 1]) and np.isnan(ref[3, 1])
    assert air.ngmi(6.0, 6) == 1.0 and air.ngmi(0.0, 6) == 0.0


def test_hd_rates_match_oracle():
    rng = np.random.default_rng(6)
    N, m = 1_000_003, 11
    sym = rng.integers(0, N, 12)
    bits = np.minimum(sym * rng.integers(1, m + 1, 12), N * m)
    counts = np.column_stack([sym, bits]).astype(np.uint64)
    counts[0] = [0, 0]                          # no errors: Q undefined
    counts[1] = [N, N * m]                      # BER 1: Q undefined
    got, ref = air.hd_rates(counts, N, m), oracle.hd_rates(counts, N, m)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    np.testing.assert_allclose(got[ok], ref[ok], rtol=1e-12, atol=0)
    assert math.isnan(got[0, 2]) and math.isnan(got[1, 2])
    np.testing.assert_array_equal(got[:, :2], ref[:, :2])
    # just below BER 0.5, erfcinv(2 BER) is ill-conditioned: both sides agree
    # with the erfc round trip to the argument's rounding
    near = air.hd_rates([[N, N * m // 2]], N, m)[0]
    assert near[0] < 0.5
    x = 10 ** (near[2] / 20) / math.sqrt(2.0)
    assert abs(math.erfc(x) - 2 * near[0]) <= 4e-16


def test_fec_net_matches_oracle():
    rng = np.random.default_rng(7)
    ber = np.concatenate([10 ** rng.uniform(-6, -0.4, 40), [0.0, 3.8e-3, 2.0e-2, np.nan, 0.5]])
    codes = [([0.067, 0.2], [3.8e-3, 2.0e-2]), ([0.2, 0.067], [2.0e-2, 3.8e-3]),
             ([0.2, 0.2], [1e-2, 1e-2]), ([0.0], [1e-3])]
    for m in (2, 3, 6):
        for oh, th in codes:
            got = air.fec_net(ber, m, oh, th, symbol_rate=1e9)
            ref = oracle.fec_net(ber, m, oh, th, symbol_rate=1e9)
            np.testing.assert_array_equal(got["pass"], ref["pass"])
            np.testing.assert_array_equal(got["code"], ref["best"])
            np.testing.assert_allclose(got["net"], ref["net"], rtol=1e-15, atol=0)


def test_fec_net_stride_reads_the_ber_column():
    lib = air.load()
    rates = np.array([[1e-3, 0.1, 9.0], [3e-2, 0.5, 5.0]])
    oh = np.array([0.067, 0.2])
    th = np.array([3.8e-3, 2.0e-2])
    pas = np.empty((2, 2), dtype=np.int32)
    net = np.empty(2)
    code = np.empty(2, dtype=np.int32)
    st = lib.air_fec_net(rates.ctypes.data, 3, 2, 4, oh.ctypes.data, th.ctypes.data, 2, 1.0,
                         pas.ctypes.data, net.ctypes.data, code.ctypes.data)
    assert st == air.AIR_OK
    assert pas.tolist() == [[1, 1], [0, 0]] and code.tolist() == [0, -1]
    assert net[0] == pytest.approx(4 / 1.067) and net[1] == 0.0


def test_host_summaries_reject_bad_arguments():
    lib = air.load()
    st4 = np.zeros((1, 4))
    out = np.empty(8)
    assert lib.air_ngmi(None, 1, 4, out.ctypes.data) == air.AIR_E_INVAL
    assert lib.air_ngmi(st4.ctypes.data, 0, 4, out.ctypes.data) == air.AIR_E_INVAL
    assert lib.air_ngmi(st4.ctypes.data, 1, 0, out.ctypes.data) == air.AIR_E_INVAL
    cnt = np.zeros(2, dtype=np.uint64)
    assert lib.air_hd_rates(cnt.ctypes.data, 1, 0, 4, out.ctypes.data) == air.AIR_E_INVAL
    assert lib.air_hd_rates(None, 1, 10, 4, out.ctypes.data) == air.AIR_E_INVAL
    b = np.array([1e-3])
    for oh, th, rate in (([-0.1], [1e-2], 1.0), ([math.inf], [1e-2], 1.0), ([0.1], [math.nan], 1.0),
                         ([0.1], [-1.0], 1.0), ([0.1], [1e-2], -1.0), ([0.1], [1e-2], math.nan)):
        with pytest.raises(air.AirError):
            air.fec_net(b, 4, oh, th, symbol_rate=rate)
    assert lib.air_fec_net(b.ctypes.data, 0, 1, 4, b.ctypes.data, b.ctypes.data, 1, 1.0,
                           None, None, None) == air.AIR_E_INVAL
    assert lib.air_aux_rates(None, None, None, None, 1, 1, None, None) == air.AIR_E_INVAL
    assert lib.air_server_destroy(None) == air.AIR_E_INVAL
