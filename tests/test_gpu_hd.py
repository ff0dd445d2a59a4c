"""GPU hard decisions (air_hard_decide / air_hard_sweep) against the oracle.

Both sides take the nearest-point decision in FP32 with the same operation
order, so decisions and error counts are compared exactly; a differing
decision is accepted only at a tie within FP32 rounding (checked in FP64)."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2108_07001_amd import air, inputs
from tests.helpers import to_dev, tx_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = air.Context(0)
    yield c
    c.close()


def _check_decisions(X, Y, got, ref):
    diff = np.nonzero(got != ref)[0]
    for n in diff:                     # only ties within FP32 rounding may differ
        y = Y[n].astype(np.float64)
        dg = np.sum((y - X[got[n]]) ** 2)
        dr = np.sum((y - X[ref[n]]) ** 2)
        assert abs(dg - dr) <= 1e-5 * max(dr, 1e-6), (n, got[n], ref[n], dg, dr)
    return len(diff)


@pytest.mark.parametrize("name,N", [("psk8x8", 40_000), ("pmqpsk", 20_000), ("gauss8d2048", 3000)])
def test_hard_sweep_matches_oracle(ctx, name, N):
    w = inputs.make(name, N=N)
    z32 = np.ascontiguousarray(w.z, dtype=np.float32)
    c = ctx.const(w.X, w.labels)
    counts, dec = ctx.hard_sweep(c, tx_dev(w.tx), to_dev(z32), w.snr_db, decided=True)
    ctx.sync()
    ref = oracle.hard_decisions_sweep(w.X, w.labels, w.tx, z32, w.snr_db, decided=True)
    got = dec.cpu().numpy().astype(np.uint32)
    ndiff = 0
    for s in range(len(w.snr_db)):
        sf = np.float32(math.sqrt(oracle.sigma2(w.X, w.snr_db[s])))
        Y = (sf * z32 + w.X[w.tx].astype(np.float32)).astype(np.float32)
        ndiff += _check_decisions(w.X, Y, got[s], ref["decided"][s])
    got_counts = counts.cpu().numpy().astype(np.uint64)
    # the counts always match the kernel's own decisions (counted here on the host) ...
    np.testing.assert_array_equal(got_counts, _counts_of(w.labels, w.tx, got))
    # ... and the oracle's counts whenever no decision differs at a tie
    if ndiff == 0:
        np.testing.assert_array_equal(got_counts, ref["counts"])
    c.close()


def _counts_of(labels, tx, decided):
    """[symbol errors, bit errors] per row of `decided` (S x N point indices)."""
    lab = np.asarray(labels, dtype=np.uint32)
    t = lab[np.asarray(tx)]
    out = np.zeros((decided.shape[0], 2), dtype=np.uint64)
    for s in range(decided.shape[0]):
        d = lab[decided[s]]
        out[s, 0] = np.count_nonzero(decided[s] != np.asarray(tx))
        x = (d ^ t).astype(np.uint32)
        out[s, 1] = int(np.unpackbits(x.view(np.uint8)).sum())
    return out


def test_hard_decide_given_block(ctx):
    X, lab = inputs.random_constellation(61, 256, 4)
    tx, z = inputs.random_block(62, 256, 5001, 4)
    sigma = math.sqrt(oracle.sigma2(X, 11.0))
    Y = (X[tx] + sigma * z.astype(np.float64)).astype(np.float32)
    c = ctx.const(X, lab)
    dec, counts = ctx.hard_decide(c, to_dev(Y), tx_dev(tx))
    dec_only, none = ctx.hard_decide(c, to_dev(Y))
    ctx.sync()
    ref = oracle.hard_decisions(X, lab, Y, tx)
    assert none is None
    assert _check_decisions(X, Y, dec.cpu().numpy().astype(np.uint32), ref["decided"]) == 0
    assert torch.equal(dec, dec_only)
    np.testing.assert_array_equal(counts.cpu().numpy().astype(np.uint64), ref["counts"])
    c.close()


@pytest.mark.parametrize("M,D,N", [(2, 1, 1), (4, 2, 257), (16, 3, 1000), (4096, 12, 300)])
def test_hard_decide_shapes(ctx, M, D, N):
    X, lab = inputs.random_constellation(M + D, M, D)
    tx, z = inputs.random_block(M * D, M, N, D)
    Y = (X[tx] + 0.3 * z.astype(np.float64)).astype(np.float32)
    c = ctx.const(X, lab)
    dec, counts = ctx.hard_decide(c, to_dev(Y), tx_dev(tx))
    ctx.sync()
    ref = oracle.hard_decisions(X, lab, Y, tx)
    assert _check_decisions(X, Y, dec.cpu().numpy().astype(np.uint32), ref["decided"]) == 0
    np.testing.assert_array_equal(counts.cpu().numpy().astype(np.uint64), ref["counts"])
    c.close()


def test_hard_decide_invalid_tx(ctx):
    X, lab = inputs.random_constellation(63, 16, 2)
    tx, z = inputs.random_block(64, 16, 100, 2)
    bad = tx.astype(np.int64).copy()
    bad[7] = 16
    c = ctx.const(X, lab)
    ctx.hard_decide(c, to_dev(z.astype(np.float32)), tx_dev(bad))
    with pytest.raises(air.AirError) as e:
        ctx.sync()
    assert e.value.status == air.AIR_E_RANGE
    c.close()


def _decide_exact(ctx, X, lab, Y, tx):
    c = ctx.const(X, lab)
    dec, counts = ctx.hard_decide(c, to_dev(Y), tx_dev(tx))
    ctx.sync()
    ref = oracle.hard_decisions(X, lab, Y, tx)
    # both sides run the FP32 procedure: identical decisions, not just ties
    np.testing.assert_array_equal(dec.cpu().numpy().astype(np.uint32), ref["decided"])
    np.testing.assert_array_equal(counts.cpu().numpy().astype(np.uint64), ref["counts"])
    c.close()


def test_hard_decide_near_ties(ctx):
    # received points at (and within a few ulps of) midpoints of pairs of
    # constellation points: the matrix-core path must hand these to the FP32
    # procedure and decide exactly as it does
    rng = np.random.default_rng(71)
    X, lab = inputs.random_constellation(72, 64, 4)
    a = rng.integers(0, 64, 4000)
    b = rng.integers(0, 64, 4000)
    mid = ((X[a] + X[b]) / 2.0).astype(np.float32)
    jitter = rng.integers(-3, 4, mid.shape).astype(np.float32)
    Y = np.nextafter(mid, np.where(jitter > 0, np.inf, -np.inf).astype(np.float32))
    Y = np.where(jitter == 0, mid, Y).astype(np.float32)
    Y = np.concatenate([mid, Y]).astype(np.float32)
    tx = np.concatenate([a, b]).astype(np.int64)
    _decide_exact(ctx, X, lab, Y, tx)


@pytest.mark.parametrize("scale", [1e-2, 0.3, 8.0, 200.0])
def test_hard_decide_coordinate_ranges(ctx, scale):
    # largest |x| outside [1/16, 64] takes the vector kernel, inside the
    # matrix cores; both decide as the FP32 procedure
    X, lab = inputs.random_constellation(73, 256, 6)
    X = X * scale
    tx, z = inputs.random_block(74, 256, 3000, 6)
    sigma = math.sqrt(oracle.sigma2(X, 4.0))
    Y = (X[tx] + sigma * z.astype(np.float64)).astype(np.float32)
    _decide_exact(ctx, X, lab, Y, tx)


@pytest.mark.parametrize("M,D,snr", [(1024, 6, -3.0), (32, 2, 0.0), (128, 16, 10.0)])
def test_hard_decide_low_snr_many_points(ctx, M, D, snr):
    X, lab = inputs.random_constellation(M + 3 * D, M, D)
    tx, z = inputs.random_block(M + 5 * D, M, 2500, D)
    sigma = math.sqrt(oracle.sigma2(X, snr))
    Y = (X[tx] + sigma * z.astype(np.float64)).astype(np.float32)
    _decide_exact(ctx, X, lab, Y, tx)


@pytest.mark.parametrize("N,S", [(1, 3), (33, 70), (5000, 70)])
def test_hard_sweep_launch_edges(ctx, N, S):
    # tiny blocks (one sample, one ragged tile pair) and more SNR points than
    # one launch takes, on the matrix-core path (M = 64)
    w = inputs.make("psk8x8", N=N, snr_db=np.linspace(-4.0, 30.0, S))
    z32 = np.ascontiguousarray(w.z, dtype=np.float32)
    c = ctx.const(w.X, w.labels)
    counts, dec = ctx.hard_sweep(c, tx_dev(w.tx), to_dev(z32), w.snr_db, decided=True)
    ctx.sync()
    ref = oracle.hard_decisions_sweep(w.X, w.labels, w.tx, z32, w.snr_db, decided=True)
    np.testing.assert_array_equal(dec.cpu().numpy().astype(np.uint32), ref["decided"])
    np.testing.assert_array_equal(counts.cpu().numpy().astype(np.uint64), ref["counts"])
    c.close()


def test_hard_decide_extreme_inputs(ctx):
    # NaN, infinite and huge received points and one at the origin among
    # ordinary ones: the matrix-core path (M = 64) decides them as the FP32
    # procedure does (an undecidable point keeps label 0)
    X, lab = inputs.random_constellation(81, 64, 4)
    tx, z = inputs.random_block(82, 64, 250, 4)
    Y = (X[tx] + 0.2 * z.astype(np.float64)).astype(np.float32)
    odd = np.array([[np.nan, 0, 0, 0], [1e20, 1e20, 0, 0], [-1e19, 3, 0, 1], [1e-30, 0, 0, 0],
                    [3e18, -2e18, 1e18, 0], [np.inf, 0, 0, 0], [0, 0, 0, 0]], dtype=np.float32)
    Y[:len(odd)] = odd
    c = ctx.const(X, lab)
    dec, _ = ctx.hard_decide(c, to_dev(Y))
    ctx.sync()
    ref = oracle.hard_decisions(X, lab, Y)
    np.testing.assert_array_equal(dec.cpu().numpy().astype(np.uint32), ref["decided"])
    c.close()
