"""GPU tests of the serving loop (air_server_*): parity with the FP64 oracle,
agreement with the one-shot entry points, bitwise alone-vs-mix identity,
admission under the footprint budget, latency stamps and error paths."""
import time

import numpy as np
import pytest
import torch

import oracle
from paper_2108_07001_amd import air, inputs
from tests.helpers import assert_llr, assert_stats, to_dev, tx_dev

pytestmark = pytest.mark.gpu

LLR_BAR = {"fp16x3": 1e-3, "bf16x3": 1e-3}
MIX = [(16, 2), (64, 4), (256, 4), (2048, 8)]     # (M, D) of the serving mix


@pytest.fixture(scope="module")
def ctx():
    c = air.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def consts(ctx):
    out = {}
    for i, (M, D) in enumerate(MIX):
        X, lab = inputs.random_constellation(100 + i, M, D)
        out[M] = (X, lab, ctx.const(X, lab))
    return out


def _block(M, D, N, seed):
    tx, z = inputs.random_block(seed, M, N, D)
    return tx.astype(np.int32), np.ascontiguousarray(z, dtype=np.float32)


def _received(X, tx, z, snr_db):
    """y = x_t + sigma z in float32 (the input of the one-shot entry point)."""
    s = np.sqrt(oracle.sigma2(X, snr_db))
    return np.ascontiguousarray((X[tx] + s * z.astype(np.float64)).astype(np.float32))


def _run_alone(sv, job):
    jid = sv.submit(**job)
    res = sv.results()
    assert len(res) == 1 and res[0]["id"] == jid
    return res[0]


@pytest.mark.parametrize("prec", ["fp16x3", "bf16x3"])
def test_serve_mi_gmi_only_high_snr(ctx, consts, prec):
    """A job without LLRs at 22 dB on the 2048-point set: only the total and
    the transmitted point's bit sides have to stay in the first tier's frame,
    so far fewer items reach the second tier; MI/GMI still match the oracle."""
    X, lab, c = consts[2048]
    N = 1201
    tx, z = _block(2048, 8, N, 11)
    sv = ctx.server(1 << 28)
    L = torch.empty((N, c.m), device=ctx.torch_device)
    r_l = _run_alone(sv, dict(c=c, inp=to_dev(z), tx=tx_dev(tx), snr_db=22.0, prec=prec, noise=True, llr=L))
    r = _run_alone(sv, dict(c=c, inp=to_dev(z), tx=tx_dev(tx), snr_db=22.0, prec=prec, noise=True))
    sv.close()
    ref = oracle.sweep(X, lab, tx.astype(np.uint32), z, [22.0], llr=False)
    for res in (r, r_l):
        assert res["status"] == air.AIR_OK
        assert_stats(np.array([_stats(res)]), ref["stats"], se_rel=2e-2)
    print(f"{prec}: recomputed {r['recomputed']} without LLRs, {r_l['recomputed']} with")
    assert r_l["recomputed"] > 500 and r["recomputed"] * 10 < r_l["recomputed"]


@pytest.mark.parametrize("prec", ["fp16x3", "bf16x3"])
@pytest.mark.parametrize("M,D", MIX)
def test_serve_oracle_parity(ctx, consts, prec, M, D):
    """Noise-mode jobs (y formed on the device) against the FP64 oracle."""
    X, lab, c = consts[M]
    N = 3001 if M < 2048 else 1201           # several tiles and a ragged tail
    tx, z = _block(M, D, N, 7 + M)
    snr = 9.5
    sv = ctx.server(1 << 28)
    L = torch.full((N, c.m), float("nan"), device=ctx.torch_device)
    r = _run_alone(sv, dict(c=c, inp=to_dev(z), tx=tx_dev(tx), snr_db=snr, prec=prec,
                            noise=True, llr=L))
    sv.close()
    ref = oracle.sweep(X, lab, tx.astype(np.uint32), z, [snr])
    assert r["status"] == air.AIR_OK
    st = np.array([[r["mi"], r["gmi"], r["se_mi"], r["se_gmi"]]])
    assert_stats(st, ref["stats"], se_rel=2e-2)
    assert_llr(L.cpu().numpy(), ref["llr"][0], LLR_BAR[prec])


@pytest.mark.parametrize("M,D", MIX)
def test_serve_matches_one_shot(ctx, consts, M, D):
    """Same received block through air_mi_gmi and through the server. The
    one-shot kernel puts each sample's terms in a frame shifted by a rounded
    per-sample constant, the serving kernel in the fixed frame: the results
    agree to FP32 rounding of the terms."""
    X, lab, c = consts[M]
    N = 4099
    tx, z = _block(M, D, N, 11 + M)
    snr = 6.0
    Y = _received(X, tx, z, snr)
    st1, L1 = ctx.mi_gmi(c, to_dev(Y), tx_dev(tx), snr, prec="fp16x3", llr=True)
    ctx.sync()
    sv = ctx.server(1 << 28)
    L2 = torch.empty((N, c.m), device=ctx.torch_device)
    r = _run_alone(sv, dict(c=c, inp=to_dev(Y), tx=tx_dev(tx), snr_db=snr, prec="fp16x3", llr=L2))
    sv.close()
    assert_llr(L2.cpu().numpy(), L1.cpu().numpy(), 1e-4)
    st1 = st1.cpu().numpy()
    st2 = np.array([r["mi"], r["gmi"], r["se_mi"], r["se_gmi"]])
    assert np.allclose(st1, st2, rtol=1e-6, atol=1e-7), (st1, st2)


def _mix_jobs(ctx, consts, n, seed, host_share=0.5):
    """n jobs of random constellation, N (1 .. 20000, ragged), SNR and buffer
    placement; LLR buffers are preallocated (a quarter of the jobs ask for
    MI/GMI only, which changes which bit sides must stay in the FP32 frame)."""
    r = np.random.default_rng(seed)
    jobs = []
    for i in range(n):
        M, D = MIX[r.integers(0, len(MIX))]
        X, lab, c = consts[M]
        N = int(r.choice([1, 31, 32, 33, 777, 2048, 5000, 20000])) if M < 2048 else int(r.choice([1, 33, 1500]))
        tx, z = _block(M, D, N, int(r.integers(1 << 30)))
        host = r.random() < host_share
        noise = bool(r.random() < 0.5)
        snr = float(r.uniform(0.0, 25.0))
        inp = z if noise else _received(X, tx, z, snr)
        if host:
            inp_b = torch.from_numpy(inp).pin_memory()
            tx_b = torch.from_numpy(tx).pin_memory()
            L = torch.empty((N, c.m), dtype=torch.float32).pin_memory()
        else:
            inp_b, tx_b = to_dev(inp), tx_dev(tx)
            L = torch.empty((N, c.m), device=ctx.torch_device)
        if r.random() < 0.25:
            L = None
        jobs.append(dict(c=c, inp=inp_b, tx=tx_b, snr_db=snr, prec=str(r.choice(["fp16x3", "bf16x3"])),
                         noise=noise, llr=L, tag=i))
    return jobs


def _stats(r):
    return np.array([r["mi"], r["gmi"], r["se_mi"], r["se_gmi"]])


def test_alone_vs_mix_bitwise(ctx, consts):
    jobs = _mix_jobs(ctx, consts, 40, seed=5)
    sv = ctx.server(1 << 28)
    alone = {}
    for jb in jobs:
        r = _run_alone(sv, jb)
        assert r["status"] == air.AIR_OK
        alone[jb["tag"]] = (_stats(r), None if jb["llr"] is None else jb["llr"].cpu().clone())
    # the same jobs, submitted together in another order
    order = np.random.default_rng(9).permutation(len(jobs))
    for jb in jobs:
        if jb["llr"] is not None:
            jb["llr"].fill_(float("nan"))
    torch.cuda.synchronize()
    for k in order:
        sv.submit(**jobs[k])
    res = sv.results()
    info = sv.info()
    sv.close()
    assert len(res) == len(jobs)
    assert info["max_batch"] > 1, info          # the jobs really shared launches
    for r in res:
        s_alone, l_alone = alone[r["tag"]]
        assert r["status"] == air.AIR_OK
        np.testing.assert_array_equal(_stats(r), s_alone)
        if l_alone is not None:
            assert torch.equal(jobs[r["tag"]]["llr"].cpu(), l_alone)


def test_admission_respects_budget(ctx, consts):
    jobs = _mix_jobs(ctx, consts, 60, seed=6, host_share=1.0)
    sv = ctx.server(1 << 20, max_inflight=8)     # 1 MiB: a few jobs at a time
    ids = []
    for jb in jobs:
        try:
            ids.append(sv.submit(**jb))
        except air.AirError as e:
            # a job whose footprint alone exceeds the budget is refused up front
            assert e.status == air.AIR_E_NOMEM
    assert len(ids) >= 20
    res = sv.results()
    info = sv.info()
    sv.close()
    assert len(res) == len(ids) and {r["id"] for r in res} == set(ids)
    assert info["peak_in_use"] <= info["budget"] == 1 << 20
    assert info["in_use"] == 0 and info["completed"] == info["submitted"] == len(ids)
    assert all(r["status"] == air.AIR_OK and 0 < r["footprint"] <= 1 << 20 for r in res)


def test_latency_stamps(ctx, consts):
    jobs = _mix_jobs(ctx, consts, 30, seed=7)
    sv = ctx.server(1 << 28)
    t0 = time.monotonic_ns()
    for jb in jobs:
        sv.submit(**jb, t_arrival_ns=time.monotonic_ns())
    res = sv.results()
    t1 = time.monotonic_ns()
    sv.close()
    for r in res:
        assert t0 <= r["t_arrival_ns"] <= r["t_admit_ns"] <= r["t_launch_ns"] <= r["t_done_ns"] <= t1, r


def test_invalid_tx_only_fails_its_job(ctx, consts):
    X, lab, c = consts[64]
    N = 700
    tx, z = _block(64, 4, N, 21)
    bad = tx.copy()
    bad[123] = 64
    sv = ctx.server(1 << 26)
    good_alone = _run_alone(sv, dict(c=c, inp=to_dev(z), tx=tx_dev(tx), snr_db=8.0, noise=True))
    L = torch.zeros((N, c.m), device=ctx.torch_device)
    sv.submit(c=c, inp=to_dev(z), tx=tx_dev(bad), snr_db=8.0, noise=True, llr=L, tag=1)
    sv.submit(c=c, inp=to_dev(z), tx=tx_dev(tx), snr_db=8.0, noise=True, tag=2)
    res = {r["tag"]: r for r in sv.results()}
    sv.close()
    assert res[1]["status"] == air.AIR_E_RANGE and np.isnan(_stats(res[1])).all()
    assert torch.isnan(L[123]).all() and not torch.isnan(L[:123]).any()
    assert res[2]["status"] == air.AIR_OK
    np.testing.assert_array_equal(_stats(res[2]), _stats(good_alone))


def test_llr_only_job(ctx, consts):
    X, lab, c = consts[256]
    N = 999
    tx, z = _block(256, 4, N, 31)
    Y = _received(X, tx, z, 12.0)
    L1 = ctx.llr(c, to_dev(Y), 12.0, prec="bf16x3")
    ctx.sync()
    sv = ctx.server(1 << 26)
    L2 = torch.empty_like(L1)
    r = _run_alone(sv, dict(c=c, inp=to_dev(Y), snr_db=12.0, prec="bf16x3", llr=L2))
    sv.close()
    assert r["status"] == air.AIR_OK and np.isnan(_stats(r)).all()
    assert_llr(L2.cpu().numpy(), L1.cpu().numpy(), 1e-4)


def test_submit_errors(ctx, consts):
    X, lab, c = consts[16]
    tx, z = _block(16, 2, 100, 41)
    sv = ctx.server(1 << 20)
    with pytest.raises(air.AirError) as e:
        sv.submit(c=c, inp=to_dev(z), tx=tx_dev(tx), snr_db=3.0, prec="fp32")
    assert e.value.status == air.AIR_E_UNSUPPORTED
    with pytest.raises(air.AirError) as e:
        sv.submit(c=c, inp=to_dev(z), snr_db=3.0, noise=True)            # noise needs tx
    assert e.value.status == air.AIR_E_INVAL
    with pytest.raises(air.AirError) as e:
        sv.submit(c=c, inp=to_dev(z), tx=tx_dev(tx), snr_db=float("nan"))
    assert e.value.status == air.AIR_E_INVAL
    with pytest.raises(air.AirError) as e:
        sv.submit(c=c, inp=to_dev(z[:0]), snr_db=3.0)                      # N = 0
    assert e.value.status == air.AIR_E_INVAL
    big = np.zeros((200_000, 2), dtype=np.float32)
    with pytest.raises(air.AirError) as e:
        sv.submit(c=c, inp=big, snr_db=3.0)                                # footprint > budget
    assert e.value.status == air.AIR_E_NOMEM
    Xq, labq = inputs.random_constellation(3, 8, 2)
    cq = ctx.const(Xq, labq)
    with pytest.raises(air.AirError) as e:
        sv.submit(c=cq, inp=to_dev(z), snr_db=3.0)                         # M < 16
    assert e.value.status == air.AIR_E_UNSUPPORTED
    assert sv.info()["submitted"] == 0
    sv.close()
    cq.close()


def test_poisson_soak(ctx):
    """A short stretch of the serving mix at its arrival rate: every job
    completes, results are finite and stamps are ordered."""
    jobs = inputs.serving_jobs(400)
    pools = {M: [ctx.const(X, lab) for X, lab in inputs.serving_pool(M)] for M, _ in MIX}
    nmax = max(j.N for j in jobs)
    r = np.random.default_rng(1)
    zpool = {D: torch.from_numpy(r.standard_normal((nmax, D)).astype(np.float32)).to(ctx.torch_device)
             for D in (2, 4, 8)}
    txpool = {M: torch.from_numpy(r.integers(0, M, nmax).astype(np.int32)).to(ctx.torch_device)
              for M, _ in MIX}
    sv = ctx.server(8 << 30)
    t0 = time.monotonic_ns()
    for jb in jobs:
        t_arr = t0 + int(jb.arrival_s * 1e9)
        while time.monotonic_ns() < t_arr:
            pass
        sv.submit(c=pools[jb.M][jb.const_id], inp=zpool[jb.D][:jb.N], tx=txpool[jb.M][:jb.N],
                  snr_db=jb.snr_db, noise=True, t_arrival_ns=t_arr)
    res = sv.results()
    sv.close()
    assert len(res) == len(jobs)
    lat = np.array([(x["t_done_ns"] - x["t_arrival_ns"]) * 1e-6 for x in res])
    print(f"soak: {len(res)} jobs, latency p50 {np.percentile(lat, 50):.3f} ms, "
          f"p99 {np.percentile(lat, 99):.3f} ms")
    assert all(x["status"] == air.AIR_OK and np.isfinite(_stats(x)[:2]).all() for x in res)
