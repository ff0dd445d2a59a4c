#!/usr/bin/env python3
"""Throughput of the soft-demapping + MI/GMI hot path on one MI355X.

One step = one air_sweep call over the whole workload: every SNR point of the
grid, LLRs written for every (SNR, sample, bit), MI/GMI and their standard
errors reduced in FP64. Inputs (tx, unit noise) are resident in HBM before the
timed region. The metric is sample*points per second, N * S * M / step time.

Prints one JSON line. With --gpus N > 1 it exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Transcendental roof of MI355X: 256 CUs x 4 SIMDs x 16 lanes per clock at half
# rate for v_exp_f32 / v_log_f32 (32 per clock per CU), 2.4 GHz.
CLOCK_HZ = 2.4e9
SIMDS = 256 * 4                        # 256 CUs x 4 SIMDs
TRANS_PEAK = 256 * 32 * CLOCK_HZ       # exp2/log2 per second (half rate)
PROFILES = os.path.join(ROOT, "profiles")

# Hard-decision FEC codes the summaries are judged against: the paper names a
# 6.7 % and a 20 % overhead code without printing their threshold BERs; these
# are the caller's choice (the usual literature values for codes of those
# overheads).
FEC_OVERHEAD = [0.067, 0.20]
FEC_THRESHOLD = [3.8e-3, 2.0e-2]


# Sources of the profiled kernels (both tiers) and of their launches (grid,
# arguments): stored counter data describes the kernels only while these are
# unchanged.
FIRST_TIER_SOURCES = ("device_common.h", "mfma_kernels.h", "mfma_wide.h", "mfma_inst_f16_0.hip",
                      "mfma_inst_bf16_0.hip", "vec_kernels.h", "vec_inst_f32_0.hip", "air_host.hip",
                      "host_state.h", "tier2_list.h", "exact_rule.h")


def source_hash() -> str:
    """Digest of the first tier's sources (comments and blank lines dropped),
    to tell whether stored counter data still describes the kernel built."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in FIRST_TIER_SOURCES:
        h.update(name.encode())
        for line in open(os.path.join(ROOT, "paper_2108_07001_amd", "csrc", name)).read().splitlines():
            code = re.sub(r"//.*$", "", line).rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def traffic_from(out_dir: str, config: str, prec: str, kernel: str, commands: list) -> dict:
    """HBM bytes per launch of `kernel` from rocprofv3 --pmc runs in out_dir:
    f/ (FETCH_SIZE) and w/ (WRITE_SIZE) of the benchmark, cf/ and cw/ of the
    1 GiB copy probe; each counter scaled by what it reads for the copy."""
    import csv
    import glob

    def rows(sub):
        f = glob.glob(os.path.join(out_dir, sub, "**", "*counter_collection.csv"), recursive=True)
        if not f:
            raise SystemExit(f"no counter_collection.csv under {out_dir}/{sub}")
        return list(csv.DictReader(open(f[0])))

    def per_dispatch(rs, pred):
        vals = {}
        for r in rs:
            if pred(r["Kernel_Name"]):
                vals[r["Dispatch_Id"]] = vals.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
        if not vals:
            raise SystemExit("kernel not found in the counter data")
        return sum(vals.values()) / len(vals), len(vals)

    fk, nf = per_dispatch(rows("f"), lambda n: kernel in n)
    wk, nw = per_dispatch(rows("w"), lambda n: kernel in n)
    cf, _ = per_dispatch(rows("cf"), lambda n: "copyBuffer" in n)
    cw, _ = per_dispatch(rows("cw"), lambda n: "copyBuffer" in n)
    gib = float(1 << 30)
    ff, wf = gib / (cf * 1024.0), gib / (cw * 1024.0)
    fb, wb = fk * 1024.0 * ff, wk * 1024.0 * wf
    return {"kernel": kernel, "workload": config, "prec": prec, "dispatches": [nf, nw],
            "fetch_size_kib_per_dispatch": fk, "write_size_kib_per_dispatch": wk,
            "copy_probe": {"bytes": int(gib), "fetch_size_kib": cf, "write_size_kib": cw,
                           "fetch_factor": ff, "write_factor": wf},
            "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb, "bytes_per_launch": fb + wb,
            "source_hash": source_hash(), "commands": commands}


def counters_from(out_dir: str, kernel: str) -> dict:
    """Per-dispatch averages of every counter of `kernel` in one rocprofv3
    --pmc run under out_dir."""
    import csv
    import glob
    f = glob.glob(os.path.join(out_dir, "**", "*counter_collection.csv"), recursive=True)
    if not f:
        raise SystemExit(f"no counter_collection.csv under {out_dir}")
    acc = {}
    for r in csv.DictReader(open(f[0])):
        if kernel in r["Kernel_Name"]:
            d = acc.setdefault(r["Counter_Name"], {})
            d[r["Dispatch_Id"]] = d.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    if not acc:
        raise SystemExit("kernel not found in the counter data")
    return {k: sum(v.values()) / len(v) for k, v in acc.items()}


def stored_issue(workload: str, prec: str, kernel_ms: float, tier: int = 1):
    """VALU issue of the main kernel from the committed SQ counter summary:
    instructions per launch and the fraction of the issue limit (one wave64
    VALU instruction per SIMD every 4 cycles) they take at the measured launch
    time; None when there is no summary or the sources changed since."""
    p = os.path.join(PROFILES, f"sq_{profile_suffix(workload, prec, tier)}.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("source_hash") != source_hash():
        return None
    cycles = kernel_ms * 1e-3 * CLOCK_HZ
    return {"valu_insts_per_launch": d["SQ_INSTS_VALU"],
            "insts_per_simd_cycle": d["SQ_INSTS_VALU"] / (SIMDS * cycles),
            "frac_of_issue_limit": d["SQ_INSTS_VALU"] * 4.0 / (SIMDS * cycles),
            "note": "exp2/log2 occupy the SIMD for two issue slots; they are counted once here"}


def stored_traffic(workload: str, prec: str, tier: int = 1):
    """HBM bytes per launch of the main kernel from the committed counter
    summary (FETCH_SIZE / WRITE_SIZE scaled by a plain copy's readings), or
    None when there is none for this workload or the sources changed since."""
    p = os.path.join(PROFILES, f"traffic_{profile_suffix(workload, prec, tier)}.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    return d["bytes_per_launch"] if d.get("source_hash") == source_hash() else None


def kernel_name(M: int, D: int, prec: str, tier: int) -> str:
    """A matrix-core demapping kernel as the profiler prints it. First tier:
    demap_mfma_w<D, bfloat16 operands, tables in LDS, exact-size log2 M or 0,
    max-log>; second tier: demap_mfma_t2<D, bfloat16, 16-point tiles, tables
    in LDS>. The tables go to LDS when they take at most 40 KB (labels, FP32
    coordinates and the point records, as the library lays them out)."""
    bf = prec == "bf16x3"
    feat = 6 * D + 6 if bf else 3 * D + 3
    nk = (feat + 1 + 15) // 16
    tbl = M * 4 + M * D * 4 + 16 + M * nk * 32 <= 40 * 1024
    b = "true" if bf else "false"
    if tier == 1:
        mb = {16: 4, 32: 5, 64: 6}.get(M, 0)
        return f"demap_mfma_w<{D}, {b}, {'true' if (tbl or mb) else 'false'}, {mb}, false>"
    half = M == 16
    return f"demap_mfma_t2<{D}, {b}, {'true' if half else 'false'}, {'true' if (half or tbl) else 'false'}>"


def profile_suffix(config: str, prec: str, tier: int) -> str:
    return f"{config}_{prec}" + ("_t2" if tier == 2 else "")


def inputs_config(name: str) -> dict:
    from paper_2108_07001_amd import inputs
    return inputs.CONFIGS[name]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def maxlog(ctx, c, w, tx, prec: str, steps: int) -> dict:
    """The same sweep in the max-log form (air_sweep_maxlog): LLRs from the
    largest term of each bit side, GMI of those LLRs; no symbol-wise MI."""
    import torch
    dev = ctx.torch_device
    S, N, m = len(w.snr_db), w.N, w.m
    zt = torch.from_numpy(w.z).to(dev)
    stats = torch.empty((S, 4), dtype=torch.float64, device=dev)
    L = torch.empty((S, N, m), dtype=torch.float32, device=dev)
    ctx.sweep_maxlog(c, tx, zt, w.snr_db, prec=prec, stats_out=stats, llr_out=L)
    ctx.sync()
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.sweep_maxlog(c, tx, zt, w.snr_db, prec=prec, stats_out=stats, llr_out=L)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    kms, launches = ctx.kernel_time()
    ctx.set_timing(False)
    ctx.sync()
    st = stats.cpu().numpy()
    return {"prec": prec, "ms_per_step": ms, "kernel_ms": kms / max(launches, 1),
            "sample_points_per_s": float(N) * S * w.M / (ms * 1e-3),
            "gmi": [float(x) for x in st[:, 1]]}


def hard_decisions(ctx, c, w, tx, steps: int) -> dict:
    """Nearest-point decisions of the same sweep (air_hard_sweep): BER, SER
    and Q-factor per SNR point, and the decision kernel's throughput."""
    import torch
    z = torch.from_numpy(np.ascontiguousarray(w.z, dtype=np.float32)).to(ctx.torch_device)
    counts, _ = ctx.hard_sweep(c, tx, z, w.snr_db)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        counts, _ = ctx.hard_sweep(c, tx, z, w.snr_db)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    from paper_2108_07001_amd import air
    rates = air.hd_rates(counts.cpu().numpy(), w.N, w.m)
    fec = air.fec_net(rates[:, 0], w.m, FEC_OVERHEAD, FEC_THRESHOLD)
    return {"ms_per_sweep": ms,
            "sample_points_per_s": float(w.N) * len(w.snr_db) * w.M / (ms * 1e-3),
            "snr_db": [float(x) for x in w.snr_db], "ber": [float(x) for x in rates[:, 0]],
            "ser": [float(x) for x in rates[:, 1]],
            "q_db": [None if (x != x) else float(x) for x in rates[:, 2]],
            "fec": {"overhead": FEC_OVERHEAD, "threshold_ber": FEC_THRESHOLD,
                    "pass": fec["pass"].astype(int).tolist(),
                    "net_bits_per_symbol": [float(x) for x in fec["net"]]}}


def streaming(ctx, n_buf: int) -> dict:
    """The paper's own formats at its buffer size: 1 GBaud 2-D M-QAM, buffers of
    2^20 symbols pushed from pinned host memory through a 3-slot pipe
    (air_pipe_*), LLRs back to pinned host memory. Rates are PCIe-inclusive
    (wall clock over n_buf buffers after two warm-up buffers, the median of
    three passes), beside the kernels alone on device-resident buffers."""
    import torch
    from paper_2108_07001_amd import inputs
    cap, snr_db, out = 1 << 20, 18.0, {}
    for mb in range(2, 7):
        M = 1 << mb
        prec = "fp16x3" if M >= 16 else "fp32"
        w = inputs.make(f"qam{M}", N=cap * n_buf)
        sigma = math.sqrt(1.0 / (w.D * 10 ** (snr_db / 10)))      # unit-energy QAM
        Y = torch.from_numpy((w.X[w.tx] + sigma * w.z.astype(np.float64)).astype(np.float32)).pin_memory()
        L = torch.empty((w.N, w.m), dtype=torch.float32).pin_memory()
        c = ctx.const(w.X, w.labels)
        p = ctx.pipe(c, cap, depth=3, prec=prec)
        for k in range(2):
            p.push(Y[k * cap:(k + 1) * cap], snr_db, L[k * cap:(k + 1) * cap])
        p.wait()
        walls = []
        for _ in range(3):                  # median of three passes over the buffers
            t0 = time.perf_counter()
            for k in range(n_buf):
                p.push(Y[k * cap:(k + 1) * cap], snr_db, L[k * cap:(k + 1) * cap])
            p.wait()
            walls.append(time.perf_counter() - t0)
        wall = sorted(walls)[1]
        Yd = Y[:cap].to(ctx.torch_device)
        Ld = torch.empty((cap, w.m), dtype=torch.float32, device=ctx.torch_device)
        ctx.llr(c, Yd, snr_db, prec, out=Ld)
        ctx.sync()
        t0 = time.perf_counter()
        for k in range(n_buf):
            ctx.llr(c, Yd, snr_db, prec, out=Ld)
        ctx.sync()
        dev = time.perf_counter() - t0
        rate = n_buf * cap / wall
        out[f"qam{M}"] = {"prec": prec, "symbols_per_s": rate, "real_time_1GBaud": rate >= 1e9,
                          "device_only_symbols_per_s": n_buf * cap / dev,
                          "pcie_bytes_per_symbol": 4 * (w.D + w.m), "buffers": n_buf,
                          "buffer_symbols": cap}
        p.close()
        c.close()
        del Y, L, Yd, Ld
    return out


def serving(ctx, n_jobs: int) -> dict:
    """Replay the Poisson serving mix through the serving loop: each job is
    submitted at its arrival time and its latency runs from that time to the
    moment its MI/GMI are on the host (LLRs stay in device memory). Inputs are
    slices of pinned host pools (unit noise and tx: their host-to-device copy
    is inside the latency) or, in a second pass, of device-resident pools."""
    import torch
    from paper_2108_07001_amd import inputs
    spec = inputs.SERVING
    jobs = inputs.serving_jobs(n_jobs)
    Ms = sorted(spec["M_choices"])
    pools = {M: [ctx.const(X, lab) for X, lab in inputs.serving_pool(M)] for M in Ms}
    nmax = max(j.N for j in jobs)
    r = np.random.default_rng(spec["seed"] + 1)
    Ds = sorted(set(spec["D_for_M"][M] for M in Ms))
    z_host = {D: torch.from_numpy(r.standard_normal((nmax, D)).astype(np.float32)).pin_memory() for D in Ds}
    tx_host = {M: torch.from_numpy(r.integers(0, M, nmax).astype(np.int32)).pin_memory() for M in Ms}
    dev = ctx.torch_device
    z_dev = {D: t.to(dev) for D, t in z_host.items()}
    tx_dev = {M: t.to(dev) for M, t in tx_host.items()}
    # device LLR slots, one per job in flight (handed back when its result is polled)
    mmax = max(int(np.log2(M)) for M in Ms)
    nslots = 128
    llr_pool = torch.empty((nslots, nmax * mmax), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    def replay(on_device: bool) -> dict:
        sv = ctx.server(16 << 30, max_inflight=nslots)
        free = list(range(nslots))
        slot_of, done = {}, []

        def reap():
            for res in sv.poll(1024):
                free.append(slot_of.pop(res["id"]))
                done.append(res)

        t0 = time.monotonic_ns() + 20_000_000
        for jb in jobs:
            c = pools[jb.M][jb.const_id]
            while not free:
                reap()
            k = free.pop()
            t_arr = t0 + int(jb.arrival_s * 1e9)
            while time.monotonic_ns() < t_arr:
                reap()
            zsrc = z_dev if on_device else z_host
            txsrc = tx_dev if on_device else tx_host
            L = llr_pool[k, :jb.N * c.m].view(jb.N, c.m)
            jid = sv.submit(c=c, inp=zsrc[jb.D][:jb.N], tx=txsrc[jb.M][:jb.N], snr_db=jb.snr_db,
                            noise=True, prec="bf16x3", llr=L, t_arrival_ns=t_arr)
            slot_of[jid] = k
        sv.drain()
        reap()
        info = sv.info()
        sv.close()
        lat = np.array([(x["t_done_ns"] - x["t_arrival_ns"]) * 1e-6 for x in done])
        wait = np.array([(x["t_launch_ns"] - x["t_arrival_ns"]) * 1e-6 for x in done])
        bad = sum(1 for x in done if x["status"] != 0)
        span = (max(x["t_done_ns"] for x in done) - t0) * 1e-9
        pts = sum(j.N * j.M for j in jobs)
        return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "max_ms": float(lat.max()), "mean_ms": float(lat.mean()),
                "p99_wait_to_launch_ms": float(np.percentile(wait, 99)),
                "jobs": len(done), "failed": bad, "batches": int(info["batches"]),
                "max_batch": int(info["max_batch"]), "peak_arena_bytes": int(info["peak_in_use"]),
                "offered_sample_points_per_s": pts / jobs[-1].arrival_s,
                "achieved_sample_points_per_s": pts / span}

    log(f"serving: {n_jobs} jobs, host inputs")
    host = replay(False)
    log(f"serving host inputs: p50 {host['p50_ms']:.3f} ms, p99 {host['p99_ms']:.3f} ms")
    devr = replay(True)
    log(f"serving device inputs: p50 {devr['p50_ms']:.3f} ms, p99 {devr['p99_ms']:.3f} ms")
    for p in pools.values():
        for c in p:
            c.close()
    return {"workload": f"Poisson {spec['rate_hz']:g} jobs/s, M in {list(Ms)} (D {spec['D_for_M']}), "
                        f"N = 10^U({spec['N_log10'][0]},{spec['N_log10'][1]}), SNR U{tuple(spec['snr_db'])} dB, "
                        f"bf16x3, LLRs to device memory",
            "latency_from": "arrival time -> MI/GMI on the host",
            "host_inputs": host, "device_inputs": devr}


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def large_sets(ctx, names, steps: int) -> dict:
    """Full-size step times of the large Gaussian sweeps: one air_sweep over
    every sample and SNR point with LLRs written, per form (the matrix-core
    forms `steps` timed steps after one warm-up, the plain FP32 kernel one),
    with the first tier's kernel time and its fraction of the transcendental
    roof, and the items the second tier and the exact path took."""
    import torch
    from paper_2108_07001_amd import air, inputs
    out = {}
    dev = ctx.torch_device
    for name in names:
        w = inputs.make(name)
        M, m, N, S = w.M, w.m, w.N, len(w.snr_db)
        c = ctx.const(w.X, w.labels)
        tx = torch.from_numpy(w.tx.astype(np.int32)).to(dev)
        z = torch.from_numpy(w.z).to(dev)
        stats = torch.empty((S, 4), dtype=torch.float64, device=dev)
        L = torch.empty((S, N, m), dtype=torch.float32, device=dev)
        res = {"workload": f"{name}: {inputs.CONFIGS[name]['desc']}, N={N}, SNR {w.snr_db[0]:g}.."
                           f"{w.snr_db[-1]:g} dB ({S} points), LLRs written (fp32)", "M": M, "D": w.D,
               "N": N, "S": S}
        trans = float(N) * S * (M + 2 * m + 1)
        for p in ("fp16x3", "bf16x3", "fp32"):
            k = steps if p != "fp32" else 1
            ctx.sweep(c, tx, z, w.snr_db, prec=p, stats_out=stats, llr_out=L)
            ctx.sync()
            ctx.set_timing(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(k):
                ctx.sweep(c, tx, z, w.snr_db, prec=p, stats_out=stats, llr_out=L)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / k
            kms, nl = ctx.kernel_time()
            ctx.set_timing(False)
            kstep = kms / k                       # first-tier time per step (all its launches)
            res[p] = {"ms_per_step": ms, "first_tier_ms_per_step": kstep,
                      "sample_points_per_s": float(N) * S * M / (ms * 1e-3),
                      "first_tier_trans_frac": trans / (kstep * 1e-3) / TRANS_PEAK,
                      "step_trans_frac": trans / (ms * 1e-3) / TRANS_PEAK,
                      "second_tier_items": int(ctx.last_recomputed()), "exact_path_items": int(ctx.last_exact()),
                      "mi_gmi_first_last": [float(x) for x in stats.cpu().numpy()[[0, -1], :2].ravel()]}
            if p != "fp32":
                # counter summaries of this build's first tier, where committed
                res[p]["first_tier_traffic_bytes"] = stored_traffic(name, p)
                res[p]["first_tier_valu_issue"] = stored_issue(name, p, kstep)
            log(f"{name} {p}: {ms:.2f} ms/step (first tier {kstep:.2f} ms), second tier "
                f"{res[p]['second_tier_items']} items, exact {res[p]['exact_path_items']}")
        for p in ("fp16x3", "bf16x3"):
            res[p]["speedup_vs_fp32"] = res["fp32"]["ms_per_step"] / res[p]["ms_per_step"]
        # the same sweep for MI/GMI alone (no LLRs written): only the total and
        # the transmitted point's bit sides then need the first tier's frame
        res["mi_gmi_only"] = {}
        for p in ("fp16x3", "fp32"):
            ctx.sweep(c, tx, z, w.snr_db, prec=p, stats_out=stats)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.sweep(c, tx, z, w.snr_db, prec=p, stats_out=stats)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            res["mi_gmi_only"][p] = {"ms_per_step": ms, "second_tier_items": int(ctx.last_recomputed()),
                                     "sample_points_per_s": float(N) * S * M / (ms * 1e-3)}
            log(f"{name} {p} MI/GMI only: {ms:.2f} ms/step, second tier {ctx.last_recomputed()} items")
        res["mi_gmi_only"]["fp16x3"]["speedup_vs_fp32"] = (res["mi_gmi_only"]["fp32"]["ms_per_step"] /
                                                           res["mi_gmi_only"]["fp16x3"]["ms_per_step"])
        out[name] = res
        del L, z, tx
        c.close()
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 200 steps of ~0.35-0.7 ms: four interleaved segments of 50 per form, so
    # that the launch latency at the start of a segment and the final
    # synchronisation (~20 us each segment) stay well under 1 % of a step
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="psk8x8")
    ap.add_argument("--prec", default=None, help="fp32 | bf16x3 | fp16x3 (default: fastest)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target duration of the oracle's CPU-baseline sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true",
                    help="skip timing the plain FP32 kernel beside the matrix-core form")
    ap.add_argument("--serving-jobs", type=int, default=20000,
                    help="jobs of the Poisson serving mix to replay (the full mix: 20000, 10 s per pass; 0: skip)")
    ap.add_argument("--stream-buffers", type=int, default=12,
                    help="2^20-symbol M-QAM buffers per format streamed from host memory (0: skip)")
    ap.add_argument("--traffic-from", default=None,
                    help="write profiles/traffic_<config>_<prec>.json from rocprofv3 --pmc "
                         "FETCH_SIZE / WRITE_SIZE runs of the benchmark (f/, w/) and of "
                         "--copy-probe (cf/, cw/) under this directory, then exit")
    ap.add_argument("--sq-from", default=None,
                    help="write profiles/sq_<config>_<prec>.json from a rocprofv3 --pmc run of "
                         "SQ counters of the benchmark under this directory, then exit")
    ap.add_argument("--large-sets", default="gauss8d2048,gauss12d4096",
                    help="large Gaussian sweeps whose full-size step times are reported beside the "
                         "headline (comma-separated workload names; empty: skip)")
    ap.add_argument("--large-steps", type=int, default=3,
                    help="timed steps per matrix-core form of each large sweep (the plain FP32 kernel: 1)")
    ap.add_argument("--roofs", action="store_true",
                    help="only measure the unit rates (air_measure_roofs) and print them as JSON")
    ap.add_argument("--tier", type=int, default=1, choices=(1, 2),
                    help="--traffic-from / --sq-from: the first tier's kernel or the second tier's")
    ap.add_argument("--profile-args", default="",
                    help="--traffic-from / --sq-from: further bench.py arguments of the profiled runs, "
                         "recorded in the summary's commands")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device-to-device copy of 1 GiB (3 times), the "
                         "reference for scaling hardware byte counters")
    args = ap.parse_args()
    if args.traffic_from:
        prec = args.prec or "fp16x3"
        w0 = inputs_config(args.config)
        kern = kernel_name(w0["M"], w0["D"], prec, args.tier)
        run = (f"python3 bench.py --config {args.config} --no-cpu --serving-jobs 0 --stream-buffers 0 "
               f"--large-sets '' {args.profile_args}").strip()
        cmds = [f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/f -o f -- {run}",
                f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d <out>/w -o w -- {run}",
                "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/cf -o cf -- python3 bench.py --copy-probe",
                "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <out>/cw -o cw -- python3 bench.py --copy-probe",
                f"python3 bench.py --config {args.config} --prec {prec} --tier {args.tier} --traffic-from <out>"]
        d = traffic_from(args.traffic_from, args.config, prec, kern, cmds)
        p = os.path.join(PROFILES, f"traffic_{profile_suffix(args.config, prec, args.tier)}.json")
        json.dump(d, open(p, "w"), indent=1)
        print(json.dumps({"wrote": p, "bytes_per_launch": d["bytes_per_launch"]}))
        return
    if args.sq_from:
        prec = args.prec or "fp16x3"
        w0 = inputs_config(args.config)
        kern = kernel_name(w0["M"], w0["D"], prec, args.tier)
        d = counters_from(args.sq_from, kern)
        run = (f"python3 bench.py --config {args.config} --no-cpu --serving-jobs 0 --stream-buffers 0 "
               f"--large-sets '' {args.profile_args}").strip()
        d.update(kernel=kern, workload=args.config, prec=prec, source_hash=source_hash(),
                 commands=[f"rocprofv3 --pmc {' '.join(sorted(k for k in d if not k[0].islower()))} "
                           f"--output-format csv -d <out> -o sq -- {run}",
                           f"python3 bench.py --config {args.config} --prec {prec} --tier {args.tier} "
                           f"--sq-from <out>"])
        p = os.path.join(PROFILES, f"sq_{profile_suffix(args.config, prec, args.tier)}.json")
        json.dump(d, open(p, "w"), indent=1)
        print(json.dumps({"wrote": p}))
        return
    if args.copy_probe:
        import torch
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read_per_launch": a.numel() * 4,
                          "copy_probe_bytes_written_per_launch": b.numel() * 4, "launches": 3}))
        return
    if args.roofs:
        from paper_2108_07001_amd import air
        ctx = air.Context(0)
        r = ctx.measure_roofs()
        clk_cu = CLOCK_HZ * 256
        r["per_cu_per_clock_at_2.4GHz"] = {"exp": r["exp_per_s"] / clk_cu, "explog": r["explog_per_s"] / clk_cu,
                                           "fma": r["fma_per_s"] / clk_cu,
                                           "mfma_f16_flop": r["mfma_f16_flops"] / clk_cu}
        print(json.dumps(r), flush=True)
        ctx.close()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU design is described in DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2108_07001_amd import air, inputs

    dev = torch.device("cuda", 0)
    w = inputs.make(args.config)
    M, D, m, N, S = w.M, w.D, w.m, w.N, len(w.snr_db)
    ctx = air.Context(0)
    roofs = ctx.measure_roofs()
    log(f"roofs: exp {roofs['exp_per_s']:.3e}/s, fma {roofs['fma_per_s']:.3e}/s, "
        f"mfma f16 {roofs['mfma_f16_flops']:.3e} flop/s, copy {roofs['copy_bytes_per_s']:.3e} B/s")
    c = ctx.const(w.X, w.labels)
    # the matrix-core forms first (the faster one that serves this
    # constellation is the headline), the plain FP32 kernel as the baseline
    precs = ["fp16x3", "bf16x3", "fp32"] if args.prec is None else [args.prec]
    if args.prec is None and args.no_fp32:
        precs.remove("fp32")
    tx = torch.from_numpy(w.tx.astype(np.int32)).to(dev)
    zt32 = torch.from_numpy(w.z).to(dev)
    L = torch.empty((S, N, m), dtype=torch.float64 if "fp64" in precs else torch.float32, device=dev)
    stats = torch.empty((S, 4), dtype=torch.float64, device=dev)

    def sweep(prec):
        ctx.sweep(c, tx, zt32.double() if prec == "fp64" else zt32, w.snr_db, prec=prec,
                  stats_out=stats, llr_out=L)

    forms = []
    for p in precs:
        try:
            sweep(p)
            ctx.sync()
            forms.append(p)
        except air.AirError as e:
            if e.status != air.AIR_E_UNSUPPORTED:
                raise
            log(f"{p}: not available ({e})")
    if not forms:
        raise SystemExit("no precision form is available for this constellation")
    # Untimed load first: the GPU's clocks need some hundreds of milliseconds
    # of work to settle, and no form should absorb that. Then every form's
    # warm-up, and the timed steps of the forms interleaved in rounds, so
    # that slow drifts of the clock fall on all forms alike.
    t_end = time.perf_counter() + 0.5
    while time.perf_counter() < t_end:
        for p in forms:
            sweep(p)
        torch.cuda.synchronize()
    for p in forms:
        for _ in range(args.warmup):
            sweep(p)
    ctx.sync()
    results = {p: dict(ms=0.0, kms=0.0, launches=0) for p in forms}
    rounds = min(4, args.steps)
    ctx.set_timing(True)
    for i in range(rounds):
        k = args.steps // rounds + (1 if i < args.steps % rounds else 0)
        for p in forms:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(k):
                sweep(p)
            torch.cuda.synchronize()
            results[p]["ms"] += (time.perf_counter() - t0) * 1e3
            kms, nl = ctx.kernel_time()
            results[p]["kms"] += kms
            results[p]["launches"] += nl
    ctx.set_timing(False)
    for p in forms:
        r = results[p]
        sweep(p)
        r.update(recomputed=ctx.last_recomputed(), exact=ctx.last_exact(),
                 ms=r["ms"] / args.steps, kernel_ms=r["kms"] / max(r["launches"], 1),
                 launches=r["launches"] / args.steps, stats=stats.cpu().numpy())
        log(f"{p}: {r['ms']:.3f} ms/step, kernel {r['kernel_ms']:.3f} ms")
    chosen = min((p for p in forms if p != "fp32"), key=lambda p: results[p]["ms"], default=forms[0])
    del L
    torch.cuda.empty_cache()

    r = results[chosen]
    pts = float(N) * S * M
    value = pts / (r["ms"] * 1e-3)
    trans = float(N) * S * (M + 2 * m + 1)
    # per step: the launches' total time (one launch per 64 SNR points)
    achieved = trans / (r["kernel_ms"] * max(r["launches"], 1.0) * 1e-3)
    line = {
        "metric": "sample*points/s for MI/GMI+LLR (N*S*M per step)",
        "value": value,
        "unit": "sample*points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": chosen,
        "data": "synthetic (seeded: constellation, labels, tx, unit noise)",
        "config": {"workload": f"{args.config}: {inputs.CONFIGS[args.config]['desc']}, "
                               f"N={N}, SNR {w.snr_db[0]:g}..{w.snr_db[-1]:g} dB ({S} points), "
                               f"LLRs written (fp32), MI/GMI+SE in fp64",
                   "M": M, "D": D, "N": N, "S": S},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": TRANS_PEAK / 1e12,
                     "unit": "Ttranscendentals/s", "frac": achieved / TRANS_PEAK,
                     "traffic": stored_traffic(args.config, chosen),
                     "valu_issue": stored_issue(args.config, chosen, r["kernel_ms"]),
                     "kernel": "first tier (demap_mfma_w)" if chosen in ("fp16x3", "bf16x3")
                               else "demap_vec",
                     "kernel_ms": r["kernel_ms"], "launches_per_step": r["launches"],
                     "per_unit": f"(M + 2m + 1) = {M + 2 * m + 1} exp2/log2 per sample per SNR",
                     "algorithmic_per_launch": trans / max(r["launches"], 1)},
        "second_tier_items": int(r["recomputed"]),
        "exact_path_items": int(r["exact"]),
        "roofs_measured": roofs,
    }
    line["forms"] = {p: {"value": pts / (results[p]["ms"] * 1e-3), "ms_per_step": results[p]["ms"],
                         "kernel_ms": results[p]["kernel_ms"], "second_tier_items": int(results[p]["recomputed"]),
                         "exact_path_items": int(results[p]["exact"])} for p in forms}
    if chosen != "fp32" and "fp32" in results:
        f = results["fp32"]
        line["fp32_plain"] = {"value": pts / (f["ms"] * 1e-3), "ms_per_step": f["ms"],
                              "kernel_ms": f["kernel_ms"]}
        line["speedup_vs_fp32"] = f["ms"] / r["ms"]
        for p in forms:
            if p != "fp32":
                line["forms"][p]["speedup_vs_fp32"] = f["ms"] / results[p]["ms"]
    line["timing"] = (f"forms timed interleaved in {rounds} rounds after 0.5 s of untimed load and "
                      f"{args.warmup} warm-up steps each; {args.steps} timed steps per form")

    if chosen in ("fp16x3", "bf16x3", "fp32"):
        line["maxlog"] = maxlog(ctx, c, w, tx, chosen, args.steps)
        line["maxlog"]["speedup_vs_exact"] = r["ms"] / line["maxlog"]["ms_per_step"]
    line["hard_decisions"] = hard_decisions(ctx, c, w, tx, max(3, args.steps // 4))

    if args.large_sets:
        line["large_sets"] = large_sets(ctx, [s for s in args.large_sets.split(",") if s], args.large_steps)

    if args.stream_buffers > 0:
        line["streaming"] = streaming(ctx, args.stream_buffers)

    if args.serving_jobs > 0:
        line["serving"] = serving(ctx, args.serving_jobs)

    if not args.no_cpu:
        import oracle
        # calibrate on a small prefix, then time a prefix worth ~cpu_seconds
        n0 = 2000
        t0 = time.perf_counter()
        oracle.sweep(w.X, w.labels, w.tx[:n0], w.z[:n0], w.snr_db, llr=True)
        t_small = time.perf_counter() - t0
        n = int(min(N, max(n0, n0 * args.cpu_seconds / max(t_small, 1e-3))))
        t0 = time.perf_counter()
        ref = oracle.sweep(w.X, w.labels, w.tx[:n], w.z[:n], w.snr_db, llr=True)
        t_cpu = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": n * S * M / t_cpu, "unit": "sample*points/s",
                                "cores": oracle.threads(), "kind": "oracle",
                                "sample": f"first {n} of {N} samples x {S} SNR points, LLRs on",
                                "seconds": t_cpu}
        line["cpu_baseline"]["cpu_model"] = cpu_model()
        # parity of every timed form on the same prefix
        zt = torch.from_numpy(np.ascontiguousarray(w.z[:n])).to(dev)
        par = {}
        for p in forms:
            zp = zt.double() if p == "fp64" else zt
            st, Lg = ctx.sweep(c, tx[:n].contiguous(), zp, w.snr_db, prec=p, llr=True)
            ctx.sync()
            st = st.cpu().numpy()
            Lg = Lg.cpu().numpy().astype(np.float64)
            rel = np.abs(Lg - ref["llr"]) / np.maximum(np.abs(ref["llr"]), 1.0)
            par[p] = {"samples": n, "max_dMI_bits": float(np.abs(st[:, 0] - ref["stats"][:, 0]).max()),
                      "max_dGMI_bits": float(np.abs(st[:, 1] - ref["stats"][:, 1]).max()),
                      "max_llr_rel": float(rel.max())}
            del Lg
        line["parity_vs_oracle"] = par[chosen]
        line["parity_vs_oracle_by_form"] = par
    print(json.dumps(line), flush=True)
    c.close()
    ctx.close()


if __name__ == "__main__":
    main()
