#!/usr/bin/env python3
"""X-engine benchmark on one MI355X.

Workload (one step = one full integration of the hot path on device-resident
input): N_I = 1024 inputs (512 antennas x 2 pols), 768 channels, 8000 complex
samples per channel, 4-bit-range values stored as int8 (re, im) pairs, drawn by
the seeded device generator.  A step is corr_correlate over the whole
integration (triangular tile schedule + int8 MFMA rank-k updates + integration
accumulator store) followed by the accumulator reset of corr_dump.

Prints one JSON line.  Besides the headline int8 figure it reports the plain
FP32 engine on the same data (and whether the two agree bit for bit), the
dump read-out latency, the kernel roofline and the CPU oracle timed on a
bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_IN, N_CH, N_T, SEED = 1024, 768, 8000, 3


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(x_dev, n_channels: int) -> dict:
    """The oracle X-engine on the first `n_channels` channels of the same input
    (all 524 800 products, 8000 samples), on the host's cores."""
    import numpy as np

    import oracle

    xs = x_dev[:n_channels].cpu().numpy()
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    oracle.xengine_ci8(xs)
    dt = time.perf_counter() - t0
    cmac = n_channels * N_IN * (N_IN + 1) // 2 * N_T
    # the paper's comparison is one CPU thread: one channel on one thread
    oracle.set_num_threads(1)
    try:
        t1 = time.perf_counter()
        oracle.xengine_ci8(xs[:1])
        dt1 = time.perf_counter() - t1
    finally:
        oracle.set_num_threads(threads)
    cmac1 = N_IN * (N_IN + 1) // 2 * N_T
    return {"value": cmac / dt / 1e12, "unit": "Tcmac/s", "cores": min(threads, n_channels), "kind": "oracle",
            "sample": f"{n_channels} of 768 channels x all 524800 products x 8000 samples "
                      f"({cmac:.3e} CMAC, {dt:.1f} s, int64 C oracle, OpenMP over channels)",
            "seconds": dt, "host_threads": threads, "nproc": os.cpu_count(),
            "one_thread": {"value": cmac1 / dt1 / 1e12, "unit": "Tcmac/s", "seconds": dt1,
                           "sample": "1 channel x all 524800 products x 8000 samples on one thread"}}


def cpu_other_configs() -> dict:
    """The oracle on the other configurations, on the host's cores (all of
    them, and one thread): C1 in full; one of C2's ten integrations (the
    direct DFT F-stage on a fifth of its blocks -- one thread on a fortieth --
    scaled, and
    the X-engine on requantised samples of the same shape); C4's FP64
    X-engine on 32 of its 1024 channels (one thread: 4 channels), scaled to
    the whole configuration (channels are independent).  Seconds per
    integration."""
    import numpy as np

    import oracle
    import synth

    threads = oracle.num_threads()

    def timed(fn, one_thread=False):
        if one_thread:
            oracle.set_num_threads(1)
        try:
            t = time.perf_counter()
            fn()
            return time.perf_counter() - t
        finally:
            oracle.set_num_threads(threads)

    res = {"host_threads": threads, "nproc": os.cpu_count(), "unit": "s per integration", "kind": "oracle"}
    x1 = synth.ci8(1, 128, 64, 1000)
    res["c1_x"] = {"all_cores": timed(lambda: oracle.xengine_ci8(x1)),
                   "one_thread": timed(lambda: oracle.xengine_ci8(x1), True), "sample": "in full"}
    v = synth.real_voltages(seed=2, index=0, n_blocks=2000, n_inputs=64)
    f_all = timed(lambda: oracle.dft_real(v, 256)) * 5.0
    f_one = timed(lambda: oracle.dft_real(v[: 250 * 256], 256), True) * 40.0
    q = synth.ci8(2, 128, 64, 10000)
    res["c2_f"] = {"all_cores": f_all, "one_thread": f_one,
                   "sample": "2000 of 10000 blocks x 64 inputs, x5 (one thread: 250 blocks, x40)"}
    res["c2_x"] = {"all_cores": timed(lambda: oracle.xengine_ci8(q)),
                   "one_thread": timed(lambda: oracle.xengine_ci8(q), True),
                   "sample": "128 channels x 64 inputs x 10000 samples, in full"}
    x4 = np.stack([synth.complex_float(4, ch, 256, 4096) for ch in range(32)])
    res["c4_x_fp64"] = {"all_cores": timed(lambda: oracle.xengine_cf64(x4)) * 1024 / 32,
                        "one_thread": timed(lambda: oracle.xengine_cf64(x4[:4]), True) * 1024 / 4,
                        "sample": "32 of 1024 channels (one thread: 4), scaled x32 (x256)"}
    return res


def serving(seconds: float, warm: float, rate: float, host: bool, seed: int = 5) -> dict:
    """Continuous-batching serving run (C5).  Fifteen streams, one per
    (N_I, N_C) in {16, 64, 128, 512, 1024} x {64, 256, 768}, each keep a
    device-resident ring of 8000 complex int8 samples per channel and input
    (filled once by the seeded generator, standing in for the instrument's
    ingest).  Integration jobs arrive as a Poisson process (rate jobs/s); each
    picks a stream at random and integrates its first T samples, T uniform in
    1000..8000.  Results go to device buffers (host=False) or to pinned host
    buffers (host=True).  Latency is measured from the job's scheduled
    arrival to the integration complete in device memory (both runs) and, in
    the host run, to the result landed in host memory (the dump end point).
    A job waits, counted in its latency, for a free result buffer of its
    shape.  Jobs arriving in the first `warm` seconds are excluded."""
    import numpy as np
    import torch

    import synth
    from paper_0906_1887_amd import Scheduler, corr_sched_now

    NIS, NCS, TMAX = (16, 64, 128, 512, 1024), (64, 256, 768), 8000
    gen = synth.DeviceGen()
    st = torch.cuda.current_stream().cuda_stream
    rings = {}
    for k, n_in in enumerate(NIS):
        for c, n_ch in enumerate(NCS):
            r = torch.empty((n_ch, n_in, TMAX, 2), dtype=torch.int8, device="cuda:0")
            gen.fill_ci8(r.data_ptr(), n_ch, n_in, TMAX, 5000 + 10 * k + c, stream=st)
            rings[(n_in, n_ch)] = r
    torch.cuda.synchronize()
    rng = np.random.default_rng(seed)
    n_jobs = int(seconds * rate * 1.2) + 10
    t_rel = np.cumsum(rng.exponential(1.0 / rate, n_jobs))
    t_rel = t_rel[t_rel < seconds]
    shapes = [(int(rng.choice(NIS)), int(rng.choice(NCS)), int(rng.integers(1000, TMAX + 1)))
              for _ in range(t_rel.size)]
    # result buffers per (N_I, N_C): 3 for the arrays of 512 and 1024 inputs, 6 for the others
    bufs = {}
    for n_in in NIS:
        for n_ch in NCS:
            P = n_in * (n_in + 1) // 2
            n_buf = 3 if n_in >= 512 else 6
            bufs[(n_in, n_ch)] = [torch.empty((n_ch, P, 2), dtype=torch.int32, pin_memory=True) if host else
                                  torch.empty((n_ch, P, 2), dtype=torch.int32, device="cuda:0")
                                  for _ in range(n_buf)]
    free = {k: list(range(len(v))) for k, v in bufs.items()}
    sched = Scheduler(16 << 30, n_streams=4)

    def submit(n_in, n_ch, T, slot, t_arr=None):
        ring = rings[(n_in, n_ch)]
        return sched.submit(n_in, n_ch, T, bufs[(n_in, n_ch)][slot], d_samples=ring.data_ptr(), row_stride=TMAX,
                            t_arrival=t_arr)

    j0 = submit(16, 64, 1000, 0)
    while sched.poll(j0) is None:
        time.sleep(0.001)
    inflight, done, waiting = {}, [], []
    t0 = corr_sched_now() + 0.05
    k = 0
    last_log = time.time()
    while k < len(shapes) or inflight or waiting:
        now = corr_sched_now()
        for jid in list(inflight):
            r = sched.poll(jid)
            if r is not None:
                kk, key, slot = inflight.pop(jid)
                if r[0] != 0:
                    raise RuntimeError(f"serving job {kk} failed with status {r[0]}")
                done.append((kk, t0 + t_rel[kk], r[2], r[4], r[3]))
                free[key].append(slot)
        while k < len(shapes) and t0 + t_rel[k] <= now:
            waiting.append(k)
            k += 1
        for kk in list(waiting):
            key = shapes[kk][:2]
            if free[key]:
                slot = free[key].pop()
                inflight[submit(*shapes[kk], slot, t0 + t_rel[kk])] = (kk, key, slot)
                waiting.remove(kk)
        if time.time() - last_log > 10.0:
            log(f"serving ({'host' if host else 'device'} results): {len(done)} of {len(shapes)} jobs done")
            last_log = time.time()
        time.sleep(0.0002)
    stats = sched.stats()
    sched.close()
    del bufs
    lat_d, lat_h, wait, tint1, tint2, cm, dump_bytes = [], [], [], [], [], 0, 0
    for kk, ta_sched, ta, tv, td in sorted(done):
        if t_rel[kk] < warm:
            continue
        n_in, n_ch, T = shapes[kk]
        lat_d.append(tv - ta_sched)
        lat_h.append(td - ta_sched)
        wait.append(ta - ta_sched)
        tint1.append(T / 10e3)                 # 10 kHz channels (1.28 MHz / 128)
        tint2.append(T * n_ch / 1.28e6)        # the 1.28 MHz band split into N_C channels
        cm += n_ch * n_in * (n_in + 1) // 2 * T
        dump_bytes += n_ch * n_in * (n_in + 1) // 2 * 8
    lat_d, lat_h = np.array(lat_d), np.array(lat_h)
    span = max(d[4] for d in done) - (t0 + warm)

    def pct(a):
        return {"p50": float(np.percentile(a, 50) * 1e3), "p99": float(np.percentile(a, 99) * 1e3),
                "max": float(a.max() * 1e3), "mean": float(a.mean() * 1e3)}

    def within(a):
        return {"T_over_10kHz": float(np.mean(a < np.array(tint1))),
                "T_times_NC_over_1.28MHz": float(np.mean(a < np.array(tint2)))}

    res = {"jobs": int(lat_d.size), "offered_rate_per_s": rate, "seconds": seconds, "warmup_s": warm,
           "throughput_jobs_per_s": lat_d.size / span, "throughput_tcmac_s": cm / span / 1e12,
           "dump_GB_per_s": dump_bytes / span / 1e9,
           "latency_device_ms": pct(lat_d),
           "latency_device_end": "integration complete in device memory (completion word seen by the scheduler)",
           "frac_within_own_integration_time_device": within(lat_d),
           "p99_device_below_50ms": bool(np.percentile(lat_d, 99) < 0.050),
           "admission_wait_ms_p99": float(np.percentile(wait, 99) * 1e3),
           "scheduler": stats, "path": "device job queue, one persistent int8 grid (128-row tiles)", "arena_GiB": 16,
           "rings_GB": 30.0}
    if host:
        res.update({"latency_host_ms": pct(lat_h),
                    "latency_host_end": "result landed in the job's pinned host buffer",
                    "frac_within_own_integration_time_host": within(lat_h),
                    "p99_host_below_50ms": bool(np.percentile(lat_h, 99) < 0.050)})
    return res


# HBM bytes per launch of the C3 int8 kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs calibrated against a 1 GiB device copy (FETCH x 2.000,
# WRITE x 1.000); valid only for the sources they were taken on: the kernel
# and its work-item order (the C3 pass has one launch shape: no K split,
# 128-row tiles).
TRAFFIC_SOURCES = [os.path.join(ROOT, "paper_0906_1887_amd", "csrc", f)
                   for f in ("xengine_mfma.hip", "common.h")]
TRAFFIC_SHA1 = "85b74776252e1fe064bc1be4b03c5cc10555dacf"
TRAFFIC_BYTES = {"read": 2 * 27766799 * 1024, "write": 3383890 * 1024}


def traffic_sources_sha1() -> str:
    h = hashlib.sha1()
    for path in TRAFFIC_SOURCES:
        with open(path, "rb") as fh:
            h.update(hashlib.sha1(fh.read()).digest())
    return h.hexdigest()


def measured_traffic():
    if traffic_sources_sha1() != TRAFFIC_SHA1:
        return None
    return TRAFFIC_BYTES["read"] + TRAFFIC_BYTES["write"]


def time_events(fn, reps, stream):
    """Average ms of fn() over reps back-to-back calls, HIP events on stream."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def other_configs(dev, stream):
    """C1, C2 and C4 at their full sizes: one timed figure per step of the
    path, against its roofline (inputs made on the device; timing only, the
    parity of these configurations is checked by the GPU tests)."""
    out = {}
    out.update(c1_config(dev, stream))
    out.update(c2_config(dev, stream))
    out.update(c4_config(dev, stream))
    out.update(prototype_config(dev, stream))
    out.update(designs_config(dev, stream))
    return out


def designs_config(dev, stream, reps=3):
    """The paper's CMAC design comparison (Tables 2-4) on this GPU: one
    second of the prototype's spectra (64 inputs, 128 channels, 10000 spectra,
    complex float32 laid out [t][input][channel]) through pair parallel, hybrid
    group and group parallel, against the memory-bound model, beside this
    library's tiled plain-FP32 engine on the same spectra ([channel][input][t])."""
    import torch
    from paper_0906_1887_amd import Correlator, cmac_design, perfmodel
    n_in, n_ch, T, B = 64, 128, 10000, 1.28e6
    g = torch.Generator(device=dev).manual_seed(12)
    xs = torch.randn((T, n_in, n_ch, 2), device=dev, generator=g)
    out = torch.zeros((n_ch, n_in * (n_in + 1) // 2, 2), dtype=torch.float32, device=dev)
    hbm = perfmodel.MI355X["hbm_Bps"]
    paper_c1060 = {"PP": (2.6, 3.1), "HG2": (3.3, 4.1), "HG4": (3.8, 4.9), "GP2": (4.8, 6.1), "GP4": (6.9, 12.0)}
    res = {}
    for name, key in (("pp", "PP"), ("hg2", "HG2"), ("hg4", "HG4"), ("gp2", "GP2"), ("gp4", "GP4")):
        cmac_design(name, xs, out=out)
        ms = time_events(lambda: cmac_design(name, xs, out=out), reps, stream)
        eps = perfmodel.PAPER_EPS[key]
        b_act = B / (ms / 1e3)
        b_th = perfmodel.max_signal_bandwidth(hbm, eps, n_in)
        res[key] = {"ms": ms, "eps": eps, "actual_MHz": b_act / 1e6, "theoretical_MHz": b_th / 1e6,
                    "frac": b_act / b_th, "tcmac_s": perfmodel.xengine_cmac(n_ch, n_in, T) / (ms / 1e3) / 1e12,
                    "paper_c1060_MHz": {"actual": paper_c1060[key][0], "theoretical": paper_c1060[key][1]}}
    xc = xs.permute(2, 1, 0, 3).contiguous()              # [ch][input][t][2]
    del xs
    c = Correlator(n_in, n_ch, engine="fp32", sample_type="cf32", max_abs=0, device=str(dev))

    def tiled():
        c.correlate(xc)
        c.dump(0)
    tiled()
    ms = time_events(tiled, reps, stream)
    c.close()
    res["tiled_fp32"] = {"ms": ms, "actual_MHz": B / (ms / 1e3) / 1e6,
                         "tcmac_s": perfmodel.xengine_cmac(n_ch, n_in, T) / (ms / 1e3) / 1e12,
                         "note": "this library's FP32 engine (LDS-tiled 64x64, split K) on [channel][input][t]"}
    return {"designs_1s": {**res, "note": "1 s of 64 inputs x 1.28 MHz, 128 channels; theoretical = 8 TB/s / "
                                          "(4 eps N_I (N_I+1)) (the paper's memory-bound model); actual = "
                                          "1.28 MHz x (1 s / time); the paper's C1060 row for context"}}


def prototype_config(dev, stream, reps=10):
    """One second of the paper's prototype (Table 3's workload): 4 capture
    streams of 1.28 M records (marker + 16 words of 5+5-bit complex samples),
    64 inputs, 128 channels.  Times each step on the device: aggregation,
    complex F-stage (16-bit words; and the 1-byte mode), and the int8 and
    plain FP32 X-engines on the F-stage's ring."""
    import torch
    from paper_0906_1887_amd import Correlator, aggregate_w16, perfmodel
    hbm = perfmodel.MI355X["hbm_Bps"]
    ns, wp, nr = 4, 16, 1_280_000
    n_in, nb = ns * wp, nr // 128
    g = torch.Generator(device=dev).manual_seed(11)
    # any 16-bit word is a valid sample (bits above 9 are ignored); counters in word 0
    rec = torch.randint(-32768, 32768, (ns, nr, 1 + wp), dtype=torch.int32, device=dev, generator=g).to(torch.int16)
    rec[:, :, 0] = (torch.arange(nr, device=dev, dtype=torch.int32) & 0xFFFF).to(torch.int16)[None, :]
    rec = rec.contiguous()
    agg, bad = aggregate_w16(rec)
    b8 = torch.randint(0, 256, (nr, n_in), dtype=torch.int32, device=dev, generator=g).to(torch.uint8)
    s_req = float(torch.tensor(1.0 / 16.0, dtype=torch.float32))
    plans = {
        "i8": Correlator(n_in, 128, engine="i8", fft_size=128, max_abs=7, requant_scale=s_req, ring_samples=nb,
                         device=str(dev), volt_format="cw16"),
        "fp32": Correlator(n_in, 128, engine="fp32", fft_size=128, max_abs=7, requant_scale=s_req,
                           ring_samples=nb, device=str(dev), volt_format="cw16"),
        "b8": Correlator(n_in, 128, engine="i8", fft_size=128, max_abs=7, requant_scale=s_req, ring_samples=nb,
                         device=str(dev), volt_format="cb8"),
    }
    seq = {k: 0 for k in plans}

    def fx(key, volt):
        c = plans[key]
        c.channelise(volt, first_seq=seq[key])
        seq[key] += nb
        c.correlate(None)
        c.dump(0)

    for k, v in (("i8", agg), ("fp32", agg), ("b8", b8)):
        fx(k, v)
    torch.cuda.synchronize()
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    t = {"aggregate": 0.0, "fstage_w16": 0.0, "x_i8": 0.0, "x_fp32": 0.0, "fstage_b8": 0.0}
    for _ in range(reps):
        e = [ev() for _ in range(9)]
        e[0].record(stream)
        aggregate_w16(rec, out=agg, bad=bad)
        e[1].record(stream)
        c = plans["i8"]
        c.channelise(agg, first_seq=seq["i8"])
        e[2].record(stream)
        c.correlate(None)
        e[3].record(stream)
        c.dump(0)
        c = plans["fp32"]
        c.channelise(agg, first_seq=seq["fp32"])
        e[4].record(stream)
        c.correlate(None)
        e[5].record(stream)
        c.dump(0)
        c = plans["b8"]
        e[6].record(stream)
        c.channelise(b8, first_seq=seq["b8"])
        e[7].record(stream)
        c.correlate(None)
        c.dump(0)
        for k in seq:
            seq[k] += nb
        torch.cuda.synchronize()
        t["aggregate"] += e[0].elapsed_time(e[1])
        t["fstage_w16"] += e[1].elapsed_time(e[2])
        t["x_i8"] += e[2].elapsed_time(e[3])
        t["x_fp32"] += e[4].elapsed_time(e[5])
        t["fstage_b8"] += e[6].elapsed_time(e[7])
    t = {k: v / reps for k, v in t.items()}
    for c in plans.values():
        c.close()
    cm = perfmodel.xengine_cmac(128, n_in, nb)
    agg_bytes = ns * nr * (1 + wp) * 2 + nr * n_in * 2
    f16_bytes = nr * n_in * 2 + 128 * n_in * nb * 2
    f8_bytes = nr * n_in + 128 * n_in * nb * 2
    paper = {"unpack": 53.0, "fft": 53.0, "cmac_gp4": 185.0, "cmac_pp": 494.0}
    return {"prototype_1s": {
        "ms": t,
        "total_ms_w16_i8": t["aggregate"] + t["fstage_w16"] + t["x_i8"],
        "aggregate_frac_of_hbm": agg_bytes / (t["aggregate"] / 1e3) / hbm,
        "fstage_w16_frac_of_hbm": f16_bytes / (t["fstage_w16"] / 1e3) / hbm,
        "fstage_b8_frac_of_hbm": f8_bytes / (t["fstage_b8"] / 1e3) / hbm,
        "x_i8_tcmac_s": cm / (t["x_i8"] / 1e3) / 1e12,
        "x_fp32_tcmac_s": cm / (t["x_fp32"] / 1e3) / 1e12,
        "paper_c1060_ms": paper,
        "note": "1 s of 64 inputs x 1.28 MHz complex samples, 128 channels (10000 spectra per input); "
                "the paper's Table 3 (Tesla C1060, FP32 CMAC) is context: its CMAC is on FP32 spectra, "
                "ours on the F-stage's 4-bit requantised ring"}}


def c1_config(dev, stream):
    import torch
    import synth
    from paper_0906_1887_amd import Correlator, perfmodel
    out = {}

    # C1: FP32 X-engine, N_I=64, 128 channels, 1000 samples, complex float32
    # (integer-valued, so both engines are exact): the plain vector engine and
    # the matrix-core engine
    n_in, n_ch, T = 64, 128, 1000
    x8 = torch.empty((n_ch, n_in, T, 2), dtype=torch.int8, device=dev)
    synth.DeviceGen().fill_ci8(x8.data_ptr(), n_ch, n_in, T, 1, stream=stream.cuda_stream)
    xf = x8.float()
    cm = perfmodel.xengine_cmac(n_ch, n_in, T)
    for engine, key, what in (("fp32", "c1_fp32_plain", "plain FP32 vector FMA"),
                              ("fp32m", "c1_fp32_mfma", "FP32 on the matrix cores (v_mfma_f32_16x16x4_f32)")):
        c = Correlator(n_in, n_ch, engine=engine, sample_type="cf32", max_abs=7, device=str(dev))

        def c1():
            c.correlate(xf)
            c.dump(0)
        c1()
        ms = time_events(c1, 200, stream)
        out[key] = {"ms_per_integration": ms, "tcmac_s": cm / (ms / 1e3) / 1e12,
                    "frac_of_fp32_peak": cm / (ms / 1e3) / perfmodel.fp32_cmac_peak(),
                    "engine": what, "note": "X + accumulator reset per integration, 200 back-to-back"}
        c.close()
    del x8, xf
    return out


def c2_config(dev, stream, reps=20):
    import torch
    from paper_0906_1887_amd import Correlator, perfmodel
    hbm = perfmodel.MI355X["hbm_Bps"]
    out = {}

    # C2: F-stage (256-pt real FFT, requantise, corner turn) and X on the ring, N_I=64
    n_in, nb = 64, 10000
    s_req = float(torch.tensor(2.0 / (16.0 * 128 ** 0.5), dtype=torch.float32))
    # the C2 streams: Gaussian sigma 16, a common tone at channel 37, 10 % of
    # the noise power common to inputs 0..7 (the tests' generator)
    import synth
    volt = torch.from_numpy(synth.real_voltages(seed=2, index=0, n_blocks=nb, n_inputs=n_in)).to(dev)
    c = Correlator(n_in, 128, engine="i8", fft_size=256, max_abs=7, requant_scale=s_req, ring_samples=nb,
                   device=str(dev))
    seq = [0]

    def f():
        c.channelise(volt, first_seq=seq[0])
        seq[0] += nb
        c.correlate(None)
        c.dump(0)
    f()
    e = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
          torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    for k in range(reps):
        e[k][0].record(stream)
        c.channelise(volt, first_seq=seq[0])
        seq[0] += nb
        e[k][1].record(stream)
        c.correlate(None)
        e[k][2].record(stream)
        c.dump(0)
    torch.cuda.synchronize()
    f_ms = sum(a.elapsed_time(b) for a, b, _ in e) / reps
    x_ms = sum(b.elapsed_time(d) for _, b, d in e) / reps
    f_bytes = nb * 256 * n_in + 128 * n_in * nb * 2
    x_bytes = 128 * n_in * nb * 2 + 128 * (n_in * (n_in + 1) // 2) * 8
    cm = perfmodel.xengine_cmac(128, n_in, nb)
    out["c2_fx"] = {"fstage_ms": f_ms, "fstage_GB_s": f_bytes / (f_ms / 1e3) / 1e9,
                    "fstage_frac_of_hbm": f_bytes / (f_ms / 1e3) / hbm,
                    "xengine_ms": x_ms, "xengine_GB_s": x_bytes / (x_ms / 1e3) / 1e9,
                    "xengine_frac_of_hbm": x_bytes / (x_ms / 1e3) / hbm,
                    "xengine_tcmac_s": cm / (x_ms / 1e3) / 1e12,
                    "note": "per integration of 10000 blocks x 64 inputs; algorithmic bytes: F 1 B in + 2 B out "
                            "per sample, X 2 B per sample in + 8 B per product out"}
    c.close()
    # the polyphase-filterbank F-stage (4 taps) on the same data, 3 blocks of history added
    vp = torch.cat([volt[: 3 * 256], volt]).contiguous()
    c = Correlator(n_in, 128, engine="i8", fft_size=256, max_abs=7, requant_scale=s_req, ring_samples=nb,
                   device=str(dev), pfb_taps=4)
    sq = [0]

    def fp():
        c.channelise(vp, first_seq=sq[0])
        sq[0] += nb
        c.correlate(None)
        c.dump(0)
    fp()
    pf = 0.0
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        c.channelise(vp, first_seq=sq[0])
        e1.record(stream)
        sq[0] += nb
        c.correlate(None)
        c.dump(0)
        torch.cuda.synchronize()
        pf += e0.elapsed_time(e1)
    pf /= reps
    c.close()
    out["c2_fx"]["fstage_pfb4_ms"] = pf
    out["c2_fx"]["fstage_pfb4_frac_of_hbm"] = f_bytes / (pf / 1e3) / hbm
    del volt, vp
    return out


def c4_samples(dev, n_ch, n_in, T, seed=4, rho=0.1):
    """The C4 inputs on the device: complex Gaussian samples of unit variance,
    per-input gains in [0.5, 2] and coherence rho on 16 disjoint input pairs
    (the recipe of synth.complex_float, with the same gains and pairs; the
    noise comes from torch's device generator, 8.6 GB being too large to draw
    on the host)."""
    import math
    import torch
    import synth
    gains = torch.tensor(synth.input_gains(seed, n_in), dtype=torch.float32, device=dev)
    g = torch.Generator(device=dev).manual_seed(seed)
    s = math.sqrt(0.5)
    x = torch.randn((n_ch, n_in, T, 2), device=dev, generator=g)
    x *= s
    for a, b in synth.coherent_pairs(seed, n_in, 16):
        c = torch.randn((n_ch, T, 2), device=dev, generator=g) * s
        x[:, a] = math.sqrt(1.0 - rho) * x[:, a] + math.sqrt(rho) * c
        x[:, b] = math.sqrt(1.0 - rho) * x[:, b] + math.sqrt(rho) * c
    x *= gains.view(1, n_in, 1, 1)
    return x


def c4_config(dev, stream):
    import torch
    from paper_0906_1887_amd import Correlator, perfmodel
    hbm = perfmodel.MI355X["hbm_Bps"]
    out = {}

    # C4: FP16 / FP8 matrix-core X-engine on complex float32 samples, N_I=256,
    # 1024 channels, 4096 samples: the converting plan (conversion inside the
    # X-engine's loads) and, beside it, the staged plan (a conversion pass
    # writes FP16 / FP8 rows that the X-engine then reads)
    n_in, n_ch, T = 256, 1024, 4096
    xf = c4_samples(dev, n_ch, n_in, T)
    cm = perfmodel.xengine_cmac(n_ch, n_in, T)
    out_bytes = n_ch * (n_in * (n_in + 1) // 2) * 8
    for engine, peak, sb in (("f16", perfmodel.MI355X["fp16_flops"], 4), ("f8", perfmodel.MI355X["fp8_flops"], 2)):
        res = {}
        for mode, ring in (("converting", 0), ("staged", T)):
            c = Correlator(n_in, n_ch, engine=engine, sample_type="cf32", max_abs=0, ring_samples=ring,
                           device=str(dev))

            def f4():
                c.correlate(xf, T)
                c.dump(0)
            f4()
            res[mode] = time_events(f4, 5, stream)
            c.close()
        nbytes = n_ch * n_in * T * 8 + out_bytes
        staged_bytes = n_ch * n_in * T * (8 + 2 * sb) + out_bytes
        best = min(res, key=res.get)
        ms = res[best]
        out[f"c4_{engine}"] = {"ms": ms, "plan": best, "tcmac_s": cm / (ms / 1e3) / 1e12,
                               "frac_of_mfma_peak": cm * 8 / (ms / 1e3) / peak,
                               "GB_s": nbytes / (ms / 1e3) / 1e9, "frac_of_hbm": nbytes / (ms / 1e3) / hbm,
                               "converting_ms": res["converting"], "staged_ms": res["staged"],
                               "staged_frac_of_hbm_incl_staging": staged_bytes / (res["staged"] / 1e3) / hbm,
                               "note": "ms, GB_s and frac_of_hbm: the faster plan, on the algorithmic bytes "
                                       "(FP32 samples read once, output written); the staged plan also "
                                       "writes and reads the FP16 / FP8 copy"}
    del xf
    torch.cuda.empty_cache()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-ci4", action="store_true")
    ap.add_argument("--cpu-channels", type=int, default=64)
    ap.add_argument("--serve-seconds", type=float, default=52.0)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-host-seconds", type=float, default=20.0)
    ap.add_argument("--serve-host-rate", type=float, default=100.0)
    ap.add_argument("--no-other-configs", action="store_true")
    ap.add_argument("--mode", choices=["bench", "copy", "c2", "c4", "proto", "designs"], default="bench",
                    help="copy: only a 1 GiB device-to-device copy, the known-size reference for "
                         "calibrating rocprofv3 FETCH_SIZE / WRITE_SIZE counters; c2: only the C2 "
                         "F-stage + X-engine timing (for profiling the F-stage); c4: only the C4 FP16 / "
                         "FP8 plans; proto: only one second of the prototype's complex front end; designs: "
                         "only the paper's CMAC designs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the channel-sharded multi-GPU design is described, not built", file=sys.stderr)
        return 2

    import torch

    if args.mode == "copy":
        a = torch.ones(1 << 30, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read": 1 << 30, "bytes_written": 1 << 30, "copies": 3}))
        return 0

    import synth
    from paper_0906_1887_amd import Correlator, perfmodel

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    if args.mode == "c2":
        print(json.dumps({"mode": "c2", **c2_config(dev, stream, reps=args.steps)}))
        return 0
    if args.mode == "c4":
        print(json.dumps({"mode": "c4", **c4_config(dev, stream)}))
        return 0
    if args.mode == "proto":
        print(json.dumps({"mode": "proto", **prototype_config(dev, stream, reps=args.steps)}))
        return 0
    if args.mode == "designs":
        print(json.dumps({"mode": "designs", **designs_config(dev, stream, reps=args.steps)}))
        return 0
    log("generating input on device")
    x = torch.empty((N_CH, N_IN, N_T, 2), dtype=torch.int8, device=dev)
    synth.DeviceGen().fill_ci8(x.data_ptr(), N_CH, N_IN, N_T, SEED, stream=stream.cuda_stream)
    torch.cuda.synchronize()

    cmac = perfmodel.xengine_cmac(N_CH, N_IN, N_T)
    log("int8 engine")
    c = Correlator(N_IN, N_CH, engine="i8", sample_type="ci8", max_abs=7, device="cuda:0")
    for _ in range(args.warmup):
        c.correlate(x)
        c.dump(0)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record(stream)
        c.correlate(x)
        evs[k][1].record(stream)
        c.dump(0)  # reset: the next step is a fresh integration
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    kern_ms = sorted(s.elapsed_time(e) for s, e in evs)
    kern_avg = sum(kern_ms) / len(kern_ms)

    # dump read-out latency of one integration (3.2 GB int32 triangle)
    c.correlate(x)
    out_dev = torch.empty((N_CH, N_IN * (N_IN + 1) // 2, 2), dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    td = time.perf_counter()
    c.dump(1, out=out_dev)
    dump_dev_ms = (time.perf_counter() - td) * 1e3
    c.correlate(x)
    out_host = torch.empty((N_CH, N_IN * (N_IN + 1) // 2, 2), dtype=torch.int32, pin_memory=True)
    torch.cuda.synchronize()
    td = time.perf_counter()
    c.dump(1, out=out_host)
    dump_host_ms = (time.perf_counter() - td) * 1e3
    del out_host
    c.close()
    del c

    fp32 = None
    if not args.no_fp32:
        log("plain FP32 engine")
        f = Correlator(N_IN, N_CH, engine="fp32", sample_type="ci8", max_abs=7, device="cuda:0")
        f.correlate(x)
        vf, _, _ = f.dump(1)
        same = bool(torch.equal(out_dev.to(torch.float32), vf))
        del vf
        reps = 3
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            f.correlate(x)
            f.dump(0)
        e1.record(stream)
        torch.cuda.synchronize()
        fms = e0.elapsed_time(e1) / reps
        f.close()
        fp32 = {"value": cmac / (fms / 1e3) / 1e12, "unit": "Tcmac/s", "ms": fms, "bitexact_vs_int8": same,
                "peak_tcmac": perfmodel.fp32_cmac_peak() / 1e12,
                "frac": cmac / (fms / 1e3) / perfmodel.fp32_cmac_peak()}
    ci4 = None
    if not args.no_ci4:
        log("int8 engine on one byte per sample (CI4)")
        b = (((x[..., 0] & 15) << 4) | (x[..., 1] & 15)).contiguous()     # the same samples, packed
        g = Correlator(N_IN, N_CH, engine="i8", sample_type="ci4", max_abs=7, device="cuda:0")
        g.correlate(b)
        v4, _, _ = g.dump(1)
        same4 = bool(torch.equal(v4, out_dev))
        del v4
        for _ in range(args.warmup):
            g.correlate(b)
            g.dump(0)
        torch.cuda.synchronize()
        evs4 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                for _ in range(args.steps)]
        for k in range(args.steps):
            evs4[k][0].record(stream)
            g.correlate(b)
            evs4[k][1].record(stream)
            g.dump(0)
        torch.cuda.synchronize()
        ms4 = sorted(s_.elapsed_time(e_) for s_, e_ in evs4)
        g.close()
        del b
        avg4 = sum(ms4) / len(ms4)
        ci4 = {"value": cmac / (avg4 / 1e3) / 1e12, "unit": "Tcmac/s", "kernel_ms_avg": avg4,
               "kernel_ms_median": ms4[len(ms4) // 2],
               "frac_of_int8_peak": perfmodel.REAL_MACS_PER_CMAC * 2 * cmac / (avg4 / 1e3) / perfmodel.MI355X["int8_ops"],
               "bitexact_vs_int8_pairs": same4, "input_bytes": N_CH * N_IN * N_T,
               "note": "the C3 samples packed one byte per sample (re in the high nibble); beside, not replacing, "
                       "the int8-pair headline"}
    del out_dev

    # roofline of the dominant kernel: int8 MFMA ops (4 real MACs = 8 ops per CMAC)
    ops = perfmodel.REAL_MACS_PER_CMAC * 2 * cmac
    achieved = ops / (kern_avg / 1e3) / 1e12
    peak = perfmodel.MI355X["int8_ops"] / 1e12
    roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": measured_traffic(), "kernel": "corr::xeng_mfma_128_kernel<0> (int8 v_mfma_i32_16x16x64_i8, 128x128 tiles, 4 waves of 64x64)",
            "kernel_ms_avg": kern_avg, "kernel_ms_min": kern_ms[0], "kernel_ms_median": kern_ms[len(kern_ms) // 2],
            "algorithmic_bytes": float(N_CH * N_IN * N_T * 2 + N_CH * (N_IN * (N_IN + 1) // 2) * 8)}

    serve = None
    if not args.no_serving:
        log("serving loop")
        del x
        torch.cuda.empty_cache()
        serve = serving(args.serve_seconds, warm=1.0, rate=200.0, host=False)
        log("serving loop, results to host memory")
        serve["host_end_point"] = serving(args.serve_host_seconds, warm=1.0, rate=args.serve_host_rate, host=True)
        serve["host_end_point"]["note"] = (
            "the mean dump of this job mix is 387 MB (N_C x N_I(N_I+1)/2 x 8 B), so 200 jobs/s would need "
            "77 GB/s from device to host, beyond a PCIe 5.0 x16 link; the host end point is measured at a "
            "rate the link carries")
        x = None

    others = None
    if not args.no_other_configs:
        log("C1, C2, C4")
        x = None
        torch.cuda.empty_cache()
        others = other_configs(dev, stream)

    cpu = None
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        if x is None:
            x = torch.empty((args.cpu_channels, N_IN, N_T, 2), dtype=torch.int8, device=dev)
            synth.DeviceGen().fill_ci8(x.data_ptr(), args.cpu_channels, N_IN, N_T, SEED,
                                       stream=stream.cuda_stream)
            torch.cuda.synchronize()
        cpu = cpu_baseline(x, args.cpu_channels)
        log("CPU oracle on C1, C2 and C4")
        cpu["other_configs"] = cpu_other_configs()
        cpu["one_thread"]["gpu_int8_over_this"] = (cmac / (ms_per_step / 1e3) / 1e12) / cpu["one_thread"]["value"]

    value = cmac / (ms_per_step / 1e3) / 1e12
    line = {
        "metric": "X-engine Tcmac/s at N_I=1024 (int8 MFMA vs FP32 plain, bit-exact); p99 dump latency",
        "value": value,
        "unit": "Tcmac/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic (seeded device generator, clipped rounded Gaussian sigma=2 in [-7,7])",
        "config": {"workload": "full-array X-engine: N_I=1024, 768 channels, 8000 samples, int8 pairs",
                   "n_inputs": N_IN, "n_channels": N_CH, "n_samples": N_T, "engine": "int8 MFMA",
                   "cmac_per_step": cmac},
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp32_plain": fp32,
        "ci4": ci4,
        "serving": serve,
        "other_configs": others,
        "dump_ms": {"device": dump_dev_ms, "host_pinned": dump_host_ms, "bytes": N_CH * N_IN * (N_IN + 1) // 2 * 8},
        "paper_context": "60x over one CPU thread at 32 antennas on 2008 NVIDIA hardware (abstract); context only",
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
