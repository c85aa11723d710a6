"""X-stage benchmark on one MI355X.

Workload: LWA-scale array, 256 antennas x 2 polarisations = 512 inputs,
4096 channels, 4096 samples per integration, 4+4-bit complex samples
(Gaussian noise plus a 5%-correlated point source with per-antenna delays),
generated on the device from a fixed seed.

One step = one integration window through the whole hot path: every sample of
every channel read from HBM, unpacked, cross-multiplied on the int8 MFMA and
integrated, and the exact int64 lower-triangle visibilities of all channels
written to HBM (xcorr_accumulate_dump with reset).  Inputs are resident in HBM
before the timed region.  The fp16-MFMA and plain fp32 kernels run the same
window for comparison, and the CPU oracle is timed on a bounded sample.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "X-engine TCMAC/s and % int8-MFMA peak vs FP32 kernel, N=256 dual-pol"
PEAK_INT8_TOPS = 5000.0       # MI355X dense int8 MFMA, vendor figure
PEAK_FP16_TFLOPS = 2500.0
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
PEAK_CLOCK_MHZ = 2400.0       # shader clock at which the vendor peaks are quoted
CLOCK_PROBE_MS = 20.0         # wall time the clock probe spans during timed windows
# HBM-traffic record of the int8 kernel (FETCH_SIZE / WRITE_SIZE counters on
# this workload plus a copy-kernel calibration), tied to the kernel sources.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "xcorr_i8_lwa_traffic.md")
# The kernel, its launch arguments, the work-item plan (xcorr_items.cpp) and
# the build flags: a change to any of them can change the kernel's traffic.
KERNEL_SOURCES = ("paper_1401_8288_amd/csrc/xcorr_i8.hip", "paper_1401_8288_amd/csrc/xcorr_device.h",
                  "paper_1401_8288_amd/csrc/xcorr_internal.h", "paper_1401_8288_amd/csrc/xcorr_items.cpp",
                  "paper_1401_8288_amd/build.py")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_path(torch, xcorr, x, w, path, steps, warmup, flags=0, per_step=None, clock=None, tile=0):
    """Average ms of one accumulate_dump window on the plan's stream (HIP
    events around all steps).  If per_step is a list, the ms of each step
    (events between steps) are appended to it.  If clock is a dict, after
    the timed steps a few more windows run untimed with a clock probe on a
    side stream beside them, and clock["mhz"] receives the shader clock it
    saw (the probe is kept out of the timed steps: its wave shares a CU with
    one workgroup of the persistent launch)."""
    p = xcorr.Plan(w.n_inputs, w.n_channels, w.fmt, path, flags=flags, tile=tile)
    out = p.new_output()
    for _ in range(warmup):
        p.accumulate_dump(x, out)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(p.stream)
    for k in range(steps):
        p.accumulate_dump(x, out)
        ev[k + 1].record(p.stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[steps]) / steps
    if clock is not None:
        probe = xcorr.ClockProbe(x.device)
        side = torch.cuda.Stream(device=x.device)
        n_extra = max(2, int(2 * CLOCK_PROBE_MS / ms) + 1)
        for _ in range(n_extra):
            p.accumulate_dump(x, out)
        probe.start(CLOCK_PROBE_MS, side)       # enqueued after the windows: starts beside the first
        torch.cuda.synchronize()
        clock["mhz"] = probe.mhz()
    if per_step is not None:
        per_step.extend(ev[k].elapsed_time(ev[k + 1]) for k in range(steps))
    info = p.query()
    p.close()
    return ms, out, info


def time_accumulate(torch, xcorr, x, w, steps, warmup, per_step=None):
    """Average ms of xcorr_accumulate alone into an int64 plan: every window
    adds into the plan's int32 accumulator (read and written), which is
    folded into the int64 one before its sums could overflow (after
    16777215 samples of 4-bit data, 65535 of 8-bit data).  If per_step is a
    list, the ms of each step are appended to it."""
    p = xcorr.Plan(w.n_inputs, w.n_channels, w.fmt, "i8")
    for _ in range(warmup):
        p.accumulate(x)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(p.stream)
    for k in range(steps):
        p.accumulate(x)
        ev[k + 1].record(p.stream)
    torch.cuda.synchronize()
    if per_step is not None:
        per_step.extend(ev[k].elapsed_time(ev[k + 1]) for k in range(steps))
    p.close()
    return ev[0].elapsed_time(ev[steps]) / steps


def pcie_leg(torch, x, out_bytes, reps=3):
    """Host-resident window: the input copied in from pinned host memory and
    the int32 result copied back out (HIP events, best of `reps`), for the
    PCIe-inclusive rate.  The boundary itself takes device buffers."""
    dev = x.device
    n_in = x.numel() * x.element_size()
    flat = torch.empty(n_in, dtype=torch.uint8, device=dev)     # scratch: x itself stays intact
    h_in = torch.empty(n_in, dtype=torch.uint8, pin_memory=True)
    h_out = torch.empty(out_bytes, dtype=torch.uint8, pin_memory=True)
    d_out = torch.empty(out_bytes, dtype=torch.uint8, device=dev)
    s = torch.cuda.Stream(device=dev)
    best_in = best_out = None
    with torch.cuda.stream(s):
        for _ in range(reps):
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record(s)
            flat.copy_(h_in, non_blocking=True)
            e1.record(s)
            h_out.copy_(d_out, non_blocking=True)
            e2.record(s)
            s.synchronize()
            t_in, t_out = e0.elapsed_time(e1), e1.elapsed_time(e2)
            best_in = t_in if best_in is None else min(best_in, t_in)
            best_out = t_out if best_out is None else min(best_out, t_out)
    return {"h2d_bytes": flat.numel(), "h2d_ms": round(best_in, 3),
            "h2d_gbs": round(flat.numel() / best_in / 1e6, 1),
            "d2h_bytes": out_bytes, "d2h_ms": round(best_out, 3),
            "d2h_gbs": round(out_bytes / best_out / 1e6, 1)}


def percentile(v, q):
    s = sorted(v)
    return s[min(len(s) - 1, max(0, int(round(q / 100.0 * (len(s) - 1)))))]


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def read_traffic():
    """HBM bytes per launch of the int8 kernel from the recorded counters.

    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are each scaled by the ratio
    of known bytes to counted bytes for the library's plain copy kernel in the
    same runs.  None if no record exists or the kernel sources changed since
    the counters were taken.
    """
    if not os.path.exists(TRAFFIC_FILE):
        return None, "no record"
    rec = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith(("#", " ", "|", "`")):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    try:
        if rec["kernel_sources_sha256"] != kernel_sources_sha256():
            return None, "kernel changed since the counters were taken"
        f_fetch = float(rec["copy_bytes"]) / (1024 * float(rec["copy_fetch_kib"]))
        f_write = float(rec["copy_bytes"]) / (1024 * float(rec["copy_write_kib"]))
        t = 1024 * (float(rec["fetch_kib"]) * f_fetch + float(rec["write_kib"]) * f_write)
    except (KeyError, ValueError, ZeroDivisionError):
        return None, "incomplete record"
    return t, "FETCH_SIZE x %.4f + WRITE_SIZE x %.4f (copy-kernel calibration)" % (f_fetch, f_write)


def pmc_summary(directory):
    """Per-kernel averages of rocprofv3 counter CSVs under a directory."""
    import collections
    import csv
    import glob
    agg = collections.OrderedDict()
    for f in sorted(glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)):
        for r in csv.DictReader(open(f)):
            key = (r["Kernel_Name"], r["Counter_Name"])
            agg.setdefault(key, []).append(float(r["Counter_Value"]))
    for (k, c), v in agg.items():
        print("%-70s %-30s dispatches=%d avg=%.6g" % (k[:70], c, len(v), sum(v) / len(v)))


def trace_summary(directory, skip, take, match):
    """Per-kernel durations of rocprofv3 kernel-trace CSVs under a directory:
    for every kernel whose name contains `match`, its dispatches in start
    order, the first `skip` left out (warm-up windows) and the next `take`
    averaged (the timed windows; all the rest if take is 0).  Prints a
    markdown table."""
    import collections
    import csv
    import glob
    runs = collections.OrderedDict()
    for f in sorted(glob.glob(os.path.join(directory, "**", "*kernel_trace.csv"), recursive=True)):
        for r in csv.DictReader(open(f)):
            if match and match not in r["Kernel_Name"]:
                continue
            runs.setdefault(r["Kernel_Name"], []).append(
                (int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    print("| Kernel | Dispatches | Used | Average ns | Min ns | Max ns |")
    print("|---|---|---|---|---|---|")
    for k, v in runs.items():
        d = [dt for _, dt in sorted(v)]
        sel = d[skip:skip + take] if take else d[skip:]
        if not sel:
            continue
        print("| `%s` | %d | %d..%d | %d | %d | %d |" % (k[:90], len(d), skip, skip + len(sel) - 1,
                                                      sum(sel) // len(sel), min(sel), max(sel)))


def copy_calibration(torch, xcorr, x, w):
    """One non-fused window, then a dump without reset: the library's copy
    kernel moves exactly output_bytes (read and written)."""
    p = xcorr.Plan(w.n_inputs, w.n_channels, w.fmt, "i8", flags=xcorr.FLAG_OUT_I32)
    out = p.new_output()
    p.accumulate(x)
    p.dump(out, reset=False)
    torch.cuda.synchronize()
    log("copy calibration: %d bytes copied" % p.query().output_bytes)
    p.close()


def run_serving(torch, xcorr, pool, shapes, seconds, speedup, seed, tune_path=None, inflight=1):
    """Streams of the given shapes feed windows of 1024-4096 samples into the
    server as Poisson processes whose mean gap is the window's duration
    (N_t x 40.96 us) divided by `speedup`; a window's deadline is that same
    duration / speedup after its arrival."""
    import random
    from paper_1401_8288_amd import synth
    rng = random.Random(seed)
    lens = (1024, 2048, 3072, 4096)
    srv = xcorr.Server(device_budget=64 << 30, max_streams=64, max_inflight=inflight, tune_path=tune_path)
    sids, outs, busy = [], [], []
    for (n_in, n_ch) in shapes:
        sids.append(srv.open(n_in, n_ch))
        srv.set_deadline(sids[-1], synth.SPECTRUM_INTERVAL_S / speedup)
        outs.append([srv.new_output(sids[-1]) for _ in range(8)])
        busy.append([None] * 8)
    events = []
    for k in range(len(sids)):
        t = 0.0
        while True:
            nt = rng.choice(lens)
            dur = nt * synth.SPECTRUM_INTERVAL_S / speedup
            t += rng.expovariate(1.0 / dur)
            if t > seconds:
                break
            events.append((t, k, nt, dur))
    events.sort()
    tickets = []
    t0 = time.perf_counter()
    for (ta, k, nt, dur) in events:
        delay = ta - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        slot = next((j for j in range(8) if busy[k][j] is None or srv.poll(busy[k][j])[0]), None)
        if slot is None:
            srv.wait(busy[k][0])
            slot = 0
        tk = srv.submit(sids[k], pool[k][nt], outs[k][slot])
        busy[k][slot] = tk
        tickets.append((tk, dur))
    for tk, dur in tickets:
        srv.wait(tk)
    st = srv.stats()
    misses = st["deadline_misses"]
    srv.close()
    cmac_rt = sum(n * (n + 1) // 2 * c for (n, c) in shapes) / synth.SPECTRUM_INTERVAL_S
    return {"speedup_vs_real_time": speedup, "seconds": seconds, "windows": st["windows_done"],
            "offered_tcmac_s": round(cmac_rt * speedup / 1e12, 3),
            "achieved_tcmac_s": round(st["cmac"] / st["elapsed_s"] / 1e12, 3) if st["elapsed_s"] else None,
            "latency_p50_ms": round(st["latency_p50_ms"], 3), "latency_p99_ms": round(st["latency_p99_ms"], 3),
            "latency_max_ms": round(st["latency_max_ms"], 3), "deadline_misses": int(misses),
            "launches": st["launches"], "mean_windows_per_launch": round(st["mean_batch"], 2),
            "mixes_tuned": st["mixes_tuned"], "max_inflight": inflight}


def serving_leg(torch, xcorr, seconds, speedups, seed=7, inflight=1):
    """Batched streaming of the five subarrays (16/48/96/200/352 dual-pol
    antennas, 512/1024/2048/256/128 channels, 4-bit), one run per arrival
    rate (multiple S of real time), with the launch configuration tuned on
    the first run and kept in a cache file for the later ones.  Reports each
    run and the largest S without a missed deadline."""
    import os
    import tempfile
    from paper_1401_8288_amd import synth
    dev = torch.device("cuda:0")
    lens = (1024, 2048, 3072, 4096)
    pool = [{t: synth.generate(synth.subarray_workload(k, t), device=dev) for t in lens}
            for k in range(len(synth.SUBARRAYS))]
    torch.cuda.synchronize()
    shapes = [(synth.subarray_workload(k, 1).n_inputs, synth.subarray_workload(k, 1).n_channels)
              for k in range(len(synth.SUBARRAYS))]
    # one step of all five at 4096 samples: autotuned batch, graph replay,
    # one launch per plan
    step = batch_step(torch, xcorr, [pool[k][4096] for k in range(len(shapes))], shapes, autotune=True)
    tune = os.path.join(tempfile.mkdtemp(prefix="xcorr_tune_"), "tune.txt")
    runs = [run_serving(torch, xcorr, pool, shapes, seconds, sp, seed, tune, inflight) for sp in speedups]
    clean = [r["speedup_vs_real_time"] for r in runs if r["deadline_misses"] == 0]
    return {"workload": "5 subarrays of 16/48/96/200/352 dual-pol antennas, 512/1024/2048/256/128 channels, "
                        "4+4-bit, Poisson windows of 1024-4096 samples",
            "step_4096_samples": step,
            "runs": runs, "largest_clean_speedup": max(clean) if clean else None}


def batch_step(torch, xcorr, xs, shapes, autotune=False, reps=20):
    """One integration step of several plans (window xs[k] for the plan of
    shapes[k]) three ways: one batched launch per time chunk (optionally
    with the autotuner's configuration), the same step captured once and
    replayed as a graph, and one launch per plan.  Direct steps and replays
    are each timed twice in turn after a warm-up (the clock settles over the
    first tens of launches) and the better block of each is kept."""
    dev = xs[0].device
    s = torch.cuda.Stream(device=dev)        # a stream of their own: the step is also captured as a graph
    plans = [xcorr.Plan(n_in, n_ch, "ci4", "i8", stream=s) for (n_in, n_ch) in shapes]
    outs = [p.new_output() for p in plans]
    b = xcorr.Batch(plans, stream=s)
    torch.cuda.synchronize()
    res = {}
    if autotune:
        cfg, _ = b.autotune(xs)
        res["autotuned_config"] = cfg
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(step):
        e0.record(s)
        for _ in range(reps):
            step()
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    g = b.capture(xs, outs)
    for _ in range(10):
        b.run(xs, outs)
        g.launch()
    torch.cuda.synchronize()
    run = lambda: b.run(xs, outs)
    ms_batch, ms_graph = timed(run), timed(g.launch)
    ms_batch, ms_graph = min(ms_batch, timed(run)), min(ms_graph, timed(g.launch))
    g.close()

    def per_plan():
        for p, x, o in zip(plans, xs, outs):
            p.accumulate_dump(x, o)
    for _ in range(3):
        per_plan()
    torch.cuda.synchronize()
    ms_seq = timed(per_plan)
    b.close()
    for p in plans:
        p.close()
    cmac = sum(n_in * (n_in + 1) // 2 * n_ch * x.shape[1] for (n_in, n_ch), x in zip(shapes, xs))
    res.update({"one_batched_launch_ms": round(ms_batch, 4), "one_launch_per_plan_ms": round(ms_seq, 4),
                "batched_speedup": round(ms_seq / ms_batch, 2), "one_graph_replay_ms": round(ms_graph, 4),
                "tcmac_s_batched": round(cmac / ms_batch / 1e9, 2)})
    return res


def many_small_leg(torch, xcorr, seconds, speedups, n_sub=32, n_ant=16, n_ch=512, seed=9, inflight=1):
    """Many small arrays: n_sub subarrays of n_ant dual-pol antennas and n_ch
    channels, 4-bit.  One step of all of them (4096 samples each) as one
    batched launch against the same windows as one launch per plan, and the
    server at each of `speedups` times real time."""
    from paper_1401_8288_amd import synth
    dev = torch.device("cuda:0")
    n_in = 2 * n_ant
    lens = (1024, 2048, 3072, 4096)
    pool = []
    for k in range(n_sub):
        w = synth.Workload("small%d" % k, n_in, n_ch, 4096, "ci4", "tone", 500 + k,
                           {"noise_sigma": 2.5, "tone_gain": 0.0})
        pool.append({t: synth.generate(synth.scaled(w, n_time=t), device=dev) for t in lens})
    torch.cuda.synchronize()
    xs = [pool[k][4096] for k in range(n_sub)]
    step = batch_step(torch, xcorr, xs, [(n_in, n_ch)] * n_sub)
    runs = [run_serving(torch, xcorr, pool, [(n_in, n_ch)] * n_sub, seconds, sp, seed, inflight=inflight)
            for sp in speedups]
    clean = [r["speedup_vs_real_time"] for r in runs if r["deadline_misses"] == 0]
    return {"workload": "%d subarrays of %d dual-pol antennas, %d channels, 4+4-bit" % (n_sub, n_ant, n_ch),
            "step_4096_samples": step,
            "serving": runs, "largest_clean_speedup": max(clean) if clean else None}


def corner_turn_leg(torch, xcorr, w, reps=5, n_fengines=16, spectra_per_packet=8):
    """The corner turn in front of the X-stage at the workload's size: packets
    of `spectra_per_packet` spectra from `n_fengines` F-engines (16 x 32 inputs
    for 512), reordered to [channel][time][input]; HBM-bound (one read, one
    write of every byte)."""
    J = w.n_inputs // n_fengines
    S = spectra_per_packet
    B = w.n_time // S
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev).manual_seed(11)
    packets = torch.randint(0, 256, (B * n_fengines * S * w.n_channels * J,), dtype=torch.uint8,
                            device=dev, generator=g)
    out = torch.empty((w.n_channels, B * S, w.n_inputs), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    xcorr.corner_turn(packets, n_fengines, J, w.n_channels, S, out=out, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        xcorr.corner_turn(packets, n_fengines, J, w.n_channels, S, out=out, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 2 * packets.numel()
    del packets, out
    torch.cuda.empty_cache()
    return {"layout": "%d F-engines x %d inputs, %d spectra per packet, %d channels, %d packets per F-engine"
                      % (n_fengines, J, S, w.n_channels, B),
            "ms": round(ms, 4), "bytes_moved": nbytes, "gbs": round(nbytes / ms / 1e6, 1),
            "hbm_frac": round(nbytes / ms / 1e6 / PEAK_HBM_GBS, 4)}


def fstage_leg(torch, xcorr, w, reps=3, n_taps=2):
    """The GPU F-stage that makes the workload's input: w.n_inputs int8 ADC
    streams through the 2-tap 8192-point PFB, all 4096 channels, w.n_time
    spectra, requantised to 4+4 bits in X-stage order (transform kernel plus
    transpose).  Algorithmic work per ADC sample: 2 P flops of filter bank and
    2.5 log2(N) of real transform; HBM bytes: the samples once, the codes
    written, read and written again by the transpose."""
    from paper_1401_8288_amd import synth
    N = 8192
    if w.n_channels != N // 2:
        return None
    dev = torch.device("cuda:0")
    n_samples = (w.n_time + n_taps - 1) * N
    adc = synth.adc_input(w.n_inputs, n_samples, 1, device=dev)
    h = synth.pfb_coefficients(n_taps, N).to(dev)
    gain = synth.fstage_gains(w.n_inputs, w.n_channels, h).to(dev)
    out = torch.empty((w.n_channels, w.n_time, w.n_inputs), dtype=torch.uint8, device=dev)
    work = torch.empty(w.n_inputs * w.n_time * w.n_channels, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    run = lambda: xcorr.fstage(adc, h, gain, 0, w.n_channels, n_taps=n_taps, out=out, work=work, stream=stream)
    run()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        run()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    samples = w.n_inputs * w.n_time * N
    flops = samples * (2 * n_taps + 2.5 * 13)
    codes = w.n_inputs * w.n_time * w.n_channels
    # algorithmic HBM bytes: the ADC samples read once and the codes written
    # once; the transpose pass's write and read-back of the input-major codes
    # is reported beside it, not counted as useful traffic
    nbytes = w.n_inputs * n_samples + codes
    extra = 2 * codes
    del adc, out, work
    torch.cuda.empty_cache()
    return {"config": "%d inputs, %d-tap %d-point PFB, %d channels, %d spectra, CI4 out in X-stage order"
                      % (w.n_inputs, n_taps, N, w.n_channels, w.n_time),
            "ms": round(ms, 4), "gsamples_s": round(samples / ms / 1e6, 1),
            "bound": "alu", "achieved": round(flops / ms / 1e9, 2), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": round(flops / ms / 1e9 / PEAK_FP32_TFLOPS, 4),
            "algorithmic_flops_per_sample": 2 * n_taps + 2.5 * 13,
            "hbm_bytes": nbytes, "hbm_gbs": round(nbytes / ms / 1e6, 1),
            "transpose_extra_bytes": extra}


def variants_leg(torch, xcorr, x, w, reps=3, period=700, on=0.09):
    """Pulsar gating and baseline-dependent integration at the workload's
    size: two gates (on-pulse for the first `on` of every `period` samples,
    off-pulse the rest) through xcorr_accumulate_gated, and a tile dump of a
    third of the 64 x 64 tiles with restart (bytes: the selected entries
    read, written out and zeroed)."""
    import numpy as np
    g = np.array([1 if (t % period) < on * period else 0 for t in range(w.n_time)], dtype=np.uint8)
    plans = [xcorr.Plan(w.n_inputs, w.n_channels, w.fmt, "i8") for _ in range(2)]
    xcorr.accumulate_gated(plans, x, g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        xcorr.accumulate_gated(plans, x, g)
    torch.cuda.synchronize()
    ms_gated = (time.perf_counter() - t0) * 1e3 / reps
    p = plans[0]
    out = p.new_output()
    nr = (w.n_inputs + 63) // 64
    sel = [1 if k % 3 == 0 else 0 for k in range(nr * (nr + 1) // 2)]
    p.dump_tiles(out, sel, reset=True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(p.stream)
    for _ in range(reps):
        p.dump_tiles(out, sel, reset=True)
    e1.record(p.stream)
    torch.cuda.synchronize()
    ms_tiles = e0.elapsed_time(e1) / reps
    frac = sum(sel) / len(sel)
    for q in plans:
        q.close()
    del out
    torch.cuda.empty_cache()
    return {"gated": {"gates": 2, "period": period, "on_fraction": on, "ms": round(ms_gated, 3),
                      "tcmac_s": round(w.cmac / ms_gated / 1e9, 1),
                      "note": "host wall clock per call (the call waits for its stream once)"},
            "tile_dump": {"tiles_selected": sum(sel), "tiles": len(sel), "ms": round(ms_tiles, 4),
                          "gbs": round(3 * frac * w.output_bytes / ms_tiles / 1e6, 1)}}


def configs_leg(torch, xcorr, steps=10, warmup=3):
    """The other array sizes of the workload list, one window each as the
    headline times it (int8 path, int32 output, fused accumulate + dump):
    PAPER-like (128 inputs, 1024 channels, 2048 samples, 4-bit: bound by
    HBM, so its fraction of the 8 TB/s roof is the figure of merit) and
    large-N (2048 inputs, 256 channels, 8192 samples, 8-bit: bound by the
    matrix cores).  Also the plain fp32 kernel on the PAPER-like window."""
    from paper_1401_8288_amd import synth
    dev = torch.device("cuda:0")
    res = {}
    for name in ("paper", "large_n"):
        w = synth.WORKLOADS[name]
        x = synth.generate(w, device=dev)
        torch.cuda.synchronize()
        ms, out, info = time_path(torch, xcorr, x, w, "i8", steps, warmup, flags=xcorr.FLAG_OUT_I32)
        del out
        ops = 8 * w.cmac
        nbytes = w.input_bytes + w.output_bytes // 2
        r = {"workload": "%s: %d inputs, %d channels, %d samples/integration, %s"
                         % (name, w.n_inputs, w.n_channels, w.n_time, w.fmt),
             "ms_per_step": round(ms, 4), "tcmac_s": round(w.cmac / ms / 1e9, 2),
             "pct_int8_peak": round(100 * ops / ms / 1e9 / PEAK_INT8_TOPS, 2),
             "algorithmic_bytes": nbytes, "hbm_gbs": round(nbytes / ms / 1e6, 1),
             "pct_hbm_peak": round(100 * nbytes / ms / 1e6 / PEAK_HBM_GBS, 2),
             "bound": "hbm" if name == "paper" else "mfma", "work_items": info.work_items}
        if name == "paper":
            fms, fout, _ = time_path(torch, xcorr, x, w, "f32", 3, 1)
            del fout
            r["f32_ms_per_step"] = round(fms, 4)
            r["speedup_int8_vs_fp32"] = round(fms / ms, 2)
        log("%s: %.4f ms/window, %.1f TCMAC/s, %.1f%% of int8 peak, %.1f%% of HBM peak"
            % (name, ms, r["tcmac_s"], r["pct_int8_peak"], r["pct_hbm_peak"]))
        res[name] = r
        del x
        torch.cuda.empty_cache()
    return res


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, budget_s=12.0):
    """The oracle on a bounded sample of the same workload (host cores)."""
    import oracle
    from paper_1401_8288_amd import synth
    threads = oracle.threads()
    sample = synth.scaled(w, n_channels=threads)
    x = synth.generate(sample, device="cpu").numpy()
    t0 = time.perf_counter()
    oracle.correlate(x, w.fmt)
    t1 = time.perf_counter() - t0
    reps = max(1, min(64, int(budget_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.correlate(x, w.fmt)
    dt = time.perf_counter() - t0
    cmac = sample.cmac * reps
    return {"value": round(cmac / dt / 1e12, 6), "unit": "TCMAC/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(), "compiler": oracle.compiler(),
            "sample": "%d passes over %d channels x %d inputs x %d samples (%.3g CMAC, %.1f s)"
                      % (reps, sample.n_channels, w.n_inputs, w.n_time, cmac, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--no-compare", action="store_true", help="skip the fp16 / fp32 kernels")
    ap.add_argument("--no-corner-turn", action="store_true", help="skip the corner-turn leg")
    ap.add_argument("--no-fstage", action="store_true", help="skip the F-stage leg")
    ap.add_argument("--no-variants", action="store_true", help="skip the gating / tile-dump leg")
    ap.add_argument("--no-configs", action="store_true", help="skip the PAPER-like and large-N windows")
    ap.add_argument("--no-pcie", action="store_true", help="skip the host-transfer (PCIe) leg")
    ap.add_argument("--workload", default="lwa",
                    help="synthetic workload of the timed window (default lwa, the headline; others for profiling)")
    ap.add_argument("--tile", type=int, default=0,
                    help="int8 tile variant of the timed plans (XCORR_TILE_*; 0 = the library's default)")
    ap.add_argument("--serving-seconds", type=float, default=2.0,
                    help="length of the batched-streaming leg (0 skips it)")
    ap.add_argument("--serving-inflight", type=int, default=1, help="launches the server queues at once")
    ap.add_argument("--serving-speedups", default="10,20,30,40,60,80,120",
                    help="arrival rates of the streaming leg, multiples of real time (comma separated)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run the library copy kernel once (for counter calibration)")
    ap.add_argument("--pmc-summary", metavar="DIR",
                    help="print per-kernel averages of rocprofv3 counter CSVs and exit")
    ap.add_argument("--trace-summary", metavar="DIR",
                    help="print per-kernel durations of rocprofv3 kernel-trace CSVs and exit "
                         "(with --trace-skip / --trace-take / --trace-match)")
    ap.add_argument("--trace-skip", type=int, default=0, help="dispatches of each kernel left out first")
    ap.add_argument("--trace-take", type=int, default=0, help="dispatches averaged after those (0: all)")
    ap.add_argument("--trace-match", default="", help="only kernels whose name contains this")
    ap.add_argument("--many-small-only", action="store_true",
                    help="run only the many-small-arrays leg (for profiling its launches); prints its JSON")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary)
        return
    if args.trace_summary:
        trace_summary(args.trace_summary, args.trace_skip, args.trace_take, args.trace_match)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the X-stage shards by channel with no exchange, "
              "so there is no multi-GPU run here (got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1401_8288_amd import synth, xcorr

    if args.many_small_only:
        # 3 + 20 batched steps, then 3 + 20 steps of one launch per plan,
        # then the server at each speed for --serving-seconds (0: none)
        sp = [40.0, 200.0, 400.0, 800.0] if args.serving_seconds > 0 else []
        print(json.dumps(many_small_leg(torch, xcorr, args.serving_seconds, sp, inflight=args.serving_inflight)))
        return

    dev = torch.device("cuda:0")
    w = synth.WORKLOADS[args.workload]
    log("generating", w.name, w.n_inputs, "inputs x", w.n_channels, "channels x", w.n_time, "samples")
    x = synth.generate(w, device=dev)
    torch.cuda.synchronize()

    # The headline plan writes int32 (re, im) pairs: the same exact integers
    # as int64 for any window up to the fold bound (65535 samples; this one
    # has 4096), in the 8 bytes per baseline a complex float takes.  The
    # int64-output plan is timed right after it for comparison.
    log("int8 MFMA path, int32 output: %d warmup + %d timed windows" % (args.warmup, args.steps))
    steps_ms = []
    clock = {}
    ms, out, info = time_path(torch, xcorr, x, w, "i8", args.steps, args.warmup, flags=xcorr.FLAG_OUT_I32,
                              per_step=steps_ms, clock=clock, tile=args.tile)
    cmac = w.cmac
    tcmac = cmac / (ms * 1e-3) / 1e12
    tops = 8 * cmac / (ms * 1e-3) / 1e12
    out_bytes_i32 = w.output_bytes // 2
    hbm_bytes = w.input_bytes + out_bytes_i32
    log("int8, int32 out: %.3f ms/window, %.1f TCMAC/s, %.1f%% of int8 peak" % (ms, tcmac, 100 * tops / PEAK_INT8_TOPS))
    # the exact result, kept as float32 (exact below 2^24) to measure the
    # fp paths' error over every entry of the window
    exact = out.to(torch.float32) if (not args.no_compare and int(out.abs().max()) < 2 ** 24) else None
    del out
    torch.cuda.empty_cache()
    log("int8 MFMA path, int64 output: %d warmup + %d timed windows" % (args.warmup, args.steps))
    ms64, out64, _ = time_path(torch, xcorr, x, w, "i8", args.steps, args.warmup, tile=args.tile)
    del out64
    tops64 = 8 * cmac / (ms64 * 1e-3) / 1e12
    log("int8, int64 out: %.3f ms/window, %.1f%% of int8 peak" % (ms64, 100 * tops64 / PEAK_INT8_TOPS))
    acc_steps = max(16, 65536 // w.n_time)
    # the int32 accumulator's bound (4-bit: 2 * 8 * 8 per sample, 8-bit: 2 * 128 * 128)
    acc_bound = 16777215 if w.fmt == "ci4" else 65535
    acc_folds = acc_steps // max(1, acc_bound // w.n_time)
    acc_ms_steps = []
    ms_acc = time_accumulate(torch, xcorr, x, w, acc_steps, 1, per_step=acc_ms_steps)
    log("int8, accumulate only (int64 accumulator): %.3f ms/window" % ms_acc)

    result = {
        "metric": METRIC, "value": round(tcmac, 3), "unit": "TCMAC/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int8", "data": "synthetic (seeded, generated on device)",
        "config": {"workload": ("lwa: 256 antennas x 2 pol = 512 inputs, 4096 channels, "
                                "4096 samples/integration, 4+4-bit complex") if w.name == "lwa" else
                               "%s: %d inputs, %d channels, %d samples/integration, %s"
                               % (w.name, w.n_inputs, w.n_channels, w.n_time, w.fmt),
                   "n_inputs": w.n_inputs, "n_channels": w.n_channels, "n_time": w.n_time,
                   "format": w.fmt,
                   "path": "int8 MFMA, int32 partials, int32 (re, im) output, bit-exact (window <= 65535 samples)",
                   "entry_point": "xcorr_accumulate_dump(reset=1), plan flag XCORR_FLAG_OUT_I32",
                   "work_items": info.work_items},
        "step_ms": {"p10": round(percentile(steps_ms, 10), 4), "p50": round(percentile(steps_ms, 50), 4),
                    "p90": round(percentile(steps_ms, 90), 4)},
        "int64_output": {"ms_per_step": round(ms64, 4), "value": round(cmac / (ms64 * 1e-3) / 1e12, 3),
                         "pct_int8_peak": round(100 * tops64 / PEAK_INT8_TOPS, 2)},
        "accumulate_only": {"ms_per_step": round(ms_acc, 4),
                            "pct_int8_peak": round(100 * 8 * cmac / (ms_acc * 1e-3) / 1e12 / PEAK_INT8_TOPS, 2),
                            "steps": acc_steps,
                            "folds_in_timed_steps": acc_folds,
                            "step_ms": {"p10": round(percentile(acc_ms_steps, 10), 4),
                                        "p50": round(percentile(acc_ms_steps, 50), 4),
                                        "p90": round(percentile(acc_ms_steps, 90), 4)},
                            "note": "xcorr_accumulate of an int64 plan: int32 accumulator read and written per "
                                    "window, folded into the int64 one every %d samples" % acc_bound},
        "roofline": {"bound": "mfma",
                     "kernel": "xcorr_i8_persist_kernel<V_%s_DMA4, int32 out>" % w.fmt.upper(),
                     "achieved": round(tops, 2), "peak": PEAK_INT8_TOPS, "unit": "TOP/s",
                     "frac": round(tops / PEAK_INT8_TOPS, 4), "traffic": None,
                     "algorithmic_ops_per_launch": 8 * cmac,
                     "algorithmic_bytes_per_launch": hbm_bytes,
                     "hbm_gbs_algorithmic": round(hbm_bytes / (ms * 1e-3) / 1e9, 1)},
        "pct_int8_peak": round(100 * tops / PEAK_INT8_TOPS, 2),
    }
    if "mhz" in clock:
        # the int8 peak scales with the shader clock (8192 ops per CU per cycle)
        peak_now = PEAK_INT8_TOPS * clock["mhz"] / PEAK_CLOCK_MHZ
        result["roofline"]["measured_clock_mhz"] = round(clock["mhz"], 1)
        result["roofline"]["peak_at_measured_clock"] = round(peak_now, 1)
        result["roofline"]["frac_at_measured_clock"] = round(tops / peak_now, 4)
        log("shader clock during the timed windows: %.0f MHz; %.1f%% of the int8 peak at that clock"
            % (clock["mhz"], 100 * tops / peak_now))
    traffic, how = read_traffic() if w.name == "lwa" else (None, "counters recorded for the lwa workload only")
    result["roofline"]["traffic"] = traffic
    result["roofline"]["traffic_source"] = how
    torch.cuda.empty_cache()
    if not args.no_pcie:
        log("host transfers of the same window (pinned memory)")
        pc = pcie_leg(torch, x, out_bytes_i32)
        t = pc["h2d_ms"] + ms + pc["d2h_ms"]
        pc["pcie_inclusive_ms"] = round(t, 3)
        pc["pcie_inclusive_tcmac_s"] = round(cmac / (t * 1e-3) / 1e12, 2)
        pc["note"] = "input in from the host, the window, the int32 result out, one after another"
        result["pcie"] = pc
        log("pcie:", pc)
        torch.cuda.empty_cache()
    if args.copy_calibration:
        copy_calibration(torch, xcorr, x, w)

    if not args.no_compare:
        comp = {}
        for path, steps, peak, unit in (("f16", max(2, args.steps // 4), PEAK_FP16_TFLOPS, "TFLOP/s"),
                                        ("f32", 2, PEAK_FP32_TFLOPS, "TFLOP/s")):
            log("%s path: 1 warmup + %d timed windows" % (path, steps))
            pms, pout, _ = time_path(torch, xcorr, x, w, path, steps, 1)
            err = float((pout - exact).abs().max()) if exact is not None else None
            del pout
            ptc = cmac / (pms * 1e-3) / 1e12
            comp[path] = {"ms_per_step": round(pms, 3), "tcmac_s": round(ptc, 3),
                          "achieved": round(8 * cmac / (pms * 1e-3) / 1e12, 2), "peak": peak,
                          "unit": unit, "frac": round(8 * cmac / (pms * 1e-3) / 1e12 / peak, 4),
                          "max_abs_err_vs_exact": err}
            log("%s: %.3f ms/window, %.2f TCMAC/s" % (path, pms, ptc))
        comp["speedup_int8_vs_fp32"] = round(comp["f32"]["ms_per_step"] / ms, 2)
        comp["speedup_int8_vs_fp16"] = round(comp["f16"]["ms_per_step"] / ms, 2)
        result["compare"] = comp
        exact = None
        torch.cuda.empty_cache()

    if not args.no_configs and w.name == "lwa":
        log("PAPER-like and large-N windows")
        result["configs"] = configs_leg(torch, xcorr)

    if not args.no_corner_turn and w.name == "lwa":
        log("corner turn at the same size")
        result["corner_turn"] = corner_turn_leg(torch, xcorr, w)
        log("corner turn:", result["corner_turn"])

    if not args.no_variants and w.name == "lwa":
        log("pulsar gating and tile dumps at the same size")
        result["accumulate_variants"] = variants_leg(torch, xcorr, x, w)
        log("accumulate variants:", result["accumulate_variants"])

    if not args.no_fstage and w.name == "lwa":
        log("F-stage making the same workload")
        result["fstage"] = fstage_leg(torch, xcorr, w)
        log("F-stage:", result["fstage"])

    if args.serving_seconds > 0:
        sp = [float(v) for v in args.serving_speedups.split(",") if v]
        log("batched streaming leg: %.1f s at each of %s x real time" % (args.serving_seconds, sp))
        result["serving"] = serving_leg(torch, xcorr, args.serving_seconds, sp, inflight=args.serving_inflight)
        log("serving:", result["serving"])
        torch.cuda.empty_cache()
        log("many small arrays")
        result["many_small_arrays"] = many_small_leg(torch, xcorr, args.serving_seconds, [40.0, 200.0, 400.0, 800.0],
                                                     inflight=args.serving_inflight)
        log("many small arrays:", result["many_small_arrays"])
        torch.cuda.empty_cache()

    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample")
        result["cpu_baseline"] = cpu_baseline(w)
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
