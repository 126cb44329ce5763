#!/usr/bin/env python3
"""Benchmark of the correlator hot path on one MI355X.

One step = one frame of the pathfinder per-GPU share (N=256 inputs, 64
channels, 16384 samples, 1% of 256-sample blocks lost) accumulated into
the device-resident integration (xe_accumulate: load, decode, mask, int8
MFMA over the upper triangle, add, count) and the integration normalised
(xe_normalize).  Inputs are synthetic and already in HBM when the timed
region starts.

Prints ONE JSON line.  Fields beyond the common ones:
  roofline      the correlation call (correlation kernel + the merge of
                its time chunks) against the int8 MFMA peak: the
                algorithmic ops per call (8 per channel, upper-triangle
                pair and sample) over its average duration, timed with HIP
                events on the stream it runs on; traffic = HBM bytes per
                call from the committed counter runs, when they were
                taken on the current kernel source
  batched       128 uneven single-channel instances (N 64..1024, 1024 to
                65536 samples) in one persistent launch replayed from a
                captured graph, against the same instances as plain
                per-instance launches; results compared bit for bit
  flags         per-input flags on the same frame: the flag Gram kernel
                (bursty 0.1% flags, and 50% as a stress case) against HBM,
                the zeroing and per-baseline normalisation kernels, and the
                flagged step against the plain one
  assembly      the same frame assembled on the GPU from 32768 F-engine
                packets (1% dropped, 0.5% duplicated, reordered) against HBM
  shift         per-input time shifting of the same frame and its flags
                against HBM
  large_n       N=2048, 16 channels, 8192 samples accumulated, against the
                int8 MFMA peak
  pipeline      one frame through the whole GPU data flow: packets ->
                assembly -> zeroing of flagged points -> correlation -> flag
                intersections -> per-baseline normalisation
  serving       8 streams of 4096-sample frames offered with Poisson
                arrivals at 51.2 Gb/s in total from pinned host memory:
                p50/p99 frame latency (arrival to accumulated); plus the
                serving loop's sustained rate on device-resident frames
                against one plain launch per frame, and its saturated rate
                fed from pinned host memory
  cpu_baseline  the oracle (plain C loops) on a bounded sample of the same
                frame, on this host's cores
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MFMA_INT8_PEAK_TOPS = 5000.0   # MI355X dense int8, tera-ops/s
HBM_PEAK_GBPS = 8000.0
PMC_FILE = os.path.join(ROOT, "profiles", "corr_pathfinder_n256_f64_t16384_pmc.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1503_06189_amd", "csrc", f)
                  for f in ("xcorr_kernels.hpp", "plan.hpp", "xengine.hip")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _device_info(torch) -> dict:
    """Name, architecture, compute units and clock of the GPU measured."""
    p = torch.cuda.get_device_properties(0)
    out = {"name": p.name, "arch": getattr(p, "gcnArchName", None),
           "compute_units": p.multi_processor_count,
           "hbm_bytes": int(p.total_memory)}
    clock = getattr(p, "clock_rate", None)
    if clock:
        out["clock_khz"] = int(clock)
    return out


def _pmc():
    """The committed rocprofv3 counter summary of the correlation call, if
    it was taken on the current kernel source; else None."""
    try:
        with open(PMC_FILE) as f:
            pmc = json.load(f)
    except (OSError, ValueError):
        return None
    if pmc.get("kernel_source_hash") != kernel_source_hash():
        return None
    return pmc


def measured_traffic():
    """HBM bytes per launch from the committed counter runs, or None."""
    pmc = _pmc()
    return None if pmc is None else pmc.get("hbm_bytes_per_launch")


def measured_execution():
    """Executed matrix-core work of corr_kernel from the committed SQ
    counter runs, or None: executed int8 ops against the algorithmic ones,
    and the fraction of the kernel's cycles the SIMDs' matrix cores were
    busy (SQ_VALU_MFMA_BUSY_CYCLES per SIMD over GRBM_GUI_ACTIVE per XCD),
    mean over the profiled dispatches and for the fastest one."""
    pmc = _pmc()
    sq = None if pmc is None else pmc.get("sq")
    if not sq:
        return None
    return {
        "executed_int8_ops": sq["executed_int8_ops"],
        "algorithmic_int8_ops": sq["algorithmic_int8_ops"],
        "mfma_busy_frac_mean": sq["mfma_busy_frac_mean"],
        "mfma_busy_frac_best": sq["mfma_busy_frac_best"],
        "source": os.path.basename(PMC_FILE),
    }


def _single_thread_oracle(fr, n_ch: int):
    """The oracle on n_ch channels of the frame in a child process limited
    to one OpenMP thread; seconds of the median of 3 runs."""
    import subprocess
    import tempfile
    import numpy as np
    with tempfile.TemporaryDirectory() as d:
        pk = os.path.join(d, "packed.npy")
        mk = os.path.join(d, "mask.npy")
        np.save(pk, np.ascontiguousarray(fr.packed[:, :n_ch, :]))
        np.save(mk, np.ascontiguousarray(fr.mask[:n_ch]))
        code = ("import sys, time, numpy as np; sys.path.insert(0, %r); import oracle; "
                "orc = oracle.load(); p = np.load(%r); m = np.load(%r); ts = []\n"
                "for _ in range(3):\n"
                "    t0 = time.perf_counter(); orc.correlate(p, m, %d); "
                "ts.append(time.perf_counter() - t0)\n"
                "print(sorted(ts)[1])" % (ROOT, pk, mk, fr.B))
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                           text=True, timeout=600)
        if r.returncode != 0:
            return None
        return float(r.stdout.strip().splitlines()[-1])


def cpu_baseline(fr, target_s: float):
    """Time the oracle on a prefix of channels of the frame: all host cores
    (median of 3 runs), and one core on a smaller prefix."""
    import numpy as np
    import oracle
    from paper_1503_06189_amd import metrics
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    os.environ["OMP_NUM_THREADS"] = str(threads)
    orc = oracle.load()
    # calibrate on one channel with a short time prefix, then size the sample
    t_pre = min(fr.T, 2048)
    sub = np.ascontiguousarray(fr.packed[:t_pre, :1, :])
    t0 = time.perf_counter()
    orc.correlate(sub, None, fr.B)
    per_sample_ch = (time.perf_counter() - t0) / t_pre
    # three runs share the time budget
    n_ch = max(1, min(fr.F, int(target_s / 3 / max(per_sample_ch * fr.T, 1e-9))))
    sub = np.ascontiguousarray(fr.packed[:, :n_ch, :])
    mask = np.ascontiguousarray(fr.mask[:n_ch]) if fr.mask is not None else None
    runs = []
    for _ in range(3):
        t0 = time.perf_counter()
        orc.correlate(sub, mask, fr.B)
        runs.append(time.perf_counter() - t0)
    dt = sorted(runs)[1]
    # one core: about 10 s of work at the calibrated multi-core rate
    n1 = max(1, min(fr.F, int(10.0 / 3 / max(per_sample_ch * fr.T * threads, 1e-9))))
    dt1 = _single_thread_oracle(fr, n1)
    return {
        "value": round(metrics.input_gbps(fr.N, n_ch, fr.T, dt), 6),
        "unit": "Gb/s",
        "cores": threads,
        "cpu": _cpu_model(),
        "kind": "oracle",
        "sample": f"{n_ch} of {fr.F} channels, full {fr.T} samples, N={fr.N}, median of 3 "
                  f"runs ({dt:.1f} s each)",
        "runs_s": [round(x, 3) for x in runs],
        "single_core": None if dt1 is None else {
            "value": round(metrics.input_gbps(fr.N, n1, fr.T, dt1), 6), "unit": "Gb/s",
            "cores": 1,
            "sample": f"{n1} of {fr.F} channels, full {fr.T} samples, median of 3 runs "
                      f"({dt1:.1f} s each)"},
        "next_paths": cpu_baseline_next(orc, fr),
    }


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_next(orc, fr):
    """The oracle's other paths on the same frame, one host thread each
    (their loops are not parallelised): flag counters and intersections
    (bursty 0.1% flags, all 64 channels), frame assembly from the frame's
    packets with faults, and the time shift of the first 8 channels; each
    as microseconds per pathfinder frame, to set beside the GPU legs."""
    import numpy as np
    from paper_1503_06189_amd import synth
    rng = np.random.default_rng(2024)
    flags = synth.fengine_flags(rng, fr.T, fr.F, fr.N, 1e-3, mean_run=32.0)
    t0 = time.perf_counter()
    orc.flag_counters(flags, fr.mask, fr.N, fr.B)
    flag_s = time.perf_counter() - t0
    pk = synth.network_faults(rng, synth.packetize(fr.packed, flags), p_drop=0.01,
                              p_dup=0.005, window=64)
    t0 = time.perf_counter()
    orc.assemble(pk, fr.N, fr.F // 8, 0, 0, fr.T)
    asm_s = time.perf_counter() - t0
    n_ch = 8
    d = rng.integers(-8, 9, fr.N).astype(np.int32)
    t0 = time.perf_counter()
    orc.time_shift(np.ascontiguousarray(fr.packed[:, :n_ch]),
                   np.ascontiguousarray(flags[:n_ch]), d)
    shift_s = (time.perf_counter() - t0) * fr.F / n_ch
    return {
        "flag_counters_us_per_frame": round(flag_s * 1e6, 1),
        "assemble_us_per_frame": round(asm_s * 1e6, 1),
        "time_shift_us_per_frame": round(shift_s * 1e6, 1),
        "sample": f"{fr.name}; time shift timed on {n_ch} of {fr.F} channels and scaled",
    }


def _events(torch, n):
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def batched_leg(torch, reps: int):
    """Uneven instances: one graph-replayed persistent launch vs plain
    per-instance launches on the same stream."""
    from paper_1503_06189_amd import synth, tune, xengine
    dev = torch.device("cuda:0")
    h = xengine.default_handle(0)
    frs = synth.batched()
    items = []
    for f in frs:
        p = torch.from_numpy(f.packed).to(dev)
        m = torch.from_numpy(f.mask).to(dev)
        v, c = xengine.new_accumulators(f.N, f.F, dev)
        items.append((p, m, f.B, v, c))
    ops = sum(8 * f.N * (f.N + 1) // 2 * f.F * f.T for f in frs)
    bits = sum(8 * f.N * f.F * f.T for f in frs)
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = _events(torch, 2)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def plain():
        for it in items:
            xengine.accumulate(*it, handle=h, stream=stream)

    choice = tune.tune(items, handle=h)
    entry = tune.lookup(items) or {}
    plan = xengine.BatchPlan(items, chunk_steps=choice.chunk_steps, handle=h,
                             geometry=choice.geometry)
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            plan.run()
    stream.wait_stream(side)
    torch.cuda.synchronize()
    ms_plain = timed(plain)
    ms_graph = timed(g.replay)
    # exactness: one plain pass and one batched pass from zero
    for _, _, _, v, c in items:
        v.zero_()
        c.zero_()
        xengine.reset_integration(v)
    plain()
    torch.cuda.synchronize()
    want = [(v.clone(), c.clone()) for _, _, _, v, c in items]
    for _, _, _, v, c in items:
        v.zero_()
        c.zero_()
        xengine.reset_integration(v)
    g.replay()
    torch.cuda.synchronize()
    exact = all(torch.equal(v, w) and torch.equal(c, n)
                for (_, _, _, v, c), (w, n) in zip(items, want))
    del g
    plan.release()
    return {
        "workload": f"{len(frs)} uneven single-channel instances, N 64..1024, T 1024..65536",
        "plain_ms": round(ms_plain, 4),
        "batched_ms": round(ms_graph, 4),
        "speedup": round(ms_plain / ms_graph, 2),
        "gbps": round(bits / (ms_graph / 1e3) / 1e9, 1),
        "plain_gbps": round(bits / (ms_plain / 1e3) / 1e9, 1),
        "tops": round(ops / (ms_graph / 1e3) / 1e12, 1),
        "mfma_frac": round(ops / (ms_graph / 1e3) / 1e12 / MFMA_INT8_PEAK_TOPS, 4),
        "chunk_steps": choice.chunk_steps,
        "geometry": choice.geometry,
        # the tuner's fastest plan per tile geometry (graph-free plan runs)
        "tuned_best_ms_by_geometry": {g: round(v, 4)
                                      for g, v in tune.best_by_geometry(entry).items()},
        "tuned_plans": len(entry.get("timings_ms", {})),
        "exact_vs_plain": bool(exact),
    }


def flags_leg(torch, reps: int):
    """Per-input flags on the pathfinder frame: the flag Gram kernel
    (xe_flag_accumulate) with bursty F-engine flags at 0.1% of points (runs
    of 32 samples) and, as a stress case, independent flags at 50%; the
    zeroing and per-baseline normalisation kernels; and the whole flagged
    step against the unflagged one.  The Gram kernel's HBM roofline counts
    the flag words read once plus the counts read and written once."""
    import numpy as np
    from paper_1503_06189_amd import synth, xengine
    dev = torch.device("cuda:0")
    h = xengine.default_handle(0)
    stream = torch.cuda.current_stream()
    fr = synth.pathfinder()
    N, F, T, B = fr.N, fr.F, fr.T, fr.B
    rng = np.random.default_rng(2024)
    bursty = synth.fengine_flags(rng, T, F, N, 1e-3, mean_run=32.0)
    dense = synth.random_flags(rng, T, F, N, 0.5, garbage_padding=False)

    def to_dev(a):
        return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(dev)

    fl_b, fl_d = to_dev(bursty), to_dev(dense)
    packed = torch.from_numpy(fr.packed).to(dev)
    mask = torch.from_numpy(fr.mask).to(dev)
    vis, cnt = xengine.new_accumulators(N, F, dev)
    dcount = xengine.new_flag_counts(N, F, dev)
    out = torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.float32, device=dev)

    def timed(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = _events(torch, 2)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    gram_b = timed(lambda: xengine.flag_accumulate(fl_b, mask, B, N, dcount, handle=h,
                                                   stream=stream))
    gram_d = timed(lambda: xengine.flag_accumulate(fl_d, mask, B, N, dcount, handle=h,
                                                   stream=stream))
    apply_b = timed(lambda: xengine.apply_flags(packed, fl_b, handle=h, stream=stream))
    norm = timed(lambda: xengine.normalize_flagged(vis, cnt, dcount, out=out, handle=h,
                                                   stream=stream))

    def flagged_step():
        xengine.apply_flags(packed, fl_b, handle=h, stream=stream)
        xengine.accumulate(packed, mask, B, vis, cnt, handle=h, stream=stream)
        xengine.flag_accumulate(fl_b, mask, B, N, dcount, handle=h, stream=stream)
        xengine.normalize_flagged(vis, cnt, dcount, out=out, handle=h, stream=stream)

    def plain_step():
        xengine.accumulate(packed, mask, B, vis, cnt, handle=h, stream=stream)
        xengine.normalize(vis, cnt, out, handle=h, stream=stream)

    step_f = timed(flagged_step)
    step_p = timed(plain_step)
    flag_bytes = F * T * synth.flag_words(N) * 4
    d_bytes = 2 * F * (N * (N + 1) // 2) * 4
    gbps = (flag_bytes + d_bytes) / (gram_b / 1e3) / 1e9
    return {
        "workload": f"{fr.name}, bursty flags 0.1% of points (runs of 32 samples)",
        "flag_gram_us": round(gram_b * 1e3, 2),
        "flag_gram_dense50_us": round(gram_d * 1e3, 2),
        "apply_flags_us": round(apply_b * 1e3, 2),
        "normalize_flagged_us": round(norm * 1e3, 2),
        "flagged_step_ms": round(step_f, 4),
        "plain_step_ms": round(step_p, 4),
        "flag_gram_roofline": {"bound": "hbm", "achieved": round(gbps, 1),
                               "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                               "frac": round(gbps / HBM_PEAK_GBPS, 4),
                               "alg_bytes": flag_bytes + d_bytes},
    }


def assembly_leg(torch, reps: int):
    """Frame assembly from F-engine packets (xe_assemble_frame) for the
    pathfinder share: 8 links x 8 bands, 16384 samples, 32768 packets of
    9232 B with 1% dropped, 0.5% duplicated and reordering, the packets
    already in device memory.  HBM roofline: packets read once, frame, flags
    and mask written once."""
    import numpy as np
    from paper_1503_06189_amd import synth, xengine
    dev = torch.device("cuda:0")
    h = xengine.default_handle(0)
    stream = torch.cuda.current_stream()
    fr = synth.pathfinder(p_loss=0.0)
    rng = np.random.default_rng(77)
    flags = synth.fengine_flags(rng, fr.T, fr.F, fr.N, 1e-3)
    pk = synth.packetize(fr.packed, flags, stream_base=0, seq0=0)
    pk = synth.network_faults(rng, pk, p_drop=0.01, p_dup=0.005, window=64)
    dpk = torch.from_numpy(pk).to(dev)
    S = fr.F // 8
    out = xengine.assemble_frame(dpk, fr.N, S, 0, 0, fr.T, handle=h, stream=stream)
    torch.cuda.synchronize()
    for _ in range(3):
        xengine.assemble_frame(dpk, fr.N, S, 0, 0, fr.T, *out, handle=h, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = _events(torch, 2)
    e0.record(stream)
    for _ in range(reps):
        xengine.assemble_frame(dpk, fr.N, S, 0, 0, fr.T, *out, handle=h, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    # the copy of the receive ring from pinned host memory, for context
    host = torch.from_numpy(pk).pin_memory()
    dpk.copy_(host, non_blocking=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(3):
        dpk.copy_(host, non_blocking=True)
    e1.record(stream)
    torch.cuda.synchronize()
    h2d_ms = e0.elapsed_time(e1) / 3
    st = out[3].cpu().tolist()
    W = synth.flag_words(fr.N)
    alg = pk.nbytes + fr.T * fr.F * fr.N + fr.F * fr.T * W * 4 + fr.F * fr.T // 4
    gbps = alg / (ms / 1e3) / 1e9
    return {
        "workload": f"{fr.name} from {len(pk)} packets of {pk.shape[1]} B, "
                    "1% dropped, 0.5% duplicated, reordered",
        "assemble_us": round(ms * 1e3, 2),
        "packets_per_s": round(len(pk) / (ms / 1e3), 0),
        "placed": st[4], "lost": st[5], "duplicates": st[0] - st[4],
        "h2d_packets_us": round(h2d_ms * 1e3, 1),
        "h2d_gbps": round(pk.nbytes / (h2d_ms / 1e3) / 1e9, 1),
        "roofline": {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(gbps / HBM_PEAK_GBPS, 4),
                     "alg_bytes": int(alg)},
    }


def shift_leg(torch, reps: int):
    """Per-input time shifting (xe_time_shift) of the pathfinder frame with
    delays in [-8, 8] samples and its bursty flags moved along: frame and
    flags read and written once against HBM."""
    import numpy as np
    from paper_1503_06189_amd import synth, xengine
    dev = torch.device("cuda:0")
    h = xengine.default_handle(0)
    stream = torch.cuda.current_stream()
    fr = synth.pathfinder()
    rng = np.random.default_rng(31)
    flags = synth.fengine_flags(rng, fr.T, fr.F, fr.N, 1e-3)
    delays = torch.from_numpy(rng.integers(-8, 9, fr.N).astype(np.int32)).to(dev)
    packed = torch.from_numpy(fr.packed).to(dev)
    fl = torch.from_numpy(flags.view(np.int32)).to(dev)
    out, fo = xengine.time_shift(packed, delays, fl, handle=h, stream=stream)
    for _ in range(3):
        xengine.time_shift(packed, delays, fl, out, fo, handle=h, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = _events(torch, 2)
    e0.record(stream)
    for _ in range(reps):
        xengine.time_shift(packed, delays, fl, out, fo, handle=h, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    alg = 2 * (packed.numel() + fl.numel() * 4)
    gbps = alg / (ms / 1e3) / 1e9
    return {
        "workload": f"{fr.name}, delays in [-8, 8] samples, bursty flags 0.1%",
        "time_shift_us": round(ms * 1e3, 2),
        "roofline": {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(gbps / HBM_PEAK_GBPS, 4),
                     "alg_bytes": int(alg)},
    }


def pipeline_leg(torch, reps: int):
    """One frame through the whole data flow on the GPU: F-engine packets
    already in HBM (1% dropped, 0.5% duplicated, reordered, 0.1% bursty
    per-input flags) -> frame assembly -> zeroing of flagged points ->
    correlation into the integration -> flag intersections -> per-baseline
    normalisation.  The integrated counts are checked against a second
    integration of the same frame (determinism)."""
    import numpy as np
    from paper_1503_06189_amd import synth, xengine
    dev = torch.device("cuda:0")
    h = xengine.default_handle(0)
    stream = torch.cuda.current_stream()
    fr = synth.pathfinder(p_loss=0.0)
    N, F, T = fr.N, fr.F, fr.T
    rng = np.random.default_rng(55)
    flags = synth.fengine_flags(rng, T, F, N, 1e-3)
    pk = synth.network_faults(rng, synth.packetize(fr.packed, flags), p_drop=0.01,
                              p_dup=0.005, window=64)
    dpk = torch.from_numpy(pk).to(dev)
    S = F // 8
    packed, mask, fl, stats = xengine.assemble_frame(dpk, N, S, 0, 0, T, handle=h, stream=stream)
    vis, cnt = xengine.new_accumulators(N, F, dev)
    dcount = xengine.new_flag_counts(N, F, dev)
    out = torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.float32, device=dev)

    def frame():
        xengine.assemble_frame(dpk, N, S, 0, 0, T, packed, mask, fl, stats, handle=h,
                               stream=stream)
        xengine.apply_flags(packed, fl, handle=h, stream=stream)
        xengine.accumulate(packed, mask, 4, vis, cnt, handle=h, stream=stream)
        xengine.flag_accumulate(fl, mask, 4, N, dcount, handle=h, stream=stream)
        xengine.normalize_flagged(vis, cnt, dcount, out=out, handle=h, stream=stream)

    frame()
    torch.cuda.synchronize()
    one = (vis.clone(), cnt.clone(), dcount.clone())
    for _ in range(2):
        frame()
    torch.cuda.synchronize()
    e0, e1 = _events(torch, 2)
    e0.record(stream)
    for _ in range(reps):
        frame()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    k = 3 + reps
    exact = (torch.equal(vis, one[0] * k) and torch.equal(cnt, one[1] * k)
             and torch.equal(dcount, one[2] * k))
    return {
        "workload": f"{fr.name} from {len(pk)} packets: assemble, zero flagged points, "
                    "correlate, flag intersections, per-baseline normalise",
        "frame_ms": round(ms, 4),
        "gbps": round(8.0 * N * F * T / (ms / 1e3) / 1e9, 1),
        "integration_exact": bool(exact),
    }


def large_n_leg(torch, reps: int):
    """The large-N scaling point: N=2048, 16 channels, 8192 samples, 0.5%
    block loss, accumulated (xe_accumulate) against the int8 MFMA peak.
    Uniform random bytes of that shape stand in for the point-source recipe
    (the correlation's cost does not depend on the values)."""
    from paper_1503_06189_amd import metrics, synth, xengine
    dev = torch.device("cuda:0")
    h = xengine.default_handle(0)
    stream = torch.cuda.current_stream()
    fr = synth.random_bytes_frame(synth.SEEDS["large_n"], 2048, 16, 8192, 256, p_loss=0.005,
                                  fill="zero")
    packed = torch.from_numpy(fr.packed).to(dev)
    mask = torch.from_numpy(fr.mask).to(dev)
    vis, cnt = xengine.new_accumulators(fr.N, fr.F, dev)
    for _ in range(3):
        xengine.accumulate(packed, mask, fr.B, vis, cnt, handle=h, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = _events(torch, 2)
    e0.record(stream)
    for _ in range(reps):
        xengine.accumulate(packed, mask, fr.B, vis, cnt, handle=h, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    tops = metrics.int_ops(fr.N, fr.F, fr.T) / (ms / 1e3) / 1e12
    return {
        "workload": f"N={fr.N}, F={fr.F}, T={fr.T}, 0.5% block loss (uniform random bytes)",
        "accumulate_ms": round(ms, 4),
        "gbps": round(metrics.input_gbps(fr.N, fr.F, fr.T, ms / 1e3), 1),
        "tops": round(tops, 1),
        "mfma_frac": round(tops / MFMA_INT8_PEAK_TOPS, 4),
    }


def serving_leg(torch, seconds: float):
    """The streaming server at the configured load: 8 streams offered 51.2
    Gb/s together (Poisson arrivals given the count, so the realised rate is
    the offered one), three distinct frames per stream, copied in
    1024-sample slices into the pre-allocated frame pool and accumulated
    slice by slice; the same load with whole-frame copies; a sweep of
    offered rates; and the loop's own rate with frames already in HBM
    against one plain launch per frame."""
    from paper_1503_06189_amd import serve, synth
    specs = synth.streaming_streams()
    pool = serve._frame_pool(specs, 3, 256)

    def summary(r):
        st = r.stats
        out = {"p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
               "frames": st["frames"], "sustained_gbps": round(st["gbps"], 1),
               "mean_batch": round(st["mean_batch"], 2)}
        if st.get("offered_gbps") is not None:
            out["offered_gbps"] = round(st["offered_gbps"], 1)
            out["offered_realized_gbps"] = round(st["offered_realized_gbps"], 1)
        return out

    # a short run first: every kernel of the loop is loaded before timing
    serve.run_load(specs, speed=4.0, duration=0.25, pool=pool, distinct=3,
                   hbm_budget=2 << 30, slice_samples=1024)
    live = serve.run_load(specs, speed=1.0, duration=seconds, pool=pool, distinct=3,
                          hbm_budget=2 << 30, slice_samples=1024)
    whole = serve.run_load(specs, speed=1.0, duration=seconds, pool=pool, distinct=3,
                           hbm_budget=2 << 30)
    sweep = []
    for speed in (2.0, 4.0, 8.0):
        r = serve.run_load(specs, speed=speed, duration=max(1.0, seconds / 3), pool=pool,
                           distinct=3, hbm_budget=2 << 30, slice_samples=1024, seed=int(speed))
        sweep.append(summary(r))
    sat = serve.run_load(specs, frames_per_stream=12, speed=float("inf"), pool=pool,
                         device_resident=True, hbm_budget=1 << 36)
    plain = serve.run_plain(specs, pool, 12)
    host_sat = serve.run_load(specs, frames_per_stream=12, speed=float("inf"), pool=pool,
                              distinct=3, hbm_budget=8 << 30, slice_samples=1024)
    st = live.stats
    bd = {k: {kk: round(vv, 3) for kk, vv in v.items()}
          for k, v in st["latency_breakdown"].items()}
    n_int = sum(len(v) for v in live.server.results.values())
    return {
        "workload": "8 streams, N in {128,256,512}, F 16..64, 4096-sample frames, "
                    "Poisson arrivals, 51.2 Gb/s offered, Gilbert-Elliott loss, "
                    "3 distinct frames per stream",
        "p50_ms": round(st["p50_ms"], 3),
        "p99_ms": round(st["p99_ms"], 3),
        "p99_breakdown_ms": bd,
        "frames": st["frames"],
        "integrations_completed": n_int,
        "offered_gbps": round(st["offered_gbps"], 1),
        "offered_realized_gbps": round(st["offered_realized_gbps"], 1),
        "arrival_span_s": round(st["arrival_span_s"], 3),
        "sustained_gbps": round(st["gbps"], 1),   # served bits / wall (arrival span + drain)
        "mean_batch": round(st["mean_batch"], 2),
        "admission_waits": st["admission_waits"],
        "submit_late_p99_ms": round(st.get("submit_late_p99_ms", 0.0), 3),
        "clock_offset_ms": round(st["clock_offset_ms"], 3),
        "slice_samples": 1024,
        "hbm_budget_bytes": st["hbm_budget"],
        "hbm_peak_used_bytes": st["hbm_peak_used"],
        "frame_pool_bytes": live.server.pool.bytes,
        "whole_frames": summary(whole),
        "sweep": sweep,
        "device_resident_gbps": round(sat.stats["gbps"], 1),
        "device_resident_plain_gbps": round(plain["gbps"], 1),
        "host_fed_saturated_gbps": round(host_sat.stats["gbps"], 1),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # about 20 ms of warm-up: clocks settle before the timed region
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-flags", action="store_true")
    ap.add_argument("--no-assembly", action="store_true")
    ap.add_argument("--no-shift", action="store_true")
    ap.add_argument("--no-pipeline", action="store_true")
    ap.add_argument("--no-large-n", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=4.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed region, copy 256 MiB once (a kernel of known "
                         "traffic, to scale HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the correlator shards by "
              "channel with no communication, so run one process per GPU "
              "and add their rates.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1503_06189_amd import metrics, synth, xengine

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    xengine.lib()

    fr = synth.pathfinder()
    N, F, T, B = fr.N, fr.F, fr.T, fr.B
    packed = torch.from_numpy(fr.packed).to(dev)
    mask = torch.from_numpy(fr.mask).to(dev)
    vis, cnt = xengine.new_accumulators(N, F, dev)
    out = torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.float32, device=dev)
    h = xengine.default_handle(0)
    stream = torch.cuda.current_stream()

    def step(ev0=None, ev1=None):
        if ev0 is not None:
            ev0.record(stream)
        xengine.accumulate(packed, mask, B, vis, cnt, handle=h, stream=stream)
        if ev1 is not None:
            ev1.record(stream)
        xengine.normalize(vis, cnt, out, handle=h, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    vis.zero_()
    cnt.zero_()
    xengine.reset_integration(vis)
    torch.cuda.synchronize()

    k_ev = [tuple(_events(torch, 2)) for _ in range(args.steps)]
    s0, s1 = _events(torch, 2)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    s0.record(stream)
    for k in range(args.steps):
        step(*k_ev[k])
    s1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    total_ms = s0.elapsed_time(s1)
    kern_ms = sum(a.elapsed_time(b) for a, b in k_ev) / args.steps

    # the integration of K identical frames is K times one frame's sums
    valid0 = int((fr.mask[0] == 0).sum()) * B   # T is a multiple of B here
    assert int(cnt[0].item()) == args.steps * valid0
    ms_per_step = total_ms / args.steps
    value = metrics.input_gbps(N, F, T, ms_per_step / 1e3)
    ops = metrics.int_ops(N, F, T)
    achieved_tops = ops / (kern_ms / 1e3) / 1e12
    alg_bytes = metrics.input_bytes(N, F, T) + 2 * metrics.output_bytes(N, F)

    if args.copy_calibration:
        a = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    res = {
        "metric": "input Gb/s + int8 MFMA util at N=256x64ch; streaming p50/p99 frame latency",
        "value": round(value, 3),
        "unit": "Gb/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic (seeded Gaussian noise + sky tone, 4+4-bit, 1% block loss)",
        "config": {"workload": fr.name, "N": N, "F": F, "T": T, "B": B,
                   "loss": "bernoulli 0.01 per 256-sample block",
                   "step": "accumulate one frame + normalize the integration"},
        "roofline": {
            "kernel": "xe_accumulate call: corr_kernel + merge_kernel (chunks 1..3)",
            "bound": "mfma",
            "achieved": round(achieved_tops, 2),
            "peak": MFMA_INT8_PEAK_TOPS,
            "unit": "TOPS",
            "frac": round(achieved_tops / MFMA_INT8_PEAK_TOPS, 4),
            "traffic": measured_traffic(),
            "executed": measured_execution(),
        },
        "kernel_ms": round(kern_ms, 5),
        "device": _device_info(torch),
        "kernel_alg_hbm_gbps": round(alg_bytes / (kern_ms / 1e3) / 1e9, 1),
        "wall_s": round(t_wall, 4),
    }
    del packed, mask, vis, cnt, out
    torch.cuda.empty_cache()
    if not args.no_batched:
        res["batched"] = batched_leg(torch, reps=max(3, min(20, args.steps)))
        torch.cuda.empty_cache()
    if not args.no_flags:
        res["flags"] = flags_leg(torch, reps=max(5, min(50, args.steps)))
        torch.cuda.empty_cache()
    if not args.no_assembly:
        res["assembly"] = assembly_leg(torch, reps=max(5, min(50, args.steps)))
        torch.cuda.empty_cache()
    if not args.no_shift:
        res["shift"] = shift_leg(torch, reps=max(5, min(50, args.steps)))
        torch.cuda.empty_cache()
    if not args.no_large_n:
        res["large_n"] = large_n_leg(torch, reps=max(5, min(20, args.steps)))
        torch.cuda.empty_cache()
    if not args.no_pipeline:
        res["pipeline"] = pipeline_leg(torch, reps=max(5, min(30, args.steps)))
        torch.cuda.empty_cache()
    if not args.no_serving:
        res["serving"] = serving_leg(torch, args.serve_seconds)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(fr, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
