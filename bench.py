"""Benchmark of the partitioned reduction on one MI355X.

Headline workload (the message-size sweep at its largest size): 8 simulated
ranks, FP32 sum, 2^26 elements (256 MiB) per rank, 64 partitions readied
one by one in a seeded random order, inputs N(0, 1) drawn on the GPU.  One
step = pcoll_start + 64 x pcoll_pready + pcoll_wait (the whole hot path:
plan is done once at init; ready flags, tile claiming, reduce, completion
flags every step).  Inputs are resident in HBM before timing starts.

Prints one JSON line: effective reduce GB/s (algorithmic bytes
P*N*4 + N*4 per step over the step time), the roofline record of the
reduce kernel (its own duration from HIP events on the stream it runs on),
and the CPU oracle timed on a bounded sample on the host cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, published
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles",
                               "reduce_f32_p8_256MiB_traffic.json")
# what the counted launch depends on: the kernel's sources, the code that
# sizes its grid and the tuned launch parameters
KERNEL_SOURCES = ["csrc/persistent.hpp", "csrc/tiles.hpp",
                  "csrc/reduce_impl.hpp", "csrc/reduce_f32.hip",
                  "csrc/layout.hpp", "csrc/runtime.cpp", "tuned_mi355x.txt"]


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2604_22228_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_record(algo_bytes):
    """HBM bytes per launch from the committed rocprofv3 counter runs,
    scaled by the copy-kernel calibration; null when the kernel source has
    changed since the counters were taken."""
    try:
        with open(PROFILE_TRAFFIC) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--ranks", type=int, default=8)
    ap.add_argument("--log2n", type=int, default=26)
    ap.add_argument("--nparts", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--probe-copy", action="store_true",
                    help="only run the streaming-copy probe (counter "
                         "calibration) and exit")
    ap.add_argument("--only-8bit", choices=sorted(EIGHT_BIT),
                    help="only time the 8-bit workload in this format "
                         "(for profiling) and exit")
    ap.add_argument("--only", choices=sorted(ONLY) + sorted(EIGHT_BIT),
                    help="only time this workload (for profiling): steps "
                         "epochs after warmup ones, one JSON line, exit")
    return ap.parse_args()


def probe_copy(pc, torch, steps):
    """Streaming copy of 2 GiB: the calibration run for the byte counters
    and the attainable-bandwidth reference."""
    nbytes = 2 << 30
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1.0)
    s = torch.cuda.current_stream()
    for _ in range(2):
        pc.pcoll_probe_copy(dst, src, nbytes, s)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), \
        torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        pc.pcoll_probe_copy(dst, src, nbytes, s)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    return {"bytes_per_launch": 2 * nbytes, "ms": ms,
            "GBps": 2 * nbytes / (ms * 1e-3) / 1e9}


def probe_streams(pc, torch, steps, P=8, log2n=26):
    """The headline's memory traffic without the reduce's protocol or
    arithmetic (pcoll_probe_stream): P reads of 2^log2n FP32 elements each
    and one write of their XOR (the reduce's P:1 read:write mix, the same
    bytes as one headline launch), and the same P reads alone, in three
    layouts (the reduce's tile schedule, grid-stride, contiguous shares per
    workgroup).  Buffers are 9x the MALL, so every launch streams from HBM.
    GB/s over the mean launch time (HIP events around `steps` launches)."""
    n = 1 << log2n
    nbytes = 4 * n
    srcs = [torch.full((n,), float(r + 1), device="cuda") for r in range(P)]
    dst = torch.empty(n, device="cuda")
    s = torch.cuda.current_stream()
    res = {}
    for layout, lname in ((1, "tiles"), (0, "grid_stride"), (2, "chunks")):
        for name, write in (("read_write", 1), ("read_only", 0)):
            for _ in range(2):
                pc.pcoll_probe_stream(srcs, dst, nbytes, write, layout, s)
            torch.cuda.synchronize()
            e0, e1 = _events(torch)
            e0.record(s)
            for _ in range(steps):
                pc.pcoll_probe_stream(srcs, dst, nbytes, write, layout, s)
            e1.record(s)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            total = (P + write) * nbytes
            res[f"{name}_{lname}"] = {
                "bytes_per_launch": total, "ms": round(ms, 4),
                "GBps": round(total / (ms * 1e-3) / 1e9, 1)}
    res["streams"] = f"{P} reads of {nbytes >> 20} MiB (+ 1 write)"
    res["layouts"] = ("tiles: the headline reduce's tile schedule "
                      "(8192-element tiles in bands of 16, taken in turn) "
                      "without its protocol, on 2 workgroups of 8 waves per "
                      "compute unit; grid_stride: thread i takes vectors i, "
                      "i + T, ...; chunks: each of 4 workgroups per compute "
                      "unit streams its own contiguous share")
    del srcs, dst
    torch.cuda.empty_cache()
    return res


def cpu_baseline(orc, xs_dev, P, seconds):
    """The oracle (FP64 rank-order sum, element-parallel over the host
    cores) on a bounded sample: the first 2^24 elements (64 MiB) of every
    rank, repeated until about `seconds` of CPU work; beside it the
    single-threaded fixed-order oracle on the first 2^22 elements for a
    quarter of that time (`single_thread_value`, same unit)."""
    m = 1 << 24
    sample = [x[:m].cpu().numpy() for x in xs_dev]
    reps, t0 = 0, time.perf_counter()
    while True:
        orc.sum_f32_f64(sample, threads=True)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    algo = (P * m * 4 + m * 4) * reps
    # the single-threaded fixed-order oracle on a quarter of the sample
    q = [x[:m // 4] for x in sample]
    reps1, t1 = 0, time.perf_counter()
    while True:
        orc.sum_f32_f64(q, threads=False)
        reps1 += 1
        el1 = time.perf_counter() - t1
        if el1 >= seconds / 4:
            break
    single = (P * m + m) * reps1 / el1 / 1e9  # (P + 1) * 4 * m / 4 bytes
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f
                          if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(algo / el / 1e9, 3), "unit": "GB/s",
            "cores": orc.omp_threads(), "cpu_model": model, "kind": "oracle",
            "single_thread_value": round(single, 3),
            "sample": f"first 2^24 elements of each of the {P} ranks, FP64 "
                      f"rank-order sum over host cores, {reps} repetitions "
                      f"in {el:.1f} s; single thread: the first 2^22 "
                      f"elements, {reps1} repetitions in {el1:.1f} s"}


def ready_array(order):
    """A ready list as a ctypes int array, built once outside the timed
    loops: the binding passes it to pcoll_pready_list as is (a numpy array
    costs about 2 us of conversion per call)."""
    import ctypes
    order = [int(p) for p in order]
    return (ctypes.c_int * len(order))(*order)


def _events(torch):
    return (torch.cuda.Event(enable_timing=True),
            torch.cuda.Event(enable_timing=True))


def time_requests(torch, reqs, orders, stream, warmup, reps):
    """Time-to-reduce of a set of requests sharing one stream: start all,
    ready every partition (each request's seeded order, one list call per
    request), wait all.  Returns (host ms per rep, device ms per rep),
    medians.  The host time comes from a pass with nothing else on the
    stream; the device time from a second pass: the kernel's own (start and
    end stamped by the launch, debug timing) for one request in
    direct-launch mode, else HIP events around the starts and the
    readiness calls."""
    import statistics
    own = len(reqs) == 1 and not reqs[0].config().graph
    host, _ = _time_pass(torch, reqs, orders, stream, warmup, reps,
                         events=False)
    _, devt = _time_pass(torch, reqs, orders, stream, 0, reps)
    if own:
        reqs[0].set_config(debug=4)
        _time_pass(torch, reqs, orders, stream, 1, 0, events=False)
        st0 = reqs[0].stats()
        _time_pass(torch, reqs, orders, stream, 0, reps, events=False)
        st1 = reqs[0].stats()
        reqs[0].set_config(debug=0)
        devt = [(st1.kernel_ms_total - st0.kernel_ms_total) /
                max(st1.kernel_timed - st0.kernel_timed, 1)]
    return statistics.median(host), statistics.median(devt)


def trace_span_ms(pc, torch, req, order, stream, reps):
    """The kernel's own span (first workgroup start to last workgroup end)
    and its busy span (first tile queued to last workgroup end, which
    leaves out the wait for the host's readiness call) from its
    per-workgroup wall-clock trace (debug bit 2), medians over `reps`
    epochs after one warmup.  It works for graph replays too, where no
    launch events can stamp the kernel."""
    import statistics
    dbg = req.config().debug
    req.set_config(debug=dbg | 2)
    spans, busy = [], []
    for it in range(1 + reps):
        torch.cuda.synchronize()
        req.start()
        req.pready_list(order)
        stream.query()
        req.wait()
        torch.cuda.synchronize()  # the last workgroup's stamp is written
        if it:
            tr, khz = pc.pcoll_debug_trace(req.h)
            end = max(e for _, _, e, _ in tr)
            spans.append((end - min(s for s, _, _, _ in tr)) / khz)
            busy.append((end - min(f for _, f, _, _ in tr if f)) / khz)
    req.set_config(debug=dbg)
    return statistics.median(spans), statistics.median(busy)


def _time_pass(torch, reqs, orders, stream, warmup, reps, events=True):
    """Host ms per rep and, with `events`, device ms per rep between HIP
    events recorded before the starts and after the readiness calls (the
    host time of a pass with events includes the markers' cost)."""
    host, devt = [], []
    for it in range(warmup + reps):
        if events:
            e0, e1 = _events(torch)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if events:
            e0.record(stream)
        for r in reqs:
            r.start()
        for r, o in zip(reqs, orders):
            r.pready_list(o)
        if events:
            e1.record(stream)
            stream.query()  # the HIP runtime may hold the record back
        for r in reqs:
            r.wait()
        t1 = time.perf_counter()
        if events:
            e1.synchronize()
        if it >= warmup:
            host.append((t1 - t0) * 1e3)
            if events:
                devt.append(e0.elapsed_time(e1))
    return host, devt


def size_sweep(pc, torch, synth, stream):
    """The message-size sweep: 8 ranks, FP32 sum, 2^k elements per rank
    (k = 0..26, 4 B .. 256 MiB), 1 / 4 / 16 / 64 partitions readied in a
    seeded random order with one list call.  Cold cache: a 1 GiB fill (4x
    the 256 MB MALL) runs on the stream before every timed epoch, outside
    the timed events.  Per point, medians over the epochs: the epoch's
    device time from HIP events recorded before start and after the
    readiness call on the bound stream (marker packets, which cost about
    5 us each on MI355X), the kernel's own time (events stamped at its
    start and end by the launch), and effective GB/s = 36 * 2^k B / the
    kernel's time.  The gate (>= 70 % of HBM peak at 64 MiB per rank and
    up) is read on the kernel's time; the events' figure is given beside
    it."""
    import statistics
    dev = torch.device("cuda:0")
    P = 8
    big = synth.normal_f32(P, 1 << 26, synth.seed_for(2), device=dev)
    out = torch.empty(1 << 26, device=dev)
    flush = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    points, gate, gate_ev = [], [], []
    for k in range(27):
        n = 1 << k
        xs = [b[:n] for b in big]
        reps = 20 if k <= 22 else 10
        for nparts in (1, 4, 16, 64):
            req = pc.Request([n], pc.FLOAT32, pc.SUM, nparts, P)
            req.set_config(debug=4)  # the kernel's own time
            req.bind([xs], [out[:max(n, 4)]], stream=stream)
            order = ready_array(synth.permutation(nparts,
                                                  k * 100 + nparts))
            ts, ks = [], []
            for it in range(2 + reps):
                pc.pcoll_probe_fill(flush, 4 << 28, 0, stream)
                e0, e1 = _events(torch)
                e0.record(stream)
                req.start()
                req.pready_list(order)
                e1.record(stream)
                stream.query()  # submits the record now
                req.wait()
                if it >= 2:
                    e1.synchronize()
                    ts.append(e0.elapsed_time(e1))
                    ks.append(req.stats().last_kernel_ms)
            req.free()
            ms, kms = statistics.median(ts), statistics.median(ks)
            gbps = 36 * n / (kms * 1e-3) / 1e9
            points.append([k, nparts, round(ms * 1e3, 2), round(kms * 1e3, 2),
                           round(gbps, 1)])
            if k >= 24:
                gate.append(gbps)
                gate_ev.append(36 * n / (ms * 1e-3) / 1e9)
    del big, out, flush
    torch.cuda.empty_cache()
    return {"columns": ["log2_elements", "partitions", "device_us",
                        "kernel_us", "GBps"],
            "points": points, "cold_cache": True,
            "min_pct_hbm_peak_at_64MiB_and_up": round(
                100 * min(gate) / HBM_PEAK_GBPS, 2),
            "min_pct_hbm_peak_at_64MiB_and_up_events": round(
                100 * min(gate_ev) / HBM_PEAK_GBPS, 2)}


def epoch_trace(pc, torch, synth, stream, reps=10):
    """Where an epoch's time goes at 2^24 and 2^26 elements per rank (8
    ranks, FP32, 64 partitions readied with one list call right after
    start, cold: a 1 GiB fill before each epoch): the epoch's device time
    from HIP events, and from the kernel's own per-workgroup wall-clock
    trace (debug bit 1): the spread of workgroup starts, the time from the
    first start until the first tile was queued, the time from that until
    the first workgroup ran out of tiles (the streaming part), the spread
    of the workgroups' ends (the last round of tiles), and the time outside
    the kernel (events minus the kernel's span).  Medians over `reps`
    epochs, in microseconds."""
    import statistics
    dev = torch.device("cuda:0")
    P = 8
    big = synth.normal_f32(P, 1 << 26, synth.seed_for(2), device=dev)
    out = torch.empty(1 << 26, device=dev)
    flush = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    res = {}
    for k in (24, 26):
        n = 1 << k
        req = pc.Request([n], pc.FLOAT32, pc.SUM, 64, P)
        req.set_config(debug=2)
        req.bind([[b[:n] for b in big]], [out[:n]], stream=stream)
        order = ready_array(synth.permutation(64, k * 100 + 64))
        rows = []
        for it in range(2 + reps):
            pc.pcoll_probe_fill(flush, 4 << 28, 0, stream)
            e0, e1 = _events(torch)
            e0.record(stream)
            req.start()
            req.pready_list(order)
            e1.record(stream)
            stream.query()
            req.wait()
            e1.synchronize()
            if it < 2:
                continue
            tr, khz = pc.pcoll_debug_trace(req.h)
            us = 1e3 / khz  # microseconds per tick
            st = [s for s, _, _, _ in tr]
            fi = [f for _, f, _, _ in tr if f]
            en = [e for _, _, e, _ in tr]
            t0 = min(st)
            rows.append({
                "events_us": e0.elapsed_time(e1) * 1e3,
                "kernel_span_us": (max(en) - t0) * us,
                "start_spread_us": (max(st) - t0) * us,
                "first_tile_queued_us": (min(fi) - t0) * us,
                "streaming_us": (min(en) - min(fi)) * us,
                "end_spread_us": (max(en) - min(en)) * us,
                "tiles_per_group_min": min(t for _, _, _, t in tr),
                "tiles_per_group_max": max(t for _, _, _, t in tr),
            })
        st = req.stats()
        req.free()
        rec = {key: round(statistics.median(r[key] for r in rows), 2)
               for key in rows[0]}
        rec["outside_kernel_us"] = round(rec["events_us"] -
                                         rec["kernel_span_us"], 2)
        rec["groups"] = st.groups
        rec["GBps"] = round(36 * n / rec["events_us"] / 1e3, 1)
        res[f"2^{k}"] = rec
    del big, out, flush
    torch.cuda.empty_cache()
    return res


def rank_readiness(pc, torch, synth, reps=5):
    """Per-rank readiness against bulk readiness, with compute-bound
    producers (the gradient-producing backward pass that per-rank readiness
    is for): 8 ranks, FP32, 2^26 elements per rank, 8 partitions; the
    producer of (rank, partition) is a 4096 x 512 by 512 x 2048 FP32 matrix
    product written into that rank's partition (a synthetic workload,
    outside the library), ranks spread over two streams.  overlapped: the
    reduction starts first and each (rank, partition) is marked on the
    device right after its product, so the kernel reduces each partition
    while later ones are produced; run in the library's producer mode
    (`producers` = 1: one resident wave per SIMD with fewer registers, so
    that the products' matrix-core waves start beside the resident kernel),
    on every compute unit and on 64 of them (a persistent kernel that waits
    holds registers the producers could use); the signalling streams are
    checked to run beside the reduce kernel's stream.  bulk: every product
    first, then start, ready everything, wait.  Host ms from the first product to the return of wait
    (median); `identical`: every run gives the same output bits."""
    import statistics
    dev = torch.device("cuda:0")
    P, n, nparts = 8, 1 << 26, 8
    m, k, q = 4096, 512, 2048
    gen = torch.Generator(device=dev).manual_seed(synth.seed_for(2) + 7)
    a_ = [torch.randn(m, k, device=dev, generator=gen) for _ in range(P)]
    b_ = torch.randn(k, q, device=dev, generator=gen)
    xs = [torch.empty(n, device=dev) for _ in range(P)]
    out = torch.empty(n, device=dev)
    from paper_2604_22228_amd.streams import independent_streams
    stream = torch.cuda.Stream(dev)
    sig = independent_streams(stream, 2)
    req = pc.Request([n], pc.FLOAT32, pc.SUM, nparts, P)
    req.bind([xs], [out], stream=stream)
    parts_dev = torch.arange(nparts, dtype=torch.int32, device=dev)
    spans = [pc.pcoll_part_info(req.h, j)[1:] for j in range(nparts)]
    assert all(ln == m * q for _, ln in spans)
    allp = ready_array(range(nparts))
    torch.cuda.synchronize()

    def produce(r, j):
        off, ln = spans[j]
        with torch.cuda.stream(sig[r % 2]):
            torch.mm(a_[r], b_, out=xs[r][off:off + ln].view(m, q))

    def overlapped():
        req.start()
        for j in range(nparts):
            for r in range(P):
                produce(r, j)
                req.pready_rank_on_stream(r, parts_dev[j:j + 1], 1,
                                          sig[r % 2])
        req.wait()

    def bulk():
        for j in range(nparts):
            for r in range(P):
                produce(r, j)
        for s_ in sig:
            s_.synchronize()
        req.start()
        req.pready_list(allp)
        req.wait()

    res = {}
    outs = []
    for name, fn, groups in (("overlapped_ms", overlapped, 0),
                             ("overlapped_64_groups_ms", overlapped, 64),
                             ("bulk_ms", bulk, 0)):
        req.set_config(groups=groups, producers=1)
        ts = []
        for it in range(2 + reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            ts.append((time.perf_counter() - t0) * 1e3)
        torch.cuda.synchronize()
        outs.append(out.clone())
        res[name] = round(statistics.median(ts[2:]), 4)
    res["identical"] = all(bool(torch.equal(o, outs[0])) for o in outs)
    req.free()
    del a_, b_, xs, out, outs
    torch.cuda.empty_cache()
    res["speedup"] = round(res["bulk_ms"] / min(
        res["overlapped_ms"], res["overlapped_64_groups_ms"]), 3)
    res["workload"] = ("8 ranks, FP32, 2^26 elements per rank, 8 partitions, "
                       "an 8.6 GFLOP FP32 product per rank and partition")
    res["reduce_config"] = "producers = 1 (one workgroup of 4 waves per "\
        "compute unit, 2 rows in flight per lane)"
    return res


def staggered_arrivals(pc, torch, synth, reps=5, gap_us=50.0):
    """Stragglers, the case per-rank readiness is for: 8 ranks, FP32, 2^26
    elements per rank (inputs resident), 8 or 64 partitions; rank r's
    partition j arrives at (j + lag_r) x D (partitions in order, as a
    backward pass emits gradient buckets; lag_r a seeded per-rank lag of up
    to 3, D = `gap_us`).  The arrivals are played on a side stream (one
    that runs beside the reduce kernel's) as timed spins in arrival order,
    each followed by a one-element kernel: the mark
    (pcoll_pready_rank_on_stream of that rank and partition) where the mode
    marks per arrival, else a one-element torch kernel, so that every mode
    plays the same kernels.  The whole schedule is enqueued behind a gate
    spin longer than the host takes to enqueue it, so the device sets the
    pace (`device_paced`: the gate was still running when the host was
    done, in every epoch).  Three ways to ready the partitions:
      per_rank: the reduce starts first and each arrival is marked right
        after its spin, so a partition is reduced as soon as its last rank
        has arrived;
      bulk_marked: the reduce starts first, but every partition is marked
        once, after the last arrival (pcoll_pready_on_stream of all);
      bulk_started: the reduce is launched after the last arrival (its
        stream waits for it), every partition ready (a reduction that
        begins when its data are complete).
    Device times from HIP events: `window_us` from the end of the gate to
    the last arrival, `after_last_us` from the last arrival to the end of
    the reduce (what readiness per rank hides), `epoch_us` from the end of
    the gate to the end of the reduce; medians over `reps` epochs.
    `identical`: every epoch of every mode gives the same output bits.  The
    reduce runs in its tuned launch (producers = 0): the spins and marks
    are small kernels."""
    import statistics
    dev = torch.device("cuda:0")
    P, n = 8, 1 << 26
    xs = synth.normal_f32(P, n, synth.seed_for(2) + 5, device=dev)
    out = torch.empty(n, device=dev)
    one = torch.zeros(1, device=dev)
    from paper_2604_22228_amd.streams import independent_streams
    stream = torch.cuda.Stream(dev)
    side = independent_streams(stream, 1)[0]
    rng = np.random.default_rng(synth.seed_for(2) + 11)
    lag = rng.uniform(0.0, 3.0, size=P)  # in units of D
    # spin cycles per microsecond: torch's spin counts shader clocks
    cyc_us = 2000
    res = {"gap_us": gap_us, "rank_lag_in_gaps": [round(float(x), 3)
                                                  for x in lag]}
    ref = None
    identical = paced = True
    for nparts in (8, 64):
        req = pc.Request([n], pc.FLOAT32, pc.SUM, nparts, P)
        req.set_config(producers=0)
        req.bind([xs], [out], stream=stream)
        ids = torch.arange(nparts, dtype=torch.int32, device=dev)
        arrivals = sorted((j + lag[r], r, j) for r in range(P)
                          for j in range(nparts))
        allp = ready_array(range(nparts))
        gate_ms = 5.0
        torch.cuda.synchronize()

        def play(mark):
            t = 0.0
            for when, r, j in arrivals:
                cycles = int((when - t) * gap_us * cyc_us)
                t = when
                with torch.cuda.stream(side):
                    if cycles > 0:
                        torch.cuda._sleep(cycles)
                    if not mark:
                        one.add_(1.0)
                if mark:
                    req.pready_rank_on_stream(r, ids[j:j + 1], 1, side)

        rec = {}
        for mode in ("per_rank", "bulk_marked", "bulk_started"):
            window, after, whole = [], [], []
            for it in range(2 + reps):
                out.fill_(float("nan"))
                torch.cuda.synchronize()
                e0, e_last = _events(torch)
                e_done = torch.cuda.Event(enable_timing=True)
                if mode != "bulk_started":
                    req.start()
                    e_done.record(stream)
                    stream.query()  # submits the launch now
                h0 = time.perf_counter()
                with torch.cuda.stream(side):
                    torch.cuda._sleep(int(gate_ms * 1e3 * cyc_us))
                e0.record(side)
                side.query()  # the gate starts now
                play(mode == "per_rank")
                e_last.record(side)
                side.query()  # submits what is still held back
                gate_open = e0.query()
                enq_ms = (time.perf_counter() - h0) * 1e3
                if mode == "bulk_marked":
                    req.pready_on_stream(ids, nparts, side)
                side.query()
                if mode == "bulk_started":
                    stream.wait_event(e_last)
                    req.start()
                    req.pready_list(allp)
                    e_done.record(stream)
                    stream.query()
                req.wait()
                torch.cuda.synchronize()
                gate_ms = max(gate_ms, 2.0 * enq_ms)
                if it < 2:
                    continue
                paced = paced and not gate_open
                window.append(e0.elapsed_time(e_last) * 1e3)
                after.append(e_last.elapsed_time(e_done) * 1e3)
                whole.append(e0.elapsed_time(e_done) * 1e3)
                if ref is None:
                    ref = out.clone()
                elif not torch.equal(out, ref):
                    identical = False
            rec[mode] = {"window_us": round(statistics.median(window), 1),
                         "after_last_us": round(statistics.median(after), 1),
                         "epoch_us": round(statistics.median(whole), 1)}
        for b in ("bulk_started", "bulk_marked"):
            rec[f"after_last_speedup_vs_{b}"] = round(
                rec[b]["after_last_us"] / rec["per_rank"]["after_last_us"], 2)
            rec[f"epoch_speedup_vs_{b}"] = round(
                rec[b]["epoch_us"] / rec["per_rank"]["epoch_us"], 3)
        st = req.stats()
        rec["groups"], rec["group_waves"] = st.groups, st.group_waves
        req.free()
        res[f"{nparts}_partitions"] = rec
    res["identical"] = identical
    res["device_paced"] = paced
    res["workload"] = ("8 ranks, FP32, 2^26 elements per rank, rank r's "
                       "partition j arriving at (j + lag_r) x gap_us")
    del xs, out, ref
    torch.cuda.empty_cache()
    return res


def pack_kernels(pc, torch, reps=10):
    """The producer-side packers, timed apart from the reduction: 2^28 FP32
    values (1 GiB) to bf16, to e4m3 or e5m2 codes with a binary32 scale per
    256 values, and to MX blocks (e4m3 codes, an E8M0 scale byte per 32).
    Mean device time of `reps` launches between HIP events; GB/s of the
    algorithmic bytes (4 B read + the codes and scales written per
    value)."""
    dev = torch.device("cuda:0")
    n = 1 << 28
    g = torch.Generator(device=dev).manual_seed(22228)
    x = torch.randn(n, generator=g, device=dev) * 1e-2
    s = torch.cuda.current_stream()
    bf = torch.empty(n, dtype=torch.int16, device=dev)
    q = torch.empty(n, dtype=torch.uint8, device=dev)
    sc = torch.empty(n // 256, device=dev)
    mx = torch.empty(n // 32, dtype=torch.uint8, device=dev)
    cases = {
        "bf16": (lambda: pc.pcoll_pack_bf16(x, bf, n, s), 6 * n),
        "e4m3": (lambda: pc.pcoll_pack_fp8(x, q, sc, n, s),
                 5 * n + 4 * (n // 256)),
        "e5m2": (lambda: pc.pcoll_pack_e5m2(x, q, sc, n, s),
                 5 * n + 4 * (n // 256)),
        "mxfp8": (lambda: pc.pcoll_pack_mxfp8(x, q, mx, n, s),
                  5 * n + n // 32),
    }
    res = {}
    for name, (fn, nbytes) in cases.items():
        fn()
        torch.cuda.synchronize()
        e0, e1 = _events(torch)
        e0.record(s)
        for _ in range(reps):
            fn()
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[name] = {"ms": round(ms, 4), "bytes": nbytes,
                     "GBps": round(nbytes / (ms * 1e-3) / 1e9, 1)}
    res["values"] = n
    del x, bf, q, sc, mx
    torch.cuda.empty_cache()
    return res


def graph_lifecycle(pc, torch, reps=20):
    """Graph against direct launch over bucket counts (equal buckets, FP32,
    8 ranks) at 2 MiB and 512 MiB per rank: bind (descriptor table upload),
    first start (graph: capture + instantiate + launch), then per epoch the
    host time of start and the device time of the epoch (medians)."""
    import statistics
    dev = torch.device("cuda:0")
    P = 8
    big = [torch.ones(1 << 27, device=dev) for _ in range(P)]
    obig = torch.empty(1 << 27, device=dev)
    stream = torch.cuda.Stream(dev)
    rows = []
    for total in (1 << 19, 1 << 27):  # elements per rank: 2 MiB, 512 MiB
        for nb in (1, 8, 32, 128):
            c = total // nb
            counts = [c] * nb
            ins = [[b[i * c:(i + 1) * c] for b in big] for i in range(nb)]
            outs = [obig[i * c:(i + 1) * c] for i in range(nb)]
            rec = {"bytes_per_rank": total * 4, "buckets": nb}
            for graph in (1, 0):
                req = pc.Request(counts, pc.FLOAT32, pc.SUM, 8, P,
                                 batched=True)
                req.set_config(graph=graph)
                t0 = time.perf_counter()
                req.bind(ins, outs, stream=stream)
                t1 = time.perf_counter()
                order = ready_array(range(req.nparts_total))
                req.start()
                t2 = time.perf_counter()
                req.pready_list(order)
                req.wait()
                hs, ds = [], []
                for it in range(reps):
                    e0, e1 = _events(torch)
                    torch.cuda.synchronize()
                    e0.record(stream)
                    h0 = time.perf_counter()
                    req.start()
                    h1 = time.perf_counter()
                    req.pready_list(order)
                    e1.record(stream)
                    stream.query()  # submits the record now
                    req.wait()
                    e1.synchronize()
                    hs.append((h1 - h0) * 1e6)
                    ds.append(e0.elapsed_time(e1))
                st = req.stats()
                key = "graph" if graph else "direct"
                rec[key] = {"bind_ms": round((t1 - t0) * 1e3, 3),
                            "first_start_ms": round((t2 - t1) * 1e3, 3),
                            "start_us": round(statistics.median(hs), 1),
                            "epoch_ms": round(statistics.median(ds), 4)}
                if graph:
                    rec[key]["capture_ms"] = round(st.last_capture_ms, 3)
                    rec[key]["instantiate_ms"] = round(
                        st.last_instantiate_ms, 3)
                req.free()
            rows.append(rec)
    del big, obig
    torch.cuda.empty_cache()
    return rows


EIGHT_BIT = {"e4m3": ("FP8_E4M3", "pcoll_pack_fp8", 256,
                      "fp8_batched_p8_1GiB"),
             "e5m2": ("FP8_E5M2", "pcoll_pack_e5m2", 256,
                      "e5m2_batched_p8_1GiB"),
             "mxfp8": ("MXFP8_E4M3", "pcoll_pack_mxfp8", 32,
                       "mxfp8_batched_p8_1GiB")}


def eight_bit(pc, torch, synth, fmt, stream, warmup, reps, errors=True):
    """The 8-bit workload: 8 ranks, 128 buckets totalling 2^30 elements per
    rank, N(0, 1e-2) with 1% outliers at 50x, packed to `fmt` (binary32
    scales per 256 elements, or E8M0 bytes per 32 for MX blocks)."""
    dev = torch.device("cuda:0")
    cur = torch.cuda.current_stream(dev)
    dname, pname, blk, key = EIGHT_BIT[fmt]
    dtype, pack = getattr(pc, dname), getattr(pc, pname)
    sdt, sbytes = (torch.uint8, 1) if blk == 32 else (torch.float32, 4)
    counts = synth.fp8_bucket_counts()
    n = sum(counts)
    nbytes = 9 * n + 9 * sbytes * sum((c + blk - 1) // blk for c in counts)
    order = ready_array(synth.permutation(len(counts) * 32, 5))
    qs, ss = [], []
    for b, c in enumerate(counts):
        qrow, srow = [], []
        for t in synth.normal_with_outliers_f32(
                8, c, synth.seed_for(5) * 1000 + b, 1e-2, device=dev):
            q = torch.empty(c, dtype=torch.uint8, device=dev)
            s = torch.empty((c + blk - 1) // blk, dtype=sdt, device=dev)
            pack(t, q, s, c, cur)
            qrow.append(q)
            srow.append(s)
        qs.append(qrow)
        ss.append(srow)
    torch.cuda.synchronize()
    ys = [torch.empty(c, dtype=torch.uint8, device=dev) for c in counts]
    yss = [torch.empty((c + blk - 1) // blk, dtype=sdt, device=dev)
           for c in counts]
    req = pc.Request(counts, dtype, pc.SUM, 32, 8, batched=True)
    req.bind(qs, ys, ss, yss, stream=stream)
    h, d = time_requests(torch, [req], [order], stream, warmup, reps)
    res = {"host_ms": round(h, 4), "kernel_ms": round(d, 4),
           "GBps": round(nbytes / d / 1e6, 1), "comp": req.config().comp}
    req.free()
    if errors:
        res["error"] = eight_bit_errors(pc, torch, synth, fmt, counts, qs, ss,
                                        ys, yss, stream)
    del qs, ss, ys, yss
    torch.cuda.empty_cache()
    return key, res


def _dequant(torch, fmt, codes, scales, c):
    """Values of 8-bit codes and their block scales, in float32 (exact):
    torch's float8 decode times the binary32 scale of each 256 elements, or
    times 2^(b - 127) of each E8M0 byte b of 32 elements."""
    f8 = torch.float8_e5m2 if fmt == "e5m2" else torch.float8_e4m3fn
    v = codes[:c].view(f8).float()
    if fmt == "mxfp8":
        s = torch.ldexp(torch.ones_like(scales, dtype=torch.float32),
                        scales.int() - 127)
        return v * s.repeat_interleave(32)[:c]
    return v * scales.repeat_interleave(256)[:c]


def eight_bit_errors(pc, torch, synth, fmt, counts, qs, ss, ys, yss, stream,
                     sample=1 << 24):
    """Error of the 8-bit result, ungated, on a sample of buckets (every
    8th bucket from the first until 2^24 elements): against the FP64 sum of
    the dequantized payload in rank order (the reduction's own error,
    torch float64 on the host) and against the library's plain FP32 path
    run on the values before quantization (end to end: packing plus
    reduction).  Max Sigma|x|-normalized error |y - ref| / max(Sigma|x|,
    tau) (tau = the output block's smallest normal, for the FP64 error) and
    the normwise ||y - ref|| / ||ref||."""
    dev = torch.device("cuda:0")
    pick, tot = [], 0
    for b in range(0, len(counts), 8):
        if tot >= sample:
            break
        pick.append(b)
        tot += counts[b]
    e64 = eend = 0.0
    n64 = d64 = nend = dend = 0.0
    for b in pick:
        c = counts[b]
        blk = 32 if fmt == "mxfp8" else 256
        y = _dequant(torch, fmt, ys[b], yss[b], c)
        xq = [_dequant(torch, fmt, q, s, c) for q, s in zip(qs[b], ss[b])]
        # FP64 reference of the payload, rank order, on the host
        y64 = torch.zeros(c, dtype=torch.float64)
        absq = torch.zeros(c, dtype=torch.float64)
        for x in xq:
            xh = x.cpu().double()
            y64 += xh
            absq += xh.abs()
        if fmt == "mxfp8":
            so = torch.ldexp(torch.ones(yss[b].numel(), dtype=torch.float64),
                             yss[b].cpu().long() - 127)
        else:
            so = yss[b].cpu().double()
        small = {"e4m3": 2.0 ** -6, "mxfp8": 2.0 ** -6, "e5m2": 2.0 ** -14}
        tau = (so * small[fmt]).repeat_interleave(blk)[:c]
        yh = y.cpu().double()
        e64 = max(e64, float(((yh - y64).abs() / torch.maximum(absq, tau))
                             .max()))
        n64 += float(((yh - y64) ** 2).sum())
        d64 += float((y64 ** 2).sum())
        # the plain FP32 path on the values before quantization
        xs = synth.normal_with_outliers_f32(
            8, c, synth.seed_for(5) * 1000 + b, 1e-2, device=dev)
        yf = torch.empty(c, device=dev)
        r = pc.Request([c], pc.FLOAT32, pc.SUM, 32, 8)
        r.bind([xs], [yf], stream=stream)
        r.start()
        r.pready_range(0, 31)
        r.wait()
        r.free()
        torch.cuda.synchronize()
        absx = torch.stack([x.abs() for x in xs]).sum(0)
        tiny = torch.full_like(absx, 2.0 ** -126)
        eend = max(eend, float(((y - yf).abs() / torch.maximum(absx, tiny))
                               .max()))
        nend += float(((y - yf).double() ** 2).sum())
        dend += float((yf.double() ** 2).sum())
        del xs, yf, xq, y
    return {"sample_buckets": len(pick), "sample_elements": tot,
            "vs_fp64_payload_max_norm": e64,
            "vs_fp64_payload_normwise": (n64 / d64) ** 0.5 if d64 else 0.0,
            "vs_plain_fp32_path_max_norm": eend,
            "vs_plain_fp32_path_normwise": (nend / dend) ** 0.5 if dend
            else 0.0,
            "gate_vs_fp64": {"e4m3": 6e-2, "mxfp8": 6e-2,
                             "e5m2": 1 / 9 + 16 * 2.0 ** -24}[fmt]}



def _bf16_buckets(pc, torch, synth, dev):
    """The batched workload's buckets: FP32 N(0, 1e-3) per rank and their
    bf16 packing."""
    cur = torch.cuda.current_stream(dev)
    counts = synth.batched_bf16_counts()
    f32 = [synth.normal_f32(8, c, synth.seed_for(3) * 1000 + b, std=1e-3,
                            device=dev) for b, c in enumerate(counts)]
    bf = []
    for bucket, c in zip(f32, counts):
        row = []
        for t in bucket:
            o = torch.empty(c, dtype=torch.int16, device=dev)
            pc.pcoll_pack_bf16(t, o, c, cur)
            row.append(o)
        bf.append(row)
    torch.cuda.synchronize()
    return counts, f32, bf


def only_workload(pc, torch, synth, name, warmup, steps):
    """One workload alone, for profiling: the batched bf16 buckets (8
    ranks, 64 buckets, 32 partitions each) as bf16 (direct launch or graph
    replay), bf16 pairs or FP32, or
    int32 sum / max at 16 ranks and 2^24 elements (256 partitions).  Same
    inputs, readiness order and timing as the extras."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    if name.startswith("int32"):
        n4 = 1 << 24
        xi = synth.uniform_i32(16, n4, synth.seed_for(4), -(1 << 20), 1 << 20,
                               device=dev)
        yi = torch.empty(n4, dtype=torch.int32, device=dev)
        o4 = ready_array(synth.permutation(256, synth.seed_for(4)))
        r = pc.Request([n4], pc.INT32, pc.SUM if name == "int32_sum"
                       else pc.MAX, 256, 16)
        r.bind([xi], [yi], stream=stream)
        h, d = time_requests(torch, [r], [o4], stream, warmup, steps)
        res = {"host_ms": round(h, 4), "kernel_ms": round(d, 4),
               "GBps": round(17 * n4 * 4 / d / 1e6, 1)}
        r.free()
        return res
    counts, f32, bf = _bf16_buckets(pc, torch, synth, dev)
    n_el = sum(counts)
    order = ready_array(synth.permutation(len(counts) * 32, 3))
    if name == "batched_fp32":
        ins, dt, nb = f32, pc.FLOAT32, 36 * n_el
        outs = [torch.empty(c, device=dev) for c in counts]
    else:
        ins = bf
        dt = pc.BF16_PAIR if name == "batched_bf16_pair" else pc.BFLOAT16
        nb = (20 if dt == pc.BF16_PAIR else 18) * n_el
        outs = [torch.empty(c, dtype=torch.int16, device=dev) for c in counts]
    lo = [torch.empty(c, dtype=torch.int16, device=dev) for c in counts] \
        if dt == pc.BF16_PAIR else None
    r = pc.Request(counts, dt, pc.SUM, 32, 8, batched=True)
    if name == "batched_bf16_graph":
        r.set_config(graph=1)
    r.bind(ins, outs, out_scales=lo, stream=stream)
    h, d = time_requests(torch, [r], [order], stream, warmup, steps)
    cfg = r.config()
    res = {"host_ms": round(h, 4),
           "events_ms" if cfg.graph else "kernel_ms": round(d, 4),
           "GBps": round(nb / d / 1e6, 1), "tile_elems": cfg.tile_elems,
           "group_waves": cfg.group_waves, "groups": r.stats().groups}
    r.free()
    return res


ONLY = ("batched_bf16", "batched_bf16_graph", "batched_bf16_pair",
        "batched_fp32", "int32_sum", "int32_max", "epoch_trace",
        "size_sweep", "staggered_arrivals", "rank_readiness",
        "pack_kernels")


def extras(pc, torch, synth, warmup, reps):
    """The other workloads, timed (correctness and error are the tests'
    job: the full-size GPU tests check them against the oracle).  A
    workload that fails leaves {"error": ...} in its place, so that the
    line is still printed."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    cur = torch.cuda.current_stream(dev)
    out = {}

    def guard(key, fn):
        try:
            fn()
        except Exception as e:  # noqa: BLE001 - reported, not hidden
            out[key] = {"error": f"{type(e).__name__}: {e}"}
            torch.cuda.synchronize()
            torch.cuda.empty_cache()

    def put(key, fn, *a):
        def run():
            out[key] = fn(*a)
        guard(key, run)

    put("copy_probe", probe_copy, pc, torch, 10)
    put("stream_probe", probe_streams, pc, torch, 10)
    put("size_sweep", size_sweep, pc, torch, synth, stream)
    put("epoch_trace", epoch_trace, pc, torch, synth, stream)
    put("rank_readiness", rank_readiness, pc, torch, synth)
    put("staggered_arrivals", staggered_arrivals, pc, torch, synth)
    put("graph_lifecycle", graph_lifecycle, pc, torch)

    def w1():
        # workload 1: 4 ranks, FP32, 262144 elements, 8 partitions in order;
        # 1000 epochs (a 1 MiB message), host time statistics, warm: its
        # 5 MiB stay in the caches between epochs
        import statistics
        xs = synth.uniform_f32(4, 262144, synth.seed_for(1), device=dev)
        y = torch.empty(262144, device=dev)
        req = pc.Request([262144], pc.FLOAT32, pc.SUM, 8, 4)
        req.bind([xs], [y], stream=stream)
        order = [list(range(8))]
        host, _ = _time_pass(torch, [req], order, stream, warmup, 1000,
                             events=False)
        _, d = time_requests(torch, [req], order, stream, 0, 50)
        host = sorted(host)
        out["plain_fp32_p4_1MiB"] = {
            "host_us": round(statistics.median(host) * 1e3, 1),
            "host_us_mean": round(statistics.mean(host) * 1e3, 1),
            "host_us_p10": round(host[len(host) // 10] * 1e3, 1),
            "host_us_p90": round(host[(9 * len(host)) // 10] * 1e3, 1),
            "kernel_us": round(d * 1e3, 1), "epochs": len(host),
            "GBps": round(5 * 262144 * 4 / d / 1e6, 1), "cache": "warm"}
        req.free()
        del xs, y

    guard("plain_fp32_p4_1MiB", w1)
    put("pack_kernels", pack_kernels, pc, torch)

    def w3():
        # workload 3: 64 bf16 gradient buckets, batched graph vs separate fp32
        counts = synth.batched_bf16_counts()
        P, nparts = 8, 32
        f32 = [synth.normal_f32(P, c, synth.seed_for(3) * 1000 + b, std=1e-3,
                                device=dev) for b, c in enumerate(counts)]
        bf = []
        for bucket, c in zip(f32, counts):
            row = []
            for t in bucket:
                o = torch.empty(c, dtype=torch.int16, device=dev)
                pc.pcoll_pack_bf16(t, o, c, cur)
                row.append(o)
            bf.append(row)
        torch.cuda.synchronize()
        n_el = sum(counts)
        res = {"buckets": len(counts), "elements_per_rank": n_el}
        # (a) batched bf16, one persistent launch per epoch: direct (the
        # default) and replayed from a captured graph
        yb = [torch.empty(c, dtype=torch.int16, device=dev) for c in counts]
        order = ready_array(synth.permutation(len(counts) * nparts, 3))
        for graph, key in ((0, "batched_bf16"), (1, "batched_bf16_graph")):
            rb = pc.Request(counts, pc.BFLOAT16, pc.SUM, nparts, P,
                            batched=True)
            rb.set_config(graph=graph)
            rb.bind(bf, yb, stream=stream)
            h, d = time_requests(torch, [rb], [order], stream, warmup, reps)
            st = rb.stats()
            span, busy = trace_span_ms(pc, torch, rb, order, stream, reps)
            # direct: the kernel's own time from its launch events; graph:
            # HIP events around the replay and the readiness call
            res[key] = {"host_ms": round(h, 4),
                        "events_ms" if graph else "kernel_ms": round(d, 4),
                        "kernel_span_ms": round(span, 4),
                        "kernel_busy_ms": round(busy, 4),
                        "GBps": round(n_el * 2 * (P + 1) / d / 1e6, 1),
                        "graph": rb.config().graph}
            if graph:
                res[key].update({
                    "graph_captures": st.graph_captures,
                    "capture_ms": round(st.last_capture_ms, 3),
                    "instantiate_ms": round(st.last_instantiate_ms, 3)})
            rb.free()
        # (a') the same bf16 buckets with the compensated pair output (hi, lo)
        ylo = [torch.empty(c, dtype=torch.int16, device=dev) for c in counts]
        rp = pc.Request(counts, pc.BF16_PAIR, pc.SUM, nparts, P, batched=True)
        rp.bind(bf, yb, out_scales=ylo, stream=stream)
        h, d = time_requests(torch, [rp], [order], stream, warmup, reps)
        res["batched_bf16_pair"] = {
            "host_ms": round(h, 4), "kernel_ms": round(d, 4),
            "GBps": round(n_el * (2 * P + 4) / d / 1e6, 1),
            "comp": rp.config().comp}
        rp.free()
        del ylo
        # (b) plain fp32: one request per bucket, no graph
        yf = [torch.empty(c, device=dev) for c in counts]
        reqs, orders = [], []
        for b, c in enumerate(counts):
            r = pc.Request([c], pc.FLOAT32, pc.SUM, nparts, P, batched=False)
            r.set_config(graph=0)
            r.bind([f32[b]], [yf[b]], stream=stream)
            reqs.append(r)
            orders.append(ready_array(synth.permutation(nparts, b)))
        h, d = time_requests(torch, reqs, orders, stream, warmup, reps)
        res["plain_fp32_separate"] = {
            "host_ms": round(h, 4), "kernel_ms": round(d, 4),
            "GBps": round(n_el * 4 * (P + 1) / d / 1e6, 1)}
        # the bf16 result against the fp32 path's result (not the oracle)
        num = den = 0.0
        for b in range(len(counts)):
            v = (yb[b].view(torch.bfloat16).float() - yf[b]).abs()
            num = max(num, float(v.max()))
            den = max(den, float(yf[b].abs().max()))
        res["bf16_vs_fp32_path_max_abs_rel_to_max"] = num / den if den else 0.0
        for r in reqs:
            r.free()
        # (c) batched fp32 (one launch): separates batching from precision
        rf = pc.Request(counts, pc.FLOAT32, pc.SUM, nparts, P, batched=True)
        rf.bind(f32, yf, stream=stream)
        h, d = time_requests(torch, [rf], [order], stream, warmup, reps)
        res["batched_fp32"] = {"host_ms": round(h, 4),
                               "kernel_ms": round(d, 4),
                               "GBps": round(n_el * 4 * (P + 1) / d / 1e6, 1)}
        rf.free()
        for k in ("span", "busy"):
            res[f"graph_vs_direct_kernel_{k}"] = round(
                res["batched_bf16_graph"][f"kernel_{k}_ms"] /
                res["batched_bf16"][f"kernel_{k}_ms"], 4)
        res["bf16_batched_speedup_vs_plain_fp32"] = round(
            res["plain_fp32_separate"]["host_ms"] /
            res["batched_bf16"]["host_ms"], 3)
        out["batched_bf16_vs_plain_fp32"] = res
        del f32, bf, yb, yf
        torch.cuda.empty_cache()

    guard("batched_bf16_vs_plain_fp32", w3)

    def w4():
        # workload 4: int32, 16 ranks, 2^24 elements, 256 partitions
        n4 = 1 << 24
        xi = synth.uniform_i32(16, n4, synth.seed_for(4), -(1 << 20), 1 << 20,
                               device=dev)
        yi = torch.empty(n4, dtype=torch.int32, device=dev)
        o4 = ready_array(synth.permutation(256, synth.seed_for(4)))
        for op, name in ((pc.SUM, "int32_sum_p16_64MiB"),
                         (pc.MAX, "int32_max_p16_64MiB")):
            r = pc.Request([n4], pc.INT32, op, 256, 16)
            r.bind([xi], [yi], stream=stream)
            h, d = time_requests(torch, [r], [o4], stream, warmup, reps)
            out[name] = {"host_ms": round(h, 4), "kernel_ms": round(d, 4),
                         "GBps": round(17 * n4 * 4 / d / 1e6, 1)}
            r.free()
        del xi, yi
        torch.cuda.empty_cache()

    guard("int32_sum_p16_64MiB", w4)

    # workload 5: 8-bit floats (e4m3; e5m2 and MX blocks on the same
    # values), 8 ranks, 128 buckets totalling 2^30 elements
    for fmt in ("e4m3", "e5m2", "mxfp8"):
        def w5(fmt=fmt):
            key, res = eight_bit(pc, torch, synth, fmt, stream, warmup, reps)
            out[key] = res
        guard(EIGHT_BIT[fmt][3], w5)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the P ranks are simulated as P "
              "buffers in one GPU's HBM; there is no multi-GPU path to "
              "measure.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2604_22228_amd import pcoll as pc
    from paper_2604_22228_amd import synth

    pc.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.probe_copy:
        print(json.dumps({"probe_copy": probe_copy(pc, torch, args.steps)}),
              flush=True)
        return
    if args.only_8bit or args.only in EIGHT_BIT:
        key, res = eight_bit(pc, torch, synth, args.only_8bit or args.only,
                             torch.cuda.Stream(dev), args.warmup, args.steps,
                             errors=False)
        print(json.dumps({key: res}), flush=True)
        return
    if args.only in ("epoch_trace", "size_sweep"):
        fn = epoch_trace if args.only == "epoch_trace" else size_sweep
        print(json.dumps({args.only: fn(pc, torch, synth,
                                        torch.cuda.Stream(dev))}), flush=True)
        return
    if args.only == "pack_kernels":
        print(json.dumps({args.only: pack_kernels(pc, torch)}), flush=True)
        return
    if args.only in ("staggered_arrivals", "rank_readiness"):
        fn = staggered_arrivals if args.only == "staggered_arrivals" \
            else rank_readiness
        print(json.dumps({args.only: fn(pc, torch, synth)}), flush=True)
        return
    if args.only:
        print(json.dumps({args.only: only_workload(
            pc, torch, synth, args.only, args.warmup, args.steps)}),
            flush=True)
        return

    P, n, nparts = args.ranks, 1 << args.log2n, args.nparts
    xs = synth.normal_f32(P, n, synth.seed_for(2), device=dev)
    out = torch.empty(n, dtype=torch.float32, device=dev)
    order = synth.permutation(nparts, synth.seed_for(2)).tolist()
    stream = torch.cuda.Stream(dev)
    req = pc.Request([n], pc.FLOAT32, pc.SUM, nparts, P)
    req.bind([xs], [out], stream=stream)
    torch.cuda.synchronize()

    def step():
        req.start()
        for p in order:
            req.pready(p)
        req.wait()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # the timed steps: nothing but the steps (no events: a marker packet
    # costs the stream about 5 us)
    marks = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    step_ms = sorted((b - a) * 1e3 for a, b in zip([t0] + marks[:-1], marks))
    ttr = {"median": round(step_ms[len(step_ms) // 2], 4),
           "mean": round(sum(step_ms) / len(step_ms), 4),
           "p10": round(step_ms[len(step_ms) // 10], 4),
           "p90": round(step_ms[(9 * len(step_ms)) // 10], 4)}
    # the epoch's device time between marker events (start .. readiness),
    # the same steps again with events around them
    evs = [(torch.cuda.Event(enable_timing=True),
            torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for e0, e1 in evs:
        e0.record(stream)
        req.start()
        for p in order:
            req.pready(p)
        e1.record(stream)  # enqueued behind the kernel on its stream
        stream.query()  # submitted now, not at the next look at the stream
        req.wait()
    torch.cuda.synchronize()
    epoch_ms_events = sum(a.elapsed_time(b) for a, b in evs) / args.steps
    # the kernel's own duration: the same steps again with debug timing
    # (start and end stamped by the launch, no instrumentation in the
    # kernel; it costs host time of its own, so `value` is taken without)
    req.set_config(debug=4)
    step()
    st0 = req.stats()
    for _ in range(args.steps):
        step()
    st1 = req.stats()
    timed = st1.kernel_timed - st0.kernel_timed
    kernel_ms = (st1.kernel_ms_total - st0.kernel_ms_total) / timed

    algo = P * n * 4 + n * 4
    value = algo / (ms_per_step * 1e-3) / 1e9
    achieved = algo / (kernel_ms * 1e-3) / 1e9
    cfg = req.config()
    st = req.stats()
    req.free()

    line = {
        "metric": "effective reduce GB/s & % HBM peak; plain FP32 vs batched "
                  "BF16/FP8 at stated err",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: N(0,1) FP32 per rank from a seeded GPU generator",
        "config": {
            "workload": f"partitioned FP32 sum, {P} simulated ranks, "
                        f"{n} elements ({n * 4 >> 20} MiB) per rank, "
                        f"{nparts} partitions readied one by one in a seeded "
                        f"random order",
            "ranks": P, "elements_per_rank": n, "partitions": nparts,
            "tile_elems": cfg.tile_elems, "groups": st.groups,
            "group_waves": cfg.group_waves, "interleave": cfg.interleave,
            "pct_hbm_peak": round(100 * value / HBM_PEAK_GBPS, 2),
            # OMB-style per-rank message rate: one rank's bytes / time
            "per_rank_message_GBps": round(n * 4 / (ms_per_step * 1e-3) / 1e9,
                                           2),
            "time_to_reduce_ms": ttr,
            "cache": "cold by construction: 2.4 GB per step, 9x the "
                     "256 MB MALL",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic_record(algo),
            "kernel_ms": round(kernel_ms, 4),
            "kernel_timing": f"{timed} launches after the timed steps, "
                             "start and end stamped by the launch "
                             "(hipExtLaunchKernel events on the kernel's "
                             "stream)",
            "epoch_ms_events": round(epoch_ms_events, 4),
            "algorithmic_bytes_per_launch": algo,
        },
    }
    if not args.no_cpu_baseline:
        from oracle import get as get_oracle
        line["cpu_baseline"] = cpu_baseline(get_oracle(), xs, P,
                                            args.cpu_seconds)
    del xs, out
    torch.cuda.empty_cache()
    if not args.no_extras:
        line["extras"] = extras(pc, torch, synth, 2, 5)
        ex = line["extras"]
        if "GBps" in ex.get("copy_probe", {}):
            line["config"]["pct_of_copy_probe"] = round(
                100 * value / ex["copy_probe"]["GBps"], 2)
        probes = [v["GBps"] for v in ex.get("stream_probe", {}).values()
                  if isinstance(v, dict) and "GBps" in v]
        if probes:
            # the reduce kernel against the fastest protocol-free stream of
            # its buffers (the same traffic, or its reads alone, in any of
            # the probe's layouts): what the device streams at best
            line["roofline"]["pct_of_attainable"] = round(
                100 * achieved / max(probes), 2)
            line["roofline"]["attainable_GBps"] = max(probes)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
