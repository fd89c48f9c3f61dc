"""Exhaustive launch-parameter search for libpcoll on the local GPU.

Section 4.4 of the paper tunes scheduling parameters offline by exhaustive
search and uses the results as defaults (environment variables override
them), tuning graph and non-graph execution separately.  This tool does the
same for the persistent reduce kernel: for each tuning key (dtype, op,
ranks, graph mode, floor(log2(bytes per rank))) it times every
(tile_elems, groups_per_cu, interleave, waves per workgroup, publish batch,
rows in flight per lane) combination of its grid on seeded synthetic
inputs and writes the fastest into the text table the library reads at
request creation (tuned_mi355x.txt next to libpcoll.so, or
PCOLL_TUNE_FILE).  Rows of one (dtype, op, ranks, graph) cover contiguous
size ranges: each key's row reaches down to the next smaller key's.  The
batched workloads are tuned for direct launches and for graph replays
apart; a graph row is written before the direct one, whose graph column is
"*" (it also serves graph replays of keys without a graph row of their
own).

Timing: median device time of `reps` epochs (HIP events on the bound
stream around start and the readiness call, submitted at once), every
partition readied at once in a seeded random order, after `warmup` epochs;
for the FP32 sweep keys, the mean of that over the sweep's partition
counts 1, 4, 16 and 64 (the table keys on size alone: at each size from
64 MiB per rank on, the four partition counts take times within 1 % of
each other).  Run on the target GPU:

    python -m paper_2604_22228_amd.autotune --out paper_2604_22228_amd/tuned_mi355x.txt
"""
import argparse
import itertools
import json
import math
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DTYPE_NAMES = {0: "i32", 1: "f32", 2: "bf16", 3: "e4m3", 4: "e5m2",
               5: "mxfp8", 6: "bf16pair"}
OP_NAMES = {0: "sum", 1: "max"}

TILES = (4096, 8192, 16384, 32768)
GROUPS_PER_CU = (1, 2)
# tile layout: bands of one launch's worth of tiles, or of 4, 8, 16 tiles
INTERLEAVE = (1, 4, 8, 16)
WAVES = (4, 8)
# finished tiles a workgroup publishes together: larger is faster all the
# way (publish batch 8 / 16 / 32 / 64: headline kernel 0.424 / 0.400 /
# 0.388 / 0.380 ms, batched bf16 1.181 / 1.082 / 0.999 / 0.964 ms), and 64
# is the most one wave-wide atomic instruction publishes, so it is not
# searched
BATCH = (64,)
# rows in flight per lane in the 16-byte-vector kernels from 3 ranks on (4
# or 2 up to 8 ranks, 2 or 1 above; the 8-bit kernels load one row per lane
# at a time)
UNROLL = (2, 4)
# 8-bit payloads: the kernels are bound by instruction issue and hide
# memory latency with more resident waves and longer tiles
TILES_8BIT = (16384, 32768, 65536)
GROUPS_PER_CU_8BIT = (2, 3)
# consecutive rows per tile too: the rows that share a line of block
# scales are then read by one workgroup
INTERLEAVE_8BIT = (0, 1, 4, 8, 16)
FALLBACK = "* * * * 0 63 8192 1 16 8 64 4"


def grid_for(dtype, ranks=8):
    if dtype in (3, 4, 5):
        return [TILES_8BIT, GROUPS_PER_CU_8BIT, INTERLEAVE_8BIT, WAVES, BATCH,
                (4,)]
    return [TILES, GROUPS_PER_CU, INTERLEAVE, WAVES, BATCH,
            UNROLL if ranks >= 3 else (4,)]


def default_keys():
    """The configurations of the five workloads: (dtype, op, ranks, graph,
    list of per-bucket element counts, partitions per bucket, or a tuple of
    partition counts whose mean time is scored)."""
    from paper_2604_22228_amd import synth
    keys = []
    for k in range(10, 27, 2):  # the FP32 sweep, 4 KiB .. 256 MiB per rank
        keys.append((1, 0, 8, 0, [1 << k], (1, 4, 16, 64)))
    keys.append((1, 0, 4, 0, [262144], 8))          # plain workload
    keys.append((0, 0, 16, 0, [1 << 24], 256))      # int32 sum
    keys.append((0, 1, 16, 0, [1 << 24], 256))      # int32 max
    # the batched workloads, direct launches and graph replays
    for graph in (0, 1):
        keys.append((2, 0, 8, graph, list(synth.batched_bf16_counts()), 32))
        keys.append((6, 0, 8, graph, list(synth.batched_bf16_counts()), 32))
        keys.append((3, 0, 8, graph, list(synth.fp8_bucket_counts()), 32))
        keys.append((4, 0, 8, graph, list(synth.fp8_bucket_counts()), 32))
        keys.append((5, 0, 8, graph, list(synth.fp8_bucket_counts()), 32))
    return keys


def time_config(pc, torch, synth, dtype, op, ranks, graph, counts, nparts,
                choice, warmup, reps, bufs):
    tile, gpc, inter, waves, batch, unroll = choice
    req = pc.Request(counts, dtype, op, nparts, ranks,
                     batched=len(counts) > 1)
    req.set_config(tile_elems=tile, min_tile_elems=min(tile, 4096),
                   groups_per_cu=gpc, graph=graph, groups=0,
                   interleave=inter, guide=0, group_waves=waves,
                   publish_batch=batch, unroll=unroll, producers=0)
    ins, outs, rsc, osc, stream = bufs
    req.bind(ins, outs, rsc, osc, stream=stream)
    order = synth.permutation(req.nparts_total, 1).astype("int32")
    times = []
    for it in range(warmup + reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        req.start()
        req.pready_list(order)
        e1.record(stream)
        stream.query()  # the runtime may hold the record back until then
        req.wait()
        if it >= warmup:
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
    req.free()
    return statistics.median(times)


def make_buffers(pc, torch, synth, dtype, ranks, counts):
    dev = torch.device("cuda:0")
    tdt = {0: torch.int32, 1: torch.float32, 2: torch.int16,
           3: torch.uint8, 4: torch.uint8, 5: torch.uint8,
           6: torch.int16}[dtype]
    ins, outs, rsc, osc = [], [], None, None
    if dtype in (3, 4, 5):
        rsc, osc = [], []
    elif dtype == 6:  # the low halves of the bf16 pairs
        osc = []
    pack8 = {3: pc.pcoll_pack_fp8, 4: pc.pcoll_pack_e5m2,
             5: pc.pcoll_pack_mxfp8}.get(dtype)
    # scale blocks: binary32 per 256 elements, or E8M0 bytes per 32
    blk, sdt = (32, torch.uint8) if dtype == 5 else (256, torch.float32)
    for b, c in enumerate(counts):
        m = max(c, 16)
        if dtype == 0:
            bucket = synth.uniform_i32(ranks, m, 10 + b, -(1 << 20), 1 << 20,
                                       device=dev)
        else:
            x = synth.normal_f32(ranks, m, 10 + b, device=dev)
            if dtype == 1:
                bucket = x
            elif dtype in (2, 6):
                bucket = []
                for t in x:
                    o = torch.empty(m, dtype=torch.int16, device=dev)
                    pc.pcoll_pack_bf16(t, o, m, torch.cuda.current_stream())
                    bucket.append(o)
            else:
                bucket, scales = [], []
                for t in x:
                    q = torch.empty(m, dtype=torch.uint8, device=dev)
                    s = torch.empty((m + blk - 1) // blk, dtype=sdt,
                                    device=dev)
                    pack8(t, q, s, m, torch.cuda.current_stream())
                    bucket.append(q)
                    scales.append(s)
                rsc.append(scales)
                osc.append(torch.empty((m + blk - 1) // blk, dtype=sdt,
                                       device=dev))
        ins.append(bucket)
        outs.append(torch.empty(m, dtype=tdt, device=dev))
        if dtype == 6:
            osc.append(torch.empty(m, dtype=tdt, device=dev))
    torch.cuda.synchronize()
    return ins, outs, rsc, osc, torch.cuda.Stream(dev)


def tune(keys, grid, warmup, reps, log=print):
    """grid: the search grid, or None for each key's dtype's grid."""
    import torch

    from paper_2604_22228_amd import pcoll as pc
    from paper_2604_22228_amd import synth

    rows = []
    for dtype, op, ranks, graph, counts, nparts in keys:
        bufs = make_buffers(pc, torch, synth, dtype, ranks, counts)
        nbytes = sum(counts) * pc.ELEM_BYTES[dtype]
        lg = int(math.floor(math.log2(max(nbytes, 1))))
        best = None
        parts_list = nparts if isinstance(nparts, tuple) else (nparts,)
        for choice in itertools.product(*(grid or grid_for(dtype, ranks))):
            ms = statistics.mean(
                time_config(pc, torch, synth, dtype, op, ranks, graph,
                            counts, np_, choice, warmup, reps, bufs)
                for np_ in parts_list)
            log(json.dumps({"dtype": DTYPE_NAMES[dtype],
                            "op": OP_NAMES[op], "ranks": ranks,
                            "graph": graph, "log2_bytes": lg,
                            "tile": choice[0], "gpc": choice[1],
                            "interleave": choice[2], "waves": choice[3],
                            "batch": choice[4], "unroll": choice[5],
                            "ms": round(ms, 5)}))
            if best is None or ms < best[0]:
                best = (ms, choice)
        # a direct launch's row also serves graph replays of keys tuned
        # for direct launches only
        rows.append((DTYPE_NAMES[dtype], OP_NAMES[op], ranks,
                     "1" if graph else "*", lg, best[1], best[0]))
        del bufs
        torch.cuda.empty_cache()
    return rows


def read_table(path):
    """The rows of an existing table (fallback excluded), in the form
    tune() returns them, so that a partial run can keep the other keys."""
    rows = []
    with open(path) as f:
        for line in f:
            body, _, note = line.partition("#")
            v = body.split()
            if len(v) not in (11, 12) or v[0] == "*":
                continue
            lg = int(note.split("2^")[1].split()[0])
            ms = float(note.split()[0])
            choice = tuple(int(x) for x in v[6:]) + ((4,) if len(v) == 11
                                                      else ())
            rows.append((v[0], v[1], int(v[2]), v[3], lg, choice, ms))
    return rows


def write_table(rows, path):
    """One line per key; the keys of one (dtype, op, ranks, graph) cover
    contiguous ranges of log2(bytes per rank), the largest up to 63."""
    groups = {}
    for r in rows:
        groups.setdefault(r[:4], []).append(r)
    lines = ["# Tuned launch parameters of libpcoll on MI355X (gfx950), "
             "written by paper_2604_22228_amd/autotune.py.",
             "# dtype op ranks graph log2_lo log2_hi tile_elems "
             "groups_per_cu interleave waves batch unroll   # median kernel ms"]
    # graph rows first: the first matching row wins, and a direct row
    # ("*") also serves graph replays
    keys = sorted(groups, key=lambda k: 0 if k[3] == "1" else 1)
    keys = sorted(keys, key=lambda k: [kk[:3] for kk in groups].index(k[:3]))
    for key in keys:
        rs = sorted(groups[key], key=lambda r: r[4])
        lo = 0
        for i, (d, o, rk, g, lg, (t, gpc, il, w, b, u), ms) in enumerate(rs):
            hi = 63 if i == len(rs) - 1 else lg
            lines.append(f"{d} {o} {rk} {g} {lo} {hi} {t} {gpc} {il} {w} {b}"
                         f" {u}   # {ms:.4f} at 2^{lg} B")
            lo = hi + 1
    lines.append(FALLBACK + "   # fallback")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(
        os.path.dirname(os.path.abspath(__file__)), "tuned_mi355x.txt"))
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--reps", type=int, default=7)
    ap.add_argument("--quick", action="store_true",
                    help="a reduced grid (for a smoke run)")
    ap.add_argument("--only", default="",
                    help="comma-separated dtypes (f32, bf16, e4m3, ...) to "
                         "tune; the other rows of --out are kept")
    ap.add_argument("--graph", choices=("0", "1", "both"), default="both",
                    help="launch modes of the batched keys to tune")
    args = ap.parse_args()
    keys = default_keys()
    if args.graph != "both":
        keys = [k for k in keys if k[3] == int(args.graph)]
    grid = None
    if args.quick:
        keys, grid = keys[-10:-8], [(16384, 65536), (1,), (1,), (4,), (64,),
                                    (4,)]
    kept = []
    if args.only:
        only = set(args.only.split(","))
        keys = [k for k in keys if DTYPE_NAMES[k[0]] in only]
        tuned = {(DTYPE_NAMES[k[0]], "1" if k[3] else "*") for k in keys}
        kept = [r for r in read_table(args.out) if (r[0], r[3]) not in tuned]
    rows = tune(keys, grid, args.warmup, args.reps,
                log=lambda s: print(s, flush=True))
    order = [DTYPE_NAMES[k[0]] + OP_NAMES[k[1]] + str(k[2])
             for k in default_keys()]
    rows = sorted(kept + rows, key=lambda r: (order.index(
        r[0] + r[1] + str(r[2])), r[3] != "1", r[4]))
    write_table(rows, args.out)
    print(f"wrote {args.out} ({len(rows)} rows)", flush=True)


if __name__ == "__main__":
    main()
