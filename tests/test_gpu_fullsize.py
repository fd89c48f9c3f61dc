"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times (library defaults), on sampled outputs the oracle computes
one by one (fp32, bf16: sampled elements; e4m3: sampled whole 256-element
blocks, since a code depends on its block's scale; int32: everything).
Error statistics against the FP64 reference are printed for the record."""
import json

import numpy as np
import pytest
import torch

from _gpu import DEV, as_u32, say
from _metrics import error_report, normalized_error
from oracle import get as get_oracle
from paper_2604_22228_amd import pcoll as pc
from paper_2604_22228_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    return get_oracle()


def _sample_idx(n, k, seed, extra=()):
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, n, size=min(k, n)) if n else np.zeros(0, np.int64)
    idx = np.unique(np.concatenate([idx, np.asarray(extra, np.int64)]))
    return idx[(idx >= 0) & (idx < n)]


def _gather(ts, idx):
    di = torch.from_numpy(idx).to(DEV)
    return [t.index_select(0, di).cpu().numpy() for t in ts]


def _run(req, nparts_total, seed, stream):
    req.start()
    req.pready_list(synth.permutation(nparts_total, seed).astype("int32"))
    req.wait()
    torch.cuda.synchronize()


def test_headline_fp32_p8_256MiB(orc):
    """The benchmark's workload: 8 ranks, 2^26 elements, 64 partitions, a
    seeded random arrival order, default launch configuration."""
    P, n, nparts = 8, 1 << 26, 64
    say(f"case headline fp32 P={P} n={n}")
    stream = torch.cuda.Stream(DEV)
    xs = synth.normal_f32(P, n, synth.seed_for(2), device=DEV)
    out = torch.full((n,), float("nan"), device=DEV)
    req = pc.Request([n], pc.FLOAT32, pc.SUM, nparts, P)
    req.bind([xs], [out], stream=stream)
    for epoch in range(2):
        out.fill_(float("nan"))
        req.start()
        for p in synth.permutation(nparts, synth.seed_for(2)):
            req.pready(int(p))
        req.wait()
        torch.cuda.synchronize()
        ps = n // nparts
        bounds = [k * ps for k in range(nparts)] + \
                 [k * ps - 1 for k in range(1, nparts + 1)]
        idx = _sample_idx(n, 200000, epoch, bounds)
        xsam = _gather(xs, idx)
        got = out.index_select(0, torch.from_numpy(idx).to(DEV)).cpu().numpy()
        want = orc.sum_f32_f32(xsam)
        assert np.array_equal(as_u32(got), as_u32(want))
        assert not torch.isnan(out).any().item()  # every element written
        y64 = orc.sum_f32_f64(xsam)
        absum = np.abs(np.stack(xsam)).astype(np.float64).sum(axis=0)
        rep = error_report(got, y64, absum)
        say("errors " + json.dumps({"workload": "headline fp32", **rep}))
        assert rep["max_norm_err"] <= 1e-6
    req.free()


def test_sweep_points_fp32_p8(orc):
    """The size sweep's grid (4 B .. 64 MiB per rank here; 256 MiB is the
    headline test) x partition counts {1, 4, 16, 64}, seeded arrival."""
    P = 8
    stream = torch.cuda.Stream(DEV)
    big = synth.normal_f32(P, 1 << 24, synth.seed_for(2) + 1, device=DEV)
    for k in range(0, 25, 3):
        n = 1 << k
        xs = [b[:n] for b in big]
        for nparts in (1, 4, 16, 64):
            say(f"case sweep n=2^{k} nparts={nparts}")
            out = torch.full((max(n, 4),), float("nan"), device=DEV)
            req = pc.Request([n], pc.FLOAT32, pc.SUM, nparts, P)
            req.bind([xs], [out], stream=stream)
            _run(req, nparts, k * 100 + nparts, stream)
            idx = _sample_idx(n, 50000, k, [0, n - 1])
            got = out[:n].index_select(0, torch.from_numpy(idx).to(DEV)) \
                .cpu().numpy()
            want = orc.sum_f32_f32(_gather(xs, idx))
            assert np.array_equal(as_u32(got), as_u32(want)), (k, nparts)
            req.free()


def test_workload4_int32_full(orc):
    P, n, nparts = 16, 1 << 24, 256
    stream = torch.cuda.Stream(DEV)
    xs = synth.uniform_i32(P, n, synth.seed_for(4), -(1 << 20), 1 << 20,
                           device=DEV)
    host = [x.cpu().numpy() for x in xs]
    for op in (pc.SUM, pc.MAX):
        say(f"case int32 full op={op}")
        out = torch.full((n,), 0x5A5A5A5A, dtype=torch.int32, device=DEV)
        req = pc.Request([n], pc.INT32, op, nparts, P)
        req.bind([xs], [out], stream=stream)
        _run(req, nparts, synth.seed_for(4), stream)
        got = out.cpu().numpy()
        want = orc.sum_i32(host) if op == pc.SUM else orc.max_i32(host)
        assert np.array_equal(got, want)
        req.free()


@pytest.mark.parametrize("graph", [0, 1])
def test_workload3_batched_bf16_full(orc, graph):
    counts = synth.batched_bf16_counts()
    P, nparts = 8, 32
    say(f"case batched bf16 full buckets={len(counts)} "
        f"elements/rank={sum(counts)} graph={graph}")
    stream = torch.cuda.Stream(DEV)
    cur = torch.cuda.current_stream(DEV)
    pays, outs = [], []
    for b, c in enumerate(counts):
        row = []
        for t in synth.normal_f32(P, c, synth.seed_for(3) * 1000 + b,
                                  std=1e-3, device=DEV):
            o = torch.empty(c, dtype=torch.int16, device=DEV)
            pc.pcoll_pack_bf16(t, o, c, cur)
            row.append(o)
        pays.append(row)
        outs.append(torch.full((c,), 0x7FC0, dtype=torch.int16, device=DEV))
    torch.cuda.synchronize()
    req = pc.Request(counts, pc.BFLOAT16, pc.SUM, nparts, P, batched=True)
    if graph:
        req.set_config(graph=1)
    assert req.config().graph == graph
    req.bind(pays, outs, stream=stream)
    _run(req, len(counts) * nparts, 3, stream)
    errs = []
    for b, c in enumerate(counts):
        idx = _sample_idx(c, 4096, b, [0, c - 1])
        sam = [s.view(np.uint16) for s in _gather(pays[b], idx)]
        got = outs[b].index_select(0, torch.from_numpy(idx).to(DEV)).cpu() \
            .numpy().view(np.uint16)
        want, _ = orc.sum_bf16_f32(sam, comp=req.config().comp == 1)
        assert np.array_equal(got, want), b
        y64 = orc.sum_bf16_f64(sam)
        dec = np.stack([torch.from_numpy(s.view(np.int16))
                        .view(torch.bfloat16).double().numpy() for s in sam])
        gv = torch.from_numpy(got.view(np.int16)).view(torch.bfloat16) \
            .double().numpy()
        errs.append(normalized_error(gv, y64, np.abs(dec).sum(axis=0)).max())
    say("errors " + json.dumps({"workload": "batched bf16",
                                "max_norm_err": float(max(errs))}))
    assert max(errs) <= 4e-3
    assert req.stats().graph_launches == graph
    req.free()


def test_workload5_fp8_full(orc):
    counts = synth.fp8_bucket_counts()
    P, nparts = 8, 32
    say(f"case fp8 full buckets={len(counts)} elements/rank={sum(counts)}")
    stream = torch.cuda.Stream(DEV)
    cur = torch.cuda.current_stream(DEV)
    qs, ss, oq, osc = [], [], [], []
    for b, c in enumerate(counts):
        qrow, srow = [], []
        for t in synth.normal_with_outliers_f32(
                P, c, synth.seed_for(5) * 1000 + b, 1e-2, device=DEV):
            q = torch.empty(c, dtype=torch.uint8, device=DEV)
            s = torch.empty((c + 255) // 256, dtype=torch.float32, device=DEV)
            pc.pcoll_pack_fp8(t, q, s, c, cur)
            qrow.append(q)
            srow.append(s)
        qs.append(qrow)
        ss.append(srow)
        oq.append(torch.full((c,), 0x7F, dtype=torch.uint8, device=DEV))
        osc.append(torch.full(((c + 255) // 256,), float("nan"), device=DEV))
    torch.cuda.synchronize()
    req = pc.Request(counts, pc.FP8_E4M3, pc.SUM, nparts, P, batched=True)
    req.bind(qs, oq, ss, osc, stream=stream)
    assert req.config().comp == 1
    _run(req, len(counts) * nparts, 5, stream)
    table = orc.e4m3_decode_table()
    worst = 0.0
    for b, c in enumerate(counts):
        nb = (c + 255) // 256
        blocks = _sample_idx(nb, 16, b, [0, nb - 1])
        idx = np.concatenate([np.arange(k * 256, min(c, k * 256 + 256))
                              for k in blocks])
        qsam = _gather(qs[b], idx)
        ssam = _gather(ss[b], blocks)
        # re-index the sampled blocks as consecutive blocks 0..len-1
        gq = oq[b].index_select(0, torch.from_numpy(idx).to(DEV)).cpu().numpy()
        gs = osc[b].index_select(0, torch.from_numpy(blocks).to(DEV)).cpu() \
            .numpy()
        wq, ws, _ = orc.sum_e4m3_f32(qsam, ssam, comp=True)
        assert np.array_equal(gq, wq), b
        assert np.array_equal(as_u32(gs), as_u32(ws)), b
        y64 = orc.sum_e4m3_f64(qsam, ssam)
        rep = lambda s: np.repeat(s.astype(np.float64), 256)[:len(idx)]  # noqa
        deq = np.stack([table[q] * rep(s) for q, s in zip(qsam, ssam)])
        yv = table[gq] * rep(gs)
        e = np.abs(yv - y64) / np.maximum(np.abs(deq).sum(axis=0),
                                          rep(gs) * 2.0 ** -6)
        worst = max(worst, float(e.max()))
    say("errors " + json.dumps({"workload": "fp8 batched",
                                "max_norm_err": worst}))
    assert worst <= 6e-2
    req.free()


def test_workload5_mx_full(orc):
    """The fp8 workload's shape (8 ranks, 128 buckets, 2^30 elements per
    rank, N(0, 1e-2) with 1% outliers at 50x) as MX blocks, at library
    defaults; sampled whole 32-element blocks against the oracle."""
    counts = synth.fp8_bucket_counts()
    P, nparts = 8, 32
    say(f"case mx full buckets={len(counts)} elements/rank={sum(counts)}")
    stream = torch.cuda.Stream(DEV)
    cur = torch.cuda.current_stream(DEV)
    qs, ss, oq, osb = [], [], [], []
    for b, c in enumerate(counts):
        qrow, srow = [], []
        for t in synth.normal_with_outliers_f32(
                P, c, synth.seed_for(5) * 1000 + b, 1e-2, device=DEV):
            q = torch.empty(c, dtype=torch.uint8, device=DEV)
            s = torch.empty((c + 31) // 32, dtype=torch.uint8, device=DEV)
            pc.pcoll_pack_mxfp8(t, q, s, c, cur)
            qrow.append(q)
            srow.append(s)
        qs.append(qrow)
        ss.append(srow)
        oq.append(torch.full((c,), 0x7F, dtype=torch.uint8, device=DEV))
        osb.append(torch.full(((c + 31) // 32,), 0xFF, dtype=torch.uint8,
                              device=DEV))
    torch.cuda.synchronize()
    req = pc.Request(counts, pc.MXFP8_E4M3, pc.SUM, nparts, P, batched=True)
    req.bind(qs, oq, ss, osb, stream=stream)
    assert req.config().comp == 1
    _run(req, len(counts) * nparts, 5, stream)
    worst = 0.0
    for b, c in enumerate(counts):
        nb = (c + 31) // 32
        blocks = _sample_idx(nb, 64, b, [0, nb - 1])
        idx = np.concatenate([np.arange(k * 32, min(c, k * 32 + 32))
                              for k in blocks])
        qsam = _gather(qs[b], idx)
        ssam = _gather(ss[b], blocks)
        gq = oq[b].index_select(0, torch.from_numpy(idx).to(DEV)).cpu().numpy()
        gs = osb[b].index_select(0, torch.from_numpy(blocks).to(DEV)).cpu() \
            .numpy()
        wq, ws, _ = orc.sum_mx_f32(qsam, ssam, comp=True)
        assert np.array_equal(gq, wq), b
        assert np.array_equal(gs, ws), b
        y64 = orc.sum_mx_f64(qsam, ssam)
        absum = np.abs(np.stack([orc.mx_dequant(q, s) for q, s in
                                 zip(qsam, ssam)])).sum(axis=0)
        X = np.repeat(2.0 ** (gs.astype(np.float64) - 127), 32)[:len(idx)]
        e = np.abs(orc.mx_dequant(gq, gs) - y64) / np.maximum(absum,
                                                              X * 2.0 ** -6)
        worst = max(worst, float(e.max()))
    say("errors " + json.dumps({"workload": "mx batched",
                                "max_norm_err": worst}))
    assert worst <= 6e-2
    req.free()
