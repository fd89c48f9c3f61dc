"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar: integer results and every encoded output (fp32 bits with the plain
left-to-right order, bf16 / e4m3 codes, e4m3 scales) bit-exact against the
oracle's mirror of the kernel's binary32 arithmetic; floating-point results
within the Sigma|x|-normalized tolerance against the FP64 reference (1e-6
fp32, 4e-3 bf16, 6e-2 e4m3).  Inputs come from the seeded generators."""
import itertools
import time

import numpy as np
import pytest
import torch

from _gpu import DEV, TEST_TIMEOUT_MS, as_u32, new_request, pack_bf16_gpu, \
    pack_fp8_gpu, run_epoch, say
from _metrics import normalized_error
from oracle import get as get_oracle
from paper_2604_22228_amd import pcoll as pc
from paper_2604_22228_amd import synth
from paper_2604_22228_amd.streams import independent_streams

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    return get_oracle()


@pytest.fixture(scope="module")
def stream():
    assert torch.cuda.is_available()
    pc.load()
    return torch.cuda.current_stream(DEV)


def _f32_case(orc, stream, P, n, nparts, seed, comp, order="random",
              **cfg):
    say(f"case fp32 sum P={P} n={n} nparts={nparts} seed={seed} comp={comp} "
        f"cfg={cfg}")
    xs = synth.normal_f32(P, n, seed)
    dx = [x.to(DEV) for x in xs]
    out = torch.full((max(n, 4),), float("nan"), device=DEV)
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P, comp=int(comp),
                      **cfg)
    req.bind([dx], [out], stream=stream)
    perm = synth.permutation(nparts, seed) if order == "random" \
        else np.arange(nparts)
    run_epoch(req, perm, stream)
    got = out[:n].cpu().numpy()
    req.free()
    xn = [x.numpy() for x in xs]
    want = orc.sum_f32_f32(xn, comp=comp)
    mism = int(np.count_nonzero(as_u32(got) != as_u32(want)))
    assert mism == 0, f"{mism} of {n} elements differ from the oracle"
    if n:
        y64 = orc.sum_f32_f64(xn)
        absum = np.abs(np.stack(xn)).astype(np.float64).sum(axis=0)
        assert normalized_error(got, y64, absum).max() <= 1e-6


@pytest.mark.parametrize("P", [1, 2, 3, 4, 8, 16])
def test_fp32_sum_small_grid(orc, stream, P):
    for n in (0, 1, 3, 4, 5, 1023, 1024, 4097, 65536 + 13):
        for nparts in (1, 3, 8):
            _f32_case(orc, stream, P, n, nparts, seed=1000 + n + P,
                      comp=False, tile_elems=1024)


@pytest.mark.parametrize("P", [2, 8, 16])
def test_fp32_sum2_small_grid(orc, stream, P):
    for n in (1, 7, 4096 + 5, 50001):
        _f32_case(orc, stream, P, n, 5, seed=2000 + n + P, comp=True,
                  tile_elems=2048)


@pytest.mark.parametrize("band", [0, 1, 2, 3, 8, 1 << 20])
def test_tile_layouts(orc, stream, band):
    """Consecutive tiles (0) and interleaved bands of the launch's width
    (1) or of 2, 3, 8 and more tiles than exist, with partitions of many
    tiles and a ragged end: bitwise against the oracle."""
    _f32_case(orc, stream, 3, 300 * 1024 + 77, 3, 90 + band % 97, False,
              tile_elems=1024, min_tile_elems=1024, interleave=band)


def test_workload1_plain_fp32(orc, stream):
    """4 ranks, FP32 sum, 262144 elements per rank, 8 partitions readied in
    order, uniform [-1, 1) inputs."""
    P, n, nparts = 4, 262144, 8
    say(f"case workload-1 P={P} n={n}")
    xs = synth.uniform_f32(P, n, synth.seed_for(1))
    dx = [x.to(DEV) for x in xs]
    out = torch.full((n,), float("nan"), device=DEV)
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P)
    req.bind([dx], [out], stream=stream)
    for epoch in range(3):
        out.fill_(float("nan"))
        run_epoch(req, range(nparts), stream)
        got = out.cpu().numpy()
        want = orc.sum_f32_f32([x.numpy() for x in xs])
        assert np.array_equal(as_u32(got), as_u32(want)), f"epoch {epoch}"
    req.free()


def test_all_arrival_orders_give_identical_bits(orc, stream):
    P, n, nparts = 3, 5 * 1024 + 17, 5
    say(f"case all orders P={P} n={n} nparts={nparts}")
    xs = synth.normal_f32(P, n, 31)
    dx = [x.to(DEV) for x in xs]
    out = torch.empty(n, device=DEV)
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P, tile_elems=1024)
    req.bind([dx], [out], stream=stream)
    want = as_u32(orc.sum_f32_f32([x.numpy() for x in xs]))
    for perm in itertools.permutations(range(nparts)):
        out.fill_(float("nan"))
        req.start()
        readied = set()
        for p in perm:
            # never arrived before it is readied (Section 4.5)
            for q in range(nparts):
                if q not in readied:
                    assert not req.parrived(q), (perm, q)
            req.pready(p)
            readied.add(p)
        req.wait()
        assert all(req.parrived(q) for q in range(nparts))
        torch.cuda.synchronize()
        assert np.array_equal(as_u32(out.cpu().numpy()), want), perm
    req.free()


def test_partitions_arrive_before_the_epoch_ends(orc, stream):
    """Readied partitions arrive by their own flags while later ones are
    still unready (so the kernel cannot have retired), even with the
    largest publish batch, and their output is final when the flag is seen:
    a second stream reads it while the kernel still runs."""
    P, n, nparts = 4, 256 * 1024 + 40, 8
    say(f"case early arrival P={P} n={n} nparts={nparts}")
    xs = synth.normal_f32(P, n, 41)
    out = torch.full((n,), float("nan"), device=DEV)
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P, tile_elems=4096,
                      publish_batch=64)
    req.bind([[x.to(DEV) for x in xs]], [out], stream=stream)
    want = as_u32(orc.sum_f32_f32([x.numpy() for x in xs]))
    side = independent_streams(stream, 1)[0]  # runs beside the kernel
    first = [5, 0, 3, 6]
    req.start()
    req.pready_list(first)
    t0 = time.monotonic()
    while not all(req.parrived(p) for p in first):
        assert time.monotonic() - t0 < 2.0, "readied partitions never arrived"
    assert not any(req.parrived(p) for p in range(nparts) if p not in first)
    snaps = []
    with torch.cuda.stream(side):
        for p in first:
            _, off, ln = req.part_info(p)
            snaps.append((off, ln, out[off:off + ln].clone()))
    done = torch.cuda.Event()
    done.record(side)
    t0 = time.monotonic()
    while not done.query() and time.monotonic() - t0 < 2.0:
        pass
    concurrent = done.query()
    req.pready_list([p for p in range(nparts) if p not in first])
    req.wait()
    torch.cuda.synchronize()
    say(f"snapshot taken while the kernel ran: {concurrent}")
    assert concurrent
    for off, ln, snap in snaps:
        assert np.array_equal(as_u32(snap.cpu().numpy()), want[off:off + ln])
    assert np.array_equal(as_u32(out.cpu().numpy()), want)
    assert all(req.parrived(p) for p in range(nparts))
    req.free()


@pytest.mark.parametrize("op", [pc.SUM, pc.MAX])
def test_int32_bit_exact(orc, stream, op):
    P, n, nparts = 16, (1 << 20) + 3, 256
    say(f"case int32 op={op} P={P} n={n}")
    xs = synth.uniform_i32(P, n, synth.seed_for(4), -(1 << 20), 1 << 20)
    dx = [x.to(DEV) for x in xs]
    out = torch.full((n,), 0x5A5A5A5A, dtype=torch.int32, device=DEV)
    req = new_request([n], pc.INT32, op, nparts, P)
    req.bind([dx], [out], stream=stream)
    run_epoch(req, synth.permutation(nparts, synth.seed_for(4)), stream)
    got = out.cpu().numpy()
    req.free()
    xn = [x.numpy() for x in xs]
    want = orc.sum_i32(xn) if op == pc.SUM else orc.max_i32(xn)
    assert np.array_equal(got, want)


def test_int32_wraps(orc, stream):
    n = 1000
    a = torch.full((n,), 2**31 - 1, dtype=torch.int32)
    b = torch.arange(n, dtype=torch.int32)
    out = torch.empty(n, dtype=torch.int32, device=DEV)
    req = new_request([n], pc.INT32, pc.SUM, 2, 2)
    req.bind([[a.to(DEV), b.to(DEV)]], [out], stream=stream)
    run_epoch(req, [1, 0], stream)
    got = out.cpu().numpy()
    req.free()
    assert np.array_equal(got, orc.sum_i32([a.numpy(), b.numpy()]))


def test_fp32_max(orc, stream):
    P, n = 5, 40000 + 3
    xs = synth.normal_f32(P, n, 77)
    out = torch.empty(n, device=DEV)
    req = new_request([n], pc.FLOAT32, pc.MAX, 4, P, tile_elems=4096)
    req.bind([[x.to(DEV) for x in xs]], [out], stream=stream)
    run_epoch(req, [3, 1, 0, 2], stream)
    got = out.cpu().numpy()
    req.free()
    assert np.array_equal(as_u32(got), as_u32(orc.max_f32([x.numpy()
                                                           for x in xs])))


# ---------------------------------------------------------------- bfloat16
def test_pack_bf16_matches_oracle_encoding(orc, stream):
    n = 100003
    x = synth.normal_f32(1, n, 5)[0] * torch.exp(
        torch.empty(n).uniform_(-60, 60, generator=torch.Generator()
                                .manual_seed(5)))
    got = pack_bf16_gpu(x.to(DEV)).cpu().numpy().view(np.uint16)
    want = orc.bf16_encode_array(x.numpy())
    assert np.array_equal(got, want)


@pytest.mark.parametrize("comp", [False, True])
@pytest.mark.parametrize("op", [pc.SUM, pc.MAX])
def test_bf16_reduce(orc, stream, comp, op):
    if op == pc.MAX and comp:
        pytest.skip("compensation applies to sums only")
    P, n, nparts = 8, 300007, 32
    say(f"case bf16 op={op} comp={comp} P={P} n={n}")
    xs = synth.normal_f32(P, n, synth.seed_for(3), std=1e-3)
    payload = [pack_bf16_gpu(x.to(DEV)) for x in xs]
    opay = [orc.bf16_encode_array(x.numpy()) for x in xs]
    for g, o in zip(payload, opay):
        assert np.array_equal(g.cpu().numpy().view(np.uint16), o)
    out = torch.full((n,), 0x7FC0, dtype=torch.int16, device=DEV)
    req = new_request([n], pc.BFLOAT16, op, nparts, P,
                      comp=int(comp and op == pc.SUM))
    req.bind([payload], [out], stream=stream)
    run_epoch(req, synth.permutation(nparts, 3), stream)
    got = out.cpu().numpy().view(np.uint16)
    req.free()
    if op == pc.MAX:
        assert np.array_equal(got, orc.max_bf16(opay))
        return
    want, _ = orc.sum_bf16_f32(opay, comp=comp)
    assert np.array_equal(got, want)
    y64 = orc.sum_bf16_f64(opay)
    dec = np.stack([torch.from_numpy(o.view(np.int16)).view(torch.bfloat16)
                    .to(torch.float64).numpy() for o in opay])
    gv = torch.from_numpy(got.view(np.int16)).view(torch.bfloat16) \
        .to(torch.float64).numpy()
    assert normalized_error(gv, y64, np.abs(dec).sum(axis=0)).max() <= 4e-3


# -------------------------------------------------------------------- e4m3
def test_pack_fp8_matches_oracle(orc, stream):
    n = 256 * 300 + 77
    x = synth.normal_with_outliers_f32(1, n, synth.seed_for(5), 1e-2)[0]
    q, s = pack_fp8_gpu(x.to(DEV))
    oq, os_ = orc.e4m3_pack(x.numpy())
    assert np.array_equal(q[:n].cpu().numpy(), oq)
    assert np.array_equal(as_u32(s.cpu().numpy()), as_u32(os_))


@pytest.mark.parametrize("comp", [False, True])
def test_fp8_identity_covers_every_code(orc, stream, comp):
    """P = 1 over blocks holding all 254 finite codes: decode and encode in
    the kernel must reproduce every code and the scale.  Sum2 returns
    p + sigma with sigma starting at +0, so it maps -0 to +0 (a value-equal
    code); plain accumulation keeps every bit."""
    codes = np.array([c for c in range(256) if c not in (0x7F, 0xFF)] +
                     [0, 0], dtype=np.uint8)
    n = 256 * 3
    q = np.concatenate([codes, codes[::-1], np.roll(codes, 7)])
    sc = np.array([1.0, 0.5, 3.0], dtype=np.float32)
    dq = torch.from_numpy(q).to(DEV)
    ds = torch.from_numpy(sc).to(DEV)
    oq = torch.full((n,), 0x7F, dtype=torch.uint8, device=DEV)
    osc = torch.zeros(3, device=DEV)
    req = new_request([n], pc.FP8_E4M3, pc.SUM, 1, 1, comp=int(comp))
    req.bind([[dq]], [oq], rank_scales=[[ds]], out_scales=[osc],
             stream=stream)
    run_epoch(req, [0], stream)
    gq, gs = oq.cpu().numpy(), osc.cpu().numpy()
    req.free()
    wq, ws, _ = orc.sum_e4m3_f32([q], [sc], comp=comp)
    assert np.array_equal(gq, wq)
    assert np.array_equal(as_u32(gs), as_u32(ws))
    assert np.array_equal(as_u32(gs), as_u32(sc))
    expect = q.copy()
    if comp:
        expect[expect == 0x80] = 0x00
    assert np.array_equal(gq, expect)


@pytest.mark.parametrize("comp", [True, False])
def test_fp8_reduce(orc, stream, comp, layout=None, P=8):
    n, nparts = 256 * 997 + 131, 32
    say(f"case fp8 comp={comp} P={P} n={n} layout={layout}")
    xs = synth.normal_with_outliers_f32(P, n, synth.seed_for(5), 1e-2)
    packs = [pack_fp8_gpu(x.to(DEV)) for x in xs]
    opacks = [orc.e4m3_pack(x.numpy()) for x in xs]
    for (gq, gs), (oq, os_) in zip(packs, opacks):
        assert np.array_equal(gq[:n].cpu().numpy(), oq)
        assert np.array_equal(as_u32(gs.cpu().numpy()), as_u32(os_))
    nb = (n + 255) // 256
    out = torch.full((n,), 0x7F, dtype=torch.uint8, device=DEV)
    osc = torch.full((nb,), float("nan"), device=DEV)
    cfg = {} if layout is None else dict(tile_elems=1024, interleave=layout)
    req = new_request([n], pc.FP8_E4M3, pc.SUM, nparts, P, comp=int(comp),
                      **cfg)
    req.bind([[q for q, _ in packs]], [out],
             rank_scales=[[s for _, s in packs]], out_scales=[osc],
             stream=stream)
    run_epoch(req, synth.permutation(nparts, 5), stream)
    gq, gs = out.cpu().numpy(), osc.cpu().numpy()
    req.free()
    oq = [q for q, _ in opacks]
    os_ = [s for _, s in opacks]
    wq, ws, _ = orc.sum_e4m3_f32(oq, os_, comp=comp)
    assert np.array_equal(gq, wq)
    assert np.array_equal(as_u32(gs), as_u32(ws))
    y64 = orc.sum_e4m3_f64(oq, os_)
    table = orc.e4m3_decode_table()
    rep = lambda s: np.repeat(s.astype(np.float64), 256)[:n]  # noqa: E731
    deq = np.stack([table[q] * rep(s) for q, s in zip(oq, os_)])
    yv = table[gq] * rep(gs)
    tau = rep(gs) * 2.0 ** -6
    e = np.abs(yv - y64) / np.maximum(np.abs(deq).sum(axis=0), tau)
    assert e.max() <= 6e-2


@pytest.mark.parametrize("band", [0, 1, 3])
def test_fp8_tile_layouts(orc, stream, band):
    """e4m3 with one-row tiles (8 per partition) in each tile layout."""
    test_fp8_reduce(orc, stream, True, layout=band)


@pytest.mark.parametrize("P", [1, 2, 5, 16])
def test_fp8_rank_counts(orc, stream, P):
    """e4m3 sums (Sum2) at other rank counts than the workload's 8."""
    test_fp8_reduce(orc, stream, True, P=P)


# ------------------------------------------------------- batched and graphs
@pytest.mark.parametrize("graph", [1, 0])
def test_batched_bf16_graph_replays(orc, stream, graph):
    counts = [c // 8 for c in synth.batched_bf16_counts()[:12]] + [0, 1, 9]
    P, nparts = 8, 32
    say(f"case batched bf16 graph={graph} buckets={len(counts)}")
    xs = [synth.normal_f32(P, c, 300 + b, std=1e-3)
          for b, c in enumerate(counts)]
    pays = [[pack_bf16_gpu(x.to(DEV)) if c else
             torch.zeros(8, dtype=torch.int16, device=DEV) for x in xb]
            for xb, c in zip(xs, counts)]
    outs = [torch.full((max(c, 8),), 0x7FC0, dtype=torch.int16, device=DEV)
            for c in counts]
    req = new_request(counts, pc.BFLOAT16, pc.SUM, nparts, P, graph=graph)
    req.bind(pays, outs, stream=stream)
    total = len(counts) * nparts
    wants = [orc.sum_bf16_f32([orc.bf16_encode_array(x.numpy())
                               for x in xb])[0] for xb in xs]
    for epoch in range(3):
        for o in outs:
            o.fill_(0x7FC0)
        order = synth.permutation(total, 40 + epoch)
        run_epoch(req, order, stream, mode="list")
        for b, (o, w) in enumerate(zip(outs, wants)):
            got = o[:counts[b]].cpu().numpy().view(np.uint16)
            assert np.array_equal(got, w), (epoch, b)
    st = req.stats()
    if graph:
        assert st.graph_captures == 1 and st.graph_launches == 3
    req.free()


def test_pready_on_stream(orc, stream):
    P, n, nparts = 4, 200000, 16
    xs = synth.normal_f32(P, n, 91)
    out = torch.empty(n, device=DEV)
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P)
    side = independent_streams(stream, 1)[0]
    req.bind([[x.to(DEV) for x in xs]], [out], stream=stream)
    parts = torch.tensor(synth.permutation(nparts, 91), dtype=torch.int32,
                         device=DEV)
    torch.cuda.synchronize()
    for epoch in range(2):
        req.start()
        req.pready_on_stream(parts, nparts, side)
        req.wait()
        torch.cuda.synchronize()
        want = orc.sum_f32_f32([x.numpy() for x in xs])
        assert np.array_equal(as_u32(out.cpu().numpy()), as_u32(want))
    with pytest.raises(pc.PcollError):
        req.start()
        try:
            req.pready_on_stream(parts, nparts, stream)  # own stream: refused
        finally:
            req.pready_range(0, nparts - 1)
            req.wait()
    req.free()


@pytest.mark.parametrize("batch", [1, 7, 64])
def test_exactly_once_tile_counts(orc, stream, batch):
    say(f"case exactly-once publish_batch={batch}")
    P, n, nparts = 2, 100 * 1024 + 3, 7
    xs = synth.normal_f32(P, n, 5)
    out = torch.empty(n, device=DEV)
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P, debug=1,
                      tile_elems=4096, min_tile_elems=1024,
                      publish_batch=batch)
    req.bind([[x.to(DEV) for x in xs]], [out], stream=stream)
    want = orc.sum_f32_f32([x.numpy() for x in xs], comp=False)
    for epoch in range(3):
        out.fill_(float("nan"))
        run_epoch(req, synth.permutation(nparts, 5 + epoch), stream)
        assert np.array_equal(as_u32(out.cpu().numpy()), as_u32(want))
        hits, tiles = req.tile_hits()
        for p in range(nparts):
            _, _, ln = req.part_info(p)
            rows = -(-ln // 256)  # fp32 rows of 256 elements
            assert hits[p] == tiles[p], (p, hits[p], tiles[p])
            assert 1 <= tiles[p] <= max(1, rows), p
        assert req.stats().last_kernel_ms > 0
    req.free()


@pytest.mark.parametrize("guide,graph", [(1, 0), (4, 0), (2, 1)])
def test_guided_tiles(orc, stream, guide, graph):
    """Guided self-scheduling (tiles shrink as the remaining work does):
    bitwise against the oracle, every tile reduced once, over epochs in
    both launch modes."""
    say(f"case guided guide={guide} graph={graph}")
    P, n, nparts = 4, 700 * 1024 + 11, 9
    xs = synth.normal_f32(P, n, 81)
    out = torch.empty(n, device=DEV)
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P, debug=1,
                      tile_elems=32768, min_tile_elems=1024, guide=guide,
                      graph=graph)
    req.bind([[x.to(DEV) for x in xs]], [out], stream=stream)
    want = as_u32(orc.sum_f32_f32([x.numpy() for x in xs]))
    for epoch in range(3):
        out.fill_(float("nan"))
        run_epoch(req, synth.permutation(nparts, 81 + epoch), stream)
        assert np.array_equal(as_u32(out.cpu().numpy()), want), epoch
        hits, tiles = req.tile_hits()
        assert all(h == t for h, t in zip(hits, tiles)), (hits, tiles)
    req.free()


def test_state_machine_errors(stream):
    n = 4096
    x = torch.zeros(n, device=DEV)
    out = torch.empty(n, device=DEV)
    req = new_request([n], pc.FLOAT32, pc.SUM, 4, 2)
    with pytest.raises(pc.PcollError) as e:
        req.start()  # not bound
    assert e.value.code == pc.ERR_STATE
    req.bind([[x, x]], [out], stream=stream)
    with pytest.raises(pc.PcollError) as e:
        req.pready(0)  # no active epoch
    assert e.value.code == pc.ERR_STATE
    with pytest.raises(pc.PcollError) as e:
        req.parrived(0)  # never started
    assert e.value.code == pc.ERR_STATE
    req.start()
    with pytest.raises(pc.PcollError) as e:
        req.start()  # already active
    assert e.value.code == pc.ERR_STATE
    req.pready(2)
    with pytest.raises(pc.PcollError) as e:
        req.pready(2)  # twice in one epoch
    assert e.value.code == pc.ERR_STATE
    with pytest.raises(pc.PcollError) as e:
        req.pready(4)  # out of range
    assert e.value.code == pc.ERR_ARG
    with pytest.raises(pc.PcollError) as e:
        req.pready_list([0, 0])  # duplicate in the list
    assert e.value.code == pc.ERR_ARG
    with pytest.raises(pc.PcollError) as e:
        req.pready_list(np.array([1, 0, 1], np.int32))  # apart, numpy
    assert e.value.code == pc.ERR_ARG
    with pytest.raises(pc.PcollError) as e:
        req.pready_list(np.array([0, 2]))  # 2 already readied: nothing is
    assert e.value.code == pc.ERR_STATE     # published, 0 stays unready
    with pytest.raises(pc.PcollError) as e:
        pc.pcoll_free(req.h)  # active
    assert e.value.code == pc.ERR_STATE
    with pytest.raises(pc.PcollError) as e:
        req.set_config(tile_elems=2048)  # active
    assert e.value.code == pc.ERR_STATE
    req.pready_list([0, 1, 3])
    req.wait()
    assert req.test()
    req.free()


def test_wait_timeout_drains_and_recovers(orc, stream):
    """A partition never readied: wait_timeout gives up, the kernel drains,
    and the next epoch is correct."""
    P, n, nparts = 2, 64 * 1024, 4
    xs = synth.normal_f32(P, n, 8)
    out = torch.empty(n, device=DEV)
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P)
    req.bind([[x.to(DEV) for x in xs]], [out], stream=stream)
    req.start()
    req.pready_list([0, 1, 2])
    with pytest.raises(pc.PcollError) as e:
        req.wait_timeout(50)
    assert e.value.code == pc.ERR_TIMEOUT
    assert not req.parrived(3)
    assert req.parrived(0)
    run_epoch(req, [3, 2, 1, 0], stream)
    want = orc.sum_f32_f32([x.numpy() for x in xs])
    assert np.array_equal(as_u32(out.cpu().numpy()), as_u32(want))
    req.free()


def test_kernel_deadline_reports_aborted(orc, stream):
    P, n, nparts = 2, 8192, 2
    xs = synth.normal_f32(P, n, 9)
    out = torch.empty(n, device=DEV)
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P, timeout_ms=30)
    req.bind([[x.to(DEV) for x in xs]], [out], stream=stream)
    req.start()
    req.pready(0)
    with pytest.raises(pc.PcollError) as e:
        req.wait()
    assert e.value.code == pc.ERR_ABORTED
    req.set_config(timeout_ms=TEST_TIMEOUT_MS)
    run_epoch(req, [0, 1], stream)
    assert np.array_equal(as_u32(out.cpu().numpy()),
                          as_u32(orc.sum_f32_f32([x.numpy() for x in xs])))
    req.free()


def test_wait_on_stream_orders_consumer(orc, stream):
    P, n = 3, 123456
    xs = synth.normal_f32(P, n, 12)
    out = torch.empty(n, device=DEV)
    req = new_request([n], pc.FLOAT32, pc.SUM, 4, P)
    side = torch.cuda.Stream(DEV)
    req.bind([[x.to(DEV) for x in xs]], [out], stream=stream)
    req.start()
    req.pready_range(0, 3)
    req.wait_on_stream(side)
    with torch.cuda.stream(side):
        copy = out.clone()
    req.wait()
    side.synchronize()
    assert np.array_equal(as_u32(copy.cpu().numpy()),
                          as_u32(orc.sum_f32_f32([x.numpy() for x in xs])))
    req.free()


def test_epochs_alternate_streams_and_modes(orc, stream):
    """Consecutive epochs of one request on two streams, direct and graph
    launches mixed: each launch follows the previous one even across
    streams (the counter sets alternate by epoch parity), and every epoch's
    output is exact."""
    P, n, nparts = 4, 300 * 1024 + 5, 6
    say(f"case alternating streams P={P} n={n} nparts={nparts}")
    xs = synth.normal_f32(P, n, 61)
    dx = [x.to(DEV) for x in xs]
    out = torch.empty(n, device=DEV)
    want = as_u32(orc.sum_f32_f32([x.numpy() for x in xs]))
    other = torch.cuda.Stream(DEV)
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P, tile_elems=4096)
    for i in range(8):
        s = stream if i % 2 == 0 else other
        req.set_config(graph=(i // 2) % 2)
        req.bind([dx], [out], stream=s)
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        run_epoch(req, synth.permutation(nparts, 61 + i), s)
        assert np.array_equal(as_u32(out.cpu().numpy()), want), i
    req.free()


def test_two_requests_run_concurrently(orc, stream):
    """Two requests on two streams, both epochs started before either is
    readied, readiness interleaved, then both waited for; both outputs
    exact.  (Whether the two kernels run side by side depends on whether
    HIP put the streams on different hardware queues; the readiness order
    here lets the epochs complete either way: no epoch waits for the other
    one's completion.)"""
    P, n, nparts = 4, 120 * 1024 + 33, 5
    say(f"case two concurrent requests P={P} n={n}")
    xa, xb = synth.normal_f32(P, n, 91), synth.normal_f32(P, n, 92)
    oa, ob = torch.empty(n, device=DEV), torch.empty(n, device=DEV)
    sa, sb = torch.cuda.Stream(DEV), torch.cuda.Stream(DEV)
    ra = new_request([n], pc.FLOAT32, pc.SUM, nparts, P, tile_elems=2048)
    rb = new_request([n], pc.FLOAT32, pc.SUM, nparts, P, tile_elems=2048)
    ra.bind([[x.to(DEV) for x in xa]], [oa], stream=sa)
    rb.bind([[x.to(DEV) for x in xb]], [ob], stream=sb)
    torch.cuda.synchronize()
    for epoch in range(2):
        ra.start()
        rb.start()
        ra.pready_list([0, 1])
        rb.pready_list(list(range(nparts)))
        ra.pready_list([2, 3, 4])
        rb.wait()
        ra.wait()
        torch.cuda.synchronize()
        for x, o in ((xa, oa), (xb, ob)):
            want = as_u32(orc.sum_f32_f32([t.numpy() for t in x]))
            assert np.array_equal(as_u32(o.cpu().numpy()), want), epoch
    ra.free()
    rb.free()


def test_rebind_hits_cache(orc, stream):
    P, n = 2, 4096
    a = [x.to(DEV) for x in synth.normal_f32(P, n, 1)]
    b = [x.to(DEV) for x in synth.normal_f32(P, n, 2)]
    out = torch.empty(n, device=DEV)
    req = new_request([n], pc.FLOAT32, pc.SUM, 2, P)
    for src in (a, b, a, b):
        req.bind([src], [out], stream=stream)
        run_epoch(req, [0, 1], stream)
        want = orc.sum_f32_f32([x.cpu().numpy() for x in src])
        assert np.array_equal(as_u32(out.cpu().numpy()), as_u32(want))
    st = req.stats()
    assert st.cache_misses == 2 and st.cache_hits == 2
    req.free()


@pytest.mark.parametrize("unroll", [2, 4])
@pytest.mark.parametrize("dtype,P", [(pc.FLOAT32, 8), (pc.BFLOAT16, 5),
                                     (pc.INT32, 3), (pc.INT32, 16),
                                     (pc.FLOAT32, 12)])
def test_unroll_depths(orc, stream, unroll, dtype, P):
    """Both row depths of the 16-byte-vector kernels, bitwise, with ragged
    partitions and several rows per wave; the rows in flight the launch
    reports (4 / 2 up to 8 ranks, 2 / 1 above)."""
    n, nparts = 65536 * 3 + 1031, 5
    say(f"case unroll={unroll} dtype={dtype} P={P}")
    if dtype == pc.INT32:
        xs = synth.uniform_i32(P, n, 77, -(1 << 20), 1 << 20)
        want = orc.sum_i32([x.numpy() for x in xs])
        out = torch.empty(n, dtype=torch.int32, device=DEV)
    elif dtype == pc.FLOAT32:
        xs = synth.normal_f32(P, n, 78)
        want = orc.sum_f32_f32([x.numpy() for x in xs], comp=False)
        out = torch.empty(n, device=DEV)
    else:
        xs = [t.to(torch.bfloat16).view(torch.int16)
              for t in synth.normal_f32(P, n, 79)]
        want, _ = orc.sum_bf16_f32([x.numpy().view(np.uint16) for x in xs],
                                   comp=False)
        out = torch.empty(n, dtype=torch.int16, device=DEV)
    req = new_request([n], dtype, pc.SUM, nparts, P, comp=0, unroll=unroll,
                      tile_elems=16384, interleave=16)
    assert req.config().unroll == unroll
    req.bind([[x.to(DEV) for x in xs]], [out], stream=stream)
    run_epoch(req, synth.permutation(nparts, unroll), stream)
    assert req.stats().unroll == (unroll if P <= 8 else unroll // 2)
    got = out.cpu().numpy()
    req.free()
    assert np.array_equal(got.view(np.uint32 if got.itemsize == 4
                                   else np.uint16),
                          np.asarray(want).view(np.uint32 if got.itemsize == 4
                                                else np.uint16))


def test_unroll_rejects_other_depths(stream):
    req = pc.Request([1024], pc.FLOAT32, pc.SUM, 1, 2)
    with pytest.raises(pc.PcollError):
        req.set_config(unroll=3)
    assert req.config().unroll == 4
    req.free()


def test_more_workgroups_than_resident_with_slow_readiness(orc, stream):
    """A launch with more workgroups than the device holds at once (bf16 at
    8 ranks, twice as many groups of 8 waves as compute units, given as an
    exact count: a count from groups_per_cu is capped at the residency)
    and readiness trickling in, so that ingestion is partial: the tiles at
    the queue's end can belong to workgroups that have not started, and
    the waiting resident ones must ingest instead.  Bitwise against the
    oracle."""
    import time
    P, nparts = 8, 64
    n = nparts * 16 * 1024  # 16 one-row-pair tiles per partition
    cus = torch.cuda.get_device_properties(DEV).multi_processor_count
    say(f"case oversubscribed grid, slow readiness n={n}")
    xs = [t.to(torch.bfloat16).view(torch.int16)
          for t in synth.normal_f32(P, n, 81)]
    want, _ = orc.sum_bf16_f32([x.numpy().view(np.uint16) for x in xs],
                               comp=False)
    out = torch.empty(n, dtype=torch.int16, device=DEV)
    req = new_request([n], pc.BFLOAT16, pc.SUM, nparts, P, comp=0,
                      tile_elems=1024, min_tile_elems=1024,
                      groups=2 * cus, group_waves=8, interleave=0)
    req.bind([[x.to(DEV) for x in xs]], [out], stream=stream)
    for epoch in range(2):
        req.start()
        for p in synth.permutation(nparts, 90 + epoch):
            req.pready(int(p))
            time.sleep(2e-4)
        req.wait()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(np.uint16), want)
    assert req.stats().groups == 2 * cus
    req.free()


def test_grid_is_capped_at_residency(orc, stream):
    """A grid asked for as 4 workgroups of 8 waves per compute unit (more
    than the fp32 kernel's registers allow at once) is capped at what the
    device holds: every workgroup starts within a few microseconds of the
    first (its per-workgroup trace), each reduces tiles, and the output is
    bitwise the oracle's.  An exact `groups` count is not capped."""
    P, nparts = 8, 64
    n = 1 << 22
    cus = torch.cuda.get_device_properties(DEV).multi_processor_count
    say(f"case residency cap n={n} cus={cus}")
    xs = synth.normal_f32(P, n, 91)
    dx = [x.to(DEV) for x in xs]
    out = torch.full((n,), float("nan"), device=DEV)
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P, comp=0,
                      tile_elems=4096, groups_per_cu=4, group_waves=8,
                      unroll=4, debug=2)
    req.bind([dx], [out], stream=stream)
    run_epoch(req, synth.permutation(nparts, 92), stream, mode="list")
    st = req.stats()
    tr, khz = pc.pcoll_debug_trace(req.h)
    assert 1 <= st.groups < 4 * cus and len(tr) == st.groups
    starts = [s for s, _, _, _ in tr]
    spread_us = (max(starts) - min(starts)) * 1e3 / khz
    say(f"groups {st.groups}, start spread {spread_us:.1f} us")
    assert spread_us < 50.0, "a workgroup started late: not all resident"
    assert all(t >= 1 for _, _, _, t in tr)
    want = orc.sum_f32_f32([x.numpy() for x in xs], comp=False)
    assert np.array_equal(as_u32(out.cpu().numpy()), as_u32(want))
    # an exact count is taken as given
    req.set_config(groups=4 * cus, debug=0)
    run_epoch(req, synth.permutation(nparts, 93), stream, mode="list")
    assert req.stats().groups == 4 * cus
    assert np.array_equal(as_u32(out.cpu().numpy()), as_u32(want))
    req.free()


@pytest.mark.parametrize("layout", [0, 1, 2])
@pytest.mark.parametrize("nsrc", [1, 8])
def test_probe_stream_writes_the_xor(stream, layout, nsrc):
    """pcoll_probe_stream with write = 1 stores the bitwise XOR of its
    sources in every layout (sizes with a ragged end where the layout
    allows one); with write = 0 it leaves the destination alone."""
    nbytes = (1 << 20) + (0 if layout == 1 else 48)
    say(f"case probe_stream layout={layout} nsrc={nsrc} bytes={nbytes}")
    g = torch.Generator(device=DEV).manual_seed(1000 + 10 * layout + nsrc)
    n = nbytes // 4
    srcs = [torch.randint(-2**31, 2**31 - 1, (n,), generator=g, device=DEV,
                          dtype=torch.int32) for _ in range(nsrc)]
    dst = torch.zeros(n, dtype=torch.int32, device=DEV)
    want = srcs[0].clone()
    for s in srcs[1:]:
        want ^= s
    pc.pcoll_probe_stream(srcs, dst, nbytes, 1, layout, stream)
    torch.cuda.synchronize()
    assert torch.equal(dst, want)
    dst.fill_(7)
    pc.pcoll_probe_stream(srcs, dst, nbytes, 0, layout, stream)
    torch.cuda.synchronize()
    assert bool((dst == 7).all())
