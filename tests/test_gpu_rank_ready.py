"""Per-rank readiness (the receive side of a partitioned allreduce): a
partition is reduced only once every rank has readied it.  Through the C
ABI, against the oracle, bitwise (fp32, left-to-right rank order)."""
import time

import numpy as np
import pytest
import torch

from _gpu import DEV, as_u32, new_request, say
from oracle import get as get_oracle
from paper_2604_22228_amd import pcoll as pc
from paper_2604_22228_amd import synth
from paper_2604_22228_amd.streams import independent_streams

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    return get_oracle()


def _case(P, n, nparts, seed):
    xs = synth.normal_f32(P, n, seed)
    return xs, [x.to(DEV) for x in xs], torch.empty(n, device=DEV)


def _signals_ran(streams, limit=3.0):
    """Whether the work queued on `streams` completes within `limit`
    seconds (while an epoch's kernel runs: diagnostics of a stall)."""
    t0 = time.monotonic()
    while not all(s.query() for s in streams):
        if time.monotonic() - t0 > limit:
            return False
    return True


def _launch(req):
    st = req.stats()
    return {"groups": st.groups, "group_waves": st.group_waves,
            "unroll": st.unroll, "epochs": st.epochs}


def test_host_rank_marks_never_arrive_early(orc):
    P, n, nparts = 4, 60 * 1024 + 9, 6
    say(f"case host per-rank P={P} n={n} nparts={nparts}")
    xs, dx, out = _case(P, n, nparts, 71)
    want = as_u32(orc.sum_f32_f32([x.numpy() for x in xs]))
    stream = torch.cuda.Stream(DEV)
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P, tile_elems=1024)
    req.bind([dx], [out], stream=stream)
    for epoch in range(2):
        out.fill_(float("nan"))
        marks = [(r, p) for r in range(P) for p in range(nparts)]
        order = synth.permutation(len(marks), 71 + epoch)
        have = [set() for _ in range(nparts)]
        req.start()
        for i in order:
            r, p = marks[int(i)]
            for q in range(nparts):  # no partition before all its ranks
                if len(have[q]) < P:
                    assert not req.parrived(q), (epoch, q, have[q])
            req.pready_rank(r, p)
            have[p].add(r)
        req.wait()
        torch.cuda.synchronize()
        assert np.array_equal(as_u32(out.cpu().numpy()), want), epoch
    req.free()


def test_host_rank_mark_errors(orc):
    P, n, nparts = 3, 4096, 4
    xs, dx, out = _case(P, n, nparts, 72)
    stream = torch.cuda.Stream(DEV)
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P)
    req.bind([dx], [out], stream=stream)
    with pytest.raises(pc.PcollError) as e:
        req.pready_rank(0, 0)  # no active epoch
    assert e.value.code == pc.ERR_STATE
    req.start()
    req.pready_rank(1, 0)
    with pytest.raises(pc.PcollError) as e:
        req.pready_rank(1, 0)  # the same rank twice
    assert e.value.code == pc.ERR_STATE
    for bad in ((P, 0), (-1, 0), (0, nparts), (0, -1)):
        with pytest.raises(pc.PcollError) as e:
            req.pready_rank(*bad)
        assert e.value.code == pc.ERR_ARG
    req.pready(2)  # readied whole
    with pytest.raises(pc.PcollError) as e:
        req.pready_rank(0, 2)
    assert e.value.code == pc.ERR_STATE
    req.pready_rank(0, 0)
    req.pready_rank(2, 0)  # completes partition 0
    with pytest.raises(pc.PcollError) as e:
        req.pready(0)  # already ready
    assert e.value.code == pc.ERR_STATE
    req.pready_list([1, 3])
    req.wait()
    torch.cuda.synchronize()
    want = as_u32(orc.sum_f32_f32([x.numpy() for x in xs]))
    assert np.array_equal(as_u32(out.cpu().numpy()), want)
    req.free()


@pytest.mark.parametrize("graph", [0, 1])
def test_device_rank_marks_per_rank_streams(orc, graph):
    """The ranks mark their partitions from two signalling streams (ranks
    alternate between them; HIP gives a process only a few hardware
    queues, and a signal queued behind the reduce kernel could not run),
    each rank in its own order, some marks repeated (idempotent); three
    epochs."""
    P, n, nparts = 5, 200 * 1024 + 3, 13
    say(f"case device per-rank P={P} n={n} nparts={nparts} graph={graph}")
    xs, dx, out = _case(P, n, nparts, 73)
    want = as_u32(orc.sum_f32_f32([x.numpy() for x in xs]))
    stream = torch.cuda.Stream(DEV)
    signal = independent_streams(stream, 2)
    rank_streams = [signal[r % 2] for r in range(P)]
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P, tile_elems=2048,
                      graph=graph)
    req.bind([dx], [out], stream=stream)
    for epoch in range(3):
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        lists = []
        for r in range(P):
            o = synth.permutation(nparts, 100 * epoch + r).astype(np.int32)
            o = np.concatenate([o, o[:3]])  # repeated marks
            lists.append(torch.from_numpy(o).to(DEV))
        torch.cuda.synchronize()
        req.start()
        for r in range(P):
            req.pready_rank_on_stream(r, lists[r], lists[r].numel(),
                                      rank_streams[r])
        ran = _signals_ran(signal)
        try:
            req.wait()
        except pc.PcollError as e:
            raise AssertionError(f"epoch {epoch}: {e}; signal kernels ran "
                                 f"beside the reduce kernel: {ran}; launch "
                                 f"{_launch(req)}") from e
        torch.cuda.synchronize()
        assert np.array_equal(as_u32(out.cpu().numpy()), want), epoch
        assert all(req.parrived(p) for p in range(nparts))
    req.free()


def test_host_and_device_readiness_mix(orc):
    """Within one epoch: some partitions readied whole on the host, some by
    per-rank marks on the host, the rest by per-rank marks on the device."""
    P, n, nparts = 4, 100 * 1024, 12
    xs, dx, out = _case(P, n, nparts, 74)
    want = as_u32(orc.sum_f32_f32([x.numpy() for x in xs]))
    stream = torch.cuda.Stream(DEV)
    side = independent_streams(stream, 1)[0]
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P, tile_elems=2048)
    req.bind([dx], [out], stream=stream)
    dev_parts = torch.tensor([8, 9, 10, 11], dtype=torch.int32, device=DEV)
    torch.cuda.synchronize()
    req.start()
    req.pready_list([0, 1, 2, 3])
    for r in range(P):
        req.pready_rank_on_stream(r, dev_parts, 4, side)
        for p in (4, 5, 6, 7):
            req.pready_rank(r, p)
    req.wait()
    torch.cuda.synchronize()
    assert np.array_equal(as_u32(out.cpu().numpy()), want)
    req.free()


def test_producer_room_with_matrix_core_producers(orc):
    """Matrix-core (MFMA) producers run beside the waiting reduce kernel in
    the producer mode at its defaults (only `producers` = 1 set): each rank
    writes each partition with an FP32 matrix product on one of two
    signalling streams and marks it on the device right after; the output
    is bitwise the oracle's sum of what the products wrote."""
    P, nparts, m, k, q = 8, 8, 1024, 512, 512
    n = nparts * m * q
    say(f"case MFMA producers P={P} n={n} nparts={nparts}")
    gen = torch.Generator(device=DEV).manual_seed(75)
    a_ = [torch.randn(m, k, device=DEV, generator=gen) for _ in range(P)]
    b_ = torch.randn(k, q, device=DEV, generator=gen)
    xs = [torch.full((n,), float("nan"), device=DEV) for _ in range(P)]
    out = torch.empty(n, device=DEV)
    stream = torch.cuda.Stream(DEV)
    sig = independent_streams(stream, 2)
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P, producers=1)
    req.bind([xs], [out], stream=stream)
    cus = pc.pcoll_device_info()["compute_units"]
    ids = torch.arange(nparts, dtype=torch.int32, device=DEV)
    spans = [req.part_info(j)[1:] for j in range(nparts)]
    torch.cuda.synchronize()
    for epoch in range(2):
        req.start()
        st = req.stats()  # one workgroup of <= 4 waves per compute unit
        assert (st.groups, st.unroll) == (cus, 2) and st.group_waves <= 4
        for j in range(nparts):
            off, ln = spans[j]
            for r in range(P):
                with torch.cuda.stream(sig[r % 2]):
                    torch.mm(a_[r], b_, out=xs[r][off:off + ln].view(m, q))
                req.pready_rank_on_stream(r, ids[j:j + 1], 1, sig[r % 2])
        req.wait()
        torch.cuda.synchronize()
        want = as_u32(orc.sum_f32_f32([x.cpu().numpy() for x in xs]))
        assert np.array_equal(as_u32(out.cpu().numpy()), want), epoch
    req.free()


def test_producer_room_is_automatic_after_a_device_signal(orc):
    """In the automatic mode (the default), a request's launches switch to
    producer room from the start after its first device-side signal.  The
    launch before the switch here has 8-wave workgroups, one per compute
    unit, which leaves the signal kernel room to run (a launch that fills
    every unit would not: that first epoch would end at its deadline)."""
    P, n, nparts = 4, 2 * 1024 * 1024, 4
    xs, dx, out = _case(P, n, nparts, 76)
    want = as_u32(orc.sum_f32_f32([x.numpy() for x in xs]))
    stream = torch.cuda.Stream(DEV)
    side = independent_streams(stream, 1)[0]
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P, tile_elems=4096,
                      groups_per_cu=1, group_waves=8, unroll=4)
    assert req.config().producers == -1
    req.bind([dx], [out], stream=stream)
    cus = pc.pcoll_device_info()["compute_units"]
    ids = torch.arange(nparts, dtype=torch.int32, device=DEV)
    torch.cuda.synchronize()
    launches = []
    for epoch in range(3):
        req.start()
        st = req.stats()
        launches.append((st.groups, st.group_waves, st.unroll))
        if epoch == 0:
            req.pready_list(list(range(nparts)))
        else:
            req.pready_on_stream(ids, nparts, side)
        req.wait()
        torch.cuda.synchronize()
        assert np.array_equal(as_u32(out.cpu().numpy()), want), epoch
    say(f"(workgroups, waves, unroll) per epoch: {launches}")
    assert launches[0] == launches[1] == (cus, 8, 4)
    assert launches[2] == (cus, 4, 2)
    assert req.config().producers == -1
    req.free()


@pytest.mark.parametrize("producers", [0, 1])
def test_staggered_rank_marks_on_the_device(orc, producers):
    """Stragglers, as the benchmark plays them: rank r's partition j is
    marked on a side stream at (j + lag_r) gaps, each mark after a bounded
    spin, while the epoch's kernel waits; every partition is reduced once
    its last rank has marked it.  Bitwise against the oracle over two
    epochs, in the tuned launch (producers = 0) and in the launch that
    leaves room for producers (producers = 1)."""
    P, n, nparts = 4, 256 * 1024 + 13, 16
    say(f"case staggered device marks P={P} n={n} nparts={nparts} "
        f"producers={producers}")
    xs, dx, out = _case(P, n, nparts, 81)
    want = as_u32(orc.sum_f32_f32([x.numpy() for x in xs]))
    stream = torch.cuda.Stream(DEV)
    side = independent_streams(stream, 1)[0]
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P, tile_elems=1024,
                      producers=producers)
    req.bind([dx], [out], stream=stream)
    ids = torch.arange(nparts, dtype=torch.int32, device=DEV)
    rng = np.random.default_rng(82)
    lag = rng.uniform(0.0, 3.0, size=P)
    arrivals = sorted((j + lag[r], r, j) for r in range(P)
                      for j in range(nparts))
    torch.cuda.synchronize()
    for epoch in range(2):
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        req.start()
        t = 0.0
        for when, r, j in arrivals:
            cycles = int((when - t) * 20000)  # about 10 us per gap
            t = when
            if cycles > 0:
                with torch.cuda.stream(side):
                    torch.cuda._sleep(cycles)
            req.pready_rank_on_stream(r, ids[j:j + 1], 1, side)
        if not _signals_ran([side]):
            pytest.fail(f"marks did not run beside the kernel: {_launch(req)}")
        req.wait()
        torch.cuda.synchronize()
        assert np.array_equal(as_u32(out.cpu().numpy()), want), epoch
        assert all(req.parrived(p) for p in range(nparts))
    req.free()
