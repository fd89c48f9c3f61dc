"""Device-side readiness across epochs, through the C ABI, bitwise against
the oracle (fp32 sum, left-to-right rank order).

A device-side ready signal names the epoch it was enqueued in.  One that
runs after its epoch ended (wait_timeout ended the epoch while the signal
was still queued behind a slow producer on its stream) must neither ready
a partition of a later epoch nor disturb that epoch's per-rank marks; ids
out of range are ignored, and a partition signalled twice counts once.
The slow producer is a bounded spin on a side stream, so every kernel ends
normally."""
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
# spin of the slow producer, in shader clocks: well above the time the
# test needs to end one epoch and start the next
SPIN_CYCLES = 600_000_000


@pytest.fixture(scope="module")
def orc():
    return get_oracle()


@pytest.fixture(scope="module")
def stream():
    assert torch.cuda.is_available()
    pc.load()
    return torch.cuda.current_stream(DEV)


def _want(orc, xs):
    return as_u32(orc.sum_f32_f32([x.cpu().numpy() for x in xs]))


def _ids(vals):
    return torch.tensor(vals, dtype=torch.int32, device=DEV)


def test_out_of_range_and_repeated_ids_over_epochs(orc, stream):
    P, n, nparts = 3, 96 * 1024 + 5, 24
    say(f"case device ids P={P} n={n} nparts={nparts}")
    xs = synth.normal_f32(P, n, 31)
    dx = [x.to(DEV) for x in xs]
    out = torch.empty(n, device=DEV)
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P, tile_elems=1024)
    req.bind([dx], [out], stream=stream)
    sides = independent_streams(stream, 2)
    want = _want(orc, xs)
    bad = [-1, nparts, nparts + 7, 1 << 20, 2**31 - 1, -(2**31)]
    for epoch in range(3):
        perm = [int(p) for p in synth.permutation(nparts, 40 + epoch)]
        half = nparts // 2
        # out-of-range ids and repeats mixed into both calls; the second
        # call repeats some partitions of the first
        first = perm[:half] + bad[:3] + perm[:2]
        second = bad[3:] + perm[half:] + perm[:3] + perm[half:half + 2]
        ids = [_ids(first), _ids(second)]
        torch.cuda.synchronize()
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        req.start()
        req.pready_on_stream(ids[0], len(first), sides[0])
        req.pready_on_stream(ids[1], len(second), sides[1])
        req.wait()
        torch.cuda.synchronize()
        assert np.array_equal(as_u32(out.cpu().numpy()), want), epoch
    # device and host readiness of disjoint partitions in one epoch (device
    # arrays are made before the start: a copy on the bound stream would
    # wait for the epoch's kernel)
    even = _ids(list(range(0, nparts, 2)))
    req.start()
    req.pready_on_stream(even, nparts // 2, sides[0])
    req.pready_list(list(range(1, nparts, 2)))
    req.wait()
    torch.cuda.synchronize()
    assert np.array_equal(as_u32(out.cpu().numpy()), want)
    req.free()


def _late_setup(P, n, nparts, seed, stream):
    xs = synth.normal_f32(P, n, seed)
    dx = [x.to(DEV) for x in xs]
    new = [x.to(DEV) for x in synth.normal_f32(P, n, seed + 1)]
    out = torch.empty(n, device=DEV)
    # the kernel's own deadline well beyond the spin
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P, tile_elems=1024,
                      timeout_ms=20000)
    req.bind([dx], [out], stream=stream)
    return xs, dx, new, out, req


def _end_epoch_with_late_signal(req, side, signal):
    """Starts an epoch, queues `signal` on `side` behind a bounded spin and
    ends the epoch with wait_timeout while the signal is still queued."""
    req.start()
    with torch.cuda.stream(side):
        torch.cuda._sleep(SPIN_CYCLES)
    signal()
    t0 = time.perf_counter()
    with pytest.raises(pc.PcollError) as e:
        req.wait_timeout(20)
    assert e.value.code == pc.ERR_TIMEOUT
    say(f"epoch ended after {1e3 * (time.perf_counter() - t0):.1f} ms")


def test_late_signal_does_not_ready_the_next_epoch(orc, stream):
    P, n, nparts = 4, 64 * 1024 + 3, 8
    say(f"case late pready_on_stream P={P} n={n} nparts={nparts}")
    xs, dx, new, out, req = _late_setup(P, n, nparts, 51, stream)
    side, copier = independent_streams(stream, 2)
    ids = _ids(list(range(nparts)))
    torch.cuda.synchronize()
    _end_epoch_with_late_signal(
        req, side, lambda: req.pready_on_stream(ids, nparts, side))
    # next epoch: the late signal runs while it is active; the rank data
    # change after that and only then are the partitions readied
    out.fill_(float("nan"))
    stream.synchronize()  # not the device: the spin must go on
    req.start()
    assert not side.query(), "the spin ended before the next epoch began"
    t0 = time.perf_counter()
    side.synchronize()
    say(f"late signal ran {1e3 * (time.perf_counter() - t0):.1f} ms into "
        "the next epoch")
    assert not any(req.parrived(p) for p in range(nparts))
    with torch.cuda.stream(copier):
        for d, v in zip(dx, new):
            d.copy_(v)
    copier.synchronize()
    for p in synth.permutation(nparts, 52):
        req.pready(int(p))
    req.wait()
    torch.cuda.synchronize()
    assert np.array_equal(as_u32(out.cpu().numpy()), _want(orc, new))
    # and the epoch after, readied on the device again
    perm = _ids([int(p) for p in synth.permutation(nparts, 53)])
    req.start()
    req.pready_on_stream(perm, nparts, side)
    req.wait()
    torch.cuda.synchronize()
    assert np.array_equal(as_u32(out.cpu().numpy()), _want(orc, new))
    req.free()


def test_late_rank_mark_keeps_newer_marks(orc, stream):
    P, n, nparts = 4, 64 * 1024 + 3, 6
    say(f"case late pready_rank_on_stream P={P} n={n} nparts={nparts}")
    xs, dx, new, out, req = _late_setup(P, n, nparts, 61, stream)
    side, other = independent_streams(stream, 2)
    ids = _ids(list(range(nparts)))
    torch.cuda.synchronize()
    _end_epoch_with_late_signal(
        req, side, lambda: req.pready_rank_on_stream(0, ids, nparts, side))
    out.fill_(float("nan"))
    stream.synchronize()  # not the device: the spin must go on
    req.start()
    assert not side.query(), "the spin ended before the next epoch began"
    for r in range(1, P):  # every rank but 0 marks in the new epoch
        req.pready_rank_on_stream(r, ids, nparts, other)
    other.synchronize()
    side.synchronize()  # the late mark of rank 0 of the ended epoch runs
    assert not any(req.parrived(p) for p in range(nparts))
    req.pready_rank_on_stream(0, ids, nparts, other)
    req.wait()
    torch.cuda.synchronize()
    assert np.array_equal(as_u32(out.cpu().numpy()), _want(orc, xs))
    req.free()


@pytest.mark.parametrize("graph", [0, 1])
def test_epoch_count_wraps(orc, stream, graph):
    P, n, nparts = 3, 40 * 1024 + 1, 5
    say(f"case epoch wrap graph={graph}")
    xs = synth.normal_f32(P, n, 71)
    dx = [x.to(DEV) for x in xs]
    out = torch.empty(n, device=DEV)
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, P, tile_elems=1024,
                      graph=graph)
    req.bind([dx], [out], stream=stream)
    side = independent_streams(stream, 1)[0]
    want = _want(orc, xs)
    run = 0

    def epoch(mode):
        nonlocal run
        run += 1
        out.fill_(float("nan"))
        perm = [int(p) for p in synth.permutation(nparts, 80 + run)]
        ids = _ids(perm)
        torch.cuda.synchronize()
        req.start()
        if mode == "host":
            req.pready_list(perm)
        elif mode == "device":
            req.pready_on_stream(ids, nparts, side)
        else:  # per rank, on the device
            for r in range(P):
                req.pready_rank_on_stream(r, ids, nparts, side)
        req.wait()
        torch.cuda.synchronize()
        assert np.array_equal(as_u32(out.cpu().numpy()), want), (mode, run)
        assert all(req.parrived(p) for p in range(nparts))

    # a few epochs first, so that every stamp holds small epochs
    for m in ("host", "device", "rank", "device"):
        epoch(m)
    # both parities of the last epoch before the wrap
    for last in (0xFFFFFFFC, 0xFFFFFFFB):
        req.debug_set_epoch(last)
        for m in ("device", "rank", "host", "device", "rank", "device"):
            epoch(m)
    req.free()
