"""Finding streams whose work can run while a request's kernel runs.

The persistent reduce kernel occupies the stream it is launched on until
every partition of its epoch is ready.  HIP multiplexes a process's streams
onto a few hardware queues (GPU_MAX_HW_QUEUES, 4 by default), and work on a
stream that shares a hardware queue with the kernel's stream waits behind
the kernel.  A device-side ready signal (pcoll_pready_on_stream,
pcoll_pready_rank_on_stream), or a producer the readiness waits for, queued
on such a stream would never run during the epoch.  HIP does not expose the
stream-to-queue mapping, so this module finds suitable streams by
behaviour: it keeps the bound stream (and the streams already chosen) busy
with a short bounded spin, and keeps a candidate stream only if a tiny
kernel on it completes while every spin is still running.

The HIP runtime may hold a launch back until the host next looks at its
stream (a query or a synchronization), so every spin is submitted with a
query, and seen running, before the candidate's kernel is launched; a
check that skipped this would see the candidate run ahead of spins that
had not started yet.

This is a helper for callers of the library (and its tests and benchmark);
it is not part of the reduction.
"""
import time

import torch

# a spin of about 50 ms at the shader clocks of an MI355X
_SPIN_CYCLES = 100_000_000
_found = {}


def independent_streams(bound, n, device=None, tries=32):
    """Returns `n` streams of torch's pool such that work on any of them runs
    while `bound` and the other returned streams are busy.  Results are
    cached per (device, bound stream, n).  Raises RuntimeError if `tries`
    candidates do not yield `n` of them."""
    device = torch.device(device or bound.device)
    key = (str(device), bound.cuda_stream, n)
    if key in _found:
        return list(_found[key])
    busy = [bound]
    chosen = []
    flag = torch.zeros(1, device=device)
    for _ in range(tries):
        cand = torch.cuda.Stream(device)
        if any(cand.cuda_stream == b.cuda_stream for b in busy):
            continue  # the pool came round to a stream already in use
        torch.cuda.synchronize(device)
        for b in busy:
            with torch.cuda.stream(b):
                torch.cuda._sleep(_SPIN_CYCLES)
        started = not any(b.query() for b in busy)  # submits the spins
        with torch.cuda.stream(cand):
            flag.add_(1.0)
        t0 = time.perf_counter()
        while not cand.query() and time.perf_counter() - t0 < 1.0:
            pass
        ran = started and cand.query() and not any(b.query() for b in busy)
        torch.cuda.synchronize(device)
        if ran:
            chosen.append(cand)
            busy.append(cand)
            if len(chosen) == n:
                _found[key] = list(chosen)
                return chosen
    raise RuntimeError(f"found {len(chosen)} of {n} streams on hardware "
                       "queues of their own (GPU_MAX_HW_QUEUES too small?)")
