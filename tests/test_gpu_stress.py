"""Stress: a thousand epochs per request, two requests on two streams,
every epoch readied in a fresh random order by a random mix of the host
readiness calls (one by one, one list, a range), direct and graph launches
alternating.  (Device-side readiness is left to its own tests: a signal on
a stream that HIP put on a bound stream's hardware queue would wait behind
that stream's kernel.)  Every epoch's output is compared
bitwise with the oracle's on the GPU, and the debug counters show every
tile reduced exactly once."""
import numpy as np
import pytest
import torch

from _gpu import DEV, new_request, say
from oracle import get as get_oracle
from paper_2604_22228_amd import pcoll as pc
from paper_2604_22228_amd import synth

pytestmark = pytest.mark.gpu

EPOCHS = 1000


def _ready(req, order, how):
    if how == 0:
        for p in order:
            req.pready(int(p))
    elif how == 1:
        req.pready_list([int(p) for p in order])
    else:
        req.pready_range(0, req.nparts_total - 1)


def test_thousand_epochs_two_requests():
    orc = get_oracle()
    rng = np.random.default_rng(2026)
    cases = [(3, 40 * 1024 + 17, 9, pc.FLOAT32), (5, 7 * 1024 + 3, 4,
                                                  pc.FLOAT32)]
    reqs, outs, wants = [], [], []
    streams = [torch.cuda.Stream(DEV) for _ in cases]
    for i, (P, n, nparts, dtype) in enumerate(cases):
        xs = synth.normal_f32(P, n, 3100 + i)
        want = orc.sum_f32_f32([x.numpy() for x in xs], comp=False)
        out = torch.empty(n, device=DEV)
        req = new_request([n], dtype, pc.SUM, nparts, P, debug=1,
                          tile_elems=4096, min_tile_elems=1024)
        req.bind([[x.to(DEV) for x in xs]], [out], stream=streams[i])
        reqs.append(req)
        outs.append(out)
        wants.append(torch.from_numpy(want.view(np.int32)).to(DEV))
    torch.cuda.synchronize()
    for e in range(EPOCHS):
        if e % 100 == 0:
            say(f"stress epoch {e}")
        graph = (e // 7) % 2
        for r, out in zip(reqs, outs):
            r.set_config(graph=graph)
            out.fill_(float("nan"))
        torch.cuda.synchronize()
        for r in reqs:
            r.start()
        for r in reqs:
            _ready(r, rng.permutation(r.nparts_total), int(rng.integers(0, 3)))
        for r in reqs:
            r.wait()
        torch.cuda.synchronize()
        for i, (r, out) in enumerate(zip(reqs, outs)):
            assert torch.equal(out.view(torch.int32), wants[i]), (e, i)
            hits, tiles = r.tile_hits()
            assert all(h == t and t >= 1 for h, t in zip(hits, tiles)), (e, i)
    for r in reqs:
        assert r.stats().epochs == EPOCHS
        r.free()
