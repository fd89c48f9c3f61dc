"""bf16 pair output (PCOLL_BF16_PAIR: bf16 in, hi = bf16(y) and lo =
bf16(y - hi) out, y the binary32 sum) through the C ABI: bitwise against
the oracle for plain and Sum2 accumulation, over tile layouts, ragged
sizes and batched launches, and within 2^-16 + the binary32 sum's error of
the FP64 reference."""
import numpy as np
import pytest
import torch

from _gpu import DEV, new_request, run_epoch, say
from oracle import get as get_oracle
from paper_2604_22228_amd import pcoll as pc
from paper_2604_22228_amd import synth

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def orc():
    return get_oracle()


@pytest.fixture(scope="module")
def stream():
    assert torch.cuda.is_available()
    pc.load()
    return torch.cuda.current_stream(DEV)


def _bf16(P, n, seed, std=1e-3):
    xs = synth.normal_f32(P, n, seed, std=std)
    return [t.to(torch.bfloat16).view(torch.int16) for t in xs]


def _u16(t):
    return t.cpu().numpy().view(np.uint16)


def _values(codes):
    return (codes.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _check(orc, xs, hi, lo, n, comp):
    host = [_u16(x) for x in xs]
    whi, wlo = orc.sum_bf16_hilo(host, comp=comp)
    ghi, glo = _u16(hi)[:n], _u16(lo)[:n]
    assert np.array_equal(ghi, whi)
    assert np.array_equal(glo, wlo)
    return host, ghi, glo


@pytest.mark.parametrize("comp", [True, False])
@pytest.mark.parametrize("P", [1, 3, 8, 16])
def test_bf16_pair_reduce(orc, stream, comp, P):
    n, nparts = 4096 * 37 + 5, 13
    say(f"case bf16 pair P={P} comp={comp} n={n}")
    xs = _bf16(P, n, 500 + P)
    hi = torch.full((n,), 0x7FC0, dtype=torch.int16, device=DEV)
    lo = torch.full((n,), 0x7FC0, dtype=torch.int16, device=DEV)
    req = new_request([n], pc.BF16_PAIR, pc.SUM, nparts, P, comp=int(comp))
    req.bind([[x.to(DEV) for x in xs]], [hi], out_scales=[lo], stream=stream)
    run_epoch(req, synth.permutation(nparts, P), stream)
    host, ghi, glo = _check(orc, xs, hi, lo, n, comp)
    req.free()
    y64 = orc.sum_bf16_f64(host)
    absum = np.abs(np.stack([_values(h) for h in host])).sum(axis=0)
    e = np.abs(_values(ghi) + _values(glo) - y64) / np.maximum(absum, 1e-38)
    bound = 2.0 ** -16 + (3 * U32 if comp else (P - 1) * U32 / (1 - (P - 1) * U32))
    say(f"bf16 pair max normalized error {e.max():.3g} (bound {bound:.3g})")
    assert e.max() <= bound


@pytest.mark.parametrize("band", [0, 1, 5])
def test_bf16_pair_tile_layouts(orc, stream, band):
    P, n, nparts = 4, 512 * 300 + 77, 6
    say(f"case bf16 pair layout band={band}")
    xs = _bf16(P, n, 600 + band, std=1.0)
    hi = torch.full((n,), 0x7FC0, dtype=torch.int16, device=DEV)
    lo = torch.full((n,), 0x7FC0, dtype=torch.int16, device=DEV)
    req = new_request([n], pc.BF16_PAIR, pc.SUM, nparts, P, tile_elems=1024,
                      interleave=band)
    req.bind([[x.to(DEV) for x in xs]], [hi], out_scales=[lo], stream=stream)
    for epoch in range(2):
        hi.fill_(0x7FC0)
        lo.fill_(0x7FC0)
        run_epoch(req, synth.permutation(nparts, epoch), stream)
        _check(orc, xs, hi, lo, n, True)
    req.free()


@pytest.mark.parametrize("graph", [0, 1])
def test_bf16_pair_batched(orc, stream, graph):
    P, nparts = 8, 4
    counts = [8 * 1000 + 3, 7, 0, 65536, 12345]
    say(f"case bf16 pair batched graph={graph}")
    ins, his, los = [], [], []
    for b, c in enumerate(counts):
        ins.append([x.to(DEV) for x in _bf16(P, c, 700 + b)])
        his.append(torch.full((max(c, 8),), 0x7FC0, dtype=torch.int16,
                              device=DEV))
        los.append(torch.full((max(c, 8),), 0x7FC0, dtype=torch.int16,
                              device=DEV))
    req = new_request(counts, pc.BF16_PAIR, pc.SUM, nparts, P, graph=graph)
    req.bind(ins, his, out_scales=los, stream=stream)
    run_epoch(req, synth.permutation(req.nparts_total, 3), stream, mode="list")
    for b, c in enumerate(counts):
        _check(orc, ins[b], his[b], los[b], c, True)
    req.free()


def test_bf16_pair_argument_rules(stream):
    with pytest.raises(pc.PcollError) as e:
        pc.Request([64], pc.BF16_PAIR, pc.MAX, 1, 2)
    assert e.value.code == pc.ERR_UNSUPPORTED
    req = pc.Request([64], pc.BF16_PAIR, pc.SUM, 1, 2)
    assert req.config().comp == 1  # compensated by default
    x = torch.zeros(64, dtype=torch.int16, device=DEV)
    with pytest.raises(pc.PcollError):
        req.bind([[x, x]], [x], stream=stream)  # the lo outputs are required
    with pytest.raises(pc.PcollError):
        req.bind([[x, x]], [x], rank_scales=[[x, x]], out_scales=[x],
                 stream=stream)  # and input scales are not taken
    req.free()
