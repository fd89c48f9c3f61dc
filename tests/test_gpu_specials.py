"""Special values through the C ABI: NaNs (quiet and signalling, both
signs, with payloads), infinities, signed zeros, overflowing sums and
subnormals, planted in fp32 and bf16 inputs, against the oracle.

Bar: float max is IEEE 754-2019 maximum (NaN wherever any rank holds a
NaN, +0 above -0, independent of rank order); sums follow IEEE arithmetic
and the compensated sum returns the running sum once that is not finite.
fp32 outputs match bit for bit except inside NaNs (whose sign and payload
are unspecified: only the positions of NaNs are compared); bf16 outputs
match bit for bit, every NaN being the code 0x7FC0 on both sides."""
import numpy as np
import pytest
import torch

from _gpu import DEV, as_u32, new_request, run_epoch, say
from oracle import get as get_oracle
from paper_2604_22228_amd import pcoll as pc
from paper_2604_22228_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    return get_oracle()


@pytest.fixture(scope="module")
def stream():
    assert torch.cuda.is_available()
    pc.load()
    return torch.cuda.current_stream(DEV)


def _f32_inputs(P, n, seed):
    xs = synth.normal_f32(P, n, seed)
    bits = synth.plant_specials([x.view(torch.int32) for x in xs], seed + 1,
                                synth.F32_SPECIAL_BITS)
    return [b.view(torch.float32) for b in bits]


def _bf16_inputs(P, n, seed):
    codes = synth.bf16_codes(P, n, seed)
    return synth.plant_specials(codes, seed + 1, synth.BF16_SPECIAL_CODES)


def _same_f32(got, want):
    """Bitwise outside NaNs, NaN exactly where the oracle has one."""
    gn, wn = np.isnan(got), np.isnan(want)
    assert np.array_equal(gn, wn), \
        f"NaN positions differ at {np.flatnonzero(gn != wn)[:8]}"
    keep = ~wn
    diff = np.flatnonzero(as_u32(got)[keep] != as_u32(want)[keep])
    assert diff.size == 0, f"{diff.size} elements differ"


@pytest.mark.parametrize("P", [2, 5, 16])
@pytest.mark.parametrize("case", ["sum", "sum2", "max"])
def test_fp32_special_values(orc, stream, P, case):
    n, nparts = 50000 + 7, 6
    say(f"case fp32 specials {case} P={P} n={n}")
    xs = _f32_inputs(P, n, 900 + P)
    op = pc.MAX if case == "max" else pc.SUM
    cfg = {} if op == pc.MAX else {"comp": int(case == "sum2")}
    out = torch.zeros(n, device=DEV)
    req = new_request([n], pc.FLOAT32, op, nparts, P, tile_elems=4096, **cfg)
    req.bind([[x.to(DEV) for x in xs]], [out], stream=stream)
    run_epoch(req, synth.permutation(nparts, P), stream)
    got = out.cpu().numpy()
    req.free()
    host = [x.numpy() for x in xs]
    want = orc.max_f32(host) if op == pc.MAX else \
        orc.sum_f32_f32(host, comp=case == "sum2")
    # the planted values reach every kind of result
    assert np.isnan(want).any() and np.isinf(want).any()
    if op == pc.MAX and P <= 5:  # -0 needs -0 at every rank
        z = want == 0
        assert (z & np.signbit(want)).any() and (z & ~np.signbit(want)).any()
    _same_f32(got, want)


@pytest.mark.parametrize("P", [2, 5, 16])
@pytest.mark.parametrize("case", ["sum", "sum2", "max", "pair"])
def test_bf16_special_values(orc, stream, P, case):
    n, nparts = 40000 + 3, 5
    say(f"case bf16 specials {case} P={P} n={n}")
    xs = _bf16_inputs(P, n, 700 + P)
    host = [x.numpy().view(np.uint16) for x in xs]
    dx = [x.to(DEV) for x in xs]
    out = torch.full((n,), 0x1234, dtype=torch.int16, device=DEV)
    if case == "pair":
        lo = torch.full((n,), 0x1234, dtype=torch.int16, device=DEV)
        req = new_request([n], pc.BF16_PAIR, pc.SUM, nparts, P,
                          tile_elems=4096)
        req.bind([dx], [out], out_scales=[lo], stream=stream)
    else:
        op = pc.MAX if case == "max" else pc.SUM
        cfg = {} if op == pc.MAX else {"comp": int(case == "sum2")}
        req = new_request([n], pc.BFLOAT16, op, nparts, P, tile_elems=4096,
                          **cfg)
        req.bind([dx], [out], stream=stream)
    run_epoch(req, synth.permutation(nparts, P + 1), stream)
    got = out.cpu().numpy().view(np.uint16)
    glo = lo.cpu().numpy().view(np.uint16) if case == "pair" else None
    req.free()
    if case == "pair":
        whi, wlo = orc.sum_bf16_hilo(host, comp=True)
        assert (whi == 0x7FC0).any() and ((whi & 0x7FFF) == 0x7F80).any()
        assert np.array_equal(got, whi)
        assert np.array_equal(glo, wlo)
        return
    if case == "max":
        want = orc.max_bf16(host)
        assert (want == 0x0000).any()
        assert P > 5 or (want == 0x8000).any()
    else:
        want, _ = orc.sum_bf16_f32(host, comp=case == "sum2")
    assert (want == 0x7FC0).any()
    diff = np.flatnonzero(got != want)
    assert diff.size == 0, \
        f"{diff.size} codes differ, first at {diff[:4]}: " \
        f"{got[diff[:4]]} vs {want[diff[:4]]}"
