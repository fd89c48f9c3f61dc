"""The allocation-free epoch (pcoll_reduce_noalloc) through the C ABI,
against the request path (pcoll_init, pcoll_bind, pcoll_start, every
partition readied, pcoll_wait) on the same inputs: bit for bit, on two
calls in a row, the second with a smaller input (the scratch array keeps
the first call's contents and the set-up must clear what matters)."""
import numpy as np
import pytest
import torch

from _gpu import DEV, new_request, say
from paper_2604_22228_amd import pcoll as pc
from paper_2604_22228_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stream():
    assert torch.cuda.is_available()
    pc.load()
    return torch.cuda.current_stream(DEV)


def _inputs(dtype, P, n, seed):
    """Rank buffers (and scales) of `dtype` on the device."""
    cur = torch.cuda.current_stream(DEV)
    if dtype == pc.INT32:
        return synth.uniform_i32(P, n, seed, -(1 << 20), 1 << 20,
                                 device=DEV), None
    xs = synth.normal_f32(P, n, seed, device=DEV)
    if dtype == pc.FLOAT32:
        return xs, None
    if dtype in (pc.BFLOAT16, pc.BF16_PAIR):
        outs = []
        for x in xs:
            b = torch.empty(n, dtype=torch.int16, device=DEV)
            pc.pcoll_pack_bf16(x, b, n, cur)
            outs.append(b)
        return outs, None
    blk = 32 if dtype == pc.MXFP8_E4M3 else 256
    pack = {pc.FP8_E4M3: pc.pcoll_pack_fp8, pc.FP8_E5M2: pc.pcoll_pack_e5m2,
            pc.MXFP8_E4M3: pc.pcoll_pack_mxfp8}[dtype]
    sdt = torch.uint8 if blk == 32 else torch.float32
    qs, ss = [], []
    for x in xs:
        q = torch.empty(max(n, 16), dtype=torch.uint8, device=DEV)
        s = torch.empty(max((n + blk - 1) // blk, 1), dtype=sdt, device=DEV)
        pack(x, q, s, n, cur)
        qs.append(q)
        ss.append(s)
    return qs, ss


def _outputs(dtype, n):
    """Output buffers prefilled with bytes the result must overwrite: the
    output and its scales (8-bit floats) or lo halves (bf16 pairs)."""
    blk = 32 if dtype == pc.MXFP8_E4M3 else 256
    if dtype in (pc.FP8_E4M3, pc.FP8_E5M2, pc.MXFP8_E4M3):
        sdt = torch.uint8 if blk == 32 else torch.float32
        return (torch.full((max(n, 16),), 0x5A, dtype=torch.uint8, device=DEV),
                torch.full((max((n + blk - 1) // blk, 1),), 3, dtype=sdt,
                           device=DEV))
    nbytes = max(n * pc.ELEM_BYTES[dtype], 16)
    y = torch.full(((nbytes + 3) // 4,), 0x7FC01234, dtype=torch.int32,
                   device=DEV)
    lo = torch.full_like(y, 0x12345678) if dtype == pc.BF16_PAIR else None
    return y, lo  # output, and the second output (lo halves) or None


def _bytes(t, nbytes):
    return t.view(torch.uint8)[:nbytes].cpu().numpy()


CASES = [
    (pc.FLOAT32, pc.SUM, 8, 300007, 24),
    (pc.FLOAT32, pc.MAX, 5, 100003, 7),
    (pc.INT32, pc.SUM, 16, 200001, 64),
    (pc.INT32, pc.MAX, 3, 70001, 5),
    (pc.BFLOAT16, pc.SUM, 8, 250003, 32),
    (pc.BF16_PAIR, pc.SUM, 4, 90001, 9),
    (pc.FP8_E4M3, pc.SUM, 8, 300000, 16),
    (pc.MXFP8_E4M3, pc.SUM, 8, 123456, 12),
]


@pytest.mark.parametrize("dtype,op,P,n,nparts", CASES)
def test_noalloc_matches_request_path(stream, dtype, op, P, n, nparts):
    fp8 = dtype in (pc.FP8_E4M3, pc.FP8_E5M2, pc.MXFP8_E4M3)
    calls = ((n, nparts), (n // 3 + 5, max(1, nparts // 2)))
    for call, (m, k) in enumerate(calls):
        say(f"case noalloc dtype={dtype} op={op} P={P} n={m} nparts={k} "
            f"call={call}")
        bufs, scales = _inputs(dtype, P, m, 600 + 10 * dtype + call)
        # the request path
        y, second = _outputs(dtype, m)
        req = new_request([m], dtype, op, k, P)
        req.bind([bufs], [y], rank_scales=[scales] if fp8 else None,
                 out_scales=None if second is None else [second],
                 stream=stream)
        req.start()
        req.pready_range(0, k - 1)
        req.wait()
        req.free()
        # the allocation-free entry point, on buffers holding other bytes
        z, zsecond = _outputs(dtype, m)
        pc.pcoll_reduce_noalloc(m, dtype, op, k, bufs, z, scales, zsecond,
                                stream)
        torch.cuda.synchronize()
        nb = m * (1 if fp8 else pc.ELEM_BYTES[dtype])
        assert np.array_equal(_bytes(z, nb), _bytes(y, nb)), call
        if second is not None:
            n2 = second.numel() * second.element_size() if fp8 else nb
            assert np.array_equal(_bytes(zsecond, n2), _bytes(second, n2)), \
                call


def test_noalloc_rejects_too_many_partitions(stream):
    xs = synth.normal_f32(2, 4096, 1, device=DEV)
    y = torch.empty(4096, device=DEV)
    with pytest.raises(pc.PcollError) as e:
        pc.pcoll_reduce_noalloc(4096, pc.FLOAT32, pc.SUM,
                                pc.NOALLOC_MAX_PARTS + 1, xs, y, None, None,
                                stream)
    assert e.value.code == pc.ERR_UNSUPPORTED
