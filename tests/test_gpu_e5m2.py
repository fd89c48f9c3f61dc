"""e5m2 payloads (OCP E5M2, per-256 binary32 scales) through the C ABI:
producer packing, the identity over every finite code, and sums (plain and
Sum2), bitwise against the oracle's binary32 mirror, within the e5m2
output-rounding bound u / (1 + u) = 1/9 against the FP64 reference."""
import numpy as np
import pytest
import torch

from _gpu import DEV, as_u32, new_request, run_epoch, say
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


def _pack(x_dev):
    n = x_dev.numel()
    q = torch.empty(max(n, 16), dtype=torch.uint8, device=DEV)
    s = torch.empty(max((n + 255) // 256, 1), dtype=torch.float32,
                    device=DEV)
    pc.pcoll_pack_e5m2(x_dev, q, s, n, torch.cuda.current_stream(DEV))
    return q, s


def test_pack_e5m2_matches_oracle(orc, stream):
    n = 256 * 300 + 77
    x = synth.normal_with_outliers_f32(1, n, synth.seed_for(5), 1e-2)[0]
    x[:256] *= 1e4  # a block with large values
    x[256:512] *= 1e-6  # and one deep in the subnormal range of the codes
    q, s = _pack(x.to(DEV))
    oq, os_ = orc.e5m2_pack(x.numpy())
    assert np.array_equal(q[:n].cpu().numpy(), oq)
    assert np.array_equal(as_u32(s.cpu().numpy()), as_u32(os_))


@pytest.mark.parametrize("comp", [False, True])
def test_e5m2_identity_covers_every_finite_code(orc, stream, comp):
    """P = 1 over blocks holding all 248 finite codes (hardware decode and
    software encode reproduce each code and the scale; Sum2 maps -0 to
    +0)."""
    finite = [c for c in range(256) if (c & 0x7C) != 0x7C]
    codes = np.array(finite + [0] * (256 - len(finite)), dtype=np.uint8)
    n = 256 * 3
    q = np.concatenate([codes, codes[::-1], np.roll(codes, 5)])
    sc = np.array([1.0, 0.5, 3.0], dtype=np.float32)
    dq = torch.from_numpy(q).to(DEV)
    ds = torch.from_numpy(sc).to(DEV)
    oq = torch.full((n,), 0x7F, dtype=torch.uint8, device=DEV)
    osc = torch.zeros(3, device=DEV)
    req = new_request([n], pc.FP8_E5M2, pc.SUM, 1, 1, comp=int(comp))
    req.bind([[dq]], [oq], rank_scales=[[ds]], out_scales=[osc],
             stream=stream)
    run_epoch(req, [0], stream)
    gq, gs = oq.cpu().numpy(), osc.cpu().numpy()
    req.free()
    wq, ws, _ = orc.sum_e5m2_f32([q], [sc], comp=comp)
    assert np.array_equal(gq, wq)
    assert np.array_equal(as_u32(gs), as_u32(ws))
    expect = q.copy()
    if comp:
        expect[expect == 0x80] = 0x00
    assert np.array_equal(gq, expect)


@pytest.mark.parametrize("comp", [True, False])
def test_e5m2_reduce(orc, stream, comp):
    P, n, nparts = 8, 256 * 997 + 131, 32
    say(f"case e5m2 comp={comp} P={P} n={n}")
    xs = synth.normal_with_outliers_f32(P, n, synth.seed_for(5) + 1, 1e-2)
    packs = [_pack(x.to(DEV)) for x in xs]
    opacks = [orc.e5m2_pack(x.numpy()) for x in xs]
    for (gq, gs), (oq, os_) in zip(packs, opacks):
        assert np.array_equal(gq[:n].cpu().numpy(), oq)
        assert np.array_equal(as_u32(gs.cpu().numpy()), as_u32(os_))
    nb = (n + 255) // 256
    out = torch.full((n,), 0x7F, dtype=torch.uint8, device=DEV)
    osc = torch.full((nb,), float("nan"), device=DEV)
    req = new_request([n], pc.FP8_E5M2, pc.SUM, nparts, P, comp=int(comp))
    assert req.config().comp == 1 or not comp
    req.bind([[q for q, _ in packs]], [out],
             rank_scales=[[s for _, s in packs]], out_scales=[osc],
             stream=stream)
    run_epoch(req, synth.permutation(nparts, 6), stream)
    gq, gs = out.cpu().numpy(), osc.cpu().numpy()
    req.free()
    oq = [q for q, _ in opacks]
    os_ = [s for _, s in opacks]
    wq, ws, _ = orc.sum_e5m2_f32(oq, os_, comp=comp)
    assert np.array_equal(gq, wq)
    assert np.array_equal(as_u32(gs), as_u32(ws))
    y64 = orc.sum_e5m2_f64(oq, os_)
    table = orc.e5m2_decode_table()
    rep = lambda s: np.repeat(s.astype(np.float64), 256)[:n]  # noqa: E731
    deq = np.stack([table[q] * rep(s) for q, s in zip(oq, os_)])
    yv = table[gq] * rep(gs)
    tau = rep(gs) * 2.0 ** -14
    e = np.abs(yv - y64) / np.maximum(np.abs(deq).sum(axis=0), tau)
    say(f"e5m2 max normalized error {e.max():.4g}")
    assert e.max() <= 1 / 9 + 16 * U32


@pytest.mark.parametrize("graph", [0, 1])
def test_e5m2_batched(orc, stream, graph):
    P, nparts = 4, 8
    counts = [256 * 40 + 3, 100, 256 * 7, 5000]
    say(f"case e5m2 batched graph={graph} counts={counts}")
    qs, ss, oqs, oss, want = [], [], [], [], []
    for b, c in enumerate(counts):
        xs = synth.normal_f32(P, c, 900 + b, std=1e-2)
        row = [_pack(x.to(DEV)) for x in xs]
        qs.append([q for q, _ in row])
        ss.append([s for _, s in row])
        nb = (c + 255) // 256
        oqs.append(torch.full((max(c, 16),), 0x7F, dtype=torch.uint8,
                              device=DEV))
        oss.append(torch.full((nb,), float("nan"), device=DEV))
        op = [orc.e5m2_pack(x.numpy()) for x in xs]
        want.append(orc.sum_e5m2_f32([q for q, _ in op], [s for _, s in op],
                                     comp=True)[:2])
    torch.cuda.synchronize()
    req = new_request(counts, pc.FP8_E5M2, pc.SUM, nparts, P, graph=graph)
    req.bind(qs, oqs, ss, oss, stream=stream)
    for epoch in range(2):
        run_epoch(req, synth.permutation(req.nparts_total, 7 + epoch),
                  stream)
        for b, c in enumerate(counts):
            assert np.array_equal(oqs[b][:c].cpu().numpy(), want[b][0]), b
            assert np.array_equal(as_u32(oss[b].cpu().numpy()),
                                  as_u32(want[b][1])), b
    req.free()
