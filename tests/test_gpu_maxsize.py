"""The largest sizes the boundary accepts, on the GPU, sampled against the
oracle bit for bit: one partition of exactly 2^31 elements (the longest a
partition may be: the kernel indexes rows and vectors within a partition
in 32 bits), ragged lengths just below it, and a message of more than 2^32
elements whose partitions start beyond 2^32 elements (offsets are 64-bit).
Two ranks keep the memory at 48 GiB at most.  Sampled elements: both ends
of every partition, the partition boundaries, and a seeded random set."""
import numpy as np
import pytest
import torch

from _gpu import DEV, as_u32, new_request, run_epoch, say
from oracle import get as get_oracle
from paper_2604_22228_amd import pcoll as pc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    return get_oracle()


@pytest.fixture(scope="module")
def stream():
    assert torch.cuda.is_available()
    pc.load()
    return torch.cuda.current_stream(DEV)


def _sample(n, dtype, nparts, seed):
    _, offs, _ = pc.pcoll_plan(n, dtype, nparts)
    edges = sorted(set([0, n] + list(offs)))
    idx = []
    for e in edges:
        idx.append(np.arange(max(e - 1024, 0), min(e + 1024, n)))
    rng = np.random.default_rng(seed)
    idx.append(rng.integers(0, n, size=1 << 20))
    return np.unique(np.concatenate(idx)).astype(np.int64)


def _gen(n, dtype, seed):
    g = torch.Generator(device=DEV).manual_seed(seed)
    return torch.randn(n, generator=g, device=DEV, dtype=dtype)


def _case_f32(orc, stream, n, nparts, seed):
    say(f"case max size fp32 P=2 n={n} nparts={nparts}")
    xs = [_gen(n, torch.float32, seed + r) for r in range(2)]
    out = torch.empty(n, device=DEV)
    req = new_request([n], pc.FLOAT32, pc.SUM, nparts, 2, comp=0)
    req.bind([xs], [out], stream=stream)
    run_epoch(req, list(range(nparts))[::-1], stream, mode="list")
    req.free()
    idx = _sample(n, pc.FLOAT32, nparts, seed)
    ti = torch.from_numpy(idx).to(DEV)
    got = out[ti].cpu().numpy()
    cols = [x[ti].cpu().numpy() for x in xs]
    del xs, out
    torch.cuda.empty_cache()
    want = orc.sum_f32_f32(cols, comp=False)
    bad = int(np.count_nonzero(as_u32(got) != as_u32(want)))
    assert bad == 0, f"{bad} of {idx.size} sampled elements differ"


def test_one_partition_of_2p31_elements(orc, stream):
    _case_f32(orc, stream, 1 << 31, 1, 301)


def test_ragged_partition_below_2p31(orc, stream):
    _case_f32(orc, stream, (1 << 31) - 3, 1, 302)


def test_message_beyond_2p32_elements(orc, stream):
    _case_f32(orc, stream, (1 << 32) + 1000, 4, 303)


def test_bf16_ragged_partition_below_2p31(orc, stream):
    n = (1 << 31) - 5
    say(f"case max size bf16 P=2 n={n}")
    xs = [_gen(n, torch.bfloat16, 310 + r).view(torch.int16) for r in range(2)]
    out = torch.empty(n, dtype=torch.int16, device=DEV)
    req = new_request([n], pc.BFLOAT16, pc.SUM, 1, 2, comp=0)
    req.bind([xs], [out], stream=stream)
    run_epoch(req, [0], stream, mode="list")
    req.free()
    idx = _sample(n, pc.BFLOAT16, 1, 311)
    ti = torch.from_numpy(idx).to(DEV)
    got = out[ti].cpu().numpy().view(np.uint16)
    cols = [x[ti].cpu().numpy().view(np.uint16) for x in xs]
    del xs, out
    torch.cuda.empty_cache()
    want, _ = orc.sum_bf16_f32(cols, comp=False)
    bad = int(np.count_nonzero(got != want))
    assert bad == 0, f"{bad} of {idx.size} sampled elements differ"
