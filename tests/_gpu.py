"""Helpers of the GPU parity tests: run one epoch through the C ABI and
bring results back for comparison with the oracle."""
import numpy as np
import torch

from paper_2604_22228_amd import pcoll as pc

DEV = torch.device("cuda:0")
# a starved kernel gives up after this long, so a bug cannot hang a test
TEST_TIMEOUT_MS = 5000


def say(*a):
    print(*a, flush=True)


def as_u32(x):
    return np.ascontiguousarray(x).view(np.uint32)


def new_request(counts, dtype, op, nparts, nranks, **cfg):
    req = pc.Request(counts, dtype, op, nparts, nranks)
    cfg.setdefault("timeout_ms", TEST_TIMEOUT_MS)
    if "tile_elems" in cfg:
        cfg.setdefault("min_tile_elems", min(cfg["tile_elems"], 4096))
    req.set_config(**cfg)
    return req


def run_epoch(req, order, stream, mode="single"):
    """start, pready every partition in `order`, wait."""
    req.start()
    if mode == "list":
        req.pready_list([int(p) for p in order])
    else:
        for p in order:
            req.pready(int(p))
    req.wait()
    torch.cuda.synchronize()


def pack_bf16_gpu(x_dev):
    out = torch.empty(x_dev.numel(), dtype=torch.int16, device=DEV)
    pc.pcoll_pack_bf16(x_dev, out, x_dev.numel(),
                       torch.cuda.current_stream(DEV))
    return out


def pack_fp8_gpu(x_dev):
    n = x_dev.numel()
    q = torch.empty(max(n, 16), dtype=torch.uint8, device=DEV)
    s = torch.empty(max((n + 255) // 256, 1), dtype=torch.float32, device=DEV)
    pc.pcoll_pack_fp8(x_dev, q, s, n, torch.cuda.current_stream(DEV))
    return q, s


def empty_out(n, dtype, fill=0x7FC00000):
    """Output buffer prefilled with a sentinel (every element must be
    overwritten)."""
    nbytes = max(n * pc.ELEM_BYTES[dtype], 16)
    t = torch.empty((nbytes + 3) // 4, dtype=torch.int32, device=DEV)
    t.fill_(fill if fill < 2**31 else fill - 2**32)
    return t
