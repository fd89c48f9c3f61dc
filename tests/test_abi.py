"""The C ABI without a GPU: the library loads, exports every entry point
that include/pcoll.h declares, and its host-only logic (partition plan,
argument checks, error strings) behaves as documented.  No kernel runs."""
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import get as get_oracle
from paper_2604_22228_amd import pcoll as pc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pcoll.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pcoll_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary_calls():
    names = _declared()
    for must in ("pcoll_init", "pcoll_pready", "pcoll_parrived",
                 "pcoll_start", "pcoll_wait", "pcoll_init_batch",
                 "pcoll_bind", "pcoll_free", "pcoll_pready_on_stream",
                 "pcoll_wait_timeout", "pcoll_wait_on_stream"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = pc.load()
    out = subprocess.run(["nm", "-D", "--defined-only", pc.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(pcoll_[a-z0-9_]+)$", out, flags=re.M))
    for name in _declared():
        assert name in exported, name
        assert getattr(lib, name) is not None
    # the binding covers the same set, one function per entry point
    for name in _declared():
        assert hasattr(pc, name), name


def test_library_links_no_oracle():
    out = subprocess.run(["nm", "-D", pc.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    assert "orc_" not in out
    ldd = subprocess.run(["ldd", pc.LIB_PATH], capture_output=True,
                         text=True).stdout
    assert "liboracle" not in ldd


def test_version_and_strerror():
    assert pc.pcoll_version() == 1
    lib = pc.load()
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -99):
        assert lib.pcoll_strerror(code)


@pytest.mark.parametrize("dtype,align", [(pc.INT32, 32), (pc.FLOAT32, 32),
                                         (pc.BFLOAT16, 64),
                                         (pc.FP8_E4M3, 256),
                                         (pc.FP8_E5M2, 256),
                                         (pc.MXFP8_E4M3, 128),
                                         (pc.BF16_PAIR, 64)])
def test_plan_matches_oracle(dtype, align):
    orc = get_oracle()
    for count in list(range(0, 70)) + [255, 256, 1000, 262144, 262144 + 37,
                                       (1 << 24) + 3]:
        for nparts in (1, 2, 3, 4, 7, 8, 16, 64, 256):
            ps, offs, lens = pc.pcoll_plan(count, dtype, nparts)
            ops, ooff, olen = orc.plan(count, nparts, align)
            assert ps == ops
            assert offs == ooff.tolist() and lens == olen.tolist()


def test_plan_rejects_bad_arguments():
    with pytest.raises(pc.PcollError) as e:
        pc.pcoll_plan(10, 7, 4)
    assert e.value.code == pc.ERR_ARG
    with pytest.raises(pc.PcollError):
        pc.pcoll_plan(10, pc.FLOAT32, 0)


@pytest.mark.parametrize("args,code", [
    ((100, 9, pc.SUM, 4, 4), pc.ERR_ARG),           # dtype
    ((100, pc.FLOAT32, 5, 4, 4), pc.ERR_ARG),       # op
    ((100, pc.FLOAT32, pc.SUM, 0, 4), pc.ERR_ARG),  # nparts
    ((100, pc.FLOAT32, pc.SUM, 4, 0), pc.ERR_ARG),  # nranks
    ((100, pc.FLOAT32, pc.SUM, 4, 17), pc.ERR_UNSUPPORTED),
    ((100, pc.FP8_E4M3, pc.MAX, 4, 4), pc.ERR_UNSUPPORTED),
    ((100, pc.FP8_E5M2, pc.MAX, 4, 4), pc.ERR_UNSUPPORTED),
    ((100, pc.MXFP8_E4M3, pc.MAX, 4, 4), pc.ERR_UNSUPPORTED),
    ((100, pc.BF16_PAIR, pc.MAX, 4, 4), pc.ERR_UNSUPPORTED),
    ((100, 7, pc.SUM, 4, 4), pc.ERR_ARG),           # no dtype 7
    # a partition beyond 2^31 elements (the kernels' 32-bit row indices)
    ((1 << 33, pc.FLOAT32, pc.SUM, 1, 4), pc.ERR_UNSUPPORTED),
    ((1 << 41, pc.INT32, pc.SUM, 4096, 4), pc.ERR_UNSUPPORTED),
    ((100, pc.FLOAT32, pc.SUM, (1 << 24) + 1, 4), pc.ERR_UNSUPPORTED),
])
def test_init_argument_errors_need_no_gpu(args, code):
    with pytest.raises(pc.PcollError) as e:
        pc.pcoll_init(*args)
    assert e.value.code == code


def test_batch_argument_errors_need_no_gpu():
    lib = pc.load()
    import ctypes as C
    h = C.c_void_p()
    assert lib.pcoll_init_batch(0, None, 1, 0, 4, 4, C.byref(h)) == pc.ERR_ARG
    arr = (C.c_size_t * 2)(10, 20)
    assert lib.pcoll_init_batch(2, arr, 1, 0, 4, 99, C.byref(h)) == \
        pc.ERR_UNSUPPORTED
    assert lib.pcoll_init(10, 1, 0, 4, 4, None) == pc.ERR_ARG


def test_null_request_is_an_argument_error():
    lib = pc.load()
    for name in ("pcoll_start", "pcoll_wait", "pcoll_free"):
        assert getattr(lib, name)(None) == pc.ERR_ARG
    assert lib.pcoll_pready(None, 0) == pc.ERR_ARG
    assert lib.pcoll_pready_rank(None, 0, 0) == pc.ERR_ARG
    assert lib.pcoll_pready_rank_on_stream(None, 0, None, 0, None) == \
        pc.ERR_ARG


def test_probe_and_pack_reject_unaligned_sizes():
    lib = pc.load()
    assert lib.pcoll_probe_copy(None, None, 15, None) == pc.ERR_ARG
    assert lib.pcoll_probe_fill(None, 17, 0, None) == pc.ERR_ARG
    assert lib.pcoll_pack_bf16(None, None, 8, None) == pc.ERR_ARG
    assert lib.pcoll_pack_fp8(None, None, None, 8, None) == pc.ERR_ARG
    assert lib.pcoll_pack_mxfp8(None, None, None, 8, None) == pc.ERR_ARG
    assert lib.pcoll_pack_mxfp8(None, None, None, 0, None) == 0
    # zero-length packs are no-ops that need no device
    assert lib.pcoll_pack_bf16(None, None, 0, None) == 0


def test_probe_stream_rejects_bad_layouts_and_sizes():
    """Argument checks of pcoll_probe_stream, all taken before any device
    call: source counts, layouts 0..2, sizes per layout, alignment."""
    import ctypes as C
    lib = pc.load()
    buf = (C.c_uint64 * 4)()  # 16-byte aligned host stand-ins: never read
    addr = C.addressof(buf)
    srcs = (C.c_void_p * 8)(*([addr] * 8))
    ok_dst = C.c_void_p(addr)
    for layout in (-1, 3):
        assert lib.pcoll_probe_stream(srcs, 8, ok_dst, 1024, 1, layout,
                                      None) == pc.ERR_ARG
    for nsrc in (0, 3, 17):
        assert lib.pcoll_probe_stream(srcs, nsrc, ok_dst, 1024, 1, 2,
                                      None) == pc.ERR_ARG
    assert lib.pcoll_probe_stream(srcs, 8, ok_dst, 1024, 2, 2,
                                  None) == pc.ERR_ARG       # write not 0/1
    assert lib.pcoll_probe_stream(srcs, 8, ok_dst, 24, 1, 2,
                                  None) == pc.ERR_ARG       # not 16 B units
    assert lib.pcoll_probe_stream(srcs, 8, ok_dst, 1040, 1, 1,
                                  None) == pc.ERR_ARG       # not whole rows
    assert lib.pcoll_probe_stream(srcs, 8, None, 1024, 1, 2,
                                  None) == pc.ERR_ARG       # no destination
    bad = (C.c_void_p * 8)(*([addr + 4] * 8))
    assert lib.pcoll_probe_stream(bad, 8, ok_dst, 1024, 1, 2,
                                  None) == pc.ERR_ARG       # misaligned


def test_plan_partitions_are_aligned_for_lines():
    """Partitions start on 128-byte lines (and 8-bit scale blocks)."""
    for dtype in (pc.INT32, pc.FLOAT32, pc.BFLOAT16, pc.FP8_E4M3,
                  pc.FP8_E5M2, pc.MXFP8_E4M3, pc.BF16_PAIR):
        for count in (1, 7, 1000, 123457):
            ps, offs, lens = pc.pcoll_plan(count, dtype, 8)
            unit = {pc.FP8_E4M3: 256, pc.FP8_E5M2: 256,
                    pc.MXFP8_E4M3: 128}.get(dtype,
                                            128 // pc.ELEM_BYTES[dtype])
            assert ps % unit == 0
            assert all(o % unit == 0 for o, n in zip(offs, lens) if n)
            assert sum(lens) == count
            assert np.all(np.diff(offs) >= 0)
