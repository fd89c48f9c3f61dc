"""Python binding of libpcoll.so: argument marshalling only.

Every function here has the name of the C entry point it calls (see
include/pcoll.h for the semantics); non-zero return codes raise PcollError.
All reduction work runs in the library's gfx950 kernels.  There is no
fallback: if libpcoll.so is missing or cannot be loaded, load() raises.

torch is used only for device memory and streams: `Request` keeps the bound
tensors alive and passes their data pointers and the stream handle.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcoll.so")

INT32, FLOAT32, BFLOAT16, FP8_E4M3, FP8_E5M2, MXFP8_E4M3 = 0, 1, 2, 3, 4, 5
BF16_PAIR = 6  # bf16 in, (hi, lo) bf16 pair out
SUM, MAX = 0, 1

SUCCESS = 0
ERR_ARG, ERR_STATE, ERR_UNSUPPORTED, ERR_HIP = -1, -2, -3, -4
ERR_TIMEOUT, ERR_NOMEM, ERR_ABORTED = -5, -6, -7
MAX_RANKS = 16
NOALLOC_MAX_PARTS = 4096  # PCOLL_NOALLOC_MAX_PARTS

ELEM_BYTES = {INT32: 4, FLOAT32: 4, BFLOAT16: 2, FP8_E4M3: 1, FP8_E5M2: 1,
              MXFP8_E4M3: 1, BF16_PAIR: 2}


class PcollError(RuntimeError):
    def __init__(self, code, call, detail):
        super().__init__(f"{call} failed with {code}: {detail}")
        self.code = code


class Config(C.Structure):
    _fields_ = [("tile_elems", C.c_int), ("min_tile_elems", C.c_int),
                ("groups", C.c_int),
                ("groups_per_cu", C.c_int), ("comp", C.c_int),
                ("graph", C.c_int), ("timeout_ms", C.c_int),
                ("debug", C.c_int), ("interleave", C.c_int),
                ("group_waves", C.c_int), ("publish_batch", C.c_int),
                ("guide", C.c_int), ("unroll", C.c_int),
                ("producers", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Stats(C.Structure):
    _fields_ = [("epochs", C.c_uint64), ("graph_launches", C.c_uint64),
                ("graph_captures", C.c_uint64), ("cache_hits", C.c_uint64),
                ("cache_misses", C.c_uint64),
                ("cache_evictions", C.c_uint64),
                ("last_capture_ms", C.c_double),
                ("last_instantiate_ms", C.c_double),
                ("last_kernel_ms", C.c_float),
                ("kernel_ms_total", C.c_double),
                ("kernel_timed", C.c_uint64), ("groups", C.c_int),
                ("group_waves", C.c_int), ("unroll", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_p, _i, _sz = C.c_void_p, C.c_int, C.c_size_t
_SIGS = {
    "pcoll_init": [_sz, _i, _i, _i, _i, C.POINTER(_p)],
    "pcoll_init_batch": [_i, C.POINTER(_sz), _i, _i, _i, _i, C.POINTER(_p)],
    "pcoll_bind": [_p, C.POINTER(_p), C.POINTER(_p), C.POINTER(_p),
                   C.POINTER(_p), _p],
    "pcoll_start": [_p],
    "pcoll_pready": [_p, _i],
    "pcoll_pready_range": [_p, _i, _i],
    "pcoll_pready_list": [_p, _i, C.POINTER(_i)],
    "pcoll_pready_on_stream": [_p, _p, _i, _p],
    "pcoll_pready_rank": [_p, _i, _i],
    "pcoll_pready_rank_on_stream": [_p, _i, _p, _i, _p],
    "pcoll_parrived": [_p, _i, C.POINTER(_i)],
    "pcoll_test": [_p, C.POINTER(_i)],
    "pcoll_wait": [_p],
    "pcoll_wait_timeout": [_p, _i],
    "pcoll_wait_on_stream": [_p, _p],
    "pcoll_free": [_p],
    "pcoll_strerror": [_i],
    "pcoll_last_error_detail": [],
    "pcoll_get_config": [_p, C.POINTER(Config)],
    "pcoll_set_config": [_p, C.POINTER(Config)],
    "pcoll_num_parts": [_p, C.POINTER(_i)],
    "pcoll_part_info": [_p, _i, C.POINTER(_i), C.POINTER(_sz),
                        C.POINTER(_sz)],
    "pcoll_get_stats": [_p, C.POINTER(Stats)],
    "pcoll_debug_tile_hits": [_p, C.POINTER(C.c_uint32),
                              C.POINTER(C.c_uint32), _i],
    "pcoll_debug_set_epoch": [_p, C.c_uint32],
    "pcoll_debug_trace": [_p, C.POINTER(C.c_uint64), _i, C.POINTER(_i),
                          C.POINTER(_i)],
    "pcoll_reduce_noalloc": [_sz, _i, _i, _i, _i, C.POINTER(_p), _p,
                             C.POINTER(_p), _p, _p],
    "pcoll_plan": [_sz, _i, _i, C.POINTER(_sz), C.POINTER(_sz),
                   C.POINTER(_sz)],
    "pcoll_pack_bf16": [_p, _p, _sz, _p],
    "pcoll_pack_fp8": [_p, _p, _p, _sz, _p],
    "pcoll_pack_e5m2": [_p, _p, _p, _sz, _p],
    "pcoll_pack_mxfp8": [_p, _p, _p, _sz, _p],
    "pcoll_probe_copy": [_p, _p, _sz, _p],
    "pcoll_probe_fill": [_p, _sz, C.c_uint32, _p],
    "pcoll_probe_stream": [C.POINTER(_p), _i, _p, _sz, _i, _i, _p],
    "pcoll_device_info": [C.POINTER(_i), C.POINTER(_i), C.c_char_p, _i],
    "pcoll_version": [],
}

_LIB = None


def load(path=None):
    """Loads libpcoll.so (built by paper_2604_22228_amd/build.py).  Raises if
    it is absent: there is no other implementation to fall back to."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() "
                           "or python paper_2604_22228_amd/build.py")
    lib = C.CDLL(path)
    for name, args in _SIGS.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_char_p if name in ("pcoll_strerror",
                                           "pcoll_last_error_detail") else _i
    if path == LIB_PATH:
        _LIB = lib
    return lib


def _check(rc, call):
    if rc != SUCCESS:
        lib = load()
        detail = lib.pcoll_strerror(rc).decode()
        if rc == ERR_HIP:
            detail = lib.pcoll_last_error_detail().decode() or detail
        raise PcollError(rc, call, detail)
    return rc


def _ptr(x):
    """Device address of a tensor, an int address, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(s):
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


# ---- the C entry points, one to one ---------------------------------------
def pcoll_init(count, dtype, op, nparts, nranks):
    h = _p()
    _check(load().pcoll_init(count, dtype, op, nparts, nranks, C.byref(h)),
           "pcoll_init")
    return h


def pcoll_init_batch(counts, dtype, op, nparts_per_bucket, nranks):
    arr = (_sz * len(counts))(*counts)
    h = _p()
    _check(load().pcoll_init_batch(len(counts), arr, dtype, op,
                                   nparts_per_bucket, nranks, C.byref(h)),
           "pcoll_init_batch")
    return h


def pcoll_bind(h, rank_bufs, outs, rank_scales=None, out_scales=None,
               stream=None):
    rb = (_p * len(rank_bufs))(*[_ptr(x) for x in rank_bufs])
    ob = (_p * len(outs))(*[_ptr(x) for x in outs])
    rs = (_p * len(rank_scales))(*[_ptr(x) for x in rank_scales]) \
        if rank_scales is not None else None
    os_ = (_p * len(out_scales))(*[_ptr(x) for x in out_scales]) \
        if out_scales is not None else None
    _check(load().pcoll_bind(h, rb, ob, rs, os_, _stream(stream)),
           "pcoll_bind")


def pcoll_start(h):
    _check(load().pcoll_start(h), "pcoll_start")


def pcoll_pready(h, part):
    _check(load().pcoll_pready(h, part), "pcoll_pready")


def pcoll_pready_range(h, first, last):
    _check(load().pcoll_pready_range(h, first, last), "pcoll_pready_range")


def pcoll_pready_list(h, parts):
    """parts: a sequence of ints, or (zero-copy) a contiguous int32 numpy
    array or ctypes int array."""
    if isinstance(parts, np.ndarray):
        if parts.dtype != np.int32 or not parts.flags.c_contiguous:
            parts = np.ascontiguousarray(parts, dtype=np.int32)
        n, arr = parts.size, parts.ctypes.data_as(C.POINTER(_i))
    elif isinstance(parts, C.Array):
        n, arr = len(parts), parts
    else:
        n = len(parts)
        arr = (_i * n)(*[int(p) for p in parts])
    _check(load().pcoll_pready_list(h, n, arr), "pcoll_pready_list")


def pcoll_pready_on_stream(h, parts_dev, n, stream):
    _check(load().pcoll_pready_on_stream(h, _ptr(parts_dev), n,
                                         _stream(stream)),
           "pcoll_pready_on_stream")


def pcoll_pready_rank(h, rank, part):
    _check(load().pcoll_pready_rank(h, rank, part), "pcoll_pready_rank")


def pcoll_pready_rank_on_stream(h, rank, parts_dev, n, stream):
    _check(load().pcoll_pready_rank_on_stream(h, rank, _ptr(parts_dev), n,
                                              _stream(stream)),
           "pcoll_pready_rank_on_stream")


def pcoll_parrived(h, part):
    f = _i()
    _check(load().pcoll_parrived(h, part, C.byref(f)), "pcoll_parrived")
    return bool(f.value)


def pcoll_test(h):
    f = _i()
    _check(load().pcoll_test(h, C.byref(f)), "pcoll_test")
    return bool(f.value)


def pcoll_wait(h):
    _check(load().pcoll_wait(h), "pcoll_wait")


def pcoll_wait_timeout(h, ms):
    _check(load().pcoll_wait_timeout(h, ms), "pcoll_wait_timeout")


def pcoll_wait_on_stream(h, stream):
    _check(load().pcoll_wait_on_stream(h, _stream(stream)),
           "pcoll_wait_on_stream")


def pcoll_free(h):
    _check(load().pcoll_free(h), "pcoll_free")


def pcoll_get_config(h):
    c = Config()
    _check(load().pcoll_get_config(h, C.byref(c)), "pcoll_get_config")
    return c


def pcoll_set_config(h, cfg):
    _check(load().pcoll_set_config(h, C.byref(cfg)), "pcoll_set_config")


def pcoll_num_parts(h):
    n = _i()
    _check(load().pcoll_num_parts(h, C.byref(n)), "pcoll_num_parts")
    return n.value


def pcoll_part_info(h, part):
    b, o, n = _i(), _sz(), _sz()
    _check(load().pcoll_part_info(h, part, C.byref(b), C.byref(o),
                                  C.byref(n)), "pcoll_part_info")
    return b.value, o.value, n.value


def pcoll_get_stats(h):
    s = Stats()
    _check(load().pcoll_get_stats(h, C.byref(s)), "pcoll_get_stats")
    return s


def pcoll_debug_tile_hits(h, n):
    hits = (C.c_uint32 * n)()
    tiles = (C.c_uint32 * n)()
    _check(load().pcoll_debug_tile_hits(h, hits, tiles, n),
           "pcoll_debug_tile_hits")
    return list(hits), list(tiles)


def pcoll_debug_trace(h, max_groups=4096):
    """(stamps as a list of (start, first tile, end, tiles) per workgroup,
    wall-clock kHz) of the last epoch."""
    buf = (C.c_uint64 * (4 * max_groups))()
    g, khz = _i(), _i()
    _check(load().pcoll_debug_trace(h, buf, 4 * max_groups, C.byref(g),
                                    C.byref(khz)), "pcoll_debug_trace")
    n = min(g.value, max_groups)
    return [tuple(buf[4 * i:4 * i + 4]) for i in range(n)], khz.value


def pcoll_debug_set_epoch(h, last):
    _check(load().pcoll_debug_set_epoch(h, last), "pcoll_debug_set_epoch")


def pcoll_reduce_noalloc(count, dtype, op, nparts, rank_bufs, out,
                         rank_scales=None, out_scale=None, stream=None):
    bufs = (_p * len(rank_bufs))(*[_ptr(b) for b in rank_bufs])
    scales = None if rank_scales is None else \
        (_p * len(rank_scales))(*[_ptr(s) for s in rank_scales])
    _check(load().pcoll_reduce_noalloc(count, dtype, op, nparts,
                                       len(rank_bufs), bufs, _ptr(out), scales,
                                       _ptr(out_scale), _stream(stream)),
           "pcoll_reduce_noalloc")


def pcoll_plan(count, dtype, nparts):
    ps = _sz()
    offs = (_sz * nparts)()
    lens = (_sz * nparts)()
    _check(load().pcoll_plan(count, dtype, nparts, C.byref(ps), offs, lens),
           "pcoll_plan")
    return ps.value, list(offs), list(lens)


def pcoll_pack_bf16(src, dst, n, stream=None):
    _check(load().pcoll_pack_bf16(_ptr(src), _ptr(dst), n, _stream(stream)),
           "pcoll_pack_bf16")


def pcoll_pack_fp8(src, dst, scales, n, stream=None):
    _check(load().pcoll_pack_fp8(_ptr(src), _ptr(dst), _ptr(scales), n,
                                 _stream(stream)), "pcoll_pack_fp8")


def pcoll_pack_e5m2(src, dst, scales, n, stream=None):
    _check(load().pcoll_pack_e5m2(_ptr(src), _ptr(dst), _ptr(scales), n,
                                  _stream(stream)), "pcoll_pack_e5m2")


def pcoll_pack_mxfp8(src, dst, scales, n, stream=None):
    """MX blocks: e4m3 codes to dst, one E8M0 scale byte per 32 elements
    to scales (uint8)."""
    _check(load().pcoll_pack_mxfp8(_ptr(src), _ptr(dst), _ptr(scales), n,
                                   _stream(stream)), "pcoll_pack_mxfp8")


def pcoll_probe_copy(dst, src, nbytes, stream=None):
    _check(load().pcoll_probe_copy(_ptr(dst), _ptr(src), nbytes,
                                   _stream(stream)), "pcoll_probe_copy")


def pcoll_probe_stream(srcs, dst, nbytes, write, layout=0, stream=None):
    arr = (_p * len(srcs))(*[_ptr(s) for s in srcs])
    _check(load().pcoll_probe_stream(arr, len(srcs), _ptr(dst), nbytes,
                                     int(write), int(layout), _stream(stream)),
           "pcoll_probe_stream")


def pcoll_probe_fill(dst, nbytes, value, stream=None):
    _check(load().pcoll_probe_fill(_ptr(dst), nbytes, value,
                                   _stream(stream)), "pcoll_probe_fill")


def pcoll_device_info():
    cus, khz = _i(), _i()
    arch = C.create_string_buffer(64)
    _check(load().pcoll_device_info(C.byref(cus), C.byref(khz), arch, 64),
           "pcoll_device_info")
    return {"compute_units": cus.value, "wall_clock_khz": khz.value,
            "arch": arch.value.decode()}


def pcoll_version():
    return load().pcoll_version()


def pcoll_strerror(code):
    return load().pcoll_strerror(code).decode()


def pcoll_last_error_detail():
    return load().pcoll_last_error_detail().decode()


# ---- convenience wrapper ---------------------------------------------------
class Request:
    """A persistent partitioned-reduction request bound to torch tensors.

    bind(): rank_bufs, a list of per-bucket lists of P rank tensors (one
    bucket for the plain form); outs, one output tensor per bucket; for the
    8-bit dtypes also rank_scales (per bucket, per rank) and out_scales (per
    bucket): binary32 per 256 elements, or E8M0 bytes per 32 for MX blocks;
    for BF16_PAIR out_scales holds the lo output of each bucket.  The
    tensors are kept referenced while bound."""

    def __init__(self, counts, dtype, op, nparts, nranks, batched=None):
        self.counts = list(counts)
        self.dtype, self.op = dtype, op
        self.nparts, self.nranks = nparts, nranks
        if batched is None:
            batched = len(self.counts) > 1
        if batched:
            self.h = pcoll_init_batch(self.counts, dtype, op, nparts, nranks)
        else:
            self.h = pcoll_init(self.counts[0], dtype, op, nparts, nranks)
        self._keep = None
        self.nparts_total = pcoll_num_parts(self.h)

    def bind(self, rank_bufs, outs, rank_scales=None, out_scales=None,
             stream=None):
        flat = [t for bucket in rank_bufs for t in bucket]
        sflat = ([t for bucket in rank_scales for t in bucket]
                 if rank_scales is not None else None)
        pcoll_bind(self.h, flat, outs, sflat, out_scales, stream)
        self._keep = (flat, list(outs), sflat, out_scales, stream)

    def config(self):
        return pcoll_get_config(self.h)

    def set_config(self, **kw):
        c = pcoll_get_config(self.h)
        for k, v in kw.items():
            setattr(c, k, int(v))
        pcoll_set_config(self.h, c)

    def start(self):
        pcoll_start(self.h)

    def pready(self, part):
        pcoll_pready(self.h, part)

    def pready_range(self, first, last):
        pcoll_pready_range(self.h, first, last)

    def pready_list(self, parts):
        pcoll_pready_list(self.h, parts)

    def pready_on_stream(self, parts_dev, n, stream):
        pcoll_pready_on_stream(self.h, parts_dev, n, stream)

    def pready_rank(self, rank, part):
        pcoll_pready_rank(self.h, rank, part)

    def pready_rank_on_stream(self, rank, parts_dev, n, stream):
        pcoll_pready_rank_on_stream(self.h, rank, parts_dev, n, stream)

    def parrived(self, part):
        return pcoll_parrived(self.h, part)

    def test(self):
        return pcoll_test(self.h)

    def wait(self):
        pcoll_wait(self.h)

    def wait_timeout(self, ms):
        pcoll_wait_timeout(self.h, ms)

    def wait_on_stream(self, stream):
        pcoll_wait_on_stream(self.h, stream)

    def part_info(self, part):
        return pcoll_part_info(self.h, part)

    def stats(self):
        return pcoll_get_stats(self.h)

    def tile_hits(self):
        return pcoll_debug_tile_hits(self.h, self.nparts_total)

    def debug_set_epoch(self, last):
        pcoll_debug_set_epoch(self.h, last)

    def free(self):
        if self.h is not None:
            pcoll_free(self.h)
            self.h = None
            self._keep = None

    def __del__(self):
        try:
            self.free()
        except Exception:  # noqa: BLE001 - never raise from a finalizer
            pass
