"""Python view of the CPU oracle.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module.  It loads liboracle.so (plain C, built by gcc from oracle.c; see
that file for every definition and its citation) through ctypes and marshals
numpy arrays.  It imports nothing from the GPU package.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _load(path=None):
    path = path or os.path.join(HERE, "liboracle.so")
    if not os.path.exists(path):
        from . import build as _b  # noqa: WPS433 - build only when absent
        _b.build(out=path)
    lib = C.CDLL(path)
    i64, i32, p = C.c_int64, C.c_int, C.c_void_p
    sig = {
        "orc_plan": (i64, [i64, i64, i64, p, p]),
        "orc_sum_i32": (None, [i32, i64, p, p]),
        "orc_max_i32": (None, [i32, i64, p, p]),
        "orc_sum_f32_f64": (None, [i32, i64, p, p]),
        "orc_sum_f32_f64_omp": (None, [i32, i64, p, p]),
        "orc_omp_threads": (i32, []),
        "orc_sum_f32_f32": (None, [i32, i64, p, i32, p]),
        "orc_max_f32": (None, [i32, i64, p, p]),
        "orc_bf16_decode": (C.c_double, [C.c_uint16]),
        "orc_bf16_encode": (C.c_uint16, [C.c_double]),
        "orc_sum_bf16_f64": (None, [i32, i64, p, p]),
        "orc_sum_bf16_f32": (None, [i32, i64, p, i32, p, p]),
        "orc_sum_bf16_hilo": (None, [i32, i64, p, i32, p, p]),
        "orc_max_bf16": (None, [i32, i64, p, p]),
        "orc_e4m3_decode": (C.c_double, [C.c_uint8]),
        "orc_e4m3_encode": (C.c_uint8, [C.c_double]),
        "orc_e4m3_pack": (None, [i64, p, p, p]),
        "orc_sum_e4m3_f64": (None, [i32, i64, p, p, p]),
        "orc_sum_e4m3_f32": (None, [i32, i64, p, p, i32, p, p, p]),
        "orc_e5m2_decode": (C.c_double, [C.c_uint8]),
        "orc_e5m2_encode": (C.c_uint8, [C.c_double]),
        "orc_e5m2_pack": (None, [i64, p, p, p]),
        "orc_sum_e5m2_f64": (None, [i32, i64, p, p, p]),
        "orc_sum_e5m2_f32": (None, [i32, i64, p, p, i32, p, p, p]),
        "orc_e8m0_decode": (C.c_double, [C.c_uint8]),
        "orc_mx_exponent": (i32, [C.c_float]),
        "orc_mx_pack": (None, [i64, p, p, p]),
        "orc_sum_mx_f64": (None, [i32, i64, p, p, p]),
        "orc_sum_mx_f32": (None, [i32, i64, p, p, i32, p, p, p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


class Oracle:
    """ctypes wrapper; every array argument is a C-contiguous numpy array."""

    def __init__(self, path=None):
        self.lib = _load(path)

    # ---- helpers -------------------------------------------------------
    @staticmethod
    def _ptr(a):
        return a.ctypes.data_as(C.c_void_p)

    def _ptrs(self, arrays, dtype):
        arrs = [np.ascontiguousarray(a, dtype=dtype) for a in arrays]
        n = len(arrs[0]) if arrs else 0
        for a in arrs:
            if a.ndim != 1 or len(a) != n:
                raise ValueError("rank arrays must be 1-D and equally long")
        tab = (C.c_void_p * max(len(arrs), 1))(
            *[a.ctypes.data for a in arrs])
        return arrs, tab, n

    # ---- partition plan (Algorithm 1 chunk rule) -----------------------
    def plan(self, count, nparts, align=1):
        off = np.zeros(nparts, np.int64)
        ln = np.zeros(nparts, np.int64)
        ps = self.lib.orc_plan(count, nparts, align, self._ptr(off),
                               self._ptr(ln))
        if ps < 0:
            raise ValueError("bad plan arguments")
        return int(ps), off, ln

    # ---- int32 ----------------------------------------------------------
    def sum_i32(self, xs):
        arrs, tab, n = self._ptrs(xs, np.int32)
        y = np.empty(n, np.int32)
        self.lib.orc_sum_i32(len(arrs), n, tab, self._ptr(y))
        return y

    def max_i32(self, xs):
        arrs, tab, n = self._ptrs(xs, np.int32)
        y = np.empty(n, np.int32)
        self.lib.orc_max_i32(len(arrs), n, tab, self._ptr(y))
        return y

    # ---- float32 ----------------------------------------------------------
    def sum_f32_f64(self, xs, threads=False):
        arrs, tab, n = self._ptrs(xs, np.float32)
        y = np.empty(n, np.float64)
        f = self.lib.orc_sum_f32_f64_omp if threads else self.lib.orc_sum_f32_f64
        f(len(arrs), n, tab, self._ptr(y))
        return y

    def omp_threads(self):
        return int(self.lib.orc_omp_threads())

    def sum_f32_f32(self, xs, comp=False):
        arrs, tab, n = self._ptrs(xs, np.float32)
        y = np.empty(n, np.float32)
        self.lib.orc_sum_f32_f32(len(arrs), n, tab, int(comp), self._ptr(y))
        return y

    def max_f32(self, xs):
        arrs, tab, n = self._ptrs(xs, np.float32)
        y = np.empty(n, np.float32)
        self.lib.orc_max_f32(len(arrs), n, tab, self._ptr(y))
        return y

    # ---- bfloat16 (payload = uint16 codes) ------------------------------
    def bf16_decode(self, h):
        return float(self.lib.orc_bf16_decode(int(h)))

    def bf16_encode(self, v):
        return int(self.lib.orc_bf16_encode(float(v)))

    def bf16_encode_array(self, x):
        x = np.asarray(x, dtype=np.float64).ravel()
        return np.fromiter((self.lib.orc_bf16_encode(float(v)) for v in x),
                           dtype=np.uint16, count=len(x))

    def bf16_decode_table(self):
        return np.array([self.lib.orc_bf16_decode(h) for h in range(1 << 16)],
                        dtype=np.float64)

    def sum_bf16_f64(self, xs):
        arrs, tab, n = self._ptrs(xs, np.uint16)
        y = np.empty(n, np.float64)
        self.lib.orc_sum_bf16_f64(len(arrs), n, tab, self._ptr(y))
        return y

    def sum_bf16_f32(self, xs, comp=False):
        """Returns (bf16 codes, binary32 sums before encoding)."""
        arrs, tab, n = self._ptrs(xs, np.uint16)
        y = np.empty(n, np.uint16)
        y32 = np.empty(n, np.float32)
        self.lib.orc_sum_bf16_f32(len(arrs), n, tab, int(comp), self._ptr(y),
                                  self._ptr(y32))
        return y, y32

    def sum_bf16_hilo(self, xs, comp=True):
        """Returns (hi, lo) bf16 codes: hi = bf16(y32), lo = bf16(y32 - hi)."""
        arrs, tab, n = self._ptrs(xs, np.uint16)
        hi = np.empty(n, np.uint16)
        lo = np.empty(n, np.uint16)
        self.lib.orc_sum_bf16_hilo(len(arrs), n, tab, int(comp),
                                   self._ptr(hi), self._ptr(lo))
        return hi, lo

    def max_bf16(self, xs):
        arrs, tab, n = self._ptrs(xs, np.uint16)
        y = np.empty(n, np.uint16)
        self.lib.orc_max_bf16(len(arrs), n, tab, self._ptr(y))
        return y

    # ---- e4m3 with per-256 FP32 scales ----------------------------------
    def e4m3_decode(self, q):
        return float(self.lib.orc_e4m3_decode(int(q)))

    def e4m3_encode(self, v):
        return int(self.lib.orc_e4m3_encode(float(v)))

    def e4m3_decode_table(self):
        return np.array([self.lib.orc_e4m3_decode(q) for q in range(256)],
                        dtype=np.float64)

    def e4m3_pack(self, x):
        x = np.ascontiguousarray(x, dtype=np.float32)
        n = len(x)
        q = np.empty(n, np.uint8)
        s = np.empty((n + 255) // 256, np.float32)
        self.lib.orc_e4m3_pack(n, self._ptr(x), self._ptr(q), self._ptr(s))
        return q, s

    def sum_e4m3_f64(self, qs, ss):
        arrs, tab, n = self._ptrs(qs, np.uint8)
        sarr, stab, _ = self._ptrs(ss, np.float32)
        y = np.empty(n, np.float64)
        self.lib.orc_sum_e4m3_f64(len(arrs), n, tab, stab, self._ptr(y))
        return y

    def sum_e4m3_f32(self, qs, ss, comp=True):
        """Returns (e4m3 codes, per-256 scales, binary32 sums)."""
        arrs, tab, n = self._ptrs(qs, np.uint8)
        sarr, stab, _ = self._ptrs(ss, np.float32)
        yq = np.empty(n, np.uint8)
        ys = np.empty((n + 255) // 256, np.float32)
        y32 = np.empty(n, np.float32)
        self.lib.orc_sum_e4m3_f32(len(arrs), n, tab, stab, int(comp),
                                  self._ptr(yq), self._ptr(ys),
                                  self._ptr(y32))
        return yq, ys, y32


    # ---- e5m2 with per-256 FP32 scales ----------------------------------
    def e5m2_decode(self, q):
        return float(self.lib.orc_e5m2_decode(int(q)))

    def e5m2_encode(self, v):
        return int(self.lib.orc_e5m2_encode(float(v)))

    def e5m2_decode_table(self):
        return np.array([self.lib.orc_e5m2_decode(q) for q in range(256)],
                        dtype=np.float64)

    def e5m2_pack(self, x):
        x = np.ascontiguousarray(x, dtype=np.float32)
        n = len(x)
        q = np.empty(n, np.uint8)
        s = np.empty((n + 255) // 256, np.float32)
        self.lib.orc_e5m2_pack(n, self._ptr(x), self._ptr(q), self._ptr(s))
        return q, s

    def sum_e5m2_f64(self, qs, ss):
        arrs, tab, n = self._ptrs(qs, np.uint8)
        sarr, stab, _ = self._ptrs(ss, np.float32)
        y = np.empty(n, np.float64)
        self.lib.orc_sum_e5m2_f64(len(arrs), n, tab, stab, self._ptr(y))
        return y

    def sum_e5m2_f32(self, qs, ss, comp=True):
        """Returns (e5m2 codes, per-256 scales, binary32 sums)."""
        arrs, tab, n = self._ptrs(qs, np.uint8)
        sarr, stab, _ = self._ptrs(ss, np.float32)
        yq = np.empty(n, np.uint8)
        ys = np.empty((n + 255) // 256, np.float32)
        y32 = np.empty(n, np.float32)
        self.lib.orc_sum_e5m2_f32(len(arrs), n, tab, stab, int(comp),
                                  self._ptr(yq), self._ptr(ys),
                                  self._ptr(y32))
        return yq, ys, y32

    # ---- MX blocks: e4m3 codes, one E8M0 scale byte per 32 elements ------
    def e8m0_decode(self, b):
        return float(self.lib.orc_e8m0_decode(int(b)))

    def mx_exponent(self, amax):
        return int(self.lib.orc_mx_exponent(float(amax)))

    def mx_pack(self, x):
        """Returns (e4m3 codes, E8M0 scale bytes, one per 32 elements)."""
        x = np.ascontiguousarray(x, dtype=np.float32)
        n = len(x)
        q = np.empty(n, np.uint8)
        sb = np.empty((n + 31) // 32, np.uint8)
        self.lib.orc_mx_pack(n, self._ptr(x), self._ptr(q), self._ptr(sb))
        return q, sb

    def mx_dequant(self, q, sb):
        """dec(q) * 2^(b - 127) per element, in double (exact)."""
        table = self.e4m3_decode_table()
        sc = np.array([self.e8m0_decode(b) for b in range(256)])
        q = np.asarray(q)
        return table[q] * np.repeat(sc[np.asarray(sb)], 32)[:len(q)]

    def sum_mx_f64(self, qs, sbs):
        arrs, tab, n = self._ptrs(qs, np.uint8)
        sarr, stab, _ = self._ptrs(sbs, np.uint8)
        y = np.empty(n, np.float64)
        self.lib.orc_sum_mx_f64(len(arrs), n, tab, stab, self._ptr(y))
        return y

    def sum_mx_f32(self, qs, sbs, comp=True):
        """Returns (e4m3 codes, E8M0 scale bytes, binary32 sums)."""
        arrs, tab, n = self._ptrs(qs, np.uint8)
        sarr, stab, _ = self._ptrs(sbs, np.uint8)
        yq = np.empty(n, np.uint8)
        ysb = np.empty((n + 31) // 32, np.uint8)
        y32 = np.empty(n, np.float32)
        self.lib.orc_sum_mx_f32(len(arrs), n, tab, stab, int(comp),
                                self._ptr(yq), self._ptr(ysb),
                                self._ptr(y32))
        return yq, ysb, y32



_DEFAULT = None


def get():
    """Process-wide oracle instance."""
    global _DEFAULT
    if _DEFAULT is None:
        _DEFAULT = Oracle()
    return _DEFAULT
