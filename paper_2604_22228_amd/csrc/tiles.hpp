// Tile reducers: one wavefront reduces `n` consecutive elements of one
// bucket, starting at element `e0`, over the P rank contributions, in rank
// order 0..P-1 per element (the operation is elementwise, so any split into
// tiles gives the same result, which is why partitions may be reduced in
// any arrival order).
//
// Layout: every rank buffer and output is 16-byte aligned and every
// partition starts on a 128-byte line of its bucket (partition lengths are
// planned in whole lines; 256 elements for the 8-bit floats), so a row of a
// 128-byte aligned buffer covers whole lines.  Each lane streams 16-byte vectors
// (dwordx4), 64 lanes cover 1 KiB per rank per step, and U steps are issued
// back to back so that U * P loads are in flight per lane before the first
// add.  Loads and stores carry the nontemporal hint: the data are touched
// once.  The ragged end (< 16 bytes) of a bucket is done element by element.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "layout.hpp"
#include "persistent.hpp"

namespace pcoll {
namespace dev {

// ------------------------------------------------------------ accumulators
// Float sum in binary32, plain or Sum2.  Non-finite values follow IEEE
// arithmetic; once the running sum is not finite the TwoSum errors are
// NaN, so the compensated result is the running sum itself (plain and
// compensated sums then agree).  FINITE: the inputs and sums are known to
// be finite (the 8-bit payloads), which spares that test.
template <bool COMP, bool FINITE = false>
struct FSum {
  float s, c;
  __device__ __forceinline__ void init(float v) { s = v; c = 0.0f; }
  __device__ __forceinline__ void add(float v) {
    if (COMP) {  // Sum2 (Ogita, Rump, Oishi 2005): carry the exact errors
      float e;
      two_sum(s, v, s, e);
      c = c + e;
    } else {
      s = s + v;
    }
  }
  __device__ __forceinline__ float get() const {
    if (!COMP) return s;
    if (FINITE) return s + c;
    return __builtin_isfinite(s) ? s + c : s;
  }
};

// Float max: the maximum operation of IEEE 754-2019 (NaN if any input is
// NaN, +0 above -0), one v_maximum3_f32 on gfx950.  It is commutative and
// associative, so the rank order does not change the result.
struct FMax {
  float m;
  __device__ __forceinline__ void init(float v) { m = v; }
  __device__ __forceinline__ void add(float v) {
    m = __builtin_elementwise_maximum(m, v);
  }
  __device__ __forceinline__ float get() const { return m; }
};

struct ISum {
  uint32_t s;  // two's-complement wrap
  __device__ __forceinline__ void init(uint32_t v) { s = v; }
  __device__ __forceinline__ void add(uint32_t v) { s = s + v; }
  __device__ __forceinline__ uint32_t get() const { return s; }
};

struct IMax {
  int32_t m;
  __device__ __forceinline__ void init(uint32_t v) { m = (int32_t)v; }
  __device__ __forceinline__ void add(uint32_t v) {
    m = (int32_t)v > m ? (int32_t)v : m;
  }
  __device__ __forceinline__ uint32_t get() const { return (uint32_t)m; }
};

// ------------------------------------------------------------------ codecs
// 32-bit words: the value is the word (float bits or int32).
struct Word32 {
  static constexpr int kPerVec = 4;
  static constexpr int kBytes = 4;
  using Val = uint32_t;
  __device__ __forceinline__ static uint32_t get(const uint4& v, int j) {
    return j == 0 ? v.x : (j == 1 ? v.y : (j == 2 ? v.z : v.w));
  }
};

__device__ __forceinline__ float as_f(uint32_t u) { return __uint_as_float(u); }

// bfloat16 -> float is exact (the upper half of a binary32).
__device__ __forceinline__ float bf16_to_f(uint32_t h) {
  return __uint_as_float(h << 16);
}
// Two floats -> a word of two bfloat16 codes (a in the low half), round
// to nearest even (ties to the even code, subnormals kept, overflow to
// infinity) with gfx950's v_cvt_pk_bf16_f32; every NaN becomes the quiet
// NaN 0x7FC0 (sign and payload dropped) by converting the quiet NaN of
// binary32 with an empty payload in its place.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t f_to_bf16x2(float a, float b) {
  const float qnan = __uint_as_float(0x7fc00000u);
  const f32x2_t v = {__builtin_isnan(a) ? qnan : a,
                     __builtin_isnan(b) ? qnan : b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}
__device__ __forceinline__ uint32_t f_to_bf16(float f) {
  return f_to_bf16x2(f, 0.0f) & 0xffffu;
}

// The two 8-bit formats: largest finite value (the block scale maps a
// block's amax onto it), the hardware decode of a code pair, and the encode
// of four values into one word (code j in byte j).  The gfx950 conversions
// round to nearest even, subnormals included, but do not saturate; values
// are clamped to +-kMax first, so that the encode saturates as the formats'
// definitions ask.
__device__ __forceinline__ float clamp_abs(float v, float m) {
  return __builtin_amdgcn_fmed3f(v, -m, m);
}

struct Fp8E4M3 {
  static constexpr float kMax = 448.0f;
  template <bool HI>
  __device__ __forceinline__ static auto dec_pair(uint32_t w) {
    return __builtin_amdgcn_cvt_pk_f32_fp8((int)w, HI);
  }
  __device__ __forceinline__ static uint32_t enc4(float a, float b, float c,
                                                  float d) {
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(clamp_abs(a, kMax),
                                            clamp_abs(b, kMax), 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(clamp_abs(c, kMax), clamp_abs(d, kMax),
                                        w, true);
    return (uint32_t)w;
  }
};
struct Fp8E5M2 {
  static constexpr float kMax = 57344.0f;
  template <bool HI>
  __device__ __forceinline__ static auto dec_pair(uint32_t w) {
    return __builtin_amdgcn_cvt_pk_f32_bf8((int)w, HI);
  }
  __device__ __forceinline__ static uint32_t enc4(float a, float b, float c,
                                                  float d) {
    int w = __builtin_amdgcn_cvt_pk_bf8_f32(clamp_abs(a, kMax),
                                            clamp_abs(b, kMax), 0, false);
    w = __builtin_amdgcn_cvt_pk_bf8_f32(clamp_abs(c, kMax), clamp_abs(d, kMax),
                                        w, true);
    return (uint32_t)w;
  }
};

// ---------------------------------------------------- 16-byte vector tiles
// Reduces one 16-byte vector per rank into one 16-byte output vector.
template <class Acc, int P, int Kind>
struct VecCombine;

// Kind 0: 32-bit float lanes; Kind 1: 32-bit int lanes; Kind 2: bf16 lanes.
template <class Acc, int P>
struct VecCombine<Acc, P, 0> {
  __device__ __forceinline__ static uint4 run(const uint4 (&x)[P]) {
    uint32_t o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      Acc a;
      a.init(as_f(Word32::get(x[0], j)));
#pragma unroll
      for (int r = 1; r < P; ++r) a.add(as_f(Word32::get(x[r], j)));
      o[j] = __float_as_uint(a.get());
    }
    return make_uint4(o[0], o[1], o[2], o[3]);
  }
};

template <class Acc, int P>
struct VecCombine<Acc, P, 1> {
  __device__ __forceinline__ static uint4 run(const uint4 (&x)[P]) {
    uint32_t o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      Acc a;
      a.init(Word32::get(x[0], j));
#pragma unroll
      for (int r = 1; r < P; ++r) a.add(Word32::get(x[r], j));
      o[j] = a.get();
    }
    return make_uint4(o[0], o[1], o[2], o[3]);
  }
};

template <class Acc, int P>
struct VecCombine<Acc, P, 2> {
  __device__ __forceinline__ static uint4 run(const uint4 (&x)[P]) {
    uint32_t o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      Acc lo, hi;
      uint32_t w = Word32::get(x[0], j);
      lo.init(bf16_to_f(w & 0xffffu));
      hi.init(bf16_to_f(w >> 16));
#pragma unroll
      for (int r = 1; r < P; ++r) {
        w = Word32::get(x[r], j);
        lo.add(bf16_to_f(w & 0xffffu));
        hi.add(bf16_to_f(w >> 16));
      }
      o[j] = f_to_bf16x2(lo.get(), hi.get());
    }
    return make_uint4(o[0], o[1], o[2], o[3]);
  }
};

// bf16 pair output of a binary32 sum y: hi = bf16(y), lo = bf16(y - hi).
// The difference is exact in binary32 (hi is y rounded to fewer bits in
// the same binade), so hi + lo carries y to 16 significant bits.  When hi
// is not finite (y is NaN, infinite or beyond bf16's range), lo = +0, so
// that hi + lo is hi.
__device__ __forceinline__ uint32_t bf16_pair(float y, uint32_t& lo) {
  const uint32_t hi = f_to_bf16(y);
  lo = (hi & 0x7f80u) == 0x7f80u ? 0u : f_to_bf16(y - bf16_to_f(hi));
  return hi;
}

// Kind 3: bf16 lanes in, the pair (hi, lo) out: run() returns the hi
// vector and leaves the lo vector in `low`.
template <class Acc, int P>
struct VecCombine<Acc, P, 3> {
  __device__ __forceinline__ static uint4 run(const uint4 (&x)[P],
                                              uint4& low) {
    uint32_t o[4], l[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      Acc a, b;
      uint32_t w = Word32::get(x[0], j);
      a.init(bf16_to_f(w & 0xffffu));
      b.init(bf16_to_f(w >> 16));
#pragma unroll
      for (int r = 1; r < P; ++r) {
        w = Word32::get(x[r], j);
        a.add(bf16_to_f(w & 0xffffu));
        b.add(bf16_to_f(w >> 16));
      }
      uint32_t la, lb;
      const uint32_t ha = bf16_pair(a.get(), la);
      const uint32_t hb = bf16_pair(b.get(), lb);
      o[j] = ha | (hb << 16);
      l[j] = la | (lb << 16);
    }
    low = make_uint4(l[0], l[1], l[2], l[3]);
    return make_uint4(o[0], o[1], o[2], o[3]);
  }
};

// Scalar path for the last (< 16 bytes) elements of a bucket.
template <class Acc, int P, int Kind>
__device__ __forceinline__ void combine_scalar(const char* const (&in)[P],
                                               char* out, char* out2,
                                               uint32_t i) {
  if (Kind == 3) {
    Acc a;
    a.init(bf16_to_f(reinterpret_cast<const uint16_t*>(in[0])[i]));
#pragma unroll
    for (int r = 1; r < P; ++r)
      a.add(bf16_to_f(reinterpret_cast<const uint16_t*>(in[r])[i]));
    uint32_t lo;
    reinterpret_cast<uint16_t*>(out)[i] = (uint16_t)bf16_pair(a.get(), lo);
    reinterpret_cast<uint16_t*>(out2)[i] = (uint16_t)lo;
  } else if (Kind == 2) {
    Acc a;
    a.init(bf16_to_f(reinterpret_cast<const uint16_t*>(in[0])[i]));
#pragma unroll
    for (int r = 1; r < P; ++r)
      a.add(bf16_to_f(reinterpret_cast<const uint16_t*>(in[r])[i]));
    reinterpret_cast<uint16_t*>(out)[i] = (uint16_t)f_to_bf16(a.get());
  } else if (Kind == 0) {
    Acc a;
    a.init(as_f(reinterpret_cast<const uint32_t*>(in[0])[i]));
#pragma unroll
    for (int r = 1; r < P; ++r)
      a.add(as_f(reinterpret_cast<const uint32_t*>(in[r])[i]));
    reinterpret_cast<uint32_t*>(out)[i] = __float_as_uint(a.get());
  } else {
    Acc a;
    a.init(reinterpret_cast<const uint32_t*>(in[0])[i]);
#pragma unroll
    for (int r = 1; r < P; ++r)
      a.add(reinterpret_cast<const uint32_t*>(in[r])[i]);
    reinterpret_cast<uint32_t*>(out)[i] = a.get();
  }
}

// Rows each lane loads at once: enough loads in flight, bounded register
// use.  DEEP (the default) keeps 4 rows in flight up to 8 ranks and 2 above
// (at 16 ranks 1.4 % faster than 1, with no spills); the shallow form keeps
// half of that from 3 ranks on, which needs fewer registers and leaves more
// room for kernels that run beside the reduction.
template <int P, bool DEEP>
struct Unroll {
  static constexpr int value = P <= 2 ? 4 : (P <= 8 ? (DEEP ? 4 : 2) : (DEEP ? 2 : 1));
};

// Rows of a tile.  A partition is cut into rows of 64 lanes x 16 bytes
// (kRowElems elements) and into nt tiles of rpt = ceil(rows / nt) rows;
// tile lt takes rows base + k * stride, k = 0, 1, ...
//  * consecutive layout (band 0): rows [lt rpt, (lt + 1) rpt);
//  * banded interleave (band B > 0): tiles are grouped into bands of B
//    consecutive tiles, band b owning rows [b B rpt, (b B + nb) rpt) (nb =
//    its tile count, B but the last), and tile j of the band takes every
//    nb-th row of it starting at row j.  The tiles running at the same time
//    (consecutive claims) then stream side by side through one band, and
//    each tile's rows stay within B rpt rows, so a tile touches few pages
//    whatever the partition's size.
struct RowSet {
  uint32_t base, stride, limit;  // rows base + k * stride, k < limit
  // nrows: rows this set may use (whole rows); rpt: ceil(all rows of the
  // partition / nt)
  __device__ __forceinline__ RowSet(uint32_t lt, uint32_t nt, uint32_t rpt,
                                    uint32_t band, uint32_t nrows) {
    if (band) {
      const uint32_t b = lt / band, j = lt - b * band;
      const uint32_t nb = min(band, nt - b * band);
      const uint32_t b0 = b * band * rpt;
      const uint32_t b1 = min(b0 + nb * rpt, nrows);
      base = b0 + j;
      stride = nb;
      limit = base < b1 ? (b1 - 1 - base) / nb + 1 : 0;
    } else {
      const uint32_t rows_per_tile = rpt;
      base = lt * rows_per_tile;
      stride = 1;
      limit = base < nrows ? min(rows_per_tile, nrows - base) : 0;
    }
  }
  __device__ __forceinline__ uint32_t row(uint32_t k) const {
    return base + k * stride;
  }
};

// Whether tile lt owns row q < nt * rpt (used for the ragged end of a
// partition), in the layout of RowSet.
__device__ __forceinline__ bool owns_row(uint32_t q, uint32_t lt, uint32_t nt,
                                         uint32_t rpt, uint32_t band) {
  if (!band) return q / rpt == lt;
  const uint64_t span = (uint64_t)band * rpt;  // rows of a full band
  const uint32_t b = (uint32_t)(q / span);
  const uint32_t nb = min(band, nt - b * band);
  return b * band + (uint32_t)(q - b * span) % nb == lt;
}

template <class Acc, int Kind, bool DEEP = true>
struct VecTile {
  static constexpr int kElemBytes = Kind >= 2 ? 2 : 4;
  static constexpr int kPerVec = 16 / kElemBytes;
  static constexpr uint32_t kRowElems = 64 * kPerVec;

  // Reduces wavefront `wave`'s rows of the tile: rows k = wave, wave +
  // nwaves, ... of the tile's row set; wavefront 0 also does the
  // partition's ragged end if this tile owns it.
  template <int P>
  __device__ __forceinline__ static void run(const_ptr<BucketDesc> bd,
                                             uint64_t poff, uint64_t plen,
                                             uint32_t lt, uint32_t nt,
                                             uint32_t inter, uint32_t wave,
                                             uint32_t nwaves) {
    const uint32_t lane = lane_id();
    const uint4* in[P];
#pragma unroll
    for (int r = 0; r < P; ++r)
      in[r] = reinterpret_cast<const uint4*>(
          static_cast<const char*>(bd->in[r]) + poff * kElemBytes);
    uint4* out = reinterpret_cast<uint4*>(static_cast<char*>(bd->out) +
                                          poff * kElemBytes);
    // Kind 3: the low halves of the pairs go to the second output
    uint4* out2 = Kind == 3 ? reinterpret_cast<uint4*>(
                                  static_cast<char*>(bd->out_scale) +
                                  poff * kElemBytes)
                            : nullptr;
    auto emit = [&](uint32_t v, const uint4(&xx)[P]) {
      if constexpr (Kind == 3) {
        uint4 low;
        st_stream(out + v, VecCombine<Acc, P, 3>::run(xx, low));
        st_stream(out2 + v, low);
      } else {
        st_stream(out + v, VecCombine<Acc, P, Kind>::run(xx));
      }
    };
    const uint32_t nv = (uint32_t)(plen / kPerVec);  // whole vectors
    const uint32_t full = nv / 64;                    // whole rows
    const uint32_t all = (uint32_t)((plen + kRowElems - 1) / kRowElems);
    const uint32_t rpt = (all + nt - 1) / nt;
    const RowSet rows(lt, nt, rpt, inter, full);
    // bf16 max holds more temporaries per value than the sums (the NaN
    // handling of IEEE maximum): at 4 rows in flight it would spill
    constexpr int U0 = Unroll<P, DEEP>::value;
    constexpr bool kBf16Max = Kind == 2 && std::is_same<Acc, FMax>::value;
    constexpr int U = kBf16Max && U0 > 2 ? 2 : U0;
    uint32_t k = wave;
    for (; k + (U - 1) * nwaves < rows.limit; k += U * nwaves) {
      uint4 x[U][P];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int r = 0; r < P; ++r)
          x[u][r] = ld_stream(in[r] + rows.row(k + u * nwaves) * 64u + lane);
#pragma unroll
      for (int u = 0; u < U; ++u) emit(rows.row(k + u * nwaves) * 64u + lane, x[u]);
    }
    for (; k < rows.limit; k += nwaves) {
      uint4 x[P];
      const uint32_t v = rows.row(k) * 64u + lane;
#pragma unroll
      for (int r = 0; r < P; ++r) x[r] = ld_stream(in[r] + v);
      emit(v, x);
    }
    // the partition's ragged end: a partial row and the last < 16 bytes,
    // done by the tile that owns row `full`
    if (wave != 0 || full >= all || !owns_row(full, lt, nt, rpt, inter))
      return;
    const uint32_t v = full * 64u + lane;
    if (v < nv) {
      uint4 x[P];
#pragma unroll
      for (int r = 0; r < P; ++r) x[r] = ld_stream(in[r] + v);
      emit(v, x);
    }
    const uint32_t tail = (uint32_t)(plen - (uint64_t)nv * kPerVec);
    if (lane < tail) {
      const char* inb[P];
#pragma unroll
      for (int r = 0; r < P; ++r) inb[r] = reinterpret_cast<const char*>(in[r]);
      combine_scalar<Acc, P, Kind>(inb, reinterpret_cast<char*>(out),
                                   reinterpret_cast<char*>(out2),
                                   nv * kPerVec + lane);
    }
  }
};

// ------------------------------------------------------ 8-bit float tiles
// Each lane owns 16 consecutive codes; a row of 16 lanes owns one block of
// 256 elements and its scale.  Inputs: y = sum_r fl(dec(q_r) * s_r) in
// binary32 (plain or Sum2), then per block amax = max |y|, s = fl(amax /
// max) (max = 448 for e4m3, 57344 for e5m2; s = 1 if that is not a normal
// number), codes enc(fl(y * fl(1/s))).
// Tiles start on block boundaries (tile and partition lengths are multiples
// of 256); only a bucket's last block can be short.
template <class Fmt>
__device__ __forceinline__ void dec16(const uint4& raw, float scale,
                                      float (&o)[16]) {
  const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    auto lo = Fmt::template dec_pair<false>(w[k]);
    auto hi = Fmt::template dec_pair<true>(w[k]);
    o[4 * k + 0] = lo[0] * scale;
    o[4 * k + 1] = lo[1] * scale;
    o[4 * k + 2] = hi[0] * scale;
    o[4 * k + 3] = hi[1] * scale;
  }
}

__device__ __forceinline__ uint4 load_codes(const uint8_t* p, uint32_t have) {
  if (have >= 16u) return ld_stream(reinterpret_cast<const uint4*>(p));
  uint32_t w[4] = {0u, 0u, 0u, 0u};
  for (uint32_t j = 0; j < have; ++j) w[j >> 2] |= (uint32_t)p[j] << (8 * (j & 3));
  return make_uint4(w[0], w[1], w[2], w[3]);
}

template <bool COMP, class Fmt>
struct Fp8Tile {
  static constexpr uint32_t kRowElems = 1024;  // 64 lanes x 16 codes

  // One row: lane `lane` owns codes el .. el + 16 of block blk.  FULL: the
  // whole row is inside the bucket (every lane has 16 codes), which spares
  // the per-lane length checks; otherwise `have` codes (0..16).
  template <int P, bool FULL>
  __device__ __forceinline__ static void row(const uint8_t* const (&in)[P],
                                             const float* const (&sc)[P],
                                             uint8_t* out, float* osc,
                                             uint32_t el, uint32_t have) {
    const uint32_t blk = el / 256u;
    uint4 raw[P];
    float s_in[P];
#pragma unroll
    for (int r = 0; r < P; ++r) {
      if (FULL) {
        raw[r] = ld_stream(reinterpret_cast<const uint4*>(in[r] + el));
        s_in[r] = sc[r][blk];
      } else {
        raw[r] = have ? load_codes(in[r] + el, have) : make_uint4(0, 0, 0, 0);
        s_in[r] = have ? sc[r][blk] : 0.0f;
      }
    }
    // every rank's codes and scale are requested before the first is used,
    // so that one memory latency covers the row
    if (FULL) __builtin_amdgcn_sched_barrier(0);
    FSum<COMP, true> acc[16];
    {
      float d[16];
      dec16<Fmt>(raw[0], s_in[0], d);
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j].init(d[j]);
    }
#pragma unroll
    for (int r = 1; r < P; ++r) {
      float d[16];
      dec16<Fmt>(raw[r], s_in[r], d);
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j].add(d[j]);
    }
    float y[16];
    float amax = 0.0f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      y[j] = acc[j].get();
      if (FULL || (uint32_t)j < have) amax = fmaxf(amax, fabsf(y[j]));
    }
    // max over the 16 lanes of the block
    amax = fmaxf(amax, __shfl_xor(amax, 8, 16));
    amax = fmaxf(amax, __shfl_xor(amax, 4, 16));
    amax = fmaxf(amax, __shfl_xor(amax, 2, 16));
    amax = fmaxf(amax, __shfl_xor(amax, 1, 16));
    float so = amax / Fmt::kMax;
    if (!(so >= 0x1p-126f)) so = 1.0f;
    const float inv = 1.0f / so;
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      w[k] = Fmt::enc4(y[4 * k] * inv, y[4 * k + 1] * inv, y[4 * k + 2] * inv,
                       y[4 * k + 3] * inv);
    if (FULL || have == 16u) {
      st_stream(reinterpret_cast<uint4*>(out + el),
                make_uint4(w[0], w[1], w[2], w[3]));
    } else if (have) {
      for (uint32_t j = 0; j < have; ++j)
        out[el + j] = (uint8_t)(w[j >> 2] >> (8 * (j & 3)));
    }
    if ((FULL || have) && (lane_id() & 15u) == 0u) osc[blk] = so;
  }

  template <int P>
  __device__ __forceinline__ static void run(const_ptr<BucketDesc> bd,
                                             uint64_t poff, uint64_t plen,
                                             uint32_t lt, uint32_t nt,
                                             uint32_t inter, uint32_t wave,
                                             uint32_t nwaves) {
    const uint32_t lane = lane_id();
    const uint8_t* in[P];
    const float* sc[P];
#pragma unroll
    for (int r = 0; r < P; ++r) {
      in[r] = static_cast<const uint8_t*>(bd->in[r]) + poff;
      sc[r] = static_cast<const float*>(bd->in_scale[r]) + poff / 256u;
    }
    uint8_t* out = static_cast<uint8_t*>(bd->out) + poff;
    float* osc = static_cast<float*>(bd->out_scale) + poff / 256u;
    const uint32_t n = (uint32_t)plen;
    const uint32_t nrows = (n + kRowElems - 1) / kRowElems;
    const RowSet rows(lt, nt, (nrows + nt - 1) / nt, inter, nrows);
    for (uint32_t k = wave; k < rows.limit; k += nwaves) {
      const uint32_t q = rows.row(k);
      const uint32_t el = q * kRowElems + lane * 16u;
      if ((q + 1u) * kRowElems <= n) {  // uniform: the row is whole
        row<P, true>(in, sc, out, osc, el, 16u);
      } else {
        const uint32_t have = el < n ? (n - el < 16u ? n - el : 16u) : 0u;
        row<P, false>(in, sc, out, osc, el, have);
      }
    }
  }
};

template <bool COMP>
using E4M3Tile = Fp8Tile<COMP, Fp8E4M3>;
template <bool COMP>
using E5M2Tile = Fp8Tile<COMP, Fp8E5M2>;

// ------------------------------------------------------------- MX blocks
// OCP MX blocks with e4m3 elements: 32 codes share one E8M0 scale byte b,
// the value of a code being dec(q) * 2^(b - 127) (exact in binary32).  The
// gfx950 scaled conversions take such a scale as a binary32 operand whose
// exponent field is b: v_cvt_scalef32_pk_f32_fp8 multiplies a decoded pair
// by 2^(b - 127), v_cvt_scalef32_pk_fp8_f32 divides a pair by it and rounds
// to nearest even (without saturating).
typedef float mx_f32x2 __attribute__((ext_vector_type(2)));
typedef short mx_i16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float e8m0_operand(uint32_t b) {
  return __uint_as_float(b << 23);
}

// Scale byte of a block whose largest magnitude is amax: e + 127 for the
// smallest e >= -127 with amax <= 448 * 2^e = 1.75 * 2^(e + 8).  For
// amax = f * 2^E (f in [1, 2)) that is e = E - 8 when f <= 1.75 (fraction
// field <= 0x600000), else E - 7; zero and subnormal amax (E < -126) give
// -127.  The codes of the block then never exceed 448 in magnitude.
__device__ __forceinline__ uint32_t mx_scale_byte(float amax) {
  const uint32_t u = __float_as_uint(amax);
  const int e = (int)(u >> 23) - 135 + ((u & 0x7fffffu) > 0x600000u ? 1 : 0);
  return u < 0x00800000u ? 0u : (uint32_t)(max(e, -127) + 127);
}

// 16 codes (one lane's half block) scaled by the operand of byte b.
__device__ __forceinline__ void mx_dec16(const uint4& raw, float scale,
                                         float (&o)[16]) {
  const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const mx_f32x2 lo =
        __builtin_amdgcn_cvt_scalef32_pk_f32_fp8(w[k], scale, false);
    const mx_f32x2 hi =
        __builtin_amdgcn_cvt_scalef32_pk_f32_fp8(w[k], scale, true);
    o[4 * k + 0] = lo[0];
    o[4 * k + 1] = lo[1];
    o[4 * k + 2] = hi[0];
    o[4 * k + 3] = hi[1];
  }
}

// Codes of y[0..16) / 2^(b - 127), four per word (code j in byte j).
__device__ __forceinline__ uint4 mx_enc16(const float (&y)[16], float scale) {
  uint32_t w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    mx_i16x2 t = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(
        mx_i16x2{0, 0}, y[4 * k], y[4 * k + 1], scale, false);
    t = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(t, y[4 * k + 2],
                                                 y[4 * k + 3], scale, true);
    w[k] = __builtin_bit_cast(uint32_t, t);
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// 4 codes (a dword, first value in the low byte) scaled by the operand.
__device__ __forceinline__ uint32_t mx_enc4(const float (&y)[4], float scale) {
  mx_i16x2 t = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(mx_i16x2{0, 0}, y[0],
                                                        y[1], scale, false);
  t = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(t, y[2], y[3], scale, true);
  return __builtin_bit_cast(uint32_t, t);
}

// Largest magnitude over a pair of lanes (2j, 2j + 1): one block.
__device__ __forceinline__ float pair_max(float v) {
  const int o = __builtin_amdgcn_mov_dpp(__float_as_int(v), 0xb1, 0xf, 0xf,
                                         false);  // quad_perm [1, 0, 3, 2]
  return fmaxf(v, __int_as_float(o));
}

// Each lane owns 16 consecutive codes, half of a block; lanes 2j and 2j + 1
// of a row share block j and its scale byte.  y = sum_r dec(q_r) *
// 2^(b_r - 127) in binary32 (plain or Sum2), per block the scale byte of
// max |y| (mx_scale_byte), codes RNE(y / 2^(b - 127)).  Partitions start on
// block boundaries (their lengths are multiples of 32); only a bucket's
// last block can be short.
template <bool COMP>
struct MxTile {
  static constexpr uint32_t kRowElems = 1024;  // 64 lanes x 16 codes

  template <int P, bool FULL>
  __device__ __forceinline__ static void row(const uint8_t* const (&in)[P],
                                             const uint8_t* const (&sc)[P],
                                             uint8_t* out, uint8_t* osc,
                                             uint32_t el, uint32_t have) {
    const uint32_t blk = el / 32u;
    uint4 raw[P];
    uint32_t b_in[P];
#pragma unroll
    for (int r = 0; r < P; ++r) {
      if (FULL) {
        raw[r] = ld_stream(reinterpret_cast<const uint4*>(in[r] + el));
        b_in[r] = sc[r][blk];
      } else {
        raw[r] = have ? load_codes(in[r] + el, have) : make_uint4(0, 0, 0, 0);
        b_in[r] = have ? sc[r][blk] : 0u;
      }
    }
    if (FULL) __builtin_amdgcn_sched_barrier(0);
    FSum<COMP, true> acc[16];
    {
      float d[16];
      mx_dec16(raw[0], e8m0_operand(b_in[0]), d);
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j].init(d[j]);
    }
#pragma unroll
    for (int r = 1; r < P; ++r) {
      float d[16];
      mx_dec16(raw[r], e8m0_operand(b_in[r]), d);
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j].add(d[j]);
    }
    float y[16];
    float amax = 0.0f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      y[j] = acc[j].get();
      if (FULL || (uint32_t)j < have) amax = fmaxf(amax, fabsf(y[j]));
    }
    amax = pair_max(amax);
    const uint32_t b = mx_scale_byte(amax);
    const uint4 codes = mx_enc16(y, e8m0_operand(b));
    if (FULL || have == 16u) {
      st_stream(reinterpret_cast<uint4*>(out + el), codes);
    } else if (have) {
      const uint32_t w[4] = {codes.x, codes.y, codes.z, codes.w};
      for (uint32_t j = 0; j < have; ++j)
        out[el + j] = (uint8_t)(w[j >> 2] >> (8 * (j & 3)));
    }
    if ((FULL || have) && (lane_id() & 1u) == 0u) osc[blk] = (uint8_t)b;
  }

  template <int P>
  __device__ __forceinline__ static void run(const_ptr<BucketDesc> bd,
                                             uint64_t poff, uint64_t plen,
                                             uint32_t lt, uint32_t nt,
                                             uint32_t inter, uint32_t wave,
                                             uint32_t nwaves) {
    const uint32_t lane = lane_id();
    const uint8_t* in[P];
    const uint8_t* sc[P];
#pragma unroll
    for (int r = 0; r < P; ++r) {
      in[r] = static_cast<const uint8_t*>(bd->in[r]) + poff;
      sc[r] = static_cast<const uint8_t*>(bd->in_scale[r]) + poff / 32u;
    }
    uint8_t* out = static_cast<uint8_t*>(bd->out) + poff;
    uint8_t* osc = static_cast<uint8_t*>(bd->out_scale) + poff / 32u;
    const uint32_t n = (uint32_t)plen;
    const uint32_t nrows = (n + kRowElems - 1) / kRowElems;
    const RowSet rows(lt, nt, (nrows + nt - 1) / nt, inter, nrows);
    for (uint32_t k = wave; k < rows.limit; k += nwaves) {
      const uint32_t q = rows.row(k);
      const uint32_t el = q * kRowElems + lane * 16u;
      if ((q + 1u) * kRowElems <= n) {  // uniform: the row is whole
        row<P, true>(in, sc, out, osc, el, 16u);
      } else {
        const uint32_t have = el < n ? (n - el < 16u ? n - el : 16u) : 0u;
        row<P, false>(in, sc, out, osc, el, have);
      }
    }
  }
};

}  // namespace dev
}  // namespace pcoll
