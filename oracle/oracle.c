/*
 * CPU oracle for the partitioned reduction.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The GPU library never links, includes or calls it,
 * and this file includes nothing from the GPU library: the two share no code.
 *
 * What it computes.  P rank contributions x_0..x_{P-1} of a message of n
 * elements are combined elementwise, y[i] = x_0[i] (op) x_1[i] (op) ...
 * (op) x_{P-1}[i], with op = sum or max.  The paper names this collective
 * (Allreduce) only as the target of future work (Section 6) and fixes none of
 * its arithmetic; the definitions below are the plain mathematical ones:
 *
 *   - int32 sum: two's-complement wrap, computed in uint32 (no C overflow UB).
 *   - int32 max: the largest input (exact; the result is an input).
 *   - float max: the maximum operation of IEEE 754-2019 (clause 9.6): NaN if
 *     any input is NaN, otherwise the largest input, with +0 counted larger
 *     than -0.  It is commutative and associative, so the result does not
 *     depend on rank order.  A NaN result of a bf16 output is encoded as the
 *     quiet NaN 0x7FC0 (see orc_bf16_encode).
 *   - float sum, FP64 reference: every input decoded exactly to double, then
 *     summed left to right in rank order 0..P-1 in double.
 *   - float sum, FP32 mirror: the same left-to-right order in binary32
 *     (plain), or Sum2 of Ogita, Rump and Oishi (SIAM J. Sci. Comput. 26(6),
 *     2005, Algorithm 4.4) built on Knuth's TwoSum (TAOCP vol. 2, 4.2.2), in
 *     binary32 (compensated).  These fix the integer decisions of the encoded
 *     outputs (bf16 / e4m3 codes) in the precision the kernel takes them in.
 *     Non-finite values follow IEEE arithmetic (an infinity absorbs finite
 *     terms, opposite infinities give NaN, NaN propagates).  Sum2's
 *     correction has no meaning once the running sum is not finite, so the
 *     compensated sum then returns the running sum itself: plain and
 *     compensated sums agree whenever the result is not finite.
 *
 * The partition plan follows the chunk rule of Algorithm 1 (Section 4.3):
 * every chunk is ceil(size / max_chunks) long, offsets are fixed in advance by
 * running sums, and the last chunk is clipped; Section 4.5 (Ordering
 * Guarantee) requires the chunks to be disjoint destination regions.
 *
 * Codecs are written from the format definitions, not from bit tricks:
 *   - bfloat16: 1 sign, 8 exponent (bias 127), 7 fraction bits; RNE.
 *   - e4m3 (OCP 8-bit floating point, "E4M3FN"): 1 sign, 4 exponent (bias 7),
 *     3 fraction bits; no infinities; S.1111.111 is NaN; max 448; subnormal
 *     quantum 2^-9.  Encoding rounds to nearest, ties to even, and saturates.
 *   - e5m2 (OCP 8-bit floating point, "E5M2"): 1 sign, 5 exponent (bias 15),
 *     2 fraction bits; S.11111.00 is infinity, S.11111.xx (xx != 0) NaN; max
 *     57344; subnormal quantum 2^-16.  Encoding rounds to nearest, ties to
 *     even, and saturates at +-57344.
 *   - MX blocks (OCP Microscaling Formats v1.0, MXFP8 with E4M3 elements):
 *     blocks of 32 e4m3 codes share one E8M0 scale byte b, which stands for
 *     2^(b - 127) (b = 255 is NaN).  A value is dec(q) * 2^(b - 127), exact
 *     in binary32.  The shared exponent of a block is read here as the
 *     smallest e >= -127 with max |x| <= 448 * 2^e, so that no code of the
 *     block saturates (parity pinned by closed forms and brute force).
 *
 * Build with -O2 -ffp-contract=off and SSE2 arithmetic (no x87, no fast-math)
 * so that every float / double operation is one IEEE-754 RNE operation.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "oracle.h"

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Partition plan (Algorithm 1 chunk rule; Section 4.5 disjointness)   */
/* ------------------------------------------------------------------ */

int64_t orc_plan(int64_t count, int64_t nparts, int64_t align, int64_t *off,
                 int64_t *len) {
  if (count < 0 || nparts < 1 || align < 1) return -1;
  /* chunk length: ceil(count / nparts), then rounded up to a multiple of
   * `align` elements (align = 1 reproduces Algorithm 1 exactly). */
  int64_t psize = (count + nparts - 1) / nparts;
  psize = ((psize + align - 1) / align) * align;
  int64_t sent = 0; /* running offset, as `sent_data` in Algorithm 1 */
  for (int64_t k = 0; k < nparts; ++k) {
    int64_t l = count - sent;
    if (l > psize) l = psize;
    if (l < 0) l = 0;
    off[k] = sent < count ? sent : count;
    len[k] = l;
    sent += l;
  }
  return psize;
}

/* ------------------------------------------------------------------ */
/* int32                                                               */
/* ------------------------------------------------------------------ */

void orc_sum_i32(int P, int64_t n, const int32_t *const *x, int32_t *y) {
  for (int64_t i = 0; i < n; ++i) {
    uint32_t acc = 0u;
    for (int r = 0; r < P; ++r) acc += (uint32_t)x[r][i]; /* mod 2^32 */
    y[i] = (int32_t)acc; /* two's complement on every supported target */
  }
}

void orc_max_i32(int P, int64_t n, const int32_t *const *x, int32_t *y) {
  for (int64_t i = 0; i < n; ++i) {
    int32_t m = x[0][i];
    for (int r = 1; r < P; ++r)
      if (x[r][i] > m) m = x[r][i];
    y[i] = m;
  }
}

/* ------------------------------------------------------------------ */
/* float32 payloads                                                    */
/* ------------------------------------------------------------------ */

void orc_sum_f32_f64(int P, int64_t n, const float *const *x, double *y) {
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int r = 0; r < P; ++r) acc += (double)x[r][i];
    y[i] = acc;
  }
}

void orc_sum_f32_f64_omp(int P, int64_t n, const float *const *x, double *y) {
  /* Same per-element arithmetic as orc_sum_f32_f64; elements are split over
   * threads, so the result is bitwise identical. */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int r = 0; r < P; ++r) acc += (double)x[r][i];
    y[i] = acc;
  }
}

int orc_omp_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Knuth's TwoSum: s = fl(a + b) and e with a + b = s + e exactly. */
static void two_sum_f32(float a, float b, float *s, float *e) {
  float sum = a + b;
  float bv = sum - a;
  float av = sum - bv;
  *e = (a - av) + (b - bv);
  *s = sum;
}

/* Left-to-right binary32 accumulation of one element's P values
 * (comp = 0), or Sum2 (comp = 1). */
static float acc_f32(int P, const float *v, int comp) {
  if (!comp) {
    float acc = v[0];
    for (int r = 1; r < P; ++r) acc = acc + v[r];
    return acc;
  }
  float p = v[0], sigma = 0.0f;
  for (int r = 1; r < P; ++r) {
    float q;
    two_sum_f32(p, v[r], &p, &q);
    sigma = sigma + q;
  }
  /* a running sum that is not finite stays so; its errors are NaN */
  return isfinite(p) ? p + sigma : p;
}

void orc_sum_f32_f32(int P, int64_t n, const float *const *x, int comp,
                     float *y) {
  float v[64];
  for (int64_t i = 0; i < n; ++i) {
    for (int r = 0; r < P; ++r) v[r] = x[r][i];
    y[i] = acc_f32(P, v, comp);
  }
}

/* maximum(a, b) of IEEE 754-2019 (clause 9.6): NaN if either operand is
 * NaN; otherwise the larger, +0 being larger than -0. */
static double maximum_ieee(double a, double b) {
  if (isnan(a) || isnan(b)) return NAN;
  if (a == b) return signbit(a) ? b : a; /* equal values: +0 over -0 */
  return a > b ? a : b;
}

void orc_max_f32(int P, int64_t n, const float *const *x, float *y) {
  for (int64_t i = 0; i < n; ++i) {
    double m = (double)x[0][i];
    for (int r = 1; r < P; ++r) m = maximum_ieee(m, (double)x[r][i]);
    y[i] = (float)m; /* exact: m is one of the inputs, or NaN */
  }
}

/* ------------------------------------------------------------------ */
/* bfloat16                                                            */
/* ------------------------------------------------------------------ */

double orc_bf16_decode(uint16_t h) {
  int s = (h >> 15) & 1;
  int e = (h >> 7) & 0xff;
  int f = h & 0x7f;
  double v;
  if (e == 0xff) return f ? NAN : (s ? -INFINITY : INFINITY);
  if (e == 0)
    v = ldexp((double)f, -126 - 7); /* subnormal: 0.f x 2^-126 */
  else
    v = ldexp((double)(128 + f), e - 127 - 7); /* 1.f x 2^(e-127) */
  return s ? -v : v;
}

/* Round |v| to an integer multiple of `quantum` (a power of two), nearest,
 * ties to the even multiple.  Exact in double for the ranges used here. */
static double round_to_quantum_rne(double a, double quantum) {
  double m = a / quantum; /* exact: power-of-two scaling */
  double lo = floor(m);
  double frac = m - lo;
  if (frac > 0.5 || (frac == 0.5 && fmod(lo, 2.0) != 0.0)) lo += 1.0;
  return lo * quantum;
}

uint16_t orc_bf16_encode(double v) {
  /* every NaN becomes the quiet NaN with sign 0 and an empty payload */
  if (isnan(v)) return 0x7fc0;
  int s = signbit(v) ? 1 : 0;
  double a = fabs(v);
  const double max_bf16 = ldexp(255.0, 127 - 7); /* 1.1111111b x 2^127 */
  double r;
  if (a == 0.0) return (uint16_t)(s << 15);
  int e;
  frexp(a, &e); /* a = m x 2^e, m in [0.5,1): unit in first place 2^(e-1) */
  int ufp = e - 1;
  if (ufp < -126) ufp = -126; /* subnormal range keeps the 2^-133 quantum */
  r = round_to_quantum_rne(a, ldexp(1.0, ufp - 7));
  /* overflow: RNE rounds to infinity at or above max + half an ulp */
  if (r > max_bf16) return (uint16_t)((s << 15) | 0x7f80);
  /* bits of the representable value r */
  uint16_t bits;
  if (r < ldexp(1.0, -126)) {
    bits = (uint16_t)(r / ldexp(1.0, -133));
  } else {
    int ee;
    double m = frexp(r, &ee); /* r = m 2^ee */
    int E = ee - 1 + 127;
    int F = (int)((m * 2.0 - 1.0) * 128.0);
    bits = (uint16_t)((E << 7) | F);
  }
  return (uint16_t)((s << 15) | bits);
}

void orc_sum_bf16_f64(int P, int64_t n, const uint16_t *const *x, double *y) {
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int r = 0; r < P; ++r) acc += orc_bf16_decode(x[r][i]);
    y[i] = acc;
  }
}

void orc_sum_bf16_f32(int P, int64_t n, const uint16_t *const *x, int comp,
                      uint16_t *y, float *y32) {
  float v[64];
  for (int64_t i = 0; i < n; ++i) {
    for (int r = 0; r < P; ++r) v[r] = (float)orc_bf16_decode(x[r][i]);
    float acc = acc_f32(P, v, comp);
    if (y32) y32[i] = acc;
    y[i] = orc_bf16_encode((double)acc);
  }
}

/* bf16 pair output of the same sum: hi = bf16(y32), lo = bf16(y32 - hi)
 * (lo = +0 when hi is not finite), y32 the binary32 sum above (left to
 * right or Sum2).  The difference is
 * exact in double (and in binary32: hi is y32 rounded to fewer bits in the
 * same binade), so hi + lo carries y32 to 16 significant bits. */
void orc_sum_bf16_hilo(int P, int64_t n, const uint16_t *const *x, int comp,
                       uint16_t *hi, uint16_t *lo) {
  float v[64];
  for (int64_t i = 0; i < n; ++i) {
    for (int r = 0; r < P; ++r) v[r] = (float)orc_bf16_decode(x[r][i]);
    float acc = acc_f32(P, v, comp);
    hi[i] = orc_bf16_encode((double)acc);
    /* hi infinite (the sum is beyond bf16's range) or NaN: lo = +0, so that
     * hi + lo is hi rather than a NaN from y - hi */
    if (!isfinite(orc_bf16_decode(hi[i]))) {
      lo[i] = 0;
      continue;
    }
    lo[i] = orc_bf16_encode((double)acc - orc_bf16_decode(hi[i]));
  }
}

void orc_max_bf16(int P, int64_t n, const uint16_t *const *x, uint16_t *y) {
  for (int64_t i = 0; i < n; ++i) {
    double m = orc_bf16_decode(x[0][i]);
    for (int r = 1; r < P; ++r) m = maximum_ieee(m, orc_bf16_decode(x[r][i]));
    y[i] = orc_bf16_encode(m);
  }
}

/* ------------------------------------------------------------------ */
/* e4m3 (OCP E4M3FN) with one FP32 scale per block of 256 elements      */
/* ------------------------------------------------------------------ */

double orc_e4m3_decode(uint8_t q) {
  int s = (q >> 7) & 1;
  int e = (q >> 3) & 0xf;
  int f = q & 0x7;
  double v;
  if (e == 0xf && f == 0x7) return NAN;
  if (e == 0)
    v = ldexp((double)f, -6 - 3); /* 0.f x 2^-6 */
  else
    v = ldexp((double)(8 + f), e - 7 - 3); /* 1.f x 2^(e-7) */
  return s ? -v : v;
}

uint8_t orc_e4m3_encode(double v) {
  if (isnan(v)) return 0x7f;
  int s = signbit(v) ? 1 : 0;
  double a = fabs(v);
  double r;
  if (a >= 448.0) {
    r = 448.0; /* saturate */
  } else if (a == 0.0) {
    return (uint8_t)(s << 7);
  } else {
    int e;
    frexp(a, &e);
    int ufp = e - 1;
    if (ufp < -6) ufp = -6; /* subnormals: quantum 2^-9 */
    r = round_to_quantum_rne(a, ldexp(1.0, ufp - 3));
    if (r > 448.0) r = 448.0; /* cannot happen below 448, kept for clarity */
  }
  uint8_t bits;
  if (r < ldexp(1.0, -6)) {
    bits = (uint8_t)(r / ldexp(1.0, -9));
  } else {
    int ee;
    double m = frexp(r, &ee);
    int E = ee - 1 + 7;
    int F = (int)((m * 2.0 - 1.0) * 8.0);
    bits = (uint8_t)((E << 3) | F);
  }
  return (uint8_t)((s << 7) | bits);
}

/* Scale of one block from its largest magnitude: s = fl32(amax / 448);
 * s = 1 when amax is 0 or s would not be a normal binary32 number. */
static float block_scale(float amax) {
  float s = amax / 448.0f;
  if (!(s >= 0x1p-126f)) s = 1.0f;
  return s;
}

/* Quantize n FP32 values to e4m3 codes with one FP32 scale per block of 256
 * elements (the last block may be short): s = block_scale(max |x|),
 * q = e4m3(fl32(x * fl32(1 / s))).  Every step is one binary32 operation. */
void orc_e4m3_pack(int64_t n, const float *x, uint8_t *q, float *s) {
  for (int64_t b = 0; b * 256 < n; ++b) {
    int64_t lo = b * 256, hi = lo + 256 < n ? lo + 256 : n;
    float amax = 0.0f;
    for (int64_t i = lo; i < hi; ++i) {
      float a = fabsf(x[i]);
      if (a > amax) amax = a;
    }
    float sc = block_scale(amax);
    float inv = 1.0f / sc;
    s[b] = sc;
    for (int64_t i = lo; i < hi; ++i) {
      float t = x[i] * inv;
      q[i] = orc_e4m3_encode((double)t);
    }
  }
}

/* FP64 reference: sum over ranks of the exactly dequantized payloads
 * dec(q_r[i]) * s_r[i / 256] (4 x 24 significant bits: exact in double). */
void orc_sum_e4m3_f64(int P, int64_t n, const uint8_t *const *q,
                      const float *const *s, double *y) {
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int r = 0; r < P; ++r)
      acc += orc_e4m3_decode(q[r][i]) * (double)s[r][i / 256];
    y[i] = acc;
  }
}

/* FP32 mirror: each input dequantized in binary32, fl32(dec(q) * s),
 * accumulated left to right (comp = 0) or by Sum2 (comp = 1), then the
 * result re-quantized with orc_e4m3_pack.  y32 (optional) receives the
 * binary32 sums before quantization. */
void orc_sum_e4m3_f32(int P, int64_t n, const uint8_t *const *q,
                      const float *const *s, int comp, uint8_t *yq,
                      float *ys, float *y32) {
  float v[64];
  float blk[256];
  for (int64_t b = 0; b * 256 < n; ++b) {
    int64_t lo = b * 256, hi = lo + 256 < n ? lo + 256 : n;
    for (int64_t i = lo; i < hi; ++i) {
      for (int r = 0; r < P; ++r)
        v[r] = (float)orc_e4m3_decode(q[r][i]) * s[r][b];
      blk[i - lo] = acc_f32(P, v, comp);
      if (y32) y32[i] = blk[i - lo];
    }
    orc_e4m3_pack(hi - lo, blk, yq + lo, ys + b);
  }
}

/* ------------------------------------------------------------------ */
/* e5m2 (OCP E5M2) with one FP32 scale per block of 256 elements        */
/* ------------------------------------------------------------------ */

double orc_e5m2_decode(uint8_t q) {
  int s = (q >> 7) & 1;
  int e = (q >> 2) & 0x1f;
  int f = q & 0x3;
  double v;
  if (e == 0x1f) {
    if (f != 0) return NAN;
    v = INFINITY;
  } else if (e == 0) {
    v = ldexp((double)f, -14 - 2); /* 0.f x 2^-14 */
  } else {
    v = ldexp((double)(4 + f), e - 15 - 2); /* 1.f x 2^(e-15) */
  }
  return s ? -v : v;
}

uint8_t orc_e5m2_encode(double v) {
  if (isnan(v)) return 0x7f;
  int s = signbit(v) ? 1 : 0;
  double a = fabs(v);
  const double max_e5m2 = 57344.0; /* 1.11b x 2^15 */
  double r;
  if (a >= max_e5m2) {
    r = max_e5m2; /* saturate (infinities included) */
  } else if (a == 0.0) {
    return (uint8_t)(s << 7);
  } else {
    int e;
    frexp(a, &e);
    int ufp = e - 1;
    if (ufp < -14) ufp = -14; /* subnormals: quantum 2^-16 */
    r = round_to_quantum_rne(a, ldexp(1.0, ufp - 2));
    if (r > max_e5m2) r = max_e5m2;
  }
  uint8_t bits;
  if (r < ldexp(1.0, -14)) {
    bits = (uint8_t)(r / ldexp(1.0, -16));
  } else {
    int ee;
    double m = frexp(r, &ee);
    int E = ee - 1 + 15;
    int F = (int)((m * 2.0 - 1.0) * 4.0);
    bits = (uint8_t)((E << 2) | F);
  }
  return (uint8_t)((s << 7) | bits);
}

/* Scale of one e5m2 block: s = fl32(amax / 57344); s = 1 when amax is 0 or
 * s would not be a normal binary32 number. */
static float block_scale_e5m2(float amax) {
  float s = amax / 57344.0f;
  if (!(s >= 0x1p-126f)) s = 1.0f;
  return s;
}

/* As orc_e4m3_pack, for e5m2: q = e5m2(fl32(x * fl32(1 / s))). */
void orc_e5m2_pack(int64_t n, const float *x, uint8_t *q, float *s) {
  for (int64_t b = 0; b * 256 < n; ++b) {
    int64_t lo = b * 256, hi = lo + 256 < n ? lo + 256 : n;
    float amax = 0.0f;
    for (int64_t i = lo; i < hi; ++i) {
      float a = fabsf(x[i]);
      if (a > amax) amax = a;
    }
    float sc = block_scale_e5m2(amax);
    float inv = 1.0f / sc;
    s[b] = sc;
    for (int64_t i = lo; i < hi; ++i) {
      float t = x[i] * inv;
      q[i] = orc_e5m2_encode((double)t);
    }
  }
}

/* FP64 reference: sum of the exactly dequantized payloads
 * dec(q_r[i]) * s_r[i / 256] (3 x 24 significant bits: exact in double). */
void orc_sum_e5m2_f64(int P, int64_t n, const uint8_t *const *q,
                      const float *const *s, double *y) {
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int r = 0; r < P; ++r)
      acc += orc_e5m2_decode(q[r][i]) * (double)s[r][i / 256];
    y[i] = acc;
  }
}

/* FP32 mirror, as orc_sum_e4m3_f32 with the e5m2 codec and scale. */
void orc_sum_e5m2_f32(int P, int64_t n, const uint8_t *const *q,
                      const float *const *s, int comp, uint8_t *yq,
                      float *ys, float *y32) {
  float v[64];
  float blk[256];
  for (int64_t b = 0; b * 256 < n; ++b) {
    int64_t lo = b * 256, hi = lo + 256 < n ? lo + 256 : n;
    for (int64_t i = lo; i < hi; ++i) {
      for (int r = 0; r < P; ++r)
        v[r] = (float)orc_e5m2_decode(q[r][i]) * s[r][b];
      blk[i - lo] = acc_f32(P, v, comp);
      if (y32) y32[i] = blk[i - lo];
    }
    orc_e5m2_pack(hi - lo, blk, yq + lo, ys + b);
  }
}

/* ------------------------------------------------------------------ */
/* MX blocks: e4m3 codes, one E8M0 scale per block of 32 elements       */
/* ------------------------------------------------------------------ */

double orc_e8m0_decode(uint8_t b) {
  if (b == 255) return NAN;
  return ldexp(1.0, (int)b - 127);
}

/* Shared exponent of one block: the smallest e >= -127 with
 * amax <= 448 * 2^e (amax = 0 gives -127).  Found by counting up, every
 * comparison exact in double. */
int orc_mx_exponent(float amax) {
  int e = -127;
  while (ldexp(448.0, e) < (double)amax) ++e;
  return e;
}

/* Quantize n FP32 values to MX blocks of 32 (the last block may be short):
 * e = orc_mx_exponent(max |x|), scale byte e + 127, q = e4m3(x / 2^e); the
 * division is exact in double and the quotient is at most 448. */
void orc_mx_pack(int64_t n, const float *x, uint8_t *q, uint8_t *sb) {
  for (int64_t b = 0; b * 32 < n; ++b) {
    int64_t lo = b * 32, hi = lo + 32 < n ? lo + 32 : n;
    float amax = 0.0f;
    for (int64_t i = lo; i < hi; ++i) {
      float a = fabsf(x[i]);
      if (a > amax) amax = a;
    }
    int e = orc_mx_exponent(amax);
    sb[b] = (uint8_t)(e + 127);
    for (int64_t i = lo; i < hi; ++i)
      q[i] = orc_e4m3_encode((double)x[i] / ldexp(1.0, e));
  }
}

/* FP64 reference: sum over ranks of dec(q_r[i]) * 2^(b_r[i / 32] - 127). */
void orc_sum_mx_f64(int P, int64_t n, const uint8_t *const *q,
                    const uint8_t *const *sb, double *y) {
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int r = 0; r < P; ++r)
      acc += orc_e4m3_decode(q[r][i]) * orc_e8m0_decode(sb[r][i / 32]);
    y[i] = acc;
  }
}

/* FP32 mirror: the dequantized inputs (exact in binary32) accumulated left
 * to right (comp = 0) or by Sum2 (comp = 1), then re-quantized with
 * orc_mx_pack.  y32 (optional) receives the binary32 sums. */
void orc_sum_mx_f32(int P, int64_t n, const uint8_t *const *q,
                    const uint8_t *const *sb, int comp, uint8_t *yq,
                    uint8_t *ysb, float *y32) {
  float v[64];
  float blk[32];
  for (int64_t b = 0; b * 32 < n; ++b) {
    int64_t lo = b * 32, hi = lo + 32 < n ? lo + 32 : n;
    for (int64_t i = lo; i < hi; ++i) {
      for (int r = 0; r < P; ++r)
        v[r] = (float)(orc_e4m3_decode(q[r][i]) * orc_e8m0_decode(sb[r][b]));
      blk[i - lo] = acc_f32(P, v, comp);
      if (y32) y32[i] = blk[i - lo];
    }
    orc_mx_pack(hi - lo, blk, yq + lo, ysb + b);
  }
}
