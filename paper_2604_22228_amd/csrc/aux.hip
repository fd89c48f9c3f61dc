// Dispatch of the reduce kernel, and the small kernels around it: the
// device-side ready signal, the producer-side packers (FP32 -> bf16,
// FP32 -> e4m3 / e5m2 with per-256 scales, FP32 -> MX blocks), and the
// measurement probes.
#include <hip/hip_runtime.h>

#include "reduce_impl.hpp"

namespace pcoll {

hipError_t launch_reduce(const ReduceArgs& a, int dtype, int op, bool comp,
                         bool deep, int nranks, int groups, int waves,
                         hipStream_t s) {
  if (nranks < 1 || nranks > kMaxRanks || groups < 1 || waves < 1 ||
      waves > kMaxWavesPerGroup)
    return hipErrorInvalidValue;
  switch (dtype) {
    case kF32:
      return launch_reduce_f32(a, op, comp, deep, nranks, groups, waves, s);
    case kI32:
      return launch_reduce_i32(a, op, deep, nranks, groups, waves, s);
    case kBF16:
      return launch_reduce_bf16(a, op, comp, deep, nranks, groups, waves, s);
    case kE4M3:
      if (op != kSum) return hipErrorInvalidValue;
      return launch_reduce_e4m3(a, comp, nranks, groups, waves, s);
    case kE5M2:
      if (op != kSum) return hipErrorInvalidValue;
      return launch_reduce_e5m2(a, comp, nranks, groups, waves, s);
    case kMX:
      if (op != kSum) return hipErrorInvalidValue;
      return launch_reduce_mx(a, comp, nranks, groups, waves, s);
    case kBF16Pair:
      if (op != kSum) return hipErrorInvalidValue;
      return launch_reduce_bf16_pair(a, comp, deep, nranks, groups, waves,
                                     s);
    default:
      return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------ ready signal
// Appends parts[0..n) to the device ready ring.  One workgroup reserves its
// entries with a single atomic on the ring's 64-bit entry counter; entry c
// goes to slot c % capacity as one 64-bit store ((uint32)c << 32) | part,
// so a reader sees either the old or the new entry and can tell them apart.
__global__ __launch_bounds__(256) void pready_kernel(PreadyArgs a) {
  __shared__ uint64_t base;
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  const uint32_t first = blockIdx.x * 256u;
  const uint32_t cnt = a.n - first < 256u ? a.n - first : 256u;
  if (threadIdx.x == 0)
    base = __hip_atomic_fetch_add(&a.ring->dreserve, (uint64_t)cnt,
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  if (i < a.n) {
    const uint64_t c = base + threadIdx.x;
    const uint64_t v = ((uint64_t)(uint32_t)c << 32) | (uint32_t)a.parts[i];
    __hip_atomic_store(&a.dlist[c % a.capacity], v, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
}

hipError_t launch_pready(const PreadyArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(pready_kernel, dim3((a.n + 255u) / 256u), dim3(256), 0,
                     s, a);
  return hipGetLastError();
}

// Per-rank marks.  Each lane sets its rank's bit in the partition's
// epoch-tagged mask with a compare-and-swap (acquire-release: the ranks'
// producers, ordered before their marks by their streams, are visible to
// the lane whose mark completes the mask, which then publishes with a
// release store).  Marks already set are idempotent, so a partition is
// appended exactly once; the completing lanes of a wavefront reserve their
// ring entries with one atomic.
__global__ __launch_bounds__(256) void pready_rank_kernel(PreadyRankArgs a) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63u;
  bool done = false;
  uint32_t part = 0;
  if (i < a.n) {
    part = (uint32_t)a.parts[i];
    if (part < a.capacity) {
      uint64_t* w = &a.rank_marks[part];
      const uint64_t tag = (uint64_t)a.epoch << 32;
      const uint64_t bit = 1ull << a.rank;
      uint64_t old = __hip_atomic_load(w, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
      for (;;) {
        const uint64_t cur = (old & ~0xffffffffull) == tag ? old : tag;
        const uint64_t nw = cur | bit;
        if (nw == old) break;  // this rank's mark is already in
        if (__hip_atomic_compare_exchange_strong(
                w, &old, nw, __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                __HIP_MEMORY_SCOPE_AGENT)) {
          done = (uint32_t)nw == a.full && (uint32_t)cur != a.full;
          break;
        }
      }
    }
  }
  const uint64_t m = __ballot(done);
  if (m == 0) return;
  const uint32_t leader = (uint32_t)(__ffsll((long long)m) - 1);
  uint64_t base = 0;
  if (lane == leader)
    base = __hip_atomic_fetch_add(&a.ring->dreserve,
                                  (uint64_t)__popcll(m), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  base = __shfl(base, (int)leader);
  if (done) {
    const uint64_t c = base + __popcll(m & ((1ull << lane) - 1ull));
    const uint64_t v = ((uint64_t)(uint32_t)c << 32) | part;
    __hip_atomic_store(&a.dlist[c % a.capacity], v, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
}

hipError_t launch_pready_rank(const PreadyRankArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(pready_rank_kernel, dim3((a.n + 255u) / 256u),
                     dim3(256), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ packers
__global__ __launch_bounds__(256) void pack_bf16_kernel(const float* src,
                                                        uint16_t* dst,
                                                        size_t n) {
  const size_t nv = n / 8;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv;
       v += stride) {
    const uint4 a = dev::ld_stream(reinterpret_cast<const uint4*>(src) + 2 * v);
    const uint4 b =
        dev::ld_stream(reinterpret_cast<const uint4*>(src) + 2 * v + 1);
    uint4 o;
    o.x = dev::f_to_bf16(__uint_as_float(a.x)) |
          (dev::f_to_bf16(__uint_as_float(a.y)) << 16);
    o.y = dev::f_to_bf16(__uint_as_float(a.z)) |
          (dev::f_to_bf16(__uint_as_float(a.w)) << 16);
    o.z = dev::f_to_bf16(__uint_as_float(b.x)) |
          (dev::f_to_bf16(__uint_as_float(b.y)) << 16);
    o.w = dev::f_to_bf16(__uint_as_float(b.z)) |
          (dev::f_to_bf16(__uint_as_float(b.w)) << 16);
    dev::st_stream(reinterpret_cast<uint4*>(dst) + v, o);
  }
  if (blockIdx.x == 0 && threadIdx.x < n - nv * 8) {
    const size_t i = nv * 8 + threadIdx.x;
    dst[i] = (uint16_t)dev::f_to_bf16(src[i]);
  }
}

hipError_t launch_pack_bf16(const float* src, uint16_t* dst, size_t n,
                            hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n / 8 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(pack_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     s, src, dst, n);
  return hipGetLastError();
}

// One row of 16 lanes per block of 256 values, 16 values per lane.
template <class Fmt>
__global__ __launch_bounds__(256) void pack_fp8_kernel(const float* src,
                                                       uint8_t* dst,
                                                       float* scales,
                                                       size_t n) {
  const uint32_t lane = threadIdx.x & 63u;
  const size_t wave = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
  const size_t nwaves = (size_t)gridDim.x * blockDim.x / 64;
  for (size_t base = wave * 1024; base < n; base += nwaves * 1024) {
    const size_t el = base + (size_t)lane * 16;
    const uint32_t have = el < n ? (n - el < 16 ? (uint32_t)(n - el) : 16u) : 0u;
    float x[16];
    if (have == 16u) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint4 v = dev::ld_stream(reinterpret_cast<const uint4*>(src + el) + k);
        x[4 * k + 0] = __uint_as_float(v.x);
        x[4 * k + 1] = __uint_as_float(v.y);
        x[4 * k + 2] = __uint_as_float(v.z);
        x[4 * k + 3] = __uint_as_float(v.w);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) x[j] = (uint32_t)j < have ? src[el + j] : 0.0f;
    }
    float amax = 0.0f;
#pragma unroll
    for (int j = 0; j < 16; ++j) amax = fmaxf(amax, fabsf(x[j]));
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
      w[k] = Fmt::enc4(x[4 * k] * inv, x[4 * k + 1] * inv, x[4 * k + 2] * inv,
                       x[4 * k + 3] * inv);
    if (have == 16u) {
      dev::st_stream(reinterpret_cast<uint4*>(dst + el),
                     make_uint4(w[0], w[1], w[2], w[3]));
    } else if (have) {
      for (uint32_t j = 0; j < have; ++j)
        dst[el + j] = (uint8_t)(w[j >> 2] >> (8 * (j & 3)));
    }
    if (have && (lane & 15u) == 0u) scales[el / 256] = so;
  }
}

template <class Fmt>
static hipError_t launch_pack_fp8(const float* src, uint8_t* dst,
                                  float* scales, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 4095) / 4096;  // 4 waves x 1024 values
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(pack_fp8_kernel<Fmt>, dim3((unsigned)blocks), dim3(256),
                     0, s, src, dst, scales, n);
  return hipGetLastError();
}

hipError_t launch_pack_e4m3(const float* src, uint8_t* dst, float* scales,
                            size_t n, hipStream_t s) {
  return launch_pack_fp8<dev::Fp8E4M3>(src, dst, scales, n, s);
}

hipError_t launch_pack_e5m2(const float* src, uint8_t* dst, float* scales,
                            size_t n, hipStream_t s) {
  return launch_pack_fp8<dev::Fp8E5M2>(src, dst, scales, n, s);
}

// One pair of lanes per MX block of 32 values, 16 values per lane.
__global__ __launch_bounds__(256) void pack_mx_kernel(const float* src,
                                                      uint8_t* dst,
                                                      uint8_t* scales,
                                                      size_t n) {
  const uint32_t lane = threadIdx.x & 63u;
  const size_t wave = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
  const size_t nwaves = (size_t)gridDim.x * blockDim.x / 64;
  for (size_t base = wave * 1024; base < n; base += nwaves * 1024) {
    const size_t el = base + (size_t)lane * 16;
    const uint32_t have = el < n ? (n - el < 16 ? (uint32_t)(n - el) : 16u) : 0u;
    float x[16];
    if (have == 16u) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint4 v = dev::ld_stream(reinterpret_cast<const uint4*>(src + el) + k);
        x[4 * k + 0] = __uint_as_float(v.x);
        x[4 * k + 1] = __uint_as_float(v.y);
        x[4 * k + 2] = __uint_as_float(v.z);
        x[4 * k + 3] = __uint_as_float(v.w);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) x[j] = (uint32_t)j < have ? src[el + j] : 0.0f;
    }
    float amax = 0.0f;
#pragma unroll
    for (int j = 0; j < 16; ++j) amax = fmaxf(amax, fabsf(x[j]));
    amax = dev::pair_max(amax);
    const uint32_t b = dev::mx_scale_byte(amax);
    const uint4 codes = dev::mx_enc16(x, dev::e8m0_operand(b));
    if (have == 16u) {
      dev::st_stream(reinterpret_cast<uint4*>(dst + el), codes);
    } else if (have) {
      const uint32_t w[4] = {codes.x, codes.y, codes.z, codes.w};
      for (uint32_t j = 0; j < have; ++j)
        dst[el + j] = (uint8_t)(w[j >> 2] >> (8 * (j & 3)));
    }
    if (have && (lane & 1u) == 0u) scales[el / 32] = (uint8_t)b;
  }
}

hipError_t launch_pack_mx(const float* src, uint8_t* dst, uint8_t* scales,
                          size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 4095) / 4096;  // 4 waves x 1024 values
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(pack_mx_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     src, dst, scales, n);
  return hipGetLastError();
}

// ------------------------------------------------------------------- probes
__global__ __launch_bounds__(256) void copy_kernel(const uint4* src, uint4* dst,
                                                   size_t nv) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < nv; i += 4 * stride) {
    uint4 a = dev::ld_stream(src + i);
    uint4 b = dev::ld_stream(src + i + stride);
    uint4 c = dev::ld_stream(src + i + 2 * stride);
    uint4 d = dev::ld_stream(src + i + 3 * stride);
    dev::st_stream(dst + i, a);
    dev::st_stream(dst + i + stride, b);
    dev::st_stream(dst + i + 2 * stride, c);
    dev::st_stream(dst + i + 3 * stride, d);
  }
  for (; i < nv; i += stride) dev::st_stream(dst + i, dev::ld_stream(src + i));
}

__global__ __launch_bounds__(256) void fill_kernel(uint4* dst, size_t nv,
                                                   uint32_t v) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const uint4 val = make_uint4(v, v, v, v);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv;
       i += stride)
    dev::st_stream(dst + i, val);
}

static unsigned probe_blocks(size_t nv) {
  size_t b = (nv + 255) / 256;
  if (b > 16384) b = 16384;
  return (unsigned)(b ? b : 1);
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes,
                       hipStream_t s) {
  const size_t nv = bytes / 16;
  if (nv == 0) return hipSuccess;
  hipLaunchKernelGGL(copy_kernel, dim3(probe_blocks(nv)), dim3(256), 0, s,
                     static_cast<const uint4*>(src), static_cast<uint4*>(dst),
                     nv);
  return hipGetLastError();
}

hipError_t launch_fill(void* dst, size_t bytes, uint32_t value,
                       hipStream_t s) {
  const size_t nv = bytes / 16;
  if (nv == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(probe_blocks(nv)), dim3(256), 0, s,
                     static_cast<uint4*>(dst), nv, value);
  return hipGetLastError();
}

}  // namespace pcoll
