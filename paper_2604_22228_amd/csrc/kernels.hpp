// Launch entry points of the gfx950 kernels, called by the host runtime.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#include "layout.hpp"

namespace pcoll {

// Largest workgroup of the persistent reduce kernel, in wavefronts (the
// kernels are compiled for up to 512 threads; the runtime picks 1..8).
constexpr int kMaxWavesPerGroup = 8;

// Dtype / op codes, equal to the public enums of pcoll.h.
enum Dtype : int {
  kI32 = 0, kF32 = 1, kBF16 = 2, kE4M3 = 3, kE5M2 = 4, kMX = 5,
  kBF16Pair = 6
};
enum Op : int { kSum = 0, kMax = 1 };

// Elements per 16-byte vector and alignment unit of partitions.
inline int elem_bytes(int dtype) {
  return dtype == kBF16 || dtype == kBF16Pair ? 2
                        : (dtype == kE4M3 || dtype == kE5M2 || dtype == kMX
                               ? 1
                               : 4);
}

// Launch shape of the persistent kernel: `groups` workgroups of `waves`
// wavefronts on `stream`; with start / stop events, those are stamped at
// the kernel's own start and end (hipExtLaunchKernel).  With `per_cu` set,
// nothing is launched: *per_cu receives how many workgroups of `waves`
// wavefronts of the selected kernel fit on one compute unit at once.
struct Launch {
  int groups;
  int waves;
  hipStream_t stream;
  hipEvent_t start;
  hipEvent_t stop;
  int* per_cu = nullptr;
};

// The persistent partitioned-reduce kernel; deep: 4 rows per lane in
// flight in the 16-byte-vector kernels at 3..8 ranks (else 2).  Returns
// hipErrorInvalidValue for an unsupported (dtype, op, comp, nranks)
// combination.
hipError_t launch_reduce(const ReduceArgs& a, int dtype, int op, bool comp,
                         bool deep, int nranks, const Launch& l);
// Device-side readiness: appends `a.n` partition ids to the device ready
// ring.
hipError_t launch_pready(const PreadyArgs& a, hipStream_t s);
// Device-side per-rank readiness: marks one rank's contribution to a.n
// partitions; each partition whose last rank this completes is appended to
// the ring.
hipError_t launch_pready_rank(const PreadyRankArgs& a, hipStream_t s);
// Producer-side packing: FP32 -> bfloat16 (RNE), FP32 -> e4m3 + per-256
// FP32 scales.
hipError_t launch_pack_bf16(const float* src, uint16_t* dst, size_t n,
                            hipStream_t s);
hipError_t launch_pack_e4m3(const float* src, uint8_t* dst, float* scales,
                            size_t n, hipStream_t s);
hipError_t launch_pack_e5m2(const float* src, uint8_t* dst, float* scales,
                            size_t n, hipStream_t s);
// FP32 -> MX blocks: e4m3 codes and one E8M0 scale byte per 32 elements.
hipError_t launch_pack_mx(const float* src, uint8_t* dst, uint8_t* scales,
                          size_t n, hipStream_t s);
// Measurement probes: a dwordx4 streaming copy and a fill.
hipError_t launch_copy(void* dst, const void* src, size_t bytes,
                       hipStream_t s);
hipError_t launch_fill(void* dst, size_t bytes, uint32_t value,
                       hipStream_t s);
// The reduce's streams without its protocol: nsrc (1, 2, 4, 8 or 16) reads
// of `bytes` each and, with `write`, one write of their XOR; grid-stride
// (tiles = null), in the reduce's tile schedule (whole 1 KiB rows), or in
// contiguous shares per workgroup (tiles->chunked).
struct StreamTiles {
  uint32_t groups, waves, tile_rows, band;
  uint32_t chunked;  // 1: each of `groups` workgroups of 256 threads
                     // streams its own contiguous share (waves, tile_rows
                     // and band unused)
};
hipError_t launch_stream(const void* const* srcs, int nsrc, void* dst,
                         size_t bytes, bool write, const StreamTiles* tiles,
                         hipStream_t s);

}  // namespace pcoll
