// Kernel template and rank-count dispatch shared by the per-dtype
// translation units (split so that they compile in parallel).
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "persistent.hpp"
#include "tiles.hpp"

namespace pcoll {

template <class Tile, int P>
__global__ __launch_bounds__(64 * kMaxWavesPerGroup) void reduce_persistent(
    ReduceArgs a) {
  dev::persistent_loop<Tile, P>(a);
}

template <class Tile>
hipError_t launch_ranks(const ReduceArgs& a, int nranks, int groups,
                        int waves, hipStream_t s) {
  const dim3 grid(groups), block(64 * waves);
  switch (nranks) {
#define PCOLL_CASE(P)                                                \
  case P:                                                            \
    hipLaunchKernelGGL((reduce_persistent<Tile, P>), grid, block, 0, \
                       s, a);                                        \
    break;
    PCOLL_CASE(1) PCOLL_CASE(2) PCOLL_CASE(3) PCOLL_CASE(4)
    PCOLL_CASE(5) PCOLL_CASE(6) PCOLL_CASE(7) PCOLL_CASE(8)
    PCOLL_CASE(9) PCOLL_CASE(10) PCOLL_CASE(11) PCOLL_CASE(12)
    PCOLL_CASE(13) PCOLL_CASE(14) PCOLL_CASE(15) PCOLL_CASE(16)
#undef PCOLL_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Per-family launchers, defined in reduce_<family>.hip.
// deep: the 16-byte-vector kernels keep 4 rows per lane in flight at 3..8
// ranks (else 2).
hipError_t launch_reduce_f32(const ReduceArgs&, int op, bool comp, bool deep,
                             int nranks, int groups, int waves, hipStream_t);
hipError_t launch_reduce_i32(const ReduceArgs&, int op, bool deep, int nranks,
                             int groups, int waves, hipStream_t);
hipError_t launch_reduce_bf16(const ReduceArgs&, int op, bool comp, bool deep,
                              int nranks, int groups, int waves, hipStream_t);
hipError_t launch_reduce_e4m3(const ReduceArgs&, bool comp, int nranks,
                              int groups, int waves, hipStream_t);
hipError_t launch_reduce_e5m2(const ReduceArgs&, bool comp, int nranks,
                              int groups, int waves, hipStream_t);
hipError_t launch_reduce_mx(const ReduceArgs&, bool comp, int nranks,
                            int groups, int waves, hipStream_t);
hipError_t launch_reduce_bf16_pair(const ReduceArgs&, bool comp, bool deep,
                                   int nranks, int groups, int waves,
                                   hipStream_t);

}  // namespace pcoll
