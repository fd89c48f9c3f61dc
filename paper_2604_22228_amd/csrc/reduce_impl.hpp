// Kernel template and rank-count dispatch shared by the per-dtype
// translation units (split so that they compile in parallel).
#pragma once
#include <hip/hip_runtime.h>

#include <hip/hip_ext.h>

#include "kernels.hpp"
#include "persistent.hpp"
#include "tiles.hpp"

namespace pcoll {

template <class Tile, int P>
__global__ __launch_bounds__(64 * kMaxWavesPerGroup) void reduce_persistent(
    ReduceArgs a) {
  dev::persistent_loop<Tile, P>(a);
}

// With timing events, the launch goes through hipExtLaunchKernel, which
// stamps the events at the kernel's own start and end (no marker packets
// around it).  With l.per_cu set, only the kernel's residency is read.
template <class Tile>
hipError_t launch_ranks(const ReduceArgs& a, int nranks, const Launch& l) {
  const dim3 grid(l.groups), block(64 * l.waves);
  switch (nranks) {
#define PCOLL_CASE(P)                                                        \
  case P:                                                                    \
    if (l.per_cu)                                                            \
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(                   \
          l.per_cu, reduce_persistent<Tile, P>, 64 * l.waves, 0);            \
    if (l.start || l.stop)                                                   \
      hipExtLaunchKernelGGL((reduce_persistent<Tile, P>), grid, block, 0,    \
                            l.stream, l.start, l.stop, 0, a);                \
    else                                                                     \
      hipLaunchKernelGGL((reduce_persistent<Tile, P>), grid, block, 0,       \
                         l.stream, a);                                       \
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
                             int nranks, const Launch&);
hipError_t launch_reduce_i32(const ReduceArgs&, int op, bool deep, int nranks, const Launch&);
hipError_t launch_reduce_bf16(const ReduceArgs&, int op, bool comp, bool deep,
                              int nranks, const Launch&);
hipError_t launch_reduce_e4m3(const ReduceArgs&, bool comp, int nranks, const Launch&);
hipError_t launch_reduce_e5m2(const ReduceArgs&, bool comp, int nranks, const Launch&);
hipError_t launch_reduce_mx(const ReduceArgs&, bool comp, int nranks, const Launch&);
hipError_t launch_reduce_bf16_pair(const ReduceArgs&, bool comp, bool deep,
                                   int nranks, const Launch&);

}  // namespace pcoll
