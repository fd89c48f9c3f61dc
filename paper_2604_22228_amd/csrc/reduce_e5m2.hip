// e5m2 payloads with per-256 binary32 scales: sum (plain or Sum2).
#include "reduce_impl.hpp"

namespace pcoll {
hipError_t launch_reduce_e5m2(const ReduceArgs& a, bool comp, int nranks,
                              int groups, int waves, hipStream_t s) {
  using namespace dev;
  if (comp) return launch_ranks<E5M2Tile<true>>(a, nranks, groups, waves, s);
  return launch_ranks<E5M2Tile<false>>(a, nranks, groups, waves, s);
}
}  // namespace pcoll
