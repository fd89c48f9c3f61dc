// e5m2 payloads with per-256 binary32 scales: sum (plain or Sum2).
#include "reduce_impl.hpp"

namespace pcoll {
hipError_t launch_reduce_e5m2(const ReduceArgs& a, bool comp, int nranks, const Launch& l) {
  using namespace dev;
  if (comp) return launch_ranks<E5M2Tile<true>>(a, nranks, l);
  return launch_ranks<E5M2Tile<false>>(a, nranks, l);
}
}  // namespace pcoll
