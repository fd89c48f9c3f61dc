// e4m3 payloads with per-256 binary32 scales: sum (plain or Sum2).
#include "reduce_impl.hpp"

namespace pcoll {
hipError_t launch_reduce_e4m3(const ReduceArgs& a, bool comp, int nranks, const Launch& l) {
  using namespace dev;
  if (comp) return launch_ranks<E4M3Tile<true>>(a, nranks, l);
  return launch_ranks<E4M3Tile<false>>(a, nranks, l);
}
}  // namespace pcoll
