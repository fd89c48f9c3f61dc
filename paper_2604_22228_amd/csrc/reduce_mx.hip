// MX blocks (e4m3 codes, one E8M0 scale per 32 elements): sum (plain or
// Sum2).
#include "reduce_impl.hpp"

namespace pcoll {
hipError_t launch_reduce_mx(const ReduceArgs& a, bool comp, int nranks,
                            int groups, int waves, hipStream_t s) {
  using namespace dev;
  if (comp) return launch_ranks<MxTile<true>>(a, nranks, groups, waves, s);
  return launch_ranks<MxTile<false>>(a, nranks, groups, waves, s);
}
}  // namespace pcoll
