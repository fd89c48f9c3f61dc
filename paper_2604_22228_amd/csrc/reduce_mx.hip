// MX blocks (e4m3 codes, one E8M0 scale per 32 elements): sum (plain or
// Sum2).
#include "reduce_impl.hpp"

namespace pcoll {
hipError_t launch_reduce_mx(const ReduceArgs& a, bool comp, int nranks, const Launch& l) {
  using namespace dev;
  if (comp) return launch_ranks<MxTile<true>>(a, nranks, l);
  return launch_ranks<MxTile<false>>(a, nranks, l);
}
}  // namespace pcoll
