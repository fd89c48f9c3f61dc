// int32 payloads: wrapping sum and max (bit-exact).
#include "reduce_impl.hpp"

namespace pcoll {
hipError_t launch_reduce_i32(const ReduceArgs& a, int op, int nranks,
                             int groups, int waves, hipStream_t s) {
  using namespace dev;
  if (op == kMax) return launch_ranks<VecTile<IMax, 1>>(a, nranks, groups, waves, s);
  return launch_ranks<VecTile<ISum, 1>>(a, nranks, groups, waves, s);
}
}  // namespace pcoll
