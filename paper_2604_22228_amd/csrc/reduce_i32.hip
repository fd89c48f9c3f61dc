// int32 payloads: wrapping sum and max (bit-exact).
#include "reduce_impl.hpp"

namespace pcoll {
namespace {
template <bool D>
hipError_t i32(const ReduceArgs& a, int op, int nranks, int groups, int waves,
               hipStream_t s) {
  using namespace dev;
  if (op == kMax) return launch_ranks<VecTile<IMax, 1, D>>(a, nranks, groups, waves, s);
  return launch_ranks<VecTile<ISum, 1, D>>(a, nranks, groups, waves, s);
}
}  // namespace

hipError_t launch_reduce_i32(const ReduceArgs& a, int op, bool deep,
                             int nranks, int groups, int waves, hipStream_t s) {
  return deep ? i32<true>(a, op, nranks, groups, waves, s)
              : i32<false>(a, op, nranks, groups, waves, s);
}
}  // namespace pcoll
