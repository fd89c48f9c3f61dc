// int32 payloads: wrapping sum and max (bit-exact).
#include "reduce_impl.hpp"

namespace pcoll {
namespace {
template <bool D>
hipError_t i32(const ReduceArgs& a, int op, int nranks, const Launch& l) {
  using namespace dev;
  if (op == kMax) return launch_ranks<VecTile<IMax, 1, D>>(a, nranks, l);
  return launch_ranks<VecTile<ISum, 1, D>>(a, nranks, l);
}
}  // namespace

hipError_t launch_reduce_i32(const ReduceArgs& a, int op, bool deep,
                             int nranks, const Launch& l) {
  return deep ? i32<true>(a, op, nranks, l)
              : i32<false>(a, op, nranks, l);
}
}  // namespace pcoll
