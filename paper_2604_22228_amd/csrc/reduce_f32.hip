// binary32 payloads: sum (plain or Sum2) and max.
#include "reduce_impl.hpp"

namespace pcoll {
namespace {
template <bool D>
hipError_t f32(const ReduceArgs& a, int op, bool comp, int nranks, const Launch& l) {
  using namespace dev;
  if (op == kMax) return launch_ranks<VecTile<FMax, 0, D>>(a, nranks, l);
  if (comp) return launch_ranks<VecTile<FSum<true>, 0, D>>(a, nranks, l);
  return launch_ranks<VecTile<FSum<false>, 0, D>>(a, nranks, l);
}
}  // namespace

hipError_t launch_reduce_f32(const ReduceArgs& a, int op, bool comp, bool deep,
                             int nranks, const Launch& l) {
  return deep ? f32<true>(a, op, comp, nranks, l)
              : f32<false>(a, op, comp, nranks, l);
}
}  // namespace pcoll
