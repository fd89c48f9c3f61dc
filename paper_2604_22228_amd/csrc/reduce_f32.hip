// binary32 payloads: sum (plain or Sum2) and max.
#include "reduce_impl.hpp"

namespace pcoll {
namespace {
template <bool D>
hipError_t f32(const ReduceArgs& a, int op, bool comp, int nranks, int groups,
               int waves, hipStream_t s) {
  using namespace dev;
  if (op == kMax) return launch_ranks<VecTile<FMax, 0, D>>(a, nranks, groups, waves, s);
  if (comp) return launch_ranks<VecTile<FSum<true>, 0, D>>(a, nranks, groups, waves, s);
  return launch_ranks<VecTile<FSum<false>, 0, D>>(a, nranks, groups, waves, s);
}
}  // namespace

hipError_t launch_reduce_f32(const ReduceArgs& a, int op, bool comp, bool deep,
                             int nranks, int groups, int waves, hipStream_t s) {
  return deep ? f32<true>(a, op, comp, nranks, groups, waves, s)
              : f32<false>(a, op, comp, nranks, groups, waves, s);
}
}  // namespace pcoll
