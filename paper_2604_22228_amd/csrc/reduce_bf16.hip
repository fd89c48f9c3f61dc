// bfloat16 payloads, binary32 accumulation: sum (plain or Sum2) and max,
// and the sum with a bf16 pair (hi, lo) output.
#include "reduce_impl.hpp"

namespace pcoll {
namespace {
template <bool D>
hipError_t bf16(const ReduceArgs& a, int op, bool comp, int nranks, const Launch& l) {
  using namespace dev;
  if (op == kMax) return launch_ranks<VecTile<FMax, 2, D>>(a, nranks, l);
  if (comp) return launch_ranks<VecTile<FSum<true>, 2, D>>(a, nranks, l);
  return launch_ranks<VecTile<FSum<false>, 2, D>>(a, nranks, l);
}

template <bool D>
hipError_t pair(const ReduceArgs& a, bool comp, int nranks, const Launch& l) {
  using namespace dev;
  if (comp) return launch_ranks<VecTile<FSum<true>, 3, D>>(a, nranks, l);
  return launch_ranks<VecTile<FSum<false>, 3, D>>(a, nranks, l);
}
}  // namespace

hipError_t launch_reduce_bf16(const ReduceArgs& a, int op, bool comp,
                              bool deep, int nranks, const Launch& l) {
  return deep ? bf16<true>(a, op, comp, nranks, l)
              : bf16<false>(a, op, comp, nranks, l);
}

hipError_t launch_reduce_bf16_pair(const ReduceArgs& a, bool comp, bool deep,
                                   int nranks, const Launch& l) {
  return deep ? pair<true>(a, comp, nranks, l)
              : pair<false>(a, comp, nranks, l);
}
}  // namespace pcoll
