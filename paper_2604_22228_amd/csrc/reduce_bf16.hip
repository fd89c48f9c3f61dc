// bfloat16 payloads, binary32 accumulation: sum (plain or Sum2) and max,
// and the sum with a bf16 pair (hi, lo) output.
#include "reduce_impl.hpp"

namespace pcoll {
namespace {
template <bool D>
hipError_t bf16(const ReduceArgs& a, int op, bool comp, int nranks,
                int groups, int waves, hipStream_t s) {
  using namespace dev;
  if (op == kMax) return launch_ranks<VecTile<FMax, 2, D>>(a, nranks, groups, waves, s);
  if (comp) return launch_ranks<VecTile<FSum<true>, 2, D>>(a, nranks, groups, waves, s);
  return launch_ranks<VecTile<FSum<false>, 2, D>>(a, nranks, groups, waves, s);
}

template <bool D>
hipError_t pair(const ReduceArgs& a, bool comp, int nranks, int groups,
                int waves, hipStream_t s) {
  using namespace dev;
  if (comp) return launch_ranks<VecTile<FSum<true>, 3, D>>(a, nranks, groups, waves, s);
  return launch_ranks<VecTile<FSum<false>, 3, D>>(a, nranks, groups, waves, s);
}
}  // namespace

hipError_t launch_reduce_bf16(const ReduceArgs& a, int op, bool comp,
                              bool deep, int nranks, int groups, int waves,
                              hipStream_t s) {
  return deep ? bf16<true>(a, op, comp, nranks, groups, waves, s)
              : bf16<false>(a, op, comp, nranks, groups, waves, s);
}

hipError_t launch_reduce_bf16_pair(const ReduceArgs& a, bool comp, bool deep,
                                   int nranks, int groups, int waves,
                                   hipStream_t s) {
  return deep ? pair<true>(a, comp, nranks, groups, waves, s)
              : pair<false>(a, comp, nranks, groups, waves, s);
}
}  // namespace pcoll
