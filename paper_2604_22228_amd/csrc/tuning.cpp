// Tuned-table parsing and lookup (see tuning.hpp).
#include "tuning.hpp"

#include <sstream>

namespace pcoll {

namespace {

int parse_dtype(const std::string& s) {
  if (s == "*") return -1;
  if (s == "i32") return 0;
  if (s == "f32") return 1;
  if (s == "bf16") return 2;
  if (s == "e4m3") return 3;
  if (s == "e5m2") return 4;
  if (s == "mxfp8") return 5;
  if (s == "bf16pair") return 6;
  return -2;
}

int parse_op(const std::string& s) {
  if (s == "*") return -1;
  if (s == "sum") return 0;
  if (s == "max") return 1;
  return -2;
}

bool parse_int_or_any(const std::string& s, int* v) {
  if (s == "*") {
    *v = -1;
    return true;
  }
  try {
    size_t used = 0;
    *v = std::stoi(s, &used);
    return used == s.size();
  } catch (...) {
    return false;
  }
}

bool match(int want, int have) { return want == -1 || want == have; }

}  // namespace

std::vector<TuneRow> parse_tune_table(const std::string& text) {
  std::vector<TuneRow> rows;
  std::istringstream in(text);
  std::string line;
  while (std::getline(in, line)) {
    auto hash = line.find('#');
    if (hash != std::string::npos) line.resize(hash);
    std::istringstream ls(line);
    std::string f[12];
    int nf = 0;
    while (nf < 12 && (ls >> f[nf])) ++nf;
    std::string extra;
    if (nf < 8 || (ls >> extra)) continue;
    TuneRow r;
    r.dtype = parse_dtype(f[0]);
    r.op = parse_op(f[1]);
    if (r.dtype == -2 || r.op == -2) continue;
    if (!parse_int_or_any(f[2], &r.ranks) || !parse_int_or_any(f[3], &r.graph))
      continue;
    if (!parse_int_or_any(f[4], &r.log2_lo) ||
        !parse_int_or_any(f[5], &r.log2_hi))
      continue;
    if (!parse_int_or_any(f[6], &r.tile_elems) ||
        !parse_int_or_any(f[7], &r.groups_per_cu))
      continue;
    if (nf >= 9 && (!parse_int_or_any(f[8], &r.interleave) ||
                    r.interleave < 0 || r.interleave > (1 << 20)))
      continue;
    if (nf >= 10 && (!parse_int_or_any(f[9], &r.group_waves) ||
                     r.group_waves < 1 || r.group_waves > 8))
      continue;
    if (nf >= 11 && (!parse_int_or_any(f[10], &r.publish_batch) ||
                     r.publish_batch < 1 || r.publish_batch > 64))
      continue;
    if (nf == 12 && (!parse_int_or_any(f[11], &r.unroll) ||
                     (r.unroll != 2 && r.unroll != 4)))
      continue;
    if (r.log2_lo < 0) r.log2_lo = 0;
    if (r.log2_hi < 0) r.log2_hi = 63;
    if (r.tile_elems <= 0 || r.tile_elems % 1024 != 0 || r.groups_per_cu <= 0)
      continue;
    rows.push_back(r);
  }
  return rows;
}

TuneChoice tune_lookup(const std::vector<TuneRow>& rows, int dtype, int op,
                       int ranks, int graph, uint64_t bytes_per_rank) {
  int lg = 0;
  while (lg < 63 && (bytes_per_rank >> (lg + 1)) != 0) ++lg;
  for (const auto& r : rows) {
    if (match(r.dtype, dtype) && match(r.op, op) && match(r.ranks, ranks) &&
        match(r.graph, graph) && lg >= r.log2_lo && lg <= r.log2_hi)
      return {r.tile_elems, r.groups_per_cu, r.interleave, r.group_waves,
              r.publish_batch, r.unroll};
  }
  // built-in default: 16 KiB of output per tile, two groups per CU
  // (element bytes: 2 for bf16 and bf16 pairs, 1 for the 8-bit floats)
  const int elem = dtype == 2 || dtype == 6 ? 2
                                            : (dtype >= 3 && dtype <= 5 ? 1 : 4);
  return {16384 / elem, 2, 0, 4, 16, 4};
}

}  // namespace pcoll
