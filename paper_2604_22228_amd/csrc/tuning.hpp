// Tuned launch parameters, looked up per request.
//
// Section 4.4: an offline exhaustive search fixes the scheduling parameters
// per configuration, separately for graph and non-graph execution; the
// tuned values are defaults that environment variables override.  Here the
// search is done by the package's autotuner, which writes a text table:
//
//   # dtype op ranks graph log2_lo log2_hi tile groups_per_cu interleave waves batch unroll
//   f32     sum 8   0     24      28      4096   1             1          4     16    4
//
// dtype in {i32, f32, bf16, e4m3, e5m2, mxfp8,
// bf16pair, *}, op in {sum, max, *}, ranks a number
// or *, graph 0 / 1 / *, and [log2_lo, log2_hi] the range of
// floor(log2(bytes per rank of the whole request)); the trailing interleave
// (tile layout, default 0; 1 = bands of the launch's workgroups, n >= 2 =
// bands of n tiles), waves-per-workgroup (default 4), publish-batch (default
// 16) and unroll (rows in flight per lane, 2 or 4, default 4) columns may be
// omitted, from the right.  The first matching row wins.  Host-only C++17.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace pcoll {

struct TuneRow {
  int dtype = -1, op = -1, ranks = -1, graph = -1;  // -1 = any
  int log2_lo = 0, log2_hi = 63;
  int tile_elems = 0, groups_per_cu = 0, interleave = 0, group_waves = 4;
  int publish_batch = 16;
  int unroll = 4;
};

struct TuneChoice {
  int tile_elems;
  int groups_per_cu;
  int interleave;
  int group_waves;
  int publish_batch;
  int unroll;
};

// Parses a table; malformed lines are skipped.  Returns the rows.
std::vector<TuneRow> parse_tune_table(const std::string& text);

// First matching row, or the built-in default.
TuneChoice tune_lookup(const std::vector<TuneRow>& rows, int dtype, int op,
                       int ranks, int graph, uint64_t bytes_per_rank);

}  // namespace pcoll
