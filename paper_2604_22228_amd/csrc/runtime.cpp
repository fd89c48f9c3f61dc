// Host runtime of libpcoll: requests, epochs, readiness, completion, the
// binding/graph cache, and the C ABI declared in include/pcoll.h.
//
// Host C++17 over the HIP runtime API; kernels are launched through the
// entry points of kernels.hpp.  Per request:
//   * host-coherent pinned memory (HostShared + ready list + arrived flags)
//     is the channel between the host thread and the running kernel:
//     pready appends to the ready list and publishes its length with a
//     store-release; the kernel stores arrived[p] = epoch when partition p
//     is final, and an epoch-stamped status if it gives up; the host's wait
//     returns once every arrived flag carries the epoch;
//   * device memory holds the partition table, the work queue and the
//     counters the kernel's wavefronts share;
//   * an LRU cache (Section 4.2's graph cache) maps each binding to its
//     descriptor table and, in graph mode, to the instantiated graph of the
//     persistent launch, created lazily on first start (Algorithm 1,
//     LaunchGraph: look up, create on a miss, launch, record an event).
#include <dlfcn.h>
#include <immintrin.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <memory>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "kernels.hpp"
#include "layout.hpp"
#include "lru_cache.hpp"
#include "noalloc.hpp"
#include "pcoll.h"

static_assert(pcoll::kNoallocMaxParts == PCOLL_NOALLOC_MAX_PARTS,
              "the header states the scratch array's partition limit");
#include "tuning.hpp"

using namespace pcoll;

namespace {

thread_local std::string g_detail;

int hip_fail(hipError_t e, const char* what) {
  g_detail = std::string(what) + ": " + hipGetErrorName(e) + " (" +
             hipGetErrorString(e) + ")";
  return PCOLL_ERR_HIP;
}

#define HIP_TRY(call)                                    \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail(e_, #call);    \
  } while (0)

int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  char* end = nullptr;
  long x = std::strtol(v, &end, 10);
  return (end && *end == '\0') ? (int)x : dflt;
}

std::string lib_dir() {
  Dl_info info;
  if (dladdr(reinterpret_cast<void*>(&lib_dir), &info) && info.dli_fname) {
    std::string p = info.dli_fname;
    auto s = p.rfind('/');
    if (s != std::string::npos) return p.substr(0, s);
  }
  return ".";
}

const std::vector<TuneRow>& tune_rows() {
  static std::once_flag once;
  static std::vector<TuneRow> rows;
  std::call_once(once, [] {
    const char* f = std::getenv("PCOLL_TUNE_FILE");
    std::string path = f && *f ? std::string(f) : lib_dir() + "/tuned_mi355x.txt";
    std::ifstream in(path);
    if (!in) return;
    std::stringstream ss;
    ss << in.rdbuf();
    rows = parse_tune_table(ss.str());
  });
  return rows;
}

bool valid_dtype(int d) { return d >= PCOLL_INT32 && d <= PCOLL_BF16_PAIR; }
// 8-bit floats: codes plus block scales (binary32 per 256 elements, or
// E8M0 bytes per 32 for MX blocks)
bool is_fp8(int d) {
  return d == PCOLL_FP8_E4M3 || d == PCOLL_FP8_E5M2 || d == PCOLL_MXFP8_E4M3;
}
bool valid_op(int o) { return o == PCOLL_SUM || o == PCOLL_MAX; }

// Partition alignment in elements: whole 128-byte cache lines, so that a
// row (1 KiB of one rank) of a partition covers exactly eight lines when
// the buffers are 128-byte aligned (rows of neighbouring tiles then never
// share a line, which each would fetch again), and whole scale blocks for
// the 8-bit floats (256 elements; 128 for MX blocks of 32).
uint64_t part_align(int dtype) {
  if (dtype == PCOLL_MXFP8_E4M3) return 128u;
  return is_fp8(dtype) ? 256u : 128u / (uint64_t)elem_bytes(dtype);
}

// Algorithm 1's chunk rule with the alignment above.
uint64_t plan_psize(uint64_t count, uint64_t nparts, uint64_t align) {
  uint64_t ps = (count + nparts - 1) / nparts;
  return (ps + align - 1) / align * align;
}

struct BindKey {
  std::vector<uintptr_t> v;
  bool operator==(const BindKey& o) const { return v == o.v; }
};
struct BindKeyHash {
  size_t operator()(const BindKey& k) const {
    uint64_t h = 1469598103934665603ull;  // FNV-1a over the words
    for (uintptr_t x : k.v) {
      h ^= (uint64_t)x;
      h *= 1099511628211ull;
    }
    return (size_t)h;
  }
};

struct Binding {
  BucketDesc* table = nullptr;   // device copy of the bucket descriptors
  hipGraphExec_t exec = nullptr; // persistent launch, captured lazily
  uint64_t exec_sig = 0;         // launch signature the graph was made for
};

}  // namespace

struct pcoll_req_s {
  int device = 0;
  int dtype = 0, op = 0, nranks = 0, nparts_per_bucket = 0, nbuckets = 0;
  std::vector<uint64_t> counts;
  uint32_t nparts_total = 0;
  std::vector<PartDesc> parts;
  pcoll_config_t cfg{};
  uint64_t total_rows = 0;
  int groups = 0;       // workgroups of the launch
  int waves = 0;        // wavefronts per workgroup of the launch
  bool deep = true;     // 4 rows in flight per lane (else 2)
  bool device_signals = false;  // a device-side ready signal was enqueued
  bool room_pending = false;    // ... and the launch does not leave room yet
  int cus = 0;
  int clock_khz = 0;

  HostShared* host = nullptr;      // host address of the pinned block
  HostShared* host_dev = nullptr;  // device address of the same block
  uint64_t* hlist = nullptr;
  uint32_t* arrived = nullptr;

  void* arena = nullptr;
  PartDesc* d_parts = nullptr;
  QEntry* d_queue = nullptr;
  uint32_t* d_done = nullptr;     // [2][nparts_total]
  uint32_t* d_queued = nullptr;
  uint32_t* d_hits = nullptr;
  uint32_t* d_tiles = nullptr;
  uint64_t* d_dlist = nullptr;       // [2][partitions] device ready rings
  uint32_t* d_dstamp = nullptr;      // [partitions] last epoch appended
  uint64_t* d_rank_marks = nullptr;  // [partitions] device per-rank marks
  uint64_t* d_trace = nullptr;       // debug trace: [trace_cap][4]
  int trace_cap = 0;
  EpochCounters* d_ctr = nullptr;  // [2]
  RingCounters* d_ring = nullptr;  // [2]

  hipStream_t stream = nullptr;
  hipStream_t launch_stream = nullptr;  // stream of the last launch
  bool bound = false;
  Binding* cur = nullptr;
  std::unique_ptr<LruCache<BindKey, Binding, BindKeyHash>> cache;
  hipStream_t capture_stream = nullptr;
  hipEvent_t ev_end = nullptr;
  // debug timing: per epoch a pair of events, stamped at a direct
  // launch's own start and end (no marker packets, which add microseconds
  // of their own), or markers around a graph replay; kTimers pairs in
  // turn, collected once complete, so that no epoch waits for the last
  // one's kernel to retire
  static constexpr int kTimers = 8;
  hipEvent_t ev_t[kTimers][2] = {};
  bool t_pending[kTimers] = {};
  int t_next = 0;
  bool ev_end_recorded = false;

  uint32_t epoch = 0;
  bool active = false;
  bool epoch_ok = false;        // the last finished epoch completed
  uint32_t scan = 0;            // first partition not yet seen arrived
  uint32_t hcount = 0;
  std::vector<uint32_t> stamp;  // epoch in which each partition was readied
  std::vector<uint64_t> mark;   // call generation that last listed it
  uint64_t mark_gen = 0;
  std::vector<int> order;       // scratch: a list in partition order
  std::vector<uint32_t> rank_mask;   // host per-rank readiness: ranks that
  std::vector<uint32_t> rank_epoch;  // readied each partition, and when
  pcoll_stats_t stats{};
  uint64_t sig = 0;             // launch signature (config-dependent args)
};

namespace {

// Waits until the kernel of the last launch has fully retired.
int drain(pcoll_req_t r) {
  if (r->ev_end_recorded) HIP_TRY(hipEventSynchronize(r->ev_end));
  return PCOLL_SUCCESS;
}

// The epoch after e: epoch 0 is never used (it tells a kernel to read the
// stamp from host memory), so after 2^32 - 1 the count goes on at 2, which
// keeps the parity alternating.  The kernel's next_epoch() is the same rule.
uint32_t epoch_after(uint32_t e) { return e + 1u == 0u ? 2u : e + 1u; }

// Opens the device ready rings for epochs `next` and the one after.
int open_rings(pcoll_req_t r, uint32_t next) {
  RingCounters rc[2];
  std::memset(rc, 0, sizeof(rc));
  const uint32_t after = epoch_after(next);
  rc[next & 1u].reserve = (uint64_t)next << 32;
  rc[after & 1u].reserve = (uint64_t)after << 32;
  HIP_TRY(hipMemcpy(r->d_ring, rc, sizeof(rc), hipMemcpyHostToDevice));
  return PCOLL_SUCCESS;
}

// Clears every epoch stamp of the request, so that the epoch after `last`
// starts from a clean slate: the device's queued stamps, ready rings,
// partition stamps, per-rank marks, counter sets and done counters, and the
// host's ready list, arrived flags, status and readiness bookkeeping.  Stamps are compared with the
// current epoch for equality (and the device's ready state by magnitude),
// so once the 32-bit count wraps, a stamp left from 2^32 epochs earlier
// could pass for a current one.  Waits for the whole device first: a
// device-side ready signal of an ended epoch may still be queued on some
// stream, and must not run after the clear.
int reset_epoch_state(pcoll_req_t r, uint32_t last) {
  HIP_TRY(hipDeviceSynchronize());
  const size_t np = r->nparts_total;
  HIP_TRY(hipMemset(r->d_queued, 0, sizeof(uint32_t) * np));
  HIP_TRY(hipMemset(r->d_dlist, 0, sizeof(uint64_t) * 2 * np));
  HIP_TRY(hipMemset(r->d_dstamp, 0, sizeof(uint32_t) * np));
  HIP_TRY(hipMemset(r->d_rank_marks, 0, sizeof(uint64_t) * np));
  // both counter sets and done halves: the next epoch's parity may be the
  // one the last launch used
  HIP_TRY(hipMemset(r->d_ctr, 0, 2 * sizeof(EpochCounters)));
  HIP_TRY(hipMemset(r->d_done, 0, sizeof(uint32_t) * 2 * np));
  std::memset(r->hlist, 0, sizeof(uint64_t) * np);
  std::memset(r->arrived, 0, sizeof(uint32_t) * np);
  r->host->status = 0;
  r->host->status_epoch = 0;
  std::fill(r->stamp.begin(), r->stamp.end(), 0u);
  std::fill(r->rank_epoch.begin(), r->rank_epoch.end(), 0u);
  std::fill(r->rank_mask.begin(), r->rank_mask.end(), 0u);
  const int rc = open_rings(r, epoch_after(last));
  if (rc) return rc;
  r->epoch = last;
  return PCOLL_SUCCESS;
}

void dispose_binding(Binding& b) {
  if (b.exec) (void)hipGraphExecDestroy(b.exec);
  if (b.table) (void)hipFree(b.table);
  b.exec = nullptr;
  b.table = nullptr;
}

uint64_t launch_signature(const pcoll_req_s* r) {
  uint64_t h = 1469598103934665603ull;
  const uint64_t v[] = {(uint64_t)r->cfg.tile_elems,
                        (uint64_t)r->cfg.min_tile_elems, (uint64_t)r->groups,
                        (uint64_t)r->cfg.comp, (uint64_t)r->cfg.debug,
                        (uint64_t)r->cfg.timeout_ms, r->total_rows,
                        (uint64_t)r->cfg.interleave, (uint64_t)r->cfg.guide,
                        (uint64_t)r->waves,
                        (uint64_t)r->cfg.publish_batch,
                        (uint64_t)r->deep};
  for (uint64_t x : v) {
    h ^= x;
    h *= 1099511628211ull;
  }
  return h;
}

int validate_config(const pcoll_req_s* r, const pcoll_config_t& c) {
  if (c.tile_elems < 1024 || c.tile_elems % 1024 != 0 ||
      c.tile_elems > (1 << 26))
    return PCOLL_ERR_ARG;
  if (c.min_tile_elems < 1024 || c.min_tile_elems % 1024 != 0 ||
      c.min_tile_elems > c.tile_elems)
    return PCOLL_ERR_ARG;
  if (c.groups < 0 || c.groups > (1 << 20)) return PCOLL_ERR_ARG;
  if (c.groups == 0 && (c.groups_per_cu < 1 || c.groups_per_cu > 64))
    return PCOLL_ERR_ARG;
  if (c.comp != 0 && c.comp != 1) return PCOLL_ERR_ARG;
  if (c.comp == 1 && (r->dtype == PCOLL_INT32 || r->op == PCOLL_MAX))
    return PCOLL_ERR_ARG;
  if (c.graph != 0 && c.graph != 1) return PCOLL_ERR_ARG;
  if (c.timeout_ms < 1 || c.timeout_ms > 3600 * 1000) return PCOLL_ERR_ARG;
  if (c.debug < 0 || c.debug > 7) return PCOLL_ERR_ARG;
  if (c.interleave < 0 || c.interleave > (1 << 20)) return PCOLL_ERR_ARG;
  if (c.guide < 0 || c.guide > 64) return PCOLL_ERR_ARG;
  if (c.unroll != 2 && c.unroll != 4) return PCOLL_ERR_ARG;
  if (c.group_waves < 1 || c.group_waves > kMaxWavesPerGroup)
    return PCOLL_ERR_ARG;
  if (c.publish_batch < 1 || c.publish_batch > kMaxPublishBatch)
    return PCOLL_ERR_ARG;
  if (c.producers < -1 || c.producers > 1) return PCOLL_ERR_ARG;
  return PCOLL_SUCCESS;
}

// Whether the launch leaves room for kernels that run beside it (the
// producers that device-side readiness follows): explicitly, or, in the
// automatic mode, once the request has seen a device-side signal.
bool producer_room(const pcoll_req_s* r, const pcoll_config_t& c) {
  return c.producers == 1 || (c.producers == -1 && r->device_signals);
}

// Elements per row: 64 lanes x 16 bytes per rank.
uint64_t row_elems(int dtype) { return 1024u / (uint64_t)elem_bytes(dtype); }

// Workgroups of a launch: the configured count, but no more than the
// launch has tiles for sure (every partition has at least max(1,
// ceil(rows / largest tile)) tiles), so that every workgroup owns a first
// tile.  `rows_of(k)` gives the rows of partition k.
template <class RowsOf>
int launch_groups(const pcoll_config_t& c, int cus, int dtype, uint32_t np,
                  RowsOf rows_of) {
  int groups = c.groups ? c.groups : c.groups_per_cu * cus;
  const uint64_t tile_rows =
      std::max<uint64_t>(1, (uint64_t)c.tile_elems / row_elems(dtype));
  uint64_t max_tiles = 0;
  for (uint32_t k = 0; k < np; ++k) {
    const uint64_t rows = rows_of(k);
    max_tiles += rows ? (rows + tile_rows - 1) / tile_rows : 1;
  }
  if ((uint64_t)groups > max_tiles) groups = (int)max_tiles;
  return groups < 1 ? 1 : groups;
}

// Workgroups of `waves` wavefronts of the selected kernel that the device
// holds at once (`cus` compute units), or 0 if HIP cannot say.  The
// persistent kernel launches no more than that: a workgroup beyond them
// would start only when a resident one has run out of tiles and exited, and
// would then reduce its own first tile alone at the end of the epoch.
int resident_groups(int dtype, int op, bool comp, bool deep, int nranks,
                    int waves, int cus) {
  int per_cu = 0;
  Launch l{1, waves, nullptr, nullptr, nullptr};
  l.per_cu = &per_cu;
  const ReduceArgs a{};
  if (launch_reduce(a, dtype, op, comp, deep, nranks, l) != hipSuccess)
    return 0;
  return per_cu > 0 ? per_cu * cus : 0;
}

// Rows of 64 lanes x 16 bytes each lane of the launch keeps loading at once
// (the 8-bit kernels: one; the others: the kernels' Unroll rule, at most 2
// for bf16 max).
int rows_in_flight(int dtype, int op, int nranks, bool deep) {
  if (is_fp8(dtype)) return 1;
  int u = nranks <= 2 ? 4 : (nranks <= 8 ? (deep ? 4 : 2) : (deep ? 2 : 1));
  if (dtype == PCOLL_BFLOAT16 && op == PCOLL_MAX && u > 2) u = 2;
  return u;
}

// Applies a configuration: workgroups and the signature of the launch.
int apply_config(pcoll_req_t r, const pcoll_config_t& c) {
  int rc = validate_config(r, c);
  if (rc) return rc;
  // Producer room: one resident wave per SIMD (one workgroup of at most 4
  // waves per compute unit, unless the workgroup count is given) and 2
  // rows in flight per lane (about 115 instead of 160-190 VGPRs per wave
  // at 8 ranks), so that producer waves, matrix-core ones included, find
  // registers and wave slots beside the resident kernel.
  const bool room = producer_room(r, c);
  const int waves = room ? std::min(c.group_waves, 4) : c.group_waves;
  pcoll_config_t eff = c;
  if (room && !c.groups) eff.groups_per_cu = 1;
  // Unless the count is given, no more workgroups than the device holds at
  // once (resident_groups).  And no more than the launch has tiles for
  // sure, so that every workgroup owns a first tile (its own number), a
  // small message does not dispatch workers that would only wait, and an
  // epoch cannot complete before every workgroup of its launch has
  // started; a graph replay, whose workgroups read the epoch stamp from
  // host memory when they start, depends on that (the host writes the next
  // stamp only after the epoch completed).
  const bool deep = !room && c.unroll != 2;
  int groups = launch_groups(eff, r->cus, r->dtype, r->nparts_total,
                             [&](uint32_t k) { return r->parts[k].rows; });
  const int fit = resident_groups(r->dtype, r->op, c.comp != 0, deep,
                                  r->nranks, waves, r->cus);
  if (!c.groups && fit > 0 && groups > fit) groups = fit;
  rc = drain(r);
  if (rc) return rc;
  if ((c.debug & 2) && groups > r->trace_cap) {  // the trace's records
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, sizeof(uint64_t) * 4 * (size_t)groups);
    if (e != hipSuccess)
      return e == hipErrorOutOfMemory ? PCOLL_ERR_NOMEM
                                      : hip_fail(e, "hipMalloc(trace)");
    if (r->d_trace) (void)hipFree(r->d_trace);
    r->d_trace = static_cast<uint64_t*>(p);
    r->trace_cap = groups;
  }
  r->cfg = c;
  r->groups = groups;
  r->waves = waves;
  r->deep = deep;
  r->room_pending = false;
  r->sig = launch_signature(r);
  if (r->cache)  // graphs captured with the old arguments are stale
    r->cache->for_each([](const BindKey&, Binding& b) {
      if (b.exec) (void)hipGraphExecDestroy(b.exec);
      b.exec = nullptr;
    });
  return PCOLL_SUCCESS;
}

// The default configuration of a request of `bytes` per rank: the tuned
// table's row, then the environment overrides.
pcoll_config_t config_for(int dtype, int op, int nranks, uint64_t bytes) {
  pcoll_config_t c{};
  // direct launch by default: the request's work is one kernel, and a
  // graph launch of one node costs more host time than a kernel launch
  c.graph = env_int("PCOLL_GRAPH", 0) ? 1 : 0;
  TuneChoice t = tune_lookup(tune_rows(), dtype, op, nranks, c.graph, bytes);
  c.tile_elems = env_int("PCOLL_TILE", t.tile_elems);
  c.min_tile_elems = env_int("PCOLL_MIN_TILE", 4096);
  if (c.min_tile_elems > c.tile_elems) c.min_tile_elems = c.tile_elems;
  c.interleave = env_int("PCOLL_INTERLEAVE", t.interleave);
  c.guide = env_int("PCOLL_GUIDE", 0);
  c.unroll = env_int("PCOLL_UNROLL", t.unroll);
  c.group_waves = env_int("PCOLL_GROUP_WAVES", t.group_waves);
  c.publish_batch = env_int("PCOLL_PUBLISH_BATCH", t.publish_batch);
  c.groups = env_int("PCOLL_GROUPS", 0);
  c.groups_per_cu = env_int("PCOLL_GROUPS_PER_CU", t.groups_per_cu);
  const bool float_sum = op == PCOLL_SUM && dtype != PCOLL_INT32;
  // compensated accumulation: on for the 8-bit floats, bf16 pairs and 16
  // ranks or more
  int comp = float_sum && (is_fp8(dtype) || dtype == PCOLL_BF16_PAIR ||
                           nranks >= 16);
  comp = env_int("PCOLL_COMP", comp);
  c.comp = float_sum && comp ? 1 : 0;
  c.timeout_ms = env_int("PCOLL_TIMEOUT_MS", 10000);
  c.debug = env_int("PCOLL_DEBUG", 0) & 7;
  c.producers = env_int("PCOLL_PRODUCERS", -1);
  if (c.producers < -1 || c.producers > 1) c.producers = -1;
  return c;
}

pcoll_config_t default_config(const pcoll_req_s* r) {
  uint64_t bytes = 0;
  for (uint64_t c : r->counts) bytes += c * (uint64_t)elem_bytes(r->dtype);
  return config_for(r->dtype, r->op, r->nranks, bytes);
}


void destroy(pcoll_req_t r) {
  if (!r) return;
  (void)hipSetDevice(r->device);
  (void)drain(r);
  r->cache.reset();
  if (r->capture_stream) (void)hipStreamDestroy(r->capture_stream);
  for (auto& pair : r->ev_t)
    for (hipEvent_t ev : pair)
      if (ev) (void)hipEventDestroy(ev);
  if (r->ev_end) (void)hipEventDestroy(r->ev_end);
  if (r->arena) (void)hipFree(r->arena);
  if (r->d_trace) (void)hipFree(r->d_trace);
  if (r->host) (void)hipHostFree(r->host);
  delete r;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int create(const std::vector<uint64_t>& counts, int dtype, int op,
           int nparts, int nranks, pcoll_req_t* out) {
  if (!out) return PCOLL_ERR_ARG;
  *out = nullptr;
  if (!valid_dtype(dtype) || !valid_op(op)) return PCOLL_ERR_ARG;
  if (nparts < 1 || nranks < 1) return PCOLL_ERR_ARG;
  if (nranks > PCOLL_MAX_RANKS) return PCOLL_ERR_UNSUPPORTED;
  if ((is_fp8(dtype) || dtype == PCOLL_BF16_PAIR) && op == PCOLL_MAX)
    return PCOLL_ERR_UNSUPPORTED;
  const uint64_t np_total = (uint64_t)nparts * counts.size();
  if (np_total > (1u << 24)) return PCOLL_ERR_UNSUPPORTED;
  for (uint64_t c : counts)
    if (c > (1ull << 40)) return PCOLL_ERR_UNSUPPORTED;

  std::unique_ptr<pcoll_req_s, void (*)(pcoll_req_t)> r(new pcoll_req_s,
                                                        destroy);
  r->dtype = dtype;
  r->op = op;
  r->nranks = nranks;
  r->nparts_per_bucket = nparts;
  r->nbuckets = (int)counts.size();
  r->counts = counts;
  r->nparts_total = (uint32_t)np_total;
  const uint64_t align = part_align(dtype);
  for (size_t b = 0; b < counts.size(); ++b) {
    const uint64_t ps = plan_psize(counts[b], (uint64_t)nparts, align);
    if (ps > (1ull << 31)) return PCOLL_ERR_UNSUPPORTED;  // 32-bit row math
    for (int k = 0; k < nparts; ++k) {
      PartDesc p{};
      const uint64_t off = std::min<uint64_t>((uint64_t)k * ps, counts[b]);
      p.off = off;
      p.len = std::min<uint64_t>(ps, counts[b] - off);
      p.bucket = (uint32_t)b;
      p.rows = (uint32_t)((p.len + row_elems(dtype) - 1) / row_elems(dtype));
      r->total_rows += p.rows;
      r->parts.push_back(p);
    }
  }
  r->stamp.assign(r->nparts_total, 0u);
  r->mark.assign(r->nparts_total, 0u);
  r->order.reserve(r->nparts_total);
  r->rank_mask.assign(r->nparts_total, 0u);
  r->rank_epoch.assign(r->nparts_total, 0u);

  HIP_TRY(hipGetDevice(&r->device));
  HIP_TRY(hipDeviceGetAttribute(&r->cus, hipDeviceAttributeMultiprocessorCount,
                                r->device));
  HIP_TRY(hipDeviceGetAttribute(&r->clock_khz, hipDeviceAttributeWallClockRate,
                                r->device));
  if (r->clock_khz <= 0) r->clock_khz = 100000;

  // host-coherent block: header, ready list, arrived flags
  const size_t hbytes =
      sizeof(HostShared) + (sizeof(uint64_t) + sizeof(uint32_t)) * np_total;
  void* hp = nullptr;
  hipError_t e = hipHostMalloc(&hp, hbytes,
                               hipHostMallocCoherent | hipHostMallocMapped);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? PCOLL_ERR_NOMEM
                                                       : hip_fail(e, "hipHostMalloc");
  std::memset(hp, 0, hbytes);
  r->host = static_cast<HostShared*>(hp);
  r->hlist = reinterpret_cast<uint64_t*>(r->host + 1);
  r->arrived = reinterpret_cast<uint32_t*>(r->hlist + np_total);
  void* dp = nullptr;
  HIP_TRY(hipHostGetDevicePointer(&dp, hp, 0));
  r->host_dev = static_cast<HostShared*>(dp);

  // device arena
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  const size_t o_parts = take(sizeof(PartDesc) * np_total);
  const size_t o_queue = take(sizeof(QEntry) * np_total);
  const size_t o_done = take(sizeof(uint32_t) * 2 * np_total);
  const size_t o_queued = take(sizeof(uint32_t) * np_total);
  const size_t o_hits = take(sizeof(uint32_t) * np_total);
  const size_t o_tiles = take(sizeof(uint32_t) * np_total);
  const size_t o_dlist = take(sizeof(uint64_t) * 2 * np_total);
  const size_t o_dstamp = take(sizeof(uint32_t) * np_total);
  const size_t o_marks = take(sizeof(uint64_t) * np_total);
  const size_t o_ctr = take(2 * sizeof(EpochCounters));
  const size_t o_ring = take(2 * sizeof(RingCounters));
  e = hipMalloc(&r->arena, off);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? PCOLL_ERR_NOMEM
                                                       : hip_fail(e, "hipMalloc");
  HIP_TRY(hipMemset(r->arena, 0, off));
  char* base = static_cast<char*>(r->arena);
  r->d_parts = reinterpret_cast<PartDesc*>(base + o_parts);
  r->d_queue = reinterpret_cast<QEntry*>(base + o_queue);
  r->d_done = reinterpret_cast<uint32_t*>(base + o_done);
  r->d_queued = reinterpret_cast<uint32_t*>(base + o_queued);
  r->d_hits = reinterpret_cast<uint32_t*>(base + o_hits);
  r->d_tiles = reinterpret_cast<uint32_t*>(base + o_tiles);
  HIP_TRY(hipMemcpy(r->d_parts, r->parts.data(),
                    sizeof(PartDesc) * r->parts.size(),
                    hipMemcpyHostToDevice));
  r->d_dlist = reinterpret_cast<uint64_t*>(base + o_dlist);
  r->d_dstamp = reinterpret_cast<uint32_t*>(base + o_dstamp);
  r->d_rank_marks = reinterpret_cast<uint64_t*>(base + o_marks);
  r->d_ctr = reinterpret_cast<EpochCounters*>(base + o_ctr);
  r->d_ring = reinterpret_cast<RingCounters*>(base + o_ring);
  // epoch stamps start at 0 (no epoch): slots, partition stamps and marks
  // are zero; the rings are open for epochs 1 and 2
  {
    const int rc = open_rings(r.get(), 1u);
    if (rc) return rc;
  }

  HIP_TRY(hipStreamCreateWithFlags(&r->capture_stream, hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&r->ev_end, hipEventDefault));
  for (auto& pair : r->ev_t)
    for (hipEvent_t& ev : pair)
      HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDefault));
  const int cap = std::max(1, env_int("PCOLL_GRAPH_CACHE", 8));
  r->cache.reset(new LruCache<BindKey, Binding, BindKeyHash>(
      (size_t)cap, [](const BindKey&, Binding& b) { dispose_binding(b); }));

  int rc = apply_config(r.get(), default_config(r.get()));
  if (rc) return rc;
  r->stats.last_kernel_ms = -1.0f;
  *out = r.release();
  return PCOLL_SUCCESS;
}

ReduceArgs make_args(const pcoll_req_s* r) {
  ReduceArgs a{};
  a.buckets = r->cur->table;
  a.parts = r->d_parts;
  a.queue = r->d_queue;
  a.done = r->d_done;
  a.queued = r->d_queued;
  a.tile_hits = (r->cfg.debug & 1) ? r->d_hits : nullptr;
  a.dlist = r->d_dlist;
  a.ctr = r->d_ctr;
  a.ring = r->d_ring;
  a.host = r->host_dev;
  a.hlist = reinterpret_cast<const uint64_t*>(r->host_dev + 1);
  a.arrived = reinterpret_cast<uint32_t*>(
      const_cast<uint64_t*>(a.hlist) + r->nparts_total);
  a.nparts_total = r->nparts_total;
  a.total_groups = (uint32_t)r->groups;
  a.total_rows = r->total_rows;
  a.row_elems = (uint32_t)row_elems(r->dtype);
  a.min_tile_rows = (uint32_t)std::max<uint64_t>(
      1, (uint64_t)r->cfg.min_tile_elems / row_elems(r->dtype));
  a.max_tile_rows = (uint32_t)std::max<uint64_t>(
      1, (uint64_t)r->cfg.tile_elems / row_elems(r->dtype));
  // 1 = bands as wide as the launch: the tiles of one round of claims
  a.interleave = r->cfg.interleave == 1 ? (uint32_t)r->groups
                                         : (uint32_t)r->cfg.interleave;
  a.tile_counts = (r->cfg.debug & 1) ? r->d_tiles : nullptr;
  a.trace = (r->cfg.debug & 2) ? r->d_trace : nullptr;
  a.guide = (uint32_t)r->cfg.guide;
  a.publish_batch = (uint32_t)r->cfg.publish_batch;
  a.timeout_ticks = (uint64_t)r->cfg.timeout_ms * (uint64_t)r->clock_khz;
  return a;
}

// One launch per epoch.  epoch == 0 makes the kernel read the stamp from
// the host struct (for graphs, whose arguments are fixed at capture).
int launch_direct(pcoll_req_t r, hipStream_t s, uint32_t epoch,
                  hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr) {
  ReduceArgs a = make_args(r);
  a.epoch = epoch;
  const Launch l{r->groups, r->waves, s, t0, t1};
  HIP_TRY(launch_reduce(a, r->dtype, r->op, r->cfg.comp != 0, r->deep,
                        r->nranks, l));
  return PCOLL_SUCCESS;
}

// Hands the work enqueued on `s` to the device now.  The HIP runtime may
// hold launches back until the host next looks at their stream (measured
// on MI355X: kernels enqueued on a stream stayed unsubmitted for 100 ms,
// and ran within microseconds of a query); a device-side ready signal held
// back that way would never run while the host waits on pinned memory, so
// every launch the host does not wait for is followed by a query.
hipError_t submit(hipStream_t s) {
  const hipError_t e = hipStreamQuery(s);
  return e == hipErrorNotReady ? hipSuccess : e;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now() - t0)
      .count();
}

// Graph mode: capture the persistent launch once per binding and
// configuration, instantiate, then replay.
int launch_graph(pcoll_req_t r) {
  Binding* b = r->cur;
  if (!b->exec || b->exec_sig != r->sig) {
    if (b->exec) {
      (void)hipGraphExecDestroy(b->exec);
      b->exec = nullptr;
    }
    auto t0 = std::chrono::steady_clock::now();
    HIP_TRY(hipStreamBeginCapture(r->capture_stream,
                                  hipStreamCaptureModeThreadLocal));
    int rc = launch_direct(r, r->capture_stream, 0);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(r->capture_stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    r->stats.last_capture_ms = ms_since(t0);
    auto t1 = std::chrono::steady_clock::now();
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      b->exec = nullptr;
      return hip_fail(e, "hipGraphInstantiate");
    }
    r->stats.last_instantiate_ms = ms_since(t1);
    b->exec_sig = r->sig;
    r->stats.graph_captures++;
  }
  HIP_TRY(hipGraphLaunch(b->exec, r->stream));
  r->stats.graph_launches++;
  return PCOLL_SUCCESS;
}

// Error recorded by the kernel for the current epoch (0 if none).
uint32_t epoch_status(const pcoll_req_s* r) {
  if (__atomic_load_n(&r->host->status_epoch, __ATOMIC_ACQUIRE) != r->epoch)
    return kStatusOk;
  return __atomic_load_n(&r->host->status, __ATOMIC_RELAXED);
}

// Whether every partition has arrived this epoch by its flag; `scan`
// remembers the first one not seen arrived, so a wait reads each flag
// about once.
bool all_arrived(pcoll_req_s* r) {
  while (r->scan < r->nparts_total &&
         __atomic_load_n(&r->arrived[r->scan], __ATOMIC_ACQUIRE) == r->epoch)
    ++r->scan;
  return r->scan == r->nparts_total;
}

// Whether the epoch's launch has retired: 1 yes, 0 not yet, or a negative
// error code (the HIP error is kept for pcoll_last_error_detail).  A launch
// that retired with no error recorded has reduced every tile, and its end
// made every store visible: then every partition has arrived, also those
// whose last tiles the kernel left unpublished.
int retired(pcoll_req_s* r) {
  const hipError_t q = hipEventQuery(r->ev_end);
  if (q == hipSuccess) return 1;
  if (q == hipErrorNotReady) return 0;
  return hip_fail(q, "hipEventQuery");
}

// Completes the epoch: every partition arrived, or the kernel gave up (then
// wait for it to drain before reporting).
int finish_epoch(pcoll_req_t r, uint32_t st) {
  r->active = false;
  r->epoch_ok = st == kStatusOk;
  if (st != kStatusOk) {
    HIP_TRY(hipEventSynchronize(r->ev_end));
    return st == kStatusTimeout ? PCOLL_ERR_ABORTED : PCOLL_ERR_TIMEOUT;
  }
  return PCOLL_SUCCESS;
}

// Debug timing: adds the times of the timed epochs whose events have
// completed (all of them, waiting, with `wait`; pair `need` at least).
int collect_timing(pcoll_req_t r, bool wait, int need = -1) {
  for (int k = 0; k < pcoll_req_s::kTimers; ++k) {
    const int i = (r->t_next + k) % pcoll_req_s::kTimers;  // oldest first
    if (!r->t_pending[i]) continue;
    if (!wait && i != need) {
      const hipError_t q = hipEventQuery(r->ev_t[i][1]);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return hip_fail(q, "hipEventQuery");
    }
    HIP_TRY(hipEventSynchronize(r->ev_t[i][1]));
    float ms = -1.0f;
    HIP_TRY(hipEventElapsedTime(&ms, r->ev_t[i][0], r->ev_t[i][1]));
    r->t_pending[i] = false;
    r->stats.last_kernel_ms = ms;
    r->stats.kernel_ms_total += ms;
    r->stats.kernel_timed++;
  }
  return PCOLL_SUCCESS;
}

// Finishes an epoch that completed: 1, or a negative error code.
int complete_ok(pcoll_req_t r) {
  const int rc = finish_epoch(r, kStatusOk);
  return rc ? rc : 1;
}

// One look at the epoch: 1 complete (then finished), 0 not yet, or a
// negative error code.  The arrived flags are read every time; the launch's
// retirement, which costs a runtime call, only with query_event.
int poll_epoch(pcoll_req_t r, bool query_event) {
  if (all_arrived(r)) return complete_ok(r);
  uint32_t st = epoch_status(r);
  if (st != kStatusOk) return finish_epoch(r, st);
  if (!query_event) return 0;
  const int rt = retired(r);
  if (rt == 0) return 0;
  if (rt < 0) {
    r->active = false;
    r->epoch_ok = false;
    return rt;
  }
  // the error word is written before the kernel retires
  st = epoch_status(r);
  if (st != kStatusOk) return finish_epoch(r, st);
  return complete_ok(r);
}

// Spins until the epoch completes.  With limit_ms >= 0, asks the kernel to
// stop waiting for unready partitions after that long.
int spin_wait(pcoll_req_t r, int limit_ms) {
  auto t0 = std::chrono::steady_clock::now();
  bool aborted = false;
  for (uint64_t it = 0;; ++it) {
    const int rc = poll_epoch(r, (it & 7) == 7);
    if (rc != 0) return rc < 0 ? rc : PCOLL_SUCCESS;
    _mm_pause();
    if (!aborted && limit_ms >= 0 && (it & 1023) == 1023 &&
        ms_since(t0) >= limit_ms) {
      __atomic_store_n(&r->host->abort, r->epoch, __ATOMIC_RELEASE);
      aborted = true;
    }
  }
}

int check_req(pcoll_req_t r) { return r ? PCOLL_SUCCESS : PCOLL_ERR_ARG; }

}  // namespace

// ===================================================================== ABI
extern "C" {

int pcoll_version(void) { return PCOLL_VERSION; }

const char* pcoll_strerror(int code) {
  switch (code) {
    case PCOLL_SUCCESS: return "success";
    case PCOLL_ERR_ARG: return "invalid argument";
    case PCOLL_ERR_STATE: return "call not valid in the request's state";
    case PCOLL_ERR_UNSUPPORTED: return "unsupported dtype/op/rank count";
    case PCOLL_ERR_HIP: return g_detail.empty() ? "HIP runtime error" : g_detail.c_str();
    case PCOLL_ERR_TIMEOUT: return "timed out before every partition arrived";
    case PCOLL_ERR_NOMEM: return "out of memory";
    case PCOLL_ERR_ABORTED: return "kernel deadline passed with partitions not ready";
    default: return "unknown error";
  }
}

int pcoll_plan(size_t count, pcoll_dtype_t dtype, int nparts, size_t* psize,
               size_t* offsets, size_t* lengths) {
  if (!valid_dtype(dtype) || nparts < 1 || !psize) return PCOLL_ERR_ARG;
  const uint64_t ps = plan_psize(count, (uint64_t)nparts, part_align(dtype));
  *psize = (size_t)ps;
  for (int k = 0; k < nparts; ++k) {
    const uint64_t off = std::min<uint64_t>((uint64_t)k * ps, count);
    if (offsets) offsets[k] = (size_t)off;
    if (lengths) lengths[k] = (size_t)std::min<uint64_t>(ps, count - off);
  }
  return PCOLL_SUCCESS;
}

int pcoll_init(size_t count, pcoll_dtype_t dtype, pcoll_op_t op, int nparts,
               int nranks, pcoll_req_t* out) {
  try {
    return create({(uint64_t)count}, (int)dtype, (int)op, nparts, nranks,
                  out);
  } catch (const std::bad_alloc&) {
    return PCOLL_ERR_NOMEM;
  } catch (...) {
    return PCOLL_ERR_HIP;
  }
}

int pcoll_init_batch(int nbuckets, const size_t* counts, pcoll_dtype_t dtype,
                     pcoll_op_t op, int nparts_per_bucket, int nranks,
                     pcoll_req_t* out) {
  if (!out) return PCOLL_ERR_ARG;
  *out = nullptr;
  if (nbuckets < 1 || !counts) return PCOLL_ERR_ARG;
  try {
    std::vector<uint64_t> c(counts, counts + nbuckets);
    return create(c, (int)dtype, (int)op, nparts_per_bucket, nranks, out);
  } catch (const std::bad_alloc&) {
    return PCOLL_ERR_NOMEM;
  } catch (...) {
    return PCOLL_ERR_HIP;
  }
}

int pcoll_bind(pcoll_req_t r, const void* const* rank_bufs, void* const* outs,
               const void* const* rank_scales, void* const* out_scales,
               void* stream) {
  if (check_req(r)) return PCOLL_ERR_ARG;
  if (!rank_bufs || !outs) return PCOLL_ERR_ARG;
  const bool fp8 = is_fp8(r->dtype);
  // second outputs: scales of the 8-bit floats, low halves of bf16 pairs
  const bool out2 = fp8 || r->dtype == PCOLL_BF16_PAIR;
  if (fp8 != (rank_scales != nullptr) || out2 != (out_scales != nullptr))
    return PCOLL_ERR_ARG;
  const int nb = r->nbuckets, P = r->nranks;
  // null is allowed only for empty buckets (never dereferenced)
  auto bad = [&](const void* p, int b, uintptr_t align) {
    return p ? ((uintptr_t)p & (align - 1)) != 0 : r->counts[(size_t)b] != 0;
  };
  for (int i = 0; i < nb * P; ++i)
    if (bad(rank_bufs[i], i / P, 16)) return PCOLL_ERR_ARG;
  for (int b = 0; b < nb; ++b)
    if (bad(outs[b], b, 16)) return PCOLL_ERR_ARG;
  if (fp8) {
    const uintptr_t sa = r->dtype == PCOLL_MXFP8_E4M3 ? 1 : 4;  // E8M0 bytes
    for (int i = 0; i < nb * P; ++i)
      if (bad(rank_scales[i], i / P, sa)) return PCOLL_ERR_ARG;
    for (int b = 0; b < nb; ++b)
      if (bad(out_scales[b], b, sa)) return PCOLL_ERR_ARG;
  } else if (out2) {
    for (int b = 0; b < nb; ++b)
      if (bad(out_scales[b], b, 16)) return PCOLL_ERR_ARG;
  }
  if (r->active) return PCOLL_ERR_STATE;
  try {
    BindKey key;
    key.v.reserve((size_t)nb * (2 * P + 2) + 1);
    for (int i = 0; i < nb * P; ++i) key.v.push_back((uintptr_t)rank_bufs[i]);
    for (int b = 0; b < nb; ++b) key.v.push_back((uintptr_t)outs[b]);
    if (fp8)
      for (int i = 0; i < nb * P; ++i) key.v.push_back((uintptr_t)rank_scales[i]);
    if (out2)
      for (int b = 0; b < nb; ++b) key.v.push_back((uintptr_t)out_scales[b]);
    key.v.push_back((uintptr_t)stream);
    HIP_TRY(hipSetDevice(r->device));
    Binding* hit = r->cache->get(key);
    if (hit) {
      r->stats.cache_hits++;
    } else {
      r->stats.cache_misses++;
      std::vector<BucketDesc> tab((size_t)nb);
      for (int b = 0; b < nb; ++b) {
        BucketDesc& d = tab[(size_t)b];
        std::memset(&d, 0, sizeof(d));
        for (int q = 0; q < P; ++q) {
          d.in[q] = rank_bufs[b * P + q];
          d.in_scale[q] = fp8 ? rank_scales[b * P + q] : nullptr;
        }
        d.out = outs[b];
        d.out_scale = out2 ? out_scales[b] : nullptr;
        d.count = r->counts[(size_t)b];
      }
      Binding nb_{};
      HIP_TRY(hipMalloc(&nb_.table, sizeof(BucketDesc) * tab.size()));
      hipError_t e = hipMemcpy(nb_.table, tab.data(),
                               sizeof(BucketDesc) * tab.size(),
                               hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        (void)hipFree(nb_.table);
        return hip_fail(e, "hipMemcpy(bucket table)");
      }
      // an eviction may free a table or graph the last kernel used
      int rc = drain(r);
      if (rc) {
        (void)hipFree(nb_.table);
        return rc;
      }
      const size_t ev0 = r->cache->evictions();
      hit = &r->cache->put(key, nb_);
      r->stats.cache_evictions += r->cache->evictions() - ev0;
    }
    r->cur = hit;
    r->stream = static_cast<hipStream_t>(stream);
    r->bound = true;
    return PCOLL_SUCCESS;
  } catch (const std::bad_alloc&) {
    return PCOLL_ERR_NOMEM;
  }
}

int pcoll_start(pcoll_req_t r) {
  if (check_req(r)) return PCOLL_ERR_ARG;
  if (!r->bound || r->active) return PCOLL_ERR_STATE;
  HIP_TRY(hipSetDevice(r->device));
  // epoch 0 means "read the stamp from host memory" to the kernel, and the
  // counter sets alternate by parity: after wrapping, continue at 2, from
  // cleared stamps
  if (r->cfg.debug) {  // completed timings; the pair this epoch reuses
    const int rc = collect_timing(r, false, r->t_next);
    if (rc) return rc;
  }
  // the first device-side signal of a request in the automatic producer
  // mode: leave room from this launch on
  if (r->room_pending) {
    const int rc = apply_config(r, r->cfg);
    if (rc) return rc;
  }
  const uint32_t e = epoch_after(r->epoch);
  if (e < r->epoch) {
    const int rc = reset_epoch_state(r, r->epoch);
    if (rc) return rc;
  }
  // the previous launch may still be draining (its epoch completes when
  // every partition has arrived): a launch on another stream must follow it
  if (r->ev_end_recorded && r->launch_stream != r->stream)
    HIP_TRY(hipStreamWaitEvent(r->stream, r->ev_end, 0));
  // a draining launch has queued every partition, so it no longer reads
  // the ready list or the abort word; list entries of earlier epochs carry
  // older tags
  r->host->abort = 0;
  __atomic_store_n(&r->host->epoch, e, __ATOMIC_RELEASE);
  r->hcount = 0;
  r->scan = 0;
  hipEvent_t* tp = r->cfg.debug ? r->ev_t[r->t_next] : nullptr;
  if (r->cfg.debug & 1) {
    HIP_TRY(hipMemsetAsync(r->d_hits, 0, sizeof(uint32_t) * r->nparts_total,
                           r->stream));
    HIP_TRY(hipMemsetAsync(r->d_tiles, 0, sizeof(uint32_t) * r->nparts_total,
                           r->stream));
  }
  // a graph replay is timed by markers around it
  if (tp && r->cfg.graph) HIP_TRY(hipEventRecord(tp[0], r->stream));
  int rc = r->cfg.graph ? launch_graph(r)
                        : launch_direct(r, r->stream, e,
                                        tp ? tp[0] : nullptr,
                                        tp ? tp[1] : nullptr);
  if (rc) return rc;
  if (tp && r->cfg.graph) HIP_TRY(hipEventRecord(tp[1], r->stream));
  if (tp) {
    r->t_pending[r->t_next] = true;
    r->t_next = (r->t_next + 1) % pcoll_req_s::kTimers;
  }
  HIP_TRY(hipEventRecord(r->ev_end, r->stream));
  // the kernel starts now, not when the host next looks at the stream: it
  // then runs while the host issues the epoch's ready signals
  HIP_TRY(submit(r->stream));
  r->ev_end_recorded = true;
  r->launch_stream = r->stream;
  r->epoch = e;
  r->active = true;
  r->epoch_ok = false;
  r->stats.epochs++;
  r->stats.groups = r->groups;
  r->stats.group_waves = r->waves;
  r->stats.unroll = rows_in_flight(r->dtype, r->op, r->nranks, r->deep);
  return PCOLL_SUCCESS;
}

// A device-side signal was enqueued: in the automatic producer mode, the
// next launch leaves room for producers (this epoch's kernel is running).
static void note_device_signal(pcoll_req_t r) {
  if (!r->device_signals) {
    r->device_signals = true;
    r->room_pending = r->cfg.producers == -1;
  }
}

// Where the device-side signals of the current epoch append.
static RingArgs ring_args(const pcoll_req_s* r) {
  RingArgs a{};
  a.dlist = r->d_dlist;
  a.ring = r->d_ring;
  a.dstamp = r->d_dstamp;
  a.capacity = r->nparts_total;
  a.epoch = r->epoch;
  return a;
}

static int publish_ready(pcoll_req_t r, const int* parts, int n, int first) {
  // validate everything first: all-or-nothing, in one pass (a list entry
  // seen earlier in the same call carries this call's mark)
  const uint64_t gen = ++r->mark_gen;
  for (int i = 0; i < n; ++i) {
    const int p = parts ? parts[i] : first + i;
    if (p < 0 || (uint32_t)p >= r->nparts_total) return PCOLL_ERR_ARG;
    if (r->stamp[(size_t)p] == r->epoch) return PCOLL_ERR_STATE;
    if (r->mark[(size_t)p] == gen) return PCOLL_ERR_ARG;  // duplicate
    r->mark[(size_t)p] = gen;
  }
  // one call readies its partitions at the same instant, so their order in
  // the call means nothing: queue them in partition order, which keeps the
  // neighbouring partitions of a bucket together in the kernel's work queue
  // (tiles claimed together then read neighbouring memory).  A long list is
  // ordered by a scan of the marks, a short one by sorting a copy.
  if (parts && n > 1) {
    r->order.clear();
    if ((uint64_t)n * 8u >= r->nparts_total) {
      for (uint32_t p = 0; p < r->nparts_total; ++p)
        if (r->mark[p] == gen) r->order.push_back((int)p);
    } else {
      r->order.assign(parts, parts + n);
      std::sort(r->order.begin(), r->order.end());
    }
    parts = r->order.data();
  }
  // each entry carries the epoch: the kernel takes the prefix of the list
  // whose entries carry the current one, so no count is published
  const uint64_t tag = (uint64_t)r->epoch << 32;
  for (int i = 0; i < n; ++i) {
    const int p = parts ? parts[i] : first + i;
    r->stamp[(size_t)p] = r->epoch;
    __atomic_store_n(&r->hlist[r->hcount++], tag | (uint32_t)p,
                     __ATOMIC_RELEASE);
  }
  return PCOLL_SUCCESS;
}

int pcoll_pready(pcoll_req_t r, int part) {
  if (check_req(r)) return PCOLL_ERR_ARG;
  if (!r->active) return PCOLL_ERR_STATE;
  return publish_ready(r, &part, 1, 0);
}

int pcoll_pready_range(pcoll_req_t r, int first, int last) {
  if (check_req(r)) return PCOLL_ERR_ARG;
  if (!r->active) return PCOLL_ERR_STATE;
  if (last < first) return PCOLL_ERR_ARG;
  return publish_ready(r, nullptr, last - first + 1, first);
}

int pcoll_pready_rank(pcoll_req_t r, int rank, int part) {
  if (check_req(r)) return PCOLL_ERR_ARG;
  if (rank < 0 || rank >= r->nranks) return PCOLL_ERR_ARG;
  if (part < 0 || (uint32_t)part >= r->nparts_total) return PCOLL_ERR_ARG;
  if (!r->active) return PCOLL_ERR_STATE;
  const size_t p = (size_t)part;
  if (r->stamp[p] == r->epoch) return PCOLL_ERR_STATE;  // already ready
  if (r->rank_epoch[p] != r->epoch) {
    r->rank_epoch[p] = r->epoch;
    r->rank_mask[p] = 0u;
  }
  const uint32_t bit = 1u << rank;
  if (r->rank_mask[p] & bit) return PCOLL_ERR_STATE;  // this rank, twice
  r->rank_mask[p] |= bit;
  if (r->rank_mask[p] != (1u << r->nranks) - 1u) return PCOLL_SUCCESS;
  return publish_ready(r, &part, 1, 0);  // the last rank: queue it
}

int pcoll_pready_rank_on_stream(pcoll_req_t r, int rank, const int* parts_dev,
                                int n, void* stream) {
  if (check_req(r)) return PCOLL_ERR_ARG;
  if (rank < 0 || rank >= r->nranks) return PCOLL_ERR_ARG;
  if (n < 0 || (n > 0 && !parts_dev)) return PCOLL_ERR_ARG;
  if (!r->active) return PCOLL_ERR_STATE;
  if (static_cast<hipStream_t>(stream) == r->stream) return PCOLL_ERR_ARG;
  HIP_TRY(hipSetDevice(r->device));
  PreadyRankArgs a{};
  a.parts = parts_dev;
  a.n = (uint32_t)n;
  a.rank = (uint32_t)rank;
  a.full = (1u << r->nranks) - 1u;
  a.rank_marks = r->d_rank_marks;
  a.ring = ring_args(r);
  HIP_TRY(launch_pready_rank(a, static_cast<hipStream_t>(stream)));
  HIP_TRY(submit(static_cast<hipStream_t>(stream)));
  note_device_signal(r);
  return PCOLL_SUCCESS;
}

int pcoll_pready_list(pcoll_req_t r, int n, const int* parts) {
  if (check_req(r)) return PCOLL_ERR_ARG;
  if (n < 0 || (n > 0 && !parts)) return PCOLL_ERR_ARG;
  if (!r->active) return PCOLL_ERR_STATE;
  try {
    return publish_ready(r, parts, n, 0);
  } catch (const std::bad_alloc&) {
    return PCOLL_ERR_NOMEM;
  }
}

int pcoll_pready_on_stream(pcoll_req_t r, const int* parts_dev, int n,
                           void* stream) {
  if (check_req(r)) return PCOLL_ERR_ARG;
  if (n < 0 || (n > 0 && !parts_dev)) return PCOLL_ERR_ARG;
  if (!r->active) return PCOLL_ERR_STATE;
  if (static_cast<hipStream_t>(stream) == r->stream) return PCOLL_ERR_ARG;
  HIP_TRY(hipSetDevice(r->device));
  PreadyArgs a{};
  a.parts = parts_dev;
  a.n = (uint32_t)n;
  a.ring = ring_args(r);
  HIP_TRY(launch_pready(a, static_cast<hipStream_t>(stream)));
  HIP_TRY(submit(static_cast<hipStream_t>(stream)));
  note_device_signal(r);
  return PCOLL_SUCCESS;
}

int pcoll_parrived(pcoll_req_t r, int part, int* flag) {
  if (check_req(r) || !flag) return PCOLL_ERR_ARG;
  if (part < 0 || (uint32_t)part >= r->nparts_total) return PCOLL_ERR_ARG;
  if (r->epoch == 0) return PCOLL_ERR_STATE;
  *flag = 0;
  if (__atomic_load_n(&r->arrived[part], __ATOMIC_ACQUIRE) == r->epoch) {
    *flag = 1;
    return PCOLL_SUCCESS;
  }
  if (!r->active) {
    *flag = r->epoch_ok ? 1 : 0;
    return PCOLL_SUCCESS;
  }
  // a launch that retired cleanly has completed every partition
  const int rt = retired(r);
  if (rt < 0) return rt;
  *flag = rt == 1 && epoch_status(r) == kStatusOk;
  return PCOLL_SUCCESS;
}

int pcoll_test(pcoll_req_t r, int* flag) {
  if (check_req(r) || !flag) return PCOLL_ERR_ARG;
  if (!r->active) {
    *flag = 1;
    return PCOLL_SUCCESS;
  }
  const int rc = poll_epoch(r, true);
  *flag = rc != 0;
  return rc < 0 ? rc : PCOLL_SUCCESS;
}

int pcoll_wait(pcoll_req_t r) {
  if (check_req(r)) return PCOLL_ERR_ARG;
  if (!r->active) return PCOLL_SUCCESS;
  return spin_wait(r, -1);
}

int pcoll_wait_timeout(pcoll_req_t r, int ms) {
  if (check_req(r) || ms < 0) return PCOLL_ERR_ARG;
  if (!r->active) return PCOLL_SUCCESS;
  return spin_wait(r, ms);
}

int pcoll_wait_on_stream(pcoll_req_t r, void* stream) {
  if (check_req(r)) return PCOLL_ERR_ARG;
  if (!r->active) return PCOLL_ERR_STATE;
  HIP_TRY(hipStreamWaitEvent(static_cast<hipStream_t>(stream), r->ev_end, 0));
  return PCOLL_SUCCESS;
}

int pcoll_free(pcoll_req_t r) {
  if (check_req(r)) return PCOLL_ERR_ARG;
  if (r->active) return PCOLL_ERR_STATE;
  destroy(r);
  return PCOLL_SUCCESS;
}

int pcoll_reduce_noalloc(size_t count, pcoll_dtype_t dtype_, pcoll_op_t op_,
                         int nparts, int nranks, const void* const* rank_bufs,
                         void* out, const void* const* rank_scales,
                         void* out_scale, void* stream) {
  const int dtype = (int)dtype_, op = (int)op_;
  // the argument rules of pcoll_init and pcoll_bind
  if (!valid_dtype(dtype) || !valid_op(op) || nparts < 1 || nranks < 1)
    return PCOLL_ERR_ARG;
  if (nranks > PCOLL_MAX_RANKS) return PCOLL_ERR_UNSUPPORTED;
  if ((is_fp8(dtype) || dtype == PCOLL_BF16_PAIR) && op == PCOLL_MAX)
    return PCOLL_ERR_UNSUPPORTED;
  // beyond the scratch array (the error path allocates nothing either)
  if ((uint32_t)nparts > kNoallocMaxParts) return PCOLL_ERR_UNSUPPORTED;
  if ((uint64_t)count > (1ull << 40)) return PCOLL_ERR_UNSUPPORTED;
  const uint64_t ps = plan_psize(count, (uint64_t)nparts, part_align(dtype));
  if (ps > (1ull << 31)) return PCOLL_ERR_UNSUPPORTED;
  const bool fp8 = is_fp8(dtype);
  const bool out2 = fp8 || dtype == PCOLL_BF16_PAIR;
  if (!rank_bufs || fp8 != (rank_scales != nullptr) ||
      out2 != (out_scale != nullptr))
    return PCOLL_ERR_ARG;
  auto bad = [&](const void* p, uintptr_t align) {
    return p ? ((uintptr_t)p & (align - 1)) != 0 : count != 0;
  };
  for (int q = 0; q < nranks; ++q)
    if (bad(rank_bufs[q], 16)) return PCOLL_ERR_ARG;
  if (bad(out, 16)) return PCOLL_ERR_ARG;
  if (fp8) {
    const uintptr_t sa = dtype == PCOLL_MXFP8_E4M3 ? 1 : 4;
    for (int q = 0; q < nranks; ++q)
      if (bad(rank_scales[q], sa)) return PCOLL_ERR_ARG;
    if (bad(out_scale, sa)) return PCOLL_ERR_ARG;
  } else if (out2 && bad(out_scale, 16)) {
    return PCOLL_ERR_ARG;
  }
  const uint32_t np = (uint32_t)nparts;
  const NoallocLayout L = noalloc_layout(np);
  if (L.total > kNoallocScratchBytes) return PCOLL_ERR_UNSUPPORTED;

  int dev = 0, cus = 0, khz = 0;
  HIP_TRY(hipGetDevice(&dev));
  void* scratch = nullptr;
  HIP_TRY(noalloc_scratch(dev, &scratch));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                                dev));
  HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  if (khz <= 0) khz = 100000;
  const pcoll_config_t c = config_for(
      dtype, op, nranks, (uint64_t)count * (uint64_t)elem_bytes(dtype));
  const uint64_t re = row_elems(dtype);
  auto len_of = [&](uint32_t k) {
    const uint64_t off = std::min<uint64_t>((uint64_t)k * ps, count);
    return std::min<uint64_t>(ps, count - off);
  };
  auto rows_of = [&](uint32_t k) { return (len_of(k) + re - 1) / re; };
  int groups = launch_groups(c, cus, dtype, np, rows_of);
  const int fit = resident_groups(dtype, op, c.comp != 0, c.unroll != 2,
                                  nranks, c.group_waves, cus);
  if (!c.groups && fit > 0 && groups > fit) groups = fit;
  uint64_t total_rows = 0;
  for (uint32_t k = 0; k < np; ++k) total_rows += rows_of(k);

  unsigned char* base = static_cast<unsigned char*>(scratch);
  NoallocSetup s{};
  s.base = base;
  s.layout = L;
  std::memset(&s.bucket, 0, sizeof(s.bucket));
  for (int q = 0; q < nranks; ++q) {
    s.bucket.in[q] = rank_bufs[q];
    s.bucket.in_scale[q] = fp8 ? rank_scales[q] : nullptr;
  }
  s.bucket.out = out;
  s.bucket.out_scale = out2 ? out_scale : nullptr;
  s.bucket.count = count;
  s.count = count;
  s.psize = ps;
  s.nparts = np;
  s.row_elems = (uint32_t)re;
  s.epoch = 1;  // every stamp is rewritten by the set-up launch
  const hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(launch_noalloc_setup(s, st));

  ReduceArgs a{};
  a.buckets = reinterpret_cast<const BucketDesc*>(base + L.bucket);
  a.parts = reinterpret_cast<const PartDesc*>(base + L.parts);
  a.queue = reinterpret_cast<QEntry*>(base + L.queue);
  a.done = reinterpret_cast<uint32_t*>(base + L.done);
  a.queued = reinterpret_cast<uint32_t*>(base + L.queued);
  a.dlist = reinterpret_cast<uint64_t*>(base + L.dlist);
  a.ctr = reinterpret_cast<EpochCounters*>(base + L.ctr);
  a.ring = reinterpret_cast<RingCounters*>(base + L.ring);
  a.host = reinterpret_cast<HostShared*>(base + L.host);
  a.hlist = reinterpret_cast<const uint64_t*>(base + L.hlist);
  a.arrived = reinterpret_cast<uint32_t*>(base + L.arrived);
  a.nparts_total = np;
  a.total_groups = (uint32_t)groups;
  a.total_rows = total_rows;
  a.row_elems = (uint32_t)re;
  a.min_tile_rows =
      (uint32_t)std::max<uint64_t>(1, (uint64_t)c.min_tile_elems / re);
  a.max_tile_rows = (uint32_t)std::max<uint64_t>(1, (uint64_t)c.tile_elems / re);
  a.interleave = c.interleave == 1 ? (uint32_t)groups : (uint32_t)c.interleave;
  a.guide = (uint32_t)c.guide;
  a.publish_batch = (uint32_t)c.publish_batch;
  a.epoch = s.epoch;
  a.timeout_ticks = (uint64_t)c.timeout_ms * (uint64_t)khz;
  const Launch l{groups, c.group_waves, st, nullptr, nullptr};
  HIP_TRY(launch_reduce(a, dtype, op, c.comp != 0, c.unroll != 2, nranks, l));
  return PCOLL_SUCCESS;
}

int pcoll_get_config(pcoll_req_t r, pcoll_config_t* cfg) {
  if (check_req(r) || !cfg) return PCOLL_ERR_ARG;
  *cfg = r->cfg;
  return PCOLL_SUCCESS;
}

int pcoll_set_config(pcoll_req_t r, const pcoll_config_t* cfg) {
  if (check_req(r) || !cfg) return PCOLL_ERR_ARG;
  if (r->active) return PCOLL_ERR_STATE;
  // the residency query and the debug trace's allocation are per device
  HIP_TRY(hipSetDevice(r->device));
  try {
    return apply_config(r, *cfg);
  } catch (const std::bad_alloc&) {
    return PCOLL_ERR_NOMEM;
  }
}

int pcoll_num_parts(pcoll_req_t r, int* n) {
  if (check_req(r) || !n) return PCOLL_ERR_ARG;
  *n = (int)r->nparts_total;
  return PCOLL_SUCCESS;
}

int pcoll_part_info(pcoll_req_t r, int part, int* bucket, size_t* offset,
                    size_t* length) {
  if (check_req(r)) return PCOLL_ERR_ARG;
  if (part < 0 || (uint32_t)part >= r->nparts_total) return PCOLL_ERR_ARG;
  const PartDesc& p = r->parts[(size_t)part];
  if (bucket) *bucket = (int)p.bucket;
  if (offset) *offset = (size_t)p.off;
  if (length) *length = (size_t)p.len;
  return PCOLL_SUCCESS;
}

int pcoll_get_stats(pcoll_req_t r, pcoll_stats_t* st) {
  if (check_req(r) || !st) return PCOLL_ERR_ARG;
  if (!r->active) {
    const int rc = collect_timing(r, true);
    if (rc) return rc;
  }
  *st = r->stats;
  return PCOLL_SUCCESS;
}

int pcoll_debug_set_epoch(pcoll_req_t r, uint32_t last) {
  if (check_req(r)) return PCOLL_ERR_ARG;
  if (r->active) return PCOLL_ERR_STATE;
  HIP_TRY(hipSetDevice(r->device));
  return reset_epoch_state(r, last);
}

int pcoll_debug_trace(pcoll_req_t r, uint64_t* stamps, int n, int* groups,
                      int* clock_khz) {
  if (check_req(r) || n < 0 || (n > 0 && !stamps)) return PCOLL_ERR_ARG;
  if (!(r->cfg.debug & 2) || r->active || r->epoch == 0)
    return PCOLL_ERR_STATE;
  HIP_TRY(hipSetDevice(r->device));
  const int rc = drain(r);
  if (rc) return rc;
  const size_t words = std::min<size_t>((size_t)n, 4 * (size_t)r->groups);
  if (words)
    HIP_TRY(hipMemcpy(stamps, r->d_trace, sizeof(uint64_t) * words,
                      hipMemcpyDeviceToHost));
  if (groups) *groups = r->groups;
  if (clock_khz) *clock_khz = r->clock_khz;
  return PCOLL_SUCCESS;
}

int pcoll_debug_tile_hits(pcoll_req_t r, uint32_t* hits, uint32_t* tiles,
                          int n) {
  if (check_req(r) || !hits || !tiles || n < (int)r->nparts_total)
    return PCOLL_ERR_ARG;
  if (!(r->cfg.debug & 1) || r->active) return PCOLL_ERR_STATE;
  HIP_TRY(hipSetDevice(r->device));
  int rc = drain(r);
  if (rc) return rc;
  HIP_TRY(hipMemcpy(hits, r->d_hits, sizeof(uint32_t) * r->nparts_total,
                    hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(tiles, r->d_tiles, sizeof(uint32_t) * r->nparts_total,
                    hipMemcpyDeviceToHost));
  return PCOLL_SUCCESS;
}

int pcoll_pack_bf16(const float* src, uint16_t* dst, size_t n, void* stream) {
  if (n && (!src || !dst || ((uintptr_t)src & 15u) || ((uintptr_t)dst & 15u)))
    return PCOLL_ERR_ARG;
  HIP_TRY(launch_pack_bf16(src, dst, n, static_cast<hipStream_t>(stream)));
  return PCOLL_SUCCESS;
}

int pcoll_pack_fp8(const float* src, uint8_t* dst, float* scales, size_t n,
                   void* stream) {
  if (n && (!src || !dst || !scales || ((uintptr_t)src & 15u) ||
            ((uintptr_t)dst & 15u) || ((uintptr_t)scales & 3u)))
    return PCOLL_ERR_ARG;
  HIP_TRY(launch_pack_e4m3(src, dst, scales, n,
                           static_cast<hipStream_t>(stream)));
  return PCOLL_SUCCESS;
}

int pcoll_pack_e5m2(const float* src, uint8_t* dst, float* scales, size_t n,
                    void* stream) {
  if (n && (!src || !dst || !scales || ((uintptr_t)src & 15u) ||
            ((uintptr_t)dst & 15u) || ((uintptr_t)scales & 3u)))
    return PCOLL_ERR_ARG;
  HIP_TRY(launch_pack_e5m2(src, dst, scales, n,
                           static_cast<hipStream_t>(stream)));
  return PCOLL_SUCCESS;
}

int pcoll_pack_mxfp8(const float* src, uint8_t* dst, uint8_t* scales,
                     size_t n, void* stream) {
  if (n && (!src || !dst || !scales || ((uintptr_t)src & 15u) ||
            ((uintptr_t)dst & 15u)))
    return PCOLL_ERR_ARG;
  HIP_TRY(launch_pack_mx(src, dst, scales, n,
                         static_cast<hipStream_t>(stream)));
  return PCOLL_SUCCESS;
}

int pcoll_probe_copy(void* dst, const void* src, size_t bytes, void* stream) {
  if (bytes % 16 || (bytes && (!src || !dst || ((uintptr_t)src & 15u) ||
                               ((uintptr_t)dst & 15u))))
    return PCOLL_ERR_ARG;
  HIP_TRY(launch_copy(dst, src, bytes, static_cast<hipStream_t>(stream)));
  return PCOLL_SUCCESS;
}

int pcoll_probe_stream(const void* const* srcs, int nsrc, void* dst,
                       size_t bytes, int write, int layout, void* stream) {
  if (!srcs || (nsrc != 1 && nsrc != 2 && nsrc != 4 && nsrc != 8 &&
                nsrc != 16) ||
      (write != 0 && write != 1) || layout < 0 || layout > 2 ||
      bytes % (layout == 1 ? 1024 : 16) ||
      (layout == 1 && bytes > (1ull << 36)) ||
      !dst ||
      ((uintptr_t)dst & 15u))
    return PCOLL_ERR_ARG;
  for (int r = 0; r < nsrc; ++r)
    if (bytes && (!srcs[r] || ((uintptr_t)srcs[r] & 15u))) return PCOLL_ERR_ARG;
  StreamTiles t{};
  if (layout) {
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                                  dev));
    if (layout == 1) {
      // the headline reduce's tile schedule: tiles of 32 rows (8192
      // binary32 elements), bands of 16 tiles, 2 workgroups of 8 waves per
      // compute unit
      t.groups = (uint32_t)(2 * std::max(cus, 1));
      t.waves = 8;
      t.tile_rows = 32;
      t.band = 16;
    } else {
      // contiguous shares: 4 workgroups of 256 threads per compute unit
      t.groups = (uint32_t)(4 * std::max(cus, 1));
      t.chunked = 1;
    }
  }
  HIP_TRY(launch_stream(srcs, nsrc, dst, bytes, write != 0,
                        layout ? &t : nullptr,
                        static_cast<hipStream_t>(stream)));
  return PCOLL_SUCCESS;
}

int pcoll_probe_fill(void* dst, size_t bytes, uint32_t value, void* stream) {
  if (bytes % 16 || (bytes && (!dst || ((uintptr_t)dst & 15u))))
    return PCOLL_ERR_ARG;
  HIP_TRY(launch_fill(dst, bytes, value, static_cast<hipStream_t>(stream)));
  return PCOLL_SUCCESS;
}

int pcoll_device_info(int* cus, int* wall_clock_khz, char* arch,
                      int arch_len) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (cus)
    HIP_TRY(hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount,
                                  dev));
  if (wall_clock_khz)
    HIP_TRY(hipDeviceGetAttribute(wall_clock_khz,
                                  hipDeviceAttributeWallClockRate, dev));
  if (arch && arch_len > 0) {
    hipDeviceProp_t p;
    HIP_TRY(hipGetDeviceProperties(&p, dev));
    std::snprintf(arch, (size_t)arch_len, "%s", p.gcnArchName);
  }
  return PCOLL_SUCCESS;
}

const char* pcoll_last_error_detail(void) { return g_detail.c_str(); }

}  // extern "C"
