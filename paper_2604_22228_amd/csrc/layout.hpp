// Memory layout shared by the host runtime (C++17, g++) and the gfx950
// kernels (HIP).  Plain structs only: no HIP types, no methods.
//
// One request reduces `nbuckets` messages ("buckets") of P rank
// contributions each.  Bucket b is split into nparts partitions by the chunk
// rule of Algorithm 1 (Section 4.3): equal lengths fixed in advance, running
// offsets, the last one clipped.  Global partition g = b * nparts + k.  A
// partition is a sequence of rows (one row = 64 lanes x 16 bytes per rank)
// and is cut into tiles, the unit one workgroup reduces: a tile is a set of
// rows, consecutive or interleaved with the partition's other tiles, and
// the number of tiles is chosen when the partition is queued.  Destination
// regions of partitions and tiles are disjoint (Section 4.5, Ordering
// Guarantee), so each is written once.
#pragma once
#include <stdint.h>

namespace pcoll {

constexpr int kMaxRanks = 16;
constexpr int kMaxPublishBatch = 64;

// Per bucket, in device memory; written once at bind time, read-only to the
// kernels.
struct BucketDesc {
  const void* in[kMaxRanks];        // rank contributions (device pointers)
  const void* in_scale[kMaxRanks];  // 8-bit floats only: block scales
                                    // (binary32 per 256 elements, or E8M0
                                    // bytes per 32 for MX blocks)
  void* out;                        // reduced message
  void* out_scale;                  // 8-bit floats only: output scales
  uint64_t count;                   // elements in the bucket
  uint64_t reserved;
};

// Per global partition, in device memory; read-only to the kernels.
struct PartDesc {
  uint64_t off;     // first element, relative to the bucket start
  uint64_t len;     // elements (0 for empty partitions)
  uint32_t bucket;  // owning bucket
  uint32_t rows;    // ceil(len / row_elems): rows of 64 lanes x 16 bytes
  uint64_t reserved;
};

// One entry of the device work queue: partitions in the order they were
// found ready, with the running total of their tiles (a partition's tile
// count is the difference of consecutive totals; it is chosen when the
// partition is queued, see persistent.hpp).
struct QEntry {
  uint32_t part;
  uint32_t cum_end;  // tiles of all entries up to and including this one
};

// Host-coherent pinned memory shared with the host thread.  Followed in the
// same allocation by the ready list hlist[nparts] (uint64 tagged entries)
// and the arrived stamps arrived[nparts] (uint32).
struct HostShared {
  uint32_t epoch;         // host: stamp of the next / running epoch, stored
                          // before the launch
  uint32_t abort;         // host: == epoch asks the kernel to give up
  uint32_t status;        // device: error code of epoch status_epoch
  uint32_t status_epoch;  // device: epoch the status belongs to
  uint32_t reserved[28];
};

// Device-memory counters of one epoch, each group on its own 128-B line so
// that polling one does not contend with atomics on another.  A request
// holds two sets: epoch e uses set e & 1, and its launch clears the other
// set (and the other half of the done counters) for epoch e + 1, which the
// stream orders after it.  So no separate reset launch precedes the reduce
// kernel.
struct EpochCounters {
  uint32_t claim;                 // tiles handed out beyond the first round
  uint32_t pad0[31];
  uint64_t qstate;                // (queue entries << 32) | queued tiles
  uint32_t pad1[30];
  uint32_t ilock;                 // ingest lock (0 free, 1 held)
  uint32_t hconsumed;             // host ready entries already queued
  uint64_t queued_rows;           // rows of the partitions queued so far
  uint32_t dconsumed;             // device ring entries already queued
  uint32_t pad2[27];
  uint32_t error;                 // first error seen this epoch
  uint32_t pad3[31];
};

// Device ready rings.  Device-side signals of epoch e append to ring e & 1
// (slots dlist[(e & 1) * nparts_total ...]).  Its reservation word holds
// (epoch << 32) | entries: a writer reserves with a compare-and-swap only
// while the word carries the writer's own epoch, so a signal that runs
// after its epoch ended (a wait_timeout ended it while the signal was still
// queued behind its producer) reserves nothing in a later epoch's ring.
// The launch of epoch e opens ring (e + 1) & 1 for epoch e + 1 by storing
// ((e + 1) << 32) | 0 (the stream orders that launch before every signal
// of epoch e + 1).  A slot holds (epoch << 32) | part, written with an
// atomic max, so a late writer never overwrites a newer epoch's entry, and
// a reader takes a slot as written only when it carries the reader's
// epoch.  A partition is appended at most once per epoch (dstamp), so a
// ring never holds more entries than partitions.
struct RingCounters {
  uint64_t reserve;               // (epoch << 32) | entries reserved
  uint32_t pad0[30];
};

// Error codes a kernel can leave in HostShared::status.
enum KernelStatus : uint32_t {
  kStatusOk = 0,
  kStatusTimeout = 1,  // its own deadline passed before all parts were ready
  kStatusAborted = 2,  // the host asked it to give up
};

// Kernel arguments (passed by value).
struct ReduceArgs {
  const BucketDesc* buckets;
  const PartDesc* parts;
  QEntry* queue;          // [nparts_total]
  uint32_t* done;         // [2][nparts_total] finished tiles per
                          // partition, one half per epoch parity
  uint32_t* queued;       // [nparts_total] epoch stamp once queued
  uint32_t* tile_hits;    // [nparts_total] debug: tiles reduced, or null
  uint64_t* dlist;        // [2][nparts_total] device ready rings, one per
                          // epoch parity: entry c of epoch e's ring is slot
                          // c, ((uint64)e << 32) | part once written
  EpochCounters* ctr;     // [2], one set per epoch parity
  RingCounters* ring;     // [2], one per epoch parity
  HostShared* host;       // device-visible address of the host struct
  const uint64_t* hlist;  // device-visible host ready list: entry i of an
                          // epoch is ((uint64)epoch << 32) | part, so a
                          // reader needs no count (stale entries carry an
                          // older epoch)
  uint32_t* arrived;      // device-visible arrived stamps
  uint32_t nparts_total;
  uint32_t total_groups;   // workgroups of the launch
  uint64_t total_rows;     // rows of all partitions
  uint32_t row_elems;      // elements per row (1024 bytes per rank)
  uint32_t min_tile_rows;  // bounds of the rows per tile chosen at queueing
  uint32_t max_tile_rows;
  uint32_t interleave;     // tile layout: 0 = consecutive rows, B > 0 =
                           // interleaved in bands of B tiles (RowSet)
  uint32_t* tile_counts;   // [nparts_total] debug: tiles chosen, or null
  uint32_t guide;          // guided-scheduling divisor f (0 = fixed tiles)
  uint32_t publish_batch;  // finished tiles a workgroup publishes together
  uint32_t epoch;          // stamp of this launch, or 0: read it from the
                           // host struct (a graph replays fixed arguments)
  uint64_t timeout_ticks; // device wall-clock ticks before giving up
  uint64_t* trace;        // debug: per workgroup 4 words (wall-clock at
                          // entry, when its first tile was queued, after
                          // its last tile; tiles reduced), or null
};

// Where a device-side ready signal appends: the rings of the request, and
// the epoch the signal was enqueued in (fixed at enqueue time, so a signal
// that runs late still names its own epoch).
struct RingArgs {
  uint64_t* dlist;        // [2][capacity]
  RingCounters* ring;     // [2]
  uint32_t* dstamp;       // [capacity] latest epoch each partition was
                          // appended in (atomic max: once per epoch)
  uint32_t capacity;      // partitions of the request
  uint32_t epoch;
};

struct PreadyArgs {
  const int32_t* parts;   // device array of partition ids
  uint32_t n;
  uint32_t reserved;
  RingArgs ring;
};

// Per-rank readiness on the device: rank `rank` marks its contribution to
// parts[0..n) in place.  rank_marks[p] = (epoch << 32) | mask of the ranks
// that marked p in that epoch (a word of an older epoch counts as empty; a
// mark never changes a word of a newer epoch); the mark that completes the
// mask appends p to the ready ring.
struct PreadyRankArgs {
  const int32_t* parts;
  uint32_t n;
  uint32_t rank;
  uint32_t full;          // mask of all ranks: (1 << nranks) - 1
  uint32_t reserved;
  uint64_t* rank_marks;   // [capacity]
  RingArgs ring;
};


}  // namespace pcoll
