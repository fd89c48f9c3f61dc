// The allocation-free epoch (noalloc.hip): its scratch array's layout, and
// the set-up launch that writes the state an epoch starts from.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "layout.hpp"

namespace pcoll {

// Size of the per-device scratch array, and the most partitions it holds
// (80 bytes per partition plus about 2 KiB of fixed state).
constexpr size_t kNoallocScratchBytes = 512u * 1024u;
constexpr uint32_t kNoallocMaxParts = 4096u;

// Byte offsets into the scratch array (256-byte aligned arrays).  host,
// hlist and arrived follow each other, as in the host-coherent block of a
// request; the two ring words follow the two counter sets.
struct NoallocLayout {
  uint64_t parts, queue, done, queued, dlist, ctr, ring, bucket, host, hlist,
      arrived, total;
};

inline NoallocLayout noalloc_layout(uint32_t np) {
  NoallocLayout L{};
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off = (off + bytes + 255u) / 256u * 256u;
    return o;
  };
  L.parts = take(sizeof(PartDesc) * np);
  L.queue = take(sizeof(QEntry) * np);
  L.done = take(sizeof(uint32_t) * 2 * np);
  L.queued = take(sizeof(uint32_t) * np);
  L.dlist = take(sizeof(uint64_t) * 2 * np);
  L.ctr = take(2 * sizeof(EpochCounters) + 2 * sizeof(RingCounters));
  L.ring = L.ctr + 2 * sizeof(EpochCounters);
  L.bucket = take(sizeof(BucketDesc));
  L.host = take(sizeof(HostShared) + sizeof(uint64_t) * np +
                sizeof(uint32_t) * np);
  L.hlist = L.host + sizeof(HostShared);
  L.arrived = L.hlist + sizeof(uint64_t) * np;
  L.total = off;
  return L;
}

struct NoallocSetup {
  unsigned char* base;  // the scratch array on this device
  NoallocLayout layout;
  BucketDesc bucket;
  uint64_t count;       // elements of the message
  uint64_t psize;       // partition length (the chunk rule)
  uint32_t nparts;
  uint32_t row_elems;   // elements per row of 64 lanes x 16 bytes
  uint32_t epoch;
};

// The scratch array's device address on `device` (the current device),
// looked up once per device and kept.
hipError_t noalloc_scratch(int device, void** ptr);
hipError_t launch_noalloc_setup(const NoallocSetup& s, hipStream_t stream);

}  // namespace pcoll
