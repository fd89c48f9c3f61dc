// Device side of the persistent partitioned reduction (gfx950, wave64).
//
// One launch serves one epoch of a request.  The epoch's counters were
// cleared by the previous launch (two counter sets alternate by epoch
// parity), so no wavefront ever has to find out that it is the last one,
// and no other launch precedes the reduce kernel.  Every wavefront is an independent
// worker; none ever waits for another, so the launch needs no co-residency
// and drains even if it is larger than the machine.  The worker is a
// workgroup of up to kMaxWavesPerGroup wavefronts that reduce the rows of one
// tile together (wavefront w of W takes every W-th row), so one claim
// and one release serve the whole group.  Wavefront 0 of the group drives
// the protocol; the group meets at a barrier before and after each tile.
// A worker loops:
//
//   1. take a global tile index t: its workgroup number the first time (no
//      atomic, so the launch does not start with a burst of atomics on one
//      address), then one atomic add per tile, issued before the current
//      tile is reduced so that its latency hides behind the tile;
//   2. wait until t is covered by the work queue.  While starved, the few
//      workers at the front of the claim order try to move newly readied
//      partitions into the queue: under a try-lock, read the host ready
//      list (host-coherent memory, written by pready) and this epoch's
//      device ready ring (written by the ready kernels), and append each
//      partition not yet queued this epoch together with the running total of its tiles.
//      Partitions are reduced in the order they became ready (the chunk
//      pipeline of Section 4.3: chunks proceed as soon as they can);
//   3. find the queue entry covering t (64 entries per wave-wide probe),
//      giving the partition and the tile inside it;
//   4. reduce the tile (rank order 0..P-1 per element), store the result;
//   5. publish: after a release fence, add the tile to its partition's done
//      counter (finished tiles are published in batches, see publish()); the
//      worker that completes the partition stores the epoch into its
//      arrived flag in host-coherent memory (completion is signalled only
//      after every chunk of the partition has landed, Section 4.5).  The
//      tiles a worker still holds when the work runs out complete with the
//      launch itself.
//
// Exit: t >= total tiles.  A worker that starves past the deadline, or sees
// the host's abort word, records the reason (also in host memory, stamped
// with the epoch) and leaves; the others follow.  The host's wait returns
// when every arrived flag carries the epoch, or the launch has retired with
// no error recorded, or an error is recorded.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.hpp"

namespace pcoll {
namespace dev {

// ---------------------------------------------------------------- atomics
__device__ __forceinline__ uint32_t ld_acq_sys(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint32_t ld_rlx_sys(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint64_t ld_rlx_sys64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint32_t ld_acq(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_rlx(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_acq64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_rlx64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rlx(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rlx64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel_sys(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Pointer into the constant address space: uniform loads through it become
// scalar loads.  Only for tables no kernel writes during the launch.
template <class T>
using const_ptr = __attribute__((address_space(4))) const T*;

// ---------------------------------------------------------- wave helpers
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint32_t uni(uint32_t v) {
  return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d);
    if (lane >= (uint32_t)d) x += y;
  }
  return x;
}

// ------------------------------------------------------------- the queue

// Appends the partitions held by the lanes with `valid` set, in lane order.
// Caller holds the ingest lock; qcount / qtiles / qrows are wave-uniform and
// updated in place.
//
// Tile count (guided self-scheduling, when `guide` f > 0): a partition
// whose first row has `rem` rows of the request from it to the end (itself
// included, partitions not yet queued counted too) is cut into tiles of
// about s = clamp(ceil(rem / (f G)), min_tile_rows, max_tile_rows) rows, G
// the workgroups of the launch: large tiles while much work remains, small
// ones near the end, so that workgroups run out of work at about the same
// time.  With f = 0 every tile has max_tile_rows rows.
//
// A partition is appended once per epoch, whatever the number of ready
// signals: queue_stamp() exchanges its queued stamp first and the append
// keeps it only if the stamp was not this epoch's already.  queue_stamp()
// issues nothing that waits, so the stamps of several chunks can be in
// flight together before their appends.
struct Stamped {
  uint32_t part;
  uint32_t rows;   // rows of the partition (when valid)
  bool valid;
};

__device__ __forceinline__ Stamped queue_stamp(const ReduceArgs& a,
                                               uint32_t epoch, bool valid,
                                               uint32_t part) {
  Stamped c{part, 0u, valid && part < a.nparts_total};
  uint32_t old = epoch;
  if (c.valid) {
    // the descriptor load does not wait for the stamp exchange
    c.rows = a.parts[part].rows;
    old = __hip_atomic_exchange(&a.queued[part], epoch, __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
  }
  c.valid = c.valid && old != epoch;
  return c;
}

__device__ __forceinline__ void queue_append(const ReduceArgs& a,
                                             const Stamped& c,
                                             uint32_t& qcount,
                                             uint32_t& qtiles,
                                             uint64_t& qrows) {
  const uint32_t lane = lane_id();
  const bool valid = c.valid;
  const uint32_t part = c.part;
  const uint32_t rows = valid ? c.rows : 0u;
  const uint32_t rincl = wave_incl_scan(rows);
  const uint64_t before = qrows + (rincl - rows);
  const uint64_t rem = a.total_rows > before ? a.total_rows - before : rows;
  uint64_t s = a.max_tile_rows;
  if (a.guide) {
    const uint64_t g = (uint64_t)a.guide * a.total_groups;
    s = (rem + g - 1) / g;
    if (s < a.min_tile_rows) s = a.min_tile_rows;
    if (s > a.max_tile_rows) s = a.max_tile_rows;
  }
  const uint32_t nt =
      valid ? (rows == 0u ? 1u : (uint32_t)((rows + s - 1) / s)) : 0u;
  const uint32_t incl = wave_incl_scan(nt);
  const uint64_t vm = __ballot(valid);
  const uint32_t rank = __popcll(vm & ((1ull << lane) - 1ull));
  const uint32_t slot = qcount + rank;
  if (valid && slot < a.nparts_total) {
    const uint64_t e = ((uint64_t)(qtiles + incl) << 32) | part;
    st_rlx64(reinterpret_cast<uint64_t*>(&a.queue[slot]), e);
    if (a.tile_counts) a.tile_counts[part] = nt;
  }
  qcount += (uint32_t)__popcll(vm);
  qtiles += uni(__shfl(incl, 63));
  qrows += uni(__shfl(rincl, 63));
}

// Entries reserved in this epoch's device ready ring (its word carries the
// epoch from the previous launch on; a word of another epoch counts as
// empty).
__device__ __forceinline__ uint32_t ring_reserved(const ReduceArgs& a,
                                                  uint32_t epoch) {
  const uint64_t w = uni64(ld_rlx64(&a.ring[epoch & 1u].reserve));
  return (uint32_t)(w >> 32) == epoch ? (uint32_t)w : 0u;
}

// Whether the ready lists may hold entries not yet queued: the host list's
// next entry carries this epoch, or the device ring has reserved entries
// beyond the consumed ones.  Relaxed reads, no lock: a stale answer only
// costs one lock attempt or one more probe.  A worker that has waited a
// while probes before it takes the lock, so an epoch that waits for its
// producers does not keep an atomic and a 2 KiB bus read in flight per
// probe; a short wait (the host's readiness calls right after the launch)
// goes straight to the lock and saves the probe's bus round trip.
__device__ __forceinline__ bool ready_lists_moved(const ReduceArgs& a,
                                                  uint32_t epoch) {
  EpochCounters* c = a.ctr;
  if (uni(ld_rlx(&c->ilock)) != 0u) return false;  // being ingested
  const uint32_t hcons = uni(ld_rlx(&c->hconsumed));
  uint64_t head = 0;
  if (hcons < a.nparts_total && lane_id() == 0)
    head = ld_rlx_sys64(&a.hlist[hcons]);
  if ((uint32_t)(uni64(head) >> 32) == epoch && hcons < a.nparts_total)
    return true;
  return ring_reserved(a, epoch) > uni(ld_rlx(&c->dconsumed));
}

// Moves newly readied partitions into the queue.  Returns true if it queued
// any tile.  Wave-wide.  The lock is taken before the host list is read, so
// at most one wavefront at a time reads host memory over the bus.
__device__ __forceinline__ bool try_ingest(const ReduceArgs& a, uint32_t epoch,
                                           bool probe) {
  const uint32_t lane = lane_id();
  EpochCounters* c = a.ctr;
  if (probe && !ready_lists_moved(a, epoch)) return false;
  uint32_t got = 0;
  if (lane == 0) {
    uint32_t expect = 0;
    got = __hip_atomic_compare_exchange_strong(
        &c->ilock, &expect, 1u, __ATOMIC_ACQUIRE, __ATOMIC_RELAXED,
        __HIP_MEMORY_SCOPE_AGENT);
  }
  if (!uni(got)) return false;

  uint64_t qs = uni64(ld_rlx64(&c->qstate));
  uint32_t qcount = (uint32_t)(qs >> 32), qtiles = (uint32_t)qs;
  // every partition queued: whatever the lists hold now belongs to the next
  // epoch (its readiness may be signalled while this launch drains)
  if (qcount >= a.nparts_total) {
    if (lane == 0) st_rel(&c->ilock, 0u);
    return false;
  }
  uint32_t hcons = uni(ld_rlx(&c->hconsumed));
  uint32_t dcons = uni(ld_rlx(&c->dconsumed));
  uint32_t dr = ring_reserved(a, epoch);
  uint64_t qrows = uni64(ld_rlx64(&c->queued_rows));
  const uint32_t qtiles0 = qtiles;

  // host ready list: entries hcons.. carrying this epoch's tag, read 256
  // per round trip over the bus; the queue state is published after every
  // 64 entries, so that workers start on them while the rest is read.  An
  // empty first read is repeated a few times while the lock is held (one
  // bus round trip per poll, instead of a lock, the counters and a read),
  // unless the device ring has entries
  for (uint32_t polls = 0; hcons < a.nparts_total; ++polls) {
    uint64_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t i = hcons + 64u * k + lane;
      v[k] = i < a.nparts_total ? ld_rlx_sys64(&a.hlist[i]) : 0ull;
    }
    // the list ends at the first entry of another epoch (not yet written):
    // lim[k] entries of chunk k, counted while the chunks before are whole
    uint32_t lim[4];
    uint32_t prefix = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bool ok = hcons + 64u * k + lane < a.nparts_total &&
                      (uint32_t)(v[k] >> 32) == epoch;
      const uint64_t bad = __ballot(!ok);
      lim[k] = bad ? (uint32_t)(__ffsll((long long)bad) - 1) : 64u;
      if (prefix != 64u * k) lim[k] = 0u;
      prefix += lim[k];
    }
    if (prefix == 0u) {
      if (qtiles != qtiles0 || polls >= 7u) break;
      dr = ring_reserved(a, epoch);
      if (dr > dcons) break;
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    // the entries were written with release stores after the host saw
    // their partitions' data in place: acquire before queueing them
    if (prefix) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
    // stamps and descriptors of every chunk in flight together
    Stamped st[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      st[k] = queue_stamp(a, epoch, lane < lim[k], (uint32_t)v[k]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (lim[k] == 0u) break;
      queue_append(a, st[k], qcount, qtiles, qrows);
      st_rel64(&c->qstate, ((uint64_t)qcount << 32) | qtiles);
    }
    hcons += prefix;
    if (prefix != 256u) break;
    polls = 8u;  // found entries: no more empty polls
  }

  // this epoch's device ready ring: entry c is slot c, stored as (epoch <<
  // 32) | part; stop at the first reserved entry whose writer has not
  // stored it yet (its slot still holds an older epoch's tag)
  const uint64_t* ring = a.dlist + (size_t)(epoch & 1u) * a.nparts_total;
  while (dcons < dr) {
    const uint32_t c = dcons + lane;
    const bool in = c < dr;
    uint64_t v = in ? ld_rlx64(&ring[c]) : 0ull;
    const bool ok = in && (uint32_t)(v >> 32) == epoch;
    const uint64_t pending = __ballot(in && !ok);
    const uint32_t lim =
        pending ? (uint32_t)(__ffsll((long long)pending) - 1) : 64u;
    // the producers of these partitions ended before their signals ran
    // (stream order), which made their stores visible device-wide;
    // acquire, so that no stale line of them is read from this XCD's caches
    if (__ballot(ok && lane < lim)) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE,
                                                            "agent");
    queue_append(a, queue_stamp(a, epoch, ok && lane < lim, (uint32_t)v),
                 qcount, qtiles, qrows);
    const uint32_t avail = dr - dcons < 64u ? dr - dcons : 64u;
    dcons += lim < avail ? lim : avail;
    if (pending) break;
  }

  st_rlx(&c->hconsumed, hcons);
  st_rlx(&c->dconsumed, dcons);
  st_rlx64(&c->queued_rows, qrows);
  st_rel64(&c->qstate, ((uint64_t)qcount << 32) | qtiles);
  if (lane == 0) st_rel(&c->ilock, 0u);
  return qtiles != qtiles0;
}

// Records the first error of the epoch; the recording wavefront also
// publishes it to the host, stamped with the epoch.
__device__ __forceinline__ void set_error(const ReduceArgs& a, uint32_t code,
                                          uint32_t epoch) {
  if (lane_id() == 0) {
    uint32_t expect = 0;
    if (__hip_atomic_compare_exchange_strong(&a.ctr->error, &expect, code,
                                             __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT)) {
      __hip_atomic_store(&a.host->status, code, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_SYSTEM);
      st_rel_sys(&a.host->status_epoch, epoch);
    }
  }
}

enum WaitResult { kBail, kStop, kReady };

// Waits until tile t is queued (kReady, with the queue state in qs_out).
// Before it first has to wait it calls publish_pending().
// kStop: every partition is queued and t is beyond the last tile.  kBail:
// give up (deadline, host abort, or another worker's error).  The few
// workers at the front of the claim order (t within 8 tiles of the queued
// total) poll the ready lists and the host's abort word; the rest re-read
// the device-side queue state at a slower pace, and after a long wait they
// also poll the lists now and then (see below).
template <class Publish>
__device__ __forceinline__ WaitResult wait_queued(const ReduceArgs& a,
                                                  uint32_t t, uint32_t epoch,
                                                  uint64_t t0,
                                                  uint64_t& qs_out,
                                                  Publish&& publish_pending) {
  // the queue state this worker acquired last: entries it covers are
  // already visible, so a tile inside it needs no new acquire
  if ((uint32_t)qs_out > t) return kReady;
  for (uint32_t spins = 0;; ++spins) {
    // polled relaxed; acquired (one fence) only once it covers t: an
    // acquire invalidates caches, which a waiting kernel should not keep
    // doing to the kernels that run beside it
    const uint64_t qs = uni64(ld_rlx64(&a.ctr->qstate));
    const uint32_t qt = (uint32_t)qs;
    if (qt > t) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      qs_out = qs;
      return kReady;
    }
    if ((uint32_t)(qs >> 32) >= a.nparts_total) return kStop;
    // about to wait: finished tiles must not sit behind the wait
    publish_pending();
    // The workers near the queue's end ingest.  So does, every 128th
    // poll, any worker that has waited 64 polls: a launch can have more
    // workgroups than fit on the device at once, and the tiles at the
    // queue's end may belong to workgroups that start only when resident
    // ones leave, so ingesting must not depend on them.  Those far from the
    // end read host memory (the ready list, the abort word) that rarely:
    // a read of host memory crosses the bus, and a few hundred waiting
    // workers that read it every few polls load the bus enough to slow
    // the dispatch of kernels on other streams (the producers an epoch
    // waits for).
    const bool near = t - qt < 8u;
    const bool stuck = spins >= 64u;
    const bool front = near || (stuck && (spins & 127u) == 0u);
    if (front && try_ingest(a, epoch, spins >= 16u)) continue;
    if (uni(ld_rlx(&a.ctr->error)) != 0u) return kBail;
    if ((spins & 7u) == 7u) {
      const bool poll_abort = near || (stuck && (spins & 255u) == 255u);
      if (poll_abort && uni(ld_rlx_sys(&a.host->abort)) == epoch) {
        set_error(a, kStatusAborted, epoch);
        return kBail;
      }
      if (wall_clock64() - t0 > a.timeout_ticks) {
        set_error(a, kStatusTimeout, epoch);
        return kBail;
      }
    }
    if (near)
      __builtin_amdgcn_s_sleep(2);
    else
      __builtin_amdgcn_s_sleep(8);
  }
}

// Finds the queue entry covering tile t among entries [cursor, qcount).
// cursor / prev_end (cum_end of entry cursor-1) only move forward, since a
// worker's claims increase; part / end hold the entry found last, so a
// tile in the same partition as the previous one needs no queue read.
__device__ __forceinline__ void locate(const ReduceArgs& a, uint32_t t,
                                       uint32_t qcount, uint32_t& cursor,
                                       uint32_t& prev_end, uint32_t& part,
                                       uint32_t& end) {
  const uint32_t lane = lane_id();
  if (t < end) return;  // t >= prev_end: claims increase
  for (;;) {
    uint32_t i = cursor + lane;
    uint64_t e = i < qcount
                     ? ld_rlx64(reinterpret_cast<const uint64_t*>(&a.queue[i]))
                     : ~0ull;
    uint32_t ce = (uint32_t)(e >> 32);
    uint64_t m = __ballot(ce > t);
    if (m) {
      uint32_t k = (uint32_t)(__ffsll((long long)m) - 1);
      uint32_t before = uni(__shfl(ce, k == 0 ? 0 : k - 1));
      if (k != 0) prev_end = before;
      cursor += k;
      part = uni(__shfl((uint32_t)e, k));
      end = uni(__shfl(ce, k));
      return;
    }
    prev_end = uni(__shfl(ce, 63));
    cursor += 64;
  }
}

// Completion of finished tiles.  Publishing a tile means: its stores are
// visible device-wide, then the partition's done counter counts it; the
// worker whose count completes the partition acquires the other workers'
// tiles and stores the epoch into the host-visible arrived flag.  Making
// stores visible device-wide takes an agent-scope release fence, which
// writes back this XCD's L2 and holds it for a fraction of a microsecond,
// serialized with every other release on the XCD; so a workgroup keeps up
// to `publish_batch` finished tiles pending and publishes them together:
// one release fence (it covers every store of the group: each wavefront
// waited for its own stores before the group's barrier), then one relaxed
// add per tile, issued by one lane each (fence followed by the atomic: the
// standard fence-to-atomic synchronization).  A group publishes when the
// batch is full and before it waits for work, so a partition is late by at
// most one batch of one group, and only while the kernel has a backlog of
// readied work.
//
// When a group runs out of tiles for good it publishes nothing: a launch
// that retires without an error has reduced every tile (a worker leaves
// without error only once every tile index below the total was claimed, and
// every claimed tile is reduced), and the kernel's end makes all its stores
// visible, so the host counts every partition as arrived once the launch
// has retired cleanly.  That saves the burst of releases at the end, which
// would serialize on each XCD.  The done counters these tiles leave
// partial are cleared by the next launch, for the one after it.
struct Pending {
  uint32_t part;
  uint32_t nt;
};

__device__ __forceinline__ void publish(const ReduceArgs& a,
                                        const Pending* pend, uint32_t& npend,
                                        uint32_t epoch) {
  if (npend == 0) return;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  // lane i publishes pending tile i: one wave-wide atomic instruction
  const uint32_t l = lane_id();
  uint32_t part = 0;
  bool last = false;
  if (l < npend) {
    part = pend[l].part;
    if (a.tile_hits)
      __hip_atomic_fetch_add(&a.tile_hits[part], 1u, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t old = __hip_atomic_fetch_add(
        &a.done[part], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    last = old + 1u == pend[l].nt;  // exactly one add completes a partition
  }
  if (__builtin_amdgcn_ballot_w64(last) != 0) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __threadfence_system();
    if (last) st_rel_sys(&a.arrived[part], epoch);
  }
  npend = 0;
}

// The group has no tiles left: its pending tiles complete with the launch.
// Only the debug tile counts see them.
__device__ __forceinline__ void retire(const ReduceArgs& a,
                                       const Pending* pend, uint32_t& npend) {
  const uint32_t l = lane_id();
  if (a.tile_hits && l < npend)
    __hip_atomic_fetch_add(&a.tile_hits[pend[l].part], 1u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  npend = 0;
}

// The tile index after the first round: one relaxed atomic add by lane 0.
__device__ __forceinline__ uint32_t claim(const ReduceArgs& a) {
  uint32_t t = 0;
  if (lane_id() == 0)
    t = __hip_atomic_fetch_add(&a.ctr->claim, 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT) +
        a.total_groups;
  return t;  // valid in lane 0; broadcast by the caller when needed
}

// What wavefront 0 hands the group for one tile.
struct TileJob {
  uint32_t part;  // global partition, or ~0u to stop
  uint32_t lt;    // tile index within the partition
  uint32_t nt;    // tiles of the partition
};

// The epoch after e (the host's rule: epoch 0 is never used, so after
// 2^32 - 1 the count goes on at 2, which keeps the parity alternating).
__device__ __forceinline__ uint32_t next_epoch(uint32_t e) {
  return e + 1u == 0u ? 2u : e + 1u;
}

// Clears the counter set and done counters of the other epoch parity, for
// the next launch, and opens the other parity's device ready ring for the
// next epoch: the previous launch, which used them, has retired (the
// stream orders launches), and the next one starts only after this one.
// Every workgroup clears its share of the done counters; workgroup 0 the
// counter set and the ring's reservation word.  A device-side signal of an
// ended epoch that still tries to reserve in that ring then finds another
// epoch in the word and appends nothing.
__device__ __forceinline__ void clear_next_epoch(const ReduceArgs& args,
                                                 uint32_t epoch) {
  const uint32_t other = (epoch & 1u) ^ 1u;
  uint32_t* done = args.done + (size_t)other * args.nparts_total;
  for (uint32_t p = blockIdx.x * 64u + lane_id(); p < args.nparts_total;
       p += args.total_groups * 64u)
    st_rlx(&done[p], 0u);
  if (blockIdx.x == 0 && lane_id() == 0) {
    EpochCounters* c = args.ctr + other;
    st_rlx(&c->claim, 0u);
    st_rlx64(&c->qstate, 0ull);
    st_rlx(&c->ilock, 0u);
    st_rlx(&c->hconsumed, 0u);
    st_rlx64(&c->queued_rows, 0ull);
    st_rlx(&c->dconsumed, 0u);
    st_rlx(&c->error, 0u);
    st_rlx64(&args.ring[other].reserve, (uint64_t)next_epoch(epoch) << 32);
  }
}

// The worker loop of one workgroup.  Tile::run<P>(bucket, partition offset,
// partition length, tile index, tiles of the partition, interleave,
// wavefront, wavefronts) reduces this wavefront's rows of a tile.
template <class Tile, int P>
__device__ __forceinline__ void persistent_loop(const ReduceArgs& args) {
  __shared__ TileJob job;
  __shared__ Pending pend[kMaxPublishBatch];
  const uint32_t wave = threadIdx.x / 64u;
  const uint32_t nwaves = blockDim.x / 64u;
  // only wavefront 0 runs the protocol and needs the epoch.  A graph
  // replay reads it from host memory: the launch has no more workgroups
  // than tiles, every workgroup's first tile is its own number, so the
  // epoch cannot complete (and the host cannot store the next stamp)
  // before every workgroup has read this one
  uint32_t epoch = 0;
  if (wave == 0)
    epoch = args.epoch ? args.epoch : uni(ld_acq_sys(&args.host->epoch));
  ReduceArgs a = args;
  a.ctr = args.ctr + (epoch & 1u);
  a.done = args.done + (size_t)(epoch & 1u) * args.nparts_total;
  if (wave == 0) clear_next_epoch(args, epoch);
  const uint64_t t0 = wall_clock64();
  uint32_t cursor = 0, prev_end = 0;
  uint32_t cur_part = 0, cur_end = 0;  // queue entry at cursor
  uint32_t t = blockIdx.x;  // first round: tile = workgroup number
  uint32_t next = 0;
  uint64_t qs = 0;          // queue state last acquired (wavefront 0)
  uint32_t npend = 0;       // finished tiles not yet published (wavefront 0)
  uint32_t ntiles = 0;      // tiles reduced (wavefront 0, for the trace)
  uint64_t t_first = 0;     // when the first tile was queued (trace)
  for (;;) {
    if (wave == 0) {
      TileJob j{~0u, 0u, 0u};
      const WaitResult w = wait_queued(a, t, epoch, t0, qs, [&] {
        publish(a, pend, npend, epoch);
      });
      if (a.trace && ntiles == 0 && w == kReady) t_first = wall_clock64();
      if (a.trace && w != kReady && lane_id() == 0) {
        uint64_t* s = a.trace + (size_t)blockIdx.x * 4u;
        s[0] = t0;
        s[1] = t_first;
        s[2] = wall_clock64();
        s[3] = ntiles;
      }
      if (w == kReady) {
        locate(a, t, (uint32_t)(qs >> 32), cursor, prev_end, cur_part,
               cur_end);
        j.part = cur_part;
        j.lt = t - prev_end;
        j.nt = cur_end - prev_end;
        next = claim(a);  // in flight while the tile is reduced
      } else if (w == kStop) {
        retire(a, pend, npend);
      }
      if (lane_id() == 0) job = j;
    }
    __syncthreads();
    const TileJob j = job;
    if (j.part == ~0u) break;
    // descriptor tables are read-only for the whole launch: scalar loads
    const const_ptr<PartDesc> pd = (const_ptr<PartDesc>)(a.parts) + j.part;
    const uint64_t poff = pd->off, plen = pd->len;
    const const_ptr<BucketDesc> bd =
        (const_ptr<BucketDesc>)(a.buckets) + pd->bucket;
    Tile::template run<P>(bd, poff, plen, j.lt, j.nt, a.interleave, wave,
                          nwaves);
    // every wavefront's stores have completed before the group's release
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (wave == 0) {
      if (lane_id() == 0) pend[npend] = Pending{j.part, j.nt};
      ++npend;
      ++ntiles;
      if (npend >= a.publish_batch) publish(a, pend, npend, epoch);
      t = uni(next);
    }
  }
}

// ------------------------------------------------------ memory streaming
// 16-byte streaming access through the global address space (global_load /
// global_store with the nontemporal hint, never the generic flat path).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4* gload_ptr;
typedef __attribute__((address_space(1))) u32x4* gstore_ptr;
__device__ __forceinline__ uint4 ld_stream(const uint4* p) {
  const u32x4 v = __builtin_nontemporal_load((gload_ptr)(p));
  return make_uint4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void st_stream(uint4* p, uint4 v) {
  const u32x4 w = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(w, (gstore_ptr)(p));
}

// Knuth's TwoSum: s = fl(a + b), e = a + b - s exactly.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  float bv = s - a;
  float av = s - bv;
  e = (a - av) + (b - bv);
}

}  // namespace dev
}  // namespace pcoll
