// The allocation-free form of one epoch: every buffer the reduce kernel
// uses beyond its inputs and outputs (partition table, bucket descriptor,
// work queue, counters, done counters, queued stamps, ready list) lives in
// a file-scope device array of fixed size, so a call needs no hipMalloc
// and no pinned host memory (for callers under graph capture or in loops
// that must not allocate).  Each device holds its own copy of the array
// until the process ends; calls on one device share it, so calls that
// overlap on one device race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "noalloc.hpp"

namespace pcoll {

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices];  // the array's device address, per device

}  // namespace

hipError_t noalloc_scratch(int device, void** ptr) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    // the symbol's address on the current device (each device has its own
    // copy); in host code the array's name is no device address
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[device] = p;
  }
  *ptr = g_ptr[device];
  return hipSuccess;
}

// Writes the state one epoch starts from into the scratch array: the
// bucket descriptor, the partition table (the chunk rule: offsets k * psize,
// lengths clipped to the message), cleared counters of both epoch parities,
// cleared done counters and queued stamps, and a ready list that holds
// every partition tagged with the epoch (all partitions ready at launch).
// The device ready rings stay empty (reservation words 0).
__global__ __launch_bounds__(256) void noalloc_setup_kernel(NoallocSetup s) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  const NoallocLayout& L = s.layout;
  unsigned char* base = s.base;
  if (i == 0) {
    *reinterpret_cast<BucketDesc*>(base + L.bucket) = s.bucket;
    HostShared* h = reinterpret_cast<HostShared*>(base + L.host);
    h->epoch = s.epoch;
    h->abort = 0;
    h->status = 0;
    h->status_epoch = 0;
  }
  // counter sets and ring words, 4-byte words
  const uint32_t nctr =
      (uint32_t)((2 * sizeof(EpochCounters) + 2 * sizeof(RingCounters)) / 4);
  if (i < nctr) reinterpret_cast<uint32_t*>(base + L.ctr)[i] = 0u;
  if (i < s.nparts) {
    PartDesc p{};
    const uint64_t off = (uint64_t)i * s.psize < s.count
                             ? (uint64_t)i * s.psize
                             : s.count;
    p.off = off;
    p.len = s.count - off < s.psize ? s.count - off : s.psize;
    p.bucket = 0;
    p.rows = (uint32_t)((p.len + s.row_elems - 1) / s.row_elems);
    reinterpret_cast<PartDesc*>(base + L.parts)[i] = p;
    uint32_t* done = reinterpret_cast<uint32_t*>(base + L.done);
    done[i] = 0u;
    done[s.nparts + i] = 0u;
    reinterpret_cast<uint32_t*>(base + L.queued)[i] = 0u;
    reinterpret_cast<uint64_t*>(base + L.hlist)[i] =
        ((uint64_t)s.epoch << 32) | i;
    reinterpret_cast<uint32_t*>(base + L.arrived)[i] = 0u;
  }
}

hipError_t launch_noalloc_setup(const NoallocSetup& s, hipStream_t stream) {
  const uint32_t nctr =
      (uint32_t)((2 * sizeof(EpochCounters) + 2 * sizeof(RingCounters)) / 4);
  const uint32_t n = s.nparts > nctr ? s.nparts : nctr;
  hipLaunchKernelGGL(noalloc_setup_kernel, dim3((n + 255u) / 256u), dim3(256),
                     0, stream, s);
  return hipGetLastError();
}

}  // namespace pcoll
