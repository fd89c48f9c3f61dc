/*
 * pcoll -- partitioned reduction of P rank contributions on one MI355X
 * (gfx950).  C ABI of libpcoll.so.
 *
 * The operation.  A request reduces one message (or, batched, many
 * messages called buckets) of `count` elements held by P ranks:
 *   out[i] = in_0[i] (op) in_1[i] (op) ... (op) in_{P-1}[i],
 * op = sum or max, each element in rank order 0..P-1.  The P rank buffers
 * live in this GPU's memory (they stand for the contributions of P peer
 * ranks).  The paper this library follows (Sojoodi et al., "Accelerating
 * Intra-Node GPU-to-GPU Communication Through Multi-Path Transfers with CUDA
 * Graphs") builds point-to-point multi-path copies and names Allreduce as
 * future work (Section 6); the reduction arithmetic is the plain definition
 * of elementwise sum / max.
 *
 * Partitions.  Each message is cut into `nparts` partitions by the chunk
 * rule of Algorithm 1 (Section 4.3): every partition has the same length
 * psize = ceil(count / nparts) rounded up to whole 128-byte cache lines
 * (and whole scale blocks for the 8-bit floats: 256 elements, 128 for MX
 * blocks of 32; with A = 1 the rule is Algorithm 1's exactly),
 * offsets are fixed in advance as running sums, and the last partitions
 * are clipped (possibly to zero length).  Destination regions are disjoint (Section 4.5, Ordering
 * Guarantee): each partition of the output is written exactly once per
 * epoch, whatever order partitions are readied in.
 *
 * Life cycle (persistent request, one epoch per start):
 *   init -> bind -> { start -> pready(p)... -> parrived / test / wait }* -> free
 * `start` launches one persistent kernel (or replays its cached graph) on
 * the bound stream and returns at once.  `pready(p)` declares that every
 * rank's contribution to partition p is in place; the kernel reduces
 * partitions in the order they become ready.  `parrived(p)` tells whether
 * partition p of the output is final.  `wait` returns once every partition
 * has arrived (completion is signalled only after every chunk has landed,
 * Section 4.5, Final Synchronization).
 *
 * Memory and ownership.  The caller owns every data buffer (device memory,
 * e.g. torch tensors); the library keeps raw pointers only.  Rank buffers of
 * partition p must stay unchanged from pready(p) until p has arrived; the
 * output region of p must not be touched by others before that.  All device
 * pointers must be 16-byte aligned; buffers aligned to 128 bytes (as
 * torch's allocations are) stream without cache lines shared between
 * tiles.  The library owns its flags, counters,
 * descriptor tables, graphs and events.
 *
 * Errors.  Every call returns PCOLL_SUCCESS (0) or a negative code; on
 * error the request state is unchanged.  No C++ exception crosses this ABI.
 * Calls on one request must come from one host thread at a time; separate
 * requests may be used from separate threads and streams.
 *
 * Streams are hipStream_t values passed as void* (NULL = the null stream).
 */
#ifndef PCOLL_H
#define PCOLL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pcoll_req_s *pcoll_req_t; /* opaque, library-owned */

typedef enum {
  PCOLL_INT32 = 0,     /* two's-complement wrap sum, max: bit-exact */
  PCOLL_FLOAT32 = 1,   /* binary32 in and out, binary32 accumulation */
  PCOLL_BFLOAT16 = 2,  /* bf16 in and out, binary32 accumulation, RNE out */
  PCOLL_FP8_E4M3 = 3,  /* OCP e4m3 codes + one binary32 scale per 256
                          elements (value = code * scale), binary32
                          accumulation, output re-quantized per 256 */
  PCOLL_FP8_E5M2 = 4,  /* OCP e5m2 codes (2 fraction bits, range 57344),
                          otherwise as PCOLL_FP8_E4M3 */
  PCOLL_MXFP8_E4M3 = 5, /* OCP MX blocks (Microscaling Formats v1.0, MXFP8
                          with e4m3 elements): e4m3 codes, one E8M0 scale
                          byte b per 32 elements (value = code * 2^(b-127),
                          exact in binary32); binary32 accumulation; output
                          re-quantized per 32 with the smallest power-of-two
                          scale (>= 2^-127) under which no code exceeds 448.
                          Scale byte 0xFF (NaN) is not accepted as input:
                          such blocks give unspecified results. */
  PCOLL_BF16_PAIR = 6  /* bf16 in; out: a pair of bf16 arrays, hi = bf16(y)
                          and lo = bf16(y - hi) for the binary32 sum y (Sum2
                          by default), so hi + lo carries y to 16
                          significant bits (compensated bf16 output).  The
                          lo arrays are passed as pcoll_bind's out_scales.
                          Sum only. */
} pcoll_dtype_t;

typedef enum { PCOLL_SUM = 0, PCOLL_MAX = 1 } pcoll_op_t;

enum {
  PCOLL_SUCCESS = 0,
  PCOLL_ERR_ARG = -1,         /* bad argument: null, range, alignment */
  PCOLL_ERR_STATE = -2,       /* call not valid in the request's state */
  PCOLL_ERR_UNSUPPORTED = -3, /* dtype/op/rank-count combination */
  PCOLL_ERR_HIP = -4,         /* a HIP runtime call failed */
  PCOLL_ERR_TIMEOUT = -5,     /* not every partition arrived in time */
  PCOLL_ERR_NOMEM = -6,       /* host or device allocation failed */
  PCOLL_ERR_ABORTED = -7      /* the kernel gave up on its own deadline */
};

#define PCOLL_MAX_RANKS 16
#define PCOLL_VERSION 1

/* ---------------------------------------------------------------- setup */

/* Creates a persistent request for one message of `count` elements
 * (count >= 0) of `dtype`, reduced with `op` over `nranks` ranks
 * (1..PCOLL_MAX_RANKS), split into `nparts` >= 1 partitions by the chunk
 * rule of Algorithm 1 (Section 4.3: equal ceil-length chunks at offsets
 * fixed in advance, the last one clipped; see "Partitions" above).  The
 * persistent-request life cycle (init once, then start / ready / wait per
 * epoch) is the MPI-4 partitioned communication model, not the paper's,
 * which issues one transfer per call.  Allocates the request's flags
 * (host-coherent pinned memory) and counters (device memory) on the
 * current HIP device; the request owns them until pcoll_free.
 * PCOLL_ERR_ARG for a null `out`, an unknown dtype or op, nparts < 1 or
 * nranks < 1; PCOLL_ERR_UNSUPPORTED for nranks > PCOLL_MAX_RANKS, max on
 * the 8-bit dtypes and bf16 pairs, more than 2^24 partitions in all, or a
 * partition longer than 2^31 elements; PCOLL_ERR_NOMEM if an allocation
 * fails.  *out is NULL on error. */
int pcoll_init(size_t count, pcoll_dtype_t dtype, pcoll_op_t op, int nparts,
               int nranks, pcoll_req_t *out);

/* Batched form: `nbuckets` >= 1 messages of counts[b] elements (host
 * array, read during the call), each split into `nparts_per_bucket`
 * partitions; partition k of bucket b has the global index
 * b * nparts_per_bucket + k.  One start launches one persistent kernel for
 * all buckets (the paper records a whole multi-chunk transfer as one graph,
 * Algorithm 1; here one kernel covers every chunk of every bucket).  Many
 * uneven gradient buckets in one request are this library's extension, not
 * the paper's.  Errors as pcoll_init, and PCOLL_ERR_ARG for nbuckets < 1 or
 * a null `counts`. */
int pcoll_init_batch(int nbuckets, const size_t *counts, pcoll_dtype_t dtype,
                     pcoll_op_t op, int nparts_per_bucket, int nranks,
                     pcoll_req_t *out);

/* Binds data buffers and the stream kernels are enqueued on (host arrays
 * of device pointers, read during the call; the library keeps the
 * pointers, the caller keeps ownership of the buffers).
 *   rank_bufs  nbuckets * nranks device pointers, bucket-major:
 *              rank_bufs[b * nranks + r] = contribution of rank r to b.
 *   outs       nbuckets device pointers (may equal a rank buffer only if
 *              the caller accepts that rank's input being overwritten
 *              partition by partition).
 *   rank_scales / out_scales: 8-bit dtypes only (else NULL), laid out
 *              like rank_bufs / outs: for PCOLL_FP8_E4M3 / _E5M2 binary32
 *              scales (4-byte aligned), ceil(count / 256) per bucket; for
 *              PCOLL_MXFP8_E4M3 E8M0 bytes (any alignment), ceil(count /
 *              32) per bucket.  For PCOLL_BF16_PAIR rank_scales is NULL
 *              and out_scales holds the nbuckets lo arrays (bf16, count
 *              elements each, 16-byte aligned).
 * Not allowed while an epoch is active (PCOLL_ERR_STATE).  PCOLL_ERR_ARG
 * for null arrays, null pointers of non-empty buckets, misaligned
 * pointers, or second-output / scale arrays given for a dtype that has
 * none (or missing for one that needs them).
 * A binding seen before (same pointers and stream) reuses its cached
 * descriptor table and graph: the cache of Section 4.2 (Framework
 * Architecture), which keeps instantiated graphs in a fixed-size hash table
 * keyed by the transfer's addresses and evicts the least recently used.
 * Each request keeps the PCOLL_GRAPH_CACHE (environment, default 8) most
 * recently used bindings and frees the least recently used beyond that
 * (after the last kernel that used it has retired). */
int pcoll_bind(pcoll_req_t req, const void *const *rank_bufs,
               void *const *outs, const void *const *rank_scales,
               void *const *out_scales, void *stream);

/* --------------------------------------------------------------- epochs */

/* Starts an epoch: asynchronously launches the persistent reduce kernel on
 * the bound stream (or, in graph mode, replays the cached graph; the graph
 * is captured and instantiated lazily on first use and launched from the
 * cache afterwards, as Algorithm 1's LaunchGraph does, Section 4.3).
 * PCOLL_ERR_STATE if unbound or an epoch is still active.  Epochs are the
 * MPI-4 persistent-request model (MPI_Start), not the paper's. 
 *
 * The kernel occupies its stream until every partition is ready.  Work on
 * a stream that HIP placed on the same hardware queue runs after it (HIP
 * spreads a process's streams over GPU_MAX_HW_QUEUES queues, 4 by
 * default): do not make the readiness of an epoch wait for such work, for
 * example for another request's epoch whose stream shares the queue, or
 * for producers on such a stream; the epoch would end at its deadline with
 * PCOLL_ERR_ABORTED.  HIP does not say which streams share a queue; the
 * Python helper paper_2604_22228_amd.streams.independent_streams finds
 * streams that run beside a given one. */
int pcoll_start(pcoll_req_t req);

/* Marks partition `part` ready (host side, non-blocking, about a store to
 * pinned memory): MPI_Pready of the MPI-4 partitioned model, which the
 * paper does not have; its nearest notion is the per-chunk synchronization
 * point after which a chunk may proceed (Section 4.5).  PCOLL_ERR_STATE if
 * no epoch is active or the partition was already readied this epoch;
 * PCOLL_ERR_ARG if out of range. */
int pcoll_pready(pcoll_req_t req, int part);

/* Marks partitions first..last (inclusive) ready; all-or-nothing
 * (MPI_Pready_range).  Errors as pcoll_pready; PCOLL_ERR_ARG if
 * last < first. */
int pcoll_pready_range(pcoll_req_t req, int first, int last);

/* Marks parts[0..n) (host array) ready; all-or-nothing, duplicates are
 * PCOLL_ERR_ARG (MPI_Pready_list).  The partitions of one call become
 * ready at the same instant, so the library queues them in partition order
 * (neighbouring partitions of a bucket are then reduced together),
 * whatever their order in `parts`. */
int pcoll_pready_list(pcoll_req_t req, int n, const int *parts);

/* Device-side ready signal: enqueues on `stream` a kernel that marks the
 * partitions in the device array parts_dev[0..n) ready when it runs, so
 * readiness can follow producer kernels in stream order (or be captured in
 * a graph).  Not in the paper (whose chunks are readied by events between
 * graph nodes, Section 4.5); the device form of MPI_Pready.  The array must
 * stay valid until the signal has run.  `stream` must not be the bound
 * stream (PCOLL_ERR_ARG: the reduce kernel occupies it until every
 * partition is ready); PCOLL_ERR_STATE if no epoch is active.  Ids out of
 * range are ignored, and a partition signalled more than once in an epoch
 * counts once.  The signal belongs to the epoch that was active when it
 * was enqueued: if that epoch has ended by the time it runs (for example
 * through pcoll_wait_timeout while it waited behind its producer), it
 * readies nothing.  The request's launches leave room for producers from
 * the next start on (config field `producers`).
 *
 * The signal must be able to run while the reduce kernel runs, so its
 * stream must not share the bound stream's hardware queue: HIP spreads a
 * process's streams over GPU_MAX_HW_QUEUES hardware queues per device (4
 * by default), and work queued behind the reduce kernel in its hardware
 * queue waits for it.  Keep the streams that signal during an epoch fewer
 * than that limit.  A signal that cannot run leaves its partitions
 * unready: the kernel reaches its deadline and the epoch fails with
 * PCOLL_ERR_ABORTED; it does not hang.
 *
 * Likewise the kernels that produce the data and precede the signal on
 * its stream must find room on the compute units beside the resident
 * reduce kernel, whose workgroups stay until the epoch ends.  A producer
 * wave that needs more registers or LDS than a unit has left cannot start,
 * so readiness never comes.  The producer mode (config field `producers`)
 * keeps one resident wave per SIMD with about 115 instead of 160-190 VGPRs
 * per wave at 8 ranks, which leaves matrix-core (MFMA) producers room; in
 * the default automatic mode a request enters it from the start after its
 * first device-side signal, so set `producers` = 1 before the first epoch
 * whose readiness follows heavy producers. */
int pcoll_pready_on_stream(pcoll_req_t req, const int *parts_dev, int n,
                           void *stream);

/* Per-rank readiness (the receive side of a partitioned allreduce; the
 * MPI-4 partitioned model, not in the paper): rank `rank` (0..nranks-1)
 * has placed its contribution to partition `part`.
 * The partition becomes ready, exactly as by pcoll_pready, once every rank
 * has readied it this epoch; until then the kernel does not touch it.
 * Host-side bookkeeping only (no GPU call unless this completes the
 * partition).  PCOLL_ERR_STATE if no epoch is active, if this rank already
 * readied the partition this epoch, or if the partition is already ready;
 * PCOLL_ERR_ARG if rank or part is out of range. */
int pcoll_pready_rank(pcoll_req_t req, int rank, int part);

/* Device-side per-rank readiness (not in the paper): enqueues on `stream`
 * a kernel that marks rank `rank`'s contributions to the partitions
 * parts_dev[0..n) (device array, valid until the kernel has run) in place
 * when it runs, so each rank's marks can follow its producer kernels in
 * that rank's stream order.  A partition is queued when the marks of all
 * ranks for the epoch that was active at enqueue time are in; repeated
 * marks of one rank are idempotent, ids out of range are ignored, and a
 * mark that runs after its epoch ended changes nothing (not even a later
 * epoch's marks).  All ranks of one partition must mark it on the device
 * (pcoll_pready_rank counts on the host, apart).  `stream` must not be the
 * bound stream (PCOLL_ERR_ARG), nor share its hardware queue (see
 * pcoll_pready_on_stream); PCOLL_ERR_ARG for a rank out of range,
 * PCOLL_ERR_STATE if no epoch is active. */
int pcoll_pready_rank_on_stream(pcoll_req_t req, int rank,
                                const int *parts_dev, int n, void *stream);

/* Non-blocking test of one partition (MPI_Parrived): *flag = 1 once its
 * output is final in the current (or last completed) epoch.  PCOLL_ERR_STATE before the first
 * start.  Arrival (Section 4.5: a partition counts only after all of its
 * chunks have landed) is signalled either by the partition's own flag,
 * which the kernel sets as soon as it has published the partition's last
 * tile, or by the retirement of the epoch's kernel with no error, which
 * implies every partition: the kernel leaves the tiles that a workgroup
 * still holds when the work runs out to its own end instead of publishing
 * them (config field publish_batch).  The second case costs one
 * hipEventQuery. */
int pcoll_parrived(pcoll_req_t req, int part, int *flag);

/* Non-blocking test of the whole epoch (MPI_Test): *flag = 1 once every
 * partition has arrived; completes the epoch like pcoll_wait when it does.
 * Returns the epoch's error as pcoll_wait does. */
int pcoll_test(pcoll_req_t req, int *flag);

/* Blocks until every partition has arrived (by its flag, or by the
 * kernel's clean retirement; see pcoll_parrived) and the epoch is complete
 * (Section 4.5, Final Synchronization: completion only after every chunk's
 * synchronization point; MPI_Wait of the MPI-4 model).
 * Returns PCOLL_ERR_ABORTED if the kernel gave up on its own deadline
 * (configurable, default 10 s) because some partition was never readied.
 * A request with no active epoch returns at once. */
int pcoll_wait(pcoll_req_t req);

/* As pcoll_wait, but gives up after `ms` milliseconds (not in the paper or
 * the MPI-4 model; a way out of an epoch whose partitions never come): the
 * kernel is told to stop waiting for unready partitions, the call returns
 * PCOLL_ERR_TIMEOUT once it has drained, and the epoch is over (partitions
 * that had arrived are final; the others are undefined).  Device-side
 * signals of that epoch still queued ready nothing when they run.
 * PCOLL_ERR_ARG for ms < 0. */
int pcoll_wait_timeout(pcoll_req_t req, int ms);

/* Makes `stream` wait (on the device) for the end of the current epoch's
 * kernel: the non-blocking final synchronization of Section 4.5, which
 * records an event after the transfer and makes the user's stream wait on
 * it instead of blocking the host.  Does not complete the epoch (call
 * pcoll_wait or pcoll_test before the next start).  PCOLL_ERR_STATE if no
 * epoch is active. */
int pcoll_wait_on_stream(pcoll_req_t req, void *stream);

/* Releases the request and everything it owns (flags, counters, cached
 * descriptor tables and graphs), after waiting for its last kernel to
 * retire (MPI_Request_free).  PCOLL_ERR_STATE while an epoch is active. */
int pcoll_free(pcoll_req_t req);

const char *pcoll_strerror(int code);

/* Detail of the last PCOLL_ERR_HIP seen by the calling thread (the failing
 * HIP call and its error name), or "". */
const char *pcoll_last_error_detail(void);

/* -------------------------------------------------------- configuration */

typedef struct {
  int tile_elems;    /* largest tile (one workgroup's unit of work), in
                        elements; a multiple of 1024.  Tiles shrink toward
                        the end of an epoch (guided self-scheduling) */
  int min_tile_elems; /* smallest tile; a multiple of 1024, <= tile_elems */
  int groups;        /* workgroups of the persistent kernel; 0 =
                        groups_per_cu x compute units, but no more than
                        the device holds at once (HIP's occupancy of the
                        selected kernel).  Either way no more than the
                        message has tiles */
  int groups_per_cu; /* used when groups = 0 */
  int comp;          /* float sums: 1 = Sum2 compensated, 0 = plain */
  int graph;         /* 1 = start replays a cached graph (captured once per
                        binding and configuration), 0 = direct launch (the
                        default: an epoch is one kernel, so a graph has no
                        launches to save and its launch costs more) */
  int timeout_ms;    /* device-side deadline of one epoch */
  int debug;         /* bit 0: count tiles reduced per partition
                        (pcoll_debug_tile_hits); bit 1: per-workgroup
                        wall-clock trace (pcoll_debug_trace); bit 2: no
                        instrumentation.  Any non-zero value also times
                        the epoch's kernel (stats last_kernel_ms) */
  int interleave;    /* tile layout: 0 = each tile is a contiguous range of
                        its partition; otherwise tiles are interleaved in
                        bands of B consecutive tiles (1: B = the launch's
                        workgroups; n >= 2: B = n): tile j of a band of m
                        tiles takes every m-th row (64 lanes x 16 bytes)
                        of the band starting at its row j */
  int group_waves;   /* wavefronts per workgroup (1..8); they share each
                        tile's rows */
  int publish_batch; /* finished tiles a workgroup publishes with one
                        release (1..64).  A workgroup also publishes before
                        it waits for readied work, so the batch only delays
                        arrival flags while the kernel has a backlog:
                        larger amortizes the L2 writeback, smaller lets
                        partitions arrive sooner under backlog */
  int guide;         /* guided self-scheduling divisor f (0..64): a
                        partition queued with R rows of work left in the
                        epoch gets tiles of about R / (f x workgroups) rows,
                        clamped to [min_tile_elems, tile_elems]; 0 = every
                        tile has tile_elems elements */
  int unroll;        /* rows (64 lanes x 16 bytes) each lane keeps loading
                        at once in the int32 / fp32 / bf16 kernels at 3..8
                        ranks: 4 (the default) or 2, which takes about 40 %
                        fewer registers per wave and leaves room for
                        kernels that run beside the reduction (see
                        pcoll_pready_on_stream); above 8 ranks 2 or 1 */
  int producers;     /* room for producer kernels beside the reduction:
                        1 = the launch keeps one resident wave per SIMD
                        (one workgroup per compute unit unless `groups` is
                        given, at most 4 waves each) and 2 rows in flight
                        per lane, so that the kernels producing the data
                        that device-side signals follow (matrix-core ones
                        included) find registers and wave slots while the
                        reduce kernel waits; 0 = the tuned launch, for
                        requests readied from the host; -1 (the default) =
                        automatic: the tuned launch until the request's
                        first device-side signal (pcoll_pready_on_stream,
                        pcoll_pready_rank_on_stream), room from the next
                        start on.  Overrides groups_per_cu, group_waves
                        above 4 and unroll while room is kept. */
} pcoll_config_t;

/* Reads the request's configuration.  The defaults come from the tuned
 * table (env PCOLL_TUNE_FILE, else the table shipped next to the library),
 * then from environment overrides: PCOLL_TILE, PCOLL_MIN_TILE, PCOLL_GROUPS,
 * PCOLL_GROUPS_PER_CU, PCOLL_COMP, PCOLL_GRAPH, PCOLL_TIMEOUT_MS,
 * PCOLL_DEBUG, PCOLL_INTERLEAVE, PCOLL_GUIDE, PCOLL_GROUP_WAVES,
 * PCOLL_PUBLISH_BATCH, PCOLL_UNROLL, PCOLL_PRODUCERS. */
int pcoll_get_config(pcoll_req_t req, pcoll_config_t *cfg);

/* Replaces the configuration (not while an epoch is active).  Fields out of
 * range give PCOLL_ERR_ARG and leave the request unchanged. */
int pcoll_set_config(pcoll_req_t req, const pcoll_config_t *cfg);

/* ------------------------------------------------- allocation-free epoch */

/* Most partitions pcoll_reduce_noalloc takes (its scratch array is fixed:
 * 512 KiB per device, 80 bytes per partition). */
#define PCOLL_NOALLOC_MAX_PARTS 4096

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops that must not call hipMalloc): one epoch of the request path for a
 * single message -- pcoll_init, pcoll_bind, pcoll_start, every partition
 * readied at once, and completion on `stream` -- with the same results,
 * enqueued on `stream` without allocating anything (no hipMalloc, no pinned
 * host memory, no events).  The partition table, bucket descriptor, work
 * queue, counters and ready list live in a file-scope device array of
 * 512 KiB that each device holds until the process ends; a set-up kernel
 * rewrites what must start at zero before the reduce kernel runs.  Calls on
 * one device share that array: calls that overlap on one device (two
 * streams, or two threads) race and must be serialized by the caller.
 * The output is final once `stream` has passed the call; nothing is
 * waited for on the host.  Arguments as pcoll_init (count, dtype, op,
 * nparts, nranks) and pcoll_bind for one bucket (rank_bufs: nranks device
 * pointers; out; rank_scales / out_scale for the 8-bit floats, the lo
 * array as out_scale for bf16 pairs); the launch configuration is the
 * tuned default (and the PCOLL_* environment).  PCOLL_ERR_UNSUPPORTED for
 * more than PCOLL_NOALLOC_MAX_PARTS partitions; other errors as pcoll_init
 * and pcoll_bind.  The first call on a device looks the array's address
 * up (and reads the tuned table once per process). */
int pcoll_reduce_noalloc(size_t count, pcoll_dtype_t dtype, pcoll_op_t op,
                         int nparts, int nranks, const void *const *rank_bufs,
                         void *out, const void *const *rank_scales,
                         void *out_scale, void *stream);

/* ----------------------------------------------------------- inspection */

/* Partitions of the request (nbuckets * nparts). */
int pcoll_num_parts(pcoll_req_t req, int *nparts_total);

/* Bucket, first element and length of a global partition. */
int pcoll_part_info(pcoll_req_t req, int part, int *bucket, size_t *offset,
                    size_t *length);

typedef struct {
  uint64_t epochs;          /* starts */
  uint64_t graph_launches;  /* starts served by a cached graph */
  uint64_t graph_captures;  /* graphs captured and instantiated */
  uint64_t cache_hits;      /* binds served by the binding cache */
  uint64_t cache_misses;
  uint64_t cache_evictions;
  double last_capture_ms;     /* host time of the last capture */
  double last_instantiate_ms; /* host time of the last instantiation */
  float last_kernel_ms;       /* device time of the last epoch's kernel,
                                 if the config field debug was non-zero,
                                 else -1: from the kernel's own start to its
                                 end for direct launches (events stamped by
                                 hipExtLaunchKernel), from a marker before
                                 the replay to one after it in graph mode */
  double kernel_ms_total;     /* sum of the timed epochs' kernel times */
  uint64_t kernel_timed;      /* epochs timed (debug non-zero) */
  int groups;                 /* workgroups of the last launch */
  int group_waves;            /* wavefronts per workgroup of the last launch */
  int unroll;                 /* rows each lane of the last launch keeps
                                 loading at once: 4 or 2 up to 8 ranks, 2
                                 or 1 above (config `unroll` 4 or 2), at
                                 most 2 for bf16 max, 1 in the 8-bit
                                 kernels */
} pcoll_stats_t;

int pcoll_get_stats(pcoll_req_t req, pcoll_stats_t *st);

/* Debug mode only: per partition, the tiles reduced in the last epoch and
 * the tile count chosen when it was queued (they must be equal: every tile
 * exactly once). */
int pcoll_debug_tile_hits(pcoll_req_t req, uint32_t *hits, uint32_t *tiles,
                          int n);

/* Debug mode bit 1 only (config field debug): the trace of the last
 * epoch, 4 words per workgroup of its launch -- the device wall clock when
 * the workgroup started, when its first tile was queued (0 if none was),
 * and when it found no tile left (or gave up), then the number of tiles it
 * reduced -- copied to stamps[0..n) (n >= 4 * groups for all of them).
 * *groups receives the launch's workgroup count and *clock_khz the wall
 * clock's rate.  Waits for the epoch's kernel to retire.  PCOLL_ERR_STATE
 * without the debug bit, while an epoch is active or before the first. */
int pcoll_debug_trace(pcoll_req_t req, uint64_t *stamps, int n, int *groups,
                      int *clock_khz);

/* Test hook: clears every epoch stamp of the request (after waiting for the
 * whole device to go idle, so that no ready signal of an ended epoch is
 * still queued) and sets the epoch count so that the next start runs epoch
 * last + 1, or epoch 2 when `last` is 2^32 - 1 (epoch 0 is never used).
 * The library does the same clear by itself when the count wraps, since
 * stamps left from 2^32 epochs earlier could pass for current ones; this
 * call lets a test cross the wrap.  PCOLL_ERR_STATE while an epoch is
 * active. */
int pcoll_debug_set_epoch(pcoll_req_t req, uint32_t last);

/* Host-only partition plan (no GPU needed): for a message of `count`
 * elements of `dtype` split into `nparts` partitions, writes the common
 * partition length to *psize and, if non-NULL, offsets/lengths of each. */
int pcoll_plan(size_t count, pcoll_dtype_t dtype, int nparts, size_t *psize,
               size_t *offsets, size_t *lengths);

/* ------------------------------------------------------ producer packing */
/* The producer side of the low-precision payloads (not in the paper, which
 * moves bytes): encoders whose codes and scales the reduce kernels decode.
 * Each enqueues one kernel on `stream`; PCOLL_ERR_ARG for null or
 * misaligned pointers, PCOLL_ERR_HIP if the launch fails. */

/* dst[i] = bf16 of src[i], round to nearest even.  n elements; src, dst
 * 16-byte aligned device pointers; enqueued on `stream`. */
int pcoll_pack_bf16(const float *src, uint16_t *dst, size_t n, void *stream);

/* e4m3 codes with one binary32 scale per block of 256 elements (the last
 * block may be short): s = amax / 448 (1 if that is not a normal number),
 * dst[i] = e4m3(src[i] * (1 / s)), saturating, round to nearest even. */
int pcoll_pack_fp8(const float *src, uint8_t *dst, float *scales, size_t n,
                   void *stream);

/* As pcoll_pack_fp8, to e5m2 codes: s = amax / 57344 (1 if that is not a
 * normal number), dst[i] = e5m2(src[i] * (1 / s)), saturating at
 * +-57344, round to nearest even. */
int pcoll_pack_e5m2(const float *src, uint8_t *dst, float *scales, size_t n,
                    void *stream);

/* MX blocks of 32 (the last block may be short): scale byte b = e + 127
 * for the smallest e >= -127 with max |src| <= 448 * 2^e (b = 0 for an
 * all-zero block), dst[i] = e4m3(src[i] / 2^e), round to nearest even
 * (never saturating).  scales holds ceil(n / 32) bytes; src and dst are
 * 16-byte aligned. */
int pcoll_pack_mxfp8(const float *src, uint8_t *dst, uint8_t *scales,
                     size_t n, void *stream);

/* --------------------------------------------------- measurement probes */

/* Streaming copy of `bytes` (a multiple of 16) with 16-byte loads/stores:
 * the attainable-bandwidth reference of the device. */
int pcoll_probe_copy(void *dst, const void *src, size_t bytes, void *stream);

/* The reduce's memory traffic without its protocol or arithmetic: reads
 * `nsrc` (1, 2, 4, 8 or 16) device buffers of `bytes` each (srcs is a host
 * array of 16-byte aligned device pointers) with 16-byte nontemporal loads
 * and, with write = 1, stores their bitwise XOR to `dst` (`bytes` bytes):
 * nsrc read streams and one write stream, the mix of a reduction over nsrc
 * ranks.  With write = 0 nothing is stored (`dst` must still hold 16
 * bytes): read streams only.  layout 0: a grid-stride stream (thread i
 * takes vectors i, i + T, ...; `bytes` a multiple of 16); layout 1: the
 * reduce's own schedule (rows of 64 x 16 bytes, tiles of 32 rows in bands
 * of 16 tiles, 2 workgroups of 8 waves per compute unit, each taking tiles
 * in turn; `bytes` a multiple of 1024, at most 64 GiB), so that the reduce
 * kernel's time against it is what its readiness and completion protocol
 * costs; layout 2: contiguous shares (4 workgroups of 256 threads per
 * compute unit, each streaming its own 1 / (4 x units) of every buffer,
 * 8 / nsrc vectors per source in flight per thread, at least 1; `bytes` a
 * multiple of 16), the fastest pattern for plain streams.  The
 * attainable-bandwidth references of the reduce kernels; PCOLL_ERR_ARG for
 * other counts, layouts or sizes, null or misaligned pointers. */
int pcoll_probe_stream(const void *const *srcs, int nsrc, void *dst,
                       size_t bytes, int write, int layout, void *stream);

/* Fills `bytes` (a multiple of 16) with a 32-bit pattern. */
int pcoll_probe_fill(void *dst, size_t bytes, uint32_t value, void *stream);

/* Device facts: compute units, wall-clock rate (kHz), gcn arch name. */
int pcoll_device_info(int *compute_units, int *wall_clock_khz, char *arch,
                      int arch_len);

int pcoll_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PCOLL_H */
