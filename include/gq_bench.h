/*
 * gq_bench.h -- workload drivers and roofline probes of libgq.so (C ABI).
 *
 * These entry points launch the paper's benchmark shapes on a queue created
 * with gq.h, optionally recording a per-operation history for the
 * linearizability checks (Section IV: fields proc, op, arg/ret, call, end).
 * Same conventions as gq.h: device pointers are caller-owned, calls are
 * stream-ordered and asynchronous, status codes are returned.
 *
 * Per-operation randomness is the counter-based SplitMix64 stream
 * r(seed, c) = mix(seed + (c + 1) * 0x9E3779B97F4A7C15) with
 * c = (lane << 32) | draw, evaluated on the device.
 */
#ifndef GQ_BENCH_H
#define GQ_BENCH_H

#include <stdint.h>

#include "gq.h"

#ifdef __cplusplus
extern "C" {
#endif

/* History buffers (device memory).  Lane g's r-th operation is stored at
 * g * per_lane + r while r < per_lane; further operations are executed but not
 * stored.  count[g] receives the number of operations lane g executed.
 * opst = op | (status << 1), op 0 = enqueue, 1 = dequeue; status as gq_status.
 * val is the enqueued argument or the dequeued value (0 for EMPTY).
 * call/ret are device real-time stamps (100 MHz) taken before the call and
 * after every memory access of the operation completed: with the default
 * atomic hand-off every such access is a device-coherent atomic, so the lane
 * only waits for them (as the unrecorded kernels' operations do); with
 * GQ_OPT_FENCED the end stamp follows an agent-scope release.                */
typedef struct gq_history {
    uint64_t *val;
    uint64_t *call;
    uint64_t *ret;
    uint8_t *opst;
    uint32_t *count;
    uint32_t per_lane;
    uint32_t reserved;
} gq_history;

/* Mixed workload (Section V-A micro-benchmark shape, fixed op count): each of
 * `lanes` lanes (a multiple of 64) performs ops_per_lane operations; op r of
 * lane g is an enqueue when the top bit of r(seed, (g << 32) | r) is 0, else
 * a dequeue.  Each op is tried once: FULL/EMPTY outcomes are counted, not
 * retried.  Lane g's j-th successful enqueue carries the token
 * (g << 32) | (j + 1) (Section IV token format).
 * Launch: workgroups of the queue's ticket group (gq_options.ticket_group,
 * 1024 lanes by default), halved until it divides `lanes`, every lane taking
 * part in its workgroup's aggregated first tickets; a group of 64 lanes means
 * per-wavefront tickets in workgroups of 256 lanes (64 when 256 does not
 * divide `lanes`).
 * d_counts[8] += {ok_enq, ok_deq, full, empty, S1_deq, S2_deq, S1_enq,
 * S2_enq}: the wrapping (mod 2^64) sums of v and v * v over the items v
 * dequeued (deq) and enqueued (enq) successfully, as in gq_run_prodcons.
 * d_lane_enq (nullable): lane g's count of successful enqueues is stored at
 * d_lane_enq[g], so its tokens are known without a history.  hist may be
 * NULL; with a history the same work runs in a recording kernel.
 * G-WFQ: all lanes must be co-resident (its wait-freedom assumes it, Section
 * III-C), else GQ_ERR_RESIDENCY.  G-WFQ-YMC: a run that may need more cells
 * than the pool holds (lanes * ops_per_lane > pool cells) is refused with
 * GQ_ERR_POOL_EXHAUSTED before anything is launched.                         */
gq_status gq_run_mix(gq_queue *q, uint64_t seed, uint32_t lanes, uint32_t ops_per_lane,
                     uint64_t *d_counts, uint32_t *d_lane_enq, const gq_history *hist,
                     void *stream);

/* ---- many independent queues in one launch ---------------------------------
 * A gq_multi binds nq queues of one kind; queue i gets lanes_per_queue[i]
 * lanes (a multiple of 64, at most that queue's max_threads), i.e. whole
 * wavefronts, laid out queue after queue; the total must fill whole
 * workgroups of `block` (64, 128 or 256) lanes.  gq_multi_run_mix runs the
 * mixed workload (as gq_run_mix, ops_per_lane each, lane ids counted within
 * each queue, tokens and draws from the global lane id) on every queue in ONE
 * kernel launch; d_counts[8 * i + 0..7] += queue i's eight gq_run_mix
 * counts {ok_enq, ok_deq, full, empty, S1_deq, S2_deq, S1_enq, S2_enq}.  gq_multi_capture records (seed bump + that launch) into a
 * hipGraph on `stream` (which must not be the legacy default stream);
 * gq_multi_replay launches it (each replay advances the seed by one).  With a
 * history (nullable) the captured launch records every operation into it, so
 * each replay overwrites the history with its own (lanes of all queues in
 * launch order).                                                             */
typedef struct gq_multi gq_multi;
gq_status gq_multi_create(uint32_t nq, gq_queue *const *queues, const uint32_t *lanes_per_queue,
                          uint32_t block, gq_multi **out);
gq_status gq_multi_run_mix(gq_multi *m, uint64_t seed, uint32_t ops_per_lane, uint64_t *d_counts,
                           const gq_history *hist, void *stream);
gq_status gq_multi_capture(gq_multi *m, uint64_t seed, uint32_t ops_per_lane, uint64_t *d_counts,
                           const gq_history *hist, void *stream);
gq_status gq_multi_replay(gq_multi *m, void *stream);
gq_status gq_multi_destroy(gq_multi *m);

/* Queue-driven level-synchronous BFS (Section V-B) in one persistent launch of
 * `lanes` lanes in workgroups of `block` (64..256): two empty queues qa, qb
 * of the same kind with item_width 4 (bounded kinds: capacity >= nv; a
 * G-WFQ-YMC pool must hold nv + levels * lanes cells), CSR graph (uint32
 * offsets[nv + 1], cols[offsets[nv]]), root < nv.  d_level[nv] receives hop
 * distances (0xFFFFFFFF = unreached).  d_ctl: caller-owned, 8-byte aligned
 * workspace of ctl_bytes >= 4 KiB; gq_bfs_ctl_bytes(nnz) is the size that
 * lets every high-degree vertex's list be split over all wavefronts (less
 * works, with such vertices beyond the room scanned by one wavefront each).
 * After the run d_ctl[160] = number of levels, d_ctl[192] = adjacency
 * entries scanned.  All workgroups must be co-resident (GQ_ERR_RESIDENCY
 * otherwise).  Device-side failures latch in qa's error word.               */
gq_status gq_bfs(gq_queue *qa, gq_queue *qb, const uint32_t *d_offsets, const uint32_t *d_cols,
                 uint32_t nv, uint32_t root, uint32_t *d_level, uint32_t lanes, uint32_t block,
                 uint64_t *d_ctl, uint64_t ctl_bytes, void *stream);
/* Workspace bytes for gq_bfs on a graph of nnz adjacency entries.            */
uint64_t gq_bfs_ctl_bytes(uint64_t nnz);

/* For callers that cannot allocate device memory -- code being captured into a
 * HIP graph, tight serving loops, harnesses that forbid hipMalloc: gq_bfs with
 * its two frontier queues (kind GQ_LFQ or GQ_WFQ, capacity the next power of
 * two >= max(nv, 64), item width 4, linear slots) and its workspace placed in a
 * static device array of GQ_BFS_STATIC_BYTES that the library holds on every
 * GPU it runs on until the process ends.  It calls no hipMalloc, hipFree or
 * allocating library routine.  Graph and outputs are the caller's device
 * memory as for gq_bfs; d_info (nullable) receives 4 uint64: [0] the latched
 * device error as -gq_status (0 = none), [1] levels, [2] adjacency entries
 * scanned, [3] 0.  Limits: nv <= GQ_BFS_STATIC_MAX_VERTICES and lanes <=
 * GQ_BFS_STATIC_MAX_LANES (GQ_ERR_TOO_LARGE beyond them), lanes a multiple of
 * block (64..256), all workgroups co-resident (GQ_ERR_RESIDENCY).  Every call
 * re-initialises the queues and workspace it uses, but all calls on one GPU
 * share the one array: calls that overlap in time on one GPU (streams not
 * ordered with each other) race and return wrong levels; calls on one stream
 * run one after another.                                                      */
#define GQ_BFS_STATIC_MAX_VERTICES (1u << 18)
#define GQ_BFS_STATIC_MAX_LANES 8192u
#define GQ_BFS_STATIC_BYTES (40ull << 20)
gq_status gq_bfs_static(gq_kind kind, const uint32_t *d_offsets, const uint32_t *d_cols,
                        uint32_t nv, uint32_t root, uint32_t *d_level, uint32_t lanes,
                        uint32_t block, uint64_t *d_info, void *stream);

/* Balanced workload (Section V-A "balanced kernel", fixed op count): every
 * lane performs `rounds` times (enqueue its next token; dequeue), each tried
 * once.  Tokens as in gq_run_mix.  d_counts[4] as above.                      */
gq_status gq_run_balanced(gq_queue *q, uint32_t lanes, uint32_t rounds, uint64_t *d_counts,
                          const gq_history *hist, void *stream);

/* Producer/consumer workload (Section V-A "split kernel" shape with retries):
 * d_lane_role[g] = 0 marks lane g a producer, 1 a consumer.  Each producer
 * enqueues items_per_producer tokens, retrying on FULL; consumers retry on
 * EMPTY until `target` items were taken in total.  In round r lane g is
 * active iff r(seed, (g << 32) | r) >> (64 - log2_inv_p) == 0 (always when
 * log2_inv_p == 0).  token_mode 0: (g << 32) | (seq + 1); token_mode 1:
 * (g << 20) | seq (32-bit payloads).  Producers and consumers wait for each
 * other, so all lanes must be co-resident (GQ_ERR_RESIDENCY otherwise).
 * jitter > 0 adds a seeded pause of up to `jitter` sleep units per round.
 * max_rounds bounds every lane's loop; exceeding it latches GQ_ERR_DEVICE.
 * time_limit_ms (0 = none) bounds the run's duration on the GPU clock: a lane
 * past it stops and latches GQ_ERR_DEVICE (a bounded wait, not a result).
 * With a history, every operation a lane performs is recorded, the polls that
 * answer FULL or EMPTY included (size per_lane for them).
 * d_counts[8] += {ok_enq, ok_deq, full, empty, S1_deq, S2_deq, S1_enq,
 * S2_enq}, where S1 and S2 are the wrapping (mod 2^64) sums of v and v * v
 * over the items v successfully dequeued (deq) or enqueued (enq): multiset
 * checksums that let a caller verify conservation without a history.        */
gq_status gq_run_prodcons(gq_queue *q, uint64_t seed, uint32_t lanes, uint32_t block,
                          const uint8_t *d_lane_role, uint32_t items_per_producer,
                          uint64_t target, uint32_t log2_inv_p, uint32_t token_mode,
                          uint32_t jitter, uint64_t max_rounds, uint32_t time_limit_ms,
                          uint64_t *d_counts, const gq_history *hist, void *stream);

/* Fixed-duration run (Section V-A's balanced and split kernels): `lanes`
 * lanes (a multiple of 256, all co-resident, at most max_threads) in
 * workgroups of 256 work until warmup_us + window_us microseconds have passed
 * on the GPU's constant clock since the first lane started; a successful
 * operation counts when it completes inside the window.  mode 0 (balanced):
 * every lane alternates enqueue and dequeue; mode 1 (split): the first
 * prod_pct percent of the wavefronts only enqueue, the rest only dequeue.
 * Each operation is tried once; tokens as in gq_run_mix.  d_counts[10] +=
 * {enqueues OK in the window, dequeues OK in the window, FULL, EMPTY,
 * S1_deq, S2_deq, S1_enq, S2_enq, enqueues OK, dequeues OK} (all but the
 * first two over the whole run; S1/S2 the wrapping sums of v and v*v of the
 * items dequeued, and of the tokens enqueued, as in gq_run_mix).
 * d_lane_enq (nullable): uint32 per lane, its successful enqueues.  hist
 * (nullable): every operation recorded; a lane stops when its history row
 * (per_lane entries) is full.  d_ctl: caller-owned device memory of at least
 * 8 bytes (the shared start time), cleared by the call.                      */
gq_status gq_run_timed(gq_queue *q, uint32_t mode, uint32_t lanes, uint32_t prod_pct,
                       uint32_t warmup_us, uint32_t window_us, uint64_t *d_counts,
                       uint64_t *d_ctl, uint32_t *d_lane_enq, const gq_history *hist,
                       void *stream);

/* Scripted run for small linearizability tests: lane g (< lanes <= 1024)
 * executes n_ops[g] operations from ops[g * max_ops ...] (0 enqueue,
 * 1 dequeue) with arguments args[...], pausing pause[g * max_ops + r] sleep
 * units before op r.  Results go to hist (required, per_lane >= max_ops).
 * spread != 0: each lane runs alone in its own wavefront (one workgroup per
 * lane), so lanes really run concurrently; spread == 0: all lanes form one
 * workgroup, and lanes of one wavefront issue their operations together.      */
gq_status gq_run_script(gq_queue *q, uint32_t lanes, uint32_t spread, const uint8_t *d_ops,
                        const uint64_t *d_args, const uint16_t *d_pause,
                        const uint32_t *d_n_ops, uint32_t max_ops, const gq_history *hist,
                        void *stream);

/* ---- roofline probes -------------------------------------------------------
 * R_ctr: lanes/64 wavefronts each perform `iters` fetch-and-adds on a counter:
 *   wavefront w uses d_ctr[(w mod ncounters) * spacing_bytes / 8] (the buffer
 *   must hold ncounters * spacing_bytes bytes); one FAA per wavefront
 *   (per_lane = 0, the WaveFAA shape) or one per lane (per_lane = 1).
 * R_slot: each lane performs `iters` 64-bit CAS on slot (t mod nslots), t from
 *   a per-lane ticket sequence, slots spaced stride_bytes apart.
 * Copy: d_dst[i] = d_src[i] for n 64-bit words (HBM stream bandwidth).
 * Fence: each wavefront performs `iters` agent-scope release+acquire fences
 *   around one relaxed atomic store to its own line.                          */
gq_status gq_probe_faa(uint64_t *d_ctr, uint32_t lanes, uint32_t iters, uint32_t per_lane,
                       uint32_t ncounters, uint32_t spacing_bytes, void *stream);
gq_status gq_probe_cas(uint64_t *d_slots, uint64_t nslots, uint32_t stride_bytes,
                       uint32_t lanes, uint32_t iters, void *stream);
gq_status gq_probe_copy(uint64_t *d_dst, const uint64_t *d_src, uint64_t n, void *stream);
gq_status gq_probe_fence(uint64_t *d_lines, uint32_t lanes, uint32_t iters, uint32_t mode,
                         void *stream);

/* Number of workgroups of `block` lanes that can be resident at once for the
 * given driver kernel, summed over all compute units: "mix" (gq_run_mix's
 * per-wavefront form), "mix_group" (its workgroup-ticket form, the kernel
 * gq_run_mix launches when the ticket group exceeds 64), "prodcons".          */
gq_status gq_resident_blocks(const char *kernel, gq_kind kind, uint32_t block,
                             uint32_t *out_blocks);

/* Device properties used by the benchmark: compute units, wavefront size,
 * and the device's name (gcnArchName) copied into name[0..len).               */
gq_status gq_device_info(uint32_t *cus, uint32_t *wave, char *name, uint32_t len);

#ifdef __cplusplus
}
#endif
#endif /* GQ_BENCH_H */
