/*
 * gq.h -- C ABI of the MI355X concurrent-queue library (libgq.so).
 *
 * The library implements the three GPU FIFO queues of "Scalable Concurrent
 * Queues for GPU" (arXiv 2606.01693):
 *   GQ_LFQ      G-LFQ, bounded and lock-free (Section III-B, Algorithm 1);
 *   GQ_WFQ      G-WFQ, bounded and wait-free under co-residency and fair
 *               scheduling (Section III-C, Algorithm 2, Theorems of III-C);
 *   GQ_WFQ_YMC  G-WFQ-YMC, a Yang/Mellor-Crummey-style wait-free queue over a
 *               preallocated cell pool (Section III-A).
 *
 * Contract (Sections I and IV): every queue is linearizable with respect to
 * the sequential FIFO -- enqueue appends, dequeue returns the head or EMPTY --
 * and delivers each item exactly once.  The bounded queues (LFQ, WFQ) hold at
 * most `capacity` items; an enqueue that finds no free slot answers GQ_FULL
 * and has no effect.  G-WFQ-YMC is unbounded within its cell pool and never
 * answers FULL; running out of pool cells latches GQ_ERR_POOL_EXHAUSTED.
 *
 * Conventions for every entry point:
 *   - Host functions return gq_status, never throw and never abort.
 *   - Pointers named d_* are device pointers (hipMalloc or torch CUDA memory)
 *     owned by the caller; they must stay valid until the stream work that
 *     uses them has finished.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     All device work is stream-ordered and asynchronous; a call returns once
 *     the work is enqueued.
 *   - Only one stream at a time may operate on a given queue.
 *   - Errors raised inside kernels (pool exhausted, invariant violated) latch
 *     into a device word read back by gq_check_error().
 */
#ifndef GQ_H
#define GQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GQ_OK = 0,
    GQ_EMPTY = 1,                 /* per-op: dequeue found the queue empty     */
    GQ_FULL = 2,                  /* per-op: enqueue found no free slot        */
    GQ_ERR_INVALID = -1,          /* bad argument                              */
    GQ_ERR_NOMEM = -2,            /* device allocation failed / buffer small   */
    GQ_ERR_HIP = -3,              /* a HIP runtime call failed                 */
    GQ_ERR_RESIDENCY = -4,        /* requested lanes cannot all be resident    */
    GQ_ERR_CYCLE_BOUND = -5,      /* G-WFQ: R <= D*k/n + 6 (Lemma 4)           */
    GQ_ERR_POOL_EXHAUSTED = -6,   /* G-WFQ-YMC ran out of preallocated cells   */
    GQ_ERR_DEVICE = -7,           /* a device-side invariant check failed      */
    GQ_ERR_TOO_LARGE = -8         /* beyond an entry point's fixed maximum size */
} gq_status;

typedef enum { GQ_LFQ = 0, GQ_WFQ = 1, GQ_WFQ_YMC = 2 } gq_kind;

/* Slot layouts of the 2n-entry index rings (the paper pads cells to a cache
 * line to avoid false sharing, Section V "Devices"):
 *   GQ_SLOTS_REMAP   8-byte entries, 16 per 128-byte line, with consecutive
 *                    tickets mapped to different lines (compact footprint);
 *   GQ_SLOTS_PADDED  one entry per 128-byte line;
 *   GQ_SLOTS_LINEAR  8-byte entries in ticket order: the consecutive tickets
 *                    of one WaveFAA share lines, so the wavefront's slot
 *                    atomics coalesce into a few line operations.            */
typedef enum { GQ_SLOTS_REMAP = 0, GQ_SLOTS_PADDED = 1, GQ_SLOTS_LINEAR = 2 } gq_slot_mode;

/* Option flags (gq_options.flags):
 *   GQ_OPT_FENCED      hand payloads over with an agent-scope release on the
 *                      install CAS and an acquire on the consume, and plain
 *                      payload stores/loads (the default instead exchanges the
 *                      payload atomically and waits for it before the install,
 *                      which needs no cache write-back or invalidate);
 *   GQ_OPT_WFQ_TUNING  use wfq_patience_enq / wfq_patience_deq / wfq_help_delay
 *                      instead of the defaults (64 / 256 / 64); a patience of 0
 *                      sends every G-WFQ operation down the slow path.          */
#define GQ_OPT_FENCED 1u
#define GQ_OPT_WFQ_TUNING 2u

typedef struct gq_options {
    uint32_t slot_mode;        /* gq_slot_mode (opts == NULL: GQ_SLOTS_LINEAR) */
    uint32_t flags;            /* GQ_OPT_* bits                               */
    uint64_t ymc_pool_cells;   /* G-WFQ-YMC pool size; 0 = 2^20 cells or
                                  64 * capacity, whichever is larger          */
    uint32_t wfq_patience_enq; /* fast-path attempts before the slow path     */
    uint32_t wfq_patience_deq;
    uint32_t wfq_help_delay;   /* D: operations between peer-record checks,
                                  1..4095                                     */
    uint32_t ticket_group;     /* lanes whose first tickets the library's
                                  workgroup-uniform drivers (gq_run_mix,
                                  batches) take with one fetch-and-add per
                                  counter: 64 = one wavefront (WaveFAA
                                  alone), 128..1024 = a workgroup of that
                                  many lanes (power of two); 0 = 1024      */
} gq_options;

/* ---- device view ---------------------------------------------------------
 * A POD snapshot of a queue's device addresses and geometry, passed by value
 * to kernels that call the device API (gq_device.h).  Fields are internal;
 * obtain one from gq_device_view().                                          */
typedef struct gq_ring_view {
    uint64_t *slots;           /* 2n packed entry words                       */
    uint64_t *head;            /* 64-bit ticket counter (own 256-byte line)   */
    uint64_t *tail;            /* 64-bit ticket counter (own 256-byte line)   */
    int64_t *threshold;        /* signed empty-detection counter              */
    void *records;             /* G-WFQ per-lane request records, else NULL   */
    uint64_t *owner;           /* G-WFQ per-slot installer hints, else NULL   */
    uint8_t *hint;             /* G-LFQ, G-WFQ per-lane "last dequeue found it empty"
                                  bytes, else NULL                            */
    uint64_t *announce;        /* G-WFQ: lane + 1 of the announced slow-path
                                  request, 0 if none (own 256-byte line)      */
} gq_ring_view;

typedef struct gq_dev {
    uint32_t kind;             /* gq_kind                                     */
    uint32_t item_width;       /* 4 or 8 bytes                                */
    uint32_t log2_cap;         /* log2(capacity)                              */
    uint32_t slot_mode;        /* gq_slot_mode                                */
    uint32_t max_threads;      /* k: lane ids passed to the device API < k    */
    uint32_t flags;            /* GQ_OPT_* bits in effect                     */
    uint64_t capacity;         /* n                                           */
    void *data;                /* n payload cells of item_width bytes         */
    gq_ring_view aq;           /* ring of allocated indices                   */
    gq_ring_view fq;           /* ring of free indices                        */
    uint64_t *err;             /* latched device error (0 = none)             */
    uint64_t *stats;           /* device counters, see gq_stats               */
    uint64_t *ymc_cells;       /* G-WFQ-YMC pool: val[P], enq[P], deq[P]      */
    uint64_t ymc_pool_cells;
    uint64_t *ymc_ctr;         /* G-WFQ-YMC T at [0], H at [32]               */
    void *ymc_handles;         /* G-WFQ-YMC per-lane handles                  */
    uint32_t patience_enq;     /* G-WFQ fast-path attempts                    */
    uint32_t patience_deq;
    uint32_t help_delay;       /* G-WFQ help delay D                          */
    uint32_t group_lanes;      /* gq_options.ticket_group (resolved)          */
    uint32_t *help_ctr;        /* G-WFQ per-lane <next peer:20 | ops:12>      */
    uint8_t *ymc_hint;         /* G-WFQ-YMC per-lane "last dequeue found the
                                  queue empty" bytes, else NULL               */
} gq_dev;

typedef struct gq_stats {
    uint64_t ok_enq, ok_deq;   /* successful operations                       */
    uint64_t full, empty;      /* failed operations                           */
    uint64_t cas_fail;         /* failed slot CAS attempts                    */
    uint64_t tickets;          /* tickets taken (all counters)                */
    uint64_t slow_enter;       /* G-WFQ / YMC slow-path entries               */
    uint64_t helps;            /* peer requests helped                        */
    uint64_t scans;            /* G-WFQ record scans to finalize an enqueue   */
    uint64_t dropped;          /* operations a device fail-safe bound stopped
                                  (error latched): an enqueue so stopped
                                  reports GQ_ERR_DEVICE and its item is lost;
                                  a dequeue that already took its item still
                                  reports GQ_OK, its free index being lost  */
} gq_stats;

/* Bytes of device memory a queue with these parameters needs.
 * capacity: power of two in [2, 2^30]; item_width: 4 or 8;
 * max_threads (k): the most lanes that may operate on the queue at once, in
 * [1, 2^20); G-WFQ and G-WFQ-YMC keep one record per lane id (< k), and all
 * queues size their empty-detection threshold for k concurrent lanes.
 * opts may be NULL.  Returns GQ_ERR_INVALID on bad parameters and
 * GQ_ERR_CYCLE_BOUND when G-WFQ's cycle tags (R = 2^15) cannot satisfy
 * R > D*k/n + 6 (Section III-C, Lemma 4).                                    */
gq_status gq_required_bytes(gq_kind kind, uint64_t capacity, uint32_t item_width,
                            uint32_t max_threads, const gq_options *opts,
                            uint64_t *bytes);

/* Create an empty queue (same parameter rules as gq_required_bytes).
 * dev_buf: optional caller-owned device buffer of buf_bytes >= required bytes
 * (256-byte aligned); NULL lets the library allocate (and later free) it.
 * The queue is initialised on the default stream and synchronised before
 * return.  *out receives an opaque handle.                                   */
typedef struct gq_queue gq_queue;
gq_status gq_create(gq_kind kind, uint64_t capacity, uint32_t item_width,
                    uint32_t max_threads, const gq_options *opts, void *dev_buf,
                    uint64_t buf_bytes, gq_queue **out);

/* Destroy the handle; frees device memory only if the library allocated it.
 * The caller must have synchronised all work on the queue.                    */
gq_status gq_destroy(gq_queue *q);

/* Return the queue to the empty state, stream-ordered.                        */
gq_status gq_reset(gq_queue *q, void *stream);

/* Batched enqueue: m items (item_width bytes each, contiguous) from d_items,
 * each tried once by its own lane, concurrently, with no order among them.
 * d_status (nullable): one byte per item, GQ_OK or GQ_FULL; an operation that
 * a device fail-safe bound stopped (the queue's error is latched, see
 * gq_stats.dropped) stores the low byte of its negative gq_status.
 * d_num_ok (nullable): a device uint64 to which the OK count is ADDED.
 * Batches issued on one stream take effect in stream order.  The first
 * ticket of each operation is taken once per gq_options.ticket_group lanes.  */
gq_status gq_enqueue_batch(gq_queue *q, const void *d_items, uint64_t m,
                           uint8_t *d_status, uint64_t *d_num_ok, void *stream);

/* Batched dequeue: m concurrent single dequeues; item i goes to d_out[i]
 * (item_width bytes; 0 when EMPTY).  d_status: GQ_OK or GQ_EMPTY.             */
gq_status gq_dequeue_batch(gq_queue *q, void *d_out, uint64_t m,
                           uint8_t *d_status, uint64_t *d_num_ok, void *stream);

/* Device view for kernels that call gq_enqueue/gq_dequeue (gq_device.h).      */
gq_status gq_device_view(const gq_queue *q, gq_dev *out);

/* Copy the device counters to *out (synchronises the stream).                 */
gq_status gq_read_stats(gq_queue *q, gq_stats *out, void *stream);

/* Clear the device counters, stream-ordered.                                  */
gq_status gq_clear_stats(gq_queue *q, void *stream);

/* Synchronise the stream and report the latched device error, if any.        */
gq_status gq_check_error(gq_queue *q, void *stream);

/* Static description of a status code.                                       */
const char *gq_status_str(gq_status s);

#ifdef __cplusplus
}
#endif
#endif /* GQ_H */
