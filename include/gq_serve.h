/*
 * gq_serve.h -- serving BFS jobs through the queues (C ABI, MI355X / gfx950).
 *
 * A persistent kernel of `teams` worker teams (one workgroup each) stays on
 * the GPU between gq_serve_create and gq_serve_destroy.  The host admits jobs
 * (breadth-first searches, the paper's application of Section V-B) while
 * others run, and their work overlaps on the device:
 *
 *   host  -- arrival schedule, admission by device-memory budget ->
 *   pinned submission ring (host memory the GPU reads) ->
 *   dispatcher (whichever idle team holds the dispatch lock) moves new jobs
 *   into a device G-LFQ job queue ->
 *   a worker team dequeues a job, sets up its two per-job queues in place
 *   (G-LFQ or G-WFQ, capacity >= the job's vertex count, in a device arena),
 *   runs the level-synchronous queue BFS with workgroup barriers, hashes the
 *   level array and posts a completion record into a pinned completion ring ->
 *   host records the completion time and frees the job's memory.
 *
 * Job memory: levels (4 B per vertex) and the two per-job queues come from an
 * arena of `budget_bytes` of device memory owned by the server.  A job is
 * admitted when the bytes of all admitted, unfinished jobs plus its own
 * (CSR + levels + 2 queues) fit the budget and its arena block can be
 * allocated; admission is first come, first served (a job that does not fit
 * waits, and so do the jobs behind it).  A job larger than the whole budget is
 * refused with status GQ_ERR_NOMEM.  G-WFQ-YMC is not offered for per-job
 * queues: its cell pool is not bounded by the capacity (Section III-A), so a
 * job's bytes are not known at admission.
 *
 * Level hash of a finished job (the check that a result is the same alone and
 * in a mix):  H = sum over v < nv of splitmix64(GQ_SERVE_HASH_SEED, v) *
 * (level[v] + 1), computed in 64-bit wrapping arithmetic with level[v] as an
 * unsigned 32-bit value (0xFFFFFFFF = unreached, so unreached vertices add
 * splitmix64(seed, v) * 2^32), splitmix64(seed, c) being the c-th output of
 * the SplitMix64 generator (Steele, Lea and Flood, OOPSLA 2014).
 *
 * Threading: one host thread drives a server.  While a server exists its
 * kernel occupies the GPU: do not call hipDeviceSynchronize (or anything that
 * waits for every stream) until gq_serve_destroy; such a wait only returns
 * once the kernel's idle timeout ends it.
 */
#ifndef GQ_SERVE_H
#define GQ_SERVE_H

#include <stdint.h>

#include "gq.h"

#ifdef __cplusplus
extern "C" {
#endif

#define GQ_SERVE_HASH_SEED 0x5EED1E7E15ull

typedef struct gq_serve gq_serve;

/* One BFS job.  The CSR graph is caller-owned device memory that must stay
 * valid until the job completes (uint32 offsets[nv + 1], cols[nnz]);
 * root < nv.  nnz counts toward the job's bytes.  d_levels_out (nullable,
 * caller-owned device memory of nv uint32) receives the job's hop distances
 * (0xFFFFFFFF = unreached); without it the levels live in the arena and only
 * their hash is returned.                                                    */
typedef struct gq_serve_request {
    const uint32_t *d_offsets;
    const uint32_t *d_cols;
    uint32_t *d_levels_out;
    uint64_t nnz;
    uint32_t nv;
    uint32_t root;
} gq_serve_request;

/* Per-job result (host memory).  Times in ns from the start of gq_serve_run
 * on the host's monotonic clock; device_ns is the job's run time on its team
 * (from the GPU's constant 100 MHz clock).                                   */
typedef struct gq_serve_result {
    int64_t arrival_ns;   /* scheduled arrival (the caller's schedule)         */
    int64_t admit_ns;     /* written to the submission ring                    */
    int64_t done_ns;      /* completion seen by the host                       */
    int64_t device_ns;    /* team start to team end                            */
    uint64_t level_hash;  /* H above                                           */
    uint64_t levels;      /* BFS levels = eccentricity of the root + 1         */
    uint64_t scanned;     /* adjacency entries scanned                         */
    uint64_t job_bytes;   /* CSR + levels + two queues                         */
    uint32_t team;        /* team that ran the job                             */
    int32_t status;       /* GQ_OK, GQ_ERR_NOMEM (larger than the budget),
                             GQ_ERR_DEVICE (a queue operation failed)          */
} gq_serve_result;

/* Create a server and launch its persistent kernel on a stream of its own.
 * teams: worker workgroups (all must be co-resident: GQ_ERR_RESIDENCY
 * otherwise); team_lanes: 64..1024, a multiple of 64; job_kind: GQ_LFQ or
 * GQ_WFQ (per-job queues); budget_bytes: device-memory budget of admitted
 * jobs, also the size of the arena the server allocates; ring_slots: 1..4096,
 * the most jobs in flight at once; idle_timeout_ms: the kernel ends itself
 * after this long without work (0 = 60000), a safety net only.              */
gq_status gq_serve_create(uint32_t teams, uint32_t team_lanes, gq_kind job_kind,
                          uint64_t budget_bytes, uint32_t ring_slots, uint32_t idle_timeout_ms,
                          gq_serve **out);

/* Serve njobs requests whose arrivals are scheduled at arrival_ns[i] (ns from
 * the call, non-decreasing).  At most max_inflight (<= ring_slots) jobs are
 * admitted and unfinished at once; max_inflight = 1 runs every job alone.
 * Blocks until every job finished or failed; results go to out[i].  Returns
 * GQ_ERR_DEVICE if the kernel stopped or no job finished for 30 s.          */
gq_status gq_serve_run(gq_serve *s, uint32_t njobs, const gq_serve_request *reqs,
                       const int64_t *arrival_ns, uint32_t max_inflight, gq_serve_result *out);

/* Bytes a job occupies under the budget (CSR + levels + two queues).        */
gq_status gq_serve_job_bytes(const gq_serve *s, uint32_t nv, uint64_t nnz, uint64_t *bytes);

/* Stop the kernel, wait for it, free everything.                            */
gq_status gq_serve_destroy(gq_serve *s);

#ifdef __cplusplus
}
#endif

#endif /* GQ_SERVE_H */
