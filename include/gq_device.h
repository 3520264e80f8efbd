/*
 * gq_device.h -- device API of the MI355X concurrent queues (HIP, gfx950).
 *
 * Kernels obtain a gq_dev with gq_device_view() (gq.h) and call
 *
 *   int gq_enqueue(const gq_dev& q, uint64_t item, uint32_t tid);
 *   int gq_dequeue(const gq_dev& q, uint64_t* item, uint32_t tid);
 *
 * which return GQ_OK, GQ_FULL (enqueue on a bounded queue with no free
 * slot) or GQ_EMPTY (dequeue), with the semantics of gq.h: each call is one
 * linearizable FIFO operation (Sections III-B and III-C; linearization at the
 * install CAS, at Consume, or at the empty observation).
 *
 * Calling rules:
 *   - Any subset of a wavefront's lanes may call, in divergent code; the
 *     lanes that arrive together share one ticket fetch-and-add (the
 *     wave-batched fast path, Section III-B, Lemma 1).
 *   - No barrier is used inside; no __syncthreads around the calls is needed.
 *   - tid identifies the calling lane among all lanes that use the queue
 *     concurrently: unique and < gq_dev.max_threads.  G-WFQ and G-WFQ-YMC
 *     index their per-lane request records with it (Section III-C, "Data
 *     structure"; Section III-A); all three keep a per-lane "last dequeue
 *     found the queue empty" byte with it (G-LFQ skips it for tid >=
 *     max_threads).
 *   - Wait-freedom of G-WFQ and G-WFQ-YMC holds while every participating
 *     lane's wavefront stays resident and is fairly scheduled (Section III-C,
 *     Theorem "GPU-resident wait-freedom"); G-LFQ is lock-free.
 *   - Items of width 4 use the low 32 bits.  G-WFQ-YMC reserves the values 0
 *     and UINT64_MAX as cell markers; enqueuing them is invalid.
 *
 * The _k variants take the queue kind as a template argument (no runtime
 * switch) and count failed slot CAS attempts into `cas_fail`.
 */
#ifndef GQ_DEVICE_H
#define GQ_DEVICE_H

#include "gq.h"
#include "gq/lfq.h"
#include "gq/wfq.h"
#include "gq/ymc.h"

template <int KIND>
__device__ __forceinline__ int gq_enqueue_k(const gq_dev& q, uint64_t item, uint32_t tid,
                                            uint32_t& cas_fail) {
  if constexpr (KIND == GQ_LFQ) {
    return gq::lfq::enqueue(q, item, cas_fail, tid < q.max_threads ? tid : gq::lfq::NO_LANE);
  } else if constexpr (KIND == GQ_WFQ) {
    return gq::wfq::enqueue(q, item, tid, cas_fail);
  } else {
    return gq::ymc::enqueue(q, item, tid, cas_fail);
  }
}

template <int KIND>
__device__ __forceinline__ int gq_dequeue_k(const gq_dev& q, uint64_t* item, uint32_t tid,
                                            uint32_t& cas_fail) {
  if constexpr (KIND == GQ_LFQ) {
    return gq::lfq::dequeue(q, item, cas_fail, tid < q.max_threads ? tid : gq::lfq::NO_LANE);
  } else if constexpr (KIND == GQ_WFQ) {
    return gq::wfq::dequeue(q, item, tid, cas_fail);
  } else {
    return gq::ymc::dequeue(q, item, tid, cas_fail);
  }
}

/* Workgroup-uniform form: every thread of the workgroup calls
 * gq_group_op_k together (uniform control flow, blockDim a multiple of 64
 * and at most 1024), each with its own role: gq::ROLE_ENQ (enqueue `item`),
 * gq::ROLE_DEQ (dequeue into `item`) or gq::ROLE_NONE.  The first ticket of
 * each inner operation is taken with one fetch-and-add per counter for the
 * whole workgroup (Lemma 1's aggregation at workgroup scale); the operation
 * is otherwise the same linearizable enqueue or dequeue as above.  `lds` is
 * one __shared__ gq::GroupLds per workgroup and `par` a per-thread word that
 * starts at 0 and is passed to every call.  `help` (G-WFQ; optional): the
 * lane's help step state held in a register across calls -- load it with
 * gq::wfq::help_load(q, tid) before the first call and store it back with
 * gq::wfq::help_store(q, tid, h) after the last; without it each operation
 * reads and writes the queue's per-lane copy.  Returns the lane's status
 * (GQ_OK for ROLE_NONE).  Contains barriers: never call it from divergent
 * code.                                                                      */
template <int KIND>
__device__ __forceinline__ int gq_group_op_k(const gq_dev& q, int role, uint64_t& item,
                                             uint32_t tid, uint32_t& cas_fail, gq::GroupLds& lds,
                                             uint32_t& par, uint32_t* help = nullptr) {
  if constexpr (KIND == GQ_LFQ) {
    (void)help;
    return gq::lfq::group_op(q, role, item, cas_fail, lds, par,
                             tid < q.max_threads ? tid : gq::lfq::NO_LANE);
  } else if constexpr (KIND == GQ_WFQ) {
    return gq::wfq::group_op(q, role, item, tid, cas_fail, lds, par, help);
  } else {
    (void)help;
    return gq::ymc::group_op(q, role, item, tid, cas_fail, lds, par);
  }
}

__device__ __forceinline__ int gq_enqueue(const gq_dev& q, uint64_t item, uint32_t tid) {
  uint32_t cf = 0;
  switch (q.kind) {
    case GQ_LFQ: return gq_enqueue_k<GQ_LFQ>(q, item, tid, cf);
    case GQ_WFQ: return gq_enqueue_k<GQ_WFQ>(q, item, tid, cf);
    default: return gq_enqueue_k<GQ_WFQ_YMC>(q, item, tid, cf);
  }
}

__device__ __forceinline__ int gq_dequeue(const gq_dev& q, uint64_t* item, uint32_t tid) {
  uint32_t cf = 0;
  switch (q.kind) {
    case GQ_LFQ: return gq_dequeue_k<GQ_LFQ>(q, item, tid, cf);
    case GQ_WFQ: return gq_dequeue_k<GQ_WFQ>(q, item, tid, cf);
    default: return gq_dequeue_k<GQ_WFQ_YMC>(q, item, tid, cf);
  }
}

#endif /* GQ_DEVICE_H */
