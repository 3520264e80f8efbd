// G-LFQ: the bounded lock-free queue of Section III-B (Algorithm 1).
//
// Structure (Section III-B, "Data structure"): an inner ring of 2n physical
// slots holding packed 64-bit entries, monotone Head/Tail ticket counters and
// a signed Threshold for empty detection; an outer queue built from two such
// rings -- `aq` (allocated indices) and `fq` (free indices) -- plus an array
// of n payload cells, so the rings move 32-bit indices, not payloads.
//
// Entry word (64 bits): Index in bits [0,32), Safe in bit 32, Cycle in bits
// [33,64) -- a 31-bit cycle tag compared modulo 2^31 (Lemma 2).  Index is a
// payload index, BOT (empty) or BOTC (consumed).
//
// Tickets: slot(t) = t mod 2n, cycle(t) = floor(t / 2n) mod 2^31, reserved
// with the wave-aggregated fetch-and-add (Lemma 1).
#pragma once
#include "common.h"

namespace gq {
namespace lfq {

constexpr uint32_t BOT = 0xFFFFFFFFu;   // empty slot
constexpr uint32_t BOTC = 0xFFFFFFFEu;  // consumed slot
// Looks a dequeuer takes at an entry whose enqueuer holds the ticket but has
// not installed yet (see ring_deq).
constexpr uint32_t DEQ_WAIT_POLLS = 64;

// "No lane id": the caller keeps no per-lane state (no empty hint).
constexpr uint32_t NO_LANE = 0xFFFFFFFFu;

// Result of an inner dequeue stopped by the fail-safe bound (error latched);
// never a valid index (indices are below n <= 2^30).
constexpr uint32_t GAVE_UP = 0xFFFFFFFDu;
constexpr uint32_t CYC_BITS = 31;
constexpr uint32_t CYC_MASK = (1u << CYC_BITS) - 1u;
constexpr uint32_t CYC_HALF = 1u << (CYC_BITS - 1);

__device__ __forceinline__ uint32_t e_idx(uint64_t e) { return (uint32_t)e; }
__device__ __forceinline__ bool e_safe(uint64_t e) { return (e >> 32) & 1u; }
__device__ __forceinline__ uint32_t e_cyc(uint64_t e) { return (uint32_t)(e >> 33); }
__device__ __forceinline__ uint64_t e_make(uint32_t cyc, bool safe, uint32_t idx) {
  return ((uint64_t)(cyc & CYC_MASK) << 33) | ((uint64_t)safe << 32) | idx;
}
__device__ __forceinline__ bool idx_free(uint32_t i) { return i >= BOTC; }  // BOT or BOTC

// a is strictly older than b: 0 < (b - a) mod R < R/2  (Lemma 2 / Lemma 4).
__device__ __forceinline__ bool older(uint32_t a, uint32_t b) {
  const uint32_t d = (b - a) & CYC_MASK;
  return d != 0 && d < CYC_HALF;
}

// Geometry of one ring, derived from the queue view.
struct Ring {
  uint64_t* slots;
  uint64_t* head;
  uint64_t* tail;
  int64_t* thr;
  uint8_t* hint;      // per-lane empty hints (see ring_deq), or nullptr
  uint32_t log2_2n;   // log2(2n)
  uint32_t log2_L;    // entries per line (remap mode)
  uint32_t mode;      // gq_slot_mode
  int64_t thr_reset;  // 3n - 1

  __device__ __forceinline__ uint64_t* at(uint64_t j) const {
    if (mode == GQ_SLOTS_LINEAR) return slots + j;
    if (mode == GQ_SLOTS_PADDED) return slots + (j << 4);  // 128-byte stride
    // remap: consecutive tickets land on different 128-byte lines
    const uint32_t log2_M = log2_2n - log2_L;
    const uint64_t pos = ((j & ((1ull << log2_M) - 1)) << log2_L) | (j >> log2_M);
    return slots + pos;
  }
  __device__ __forceinline__ uint64_t slot_of(uint64_t t) const {
    return t & ((1ull << log2_2n) - 1);
  }
  __device__ __forceinline__ uint32_t cycle_of(uint64_t t) const {
    return (uint32_t)(t >> log2_2n) & CYC_MASK;
  }
};

// Threshold reset value.  Algorithm 1 resets Threshold to 3n - 1, which is
// 2n (the most tickets that can separate Head from a newly installed entry)
// plus n - 1 concurrent dequeuers that may still fail after the reset; that
// accounting assumes at most n lanes use the queue (the configuration of
// Lemma 4, k <= n).  With k lanes the same accounting gives 2n + k - 1, so
// the value used is 2n + max(n, k) - 1, equal to 3n - 1 whenever k <= n.
__host__ __device__ __forceinline__ int64_t threshold_reset(const gq_dev& q) {
  const int64_t n = (int64_t)q.capacity;
  const int64_t k = (int64_t)q.max_threads;
  return 2 * n + (k > n ? k : n) - 1;
}

__device__ __forceinline__ Ring make_ring(const gq_ring_view& v, const gq_dev& q) {
  Ring r;
  r.slots = v.slots;
  r.head = v.head;
  r.tail = v.tail;
  r.thr = v.threshold;
  r.hint = v.hint;
  r.log2_2n = q.log2_cap + 1;
  r.log2_L = r.log2_2n < 4 ? r.log2_2n : 4;
  r.mode = q.slot_mode;
  r.thr_reset = threshold_reset(q);
  return r;
}

// Move Tail forward to at least `target` (Algorithm 1 "catch up Tail").  The
// CAS only ever raises Tail: it is attempted while the Tail it last read is
// below the target, and a failed CAS returns the newer Tail.  (A CAS from a
// freshly read Tail to a target below it would move Tail backward and hand a
// used ticket to a later enqueuer.)
__device__ __forceinline__ void catchup(const Ring& r, uint64_t target) {
  uint64_t t = ld(r.tail);
  for (uint32_t spin = 0; t < target && spin < SPIN_LIMIT; spin++)
    if (cas(r.tail, t, target)) break;
}

// Inner enqueue of index `idx` (Algorithm 1, TryEnq, retried until success).
// RELEASE makes the install CAS an agent-scope release (fenced hand-off).  An
// index ring never holds more than n indices in 2n slots, so the retry loop
// ends (lock-freedom, Section III-B).  Returns false only when the fail-safe
// bound (spin_out) stopped it: the index was not installed.
// `first`: a Tail ticket already reserved for this operation (workgroup
// aggregation), used for the first attempt; GROUP_NONE to take one here.
template <bool RELEASE>
__device__ __forceinline__ bool ring_enq(const Ring& r, uint32_t idx, uint32_t& cas_fail,
                                         uint64_t* err, uint64_t first = GROUP_NONE) {
  bool done = false;
  for (uint32_t spin = 0; !done; spin++) {
    if (spin_out(spin, err)) {
      latch_error(err, (uint64_t)(-GQ_ERR_DEVICE));
      return false;  // the index is lost: the caller reports the drop
    }
    uint64_t t;
    if (first != GROUP_NONE) {
      t = first;
      first = GROUP_NONE;
    } else {
      t = wave_faa(r.tail, 1);
    }
    const uint32_t c = r.cycle_of(t);
    uint64_t* p = r.at(r.slot_of(t));
    uint64_t e = ld(p);
    while (true) {
      if (older(e_cyc(e), c) && (e_safe(e) || ld(r.head) <= t) && idx_free(e_idx(e))) {
        const uint64_t ne = e_make(c, true, idx);
        const bool ok = RELEASE ? cas_rel(p, e, ne) : cas(p, e, ne);
        if (ok) {
          if (ld(r.thr) != r.thr_reset) st(r.thr, r.thr_reset);
          done = true;
          break;
        }
        cas_fail++;
        continue;  // re-test the entry the CAS returned, same ticket
      }
      break;  // this ticket is unusable: take a new one
    }
  }
  return true;
}

// poll_avail (common.h) is the empty pre-check of ring_deq: when fewer
// entries than polling lanes are available, only that many lanes of a
// wavefront take tickets; the others look again instead of taking tickets
// past Tail, each of which would mark a slot and make Tail catch up.

// Inner dequeue (Algorithm 1, TryDeq, retried until an index or EMPTY).
// Returns the index, BOT for EMPTY, or GAVE_UP when the fail-safe bound
// stopped it (error latched).  ACQUIRE makes Consume an agent-scope
// acquire (fenced hand-off).  Consume is an atomic XOR that turns
// the index field into BOTC and leaves Cycle/Safe alone; between install and
// consume only Safe can change, so the XOR is exact.
//
// `first`: a Head ticket already reserved for this operation (workgroup
// aggregation; the caller checked Threshold before reserving it).  It is
// always used: a Head ticket that no dequeuer visits could let an enqueuer
// install behind Head, where no later ticket reaches the item.
// `lane`: the caller's lane id below max_threads, or NO_LANE.  A lane whose
// last dequeue here answered EMPTY through the look below keeps looking
// before it takes a ticket, even after an install has reset Threshold (one
// byte per lane, cleared when the lane takes a ticket): without it, every
// polling lane takes a ticket at each install, and all but one of them mark
// a slot and send Tail after them.
template <bool ACQUIRE>
__device__ __forceinline__ uint32_t ring_deq(const Ring& r, uint32_t& cas_fail, uint64_t* err,
                                             uint64_t first = GROUP_NONE,
                                             uint32_t lane = NO_LANE) {
  for (uint32_t spin = 0;; spin++) {
    if (spin_out(spin, err)) {
      latch_error(err, (uint64_t)(-GQ_ERR_DEVICE));
      return GAVE_UP;
    }
    uint64_t h;
    if (first != GROUP_NONE) {
      h = first;
      first = GROUP_NONE;
    } else {
      const int64_t th = ld(r.thr);
      if (th < 0) return BOT;
      // Threshold below its reset value: a dequeue failed since the last
      // install, so the queue may be nearly empty -- look before taking a
      // ticket.  (On a queue that keeps items, the look would only add two
      // loads on the hottest lines.)
      const bool hinted = lane != NO_LANE && r.hint && r.hint[lane] != 0;
      if (th < r.thr_reset || hinted) {
        // Bounded grab: with a entries between Head and Tail, the wavefront
        // takes at most a tickets (its other lanes look again).  A full
        // wavefront takes them with one CAS that moves Head from the value
        // it read, so no ticket of the grab lies past Tail: with thousands
        // of polling lanes, FAA tickets taken on the seen entries overshoot
        // Tail by all but one wavefront's share, and each overshooting
        // ticket marks a slot an enqueuer is about to use.  A partial
        // wavefront takes FAA tickets: its overshoot is at most its few
        // lanes, while hundreds of such wavefronts racing one CAS each would
        // win one per round trip.  A lost CAS looks again.
        const uint64_t hh = read_first_lane(ld(r.head));
        keep(hh);
        wait_mem();
        const uint64_t tt = read_first_lane(ld(r.tail));
        const uint64_t avail = tt > hh ? tt - hh : 0;
        if (avail == 0) {
          if (lane != NO_LANE && r.hint && !hinted) r.hint[lane] = 1;
          return BOT;
        }
        const uint64_t mask = active_mask();
        const uint32_t rank = lane_rank(mask);
        const uint64_t act = (uint64_t)__popcll(mask);
        const uint64_t want = avail < act ? avail : act;
        if (act == 64) {
          uint64_t won = 0;
          if (rank == 0) {
            uint64_t e = hh;
            won = cas(r.head, e, hh + want) ? 1 : 0;
          }
          won = read_first_lane(won);
          if (!won || rank >= want) {
            pause(1);
            continue;
          }
          if (hinted) r.hint[lane] = 0;  // the lane takes a ticket
          h = hh + rank;
        } else {
          if (rank >= want) {
            pause(1);
            continue;
          }
          if (hinted) r.hint[lane] = 0;
          h = wave_faa(r.head, 1);
        }
      } else {
        h = wave_faa(r.head, 1);
      }
    }
    const uint32_t c = r.cycle_of(h);
    uint64_t* p = r.at(r.slot_of(h));
    uint64_t e = ld(p);
    // The entry is still from an older cycle but Tail shows ticket h handed
    // to an enqueuer, whose install follows its Tail increment closely: look
    // at the entry a bounded number of times before marking it, rather than
    // spoil that enqueuer's attempt (with many dequeuers polling a nearly
    // empty queue, marking sends producer after producer back for a new
    // ticket).  The wait is bounded, so the operation stays lock-free.
    if (older(e_cyc(e), c) && idx_free(e_idx(e)) && ld(r.tail) > h) {
      for (uint32_t w = 0; w < DEQ_WAIT_POLLS && older(e_cyc(e), c) && idx_free(e_idx(e)); w++) {
        pause(1);
        e = ld(p);
      }
    }
    while (true) {
      if (e_cyc(e) == c && !idx_free(e_idx(e))) {
        const uint64_t x = (uint64_t)(e_idx(e) ^ BOTC);
        if (ACQUIRE) fxor_acq(p, x); else fxor(p, x);
        return e_idx(e);
      }
      if (older(e_cyc(e), c)) {
        // the slot is stale for ticket h: mark it empty at cycle c, or, when
        // it still holds an older live index, clear Safe so no enqueuer with
        // an earlier ticket than Head installs behind it
        const uint64_t ne = idx_free(e_idx(e)) ? e_make(c, e_safe(e), BOT)
                                               : e_make(e_cyc(e), false, e_idx(e));
        if (!cas(p, e, ne)) {
          cas_fail++;
          continue;  // re-examine the returned entry
        }
      }
      break;
    }
    const uint64_t t = ld(r.tail);
    if (t <= h + 1) {
      // Every lane of the wavefront that is here catches Tail up to its h + 1
      // and decrements Threshold.  Catching up to the largest h + 1 among
      // them covers all of them, so one lane does it, and the decrements are
      // one aggregated add: with thousands of lanes finding the queue empty
      // together this avoids a storm of CAS retries on Tail.
      const uint64_t target = wave_max(h + 1);
      const uint64_t mask = active_mask();
      if (lane_rank(mask) == 0) {
        catchup(r, target);
        faa(r.thr, -(int64_t)__popcll(mask));
      }
      return BOT;
    }
    if (wave_fdec(r.thr) <= 0) return BOT;
  }
}

// ---- payload hand-off -----------------------------------------------------
// The enqueuer owning index idx writes data[idx]; the dequeuer that consumes
// idx reads it.  Default: the write is an agent-scope atomic exchange that has
// completed (wait_mem) before the install CAS is issued, and the read is an
// agent-scope atomic load issued after the consumer saw the installed entry,
// and completed before idx is returned to the free ring.  All three accesses
// are atomics on one cell ordered by those waits, so no L2 write-back or
// invalidate is needed.  With GQ_OPT_FENCED the hand-off instead uses plain
// accesses with an agent-scope release on the install and an acquire on the
// consume (Section III's ordering, at the cost of cache maintenance).
template <bool FENCED>
__device__ __forceinline__ void payload_put(const gq_dev& q, uint32_t idx, uint64_t item) {
  if (FENCED) {
    if (q.item_width == 8) ((uint64_t*)q.data)[idx] = item;
    else ((uint32_t*)q.data)[idx] = (uint32_t)item;
  } else {
    if (q.item_width == 8) keep(xchg((uint64_t*)q.data + idx, item));
    else keep(xchg((uint32_t*)q.data + idx, (uint32_t)item));
    wait_mem();
  }
}

template <bool FENCED>
__device__ __forceinline__ uint64_t payload_get(const gq_dev& q, uint32_t idx) {
  uint64_t v;
  if (FENCED) {
    v = q.item_width == 8 ? ((const uint64_t*)q.data)[idx]
                          : (uint64_t)((const uint32_t*)q.data)[idx];
  } else {
    v = q.item_width == 8 ? ld((const uint64_t*)q.data + idx)
                          : (uint64_t)ld((const uint32_t*)q.data + idx);
    keep(v);
    wait_mem();  // the read completes before idx goes back to the free ring
  }
  return v;
}

// ---- outer queue (Section III-B: indices move through aq/fq) -------------
// enqueue: idx <- fq.deq (EMPTY means FULL); data[idx] <- x; aq.enq(idx).
// dequeue: idx <- aq.deq (EMPTY means EMPTY); x <- data[idx]; fq.enq(idx).
// A fail-safe stop of the second inner operation (ring_enq gave up, error
// latched) loses the index: an enqueue then reports GQ_ERR_DEVICE (its item
// is lost with the index); a dequeue keeps its item (it was read before) and
// reports GQ_OK, the lost free index shrinking the queue.  Both count one
// drop.
__device__ __forceinline__ void count_drop(const gq_dev& q) { faa(q.stats + S_DROP, 1ull); }

template <bool FENCED>
__device__ __forceinline__ int enqueue_impl(const gq_dev& q, uint64_t item, uint32_t& cas_fail,
                                            uint32_t lane) {
  const Ring fq = make_ring(q.fq, q);
  const Ring aq = make_ring(q.aq, q);
  // The payload write below depends on idx, and the previous holder of idx
  // finished reading the cell before releasing idx into fq: no acquire needed.
  const uint32_t idx = ring_deq<false>(fq, cas_fail, q.err, GROUP_NONE, lane);
  if (idx == BOT) return GQ_FULL;
  if (idx >= q.capacity) {  // GAVE_UP; guards the payload array
    latch_error(q.err, (uint64_t)(-GQ_ERR_DEVICE));
    count_drop(q);
    return GQ_ERR_DEVICE;
  }
  payload_put<FENCED>(q, idx, item);
  if (!ring_enq<FENCED>(aq, idx, cas_fail, q.err)) {
    count_drop(q);
    return GQ_ERR_DEVICE;
  }
  return GQ_OK;
}

template <bool FENCED>
__device__ __forceinline__ int dequeue_impl(const gq_dev& q, uint64_t* item, uint32_t& cas_fail,
                                            uint32_t lane) {
  const Ring aq = make_ring(q.aq, q);
  const Ring fq = make_ring(q.fq, q);
  const uint32_t idx = ring_deq<FENCED>(aq, cas_fail, q.err, GROUP_NONE, lane);
  if (idx == BOT) return GQ_EMPTY;
  if (idx >= q.capacity) {  // GAVE_UP; guards the payload array
    latch_error(q.err, (uint64_t)(-GQ_ERR_DEVICE));
    count_drop(q);
    return GQ_ERR_DEVICE;
  }
  *item = payload_get<FENCED>(q, idx);
  if (!ring_enq<FENCED>(fq, idx, cas_fail, q.err)) count_drop(q);
  return GQ_OK;
}

// ---- workgroup-uniform form ----------------------------------------------
// Every thread of the workgroup calls group_op together, each with its own
// role (enqueue `item`, dequeue into `item`, or nothing).  The first ticket of
// each inner operation comes from one FAA per counter per workgroup
// (group_ticket); retries take WaveFAA tickets as usual.  Phase A takes an
// index (fq.Head for enqueues, aq.Head for dequeues), phase B passes it on
// (aq.Tail for enqueues, fq.Tail for dequeues).  Returns the lane's status
// (GQ_OK for ROLE_NONE).
template <bool FENCED>
__device__ __forceinline__ int group_op_impl(const gq_dev& q, int role, uint64_t& item,
                                             uint32_t& cas_fail, GroupLds& s, uint32_t& par,
                                             uint32_t lane) {
  const Ring fq = make_ring(q.fq, q);
  const Ring aq = make_ring(q.aq, q);
  // The Threshold test of a dequeue precedes its ticket, as in ring_deq.
  const bool wf = role == ROLE_ENQ && ld(fq.thr) >= 0;
  const bool wa = role == ROLE_DEQ && ld(aq.thr) >= 0;
  uint64_t t = group_ticket(s, par, fq.head, 1, wf, aq.head, 1, wa);
  uint32_t idx = BOT;
  if (wf) idx = ring_deq<false>(fq, cas_fail, q.err, t, lane);
  else if (wa) idx = ring_deq<FENCED>(aq, cas_fail, q.err, t, lane);
  int st = role == ROLE_ENQ ? GQ_FULL : role == ROLE_DEQ ? GQ_EMPTY : GQ_OK;
  if (idx != BOT && idx >= q.capacity) {  // GAVE_UP; guards the payload array
    latch_error(q.err, (uint64_t)(-GQ_ERR_DEVICE));
    count_drop(q);
    idx = BOT;
    st = GQ_ERR_DEVICE;
  }
  if (idx != BOT) {
    if (role == ROLE_ENQ) payload_put<FENCED>(q, idx, item);
    else item = payload_get<FENCED>(q, idx);
    st = GQ_OK;
  }
  const bool we = role == ROLE_ENQ && idx != BOT;
  const bool wd = role == ROLE_DEQ && idx != BOT;
  t = group_ticket(s, par, aq.tail, 1, we, fq.tail, 1, wd);
  bool placed = true;
  if (we) placed = ring_enq<FENCED>(aq, idx, cas_fail, q.err, t);
  else if (wd) placed = ring_enq<FENCED>(fq, idx, cas_fail, q.err, t);
  if (!placed) {
    count_drop(q);
    if (we) st = GQ_ERR_DEVICE;
  }
  return st;
}

// `lane`: the caller's lane id, if it is below max_threads (its empty hints,
// see ring_deq), else NO_LANE.
__device__ __forceinline__ int group_op(const gq_dev& q, int role, uint64_t& item,
                                        uint32_t& cas_fail, GroupLds& s, uint32_t& par,
                                        uint32_t lane = NO_LANE) {
  return (q.flags & GQ_OPT_FENCED) ? group_op_impl<true>(q, role, item, cas_fail, s, par, lane)
                                   : group_op_impl<false>(q, role, item, cas_fail, s, par, lane);
}

__device__ __forceinline__ int enqueue(const gq_dev& q, uint64_t item, uint32_t& cas_fail,
                                       uint32_t lane = NO_LANE) {
  return (q.flags & GQ_OPT_FENCED) ? enqueue_impl<true>(q, item, cas_fail, lane)
                                   : enqueue_impl<false>(q, item, cas_fail, lane);
}

__device__ __forceinline__ int dequeue(const gq_dev& q, uint64_t* item, uint32_t& cas_fail,
                                       uint32_t lane = NO_LANE) {
  return (q.flags & GQ_OPT_FENCED) ? dequeue_impl<true>(q, item, cas_fail, lane)
                                   : dequeue_impl<false>(q, item, cas_fail, lane);
}

}  // namespace lfq
}  // namespace gq
