// G-WFQ-YMC: the Yang / Mellor-Crummey wait-free queue adapted to the GPU
// (Section III-A).
//
// An unbounded array of cells {val, enq, deq} indexed by two monotone
// counters T and H.  Fast path: an enqueue takes a cell with FAA(T) and CASes
// its value in; a dequeue takes a cell with FAA(H) and claims the value there.
// After `patience` failures an operation publishes a per-lane request that
// other lanes complete: dequeuers help pending enqueue requests of peers on
// the cells they visit, and every successful dequeue helps one peer's pending
// dequeue request.  The queue logic, helping structure and linearization
// points follow the original algorithm.
//
// GPU adaptation (Section III-A): the linked segments and their hazard-
// pointer reclamation are replaced by one preallocated pool with direct
// arithmetic lookup; running past the pool latches GQ_ERR_POOL_EXHAUSTED.
// The pool is a structure of arrays -- val[P], enq[P], deq[P] -- so cell i's
// words are val + i, enq + i and deq + i: the consecutive cells that one
// ticket FAA hands to a wavefront (or workgroup) sit in consecutive words, and
// their atomics coalesce into a few lines instead of one sector per lane.  Request "pointers" in cells are lane ids + 1 (0 is
// the empty marker, all ones the taken marker); request states pack
// <pending:1 | id:63> into one 64-bit word.  Tickets come from the wave-
// aggregated fetch-and-add, which yields the same ticket order as per-lane
// FAA (Lemma 1).
//
// Values: a cell stores item + 1, so 0 can mark an empty cell, all ones an
// unusable one and all ones - 1 the internal "empty" result; 8-byte queues
// therefore reject the items 2^64 - 3 .. 2^64 - 1 (GQ_ERR_INVALID).
// G-WFQ-YMC is unbounded within its pool and never answers FULL.
#pragma once
#include "common.h"

namespace gq {
namespace ymc {

constexpr uint64_t BOT = 0;               // empty cell value / no request
constexpr uint64_t TOP = ~0ull;           // unusable cell value / taken
constexpr uint64_t PENDING = 1ull << 63;
constexpr uint64_t ID_MASK = PENDING - 1;
constexpr uint64_t RES_EMPTY = TOP - 1;   // internal: "queue was empty"
// A helping walk over cells that is still undecided after this many ticks of
// the 100 MHz clock latches GQ_ERR_DEVICE and stops (fail-safe; the walk is
// bounded, see help_deq).
constexpr uint64_t WALK_LIMIT_TICKS = 1000000000ull;  // 10 s

// Addresses of one cell's three words.
struct Cell {
  uint64_t* val;
  uint64_t* enq;  // 0, lane + 1 of the enqueue request reserved here, or TOP
  uint64_t* deq;  // 0, lane + 1 of the dequeue request served here, or TOP
};
constexpr uint32_t CELL_WORDS = 3;  // pool bytes = 24 per cell

struct Handle {          // one per lane, 64 bytes
  uint64_t enq_val;      // enqueue request: value (stored form)
  uint64_t enq_state;    // <pending | id>: id = first cell tried, then the claimed cell
  uint64_t deq_id;       // dequeue request: id = first cell tried
  uint64_t deq_state;    // <pending | idx>: idx = announced candidate cell
  uint64_t enq_help_id;  // private: remembered id of the enqueue request being helped
  uint32_t enq_peer;     // private: next lane whose enqueue request to look at
  uint32_t deq_peer;     // private: next lane whose dequeue request to help
  uint64_t pad[3];
};

struct Q {
  uint64_t* pool;   // val[cells], then enq[cells], then deq[cells]
  uint64_t cells;
  uint64_t* T;
  uint64_t* H;
  Handle* hd;
  uint8_t* hint;    // per lane: its last dequeue answered EMPTY (a wavefront's 64 share a line)
  uint32_t k;
  uint32_t patience_enq, patience_deq;
  uint64_t* err;
  uint64_t* stats;
};

__device__ __forceinline__ Q make_q(const gq_dev& q) {
  Q y;
  y.pool = q.ymc_cells;
  y.cells = q.ymc_pool_cells;
  y.T = q.ymc_ctr;
  y.H = q.ymc_ctr + 32;
  y.hd = (Handle*)q.ymc_handles;
  y.hint = q.ymc_hint;
  y.k = q.max_threads;
  y.patience_enq = q.patience_enq;
  y.patience_deq = q.patience_deq;
  y.err = q.err;
  y.stats = q.stats;
  return y;
}

// Cell lookup into the preallocated pool; false (and a latched error) when the
// pool is exhausted.
__device__ __forceinline__ bool cell(const Q& y, uint64_t i, Cell& c) {
  if (i >= y.cells) {
    latch_error(y.err, (uint64_t)(-GQ_ERR_POOL_EXHAUSTED));
    return false;
  }
  c.val = y.pool + i;
  c.enq = y.pool + y.cells + i;
  c.deq = y.pool + 2 * y.cells + i;
  return true;
}

__device__ __forceinline__ void advance_end(uint64_t* E, uint64_t v) {
  uint64_t e = ld(E);
  while (e < v)
    if (cas(E, e, v)) break;
}

__device__ __forceinline__ bool try_claim(uint64_t* state, uint64_t id, uint64_t cell_id) {
  uint64_t e = PENDING | id;
  return cas_acqrel(state, e, cell_id);
}

__device__ __forceinline__ void enq_commit(const Q& y, const Cell& c, uint64_t v, uint64_t cid) {
  advance_end(y.T, cid + 1);
  st(c.val, v);
}

// help_enq: make cell i decided for dequeuers.  Returns the cell's value, TOP
// (no value will come to this cell), or RES_EMPTY (the queue was empty).
// The cell's own words carry the value, so the cell CASes of the fast paths
// are relaxed; request records (value, then state) are published with
// release and read with acquire.
__device__ __forceinline__ uint64_t help_enq(const Q& y, Handle* h, const Cell& c, uint64_t i) {
  // Look first: a value already in the cell is what the CAS below would
  // return on failure, and the look is a load instead of a read-modify-write.
  uint64_t e = ld(c.val);
  if (e != BOT && e != TOP) return e;
  if (e == BOT && !cas(c.val, e, TOP) && e != TOP) return e;
  // the cell holds TOP: help a pending slow-path enqueue use this cell
  if (ld_acq(c.enq) == BOT) {
    uint32_t p = 0;
    uint64_t s = 0;
    for (uint32_t spin = 0;; spin++) {
      p = h->enq_peer;
      if (p >= y.k) p = 0;
      s = ld_acq(&y.hd[p].enq_state);
      if (h->enq_help_id == 0 || h->enq_help_id == (s & ID_MASK) || spin >= y.k) break;
      h->enq_help_id = 0;
      h->enq_peer = p + 1 >= y.k ? 0 : p + 1;
    }
    uint64_t ee = BOT;
    if ((s & PENDING) && (s & ID_MASK) <= i && !cas_acqrel(c.enq, ee, (uint64_t)p + 1)) {
      h->enq_help_id = s & ID_MASK;  // could not reserve: retry this request next time
    } else {
      h->enq_peer = p + 1 >= y.k ? 0 : p + 1;
    }
    ee = BOT;
    if (ld_acq(c.enq) == BOT) cas_acqrel(c.enq, ee, TOP);
  }
  const uint64_t ce = ld_acq(c.enq);
  if (ce == TOP) return ld(y.T) <= i ? RES_EMPTY : TOP;
  Handle* r = &y.hd[ce - 1];
  const uint64_t s = ld_acq(&r->enq_state);
  const uint64_t v = ld_acq(&r->enq_val);
  if ((s & PENDING) && (s & ID_MASK) > i) {
    // a pending request that started after this cell cannot use it
    if (ld(c.val) == TOP && ld(y.T) <= i) return RES_EMPTY;
  } else {
    // Claim the pending request for cell i.  A failed claim leaves the state
    // it met in cur: if that is a claim for cell i (made by the request's
    // owner or another helper, whose value store may still be on its way),
    // the value is stored here too, so this dequeuer does not leave cell i
    // for a value that lands after it moved on.
    uint64_t cur = s;
    const bool claimed = (s & PENDING) && cas_acqrel(&r->enq_state, cur, i);
    if (claimed || (cur == i && ld(c.val) == TOP)) enq_commit(y, c, v, i);
  }
  return ld_acq(c.val);
}

// ---- enqueue -------------------------------------------------------------------
// `first`: a T ticket already reserved for this attempt (workgroup
// aggregation), or GROUP_NONE.  Returns ENQ_DONE when v is in cell `first`
// (or the next T cell), ENQ_RETRY when that cell was lost to a dequeuer (id
// = the cell), ENQ_NO_POOL when the pool is exhausted (error latched).
enum EnqFast { ENQ_RETRY = 0, ENQ_DONE = 1, ENQ_NO_POOL = 2 };
__device__ __forceinline__ int enq_fast(const Q& y, uint64_t v, uint64_t& id,
                                        uint64_t first = GROUP_NONE) {
  const uint64_t i = first != GROUP_NONE ? first : wave_faa(y.T, 1);
  Cell c;
  if (!cell(y, i, c)) return ENQ_NO_POOL;
  uint64_t e = BOT;
  if (cas(c.val, e, v)) return ENQ_DONE;
  id = i;
  return ENQ_RETRY;
}

// Returns false when the request was abandoned (pool exhausted or a
// fail-safe bound, error latched): the item may be lost.
__device__ __forceinline__ bool enq_slow(const Q& y, uint32_t tid, uint64_t v, uint64_t cell_id) {
  Handle* me = &y.hd[tid];
  st(&me->enq_val, v);
  st_rel(&me->enq_state, PENDING | cell_id);
  for (uint32_t spin = 0;; spin++) {
    if (spin_out(spin, y.err)) { latch_error(y.err, (uint64_t)(-GQ_ERR_DEVICE)); return false; }
    const uint64_t i = wave_faa(y.T, 1);
    Cell c;
    if (!cell(y, i, c)) return false;
    uint64_t e = BOT;
    if (cas_acqrel(c.enq, e, (uint64_t)tid + 1) && ld(c.val) == BOT) {
      try_claim(&me->enq_state, cell_id, i);
      break;
    }
    if (!(ld_acq(&me->enq_state) & PENDING)) break;
  }
  const uint64_t id = ld_acq(&me->enq_state) & ID_MASK;
  Cell c;
  if (!cell(y, id, c)) return false;
  enq_commit(y, c, v, id);
  return true;
}

__device__ __forceinline__ bool enq_valid(const gq_dev& q, uint64_t item, uint32_t tid) {
  return tid < q.max_threads && !(q.item_width == 8 && item >= RES_EMPTY - 1);
}

__device__ __forceinline__ int enqueue_impl(const Q& y, const gq_dev& q, uint64_t item,
                                            uint32_t tid, uint32_t& cf, uint64_t first) {
  const uint64_t v = (q.item_width == 8 ? item : (item & 0xFFFFFFFFull)) + 1;
  uint64_t id = 0;
  // At least one fast attempt: the slow path starts from the cell that
  // attempt took (patience 0 means "one attempt, then the slow path").
  const uint32_t pat = y.patience_enq ? y.patience_enq : 1;
  for (uint32_t p = 0; p < pat; p++) {
    const int r = enq_fast(y, v, id, p == 0 ? first : GROUP_NONE);
    if (r == ENQ_DONE) return GQ_OK;  // the value is in its cell
    if (r == ENQ_NO_POOL) return GQ_ERR_POOL_EXHAUSTED;
    cf++;
  }
  faa(y.stats + S_SLOW, 1ull);
  if (!enq_slow(y, tid, v, id)) {
    faa(y.stats + S_DROP, 1ull);
    return ld(y.err) == (uint64_t)(-GQ_ERR_POOL_EXHAUSTED) ? GQ_ERR_POOL_EXHAUSTED : GQ_ERR_DEVICE;
  }
  return GQ_OK;
}

__device__ __forceinline__ int enqueue(const gq_dev& q, uint64_t item, uint32_t tid, uint32_t& cf) {
  if (!enq_valid(q, item, tid)) {
    latch_error(q.err, (uint64_t)(-GQ_ERR_INVALID));
    return GQ_ERR_INVALID;
  }
  return enqueue_impl(make_q(q), q, item, tid, cf, GROUP_NONE);
}

// ---- dequeue -------------------------------------------------------------------
// A relaxed look at the helpee's state comes first: with no request pending
// (the common case) helping costs one load and no cache invalidation; a
// request published after the look is helped on a later visit.
//
// The candidate walk.  In the original algorithm a helper visits the cells
// after the request's id one by one until it finds one whose value is still
// unclaimed, or one that shows the queue empty.  On the GPU that walk can be
// as long as the run: with tens of thousands of lanes taking H tickets, every
// cell the walker reaches has already been claimed by the dequeuer holding
// its ticket, and a walker visits one cell per few atomics while H advances
// by thousands.  Every cell below H, however, already belongs to a dequeuer
// that took its ticket (or was decided by an earlier request's walk before
// H was moved past it), and that dequeuer decides the cell itself: the
// walker may start from H instead, as if it had arrived after those
// dequeuers.  Cells at or above H are visited one by one as before, so a
// value is never skipped and an EMPTY candidate still means T <= i.  The walk
// is thus bounded by the race for the few cells at H, and a fail-safe bound
// (iterations, time, a latched error) ends it in any case.  Returns false
// when that fail-safe stopped it.
__device__ bool help_deq(const Q& y, Handle* h, uint32_t helpee) {
  Handle* r = &y.hd[helpee];
  if (!(ld(&r->deq_state) & PENDING)) return true;
  uint64_t s = ld_acq(&r->deq_state);
  const uint64_t id = ld_acq(&r->deq_id);
  if (!(s & PENDING) || (s & ID_MASK) < id) return true;
  const uint64_t deadline = stamp() + WALK_LIMIT_TICKS;
  uint64_t prior = id, i = id, cand = 0;
  uint32_t steps = 0;  // one bound for both loops
  for (;;) {
    // look for a candidate cell until one is found or another helper announces one
    while (!cand && (s & ID_MASK) == prior) {
      if (spin_out(steps++, y.err) || ((steps & 255) == 0 && stamp() > deadline)) {
        latch_error(y.err, (uint64_t)(-GQ_ERR_DEVICE));
        return false;
      }
      const uint64_t hn = ld(y.H);
      if (hn > i + 1) i = hn - 1;  // cells below H belong to their ticket holders
      Cell c;
      if (!cell(y, ++i, c)) return false;
      const uint64_t v = help_enq(y, h, c, i);
      if (v == RES_EMPTY || (v != TOP && ld_acq(c.deq) == BOT)) cand = i;
      else s = ld_acq(&r->deq_state);
    }
    if (spin_out(steps++, y.err)) {
      latch_error(y.err, (uint64_t)(-GQ_ERR_DEVICE));
      return false;
    }
    if (cand) {
      uint64_t e = PENDING | prior;
      cas_acqrel(&r->deq_state, e, PENDING | cand);
      s = ld_acq(&r->deq_state);
    }
    if (!(s & PENDING) || ld_acq(&r->deq_id) != id) return true;
    Cell c;
    if (!cell(y, s & ID_MASK, c)) return false;
    uint64_t d = BOT;
    if (ld_acq(c.val) == TOP || cas_acqrel(c.deq, d, (uint64_t)helpee + 1) ||
        d == (uint64_t)helpee + 1) {
      uint64_t e = s;
      cas_acqrel(&r->deq_state, e, s & ID_MASK);
      return true;
    }
    prior = s & ID_MASK;
    if ((s & ID_MASK) >= i) {
      cand = 0;
      i = s & ID_MASK;
    }
  }
}

// deq_fast: returns a stored value, RES_EMPTY, or TOP (try again / go slow).
// `t`: the H ticket of this attempt.
__device__ __forceinline__ uint64_t deq_fast(const Q& y, Handle* h, uint64_t& id, uint64_t t) {
  const uint64_t i = t;
  Cell c;
  if (!cell(y, i, c)) return RES_EMPTY;
  const uint64_t v = help_enq(y, h, c, i);
  if (v == RES_EMPTY) return RES_EMPTY;
  uint64_t d = BOT;
  if (v != TOP && cas(c.deq, d, TOP)) return v;
  id = i;
  return TOP;
}

// Slow-path dequeue.  Sets `ok` to false when the request could not be
// completed (fail-safe stop or pool exhausted, error latched).
__device__ __forceinline__ uint64_t deq_slow(const Q& y, uint32_t tid, uint64_t cid, bool& ok) {
  Handle* me = &y.hd[tid];
  st(&me->deq_id, cid);
  st_rel(&me->deq_state, PENDING | cid);
  help_deq(y, me, tid);
  const uint64_t s = ld_acq(&me->deq_state);
  if (s & PENDING) {  // the walk was stopped before the request was decided
    ok = false;
    return RES_EMPTY;
  }
  const uint64_t i = s & ID_MASK;
  Cell c;
  if (!cell(y, i, c)) {
    ok = false;
    return RES_EMPTY;
  }
  const uint64_t v = ld_acq(c.val);
  advance_end(y.H, i + 1);
  return v == TOP ? RES_EMPTY : v;
}

// Ticket grab of a dequeue that looks before it takes a ticket (the lane's
// last dequeue here answered EMPTY).  The first active lane reads H, waits for
// it, then reads T.  With T <= H every value in the pool sits in a cell below
// H, whose dequeuer already holds its ticket (or whose request walk already
// decided it): those dequeues can be linearized just before the T read, and
// the queue is empty there -- EMPTY without a ticket for every lane here
// (the same argument as the ring queues' empty pre-check).  Otherwise it moves
// H forward by at most T - H with a CAS, so that polling dequeuers never take
// cells beyond T: each cell taken by a dequeue that then finds nothing is a
// pool cell used up (the pool is not recycled), and polling through
// fetch-and-adds would use up one per poll.  After a failed CAS, T is read
// again after the new H has returned.  Lanes beyond the tickets won look
// again.  Returns the lane's ticket, GROUP_NONE for EMPTY or LOOK_AGAIN.
constexpr uint64_t LOOK_AGAIN = GROUP_NONE - 1;

__device__ __forceinline__ uint64_t grab_below_tail(const Q& y) {
  const uint64_t mask = active_mask();
  const uint32_t rank = lane_rank(mask);
  const uint64_t want_all = (uint64_t)__popcll(mask);
  uint64_t base = 0, got = 0, empty = 0;
  if (rank == 0) {
    uint64_t h = ld(y.H);
    for (uint32_t spin = 0; !spin_out(spin, y.err); spin++) {
      keep(h);
      wait_mem();
      const uint64_t t = ld(y.T);
      if (t <= h) {
        empty = 1;
        break;
      }
      const uint64_t want = t - h < want_all ? t - h : want_all;
      if (cas(y.H, h, h + want)) {
        base = h;
        got = want;
        break;
      }
    }
  }
  base = read_first_lane(base);
  got = read_first_lane(got);
  empty = read_first_lane(empty);
  if (empty) return GROUP_NONE;
  if (rank < got) return base + rank;
  return LOOK_AGAIN;
}

// `first`: an H ticket already reserved for the first attempt (workgroup
// aggregation), or GROUP_NONE.
__device__ __forceinline__ int dequeue_impl(const Q& y, uint64_t* item, uint32_t tid,
                                            uint32_t& cf, uint64_t first) {
  Handle* me = &y.hd[tid];
  uint64_t v = TOP, id = 0;
  const bool looking = first == GROUP_NONE && y.hint[tid] != 0;
  // At least one fast attempt: every cell a dequeuer takes from H must be
  // visited, and the slow path walks forward from the cell of the last one.
  const uint32_t pat = y.patience_deq ? y.patience_deq : 1;
  for (uint32_t p = 0, spin = 0; p < pat;) {
    uint64_t t = p == 0 ? first : GROUP_NONE;
    if (t == GROUP_NONE) {
      if (looking) {
        t = grab_below_tail(y);
        if (t == GROUP_NONE) return ld(y.err) ? GQ_ERR_DEVICE : GQ_EMPTY;  // hint stays set
        if (t == LOOK_AGAIN) {
          if (spin_out(spin++, y.err)) {
            latch_error(y.err, (uint64_t)(-GQ_ERR_DEVICE));
            return GQ_ERR_DEVICE;
          }
          pause(1);
          continue;
        }
      } else {
        t = wave_faa(y.H, 1);
      }
    }
    v = deq_fast(y, me, id, t);
    if (v != TOP) break;
    cf++;
    p++;
  }
  bool ok = true;
  if (v == TOP) {
    faa(y.stats + S_SLOW, 1ull);
    v = deq_slow(y, tid, id, ok);
  }
  if (!ok) {
    faa(y.stats + S_DROP, 1ull);
    return ld(y.err) == (uint64_t)(-GQ_ERR_POOL_EXHAUSTED) ? GQ_ERR_POOL_EXHAUSTED : GQ_ERR_DEVICE;
  }
  if (v == RES_EMPTY) {
    if (ld(y.err)) return GQ_ERR_POOL_EXHAUSTED;
    if (!y.hint[tid]) y.hint[tid] = 1;
    return GQ_EMPTY;
  }
  if (y.hint[tid]) y.hint[tid] = 0;
  // a successful dequeue helps one peer's pending dequeue request
  uint32_t p = me->deq_peer;
  if (p >= y.k) p = 0;
  if (p != tid) help_deq(y, me, p);
  me->deq_peer = p + 1 >= y.k ? 0 : p + 1;
  *item = v - 1;
  return GQ_OK;
}

__device__ __forceinline__ int dequeue(const gq_dev& q, uint64_t* item, uint32_t tid, uint32_t& cf) {
  if (tid >= q.max_threads) {
    latch_error(q.err, (uint64_t)(-GQ_ERR_INVALID));
    return GQ_ERR_INVALID;
  }
  return dequeue_impl(make_q(q), item, tid, cf, GROUP_NONE);
}

// ---- workgroup-uniform form (see lfq::group_op): one phase, the T ticket
// of an enqueue or the H ticket of a dequeue comes from group_ticket.
__device__ __forceinline__ int group_op(const gq_dev& q, int role, uint64_t& item, uint32_t tid,
                                        uint32_t& cf, GroupLds& s, uint32_t& par) {
  const Q y = make_q(q);
  int st = GQ_OK;
  if ((role == ROLE_ENQ && !enq_valid(q, item, tid)) || (role == ROLE_DEQ && tid >= y.k)) {
    latch_error(q.err, (uint64_t)(-GQ_ERR_INVALID));
    st = GQ_ERR_INVALID;
    role = ROLE_NONE;
  }
  // a lane whose last dequeue found the queue empty looks before it takes a
  // ticket (dequeue_impl), so it takes no share of the group's H ticket
  const bool looking = role == ROLE_DEQ && y.hint[tid] != 0;
  const uint64_t t =
      group_ticket(s, par, y.T, 1, role == ROLE_ENQ, y.H, 1, role == ROLE_DEQ && !looking);
  if (role == ROLE_ENQ) st = enqueue_impl(y, q, item, tid, cf, t);
  else if (role == ROLE_DEQ) st = dequeue_impl(y, &item, tid, cf, looking ? GROUP_NONE : t);
  return st;
}

}  // namespace ymc
}  // namespace gq
