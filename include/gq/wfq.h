// G-WFQ: the bounded wait-free queue of Section III-C.
//
// Same 2n-slot rings and outer aq/fq queue as G-LFQ, plus a cooperative slow
// path: an operation that fails `patience` fast attempts publishes a request
// in its per-lane record, and helpers (every lane inspects one peer record
// every D operations) drive it to completion.  Every shared word is one 64-bit
// atomic (Lemma 3): slot entries, the global Head/Tail words and the per-lane
// local words.
//
// Words:
//   Entry  = <Note:15 | Cycle:15 | Safe:1 | Enq:1 | Index:32>   (bits 63..0)
//   Global = <Counter:44 | ThrIdx:20>  ThrIdx = 0 (NULL) or lane id + 1
//   Local  = <Tag:18 | Counter:44 | INC:1 | FIN:1>
// Cycle and Note are compared modulo R = 2^15 (Lemma 4; gq_create refuses
// configurations with R <= D*k/n + 6).  Tag is the request's sequence number:
// it lets helpers tell one request of a lane from the next.
//
// Slow path (Algorithm 2 and the text around it):
//   * the owner writes init/index, sets its Local word to <tag, init>, then
//     publishes <seq, enqueue, pending> with a release store;
//   * SlowFAA agrees on one ticket per round: a helper sets INC on the Local
//     word together with the counter c it read from the Global word (only
//     while ThrIdx is NULL), then races CAS(Global, <c, NULL>, <c+1, lane>);
//     exactly one CAS succeeds per round (Lemma 5); the Local word itself is
//     the phase-2 record: clearing INC commits ticket c, and ThrIdx is cleared
//     only after that;
//   * TryEnqSlow installs <c, Safe, Enq = 0, index> on the agreed ticket or
//     advances Note to c when the slot cannot be used (Lemma 6); the installer
//     then sets FIN and flips Enq to 1; a dequeuer meeting an Enq = 0 entry
//     first sets FIN on the owning request (found through a per-slot hint,
//     else by scanning the records) so no helper starts another round;
//   * TryDeqSlow finishes on the matching current-cycle entry or on an empty
//     decision (Tail <= H + 1, or Threshold < 0), recording FIN; the owner
//     then consumes the entry at its final ticket, if one is there.
#pragma once
#include "common.h"
#include "lfq.h"

namespace gq {
namespace wfq {

using lfq::BOT;
using lfq::BOTC;
using lfq::GAVE_UP;
using lfq::idx_free;

constexpr uint32_t TAG_BITS = 15;
constexpr uint32_t TAG_MASK = (1u << TAG_BITS) - 1u;
constexpr uint32_t TAG_HALF = 1u << (TAG_BITS - 1);
constexpr uint64_t ENQ_BIT = 1ull << 32;
constexpr uint64_t SAFE_BIT = 1ull << 33;
constexpr uint32_t CYC_SHIFT = 34;
constexpr uint32_t NOTE_SHIFT = 49;

constexpr uint32_t TID_BITS = 20;
constexpr uint64_t TID_MASK = (1ull << TID_BITS) - 1;
constexpr uint64_t UNIT = 1ull << TID_BITS;        // one ticket on the Global word
constexpr uint64_t CTR_MASK = (1ull << 44) - 1;   // 44-bit counters
constexpr uint64_t NO_TICKET = CTR_MASK;          // "no fast-path ticket taken"
constexpr uint64_t SLOW_GAVE_UP = CTR_MASK - 1;   // run_slow stopped by a fail-safe bound

constexpr uint64_t L_FIN = 1;
constexpr uint64_t L_INC = 2;
constexpr uint32_t L_TAG_SHIFT = 46;
constexpr uint64_t L_TAG_MASK = (1ull << 18) - 1;

// Looks a dequeuer takes at an entry whose enqueuer holds the ticket but has
// not installed yet (see try_deq).
constexpr uint32_t DEQ_WAIT_POLLS = 64;
constexpr uint32_t DEQ_WAIT_POLLS_SLOW = 2048;
constexpr uint64_t SLOW_LIMIT_TICKS = 1000000000ull;  // 10 s at 100 MHz

// ---- entry word ------------------------------------------------------------
__device__ __forceinline__ uint32_t e_idx(uint64_t e) { return (uint32_t)e; }
__device__ __forceinline__ bool e_enq(uint64_t e) { return (e & ENQ_BIT) != 0; }
__device__ __forceinline__ bool e_safe(uint64_t e) { return (e & SAFE_BIT) != 0; }
__device__ __forceinline__ uint32_t e_cyc(uint64_t e) { return (uint32_t)(e >> CYC_SHIFT) & TAG_MASK; }
__device__ __forceinline__ uint32_t e_note(uint64_t e) { return (uint32_t)(e >> NOTE_SHIFT) & TAG_MASK; }
__host__ __device__ __forceinline__ uint64_t e_make(uint32_t note, uint32_t cyc, bool safe, bool enq,
                                                    uint32_t idx) {
  return ((uint64_t)(note & TAG_MASK) << NOTE_SHIFT) | ((uint64_t)(cyc & TAG_MASK) << CYC_SHIFT) |
         (safe ? SAFE_BIT : 0) | (enq ? ENQ_BIT : 0) | idx;
}
// a strictly older than b: 0 < (b - a) mod R < R/2  (Lemma 4)
__device__ __forceinline__ bool older(uint32_t a, uint32_t b) {
  const uint32_t d = (b - a) & TAG_MASK;
  return d != 0 && d < TAG_HALF;
}

// ---- global and local words -------------------------------------------------
__device__ __forceinline__ uint64_t g_ctr(uint64_t g) { return g >> TID_BITS; }
__device__ __forceinline__ uint32_t g_thr(uint64_t g) { return (uint32_t)(g & TID_MASK); }
__device__ __forceinline__ uint64_t l_make(uint64_t tag, uint64_t ctr, bool inc, bool fin) {
  return ((tag & L_TAG_MASK) << L_TAG_SHIFT) | ((ctr & CTR_MASK) << 2) | (inc ? L_INC : 0) |
         (fin ? L_FIN : 0);
}
__device__ __forceinline__ uint64_t l_tag(uint64_t l) { return l >> L_TAG_SHIFT; }
__device__ __forceinline__ uint64_t l_ctr(uint64_t l) { return (l >> 2) & CTR_MASK; }
__device__ __forceinline__ bool l_inc(uint64_t l) { return (l & L_INC) != 0; }
__device__ __forceinline__ bool l_fin(uint64_t l) { return (l & L_FIN) != 0; }

// Per-lane request record, one per ring (64 bytes).
struct Rec {
  uint64_t local;     // Local word
  uint64_t init;      // initial ticket (the last failed fast-path ticket)
  uint64_t index;     // payload index of an enqueue request
  uint64_t req;       // <seq:62 | enqueue:1 | pending:1>, published last
  uint64_t next_seq;  // owner-private: sequence number of the next request
  uint64_t pad[3];
};

struct WRing {
  lfq::Ring g;        // slots / Head / Tail / Threshold / geometry
  Rec* rec;
  uint64_t* owner;    // per-slot hint <ticket:44 | lane + 1:20> of the last slow installer
  uint8_t* hint;      // per-lane byte: the lane's last dequeue here found the ring empty
  uint64_t* announce; // lane + 1 of the announced slow-path request, 0 if none
  uint32_t k;
  uint64_t* err;
  uint64_t* stats;

  __device__ __forceinline__ uint32_t cycle_of(uint64_t t) const {
    return (uint32_t)(t >> g.log2_2n) & TAG_MASK;
  }
  __device__ __forceinline__ uint64_t slot_of(uint64_t t) const { return g.slot_of(t); }
};

__device__ __forceinline__ WRing make_wring(const gq_ring_view& v, const gq_dev& q) {
  WRing r;
  r.g = lfq::make_ring(v, q);
  r.rec = (Rec*)v.records;
  r.owner = v.owner;
  r.hint = v.hint;
  r.announce = v.announce;
  r.k = q.max_threads;
  r.err = q.err;
  r.stats = q.stats;
  return r;
}

__device__ __forceinline__ uint64_t ticket(uint64_t word_after_rank) { return word_after_rank >> TID_BITS; }

__device__ __forceinline__ void reset_threshold(const WRing& r) {
  if (ld(r.g.thr) != r.g.thr_reset) st(r.g.thr, r.g.thr_reset);
}

// Move Tail's counter to at least `target`, keeping ThrIdx.
__device__ __forceinline__ void catchup(const WRing& r, uint64_t target) {
  uint64_t g = ld(r.g.tail);
  for (uint32_t spin = 0; g_ctr(g) < target; spin++) {
    if (spin_out(spin, r.err)) { latch_error(r.err, (uint64_t)(-GQ_ERR_DEVICE)); return; }
    if (cas(r.g.tail, g, (target << TID_BITS) | g_thr(g))) return;
  }
}

// ---- announced requests -------------------------------------------------------
// Every lane helps the one announced slow-path request of a ring before each
// fast-path attempt there (help_announced).  The announcement complements the
// every-D-operations peer visits of the help step: with tens of thousands of
// lanes a request would wait k*D operations for its turn, while the Global
// word's stream of fast-path fetch-and-adds keeps defeating its own
// compare-and-swap.  Helping the announced request stops that stream.
__device__ __forceinline__ bool try_announce(const WRing& r, uint32_t rid) {
  uint64_t z = 0;
  return ld(r.announce) == 0 && cas(r.announce, z, (uint64_t)rid + 1);
}

__device__ __forceinline__ void withdraw(const WRing& r, uint32_t rid) {
  uint64_t me = (uint64_t)rid + 1;
  cas(r.announce, me, 0ull);
}

// ---- finalization of slow-path enqueues ------------------------------------
// Set FIN on lane p's enqueue request if its committed ticket is h.
__device__ __forceinline__ bool try_fin(Rec* rec, uint32_t p, uint64_t h) {
  Rec* R = &rec[p];
  const uint64_t q1 = ld_acq(&R->req);
  if ((q1 & 3) != 3) return false;  // not a pending enqueue
  const uint64_t tag = (q1 >> 2) & L_TAG_MASK;
  uint64_t l = ld_acq(&R->local);
  for (uint32_t spin = 0; spin < 64; spin++) {
    if (l_tag(l) != tag || l_ctr(l) != h || l_inc(l)) return false;
    if (l_fin(l)) return true;
    if (cas_acqrel(&R->local, l, l | L_FIN)) return true;
  }
  return false;
}

// A dequeuer found an Enq = 0 entry for its ticket h: the slow enqueue that
// installed it may not have set FIN yet.  Set it before consuming, so that no
// helper of that request starts another round after the slot is reused.
// It takes the ring's fields as scalars: a reference to the ring would make
// the caller keep its ring descriptors in private memory on every operation.
__device__ __noinline__ void finalize_enq(Rec* rec, const uint64_t* owner, uint32_t k,
                                          uint64_t* stats, uint64_t h, uint64_t j) {
  const uint64_t o = ld(&owner[j]);
  if ((o >> TID_BITS) == (h & CTR_MASK) && (o & TID_MASK) && (o & TID_MASK) <= k) {
    if (try_fin(rec, (uint32_t)(o & TID_MASK) - 1, h)) return;
  }
  faa(stats + S_SCAN, 1ull);
  for (uint32_t p = 0; p < k; p++)
    if (try_fin(rec, p, h)) return;
}

// ---- fast path (the G-LFQ fast path on this entry layout) -------------------
template <bool RELEASE>
__device__ __forceinline__ bool try_enq(const WRing& r, uint64_t t, uint32_t idx, uint32_t& cf) {
  const uint32_t c = r.cycle_of(t);
  uint64_t* p = r.g.at(r.slot_of(t));
  uint64_t e = ld(p);
  while (true) {
    if (older(e_cyc(e), c) && (e_safe(e) || g_ctr(ld(r.g.head)) <= t) && idx_free(e_idx(e))) {
      const uint64_t ne = e_make(e_note(e), c, true, true, idx);
      if (RELEASE ? cas_rel(p, e, ne) : cas(p, e, ne)) {
        reset_threshold(r);
        return true;
      }
      cf++;
      continue;
    }
    return false;
  }
}

constexpr uint32_t DEQ_RETRY = BOTC;  // try_deq result: take another ticket

template <bool ACQUIRE>
__device__ __forceinline__ uint32_t try_deq(const WRing& r, uint64_t h, uint32_t& cf) {
  const uint32_t c = r.cycle_of(h);
  const uint64_t j = r.slot_of(h);
  uint64_t* p = r.g.at(j);
  uint64_t e = ld(p);
  // The entry is still from an older cycle but Tail shows ticket h handed
  // to an enqueuer, whose install follows its Tail increment closely: look
  // at the entry a bounded number of times before marking it, rather than
  // spoil that enqueuer's attempt (a slow-path enqueuer can otherwise lose
  // every round to a crowd of polling dequeuers).
  // A slow-path install takes longer (SlowFAA's two phases, helpers): while
  // a slow-path request is announced on the ring the wait is longer too.
  if (older(e_cyc(e), c) && idx_free(e_idx(e)) && g_ctr(ld(r.g.tail)) > h) {
    const uint32_t polls = ld(r.announce) ? DEQ_WAIT_POLLS_SLOW : DEQ_WAIT_POLLS;
    for (uint32_t w = 0; w < polls && older(e_cyc(e), c) && idx_free(e_idx(e)); w++) {
      pause(1);
      e = ld(p);
    }
  }
  while (true) {
    if (e_cyc(e) == c && !idx_free(e_idx(e))) {
      if (!e_enq(e)) finalize_enq(r.rec, r.owner, r.k, r.stats, h, j);
      const uint64_t x = (uint64_t)(e_idx(e) ^ BOTC);
      if (ACQUIRE) fxor_acq(p, x); else fxor(p, x);
      return e_idx(e);
    }
    if (older(e_cyc(e), c)) {
      const uint64_t ne = idx_free(e_idx(e))
                              ? e_make(e_note(e), c, e_safe(e), true, BOT)
                              : e_make(e_note(e), e_cyc(e), false, e_enq(e), e_idx(e));
      if (!cas(p, e, ne)) {
        cf++;
        continue;
      }
    }
    break;
  }
  const uint64_t t = g_ctr(ld(r.g.tail));
  if (t <= h + 1) {
    // one catch-up to the wavefront's largest h + 1 and one aggregated
    // Threshold decrement for all lanes here (as in the G-LFQ fast path)
    const uint64_t target = wave_max(h + 1);
    const uint64_t mask = active_mask();
    if (lane_rank(mask) == 0) {
      catchup(r, target);
      faa(r.g.thr, -(int64_t)__popcll(mask));
    }
    return BOT;
  }
  if (wave_fdec(r.g.thr) <= 0) return BOT;
  return DEQ_RETRY;
}

// ---- slow path ---------------------------------------------------------------
// Clear ThrIdx = lane q2 + 1 from the Global word after committing that
// lane's pending increment.  The INC bit is cleared only when the Local
// word's counter is below the Global counter read before it: then the INC
// belongs to the round whose increment set ThrIdx (a later round's INC can
// only be set after ThrIdx was cleared, at a counter no smaller than the one
// read here).
__device__ __forceinline__ void clear_thr(const WRing& r, uint64_t* G, uint32_t q2) {
  Rec* R2 = &r.rec[q2];
  uint64_t g = ld_acq(G);
  for (uint32_t spin = 0; g_thr(g) == q2 + 1; spin++) {
    if (spin_out(spin, r.err)) { latch_error(r.err, (uint64_t)(-GQ_ERR_DEVICE)); return; }
    const uint64_t l2 = ld_acq(&R2->local);
    if (l_inc(l2)) {
      if (l_ctr(l2) >= g_ctr(g)) {  // stale view of Global: read it again
        g = ld_acq(G);
        continue;
      }
      uint64_t le = l2;
      cas_acqrel(&R2->local, le, l2 & ~L_INC);
    }
    if (cas_acqrel(G, g, g & ~TID_MASK)) return;
  }
}

// SlowFAA (Algorithm 2): returns true with v = the Local word holding the
// next agreed ticket, or false once the request is finished (FIN) or replaced
// (tag changed), or when a fail-safe bound stopped it (gave_up set, error
// latched).  thld: Threshold for dequeue rounds (decremented once per round by
// the helper whose increment succeeded), NULL for enqueues.
__device__ __forceinline__ bool slow_faa(const WRing& r, uint64_t* G, uint32_t rid, uint64_t tag,
                                         uint64_t& v, int64_t* thld, uint64_t deadline,
                                         bool* announced, bool& gave_up) {
  Rec* R = &r.rec[rid];
  for (uint32_t spin = 0;; spin++) {
    if (spin_out(spin, r.err) || ((spin & 255) == 255 && stamp() > deadline)) {
      latch_error(r.err, (uint64_t)(-GQ_ERR_DEVICE));
      gave_up = true;
      return false;
    }
    if (announced && !*announced && (spin & 63) == 63) *announced = try_announce(r, rid);
    const uint64_t l = ld_acq(&R->local);
    if (l_tag(l) != (tag & L_TAG_MASK) || l_fin(l)) return false;
    if (!l_inc(l) && l != v) {  // a newer committed ticket
      v = l;
      return true;
    }
    const uint64_t g = ld_acq(G);
    if (g_thr(g)) {  // help the pending phase 2 first
      clear_thr(r, G, g_thr(g) - 1);
      continue;
    }
    const uint64_t c = g_ctr(g);
    uint64_t le = l;
    if (l_inc(l) && l_ctr(l) == c) {
      uint64_t ge = g;
      if (cas_acqrel(G, ge, ((c + 1) << TID_BITS) | (rid + 1))) {
        if (thld) faa(thld, (int64_t)-1);
        cas_acqrel(&R->local, le, l & ~L_INC);
        clear_thr(r, G, rid);
        v = l & ~L_INC;
        return true;
      }
    } else {
      // start the next round at c, or retarget a pending one that Global
      // has moved past without this request's increment
      cas_acqrel(&R->local, le, l_make(tag, c, true, false));
    }
  }
}

__device__ __forceinline__ void hint_owner(const WRing& r, uint64_t j, uint64_t T, uint32_t rid) {
  const uint64_t nw = ((T & CTR_MASK) << TID_BITS) | (rid + 1);
  uint64_t o = ld(&r.owner[j]);
  while ((o >> TID_BITS) < (T & CTR_MASK))
    if (cas(&r.owner[j], o, nw)) break;
}

// TryEnqSlow on the agreed ticket T.  Returns 1 when the request's item is
// installed at T (by this or another helper), 0 to go to the next round, -1
// when the fail-safe bound stopped it (error latched).
__device__ __forceinline__ int try_enq_slow(const WRing& r, uint64_t T, uint32_t idx, uint32_t rid,
                                            uint64_t tag) {
  const uint32_t c = r.cycle_of(T);
  const uint64_t j = r.slot_of(T);
  uint64_t* p = r.g.at(j);
  uint64_t e = ld_acq(p);
  for (uint32_t spin = 0;; spin++) {
    if (spin_out(spin, r.err)) { latch_error(r.err, (uint64_t)(-GQ_ERR_DEVICE)); return -1; }
    if (e_cyc(e) == c) return e_idx(e) != BOT ? 1 : 0;  // ours (maybe consumed), or dequeuer T left it empty
    if (!older(e_cyc(e), c) || !older(e_note(e), c)) return 0;  // moved on, or already noted
    if (!((e_safe(e) || g_ctr(ld(r.g.head)) <= T) && idx_free(e_idx(e)))) {
      // Lemma 6: record that this slot is ruled out for cycle c
      const uint64_t ne = (e & ~((uint64_t)TAG_MASK << NOTE_SHIFT)) | ((uint64_t)c << NOTE_SHIFT);
      if (cas_acqrel(p, e, ne)) return 0;
      continue;
    }
    hint_owner(r, j, T, rid);
    const uint64_t ne = e_make(e_note(e), c, true, false, idx);
    if (cas_acqrel(p, e, ne)) {
      Rec* R = &r.rec[rid];
      uint64_t le = l_make(tag, T, false, false);
      if (cas_acqrel(&R->local, le, le | L_FIN)) {
        // make the entry an ordinary one (Enq 0 -> 1) while it is still ours
        uint64_t e2 = ne;
        while (e_cyc(e2) == c && e_idx(e2) == idx && !e_enq(e2))
          if (cas_acqrel(p, e2, e2 | ENQ_BIT)) break;
      }
      reset_threshold(r);
      return 1;
    }
  }
}

__device__ __forceinline__ void fin_at(Rec* R, uint64_t tag, uint64_t H) {
  uint64_t le = l_make(tag, H, false, false);
  cas_acqrel(&R->local, le, le | L_FIN);
}

// TryDeqSlow on the agreed ticket H.  Returns true when the request is decided
// (an entry for H is there, or the queue was seen empty), false otherwise.
__device__ __forceinline__ bool try_deq_slow(const WRing& r, uint64_t H, uint32_t rid, uint64_t tag) {
  Rec* R = &r.rec[rid];
  const uint32_t c = r.cycle_of(H);
  uint64_t* p = r.g.at(r.slot_of(H));
  uint64_t e = ld_acq(p);
  for (uint32_t spin = 0;; spin++) {
    if (spin_out(spin, r.err)) { latch_error(r.err, (uint64_t)(-GQ_ERR_DEVICE)); return true; }
    if (e_cyc(e) == c && e_idx(e) != BOT) {
      fin_at(R, tag, H);
      return true;
    }
    if (older(e_cyc(e), c)) {
      const uint64_t ne = idx_free(e_idx(e))
                              ? e_make(e_note(e), c, e_safe(e), true, BOT)
                              : e_make(e_note(e), e_cyc(e), false, e_enq(e), e_idx(e));
      if (!cas_acqrel(p, e, ne)) continue;
    }
    break;
  }
  const uint64_t t = g_ctr(ld_acq(r.g.tail));
  if (t <= H + 1) {
    catchup(r, H + 1);
    fin_at(R, tag, H);
    return true;
  }
  if (ld(r.g.thr) < 0) {
    fin_at(R, tag, H);
    return true;
  }
  return false;
}

// Drive request (rid, tag) until it is decided; used by owners and helpers.
// An enqueue stops as soon as its item is installed at the current ticket
// (starting another round then would install it twice) and returns that
// ticket.  A dequeue keeps going until FIN: helpers may disagree about an
// empty decision, and the request follows whichever change of its Local word
// lands first.  Returns NO_TICKET when the request was found finished, and
// SLOW_GAVE_UP when a fail-safe bound stopped this lane's part (error
// latched).
__device__ __forceinline__ uint64_t run_slow(const WRing& r, uint32_t rid, uint64_t tag, bool is_enq,
                                             uint32_t idx, uint64_t v, bool* announced = nullptr) {
  uint64_t* G = is_enq ? r.g.tail : r.g.head;
  int64_t* thld = is_enq ? nullptr : r.g.thr;
  // Fail-safe: a request that is still undecided after SLOW_LIMIT_TICKS of
  // the GPU clock latches GQ_ERR_DEVICE instead of occupying its lane longer
  // (the bound Lemma 4 gives is far shorter in every configuration tested).
  const uint64_t deadline = stamp() + SLOW_LIMIT_TICKS;
  bool gave_up = false;
  for (uint32_t rounds = 0; slow_faa(r, G, rid, tag, v, thld, deadline, announced, gave_up);
       rounds++) {
    if (spin_out(rounds, r.err) || stamp() > deadline) {
      latch_error(r.err, (uint64_t)(-GQ_ERR_DEVICE));
      return SLOW_GAVE_UP;
    }
    const uint64_t T = l_ctr(v);
    if (is_enq) {
      const int res = try_enq_slow(r, T, idx, rid, tag);
      if (res > 0) return T;
      if (res < 0) return SLOW_GAVE_UP;
    } else {
      try_deq_slow(r, T, rid, tag);
    }
  }
  return gave_up ? SLOW_GAVE_UP : NO_TICKET;
}

// Publish a request (Section III-C, "GPU publication discipline"): payload
// fields first, then <seq, enqueue, pending> with release.  Returns the tag.
__device__ __forceinline__ uint64_t publish(Rec* R, bool is_enq, uint64_t init, uint32_t idx,
                                            uint64_t& seq, uint64_t& v0) {
  seq = R->next_seq;  // owner-private
  R->next_seq = seq + 1;
  const uint64_t tag = seq & L_TAG_MASK;
  st(&R->init, init);
  st(&R->index, (uint64_t)idx);
  v0 = l_make(tag, init, false, false);
  st(&R->local, v0);
  st_rel(&R->req, (seq << 2) | (is_enq ? 2ull : 0ull) | 1ull);
  return tag;
}

__device__ __forceinline__ void unpublish(Rec* R, bool is_enq, uint64_t seq) {
  st_rel(&R->req, (seq << 2) | (is_enq ? 2ull : 0ull));
}

// Help lane p's pending request on ring r, if any (the help step, D = help delay).
// A relaxed look at the request word comes first: with no request pending
// (the common case) the check costs one load and no cache invalidation; a
// request published after this look is simply helped on a later visit.
__device__ __forceinline__ void help_peer(const WRing& r, uint32_t p) {
  Rec* R = &r.rec[p];
  if (!(ld(&R->req) & 1)) return;
  const uint64_t q1 = ld_acq(&R->req);
  if (!(q1 & 1)) return;
  const uint64_t init = ld_acq(&R->init);
  const uint64_t idx = ld_acq(&R->index);
  const uint64_t q2 = ld_acq(&R->req);
  if (q2 != q1) return;  // the request changed while its fields were read
  const uint64_t tag = (q1 >> 2) & L_TAG_MASK;
  faa(r.stats + S_HELPS, 1ull);
  run_slow(r, p, tag, (q1 & 2) != 0, (uint32_t)idx, l_make(tag, init, false, false));
}

__device__ __forceinline__ void help_announced(const WRing& r, uint32_t tid) {
  const uint64_t a = ld(r.announce);
  if (a == 0 || a - 1 == tid || a - 1 >= r.k) return;
  // One helper per wavefront: the wavefront waits while its first lane
  // helps, which already keeps its fetch-and-adds off the Global word, and
  // a request with tens of thousands of helpers would spend its rounds on
  // their CAS traffic to its Local and Global words.
  if (lane_rank(active_mask()) == 0) help_peer(r, (uint32_t)(a - 1));
}

// Every D operations of a lane, inspect one peer's records on both rings.
// The lane's counter and next peer form one 32-bit word <peer:20 | count:12>
// (help step state).  help_step advances it in a register; help_check keeps
// it in the queue's compact per-lane array (a wavefront's 64 words share 2
// lines) for callers that hold no state between operations.
__device__ __forceinline__ void help_step(const gq_dev& q, uint32_t tid, uint32_t& h) {
  uint32_t cnt = (h & 0xFFFu) + 1;
  uint32_t peer = h >> 12;
  if (cnt >= q.help_delay) {
    cnt = 0;
    if (peer >= q.max_threads) peer = 0;
    if (peer != tid) {
      help_peer(make_wring(q.aq, q), peer);
      help_peer(make_wring(q.fq, q), peer);
    }
    peer = peer + 1 >= q.max_threads ? 0 : peer + 1;
  }
  h = (peer << 12) | cnt;
}

__device__ __forceinline__ void help_check(const gq_dev& q, uint32_t tid) {
  uint32_t* hp = q.help_ctr + tid;
  uint32_t h = *hp;  // owner-private
  help_step(q, tid, h);
  *hp = h;
}

// The help step state of lane tid, to hold in a register across a run of
// group_op calls that pass it (help_load before the first, help_store after
// the last): each operation then saves the array's load and store, whose
// load would otherwise sit on the operation's dependency chain.
__device__ __forceinline__ uint32_t help_load(const gq_dev& q, uint32_t tid) {
  return q.help_ctr[tid];
}
__device__ __forceinline__ void help_store(const gq_dev& q, uint32_t tid, uint32_t h) {
  q.help_ctr[tid] = h;
}

// Inner enqueue of idx: fast path up to patience_enq attempts, then the slow path.
// `first`: a Tail ticket already reserved for this operation (workgroup
// aggregation), tried before the fast-path loop; NO_TICKET if none.
// Returns false only when a fail-safe bound stopped the slow path before the
// index was installed (error latched).
template <bool RELEASE>
__device__ __forceinline__ bool ring_enq(const WRing& r, const gq_dev& q, uint32_t tid, uint32_t idx,
                                         uint32_t& cf, uint64_t first = NO_TICKET) {
  uint64_t last = NO_TICKET;
  if (first != NO_TICKET) {
    if (try_enq<RELEASE>(r, first, idx, cf)) return true;
    last = first;
  }
  for (uint32_t a = first != NO_TICKET ? 1u : 0u; a < q.patience_enq; a++) {
    help_announced(r, tid);
    const uint64_t t = ticket(wave_faa(r.g.tail, UNIT));
    if (try_enq<RELEASE>(r, t, idx, cf)) return true;
    last = t;
  }
  faa(r.stats + S_SLOW, 1ull);
  Rec* R = &r.rec[tid];
  uint64_t seq, v0;
  const uint64_t tag = publish(R, true, last, idx, seq, v0);
  bool announced = try_announce(r, tid);
  const uint64_t T = run_slow(r, tid, tag, true, idx, v0, &announced);
  if (T != NO_TICKET && T != SLOW_GAVE_UP) {
    // The item sits at T; make sure FIN is set and the entry is ordinary
    // before the record is reused (otherwise a dequeuer meeting Enq = 0
    // would have to scan every record for the finished request).
    fin_at(R, tag, T);
    const uint32_t c = r.cycle_of(T);
    uint64_t* p = r.g.at(r.slot_of(T));
    uint64_t e = ld_acq(p);
    while (e_cyc(e) == c && e_idx(e) == idx && !e_enq(e))
      if (cas_acqrel(p, e, e | ENQ_BIT)) break;
  }
  if (announced) withdraw(r, tid);
  unpublish(R, true, seq);
  return T != SLOW_GAVE_UP;
}

// Inner dequeue: returns an index, BOT (EMPTY), or GAVE_UP when a fail-safe
// bound stopped the slow path (error latched).
// `first`: a Head ticket already reserved for this operation (workgroup
// aggregation; Threshold was checked before reserving it).  It is always
// tried: a Head ticket that no dequeuer visits could strand an item.
template <bool ACQUIRE>
__device__ __forceinline__ uint32_t ring_deq(const WRing& r, const gq_dev& q, uint32_t tid,
                                             uint32_t& cf, uint64_t first = NO_TICKET) {
  uint64_t last = NO_TICKET;
  if (first != NO_TICKET) {
    const uint32_t res = try_deq<ACQUIRE>(r, first, cf);
    if (res != DEQ_RETRY) return res;
    last = first;
  }
  for (uint32_t a = first != NO_TICKET ? 1u : 0u;; a++) {
    const int64_t th = ld(r.g.thr);
    if (th < 0) return BOT;
    if (a >= q.patience_deq) break;
    help_announced(r, tid);
    // empty pre-check and bounded grab on the counters while Threshold shows
    // recent failures or this lane's last dequeue here found the ring empty
    // (see lfq::ring_deq and poll_avail)
    const bool hinted = r.hint[tid] != 0;
    if (th < r.g.thr_reset || hinted) {
      const uint64_t avail = poll_avail(r.g.head, r.g.tail, TID_BITS);
      if (avail == 0) {
        if (!hinted) r.hint[tid] = 1;
        return BOT;
      }
      if (lane_rank(active_mask()) >= avail) {  // looking again uses up an attempt
        pause(1);
        continue;
      }
      if (hinted) r.hint[tid] = 0;  // the lane takes a ticket
    }
    const uint64_t h = ticket(wave_faa(r.g.head, UNIT));
    const uint32_t res = try_deq<ACQUIRE>(r, h, cf);
    if (res != DEQ_RETRY) return res;
    last = h;
  }
  faa(r.stats + S_SLOW, 1ull);
  Rec* R = &r.rec[tid];
  uint64_t seq, v0;
  const uint64_t tag = publish(R, false, last, 0, seq, v0);
  bool announced = try_announce(r, tid);
  run_slow(r, tid, tag, false, 0, v0, &announced);
  const uint64_t l = ld_acq(&R->local);
  if (announced) withdraw(r, tid);
  unpublish(R, false, seq);
  if (!l_fin(l) || l_tag(l) != (tag & L_TAG_MASK)) {  // only after a fail-safe stop
    latch_error(r.err, (uint64_t)(-GQ_ERR_DEVICE));
    return GAVE_UP;
  }
  const uint64_t H = l_ctr(l);
  const uint64_t j = r.slot_of(H);
  uint64_t* p = r.g.at(j);
  const uint64_t e = ld_acq(p);
  if (e_cyc(e) == r.cycle_of(H) && !idx_free(e_idx(e))) {
    if (!e_enq(e)) finalize_enq(r.rec, r.owner, r.k, r.stats, H, j);
    const uint64_t x = (uint64_t)(e_idx(e) ^ BOTC);
    if (ACQUIRE) fxor_acq(p, x); else fxor(p, x);
    return e_idx(e);
  }
  return BOT;
}

// ---- outer queue ---------------------------------------------------------------
template <bool FENCED>
__device__ __forceinline__ int enqueue_impl(const gq_dev& q, uint64_t item, uint32_t tid,
                                            uint32_t& cf) {
  if (tid >= q.max_threads) {
    latch_error(q.err, (uint64_t)(-GQ_ERR_INVALID));
    return GQ_ERR_INVALID;
  }
  help_check(q, tid);
  const WRing fq = make_wring(q.fq, q);
  const WRing aq = make_wring(q.aq, q);
  const uint32_t idx = ring_deq<false>(fq, q, tid, cf);
  if (idx == BOT) return GQ_FULL;
  if (idx >= q.capacity) {  // GAVE_UP; guards the payload array
    latch_error(q.err, (uint64_t)(-GQ_ERR_DEVICE));
    lfq::count_drop(q);
    return GQ_ERR_DEVICE;
  }
  lfq::payload_put<FENCED>(q, idx, item);
  if (!ring_enq<FENCED>(aq, q, tid, idx, cf)) {  // the item is lost with its index
    lfq::count_drop(q);
    return GQ_ERR_DEVICE;
  }
  return GQ_OK;
}

template <bool FENCED>
__device__ __forceinline__ int dequeue_impl(const gq_dev& q, uint64_t* item, uint32_t tid,
                                            uint32_t& cf) {
  if (tid >= q.max_threads) {
    latch_error(q.err, (uint64_t)(-GQ_ERR_INVALID));
    return GQ_ERR_INVALID;
  }
  help_check(q, tid);
  const WRing aq = make_wring(q.aq, q);
  const WRing fq = make_wring(q.fq, q);
  const uint32_t idx = ring_deq<FENCED>(aq, q, tid, cf);
  if (idx == BOT) return GQ_EMPTY;
  if (idx >= q.capacity) {  // GAVE_UP; guards the payload array
    latch_error(q.err, (uint64_t)(-GQ_ERR_DEVICE));
    lfq::count_drop(q);
    return GQ_ERR_DEVICE;
  }
  *item = lfq::payload_get<FENCED>(q, idx);
  if (!ring_enq<FENCED>(fq, q, tid, idx, cf)) lfq::count_drop(q);  // the item was delivered
  return GQ_OK;
}

// ---- workgroup-uniform form (see lfq::group_op) ----------------------------
__device__ __forceinline__ uint64_t group_decode(uint64_t word) {
  return word == GROUP_NONE ? NO_TICKET : ticket(word);
}

template <bool FENCED>
__device__ __forceinline__ int group_op_impl(const gq_dev& q, int role, uint64_t& item,
                                             uint32_t tid, uint32_t& cf, GroupLds& s,
                                             uint32_t& par, uint32_t* help) {
  int st = role == ROLE_ENQ ? GQ_FULL : role == ROLE_DEQ ? GQ_EMPTY : GQ_OK;
  if (role != ROLE_NONE && tid >= q.max_threads) {
    latch_error(q.err, (uint64_t)(-GQ_ERR_INVALID));
    st = GQ_ERR_INVALID;
    role = ROLE_NONE;
  }
  if (role != ROLE_NONE) {
    if (help) help_step(q, tid, *help);
    else help_check(q, tid);
  }
  const WRing fq = make_wring(q.fq, q);
  const WRing aq = make_wring(q.aq, q);
  const bool wf = role == ROLE_ENQ && ld(fq.g.thr) >= 0;
  const bool wa = role == ROLE_DEQ && ld(aq.g.thr) >= 0;
  uint64_t t = group_decode(group_ticket(s, par, fq.g.head, UNIT, wf, aq.g.head, UNIT, wa));
  uint32_t idx = BOT;
  if (wf) idx = ring_deq<false>(fq, q, tid, cf, t);
  else if (wa) idx = ring_deq<FENCED>(aq, q, tid, cf, t);
  if (idx != BOT && idx >= q.capacity) {  // GAVE_UP; guards the payload array
    latch_error(q.err, (uint64_t)(-GQ_ERR_DEVICE));
    lfq::count_drop(q);
    idx = BOT;
    st = GQ_ERR_DEVICE;
  }
  if (idx != BOT) {
    if (role == ROLE_ENQ) lfq::payload_put<FENCED>(q, idx, item);
    else item = lfq::payload_get<FENCED>(q, idx);
    st = GQ_OK;
  }
  const bool we = role == ROLE_ENQ && idx != BOT;
  const bool wd = role == ROLE_DEQ && idx != BOT;
  t = group_decode(group_ticket(s, par, aq.g.tail, UNIT, we, fq.g.tail, UNIT, wd));
  bool placed = true;
  if (we) placed = ring_enq<FENCED>(aq, q, tid, idx, cf, t);
  else if (wd) placed = ring_enq<FENCED>(fq, q, tid, idx, cf, t);
  if (!placed) {
    lfq::count_drop(q);
    if (we) st = GQ_ERR_DEVICE;
  }
  return st;
}

// `help`: the lane's help step state held by the caller (help_load /
// help_store), or nullptr to keep it in the queue's per-lane array.
__device__ __forceinline__ int group_op(const gq_dev& q, int role, uint64_t& item, uint32_t tid,
                                        uint32_t& cf, GroupLds& s, uint32_t& par,
                                        uint32_t* help = nullptr) {
  return (q.flags & GQ_OPT_FENCED) ? group_op_impl<true>(q, role, item, tid, cf, s, par, help)
                                   : group_op_impl<false>(q, role, item, tid, cf, s, par, help);
}

__device__ __forceinline__ int enqueue(const gq_dev& q, uint64_t item, uint32_t tid, uint32_t& cf) {
  return (q.flags & GQ_OPT_FENCED) ? enqueue_impl<true>(q, item, tid, cf)
                                   : enqueue_impl<false>(q, item, tid, cf);
}

__device__ __forceinline__ int dequeue(const gq_dev& q, uint64_t* item, uint32_t tid, uint32_t& cf) {
  return (q.flags & GQ_OPT_FENCED) ? dequeue_impl<true>(q, item, tid, cf)
                                   : dequeue_impl<false>(q, item, tid, cf);
}

}  // namespace wfq
}  // namespace gq
