// Device primitives shared by the three queues: scoped atomics, the
// wave-aggregated fetch-and-add, timestamps and the counter-based random
// stream used by the benchmark kernels.  gfx950 (CDNA4), 64-lane wavefronts.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../gq.h"

namespace gq {

// ---------------------------------------------------------------------------
// Agent-scope atomics.  Every shared word is read with an agent-scope atomic
// load (on gfx950 a plain load may hit a stale line in this XCD's L2), and
// every update is one 64-bit atomic: the paper's single-word atomicity
// requirement (Section III-C, Lemma 3) and the absence of CAS2 on GPUs.
// ---------------------------------------------------------------------------
#define GQ_AGENT __HIP_MEMORY_SCOPE_AGENT

__device__ __forceinline__ uint64_t ld(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, GQ_AGENT);
}
__device__ __forceinline__ int64_t ld(const int64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, GQ_AGENT);
}
__device__ __forceinline__ uint32_t ld(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, GQ_AGENT);
}
__device__ __forceinline__ uint64_t ld_acq(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, GQ_AGENT);
}
__device__ __forceinline__ void st(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, GQ_AGENT);
}
__device__ __forceinline__ void st(int64_t* p, int64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, GQ_AGENT);
}
__device__ __forceinline__ void st(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, GQ_AGENT);
}
__device__ __forceinline__ void st_rel(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, GQ_AGENT);
}
// CAS; on failure `expected` receives the current value.
__device__ __forceinline__ bool cas(uint64_t* p, uint64_t& expected, uint64_t desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, GQ_AGENT);
}
__device__ __forceinline__ bool cas32(uint32_t* p, uint32_t& expected, uint32_t desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, GQ_AGENT);
}
__device__ __forceinline__ bool cas_rel(uint64_t* p, uint64_t& expected, uint64_t desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELEASE,
                                              __ATOMIC_RELAXED, GQ_AGENT);
}
__device__ __forceinline__ bool cas_acqrel(uint64_t* p, uint64_t& expected, uint64_t desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_ACQ_REL,
                                              __ATOMIC_ACQUIRE, GQ_AGENT);
}
__device__ __forceinline__ uint64_t xchg(uint64_t* p, uint64_t v) {
  return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, GQ_AGENT);
}
__device__ __forceinline__ uint32_t xchg(uint32_t* p, uint32_t v) {
  return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, GQ_AGENT);
}
__device__ __forceinline__ uint64_t faa(uint64_t* p, uint64_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, GQ_AGENT);
}
__device__ __forceinline__ int64_t faa(int64_t* p, int64_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, GQ_AGENT);
}
__device__ __forceinline__ uint64_t fxor(uint64_t* p, uint64_t v) {
  return __hip_atomic_fetch_xor(p, v, __ATOMIC_RELAXED, GQ_AGENT);
}
__device__ __forceinline__ uint64_t fxor_acq(uint64_t* p, uint64_t v) {
  return __hip_atomic_fetch_xor(p, v, __ATOMIC_ACQUIRE, GQ_AGENT);
}
__device__ __forceinline__ uint64_t f_or(uint64_t* p, uint64_t v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, GQ_AGENT);
}
__device__ __forceinline__ uint64_t f_and(uint64_t* p, uint64_t v) {
  return __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, GQ_AGENT);
}
// Wait until every memory operation this wavefront issued has completed
// (returned its value or been acknowledged).  Orders an atomic that must be
// performed before a later one without any cache maintenance.
__device__ __forceinline__ void wait_mem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
// Keep a value live in a register so the atomic producing it returns it.
template <typename T>
__device__ __forceinline__ void keep(T v) { asm volatile("" ::"v"(v)); }

__device__ __forceinline__ void fence_acq() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ void fence_rel() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void fence_acqrel() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent"); }

// ---------------------------------------------------------------------------
// Wavefront helpers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t active_mask() { return __ballot(1); }

// Number of active lanes below this lane in `mask` (the lane's prefix rank).
__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t read_first_lane(uint64_t v) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// WaveFAA (Section III-B, Algorithm 1; Lemma 1).  Every lane that reaches
// this call together forms the mask; the lowest active lane (the leader)
// performs one fetch-and-add of popcount(mask) * unit on *ctr; the old value
// is broadcast and each lane receives base + rank * unit, where rank is its
// prefix count in the mask.  The returned tickets are distinct and
// consecutive, in the same total order per-lane FAAs would give.  `unit`
// lets packed counters (G-WFQ's <Counter, ThrIdx> word) step their counter
// field; the caller decodes.
__device__ __forceinline__ uint64_t wave_faa(uint64_t* ctr, uint64_t unit) {
  const uint64_t mask = active_mask();
  const uint32_t rank = lane_rank(mask);
  const uint32_t cnt = (uint32_t)__popcll(mask);
  uint64_t base = 0;
  if (rank == 0) base = faa(ctr, (uint64_t)cnt * unit);
  base = read_first_lane(base);
  return base + (uint64_t)rank * unit;
}

// Largest value of v over the lanes active at this call (all of them get it).
__device__ __forceinline__ uint64_t wave_max(uint64_t v) {
  uint64_t m = active_mask(), mx = 0;
  while (m) {
    const int l = __ffsll((unsigned long long)m) - 1;
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), l);
    const uint64_t x = ((uint64_t)hi << 32) | lo;
    mx = x > mx ? x : mx;
    m &= m - 1;
  }
  return mx;
}

// WaveFAA on a signed counter stepping by -1 per lane: the lanes active at
// this call receive old, old - 1, old - 2, ... in lane order (the values
// per-lane decrements would return, in some order), with one atomic.
__device__ __forceinline__ int64_t wave_fdec(int64_t* ctr) {
  return (int64_t)wave_faa((uint64_t*)ctr, ~0ull);
}

// ---------------------------------------------------------------------------
// Workgroup-aggregated tickets.  Lemma 1's argument does not depend on the
// lanes sharing a fetch-and-add being one wavefront: any set of requests that
// are all pending when one FAA of their count is performed can take
// base, base + 1, ... in a fixed order, exactly as if each had performed its
// own FAA at that instant.  group_ticket applies it to a whole workgroup
// (up to 16 wavefronts), so each ticket counter sees one FAA per workgroup
// instead of one per wavefront.  Every thread of the workgroup must call it
// with uniform control flow (it contains two barriers).
//
// Two counters are served per call (an operation mix takes tickets on two
// different counters in the same phase); a lane requests from at most one of
// them (w0 and w1 exclusive).  `unit` is the FAA step per ticket (packed
// counters).  The result is the counter value the lane's own FAA would have
// returned, or GROUP_NONE if the lane requested nothing.
// ---------------------------------------------------------------------------
constexpr uint64_t GROUP_NONE = ~0ull;
constexpr uint32_t GROUP_MAX_WAVES = 16;

struct GroupLds {
  uint64_t base[2][GROUP_MAX_WAVES][2];
  uint32_t cnt[2][GROUP_MAX_WAVES][2];
};

// `par` alternates the LDS buffers between consecutive calls: a wavefront
// may enter call i + 1 while a slower one still reads call i's bases, but it
// cannot reach call i + 2 before every wavefront has passed call i + 1's first
// barrier, i.e. finished reading call i.
__device__ __forceinline__ uint64_t group_ticket(GroupLds& s, uint32_t& par, uint64_t* c0,
                                                 uint64_t u0, bool w0, uint64_t* c1, uint64_t u1,
                                                 bool w1) {
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t nw = blockDim.x >> 6;
  const uint64_t m0 = __ballot(w0);
  const uint64_t m1 = __ballot(w1);
  const uint32_t p = par;
  par ^= 1u;
  if ((threadIdx.x & 63) == 0) {
    s.cnt[p][wave][0] = (uint32_t)__popcll(m0);
    s.cnt[p][wave][1] = (uint32_t)__popcll(m1);
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const uint32_t j = threadIdx.x;
    uint64_t tot = 0;
    for (uint32_t w = 0; w < nw; w++) tot += s.cnt[p][w][j];
    const uint64_t u = j ? u1 : u0;
    uint64_t b = tot ? faa(j ? c1 : c0, tot * u) : 0;
    for (uint32_t w = 0; w < nw; w++) {
      s.base[p][w][j] = b;
      b += (uint64_t)s.cnt[p][w][j] * u;
    }
  }
  __syncthreads();
  if (w0) return s.base[p][wave][0] + (uint64_t)lane_rank(m0) * u0;
  if (w1) return s.base[p][wave][1] + (uint64_t)lane_rank(m1) * u1;
  return GROUP_NONE;
}

// Operation roles of a workgroup-uniform call.
enum GroupRole { ROLE_ENQ = 0, ROLE_DEQ = 1, ROLE_NONE = 2 };

// Wave sum of a per-lane value; every lane receives the total.
__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One atomic per wave: add the wave total of v to *dst.
__device__ __forceinline__ void wave_add(uint64_t* dst, uint64_t v) {
  const uint64_t mask = active_mask();
  // Inactive lanes contribute nothing; shuffles read 0 from them by zeroing
  // before the reduction in fully converged code only, so reduce with a
  // ballot-driven loop that is correct under any mask.
  uint64_t total = 0;
  uint64_t m = mask;
  while (m) {
    const int l = __ffsll((unsigned long long)m) - 1;
    total += __shfl(v, l, 64);
    m &= m - 1;
  }
  if (lane_rank(mask) == 0 && total) faa(dst, total);
}

// ---------------------------------------------------------------------------
// Device timestamp: the constant-rate (100 MHz) real-time counter, read with
// the wait that makes the value available before any later memory access.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t stamp() {
  uint64_t t;
  asm volatile("s_memrealtime %0\n\ts_waitcnt lgkmcnt(0)" : "=s"(t)::"memory");
  return t;
}

// Short pause (used by seeded jitter in tests and by bounded back-off).
__device__ __forceinline__ void pause(uint32_t units) {
  for (uint32_t i = 0; i < units; i++) __builtin_amdgcn_s_sleep(1);
}

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the c-th output of the
// generator seeded with `seed` is the finalizer applied to
// seed + (c + 1) * 0x9E3779B97F4A7C15.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Device error latch: first error wins.
__device__ __forceinline__ void latch_error(uint64_t* err, uint64_t code) {
  uint64_t zero = 0;
  cas(err, zero, code);
}

// Statistics slots (gq_stats order).
enum StatSlot {
  S_OK_ENQ = 0, S_OK_DEQ, S_FULL, S_EMPTY, S_CAS_FAIL, S_TICKETS, S_SLOW, S_HELPS, S_SCAN,
  S_DROP,  // operations abandoned by a fail-safe bound (item or index lost, error latched)
  S_NUM
};

// Fail-safe bound of every retry loop in the queues.  The algorithms retry
// only while other lanes make progress, so reaching SPIN_LIMIT iterations
// means an invariant broke.  Once any lane has latched an error on the queue
// (a broken invariant, an exhausted pool, or a driver's time limit) every
// loop also stops within SPIN_POLL iterations: then no kernel that uses the
// queue can stay inside a queue operation after its driver gave up.
constexpr uint32_t SPIN_LIMIT = 1u << 22;
constexpr uint32_t SPIN_POLL = 1024;
__device__ __forceinline__ bool spin_out(uint32_t spin, const uint64_t* err) {
  if (spin >= SPIN_LIMIT) return true;
  return (spin & (SPIN_POLL - 1)) == SPIN_POLL - 1 &&
         __hip_atomic_load(err, __ATOMIC_RELAXED, GQ_AGENT) != 0;
}

// Entries a dequeuer could find right now on a pair of monotone ticket
// counters: Tail - Head, read in that order (Head first, and only after its
// value has returned, Tail), or 0 when Tail <= Head.  Both counters sit in
// the bits above `shift` of their words.  With Tail <= Head every item
// already in the queue was handed a Head ticket before the Tail read, so the
// dequeuers holding those tickets will take them: they can be linearized
// just before the Tail read, in ticket order, and the queue is empty there --
// an EMPTY answer that takes (and burns) no ticket.
__device__ __forceinline__ uint64_t poll_avail(uint64_t* head, uint64_t* tail, uint32_t shift) {
  const uint64_t hh = read_first_lane(ld(head));
  keep(hh);
  wait_mem();
  const uint64_t tt = read_first_lane(ld(tail));
  const uint64_t hc = hh >> shift, tc = tt >> shift;
  return tc > hc ? tc - hc : 0;
}

}  // namespace gq
