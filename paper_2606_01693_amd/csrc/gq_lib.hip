// libgq.so: host side of the C ABI (include/gq.h, include/gq_bench.h) and the
// kernels it launches.  One process, one GPU, HIP streams passed in by the
// caller; every device word the queues share lives in one allocation.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>

#include "../../include/gq.h"
#include "../../include/gq_bench.h"
#include "../../include/gq_device.h"

using namespace gq;

// A failed HIP call returns GQ_ERR_HIP; with GQ_VERBOSE set in the
// environment the HIP error is also printed to stderr.
static gq_status hip_fail(hipError_t e, const char* what, int line) {
  if (getenv("GQ_VERBOSE"))
    fprintf(stderr, "libgq: %s failed at line %d: %s\n", what, line, hipGetErrorString(e));
  return GQ_ERR_HIP;
}
#define HIP_OK(expr)                                           \
  do {                                                         \
    hipError_t e_ = (expr);                                    \
    if (e_ != hipSuccess) return hip_fail(e_, #expr, __LINE__); \
  } while (0)
// Kernel launches report through hipGetLastError, which also returns errors
// left behind by earlier, unrelated runtime calls (e.g. a not-ready stream
// query); clear it before every launch so only the launch is judged.
#define LAUNCH(...)              \
  do {                           \
    (void)hipGetLastError();     \
    hipLaunchKernelGGL(__VA_ARGS__); \
  } while (0)

namespace {

constexpr uint32_t kBlock = 256;
constexpr uint32_t kDefaultGroupLanes = 1024;  // gq_options.ticket_group == 0
constexpr uint64_t kCtrlBytes = 8192;
constexpr uint64_t kLine = 256;  // counters live on separate 256-byte lines

// Control block layout (byte offsets).
enum : uint64_t {
  OFF_AQ_HEAD = 0 * kLine,
  OFF_AQ_TAIL = 1 * kLine,
  OFF_AQ_THR = 2 * kLine,
  OFF_FQ_HEAD = 3 * kLine,
  OFF_FQ_TAIL = 4 * kLine,
  OFF_FQ_THR = 5 * kLine,
  OFF_ERR = 6 * kLine,
  OFF_STATS = 7 * kLine,   // up to 32 words
  OFF_YMC_T = 9 * kLine,
  OFF_YMC_H = 10 * kLine,
  OFF_TAKEN = 11 * kLine,  // producer/consumer driver: items taken so far
  OFF_AQ_ANN = 12 * kLine,  // G-WFQ announced slow-path request, aq
  OFF_FQ_ANN = 13 * kLine,  // and fq
};

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }
inline bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }
inline uint32_t ilog2(uint64_t x) {
  uint32_t l = 0;
  while ((1ull << l) < x) l++;
  return l;
}

struct Layout {
  uint64_t slots_aq, slots_fq, data, rec_aq, rec_fq, own_aq, own_fq, help, hint, ymc_pool, ymc_handles,
      ymc_hint, total;
};

bool kind_supported(gq_kind kind) {
  return kind == GQ_LFQ || kind == GQ_WFQ || kind == GQ_WFQ_YMC;
}

uint64_t ymc_default_cells(uint64_t n) {
  const uint64_t c = 64 * n;
  return c > (1ull << 20) ? c : (1ull << 20);
}

// G-WFQ: Lemma 4 requires R > D*k/n + 6 for the cycle range R of its tags.
bool wfq_cycle_bound_ok(uint64_t n, uint64_t k, uint64_t D) {
  const uint64_t R = 1ull << wfq::TAG_BITS;
  return D * k < (R - 6) * n;
}

gq_status plan(gq_kind kind, uint64_t n, uint32_t w, uint32_t k, const gq_options* o,
               Layout* L) {
  if (!kind_supported(kind)) return GQ_ERR_INVALID;
  if (!is_pow2(n) || n < 2 || n > (1ull << 30)) return GQ_ERR_INVALID;
  if (w != 4 && w != 8) return GQ_ERR_INVALID;
  if (k == 0 || k > (1u << 24)) return GQ_ERR_INVALID;
  if (o && ((o->flags & ~(GQ_OPT_FENCED | GQ_OPT_WFQ_TUNING)) || o->slot_mode > GQ_SLOTS_LINEAR))
    return GQ_ERR_INVALID;
  if (o && o->ticket_group &&
      (!is_pow2(o->ticket_group) || o->ticket_group < 64 || o->ticket_group > 1024))
    return GQ_ERR_INVALID;
  if (kind == GQ_WFQ) {
    if (k >= (1u << wfq::TID_BITS)) return GQ_ERR_INVALID;
    const bool tuned = o && (o->flags & GQ_OPT_WFQ_TUNING);
    const uint64_t D = tuned ? o->wfq_help_delay : 64;
    if (tuned && (D == 0 || D > 4095)) return GQ_ERR_INVALID;
    if (!wfq_cycle_bound_ok(n, k, D)) return GQ_ERR_CYCLE_BOUND;
  }
  const uint32_t mode = o ? o->slot_mode : GQ_SLOTS_LINEAR;
  const uint64_t slot_bytes = 2 * n * (mode == GQ_SLOTS_PADDED ? 128 : 8);
  uint64_t off = kCtrlBytes;
  L->slots_aq = off;
  off = align_up(off + slot_bytes, 4096);
  L->slots_fq = off;
  off = align_up(off + slot_bytes, 4096);
  L->data = off;
  off = align_up(off + n * w, 4096);
  L->rec_aq = L->rec_fq = L->own_aq = L->own_fq = L->help = L->hint = L->ymc_pool = L->ymc_handles =
      L->ymc_hint = 0;
  if (kind == GQ_WFQ) {
    L->rec_aq = off;
    off = align_up(off + (uint64_t)k * sizeof(wfq::Rec), 4096);
    L->rec_fq = off;
    off = align_up(off + (uint64_t)k * sizeof(wfq::Rec), 4096);
    L->own_aq = off;
    off = align_up(off + 2 * n * 8, 4096);
    L->own_fq = off;
    off = align_up(off + 2 * n * 8, 4096);
    L->help = off;
    off = align_up(off + (uint64_t)k * 4, 4096);
  }
  if (kind == GQ_WFQ || kind == GQ_LFQ) {
    L->hint = off;  // per-lane empty hints: k bytes for aq, then k for fq
    off = align_up(off + 2 * (uint64_t)k, 4096);
  }
  if (kind == GQ_WFQ_YMC) {
    const uint64_t cells = (o && o->ymc_pool_cells) ? o->ymc_pool_cells : ymc_default_cells(n);
    if (cells < 2 || cells > (1ull << 34)) return GQ_ERR_INVALID;
    if (k >= (1u << 31)) return GQ_ERR_INVALID;
    L->ymc_pool = off;
    off = align_up(off + cells * ymc::CELL_WORDS * 8, 4096);
    L->ymc_handles = off;
    off = align_up(off + (uint64_t)k * sizeof(ymc::Handle), 4096);
    L->ymc_hint = off;
    off = align_up(off + (uint64_t)k, 4096);
  }
  L->total = off;
  return GQ_OK;
}

// ---- initialisation --------------------------------------------------------
// Empty ring: every entry all ones (cycle = -1 mod 2^31, Safe = 1, BOT), Head
// = Tail = 0, Threshold = -1.  Full free ring: tickets 0..n-1 already
// enqueued in cycle 0 -- slots [0, n) hold <0, 1, i>, slots [n, 2n) empty --
// Head = 0, Tail = n, Threshold = its reset value (3n - 1 when k <= n).
// The init functions take the calling lane's index g0 among `stride` lanes,
// so that a whole grid (k_init_*) or one workgroup (a serving team setting
// up a per-job queue in place) can run them.  Lane 0 writes the control words.
__device__ void init_lfq_range(const gq_dev& q, uint64_t g0, uint64_t stride) {
  const uint64_t two_n = 2 * q.capacity;
  const lfq::Ring aq = lfq::make_ring(q.aq, q);
  const lfq::Ring fq = lfq::make_ring(q.fq, q);
  for (uint64_t j = g0; j < two_n; j += stride) {
    st(aq.at(j), ~0ull);
    st(fq.at(j), j < q.capacity ? lfq::e_make(0, true, (uint32_t)j) : ~0ull);
  }
  if (g0 == 0) {
    st(q.aq.head, 0ull);
    st(q.aq.tail, 0ull);
    st(q.aq.threshold, (int64_t)-1);
    st(q.fq.head, 0ull);
    st(q.fq.tail, q.capacity);
    st(q.fq.threshold, lfq::threshold_reset(q));
    st(q.err, 0ull);
    for (int s = 0; s < S_NUM; s++) st(q.stats + s, 0ull);
  }
  if (q.aq.hint)
    for (uint64_t t = g0; t < q.max_threads; t += stride) {
      q.aq.hint[t] = 0;
      q.fq.hint[t] = 0;
    }
}

__global__ void k_init_lfq(gq_dev q) {
  init_lfq_range(q, blockIdx.x * (uint64_t)blockDim.x + threadIdx.x,
                 (uint64_t)gridDim.x * blockDim.x);
}

// G-WFQ rings: entries all ones in every field (Note = Cycle = -1 mod R,
// Safe, Enq, BOT); the free ring holds <Note -1, cycle 0, Safe, Enq, i> in
// slots [0, n).  Global words <counter, NULL>; records cleared, sequence
// numbers start at 1, help counters staggered by lane.
__device__ void init_wfq_range(const gq_dev& q, uint64_t g0, uint64_t stride) {
  const uint64_t two_n = 2 * q.capacity;
  const lfq::Ring aq = lfq::make_ring(q.aq, q);
  const lfq::Ring fq = lfq::make_ring(q.fq, q);
  for (uint64_t j = g0; j < two_n; j += stride) {
    st(aq.at(j), ~0ull);
    st(fq.at(j), j < q.capacity ? wfq::e_make(wfq::TAG_MASK, 0, true, true, (uint32_t)j) : ~0ull);
    st(q.aq.owner + j, 0ull);
    st(q.fq.owner + j, 0ull);
  }
  wfq::Rec* ra = (wfq::Rec*)q.aq.records;
  wfq::Rec* rf = (wfq::Rec*)q.fq.records;
  for (uint64_t t = g0; t < q.max_threads; t += stride) {
    for (wfq::Rec* R : {ra + t, rf + t}) {
      st(&R->local, 0ull);
      st(&R->init, 0ull);
      st(&R->index, 0ull);
      st(&R->req, 0ull);
      st(&R->next_seq, 1ull);
    }
    // The lanes of a wavefront share one phase of the help step (count
    // (t / 64) mod D; wavefronts are staggered): together they inspect 64
    // peers once every D operations, their loads in flight at once.  With
    // a phase per lane, one lane of every wavefront would run the help
    // step on every operation, and its load of a peer's request word would
    // stand in every operation's dependency chain.
    const uint32_t peer = (uint32_t)((t + 1) % q.max_threads);
    st(q.help_ctr + t, (peer << 12) | (uint32_t)((t / 64) % (q.help_delay ? q.help_delay : 1)));
    q.aq.hint[t] = 0;
    q.fq.hint[t] = 0;
  }
  if (g0 == 0) {
    st(q.aq.head, 0ull);
    st(q.aq.tail, 0ull);
    st(q.aq.threshold, (int64_t)-1);
    st(q.fq.head, 0ull);
    st(q.fq.tail, q.capacity << wfq::TID_BITS);
    st(q.fq.threshold, lfq::threshold_reset(q));
    st(q.aq.announce, 0ull);
    st(q.fq.announce, 0ull);
    st(q.err, 0ull);
    for (int s = 0; s < S_NUM; s++) st(q.stats + s, 0ull);
  }
}

__global__ void k_init_wfq(gq_dev q) {
  init_wfq_range(q, blockIdx.x * (uint64_t)blockDim.x + threadIdx.x,
                 (uint64_t)gridDim.x * blockDim.x);
}

// G-WFQ-YMC: every cell word 0 (val, enq and deq empty), T = H = 1 (cell id 0 doubles as
// "no id"), handles cleared with peers staggered by lane.
__global__ void k_init_ymc(gq_dev q) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t g0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t words = (uint64_t)ymc::CELL_WORDS * q.ymc_pool_cells;  // val, enq, deq arrays
  for (uint64_t i = g0; i < words; i += stride) st(q.ymc_cells + i, 0ull);
  ymc::Handle* hd = (ymc::Handle*)q.ymc_handles;
  for (uint64_t t = g0; t < q.max_threads; t += stride) {
    st(&hd[t].enq_val, 0ull);
    st(&hd[t].enq_state, 0ull);
    st(&hd[t].deq_id, 0ull);
    st(&hd[t].deq_state, 0ull);
    st(&hd[t].enq_help_id, 0ull);
    const uint32_t peer = (uint32_t)((t + 1) % q.max_threads);
    hd[t].enq_peer = peer;
    hd[t].deq_peer = peer;
    q.ymc_hint[t] = 0;
  }
  if (g0 == 0) {
    st(q.ymc_ctr, 1ull);
    st(q.ymc_ctr + 32, 1ull);
    st(q.err, 0ull);
    for (int s = 0; s < S_NUM; s++) st(q.stats + s, 0ull);
  }
}

uint32_t grid_for(uint64_t work, uint32_t block, uint32_t cap) {
  uint64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

// ---- batched operations ----------------------------------------------------
template <int KIND>
__global__ void k_enqueue_batch(gq_dev q, const void* items, uint64_t m, uint8_t* status,
                                uint64_t* nok) {
  const uint64_t gtid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t launched = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t stride = launched < q.max_threads ? launched : q.max_threads;
  uint64_t ok = 0;
  uint32_t cf = 0;
  for (uint64_t i = gtid; gtid < stride && i < m; i += stride) {
    const uint64_t item = q.item_width == 8 ? ((const uint64_t*)items)[i]
                                            : (uint64_t)((const uint32_t*)items)[i];
    const int s = gq_enqueue_k<KIND>(q, item, (uint32_t)gtid, cf);
    if (status) status[i] = (uint8_t)s;
    ok += s == GQ_OK;
  }
  wave_add(q.stats + S_OK_ENQ, ok);
  wave_add(q.stats + S_CAS_FAIL, cf);
  if (nok) wave_add(nok, ok);
}

template <int KIND>
__global__ void k_dequeue_batch(gq_dev q, void* out, uint64_t m, uint8_t* status, uint64_t* nok) {
  const uint64_t gtid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t launched = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t stride = launched < q.max_threads ? launched : q.max_threads;
  uint64_t ok = 0;
  uint32_t cf = 0;
  for (uint64_t i = gtid; gtid < stride && i < m; i += stride) {
    uint64_t v = 0;
    const int s = gq_dequeue_k<KIND>(q, &v, (uint32_t)gtid, cf);
    if (s != GQ_OK) v = 0;
    if (q.item_width == 8) ((uint64_t*)out)[i] = v;
    else ((uint32_t*)out)[i] = (uint32_t)v;
    if (status) status[i] = (uint8_t)s;
    ok += s == GQ_OK;
  }
  wave_add(q.stats + S_OK_DEQ, ok);
  wave_add(q.stats + S_CAS_FAIL, cf);
  if (nok) wave_add(nok, ok);
}

// Workgroup-uniform batches: every lane of a workgroup steps through the
// items together (strides of the whole launch); lanes past the end take part
// with ROLE_NONE so the group's ticket FAAs stay uniform.  The launch has at
// most max_threads lanes, so lane ids are valid tids.
template <int KIND>
__global__ __launch_bounds__(1024) void k_enqueue_batch_group(gq_dev q, const void* items,
                                                              uint64_t m, uint8_t* status,
                                                              uint64_t* nok) {
  __shared__ GroupLds lds;
  uint32_t par = 0;
  const uint64_t gtid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t ok = 0;
  uint32_t cf = 0;
  for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x; base < m; base += stride) {
    const uint64_t i = base + threadIdx.x;
    const bool act = i < m;
    uint64_t item = 0;
    if (act) item = q.item_width == 8 ? ((const uint64_t*)items)[i]
                                      : (uint64_t)((const uint32_t*)items)[i];
    const int s = gq_group_op_k<KIND>(q, act ? ROLE_ENQ : ROLE_NONE, item, (uint32_t)gtid, cf,
                                      lds, par);
    if (act) {
      if (status) status[i] = (uint8_t)s;
      ok += s == GQ_OK;
    }
  }
  wave_add(q.stats + S_OK_ENQ, ok);
  wave_add(q.stats + S_CAS_FAIL, cf);
  if (nok) wave_add(nok, ok);
}

template <int KIND>
__global__ __launch_bounds__(1024) void k_dequeue_batch_group(gq_dev q, void* out, uint64_t m,
                                                              uint8_t* status, uint64_t* nok) {
  __shared__ GroupLds lds;
  uint32_t par = 0;
  const uint64_t gtid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t ok = 0;
  uint32_t cf = 0;
  for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x; base < m; base += stride) {
    const uint64_t i = base + threadIdx.x;
    const bool act = i < m;
    uint64_t v = 0;
    const int s = gq_group_op_k<KIND>(q, act ? ROLE_DEQ : ROLE_NONE, v, (uint32_t)gtid, cf, lds,
                                      par);
    if (act) {
      if (s != GQ_OK) v = 0;
      if (q.item_width == 8) ((uint64_t*)out)[i] = v;
      else ((uint32_t*)out)[i] = (uint32_t)v;
      if (status) status[i] = (uint8_t)s;
      ok += s == GQ_OK;
    }
  }
  wave_add(q.stats + S_OK_DEQ, ok);
  wave_add(q.stats + S_CAS_FAIL, cf);
  if (nok) wave_add(nok, ok);
}

// ---- history recording -----------------------------------------------------
struct Rec {
  gq_history h;
  bool on;
  __device__ __forceinline__ void put(uint64_t g, uint32_t r, int op, int s, uint64_t val,
                                      uint64_t t0, uint64_t t1) const {
    if (!on || r >= h.per_lane) return;
    const uint64_t i = g * h.per_lane + r;
    h.val[i] = val;
    h.call[i] = t0;
    h.ret[i] = t1;
    h.opst[i] = (uint8_t)(op | (s << 1));
  }
};

// The end stamp is taken once every memory access of the operation has
// completed.  With the atomic hand-off every access that another lane reads
// is a device-coherent atomic, visible once complete, so the lane only waits
// for its outstanding accesses -- exactly what the unrecorded kernels'
// operations do; the fenced hand-off's plain payload stores need an
// agent-scope release before they are visible.
__device__ __forceinline__ uint64_t end_stamp(const gq_dev& q) {
  if (q.flags & GQ_OPT_FENCED) fence_rel();
  else wait_mem();
  return stamp();
}

// ---- mixed workload --------------------------------------------------------
// One lane's part of the mixed workload on queue q: `ops` operations, op r an
// enqueue iff the top bit of r(seed, (g << 32) | r) is 0, tried once.  g is
// the lane's global id (tokens and draws), tid its id within the queue.
// Per-lane tallies of the mixed workload: counts and the wrapping sums of v
// and v * v of the items moved (the multiset checksums of gq_run_mix).  The
// dequeued items' sums accumulate per operation; the enqueued items of lane g
// are its tokens (g << 32) | j, j = 1..c, whose sums have a closed form in c:
// with x = g << 32, sum = c x + c(c+1)/2 and sum of squares =
// c x^2 + x c(c+1) + c(c+1)(2c+1)/6, both mod 2^64 (the divisions are exact
// on the integers, so they are taken before the wrap).
__device__ __forceinline__ void token_sums(uint64_t g, uint64_t c, uint64_t& s1, uint64_t& s2) {
  const uint64_t x = g << 32;
  const uint64_t tri = (c & 1) ? c * ((c + 1) >> 1) : (c >> 1) * (c + 1);  // c(c+1)/2
  // c(c+1)(2c+1)/6 = tri * (2c+1) / 3: one of tri and 2c+1 is a multiple of 3
  const uint64_t sq = (tri % 3 == 0) ? (tri / 3) * (2 * c + 1) : tri * ((2 * c + 1) / 3);
  s1 = c * x + tri;
  s2 = c * x * x + 2 * x * tri + sq;
}

struct MixTally {
  uint32_t ok_e = 0, ok_d = 0, full = 0, empty = 0, cf = 0;
  uint64_t s1d = 0, s2d = 0;
  __device__ __forceinline__ void enq(int s, uint64_t) {
    if (s == GQ_OK) ok_e++;
    else full++;
  }
  __device__ __forceinline__ void deq(int s, uint64_t v) {
    if (s == GQ_OK) {
      ok_d++;
      s1d += v;
      s2d += v * v;
    } else {
      empty++;
    }
  }
  // counts[0..7] += {ok_enq, ok_deq, full, empty, S1_deq, S2_deq, S1_enq, S2_enq}
  // for lane g, whose tokens are (g << 32) | j
  __device__ __forceinline__ void flush(uint64_t* counts, uint64_t* stats, uint64_t g) const {
    uint64_t s1e, s2e;
    token_sums(g, ok_e, s1e, s2e);
    wave_add(counts + 0, ok_e);
    wave_add(counts + 1, ok_d);
    wave_add(counts + 2, full);
    wave_add(counts + 3, empty);
    wave_add(counts + 4, s1d);
    wave_add(counts + 5, s2d);
    wave_add(counts + 6, s1e);
    wave_add(counts + 7, s2e);
    wave_add(stats + S_CAS_FAIL, cf);
  }
  // The same sums for a whole workgroup, whose lanes all arrive here
  // together: each wavefront's total goes into the workgroup's `acc` words
  // (LDS, zeroed at kernel start), then one lane per counter adds it to the
  // device word.  With one device atomic per wavefront and counter, the
  // thousands of wavefronts of a launch ending together queued on the same
  // few words (one L2 line) for a tenth of a G-WFQ launch.
  __device__ __forceinline__ void flush_group(uint64_t* counts, uint64_t* stats, uint64_t g,
                                              uint64_t* acc) const {
    add_to(acc, g);
    __syncthreads();
    flush_acc(acc, counts, stats);
  }
  // This wavefront's sums (all its lanes present) added into the LDS words.
  __device__ __forceinline__ void add_to(uint64_t* acc, uint64_t g) const {
    uint64_t s1e, s2e;
    token_sums(g, ok_e, s1e, s2e);
    const uint64_t v[9] = {ok_e, ok_d, full, empty, s1d, s2d, s1e, s2e, cf};
    const bool lead = (threadIdx.x & 63) == 0;
#pragma unroll
    for (int i = 0; i < 9; i++) {
      const uint64_t w = wave_sum(v[i]);
      if (lead && w) atomicAdd((unsigned long long*)&acc[i], (unsigned long long)w);
    }
  }
  // The workgroup's LDS sums to the device words (after a barrier).
  __device__ __forceinline__ static void flush_acc(const uint64_t* acc, uint64_t* counts,
                                                   uint64_t* stats) {
    if (threadIdx.x < 9 && acc[threadIdx.x])
      faa(threadIdx.x < 8 ? counts + threadIdx.x : stats + S_CAS_FAIL, acc[threadIdx.x]);
  }
};

// The queue's device view with every control word addressed from one base.
// The control words sit at fixed offsets of the queue's allocation (OFF_*),
// so the compiler can reach them all as base + immediate offset instead of
// holding a 64-bit address per word in scalar registers: G-WFQ's group
// kernel otherwise needs more scalar registers than a wavefront has, parks
// the overflow in vector-register lanes and reloads it with VALU
// instructions on every operation.  LIN pins the linear slot layout (the
// caller checks that the queue uses it), which removes the layout branches
// from every slot access.  Valid for queues made by gq_create only.
template <int KIND, bool LIN>
__device__ __forceinline__ gq_dev kernel_view(const gq_dev& q) {
  gq_dev l = q;
  uint8_t* base = (uint8_t*)q.err - OFF_ERR;
  l.aq.head = (uint64_t*)(base + OFF_AQ_HEAD);
  l.aq.tail = (uint64_t*)(base + OFF_AQ_TAIL);
  l.aq.threshold = (int64_t*)(base + OFF_AQ_THR);
  l.fq.head = (uint64_t*)(base + OFF_FQ_HEAD);
  l.fq.tail = (uint64_t*)(base + OFF_FQ_TAIL);
  l.fq.threshold = (int64_t*)(base + OFF_FQ_THR);
  l.stats = (uint64_t*)(base + OFF_STATS);
  if (KIND == GQ_WFQ) {
    l.aq.announce = (uint64_t*)(base + OFF_AQ_ANN);
    l.fq.announce = (uint64_t*)(base + OFF_FQ_ANN);
  }
  if (LIN) l.slot_mode = GQ_SLOTS_LINEAR;
  return l;
}

template <int KIND, bool REC>
__device__ __forceinline__ MixTally mix_lane(const gq_dev& q, uint64_t g, uint32_t tid,
                                             uint64_t seed, uint32_t ops, uint32_t* lane_enq,
                                             const Rec& rec) {
  MixTally t;
  for (uint32_t r = 0; r < ops; r++) {
    const bool is_enq = (splitmix64(seed, (g << 32) | r) >> 63) == 0;
    const uint64_t t0 = REC ? stamp() : 0;
    uint64_t v;
    int s;
    if (is_enq) {
      v = (g << 32) | (uint64_t)(t.ok_e + 1);
      s = gq_enqueue_k<KIND>(q, v, tid, t.cf);
      t.enq(s, v);
    } else {
      v = 0;
      s = gq_dequeue_k<KIND>(q, &v, tid, t.cf);
      if (s != GQ_OK) v = 0;
      t.deq(s, v);
    }
    if (REC) rec.put(g, r, is_enq ? 0 : 1, s, v, t0, end_stamp(q));
  }
  if (REC && rec.h.count) rec.h.count[g] = ops;
  if (lane_enq) lane_enq[g] = t.ok_e;
  return t;
}

template <int KIND, bool REC>
__global__ __launch_bounds__(256) void k_mix(gq_dev q, uint64_t seed, uint32_t ops,
                                             uint64_t* counts, uint32_t* lane_enq, Rec rec) {
  __shared__ uint64_t acc[9];
  if (threadIdx.x < 9) acc[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const MixTally t = mix_lane<KIND, REC>(q, g, (uint32_t)g, seed, ops, lane_enq, rec);
  t.flush_group(counts, q.stats, g, acc);
}

// The same workload with workgroup-aggregated first tickets: every lane of
// the workgroup performs its op r together with the others (group_op), so
// each ticket counter sees one FAA per workgroup per phase.  Same draws,
// tokens and counts as k_mix.
template <int KIND, bool REC, bool LIN>
__device__ __forceinline__ void mix_group_body(const gq_dev& q0, uint64_t seed, uint32_t ops,
                                               uint64_t* counts, uint32_t* lane_enq,
                                               const Rec& rec, GroupLds& lds, uint64_t* acc) {
  const gq_dev q = kernel_view<KIND, LIN>(q0);
  uint32_t par = 0;
  const uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  // G-WFQ: the lane's help step state stays in a register for the run
  const bool own_help = KIND == GQ_WFQ && g < q.max_threads;
  uint32_t help = own_help ? wfq::help_load(q, (uint32_t)g) : 0;
  // per-lane counts never exceed `ops` (< 2^32): 32-bit registers suffice
  MixTally t;
  for (uint32_t r = 0; r < ops; r++) {
    const bool is_enq = (splitmix64(seed, (g << 32) | r) >> 63) == 0;
    const uint64_t t0 = REC ? stamp() : 0;
    uint64_t v = is_enq ? ((g << 32) | (uint64_t)(t.ok_e + 1)) : 0;
    const int s = gq_group_op_k<KIND>(q, is_enq ? ROLE_ENQ : ROLE_DEQ, v, (uint32_t)g, t.cf, lds,
                                      par, KIND == GQ_WFQ ? &help : nullptr);
    if (is_enq) {
      t.enq(s, v);
    } else {
      if (s != GQ_OK) v = 0;
      t.deq(s, v);
    }
    if (REC) rec.put(g, r, is_enq ? 0 : 1, s, v, t0, end_stamp(q));
  }
  if (REC && rec.h.count) rec.h.count[g] = ops;
  if (own_help) wfq::help_store(q, (uint32_t)g, help);
  if (lane_enq) lane_enq[g] = t.ok_e;
  t.flush_group(counts, q.stats, g, acc);
}

template <int KIND, bool REC, bool LIN>
__global__ __launch_bounds__(1024) void k_mix_group(gq_dev q, uint64_t seed, uint32_t ops,
                                                    uint64_t* counts, uint32_t* lane_enq, Rec rec) {
  __shared__ GroupLds lds;
  __shared__ uint64_t acc[9];
  if (threadIdx.x < 9) acc[threadIdx.x] = 0;
  __syncthreads();
  mix_group_body<KIND, REC, LIN>(q, seed, ops, counts, lane_enq, rec, lds, acc);
}

// G-LFQ's copy of the group kernel, compiled for 8 wavefronts per SIMD (at
// most 64 VGPRs; it needs 67 otherwise, with a few bytes spilled at the cap):
// the sweep's largest grid, 2^19 lanes, is then resident all at once instead
// of in two rounds of workgroups (measured 2.41 -> 2.21 ms per 2^26 ops).
// G-WFQ and G-WFQ-YMC need 100-126 VGPRs; capped at 64 (272 and 168 bytes of
// spills per lane), their 2^19 resident lanes are slower than 2^18 lanes at 4
// wavefronts per SIMD (2.16 -> 2.84 ms and 1.72 -> 2.12 ms).
template <bool REC, bool LIN>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_mix_group_lfq(
    gq_dev q, uint64_t seed, uint32_t ops, uint64_t* counts, uint32_t* lane_enq, Rec rec) {
  __shared__ GroupLds lds;
  __shared__ uint64_t acc[9];
  if (threadIdx.x < 9) acc[threadIdx.x] = 0;
  __syncthreads();
  mix_group_body<GQ_LFQ, REC, LIN>(q, seed, ops, counts, lane_enq, rec, lds, acc);
}

// Dequeue for the level-synchronous BFS loops (queue BFS, serving teams).
// A level's dequeues end at its first EMPTY and nothing is enqueued into the
// level's queue meanwhile, so G-LFQ's per-lane empty hints (for lanes that
// poll a queue others refill) would only add a look before every lane's
// first ticket two levels later: G-LFQ is called without a lane id.
template <int KIND>
__device__ __forceinline__ int level_dequeue(const gq_dev& q, uint64_t* v, uint32_t tid,
                                             uint32_t& cf) {
  if constexpr (KIND == GQ_LFQ) return lfq::dequeue(q, v, cf);
  else return gq_dequeue_k<KIND>(q, v, tid, cf);
}

// Many independent queues in one launch: wavefront w works on queue
// wave_q[w]; lane ids inside a queue start at q_lane0[queue].  The seed is
// read from device memory so that a captured graph can advance it.
template <int KIND, bool REC>
__global__ __launch_bounds__(256) void k_multi_mix(const gq_dev* qs, const uint32_t* wave_q,
                                                   const uint32_t* q_lane0, const uint64_t* seed,
                                                   uint32_t ops, uint64_t* counts, Rec rec) {
  __shared__ uint64_t acc[9];
  if (threadIdx.x < 9) acc[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint32_t qi = __builtin_amdgcn_readfirstlane(wave_q[g / 64]);
  const gq_dev q = qs[qi];
  const uint32_t tid = (uint32_t)(g - q_lane0[qi]);
  const MixTally t = mix_lane<KIND, REC>(q, g, tid, ld(seed), ops, nullptr, rec);
  // The wavefronts of the workgroup's first queue (all of them unless the
  // workgroup straddles queues) sum into LDS and flush once; the others flush
  // their own sums.
  const uint32_t q0 = __builtin_amdgcn_readfirstlane(wave_q[blockIdx.x * (blockDim.x / 64)]);
  if (qi == q0) t.add_to(acc, g);
  else t.flush(counts + 8 * (uint64_t)qi, q.stats, g);
  __syncthreads();
  MixTally::flush_acc(acc, counts + 8 * (uint64_t)q0, qs[q0].stats);
}

__global__ void k_seed(uint64_t* seed, uint64_t value, uint32_t bump) {
  if (blockIdx.x == 0 && threadIdx.x == 0) st(seed, bump ? ld(seed) + 1 : value);
}

// ---- balanced workload -----------------------------------------------------
template <int KIND, bool REC>
__global__ __launch_bounds__(256) void k_balanced(gq_dev q, uint32_t rounds, uint64_t* counts,
                                                  Rec rec) {
  const uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint64_t seq = 0, ok_e = 0, ok_d = 0, full = 0, empty = 0;
  uint32_t cf = 0, r = 0;
  for (uint32_t k = 0; k < rounds; k++) {
    uint64_t t0 = REC ? stamp() : 0;
    uint64_t v = (g << 32) | (seq + 1);
    int s = gq_enqueue_k<KIND>(q, v, (uint32_t)g, cf);
    if (s == GQ_OK) { seq++; ok_e++; } else full++;
    if (REC) rec.put(g, r, 0, s, v, t0, end_stamp(q));
    r++;
    t0 = REC ? stamp() : 0;
    v = 0;
    s = gq_dequeue_k<KIND>(q, &v, (uint32_t)g, cf);
    if (s == GQ_OK) ok_d++; else { empty++; v = 0; }
    if (REC) rec.put(g, r, 1, s, v, t0, end_stamp(q));
    r++;
  }
  if (REC && rec.h.count) rec.h.count[g] = r;
  wave_add(counts + 0, ok_e);
  wave_add(counts + 1, ok_d);
  wave_add(counts + 2, full);
  wave_add(counts + 3, empty);
  wave_add(q.stats + S_CAS_FAIL, cf);
}

// ---- producer / consumer workload -----------------------------------------
template <int KIND, bool REC>
__global__ void k_prodcons(gq_dev q, uint64_t seed, const uint8_t* role, uint32_t quota,
                           uint64_t target, uint32_t log2_inv_p, uint32_t token_mode,
                           uint32_t jitter, uint64_t max_rounds, uint64_t limit_ticks,
                           uint64_t* taken, uint64_t* counts, Rec rec) {
  const uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const bool producer = role[g] == 0;
  uint64_t seq = 0, ok_e = 0, ok_d = 0, full = 0, empty = 0;
  uint64_t s1d = 0, s2d = 0, s1e = 0, s2e = 0;
  uint32_t cf = 0, r = 0;
  const uint64_t t_start = limit_ticks ? stamp() : 0;
  for (uint64_t k = 0;; k++) {
    if (producer ? seq >= quota : ld(taken) >= target) break;
    if (k >= max_rounds || (limit_ticks && (k & 63) == 0 && stamp() - t_start > limit_ticks)) {
      latch_error(q.err, (uint64_t)(-GQ_ERR_DEVICE));
      break;
    }
    const uint64_t draw = splitmix64(seed, (g << 32) | (k & 0xFFFFFFFFull));
    if (jitter) pause((uint32_t)(draw & 0xFFFF) % (jitter + 1));
    const bool active = log2_inv_p == 0 || (draw >> (64 - log2_inv_p)) == 0;
    if (!active) continue;
    const uint64_t t0 = REC ? stamp() : 0;
    if (producer) {
      const uint64_t v = token_mode == 0 ? ((g << 32) | (seq + 1)) : ((g << 20) | seq);
      const int s = gq_enqueue_k<KIND>(q, v, (uint32_t)g, cf);
      if (s == GQ_OK) {
        seq++;
        ok_e++;
        s1e += v;
        s2e += v * v;
      } else {
        full++;
      }
      if (REC) rec.put(g, r++, 0, s, v, t0, end_stamp(q));
    } else {
      uint64_t v = 0;
      const int s = gq_dequeue_k<KIND>(q, &v, (uint32_t)g, cf);
      if (s == GQ_OK) {
        ok_d++;
        s1d += v;
        s2d += v * v;
        faa(taken, 1ull);
      } else {
        empty++;
        v = 0;
      }
      if (REC) rec.put(g, r++, 1, s, v, t0, end_stamp(q));
    }
  }
  if (REC && rec.h.count) rec.h.count[g] = r;
  wave_add(counts + 0, ok_e);
  wave_add(counts + 1, ok_d);
  wave_add(counts + 2, full);
  wave_add(counts + 3, empty);
  wave_add(counts + 4, s1d);
  wave_add(counts + 5, s2d);
  wave_add(counts + 6, s1e);
  wave_add(counts + 7, s2e);
  wave_add(q.stats + S_CAS_FAIL, cf);
}

// ---- fixed-duration runs -----------------------------------------------------
// Every lane reads the shared start time (the first lane to arrive sets it),
// then works until start + warmup + window.  The clock is the scalar 100 MHz
// counter, so all lanes of a wavefront leave the loop together.  Besides the
// window counts the kernel keeps the whole run's books for the oracle: OK
// counts, the dequeued items' wrapping sums of v and v * v, the enqueued
// tokens' sums in closed form (token_sums), per-lane enqueue counts, and --
// with a history -- every operation; a lane whose history is full stops (all
// lanes of a wavefront reach that point together).
template <int KIND, bool REC>
__global__ __launch_bounds__(256) void k_timed(gq_dev q, uint32_t mode, uint32_t prod_waves,
                                               uint64_t warm_ticks, uint64_t win_ticks,
                                               uint64_t* counts, uint64_t* ctl,
                                               uint32_t* lane_enq, Rec rec) {
  const uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint64_t start = ld(ctl);
  if (start == 0) {
    uint64_t z = 0;
    const uint64_t now = stamp();
    start = cas(ctl, z, now) ? now : z;
  }
  const uint64_t w0 = start + warm_ticks, w1 = w0 + win_ticks;
  const bool producer = (g >> 6) < prod_waves;
  uint32_t seq = 0, ok_e = 0, ok_d = 0, all_d = 0, full = 0, empty = 0, cf = 0;
  uint64_t s1d = 0, s2d = 0;
  uint32_t r = 0;
  for (;; r++) {
    if (REC && r >= rec.h.per_lane) break;
    const bool enq = mode == 0 ? (r & 1) == 0 : producer;
    const uint64_t t0 = REC ? stamp() : 0;
    int st;
    uint64_t v = 0;
    if (enq) {
      v = (g << 32) | (uint64_t)(seq + 1);
      st = gq_enqueue_k<KIND>(q, v, (uint32_t)g, cf);
      if (st == GQ_OK) seq++;
    } else {
      st = gq_dequeue_k<KIND>(q, &v, (uint32_t)g, cf);
      if (st == GQ_OK) {
        all_d++;
        s1d += v;
        s2d += v * v;
      } else {
        v = 0;
      }
    }
    const uint64_t t = REC ? end_stamp(q) : stamp();
    if (REC) rec.put(g, r, enq ? 0 : 1, st, v, t0, t);
    if (st == GQ_OK) {
      if (t >= w0 && t < w1) {
        if (enq) ok_e++; else ok_d++;
      }
    } else {
      if (enq) full++; else empty++;
    }
    if (t >= w1) {
      r++;
      break;
    }
  }
  if (REC && rec.h.count) rec.h.count[g] = r;
  if (lane_enq) lane_enq[g] = seq;
  uint64_t s1e, s2e;
  token_sums(g, seq, s1e, s2e);
  wave_add(counts + 0, ok_e);
  wave_add(counts + 1, ok_d);
  wave_add(counts + 2, full);
  wave_add(counts + 3, empty);
  wave_add(counts + 4, s1d);
  wave_add(counts + 5, s2d);
  wave_add(counts + 6, s1e);
  wave_add(counts + 7, s2e);
  wave_add(counts + 8, seq);
  wave_add(counts + 9, all_d);
  wave_add(q.stats + S_CAS_FAIL, cf);
}

// ---- scripted small runs ---------------------------------------------------
template <int KIND>
__global__ void k_script(gq_dev q, uint32_t lanes, uint32_t spread, const uint8_t* ops,
                         const uint64_t* args, const uint16_t* pauses, const uint32_t* n_ops,
                         uint32_t max_ops, Rec rec) {
  uint32_t g;
  if (spread) {
    if (threadIdx.x != 0) return;  // one active lane per wavefront
    g = blockIdx.x;
  } else {
    g = threadIdx.x;
  }
  if (g >= lanes) return;
  uint32_t cf = 0;
  for (uint32_t r = 0; r < n_ops[g]; r++) {
    const uint64_t i = (uint64_t)g * max_ops + r;
    pause(pauses[i]);
    const uint64_t t0 = stamp();
    uint64_t v = args[i];
    int s;
    if (ops[i] == 0) {
      s = gq_enqueue_k<KIND>(q, v, g, cf);
    } else {
      v = 0;
      s = gq_dequeue_k<KIND>(q, &v, g, cf);
      if (s != GQ_OK) v = 0;
    }
    rec.put(g, r, ops[i], s, v, t0, end_stamp(q));
  }
  if (rec.h.count) rec.h.count[g] = n_ops[g];
}

// ---- roofline probes ---------------------------------------------------------
__global__ void k_probe_faa(uint64_t* ctr, uint32_t iters, uint32_t per_lane, uint32_t ncounters,
                            uint32_t spacing_words, uint64_t* sink) {
  const uint64_t w = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) / 64;
  uint64_t* c = ctr + (w % ncounters) * spacing_words;
  uint64_t acc = 0;
  for (uint32_t i = 0; i < iters; i++) {
    if (per_lane) acc += faa(c, 1ull);
    else acc += wave_faa(c, 1ull);
  }
  if (acc == 0x5555555555555555ull) sink[0] = acc;
}

__global__ void k_probe_cas(uint64_t* slots, uint64_t nslots, uint32_t stride_words,
                            uint32_t iters, uint64_t* sink) {
  const uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t nl = (uint64_t)gridDim.x * blockDim.x;
  uint64_t acc = 0;
  for (uint32_t i = 0; i < iters; i++) {
    const uint64_t t = (g + i * nl) % nslots;
    uint64_t* p = slots + t * stride_words;
    uint64_t e = ld(p);
    if (!cas(p, e, e + 1)) acc++;
  }
  if (acc == 0x5555555555555555ull) sink[0] = acc;
}

__global__ void k_probe_copy(uint64_t* dst, const uint64_t* src, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * 2;
  for (uint64_t i = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) * 2; i < n; i += stride) {
    if (i + 1 < n) {
      const ulonglong2 v = *(const ulonglong2*)(src + i);
      *(ulonglong2*)(dst + i) = v;
    } else {
      dst[i] = src[i];
    }
  }
}

__global__ void k_probe_fence(uint64_t* lines, uint32_t iters, uint32_t mode) {
  const uint64_t w = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) / 64;
  uint64_t* p = lines + w * 32;  // one 256-byte line per wavefront
  for (uint32_t i = 0; i < iters; i++) {
    if (mode & 1) fence_rel();
    if ((threadIdx.x & 63) == 0) st(p, (uint64_t)i);
    if (mode & 2) fence_acq();
  }
}

__global__ void k_sink() {}

#include "gq_bfs.inc"

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
struct gq_queue {
  gq_kind kind;
  uint64_t n;
  uint32_t w, k;
  gq_options opt;
  char* buf;
  uint64_t bytes;
  bool owns;
  gq_dev dev;
  Layout L;
};

static hipStream_t S(void* s) { return (hipStream_t)s; }

static gq_status launch_init(gq_queue* q, hipStream_t s) {
  const uint64_t slots = 2 * q->n > q->k ? 2 * q->n : q->k;
  const uint32_t grid = grid_for(slots, kBlock, 4096);
  switch (q->kind) {
    case GQ_LFQ:
      LAUNCH(k_init_lfq, dim3(grid), dim3(kBlock), 0, s, q->dev);
      break;
    case GQ_WFQ:
      LAUNCH(k_init_wfq, dim3(grid), dim3(kBlock), 0, s, q->dev);
      break;
    case GQ_WFQ_YMC:
      LAUNCH(k_init_ymc, dim3(8192), dim3(kBlock), 0, s, q->dev);
      break;
    default:
      return GQ_ERR_INVALID;
  }
  HIP_OK(hipGetLastError());
  return GQ_OK;
}

// Batches run on at most max_threads lanes (grid-stride over the items): the
// queues' empty detection and G-WFQ's records are sized for that many lanes.
static uint32_t batch_grid(const gq_queue* q, uint64_t m) {
  uint32_t cap = (q->k + kBlock - 1) / kBlock;
  if (cap < 1) cap = 1;
  if (cap > 8192) cap = 8192;
  return grid_for(m, kBlock, cap);
}

// Workgroup-ticket batches: workgroups of the queue's ticket group (at most
// max_threads lanes in all, capped like the per-wavefront form); 0 when the
// group is a single wavefront or max_threads is too small for a group.
static uint32_t batch_group_block(const gq_queue* q, uint64_t m, uint32_t* grid) {
  uint32_t b = q->dev.group_lanes;
  while (b > 64 && b > q->k) b >>= 1;
  if (b <= 64) return 0;
  uint64_t g = (m + b - 1) / b;
  uint64_t cap = q->k / b;
  if (cap > 8192ull * kBlock / b) cap = 8192ull * kBlock / b;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  *grid = (uint32_t)g;
  return b;
}

template <int KIND>
static void launch_enq(gq_queue* q, const void* items, uint64_t m, uint8_t* st, uint64_t* nok,
                       hipStream_t s) {
  uint32_t ggrid = 0;
  const uint32_t gb = batch_group_block(q, m, &ggrid);
  if (gb) {
    LAUNCH(k_enqueue_batch_group<KIND>, dim3(ggrid), dim3(gb), 0, s, q->dev, items, m, st, nok);
    return;
  }
  const uint32_t grid = batch_grid(q, m);
  LAUNCH(k_enqueue_batch<KIND>, dim3(grid), dim3(kBlock), 0, s, q->dev, items, m, st,
                     nok);
}
template <int KIND>
static void launch_deq(gq_queue* q, void* out, uint64_t m, uint8_t* st, uint64_t* nok,
                       hipStream_t s) {
  uint32_t ggrid = 0;
  const uint32_t gb = batch_group_block(q, m, &ggrid);
  if (gb) {
    LAUNCH(k_dequeue_batch_group<KIND>, dim3(ggrid), dim3(gb), 0, s, q->dev, out, m, st, nok);
    return;
  }
  const uint32_t grid = batch_grid(q, m);
  LAUNCH(k_dequeue_batch<KIND>, dim3(grid), dim3(kBlock), 0, s, q->dev, out, m, st,
                     nok);
}

// The exported functions below were declared extern "C" in gq.h/gq_bench.h,
// so their definitions keep C linkage; helper templates stay C++.

const char* gq_status_str(gq_status s) {
  switch (s) {
    case GQ_OK: return "ok";
    case GQ_EMPTY: return "empty";
    case GQ_FULL: return "full";
    case GQ_ERR_INVALID: return "invalid argument";
    case GQ_ERR_NOMEM: return "out of device memory or buffer too small";
    case GQ_ERR_HIP: return "HIP runtime error";
    case GQ_ERR_RESIDENCY: return "lanes cannot all be co-resident";
    case GQ_ERR_CYCLE_BOUND: return "cycle-tag bound R > D*k/n + 6 violated";
    case GQ_ERR_POOL_EXHAUSTED: return "G-WFQ-YMC cell pool exhausted";
    case GQ_ERR_DEVICE: return "device-side invariant or bound violated";
    case GQ_ERR_TOO_LARGE: return "size beyond the entry point's fixed maximum";
  }
  return "unknown status";
}

gq_status gq_required_bytes(gq_kind kind, uint64_t capacity, uint32_t item_width,
                            uint32_t max_threads, const gq_options* opts, uint64_t* bytes) {
  if (!bytes) return GQ_ERR_INVALID;
  Layout L;
  gq_status st = plan(kind, capacity, item_width, max_threads, opts, &L);
  if (st != GQ_OK) return st;
  *bytes = L.total;
  return GQ_OK;
}

// The device view of a queue laid out by plan() at `buf` (device memory).
static gq_dev make_dev(gq_kind kind, uint64_t capacity, uint32_t item_width,
                       uint32_t max_threads, const gq_options& o, char* buf,
                       const Layout& L) {
  gq_dev d;
  memset(&d, 0, sizeof(d));
  d.kind = kind;
  d.item_width = item_width;
  d.log2_cap = ilog2(capacity);
  d.slot_mode = o.slot_mode;
  d.max_threads = max_threads;
  d.flags = o.flags;
  d.capacity = capacity;
  d.group_lanes = o.ticket_group ? o.ticket_group : kDefaultGroupLanes;
  d.patience_enq = 64;
  d.patience_deq = 256;
  d.help_delay = 64;
  if (o.flags & GQ_OPT_WFQ_TUNING) {
    d.patience_enq = o.wfq_patience_enq;
    d.patience_deq = o.wfq_patience_deq;
    d.help_delay = o.wfq_help_delay;
  }
  d.data = buf + L.data;
  d.aq.slots = (uint64_t*)(buf + L.slots_aq);
  d.aq.head = (uint64_t*)(buf + OFF_AQ_HEAD);
  d.aq.tail = (uint64_t*)(buf + OFF_AQ_TAIL);
  d.aq.threshold = (int64_t*)(buf + OFF_AQ_THR);
  d.fq.slots = (uint64_t*)(buf + L.slots_fq);
  d.fq.head = (uint64_t*)(buf + OFF_FQ_HEAD);
  d.fq.tail = (uint64_t*)(buf + OFF_FQ_TAIL);
  d.fq.threshold = (int64_t*)(buf + OFF_FQ_THR);
  if (kind == GQ_WFQ_YMC) {
    d.ymc_cells = (uint64_t*)(buf + L.ymc_pool);
    d.ymc_pool_cells = (o.ymc_pool_cells ? o.ymc_pool_cells : ymc_default_cells(capacity));
    d.ymc_handles = buf + L.ymc_handles;
    d.ymc_hint = (uint8_t*)(buf + L.ymc_hint);
    d.patience_enq = 10;  // the original algorithm's PATIENCE
    d.patience_deq = 10;
    if (o.flags & GQ_OPT_WFQ_TUNING) {
      d.patience_enq = o.wfq_patience_enq;
      d.patience_deq = o.wfq_patience_deq;
    }
  }
  if (kind == GQ_WFQ) {
    d.aq.records = buf + L.rec_aq;
    d.fq.records = buf + L.rec_fq;
    d.aq.owner = (uint64_t*)(buf + L.own_aq);
    d.fq.owner = (uint64_t*)(buf + L.own_fq);
    d.aq.hint = (uint8_t*)(buf + L.hint);
    d.fq.hint = (uint8_t*)(buf + L.hint) + max_threads;
    d.help_ctr = (uint32_t*)(buf + L.help);
    d.aq.announce = (uint64_t*)(buf + OFF_AQ_ANN);
    d.fq.announce = (uint64_t*)(buf + OFF_FQ_ANN);
  }
  if (kind == GQ_LFQ) {
    d.aq.hint = (uint8_t*)(buf + L.hint);
    d.fq.hint = (uint8_t*)(buf + L.hint) + max_threads;
  }
  d.err = (uint64_t*)(buf + OFF_ERR);
  d.stats = (uint64_t*)(buf + OFF_STATS);
  d.ymc_ctr = (uint64_t*)(buf + OFF_YMC_T);
  return d;
}

gq_status gq_create(gq_kind kind, uint64_t capacity, uint32_t item_width, uint32_t max_threads,
                    const gq_options* opts, void* dev_buf, uint64_t buf_bytes, gq_queue** out) {
  if (!out) return GQ_ERR_INVALID;
  *out = nullptr;
  Layout L;
  gq_status st = plan(kind, capacity, item_width, max_threads, opts, &L);
  if (st != GQ_OK) return st;
  gq_queue* q = new (std::nothrow) gq_queue();
  if (!q) return GQ_ERR_NOMEM;
  q->kind = kind;
  q->n = capacity;
  q->w = item_width;
  q->k = max_threads;
  memset(&q->opt, 0, sizeof(q->opt));
  q->opt.slot_mode = GQ_SLOTS_LINEAR;
  if (opts) q->opt = *opts;
  q->L = L;
  if (dev_buf) {
    if (buf_bytes < L.total || ((uintptr_t)dev_buf & 255)) {
      delete q;
      return GQ_ERR_NOMEM;
    }
    q->buf = (char*)dev_buf;
    q->bytes = buf_bytes;
    q->owns = false;
  } else {
    void* p = nullptr;
    if (hipMalloc(&p, L.total) != hipSuccess) {
      delete q;
      return GQ_ERR_NOMEM;
    }
    q->buf = (char*)p;
    q->bytes = L.total;
    q->owns = true;
  }
  q->dev = make_dev(kind, capacity, item_width, max_threads, q->opt, q->buf, L);
  st = launch_init(q, nullptr);
  if (st == GQ_OK) {
    // waits for the init kernel only (not for a serving kernel on its own
    // non-blocking stream)
    hipError_t e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize", __LINE__);
  }
  if (st != GQ_OK) {
    if (q->owns) (void)hipFree(q->buf);
    delete q;
    return st;
  }
  *out = q;
  return GQ_OK;
}

gq_status gq_destroy(gq_queue* q) {
  if (!q) return GQ_ERR_INVALID;
  if (q->owns && q->buf) (void)hipFree(q->buf);
  delete q;
  return GQ_OK;
}

gq_status gq_reset(gq_queue* q, void* stream) {
  if (!q) return GQ_ERR_INVALID;
  return launch_init(q, S(stream));
}

gq_status gq_enqueue_batch(gq_queue* q, const void* d_items, uint64_t m, uint8_t* d_status,
                           uint64_t* d_num_ok, void* stream) {
  if (!q || (!d_items && m)) return GQ_ERR_INVALID;
  if (m == 0) return GQ_OK;
  switch (q->kind) {
    case GQ_LFQ: launch_enq<GQ_LFQ>(q, d_items, m, d_status, d_num_ok, S(stream)); break;
    case GQ_WFQ: launch_enq<GQ_WFQ>(q, d_items, m, d_status, d_num_ok, S(stream)); break;
    case GQ_WFQ_YMC: launch_enq<GQ_WFQ_YMC>(q, d_items, m, d_status, d_num_ok, S(stream)); break;
    default: return GQ_ERR_INVALID;
  }
  HIP_OK(hipGetLastError());
  return GQ_OK;
}

gq_status gq_dequeue_batch(gq_queue* q, void* d_out, uint64_t m, uint8_t* d_status,
                           uint64_t* d_num_ok, void* stream) {
  if (!q || (!d_out && m)) return GQ_ERR_INVALID;
  if (m == 0) return GQ_OK;
  switch (q->kind) {
    case GQ_LFQ: launch_deq<GQ_LFQ>(q, d_out, m, d_status, d_num_ok, S(stream)); break;
    case GQ_WFQ: launch_deq<GQ_WFQ>(q, d_out, m, d_status, d_num_ok, S(stream)); break;
    case GQ_WFQ_YMC: launch_deq<GQ_WFQ_YMC>(q, d_out, m, d_status, d_num_ok, S(stream)); break;
    default: return GQ_ERR_INVALID;
  }
  HIP_OK(hipGetLastError());
  return GQ_OK;
}

gq_status gq_device_view(const gq_queue* q, gq_dev* out) {
  if (!q || !out) return GQ_ERR_INVALID;
  *out = q->dev;
  return GQ_OK;
}

gq_status gq_read_stats(gq_queue* q, gq_stats* out, void* stream) {
  if (!q || !out) return GQ_ERR_INVALID;
  uint64_t s[S_NUM];
  HIP_OK(hipMemcpyAsync(s, q->dev.stats, sizeof(s), hipMemcpyDeviceToHost, S(stream)));
  HIP_OK(hipStreamSynchronize(S(stream)));
  out->ok_enq = s[S_OK_ENQ];
  out->ok_deq = s[S_OK_DEQ];
  out->full = s[S_FULL];
  out->empty = s[S_EMPTY];
  out->cas_fail = s[S_CAS_FAIL];
  out->tickets = s[S_TICKETS];
  out->slow_enter = s[S_SLOW];
  out->helps = s[S_HELPS];
  out->scans = s[S_SCAN];
  out->dropped = s[S_DROP];
  return GQ_OK;
}

gq_status gq_clear_stats(gq_queue* q, void* stream) {
  if (!q) return GQ_ERR_INVALID;
  HIP_OK(hipMemsetAsync(q->dev.stats, 0, S_NUM * sizeof(uint64_t), S(stream)));
  return GQ_OK;
}

gq_status gq_check_error(gq_queue* q, void* stream) {
  if (!q) return GQ_ERR_INVALID;
  uint64_t e = 0;
  HIP_OK(hipMemcpyAsync(&e, q->dev.err, sizeof(e), hipMemcpyDeviceToHost, S(stream)));
  HIP_OK(hipStreamSynchronize(S(stream)));
  if (e == 0) return GQ_OK;
  return (gq_status)(-(int64_t)e);
}

// ---- drivers ----------------------------------------------------------------
static Rec make_rec(const gq_history* h) {
  Rec r;
  memset(&r, 0, sizeof(r));
  if (h) {
    r.h = *h;
    r.on = true;
  }
  return r;
}

static gq_status resident_blocks_of(const void* fn, uint32_t block, uint32_t* out) {
  int dev = 0, cus = 0, nb = 0;
  HIP_OK(hipGetDevice(&dev));
  HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, (int)block, 0));
  *out = (uint32_t)(nb * cus);
  return GQ_OK;
}

// Each driver is instantiated per queue kind; KIND_SWITCH picks the
// instantiation for q->kind.
#define KIND_SWITCH(kind, CALL)                      \
  switch (kind) {                                    \
    case GQ_LFQ: { constexpr int K = GQ_LFQ; CALL; } break; \
    case GQ_WFQ: { constexpr int K = GQ_WFQ; CALL; } break; \
    case GQ_WFQ_YMC: { constexpr int K = GQ_WFQ_YMC; CALL; } break; \
    default: return GQ_ERR_INVALID;                  \
  }

// Workgroup size of the group-ticket drivers: the queue's ticket group,
// halved until it divides `lanes`; 64 (or less) means the per-wavefront form.
static uint32_t group_block(const gq_queue* q, uint64_t lanes) {
  uint32_t b = q->dev.group_lanes;
  while (b > 64 && lanes % b) b >>= 1;
  return b;
}

// The mixed workload's launch shape: workgroups of `block` lanes running the
// group-ticket kernel (block > 64), or the per-wavefront kernel in workgroups
// of `block` (256 or 64).  *fn receives the kernel.
template <int KIND>
static uint32_t mix_shape(const gq_queue* q, uint32_t lanes, bool hist, const void** fn) {
  const uint32_t gb = group_block(q, lanes);
  if (gb > 64) {
    *fn = hist ? (const void*)k_mix_group<KIND, true, false> : (const void*)k_mix_group<KIND, false, false>;
    return gb;
  }
  *fn = hist ? (const void*)k_mix<KIND, true> : (const void*)k_mix<KIND, false>;
  return lanes % kBlock == 0 ? kBlock : 64;
}

template <int KIND>
static void launch_mix(gq_queue* q, uint64_t seed, uint32_t lanes, uint32_t ops, uint64_t* counts,
                       uint32_t* lane_enq, const gq_history* hist, hipStream_t s) {
  const Rec rec = make_rec(hist);
  const void* fn = nullptr;
  const uint32_t b = mix_shape<KIND>(q, lanes, hist != nullptr, &fn);
  const dim3 grid(lanes / b), block(b);
  if (fn == (const void*)k_mix_group<KIND, true, false> ||
      fn == (const void*)k_mix_group<KIND, false, false>) {
    // the timed form (no history) has a copy for linear slots, the default
    const bool lin = !hist && q->dev.slot_mode == GQ_SLOTS_LINEAR;
    if (KIND == GQ_LFQ) {
      if (hist)
        LAUNCH((k_mix_group_lfq<true, false>), grid, block, 0, s, q->dev, seed, ops, counts, lane_enq, rec);
      else if (lin)
        LAUNCH((k_mix_group_lfq<false, true>), grid, block, 0, s, q->dev, seed, ops, counts, lane_enq, rec);
      else
        LAUNCH((k_mix_group_lfq<false, false>), grid, block, 0, s, q->dev, seed, ops, counts, lane_enq, rec);
    } else if (hist) {
      LAUNCH((k_mix_group<KIND, true, false>), grid, block, 0, s, q->dev, seed, ops, counts, lane_enq, rec);
    } else if (lin) {
      LAUNCH((k_mix_group<KIND, false, true>), grid, block, 0, s, q->dev, seed, ops, counts, lane_enq, rec);
    } else {
      LAUNCH((k_mix_group<KIND, false, false>), grid, block, 0, s, q->dev, seed, ops, counts, lane_enq, rec);
    }
    return;
  }
  if (hist) LAUNCH((k_mix<KIND, true>), grid, block, 0, s, q->dev, seed, ops, counts, lane_enq, rec);
  else LAUNCH((k_mix<KIND, false>), grid, block, 0, s, q->dev, seed, ops, counts, lane_enq, rec);
}

gq_status gq_run_mix(gq_queue* q, uint64_t seed, uint32_t lanes, uint32_t ops_per_lane,
                     uint64_t* d_counts, uint32_t* d_lane_enq, const gq_history* hist,
                     void* stream) {
  if (!q || !d_counts || lanes == 0 || lanes % 64 || lanes > q->k) return GQ_ERR_INVALID;
  if (hist && (!hist->val || !hist->call || !hist->ret || !hist->opst)) return GQ_ERR_INVALID;
  // G-WFQ-YMC: every operation takes at least one cell; a run that could
  // need more cells than the pool holds is refused up front.
  if (q->kind == GQ_WFQ_YMC && (uint64_t)lanes * ops_per_lane > q->dev.ymc_pool_cells)
    return GQ_ERR_POOL_EXHAUSTED;
  // No residency check here.  G-WFQ's wait-freedom (Section III-C) assumes
  // that every lane taking part in an operation is resident and scheduled.
  // A lane takes part only once its workgroup has started, a started
  // workgroup stays resident until it ends, and no lane of this driver waits
  // for a lane that has not started (each runs its own operations; helpers
  // only act on published requests), so a grid larger than the device holds
  // at once -- it then runs in rounds of workgroups -- keeps the premise.
  // Drivers whose lanes wait for other lanes (shared targets, barriers)
  // refuse grids that cannot be resident all at once.
  KIND_SWITCH(q->kind, launch_mix<K>(q, seed, lanes, ops_per_lane, d_counts, d_lane_enq, hist,
                                     S(stream)));
  HIP_OK(hipGetLastError());
  return GQ_OK;
}

template <int KIND>
static void launch_balanced(gq_queue* q, uint32_t lanes, uint32_t rounds, uint64_t* counts,
                            const gq_history* hist, hipStream_t s) {
  const dim3 grid(lanes / kBlock), block(kBlock);
  const Rec rec = make_rec(hist);
  if (hist) LAUNCH((k_balanced<KIND, true>), grid, block, 0, s, q->dev, rounds, counts, rec);
  else LAUNCH((k_balanced<KIND, false>), grid, block, 0, s, q->dev, rounds, counts, rec);
}

gq_status gq_run_balanced(gq_queue* q, uint32_t lanes, uint32_t rounds, uint64_t* d_counts,
                          const gq_history* hist, void* stream) {
  if (!q || !d_counts || lanes == 0 || lanes % kBlock || lanes > q->k) return GQ_ERR_INVALID;
  if (hist && (!hist->val || !hist->call || !hist->ret || !hist->opst)) return GQ_ERR_INVALID;
  KIND_SWITCH(q->kind, launch_balanced<K>(q, lanes, rounds, d_counts, hist, S(stream)));
  HIP_OK(hipGetLastError());
  return GQ_OK;
}


template <int KIND>
static const void* prodcons_fn(bool hist) {
  return hist ? (const void*)k_prodcons<KIND, true> : (const void*)k_prodcons<KIND, false>;
}

template <int KIND>
static void launch_prodcons(gq_queue* q, uint64_t seed, uint32_t lanes, uint32_t block,
                            const uint8_t* role, uint32_t quota, uint64_t target,
                            uint32_t log2_inv_p, uint32_t token_mode, uint32_t jitter,
                            uint64_t max_rounds, uint64_t limit_ticks, uint64_t* taken,
                            uint64_t* counts, const gq_history* hist, hipStream_t s) {
  const Rec rec = make_rec(hist);
  const dim3 grid(lanes / block), blk(block);
  if (hist)
    LAUNCH((k_prodcons<KIND, true>), grid, blk, 0, s, q->dev, seed, role, quota, target,
           log2_inv_p, token_mode, jitter, max_rounds, limit_ticks, taken, counts, rec);
  else
    LAUNCH((k_prodcons<KIND, false>), grid, blk, 0, s, q->dev, seed, role, quota, target,
           log2_inv_p, token_mode, jitter, max_rounds, limit_ticks, taken, counts, rec);
}

gq_status gq_run_prodcons(gq_queue* q, uint64_t seed, uint32_t lanes, uint32_t block,
                          const uint8_t* d_lane_role, uint32_t items_per_producer,
                          uint64_t target, uint32_t log2_inv_p, uint32_t token_mode,
                          uint32_t jitter, uint64_t max_rounds, uint32_t time_limit_ms,
                          uint64_t* d_counts, const gq_history* hist, void* stream) {
  if (!q || !d_counts || !d_lane_role || lanes == 0 || block == 0 || block > 1024 ||
      block % 64 || lanes % block || log2_inv_p > 63 || token_mode > 1 || lanes > q->k)
    return GQ_ERR_INVALID;
  if (hist && (!hist->val || !hist->call || !hist->ret || !hist->opst)) return GQ_ERR_INVALID;
  const void* fn = nullptr;
  KIND_SWITCH(q->kind, fn = prodcons_fn<K>(hist != nullptr));
  uint32_t resident = 0;
  gq_status st = resident_blocks_of(fn, block, &resident);
  if (st != GQ_OK) return st;
  if (lanes / block > resident) return GQ_ERR_RESIDENCY;
  // The shared "taken" counter sits in the queue's control block.
  uint64_t* taken = (uint64_t*)(q->buf + OFF_TAKEN);
  HIP_OK(hipMemsetAsync(taken, 0, sizeof(uint64_t), S(stream)));
  const uint64_t limit_ticks = (uint64_t)time_limit_ms * 100000ull;  // 100 MHz clock
  KIND_SWITCH(q->kind, launch_prodcons<K>(q, seed, lanes, block, d_lane_role, items_per_producer,
                                          target, log2_inv_p, token_mode, jitter, max_rounds,
                                          limit_ticks, taken, d_counts, hist, S(stream)));
  HIP_OK(hipGetLastError());
  return GQ_OK;
}

template <int KIND>
static const void* timed_fn(bool hist) {
  return hist ? (const void*)k_timed<KIND, true> : (const void*)k_timed<KIND, false>;
}

template <int KIND>
static void launch_timed(gq_queue* q, uint32_t lanes, uint32_t mode, uint32_t prod_waves,
                         uint64_t warm, uint64_t win, uint64_t* counts, uint64_t* ctl,
                         uint32_t* lane_enq, const gq_history* hist, hipStream_t s) {
  const Rec rec = make_rec(hist);
  const dim3 grid(lanes / kBlock), block(kBlock);
  if (hist)
    LAUNCH((k_timed<KIND, true>), grid, block, 0, s, q->dev, mode, prod_waves, warm, win, counts,
           ctl, lane_enq, rec);
  else
    LAUNCH((k_timed<KIND, false>), grid, block, 0, s, q->dev, mode, prod_waves, warm, win, counts,
           ctl, lane_enq, rec);
}

gq_status gq_run_timed(gq_queue* q, uint32_t mode, uint32_t lanes, uint32_t prod_pct,
                       uint32_t warmup_us, uint32_t window_us, uint64_t* d_counts,
                       uint64_t* d_ctl, uint32_t* d_lane_enq, const gq_history* hist,
                       void* stream) {
  if (!q || !d_counts || !d_ctl || mode > 1 || lanes == 0 || lanes % kBlock || lanes > q->k ||
      prod_pct > 100 || window_us == 0)
    return GQ_ERR_INVALID;
  if (hist && (!hist->val || !hist->call || !hist->ret || !hist->opst || hist->per_lane == 0))
    return GQ_ERR_INVALID;
  const void* fn = nullptr;
  KIND_SWITCH(q->kind, fn = timed_fn<K>(hist != nullptr));
  uint32_t resident = 0;
  gq_status st = resident_blocks_of(fn, kBlock, &resident);
  if (st != GQ_OK) return st;
  if (lanes / kBlock > resident) return GQ_ERR_RESIDENCY;
  const uint32_t waves = lanes / 64;
  const uint32_t prod_waves = mode == 0 ? waves : (uint32_t)((uint64_t)waves * prod_pct / 100);
  HIP_OK(hipMemsetAsync(d_ctl, 0, sizeof(uint64_t), S(stream)));
  const uint64_t warm = (uint64_t)warmup_us * 100, win = (uint64_t)window_us * 100;
  KIND_SWITCH(q->kind, launch_timed<K>(q, lanes, mode, prod_waves, warm, win, d_counts, d_ctl,
                                       d_lane_enq, hist, S(stream)));
  HIP_OK(hipGetLastError());
  return GQ_OK;
}

template <int KIND>
static void launch_script(gq_queue* q, uint32_t lanes, uint32_t spread, const uint8_t* ops,
                          const uint64_t* args, const uint16_t* pauses, const uint32_t* n_ops,
                          uint32_t max_ops, const gq_history* hist, hipStream_t s) {
  const Rec rec = make_rec(hist);
  const dim3 grid(spread ? lanes : 1), block(spread ? 64 : ((lanes + 63) / 64) * 64);
  LAUNCH((k_script<KIND>), grid, block, 0, s, q->dev, lanes, spread, ops, args, pauses, n_ops,
         max_ops, rec);
}

gq_status gq_run_script(gq_queue* q, uint32_t lanes, uint32_t spread, const uint8_t* d_ops,
                        const uint64_t* d_args, const uint16_t* d_pause, const uint32_t* d_n_ops,
                        uint32_t max_ops, const gq_history* hist, void* stream) {
  if (!q || !hist || !d_ops || !d_args || !d_pause || !d_n_ops || lanes == 0 || lanes > 1024 ||
      lanes > q->k)
    return GQ_ERR_INVALID;
  if (!hist->val || !hist->call || !hist->ret || !hist->opst || hist->per_lane < max_ops)
    return GQ_ERR_INVALID;
  KIND_SWITCH(q->kind, launch_script<K>(q, lanes, spread, d_ops, d_args, d_pause, d_n_ops,
                                        max_ops, hist, S(stream)));
  HIP_OK(hipGetLastError());
  return GQ_OK;
}

// ---- probes -------------------------------------------------------------------
static uint64_t* probe_sink() {
  static uint64_t* s = nullptr;
  if (!s) (void)hipMalloc(&s, 256);
  return s;
}

gq_status gq_probe_faa(uint64_t* d_ctr, uint32_t lanes, uint32_t iters, uint32_t per_lane,
                       uint32_t ncounters, uint32_t spacing_bytes, void* stream) {
  if (!d_ctr || lanes == 0 || lanes % kBlock || ncounters == 0 || spacing_bytes % 8)
    return GQ_ERR_INVALID;
  LAUNCH(k_probe_faa, dim3(lanes / kBlock), dim3(kBlock), 0, S(stream), d_ctr, iters, per_lane,
         ncounters, spacing_bytes / 8, probe_sink());
  HIP_OK(hipGetLastError());
  return GQ_OK;
}

gq_status gq_probe_cas(uint64_t* d_slots, uint64_t nslots, uint32_t stride_bytes, uint32_t lanes,
                       uint32_t iters, void* stream) {
  if (!d_slots || nslots == 0 || lanes == 0 || lanes % kBlock || stride_bytes < 8 ||
      stride_bytes % 8)
    return GQ_ERR_INVALID;
  LAUNCH(k_probe_cas, dim3(lanes / kBlock), dim3(kBlock), 0, S(stream), d_slots,
                     nslots, stride_bytes / 8, iters, probe_sink());
  HIP_OK(hipGetLastError());
  return GQ_OK;
}

gq_status gq_probe_copy(uint64_t* d_dst, const uint64_t* d_src, uint64_t n, void* stream) {
  if (!d_dst || !d_src) return GQ_ERR_INVALID;
  const uint32_t grid = grid_for(n / 2, kBlock, 8192);
  LAUNCH(k_probe_copy, dim3(grid), dim3(kBlock), 0, S(stream), d_dst, d_src, n);
  HIP_OK(hipGetLastError());
  return GQ_OK;
}

gq_status gq_probe_fence(uint64_t* d_lines, uint32_t lanes, uint32_t iters, uint32_t mode,
                         void* stream) {
  if (!d_lines || lanes == 0 || lanes % kBlock || mode > 3) return GQ_ERR_INVALID;
  LAUNCH(k_probe_fence, dim3(lanes / kBlock), dim3(kBlock), 0, S(stream), d_lines,
                     iters, mode);
  HIP_OK(hipGetLastError());
  return GQ_OK;
}

template <int KIND>
static const void* driver_fn(const char* kernel) {
  if (!strcmp(kernel, "mix")) return (const void*)k_mix<KIND, false>;
  if (!strcmp(kernel, "mix_group"))  // the kernel launch_mix starts for the group form
    return KIND == GQ_LFQ ? (const void*)k_mix_group_lfq<false, true>
                          : (const void*)k_mix_group<KIND, false, true>;
  if (!strcmp(kernel, "prodcons")) return (const void*)k_prodcons<KIND, false>;
  return nullptr;
}

gq_status gq_resident_blocks(const char* kernel, gq_kind kind, uint32_t block,
                             uint32_t* out_blocks) {
  if (!kernel || !out_blocks || block == 0 || block > 1024) return GQ_ERR_INVALID;
  const void* fn = nullptr;
  KIND_SWITCH(kind, fn = driver_fn<K>(kernel));
  if (!fn) return GQ_ERR_INVALID;
  return resident_blocks_of(fn, block, out_blocks);
}

gq_status gq_device_info(uint32_t* cus, uint32_t* wave, char* name, uint32_t len) {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  hipDeviceProp_t p;
  HIP_OK(hipGetDeviceProperties(&p, dev));
  if (cus) *cus = (uint32_t)p.multiProcessorCount;
  if (wave) *wave = (uint32_t)p.warpSize;
  if (name && len) {
    strncpy(name, p.gcnArchName, len - 1);
    name[len - 1] = 0;
  }
  return GQ_OK;
}



// ---- many queues in one launch ----------------------------------------------
struct gq_multi {
  gq_kind kind;
  uint32_t nq, waves, block;
  gq_dev* d_qs;
  uint32_t* d_wave_q;
  uint32_t* d_q_lane0;
  uint64_t* d_seed;
  hipGraph_t graph;
  hipGraphExec_t exec;
  bool captured;
};

gq_status gq_multi_create(uint32_t nq, gq_queue* const* queues, const uint32_t* lanes_per_queue,
                          uint32_t block, gq_multi** out) {
  if (!out || !queues || !lanes_per_queue || nq == 0 || (block != 64 && block != 128 &&
      block != 256))
    return GQ_ERR_INVALID;
  *out = nullptr;
  uint64_t waves = 0;
  for (uint32_t i = 0; i < nq; i++) {
    if (!queues[i] || queues[i]->kind != queues[0]->kind) return GQ_ERR_INVALID;
    const uint32_t L = lanes_per_queue[i];
    if (L == 0 || L % 64 || L > queues[i]->k) return GQ_ERR_INVALID;
    waves += L / 64;
  }
  const uint32_t wpb = block / 64;
  const uint64_t waves_padded = (waves + wpb - 1) / wpb * wpb;
  if (waves_padded * 64 > (1ull << 31)) return GQ_ERR_INVALID;
  // The wavefronts must fill whole workgroups: a ragged total is refused.
  if (waves_padded != waves) return GQ_ERR_INVALID;
  gq_dev* h_qs = (gq_dev*)malloc(sizeof(gq_dev) * nq);
  uint32_t* h_wave_q = (uint32_t*)malloc(sizeof(uint32_t) * waves);
  uint32_t* h_lane0 = (uint32_t*)malloc(sizeof(uint32_t) * nq);
  if (!h_qs || !h_wave_q || !h_lane0) {
    free(h_qs); free(h_wave_q); free(h_lane0);
    return GQ_ERR_NOMEM;
  }
  uint64_t w = 0;
  for (uint32_t i = 0; i < nq; i++) {
    h_qs[i] = queues[i]->dev;
    h_lane0[i] = (uint32_t)(w * 64);
    for (uint32_t j = 0; j < lanes_per_queue[i] / 64; j++) h_wave_q[w++] = i;
  }
  gq_multi* m = new (std::nothrow) gq_multi();
  if (!m) { free(h_qs); free(h_wave_q); free(h_lane0); return GQ_ERR_NOMEM; }
  m->kind = queues[0]->kind;
  m->nq = nq;
  m->waves = (uint32_t)waves;
  m->block = block;
  m->captured = false;
  gq_status st = GQ_OK;
  if (hipMalloc(&m->d_qs, sizeof(gq_dev) * nq) != hipSuccess ||
      hipMalloc(&m->d_wave_q, sizeof(uint32_t) * waves) != hipSuccess ||
      hipMalloc(&m->d_q_lane0, sizeof(uint32_t) * nq) != hipSuccess ||
      hipMalloc(&m->d_seed, 256) != hipSuccess)
    st = GQ_ERR_NOMEM;
  if (st == GQ_OK &&
      (hipMemcpy(m->d_qs, h_qs, sizeof(gq_dev) * nq, hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(m->d_wave_q, h_wave_q, sizeof(uint32_t) * waves, hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(m->d_q_lane0, h_lane0, sizeof(uint32_t) * nq, hipMemcpyHostToDevice) != hipSuccess))
    st = GQ_ERR_HIP;
  free(h_qs); free(h_wave_q); free(h_lane0);
  if (st != GQ_OK) {
    gq_multi_destroy(m);
    return st;
  }
  *out = m;
  return GQ_OK;
}

template <int KIND>
static void launch_multi(gq_multi* m, uint32_t ops, uint64_t* counts, const gq_history* hist,
                         hipStream_t s) {
  const dim3 grid(m->waves * 64 / m->block), block(m->block);
  const Rec rec = make_rec(hist);
  if (hist)
    LAUNCH((k_multi_mix<KIND, true>), grid, block, 0, s, m->d_qs, m->d_wave_q, m->d_q_lane0,
           m->d_seed, ops, counts, rec);
  else
    LAUNCH((k_multi_mix<KIND, false>), grid, block, 0, s, m->d_qs, m->d_wave_q, m->d_q_lane0,
           m->d_seed, ops, counts, rec);
}

gq_status gq_multi_run_mix(gq_multi* m, uint64_t seed, uint32_t ops_per_lane, uint64_t* d_counts,
                           const gq_history* hist, void* stream) {
  if (!m || !d_counts) return GQ_ERR_INVALID;
  if (hist && (!hist->val || !hist->call || !hist->ret || !hist->opst)) return GQ_ERR_INVALID;
  LAUNCH(k_seed, dim3(1), dim3(64), 0, S(stream), m->d_seed, seed, 0u);
  HIP_OK(hipGetLastError());
  KIND_SWITCH(m->kind, launch_multi<K>(m, ops_per_lane, d_counts, hist, S(stream)));
  HIP_OK(hipGetLastError());
  return GQ_OK;
}

gq_status gq_multi_capture(gq_multi* m, uint64_t seed, uint32_t ops_per_lane, uint64_t* d_counts,
                           const gq_history* hist, void* stream) {
  if (!m || !d_counts || !stream) return GQ_ERR_INVALID;
  if (hist && (!hist->val || !hist->call || !hist->ret || !hist->opst)) return GQ_ERR_INVALID;
  if (m->captured) {
    (void)hipGraphExecDestroy(m->exec);
    (void)hipGraphDestroy(m->graph);
    m->captured = false;
  }
  // the first replay runs with seed + 1, each later one with the next seed
  LAUNCH(k_seed, dim3(1), dim3(64), 0, S(stream), m->d_seed, seed, 0u);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamBeginCapture(S(stream), hipStreamCaptureModeRelaxed));
  LAUNCH(k_seed, dim3(1), dim3(64), 0, S(stream), m->d_seed, 0ull, 1u);
  gq_status st = GQ_OK;
  switch (m->kind) {
    case GQ_LFQ: launch_multi<GQ_LFQ>(m, ops_per_lane, d_counts, hist, S(stream)); break;
    case GQ_WFQ: launch_multi<GQ_WFQ>(m, ops_per_lane, d_counts, hist, S(stream)); break;
    case GQ_WFQ_YMC: launch_multi<GQ_WFQ_YMC>(m, ops_per_lane, d_counts, hist, S(stream)); break;
    default: st = GQ_ERR_INVALID;
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(S(stream), &g);
  if (st != GQ_OK) return st;
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture", __LINE__);
  e = hipGraphInstantiate(&m->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(e, "hipGraphInstantiate", __LINE__);
  }
  m->graph = g;
  m->captured = true;
  return GQ_OK;
}

gq_status gq_multi_replay(gq_multi* m, void* stream) {
  if (!m || !m->captured) return GQ_ERR_INVALID;
  HIP_OK(hipGraphLaunch(m->exec, S(stream)));
  return GQ_OK;
}

gq_status gq_multi_destroy(gq_multi* m) {
  if (!m) return GQ_ERR_INVALID;
  if (m->captured) {
    (void)hipGraphExecDestroy(m->exec);
    (void)hipGraphDestroy(m->graph);
  }
  if (m->d_qs) (void)hipFree(m->d_qs);
  if (m->d_wave_q) (void)hipFree(m->d_wave_q);
  if (m->d_q_lane0) (void)hipFree(m->d_q_lane0);
  if (m->d_seed) (void)hipFree(m->d_seed);
  delete m;
  return GQ_OK;
}

// ---- queue-driven BFS ----------------------------------------------------------
template <int KIND>
static const void* bfs_fn() { return (const void*)bfs::k_bfs<KIND>; }

template <int KIND>
static void launch_bfs(const gq_dev& qa, const gq_dev& qb, const uint32_t* off,
                       const uint32_t* cols, uint32_t nv, uint32_t root, uint32_t* level,
                       uint64_t* ctl, uint64_t hub_cap, uint32_t lanes, uint32_t block,
                       hipStream_t s) {
  const uint32_t nblocks = lanes / block;
  LAUNCH((bfs::k_bfs<KIND>), dim3(nblocks), dim3(block), 0, s, qa, qb, off, cols, nv, root, level,
         ctl, hub_cap, nblocks);
}

// Checks shared by the BFS entry points: the launch shape and co-residency
// of the persistent kernel.
static gq_status bfs_launch_ok(gq_kind kind, uint32_t lanes, uint32_t block) {
  if (block == 0 || block > 256 || block % 64 || lanes == 0 || lanes % block)
    return GQ_ERR_INVALID;
  const void* fn = nullptr;
  KIND_SWITCH(kind, fn = bfs_fn<K>());
  uint32_t resident = 0;
  gq_status st = resident_blocks_of(fn, block, &resident);
  if (st != GQ_OK) return st;
  if (lanes / block > resident) return GQ_ERR_RESIDENCY;
  return GQ_OK;
}

// Clear the control block, initialise the levels, run the persistent kernel.
static gq_status bfs_launch(gq_kind kind, const gq_dev& qa, const gq_dev& qb,
                            const uint32_t* d_offsets, const uint32_t* d_cols, uint32_t nv,
                            uint32_t root, uint32_t* d_level, uint32_t lanes, uint32_t block,
                            uint64_t* d_ctl, uint64_t ctl_bytes, hipStream_t s) {
  const uint64_t words = ctl_bytes / 8;
  const uint64_t hub_cap = words > bfs::HUB_LIST ? words - bfs::HUB_LIST : 0;
  LAUNCH(bfs::k_bfs_ctl_clear, dim3(2), dim3(kBlock), 0, s, d_ctl);
  HIP_OK(hipGetLastError());
  LAUNCH(bfs::k_bfs_init, dim3(grid_for(nv, kBlock, 8192)), dim3(kBlock), 0, s, d_level,
         d_offsets, nv, d_ctl);
  HIP_OK(hipGetLastError());
  KIND_SWITCH(kind, launch_bfs<K>(qa, qb, d_offsets, d_cols, nv, root, d_level, d_ctl, hub_cap,
                                  lanes, block, s));
  HIP_OK(hipGetLastError());
  return GQ_OK;
}

uint64_t gq_bfs_ctl_bytes(uint64_t nnz) {
  return 8 * (bfs::HUB_LIST + nnz / bfs::HUB_MIN + 1);
}

gq_status gq_bfs(gq_queue* qa, gq_queue* qb, const uint32_t* d_offsets, const uint32_t* d_cols,
                 uint32_t nv, uint32_t root, uint32_t* d_level, uint32_t lanes, uint32_t block,
                 uint64_t* d_ctl, uint64_t ctl_bytes, void* stream) {
  if (!qa || !qb || qa == qb || !d_offsets || !d_cols || !d_level || !d_ctl || nv == 0 ||
      root >= nv || qa->kind != qb->kind || qa->w != 4 || qb->w != 4 || lanes > qa->k ||
      lanes > qb->k || ctl_bytes < 8 * (uint64_t)bfs::CTL_MIN_WORDS || ((uintptr_t)d_ctl & 7))
    return GQ_ERR_INVALID;
  if (qa->kind != GQ_WFQ_YMC && (qa->n < nv || qb->n < nv)) return GQ_ERR_INVALID;
  const gq_status st = bfs_launch_ok(qa->kind, lanes, block);
  if (st != GQ_OK) return st;
  return bfs_launch(qa->kind, qa->dev, qb->dev, d_offsets, d_cols, nv, root, d_level, lanes, block,
                    d_ctl, ctl_bytes, S(stream));
}

// ---- BFS with no allocation ------------------------------------------------
// The two frontier queues and the control block of gq_bfs_static live in
// this file-scope array (one copy per GPU, alive until the process ends).
// Host code never passes `g_bfs_scratch` itself to a kernel -- on the host it
// is only a stand-in symbol -- but the device address hipGetSymbolAddress
// returns for it, looked up once per device on the first call there.
static __device__ __align__(256) unsigned char g_bfs_scratch[GQ_BFS_STATIC_BYTES];
static constexpr int kMaxDevices = 64;

static constexpr uint64_t kStaticCtlBytes = 64 * 1024;  // 7680 hub-list entries

static gq_status static_scratch(char** out) {
  static std::mutex mu;
  static char* ptr[kMaxDevices] = {};
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return GQ_ERR_INVALID;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(g_bfs_scratch)));
    if (!p) return GQ_ERR_HIP;
    ptr[dev] = (char*)p;
  }
  *out = ptr[dev];
  return GQ_OK;
}

// Queue initialisation from a device view (the kernels of launch_init).
static gq_status init_view(gq_kind kind, const gq_dev& d, uint64_t n, uint32_t k, hipStream_t s) {
  const uint64_t slots = 2 * n > k ? 2 * n : k;
  const uint32_t grid = grid_for(slots, kBlock, 4096);
  if (kind == GQ_LFQ) LAUNCH(k_init_lfq, dim3(grid), dim3(kBlock), 0, s, d);
  else if (kind == GQ_WFQ) LAUNCH(k_init_wfq, dim3(grid), dim3(kBlock), 0, s, d);
  else return GQ_ERR_INVALID;
  HIP_OK(hipGetLastError());
  return GQ_OK;
}

__global__ void k_bfs_static_info(const uint64_t* err_a, const uint64_t* err_b,
                                  const uint64_t* ctl, uint64_t* info) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const uint64_t ea = ld(err_a), eb = ld(err_b);
    st(info + 0, ea ? ea : eb);
    st(info + 1, ld(ctl + bfs::LEVELS));
    st(info + 2, ld(ctl + bfs::SCANNED));
    st(info + 3, 0ull);
  }
}

gq_status gq_bfs_static(gq_kind kind, const uint32_t* d_offsets, const uint32_t* d_cols,
                        uint32_t nv, uint32_t root, uint32_t* d_level, uint32_t lanes,
                        uint32_t block, uint64_t* d_info, void* stream) {
  if (kind != GQ_LFQ && kind != GQ_WFQ) return GQ_ERR_INVALID;
  if (nv > GQ_BFS_STATIC_MAX_VERTICES || lanes > GQ_BFS_STATIC_MAX_LANES)
    return GQ_ERR_TOO_LARGE;
  if (!d_offsets || !d_cols || !d_level || nv == 0 || root >= nv) return GQ_ERR_INVALID;
  uint64_t cap = 64;  // G-WFQ's cycle bound (Lemma 4) holds for 8192 lanes from here on
  while (cap < nv) cap <<= 1;
  Layout L;
  gq_status st = plan(kind, cap, 4, lanes, nullptr, &L);
  if (st != GQ_OK) return st;
  const uint64_t qbytes = align_up(L.total, 256);
  if (2 * qbytes + kStaticCtlBytes > GQ_BFS_STATIC_BYTES) return GQ_ERR_TOO_LARGE;
  st = bfs_launch_ok(kind, lanes, block);
  if (st != GQ_OK) return st;
  char* base = nullptr;
  st = static_scratch(&base);
  if (st != GQ_OK) return st;
  gq_options o;
  memset(&o, 0, sizeof(o));
  o.slot_mode = GQ_SLOTS_LINEAR;
  const gq_dev qa = make_dev(kind, cap, 4, lanes, o, base, L);
  const gq_dev qb = make_dev(kind, cap, 4, lanes, o, base + qbytes, L);
  uint64_t* ctl = (uint64_t*)(base + 2 * qbytes);
  const hipStream_t s = S(stream);
  st = init_view(kind, qa, cap, lanes, s);
  if (st == GQ_OK) st = init_view(kind, qb, cap, lanes, s);
  if (st == GQ_OK)
    st = bfs_launch(kind, qa, qb, d_offsets, d_cols, nv, root, d_level, lanes, block, ctl,
                    kStaticCtlBytes, s);
  if (st == GQ_OK && d_info) {
    LAUNCH(k_bfs_static_info, dim3(1), dim3(64), 0, s, qa.err, qb.err, ctl, d_info);
    HIP_OK(hipGetLastError());
  }
  return st;
}

#include "gq_serve.inc"
#include "gq_rt.inc"
