/*
 * gq_oracle.c -- the CPU oracle for the concurrent-queue hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the HIP queues it checks, and it never runs
 * on the product path.
 *
 * The queues are correct iff every execution is linearizable with respect to
 * the sequential FIFO specification (paper, Section IV, "Linearizability via
 * Porcupine": enqueues append to the state list, dequeues return the head or
 * report empty) and deliver every token exactly once, in per-producer order
 * (Section IV, "Device-side FIFO conformance").  A concurrent run has many
 * correct outcomes, so this oracle does not re-run any GPU algorithm: it checks
 * recorded histories against those definitions.
 *
 * History layout (struct of arrays, one entry per completed operation, grouped
 * by process and in program order inside a process):
 *   proc[i]  the issuing lane
 *   op[i]    0 = enqueue, 1 = dequeue            (the paper's op field)
 *   st[i]    0 = OK, 1 = EMPTY, 2 = FULL
 *   val[i]   the enqueued argument, or the dequeued return value
 *   call[i], ret_t[i]  device timestamps taken before the call and after the
 *            return (the paper's call/end fields); equal stamps are overlap.
 *
 * Parts:
 *   O1/O2  orc_fifo_replay      sequential bounded FIFO (textbook definition)
 *   O3     orc_conservation     multiset equality: nothing lost, duplicated
 *                               or invented
 *   O4     orc_producer_order   per-producer monotone sequence (Section IV)
 *   O6     orc_violation_scan   sound violation patterns on large histories
 *   O7     orc_bfs              sequential queue BFS (Section V-B)
 *          orc_locked_queue_run host mutex + ring baseline (measurement only)
 * The brute-force linearizability search (O5) is in linearize.py; the
 * linearization witness search for large histories (O10) in gq_linsearch.c.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

enum { ORC_ENQ = 0, ORC_DEQ = 1 };
enum { ORC_OK = 0, ORC_EMPTY = 1, ORC_FULL = 2 };

/* ------------------------------------------------------------------------ */
/* O1/O2: sequential FIFO replay.                                            */
/* Replays m operations, in the given total order, through a FIFO of bounded */
/* capacity (0 = unbounded).  Enqueue appends and answers OK, or FULL when   */
/* the FIFO already holds `capacity` items; dequeue pops the head, or        */
/* answers EMPTY.  This is the state machine of the paper's queue model with  */
/* the bounded-capacity rule of the ring (logical capacity n, Section III-B). */
/* The FIFO is an array with a read and a write cursor: every item ever      */
/* held gets its own cell, so no wrap-around arithmetic is involved.          */
/* Returns the final size, or -1 on allocation failure.                       */
/* ------------------------------------------------------------------------ */
int64_t orc_fifo_replay(uint64_t m, const uint8_t *op, const uint64_t *arg,
                        uint64_t capacity, uint64_t n_prefill,
                        const uint64_t *prefill, uint8_t *st_out,
                        uint64_t *val_out, uint64_t *residual_out)
{
    uint64_t cells = n_prefill + m + 1;
    uint64_t *q = (uint64_t *)malloc(cells * sizeof(uint64_t));
    if (!q) return -1;
    uint64_t rd = 0, wr = 0;
    for (uint64_t i = 0; i < n_prefill; i++) q[wr++] = prefill[i];
    for (uint64_t i = 0; i < m; i++) {
        uint64_t size = wr - rd;
        if (op[i] == ORC_ENQ) {
            if (capacity != 0 && size >= capacity) {
                st_out[i] = ORC_FULL;
                val_out[i] = arg[i];
            } else {
                q[wr++] = arg[i];
                st_out[i] = ORC_OK;
                val_out[i] = arg[i];
            }
        } else {
            if (size == 0) {
                st_out[i] = ORC_EMPTY;
                val_out[i] = 0;
            } else {
                st_out[i] = ORC_OK;
                val_out[i] = q[rd++];
            }
        }
    }
    int64_t final_size = (int64_t)(wr - rd);
    if (residual_out)
        for (uint64_t i = rd; i < wr; i++) residual_out[i - rd] = q[i];
    free(q);
    return final_size;
}

/* ------------------------------------------------------------------------ */
/* O3: conservation.  The multiset of items put in (prefill plus every OK    */
/* enqueue) must equal the multiset taken out (every OK dequeue plus the     */
/* final drain).  Both sides are sorted and merged.                          */
/*   out_counts[0] = items put in but never taken out      (loss)            */
/*   out_counts[1] = items taken out but never put in, or taken out more     */
/*                   often than put in                     (fresh/duplicate) */
/*   out_counts[2] = values put in more than once (tokens must be unique)     */
/* Returns 0 iff all three are zero.                                          */
/* ------------------------------------------------------------------------ */
static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

int orc_conservation(uint64_t n_in, const uint64_t *in_vals, uint64_t n_out,
                     const uint64_t *out_vals, uint64_t *out_counts)
{
    uint64_t *a = (uint64_t *)malloc((n_in + 1) * sizeof(uint64_t));
    uint64_t *b = (uint64_t *)malloc((n_out + 1) * sizeof(uint64_t));
    if (!a || !b) { free(a); free(b); return -1; }
    memcpy(a, in_vals, n_in * sizeof(uint64_t));
    memcpy(b, out_vals, n_out * sizeof(uint64_t));
    qsort(a, n_in, sizeof(uint64_t), cmp_u64);
    qsort(b, n_out, sizeof(uint64_t), cmp_u64);
    uint64_t lost = 0, extra = 0, dup_in = 0;
    for (uint64_t i = 1; i < n_in; i++)
        if (a[i] == a[i - 1]) dup_in++;
    uint64_t i = 0, j = 0;
    while (i < n_in && j < n_out) {
        if (a[i] == b[j]) { i++; j++; }
        else if (a[i] < b[j]) { lost++; i++; }
        else { extra++; j++; }
    }
    lost += n_in - i;
    extra += n_out - j;
    out_counts[0] = lost;
    out_counts[1] = extra;
    out_counts[2] = dup_in;
    free(a);
    free(b);
    return (lost | extra | dup_in) ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Shared helpers for the interval checks.                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t key;   /* sort key */
    uint64_t idx;   /* payload: index into the owning array */
} kv_t;

static int cmp_kv(const void *a, const void *b)
{
    const kv_t *x = (const kv_t *)a, *y = (const kv_t *)b;
    if (x->key != y->key) return (x->key > y->key) - (x->key < y->key);
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* ------------------------------------------------------------------------ */
/* O4: per-producer order (Section IV, check (iii)), for tokens that encode  */
/* producer = val >> shift and seq = val & ((1 << shift) - 1).               */
/*   counts[0]: a consumer saw two tokens of one producer with the sequence  */
/*              numbers not strictly increasing in its program order;        */
/*   counts[1]: for one producer's seq i < j, deq(j) ended before deq(i)     */
/*              was called (FIFO: i is dequeued first);                       */
/*   counts[2]: a token was dequeued before its enqueue was called.           */
/* enq_* give the OK enqueues (value, call stamp); the history gives the     */
/* dequeues.  Returns 0 iff all counts are zero.                              */
/* ------------------------------------------------------------------------ */
int orc_producer_order(uint64_t m, const uint32_t *proc, const uint8_t *op,
                       const uint8_t *st, const uint64_t *val,
                       const uint64_t *call, const uint64_t *ret_t,
                       uint32_t shift, uint64_t *counts)
{
    uint64_t seq_mask = (shift >= 64) ? ~0ull : ((1ull << shift) - 1);
    counts[0] = counts[1] = counts[2] = 0;

    /* Collect OK dequeues and OK enqueues. */
    uint64_t nd = 0, ne = 0;
    for (uint64_t i = 0; i < m; i++) {
        if (st[i] != ORC_OK) continue;
        if (op[i] == ORC_DEQ) nd++; else ne++;
    }
    kv_t *d = (kv_t *)malloc((nd + 1) * sizeof(kv_t));
    kv_t *e = (kv_t *)malloc((ne + 1) * sizeof(kv_t));
    if (!d || !e) { free(d); free(e); return -1; }

    /* (1) per consumer: walk its dequeues in program order, remembering the */
    /* last sequence number seen from each producer.  The history is grouped */
    /* by process, so one consumer's dequeues are contiguous; sort them by   */
    /* (producer, position) and check the sequence numbers rise.             */
    uint64_t i = 0;
    while (i < m) {
        uint64_t j = i;
        while (j < m && proc[j] == proc[i]) j++;
        uint64_t k = 0;
        for (uint64_t x = i; x < j; x++)
            if (op[x] == ORC_DEQ && st[x] == ORC_OK) {
                d[k].key = val[x] >> shift;
                d[k].idx = x; /* program position */
                k++;
            }
        qsort(d, k, sizeof(kv_t), cmp_kv);
        for (uint64_t x = 1; x < k; x++)
            if (d[x].key == d[x - 1].key &&
                (val[d[x].idx] & seq_mask) <= (val[d[x - 1].idx] & seq_mask))
                counts[0]++;
        i = j;
    }

    /* (2) per producer: dequeues sorted by token (producer, seq). */
    nd = 0;
    ne = 0;
    for (uint64_t x = 0; x < m; x++) {
        if (st[x] != ORC_OK) continue;
        if (op[x] == ORC_DEQ) { d[nd].key = val[x]; d[nd].idx = x; nd++; }
        else { e[ne].key = val[x]; e[ne].idx = x; ne++; }
    }
    qsort(d, nd, sizeof(kv_t), cmp_kv);
    qsort(e, ne, sizeof(kv_t), cmp_kv);
    /* Within one producer, tokens ascend with seq.  Keep the latest call   */
    /* stamp among the producer's earlier tokens; deq(j).end before it is a */
    /* violation.                                                           */
    uint64_t x = 0;
    while (x < nd) {
        uint64_t y = x;
        uint64_t prod = d[x].key >> shift;
        uint64_t max_call = 0;
        int have = 0;
        while (y < nd && (d[y].key >> shift) == prod) {
            uint64_t r = d[y].idx;
            if (have && ret_t[r] < max_call) counts[1]++;
            if (!have || call[r] > max_call) max_call = call[r];
            have = 1;
            y++;
        }
        x = y;
    }
    /* (3) a dequeue must not end before the matching enqueue was called. */
    uint64_t a = 0, b = 0;
    while (a < nd && b < ne) {
        if (d[a].key == e[b].key) {
            if (ret_t[d[a].idx] < call[e[b].idx]) counts[2]++;
            a++;
        } else if (d[a].key < e[b].key) a++;
        else b++;
    }
    free(d);
    free(e);
    return (counts[0] | counts[1] | counts[2]) ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* O6: violation scan for histories too large for the exhaustive search.     */
/* Every pattern below is a proof that no linearization exists, so any hit  */
/* is a real violation (the scan is sound, not complete).  The patterns are  */
/* the classic queue-violation shapes:                                       */
/*   [0] VFresh  a dequeue returned a value never enqueued, or returned it   */
/*               before the enqueue was called;                               */
/*   [1] VRepet  a value was dequeued more than once;                         */
/*   [2] VOrd    enq(a) finished before enq(b) was called, yet deq(b)        */
/*               finished before deq(a) was called (a value never dequeued   */
/*               counts as dequeued at +infinity);                            */
/*   [3] VWit    an EMPTY dequeue ran while some value was certainly in the  */
/*               queue (its enqueue ended before the EMPTY was called and its */
/*               dequeue was called after the EMPTY ended, or never);         */
/*   [4] VWitN   an EMPTY dequeue ran while the count of certainly finished  */
/*               enqueues exceeded the count of possibly started dequeues;    */
/*   [5] VFull   a FULL enqueue ran while the queue could never have held    */
/*               `capacity` items (capacity 0 disables this check);          */
/*   [6] VLoss   a value was enqueued and never dequeued nor drained;         */
/*   [7] VWitU   an EMPTY dequeue ran while, at every instant of it, some     */
/*               value was certainly in the queue: the open intervals         */
/*               (enqueue end, dequeue call) of the values cover the EMPTY's  */
/*               whole [call, end], though no single one may (this finds      */
/*               EMPTY answers that VWit and VWitN miss).                     */
/* Prefill values count as enqueued, in order, before the history; drained  */
/* values count as dequeued, in order, after it.                             */
/* Returns 0 iff every count is zero.                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t val;
    int64_t ec, ee;   /* enqueue call / end   */
    int64_t dc, de;   /* dequeue call / end (INT64_MAX when never dequeued) */
} item_t;

static int cmp_item_val(const void *a, const void *b)
{
    const item_t *x = (const item_t *)a, *y = (const item_t *)b;
    return (x->val > y->val) - (x->val < y->val);
}

typedef struct { int64_t t; int64_t v; } tv_t;

static int cmp_tv(const void *a, const void *b)
{
    const tv_t *x = (const tv_t *)a, *y = (const tv_t *)b;
    if (x->t != y->t) return (x->t > y->t) - (x->t < y->t);
    return (x->v > y->v) - (x->v < y->v);
}

typedef struct { int64_t t0, t1; } iv_t;

static int cmp_iv_t0(const void *a, const void *b)
{
    const iv_t *x = (const iv_t *)a, *y = (const iv_t *)b;
    return (x->t0 > y->t0) - (x->t0 < y->t0);
}

/* Number of entries of the ascending array s[0..n) that are < t (or <= t). */
static uint64_t count_below(const int64_t *s, uint64_t n, int64_t t, int inclusive)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        int below = inclusive ? (s[mid] <= t) : (s[mid] < t);
        if (below) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* For each query interval q (t0 = call, t1 = end), decide whether some item */
/* has ee < q.t0 and dc > q.t1.  Items are given as (ee, dc) pairs sorted by */
/* ee; queries sorted by t0.  Returns the number of queries that match.      */
static uint64_t sweep_present(const tv_t *items_by_ee, uint64_t ni,
                              const iv_t *queries, uint64_t nq)
{
    uint64_t hits = 0, p = 0;
    int64_t best = INT64_MIN;
    for (uint64_t q = 0; q < nq; q++) {
        while (p < ni && items_by_ee[p].t < queries[q].t0) {
            if (items_by_ee[p].v > best) best = items_by_ee[p].v;
            p++;
        }
        if (p > 0 && best > queries[q].t1) hits++;
    }
    return hits;
}

int orc_violation_scan(uint64_t m, const uint8_t *op, const uint8_t *st,
                       const uint64_t *val, const uint64_t *call,
                       const uint64_t *ret_t, uint64_t n_prefill,
                       const uint64_t *prefill, uint64_t n_drain,
                       const uint64_t *drain, uint64_t capacity,
                       uint64_t *counts)
{
    for (int c = 0; c < 8; c++) counts[c] = 0;

    /* Map stamps to one signed time line: prefill item k occupies the      */
    /* instant 2k+1, the history starts after all of them, and drain item k */
    /* occupies tmax + 2 + 2k.                                              */
    uint64_t tmin = UINT64_MAX, tmax = 0;
    for (uint64_t i = 0; i < m; i++) {
        if (call[i] < tmin) tmin = call[i];
        if (ret_t[i] > tmax) tmax = ret_t[i];
    }
    if (m == 0) { tmin = 0; tmax = 0; }
    const int64_t base = 2 * (int64_t)n_prefill + 2;
#define T_OF(x) ((int64_t)((x) - tmin) + base)
    const int64_t drain0 = T_OF(tmax) + 2;

    uint64_t n_enq = n_prefill, n_deq = n_drain;
    for (uint64_t i = 0; i < m; i++)
        if (st[i] == ORC_OK) { if (op[i] == ORC_ENQ) n_enq++; else n_deq++; }

    item_t *E = (item_t *)malloc((n_enq + 1) * sizeof(item_t));
    item_t *D = (item_t *)malloc((n_deq + 1) * sizeof(item_t));
    if (!E || !D) { free(E); free(D); return -1; }
    uint64_t ie = 0, id = 0;
    for (uint64_t k = 0; k < n_prefill; k++) {
        E[ie].val = prefill[k];
        E[ie].ec = E[ie].ee = 2 * (int64_t)k + 1;
        ie++;
    }
    for (uint64_t i = 0; i < m; i++) {
        if (st[i] != ORC_OK) continue;
        if (op[i] == ORC_ENQ) {
            E[ie].val = val[i]; E[ie].ec = T_OF(call[i]); E[ie].ee = T_OF(ret_t[i]); ie++;
        } else {
            D[id].val = val[i]; D[id].dc = T_OF(call[i]); D[id].de = T_OF(ret_t[i]); id++;
        }
    }
    for (uint64_t k = 0; k < n_drain; k++) {
        D[id].val = drain[k];
        D[id].dc = D[id].de = drain0 + 2 * (int64_t)k;
        id++;
    }
    qsort(E, n_enq, sizeof(item_t), cmp_item_val);
    qsort(D, n_deq, sizeof(item_t), cmp_item_val);

    /* Match dequeues to enqueues by value (VFresh, VRepet, VLoss). */
    uint64_t a = 0, b = 0;
    while (a < n_enq || b < n_deq) {
        if (b >= n_deq || (a < n_enq && E[a].val < D[b].val)) {
            E[a].dc = E[a].de = INT64_MAX; /* never dequeued */
            counts[6]++;
            a++;
        } else if (a >= n_enq || D[b].val < E[a].val) {
            counts[0]++; /* value never enqueued */
            b++;
        } else {
            uint64_t v = E[a].val;
            E[a].dc = D[b].dc;
            E[a].de = D[b].de;
            if (D[b].de < E[a].ec) counts[0]++; /* returned before enqueue began */
            b++;
            while (b < n_deq && D[b].val == v) { counts[1]++; b++; }
            a++;
            /* further enqueues of the same value stay unmatched */
            while (a < n_enq && E[a].val == v) {
                E[a].dc = E[a].de = INT64_MAX;
                counts[6]++;
                a++;
            }
        }
    }

    /* VOrd: queries are the items b (by enqueue call); the candidates a are */
    /* items whose enqueue ended before b's enqueue call; violation when the */
    /* latest dequeue call among them exceeds b's dequeue end.  Items never  */
    /* dequeued cannot play b (their dequeue end is +infinity).              */
    tv_t *by_ee = (tv_t *)malloc((n_enq + 1) * sizeof(tv_t));
    iv_t *qs = (iv_t *)malloc((n_enq + m + 1) * sizeof(iv_t));
    if (!by_ee || !qs) { free(E); free(D); free(by_ee); free(qs); return -1; }
    for (uint64_t k = 0; k < n_enq; k++) { by_ee[k].t = E[k].ee; by_ee[k].v = E[k].dc; }
    qsort(by_ee, n_enq, sizeof(tv_t), cmp_tv);
    uint64_t nq = 0;
    for (uint64_t k = 0; k < n_enq; k++)
        if (E[k].de != INT64_MAX) { qs[nq].t0 = E[k].ec; qs[nq].t1 = E[k].de; nq++; }
    qsort(qs, nq, sizeof(iv_t), cmp_iv_t0);
    counts[2] = sweep_present(by_ee, n_enq, qs, nq);

    /* VWit: queries are the EMPTY dequeues. */
    nq = 0;
    for (uint64_t i = 0; i < m; i++)
        if (op[i] == ORC_DEQ && st[i] == ORC_EMPTY) {
            qs[nq].t0 = T_OF(call[i]); qs[nq].t1 = T_OF(ret_t[i]); nq++;
        }
    qsort(qs, nq, sizeof(iv_t), cmp_iv_t0);
    counts[3] = sweep_present(by_ee, n_enq, qs, nq);

    /* VWitU: merge the values' open presence intervals (ee, dc) -- sorted   */
    /* by ee in by_ee -- into disjoint segments; an EMPTY [t0, t1] is a hit  */
    /* when one segment (a, b) has a < t0 and t1 < b.  Two intervals merge   */
    /* only when they overlap (a shared end point is an uncovered instant).  */
    {
        iv_t *seg = (iv_t *)malloc((n_enq + 1) * sizeof(iv_t));
        if (!seg) { free(E); free(D); free(by_ee); free(qs); return -1; }
        uint64_t ns = 0;
        for (uint64_t k = 0; k < n_enq; k++) {
            const int64_t a = by_ee[k].t, b = by_ee[k].v;
            if (b <= a) continue;
            if (ns > 0 && a < seg[ns - 1].t1) {
                if (b > seg[ns - 1].t1) seg[ns - 1].t1 = b;
            } else {
                seg[ns].t0 = a;
                seg[ns].t1 = b;
                ns++;
            }
        }
        for (uint64_t q = 0; q < nq; q++) {
            /* last segment with t0 < query start */
            uint64_t lo = 0, hi = ns;
            while (lo < hi) {
                const uint64_t mid = (lo + hi) / 2;
                if (seg[mid].t0 < qs[q].t0) lo = mid + 1; else hi = mid;
            }
            if (lo > 0 && seg[lo - 1].t1 > qs[q].t1) counts[7]++;
        }
        free(seg);
    }

    /* VWitN and VFull use counts of stamps. */
    int64_t *enq_end = (int64_t *)malloc((n_enq + 1) * sizeof(int64_t));
    int64_t *enq_call = (int64_t *)malloc((n_enq + 1) * sizeof(int64_t));
    int64_t *deq_end = (int64_t *)malloc((n_deq + 1) * sizeof(int64_t));
    int64_t *deq_call = (int64_t *)malloc((n_deq + 1) * sizeof(int64_t));
    if (!enq_end || !enq_call || !deq_end || !deq_call) {
        free(E); free(D); free(by_ee); free(qs);
        free(enq_end); free(enq_call); free(deq_end); free(deq_call);
        return -1;
    }
    /* Only dequeues inside the history count here; drained values are     */
    /* dequeued after every history operation ended.                        */
    uint64_t nde = 0;
    for (uint64_t k = 0; k < n_enq; k++) { enq_end[k] = E[k].ee; enq_call[k] = E[k].ec; }
    for (uint64_t k = 0; k < n_deq; k++)
        if (D[k].dc < drain0) { deq_end[nde] = D[k].de; deq_call[nde] = D[k].dc; nde++; }
    qsort(enq_end, n_enq, sizeof(int64_t), cmp_i64);
    qsort(enq_call, n_enq, sizeof(int64_t), cmp_i64);
    qsort(deq_end, nde, sizeof(int64_t), cmp_i64);
    qsort(deq_call, nde, sizeof(int64_t), cmp_i64);
    for (uint64_t i = 0; i < m; i++) {
        if (op[i] == ORC_DEQ && st[i] == ORC_EMPTY) {
            /* lower bound on the size anywhere inside [call, end] */
            int64_t c = T_OF(call[i]), r = T_OF(ret_t[i]);
            int64_t lb = (int64_t)count_below(enq_end, n_enq, c, 0) -
                         (int64_t)count_below(deq_call, nde, r, 1);
            if (lb > 0) counts[4]++;
        } else if (op[i] == ORC_ENQ && st[i] == ORC_FULL && capacity != 0) {
            /* upper bound on the size anywhere inside [call, end] */
            int64_t c = T_OF(call[i]), r = T_OF(ret_t[i]);
            int64_t ub = (int64_t)count_below(enq_call, n_enq, r, 1) -
                         (int64_t)count_below(deq_end, nde, c, 0);
            if (ub < (int64_t)capacity) counts[5]++;
        }
    }
#undef T_OF
    free(E); free(D); free(by_ee); free(qs);
    free(enq_end); free(enq_call); free(deq_end); free(deq_call);
    for (int c = 0; c < 8; c++)
        if (counts[c]) return 1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O7: sequential queue BFS over a CSR graph (Section V-B).  level[v] is the  */
/* hop distance from root, UINT32_MAX when unreachable.  Returns the number  */
/* of levels (max level + 1); *edges_scanned counts adjacency entries read.   */
/* ------------------------------------------------------------------------ */
int64_t orc_bfs(uint64_t nv, const uint64_t *offsets, const uint32_t *cols,
                uint32_t root, uint32_t *level, uint64_t *edges_scanned)
{
    for (uint64_t v = 0; v < nv; v++) level[v] = UINT32_MAX;
    if (root >= nv) return -1;
    uint32_t *fifo = (uint32_t *)malloc((nv + 1) * sizeof(uint32_t));
    if (!fifo) return -1;
    uint64_t rd = 0, wr = 0, scanned = 0;
    uint32_t maxl = 0;
    level[root] = 0;
    fifo[wr++] = root;
    while (rd < wr) {
        uint32_t v = fifo[rd++];
        for (uint64_t e = offsets[v]; e < offsets[v + 1]; e++) {
            uint32_t u = cols[e];
            scanned++;
            if (level[u] == UINT32_MAX) {
                level[u] = level[v] + 1;
                if (level[u] > maxl) maxl = level[u];
                fifo[wr++] = u;
            }
        }
    }
    free(fifo);
    if (edges_scanned) *edges_scanned = scanned;
    return (int64_t)maxl + 1;
}

/* ------------------------------------------------------------------------ */
/* Host locked-queue baseline: a ring of `capacity` cells behind one mutex,  */
/* driven by nthreads host threads.  Thread t replays its own operation      */
/* stream roles[t*ops .. t*ops+ops) (0 = enqueue, 1 = dequeue), each op      */
/* tried once, enqueuing the token (t << 32) | (seq + 1).  The ring starts   */
/* with `prefill` items.  Reports successful enqueues and dequeues and the   */
/* elapsed wall time.  Measurement only: it is not a correctness check.      */
/* ------------------------------------------------------------------------ */
typedef struct {
    pthread_mutex_t mu;
    uint64_t *cells;
    uint64_t cap, rd, wr;
} locked_ring_t;

typedef struct {
    locked_ring_t *ring;
    const uint8_t *roles;
    uint64_t ops;
    uint32_t tid;
    uint64_t ok_enq, ok_deq;
} locked_arg_t;

static void *locked_worker(void *p)
{
    locked_arg_t *a = (locked_arg_t *)p;
    locked_ring_t *r = a->ring;
    uint64_t seq = 0, oke = 0, okd = 0;
    volatile uint64_t sink = 0;
    for (uint64_t k = 0; k < a->ops; k++) {
        uint8_t role = a->roles[k];
        pthread_mutex_lock(&r->mu);
        if (role == ORC_ENQ) {
            if (r->wr - r->rd < r->cap) {
                r->cells[r->wr % r->cap] = ((uint64_t)a->tid << 32) | (seq + 1);
                r->wr++;
                seq++;
                oke++;
            }
        } else if (r->wr != r->rd) {
            sink += r->cells[r->rd % r->cap];
            r->rd++;
            okd++;
        }
        pthread_mutex_unlock(&r->mu);
    }
    a->ok_enq = oke;
    a->ok_deq = okd;
    return NULL;
}

int orc_locked_queue_run(uint32_t nthreads, uint64_t ops_per_thread,
                         const uint8_t *roles, uint64_t capacity,
                         uint64_t prefill, uint64_t *ok_out, double *seconds)
{
    locked_ring_t ring;
    ring.cap = capacity;
    ring.cells = (uint64_t *)malloc(capacity * sizeof(uint64_t));
    if (!ring.cells) return -1;
    ring.rd = 0;
    ring.wr = 0;
    for (uint64_t i = 0; i < prefill && i < capacity; i++) ring.cells[ring.wr++] = i + 1;
    pthread_mutex_init(&ring.mu, NULL);
    pthread_t *th = (pthread_t *)malloc(nthreads * sizeof(pthread_t));
    locked_arg_t *args = (locked_arg_t *)malloc(nthreads * sizeof(locked_arg_t));
    if (!th || !args) { free(ring.cells); free(th); free(args); return -1; }
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    for (uint32_t t = 0; t < nthreads; t++) {
        args[t].ring = &ring;
        args[t].roles = roles + (uint64_t)t * ops_per_thread;
        args[t].ops = ops_per_thread;
        args[t].tid = t;
        args[t].ok_enq = args[t].ok_deq = 0;
        pthread_create(&th[t], NULL, locked_worker, &args[t]);
    }
    for (uint32_t t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    clock_gettime(CLOCK_MONOTONIC, &t1);
    ok_out[0] = ok_out[1] = 0;
    for (uint32_t t = 0; t < nthreads; t++) {
        ok_out[0] += args[t].ok_enq;
        ok_out[1] += args[t].ok_deq;
    }
    *seconds = (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
    pthread_mutex_destroy(&ring.mu);
    free(ring.cells);
    free(th);
    free(args);
    return 0;
}
