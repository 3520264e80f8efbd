/*
 * gq_linsearch.c -- O10: linearization witness search for queue histories.
 *
 * TEST INFRASTRUCTURE ONLY (part of the CPU oracle; shares nothing with the
 * HIP queues).
 *
 * The paper checks its queues by searching for a linearization of recorded
 * histories against the sequential FIFO model (Section IV, "Linearizability
 * via Porcupine").  The exhaustive search (O5) only scales to ~20 operations
 * and the violation scan (O6) is sound but not complete, so an EMPTY answer in
 * a large history could be wrong without O6 noticing.  This search constructs
 * a linearization -- a total order of every operation that keeps real-time
 * precedence (x before y whenever x returned before y was called) and is a
 * legal run of the bounded FIFO -- and returns it.  A returned order is a
 * certificate: it can be checked independently by replaying it (O2) and
 * checking real time, which the Python wrapper's caller does.
 *
 * Model (the same as O5): an enqueue answered OK appends its value (illegal
 * when the state already holds `capacity` items, capacity 0 = unbounded); a
 * FULL enqueue has no effect and is legal in any state; a dequeue answered OK
 * returns and removes the head; an EMPTY dequeue is legal only in the empty
 * state.  Items are distinct (the token format makes them so).  Prefilled
 * items are in the state before the first operation; drained items are
 * dequeued one by one after the last operation, optionally followed by the
 * drain's final EMPTY answer.
 *
 * Search (the Wing-Gong / Lowe depth-first search, specialised to the FIFO).
 * An unlinearized operation is eligible when no unlinearized operation
 * returned before it was called, i.e. its call stamp is at most the smallest
 * return stamp among the unlinearized ones.  Three kinds of step are taken as
 * soon as they are eligible and legal, without branching, because taking them
 * earlier never removes a solution:
 *   - a FULL enqueue (no effect);
 *   - the dequeue of the item at the head (a smaller state only helps later
 *     enqueues and EMPTY answers; no other dequeue or EMPTY can come between);
 *   - an EMPTY dequeue when the state is empty (no effect).
 * Otherwise the next step must be an enqueue, and the search branches over the
 * eligible enqueues.  The first one tried is chosen just in time, from the
 * operation with the smallest return stamp: if it is a dequeue of an item not
 * yet enqueued, that item's enqueue; if it is an enqueue, that enqueue, unless
 * an eligible item must leave the queue before its item does (its dequeue
 * returns before the other dequeue is called), which then goes first.  The
 * others follow in the order in which their items must leave the queue at the
 * latest (the return stamp of the item's dequeue; items never dequeued last).
 * A dead end -- the operation with the smallest return stamp can never be
 * linearized (a dequeue whose item sits behind another, an EMPTY answer with
 * items present, an enqueue into a full state) -- backtracks.
 *
 * Modes: width 0 tries every eligible enqueue at each branch and memoises the
 * (linearized set, queue contents) states that failed, so a negative answer
 * is a proof; width w > 0 tries only the w best candidates per branch, for
 * histories of millions of operations, where a positive answer is still a
 * proof and a negative one is "unknown".  Either mode gives up (undecided)
 * after `budget` dead ends.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { LS_ENQ = 0, LS_DEQ = 1 };
enum { LS_OK = 0, LS_EMPTY = 1, LS_FULL = 2 };
enum { K_ENQ = 0, K_FULL = 1, K_DEQ = 2, K_EMP = 3 };

#define NONE32 0xFFFFFFFFu
#define INF64 UINT64_MAX

/* ---- min segment tree over u64 (iterative, n leaves at [n, 2n)) ---------- */
typedef struct {
    uint64_t *t;
    uint64_t n;
} seg_t;

static int seg_init(seg_t *s, uint64_t n)
{
    s->n = n;
    s->t = (uint64_t *)malloc(2 * n * sizeof(uint64_t));
    if (!s->t) return -1;
    memset(s->t, 0xFF, 2 * n * sizeof(uint64_t));
    return 0;
}

static void seg_build(seg_t *s)
{
    for (uint64_t i = s->n - 1; i >= 1; i--) {
        const uint64_t a = s->t[2 * i], b = s->t[2 * i + 1];
        s->t[i] = a < b ? a : b;
    }
}

static void seg_set(seg_t *s, uint64_t i, uint64_t v)
{
    i += s->n;
    s->t[i] = v;
    for (i >>= 1; i >= 1; i >>= 1) {
        const uint64_t a = s->t[2 * i], b = s->t[2 * i + 1];
        s->t[i] = a < b ? a : b;
    }
}

/* the minimum over all leaves (node 1 is the root for any n >= 1) */
static uint64_t seg_all(const seg_t *s) { return s->t[1]; }

static uint64_t seg_min(const seg_t *s, uint64_t l, uint64_t r)
{
    uint64_t res = INF64;
    for (l += s->n, r += s->n; l < r; l >>= 1, r >>= 1) {
        if (l & 1) {
            if (s->t[l] < res) res = s->t[l];
            l++;
        }
        if (r & 1) {
            r--;
            if (s->t[r] < res) res = s->t[r];
        }
    }
    return res;
}

/* ---- stable LSD radix sort of (key, id) pairs by key ---------------------- */
static int radix_sort(uint64_t *key, uint32_t *id, uint64_t n)
{
    uint64_t *k2 = (uint64_t *)malloc(n * sizeof(uint64_t) + 1);
    uint32_t *i2 = (uint32_t *)malloc(n * sizeof(uint32_t) + 1);
    if (!k2 || !i2) {
        free(k2);
        free(i2);
        return -1;
    }
    for (int pass = 0; pass < 4; pass++) {
        const int sh = 16 * pass;
        uint64_t cnt[65537];
        memset(cnt, 0, sizeof(cnt));
        for (uint64_t i = 0; i < n; i++) cnt[((key[i] >> sh) & 0xFFFF) + 1]++;
        for (int d = 0; d < 65536; d++) cnt[d + 1] += cnt[d];
        for (uint64_t i = 0; i < n; i++) {
            const uint64_t d = (key[i] >> sh) & 0xFFFF;
            k2[cnt[d]] = key[i];
            i2[cnt[d]] = id[i];
            cnt[d]++;
        }
        memcpy(key, k2, n * sizeof(uint64_t));
        memcpy(id, i2, n * sizeof(uint32_t));
    }
    free(k2);
    free(i2);
    return 0;
}

/* ---- failed-state memo (open addressing over 128-bit hashes) ------------- */
typedef struct {
    uint64_t *a, *b;
    uint64_t cap, used;
} memo_t;

static uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int memo_has(const memo_t *mm, uint64_t x, uint64_t y)
{
    if (!mm->cap) return 0;
    for (uint64_t i = x & (mm->cap - 1);; i = (i + 1) & (mm->cap - 1)) {
        if (mm->a[i] == 0 && mm->b[i] == 0) return 0;
        if (mm->a[i] == x && mm->b[i] == y) return 1;
    }
}

static int memo_put(memo_t *mm, uint64_t x, uint64_t y)
{
    if (x == 0 && y == 0) x = 1;
    if (2 * (mm->used + 1) > mm->cap) {
        const uint64_t nc = mm->cap ? 2 * mm->cap : 1024;
        uint64_t *na = (uint64_t *)calloc(nc, sizeof(uint64_t));
        uint64_t *nb = (uint64_t *)calloc(nc, sizeof(uint64_t));
        if (!na || !nb) {
            free(na);
            free(nb);
            return -1;
        }
        for (uint64_t i = 0; i < mm->cap; i++) {
            if (mm->a[i] == 0 && mm->b[i] == 0) continue;
            uint64_t j = mm->a[i] & (nc - 1);
            while (na[j] || nb[j]) j = (j + 1) & (nc - 1);
            na[j] = mm->a[i];
            nb[j] = mm->b[i];
        }
        free(mm->a);
        free(mm->b);
        mm->a = na;
        mm->b = nb;
        mm->cap = nc;
    }
    uint64_t i = x & (mm->cap - 1);
    while (mm->a[i] || mm->b[i]) {
        if (mm->a[i] == x && mm->b[i] == y) return 0;
        i = (i + 1) & (mm->cap - 1);
    }
    mm->a[i] = x;
    mm->b[i] = y;
    mm->used++;
    return 0;
}

/* ---- search state ---------------------------------------------------------- */
typedef struct {
    uint64_t M;                 /* operations, drain included */
    uint8_t *kind;              /* K_* */
    uint64_t *C, *R;            /* call / return stamps */
    uint64_t *V;                /* item values */
    uint32_t *byc;              /* operations sorted by call */
    uint32_t *posof;            /* position of an operation in byc */
    uint64_t *csorted;          /* call stamps in byc order */
    uint32_t *rrank;            /* rank of an operation's return stamp */
    uint32_t *partner;          /* enqueue -> its item's dequeue; dequeue -> enqueue; NONE32 */
    uint8_t *lin;               /* linearized? */
    seg_t tret, tenq, tfull, temp;
    uint32_t *qd;               /* queue: the dequeue op of each queued item (or NONE32) */
    uint64_t *qv;               /* queue: item values */
    uint64_t head, tail;
    uint64_t nlin;
    uint64_t *order;            /* the linearization built so far (the trail) */
    uint64_t zob;               /* Zobrist hash of the linearized set */
} ls_t;

static uint64_t enq_key(const ls_t *s, uint32_t o)
{
    const uint32_t d = s->partner[o];
    const uint64_t r = d == NONE32 ? s->M : s->rrank[d];
    return (r << 32) | s->posof[o];
}

static void do_lin(ls_t *s, uint32_t o)
{
    const uint32_t p = s->posof[o];
    s->lin[o] = 1;
    s->order[s->nlin++] = o;
    s->zob ^= mix64((uint64_t)o + 0x51ull);
    seg_set(&s->tret, p, INF64);
    switch (s->kind[o]) {
    case K_ENQ:
        seg_set(&s->tenq, p, INF64);
        s->qv[s->tail] = s->V[o];
        s->qd[s->tail] = s->partner[o];
        s->tail++;
        break;
    case K_FULL:
        seg_set(&s->tfull, p, INF64);
        break;
    case K_DEQ:
        s->head++;
        break;
    default:
        seg_set(&s->temp, p, INF64);
        break;
    }
}

static void undo_lin(ls_t *s)
{
    const uint32_t o = (uint32_t)s->order[--s->nlin];
    const uint32_t p = s->posof[o];
    s->lin[o] = 0;
    s->zob ^= mix64((uint64_t)o + 0x51ull);
    seg_set(&s->tret, p, ((uint64_t)s->rrank[o] << 32) | p);
    switch (s->kind[o]) {
    case K_ENQ:
        seg_set(&s->tenq, p, enq_key(s, o));
        s->tail--;
        break;
    case K_FULL:
        seg_set(&s->tfull, p, p);
        break;
    case K_DEQ:
        s->head--;
        break;
    default:
        seg_set(&s->temp, p, p);
        break;
    }
}

/* number of positions whose call stamp is <= x */
static uint64_t upper_bound(const uint64_t *a, uint64_t n, uint64_t x)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (a[mid] <= x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

typedef struct {
    uint64_t trail;             /* nlin when the branch was opened */
    uint64_t cstart, cn, cnext; /* its candidates in the candidate stack */
    uint64_t h1, h2;            /* state hash (exhaustive mode) */
} frame_t;

static void state_hash(const ls_t *s, uint64_t *h1, uint64_t *h2)
{
    uint64_t a = s->zob, b = mix64(s->zob ^ 0xA5A5ull);
    for (uint64_t i = s->head; i < s->tail; i++) {
        a = mix64(a ^ s->qv[i]);
        b = mix64(b + s->qv[i] * 0x100000001B3ull);
    }
    a = mix64(a ^ (s->tail - s->head));
    *h1 = a;
    *h2 = b;
}

static int cmp_u64(const void *x, const void *y)
{
    const uint64_t a = *(const uint64_t *)x, b = *(const uint64_t *)y;
    return a < b ? -1 : a > b;
}

/*
 * Returns 1 (order[] holds a linearization: indices < m are history
 * operations, m + j is the j-th drained item's dequeue, m + n_drain the
 * drain's final EMPTY), 0 (no linearization exists; only when the search was
 * complete), -1 (undecided: dead-end budget or candidate width exhausted), -2
 * (unsupported input: an item enqueued twice, an impossible op/status pair,
 * 2^32 or more operations), -3 (out of memory).
 * info[0] = branch points opened, info[1] = backtracks, info[2] = the longest
 * linearized prefix reached, info[3] = the operation with the smallest return
 * stamp at the dead end that ended that prefix (or ~0).
 */
int orc_lin_witness(uint64_t m, const uint8_t *op, const uint8_t *st, const uint64_t *val,
                    const uint64_t *call, const uint64_t *ret_t, uint64_t n_pre,
                    const uint64_t *pre, uint64_t n_drain, const uint64_t *drain,
                    int drain_ends_empty, uint64_t capacity, uint64_t budget, uint32_t width,
                    uint64_t *order, uint64_t *info)
{
    const uint64_t M = m + n_drain + (drain_ends_empty ? 1 : 0);
    info[0] = info[1] = info[2] = 0;
    info[3] = ~0ull;
    if (M == 0) return 1;
    if (M >= NONE32) return -2;
    int rc = -3;
    ls_t s;
    memset(&s, 0, sizeof(s));
    s.M = M;
    s.order = order;
    frame_t *fr = NULL;
    uint64_t *cand = NULL, *keys = NULL, *vk = NULL;
    uint32_t *vid = NULL, *bid = NULL;
    memo_t memo = {0};
    uint64_t nfr = 0, frcap = 0, ncand = 0, candcap = 0;

    s.kind = (uint8_t *)malloc(M);
    s.C = (uint64_t *)malloc(M * 8);
    s.R = (uint64_t *)malloc(M * 8);
    s.V = (uint64_t *)malloc(M * 8);
    s.byc = (uint32_t *)malloc(M * 4);
    s.posof = (uint32_t *)malloc(M * 4);
    s.csorted = (uint64_t *)malloc(M * 8);
    s.rrank = (uint32_t *)malloc(M * 4);
    s.partner = (uint32_t *)malloc(M * 4);
    s.lin = (uint8_t *)calloc(M, 1);
    keys = (uint64_t *)malloc(M * 8);
    bid = (uint32_t *)malloc(M * 4);
    if (!s.kind || !s.C || !s.R || !s.V || !s.byc || !s.posof || !s.csorted || !s.rrank ||
        !s.partner || !s.lin || !keys || !bid)
        goto out;

    /* operations: the history, then the drain's dequeues (and final EMPTY)
       stamped after everything, one after another */
    uint64_t tmax = 0;
    for (uint64_t i = 0; i < m; i++) {
        if (ret_t[i] > tmax) tmax = ret_t[i];
        if (call[i] > tmax) tmax = call[i];
    }
    for (uint64_t i = 0; i < m; i++) {
        s.C[i] = call[i];
        s.R[i] = ret_t[i];
        s.V[i] = val[i];
        if (op[i] == LS_ENQ && st[i] == LS_OK) s.kind[i] = K_ENQ;
        else if (op[i] == LS_ENQ && st[i] == LS_FULL) s.kind[i] = K_FULL;
        else if (op[i] == LS_DEQ && st[i] == LS_OK) s.kind[i] = K_DEQ;
        else if (op[i] == LS_DEQ && st[i] == LS_EMPTY) s.kind[i] = K_EMP;
        else {
            rc = -2;
            goto out;
        }
        if (ret_t[i] < call[i]) {
            rc = -2;
            goto out;
        }
    }
    for (uint64_t j = 0; j < M - m; j++) {
        const uint64_t i = m + j;
        s.C[i] = tmax + 1 + 2 * j;
        s.R[i] = tmax + 2 + 2 * j;
        if (j < n_drain) {
            s.kind[i] = K_DEQ;
            s.V[i] = drain[j];
        } else {
            s.kind[i] = K_EMP;
            s.V[i] = 0;
        }
    }

    /* sort by call (positions), and rank return stamps */
    for (uint64_t i = 0; i < M; i++) {
        keys[i] = s.C[i];
        bid[i] = (uint32_t)i;
    }
    if (radix_sort(keys, bid, M)) goto out;
    for (uint64_t k = 0; k < M; k++) {
        s.byc[k] = bid[k];
        s.posof[bid[k]] = (uint32_t)k;
        s.csorted[k] = keys[k];
    }
    for (uint64_t i = 0; i < M; i++) {
        keys[i] = s.R[i];
        bid[i] = (uint32_t)i;
    }
    if (radix_sort(keys, bid, M)) goto out;
    for (uint64_t k = 0; k < M; k++) s.rrank[bid[k]] = (uint32_t)k;

    /* pair every item's enqueue (or prefill slot) with its dequeue */
    {
        uint64_t ne = n_pre, nd = 0;
        for (uint64_t i = 0; i < M; i++) {
            if (s.kind[i] == K_ENQ) ne++;
            if (s.kind[i] == K_DEQ) nd++;
        }
        vk = (uint64_t *)malloc((ne + nd + 1) * 8);
        vid = (uint32_t *)malloc((ne + nd + 1) * 4);
        if (!vk || !vid) goto out;
        /* enqueue side: ids M + j for prefill slot j, i for operations */
        uint64_t c = 0;
        for (uint64_t j = 0; j < n_pre; j++) {
            vk[c] = pre[j];
            vid[c++] = (uint32_t)(M + j) ;
        }
        if (M + n_pre >= NONE32) {
            rc = -2;
            goto out;
        }
        for (uint64_t i = 0; i < M; i++)
            if (s.kind[i] == K_ENQ) {
                vk[c] = s.V[i];
                vid[c++] = (uint32_t)i;
            }
        if (radix_sort(vk, vid, ne)) goto out;
        for (uint64_t k = 1; k < ne; k++)
            if (vk[k] == vk[k - 1]) {
                rc = -2;  /* an item enqueued twice: outside this search's model */
                goto out;
            }
        uint64_t *dk = vk + ne;
        uint32_t *did = vid + ne;
        c = 0;
        for (uint64_t i = 0; i < M; i++)
            if (s.kind[i] == K_DEQ) {
                dk[c] = s.V[i];
                did[c++] = (uint32_t)i;
            }
        if (radix_sort(dk, did, nd)) goto out;
        for (uint64_t i = 0; i < M; i++) s.partner[i] = NONE32;
        uint32_t *pre_partner = (uint32_t *)malloc((n_pre + 1) * 4);
        if (!pre_partner) goto out;
        for (uint64_t j = 0; j < n_pre; j++) pre_partner[j] = NONE32;
        uint64_t a = 0;
        int bad = 0;
        for (uint64_t k = 0; k < nd; k++) {
            if (k && dk[k] == dk[k - 1]) bad = 1;  /* dequeued twice */
            while (a < ne && vk[a] < dk[k]) a++;
            if (a >= ne || vk[a] != dk[k]) {
                bad = 1;                            /* never enqueued */
                continue;
            }
            if (vid[a] >= M) pre_partner[vid[a] - M] = did[k];
            else s.partner[vid[a]] = did[k];
            s.partner[did[k]] = vid[a] >= M ? NONE32 - 1 : vid[a];  /* NONE32-1: prefill */
        }
        if (bad) {
            free(pre_partner);
            rc = 0;
            goto out;
        }
        /* the queue starts with the prefill */
        s.qv = (uint64_t *)malloc((ne + 1) * 8);
        s.qd = (uint32_t *)malloc((ne + 1) * 4);
        if (!s.qv || !s.qd) {
            free(pre_partner);
            goto out;
        }
        for (uint64_t j = 0; j < n_pre; j++) {
            s.qv[j] = pre[j];
            s.qd[j] = pre_partner[j];
        }
        free(pre_partner);
        s.head = 0;
        s.tail = n_pre;
    }
    free(vk);
    free(vid);
    vk = NULL;
    vid = NULL;

    if (seg_init(&s.tret, M) || seg_init(&s.tenq, M) || seg_init(&s.tfull, M) ||
        seg_init(&s.temp, M))
        goto out;
    for (uint64_t i = 0; i < M; i++) {
        const uint64_t p = s.posof[i];
        s.tret.t[M + p] = ((uint64_t)s.rrank[i] << 32) | p;
        if (s.kind[i] == K_ENQ) s.tenq.t[M + p] = enq_key(&s, (uint32_t)i);
        if (s.kind[i] == K_FULL) s.tfull.t[M + p] = p;
        if (s.kind[i] == K_EMP) s.temp.t[M + p] = p;
    }
    seg_build(&s.tret);
    seg_build(&s.tenq);
    seg_build(&s.tfull);
    seg_build(&s.temp);
    free(keys);
    free(bid);
    keys = NULL;
    bid = NULL;

    int truncated = 0;
    uint64_t branches = 0, backtracks = 0;
    for (;;) {
        if (s.nlin == M) {
            rc = 1;
            break;
        }
        const uint64_t top = seg_all(&s.tret);
        const uint32_t om = s.byc[(uint32_t)top];
        const uint64_t E = upper_bound(s.csorted, M, s.R[om]);
        /* steps that never need a branch */
        const uint64_t f = seg_all(&s.tfull);
        if (f < E) {
            do_lin(&s, s.byc[f]);
            continue;
        }
        if (s.head < s.tail) {
            const uint32_t d = s.qd[s.head];
            if (d < NONE32 - 1 && s.posof[d] < E) {
                do_lin(&s, d);
                continue;
            }
        } else {
            const uint64_t e = seg_all(&s.temp);
            if (e < E) {
                do_lin(&s, s.byc[e]);
                continue;
            }
        }
        /* a branch over eligible enqueues, or a dead end */
        int dead = 0;
        uint32_t first = NONE32;
        if (capacity && s.tail - s.head >= capacity) {
            dead = 1;
        } else if (s.kind[om] == K_DEQ) {
            const uint32_t e = s.partner[om];
            if (e >= NONE32 - 1 || s.lin[e] || s.posof[e] >= E) dead = 1;
            else first = e;
        } else if (s.kind[om] == K_ENQ) {
            /* om's enqueue is due.  An eligible item whose dequeue must end
               before om's item's dequeue starts has to be ahead of it in the
               queue; the one with the earliest deadline is tried first.  Any
               other item waits: enqueued now it could block an item that
               arrives later with an earlier deadline. */
            const uint32_t w = s.byc[(uint32_t)seg_min(&s.tenq, 0, E)];
            const uint32_t dw = s.partner[w], dz = s.partner[om];
            first = (w != om && dw != NONE32 && (dz == NONE32 || s.R[dw] < s.C[dz])) ? w : om;
        } else {
            dead = 1;  /* an EMPTY answer with items present */
        }
        uint64_t h1 = 0, h2 = 0;
        if (!dead && width == 0) {
            state_hash(&s, &h1, &h2);
            if (memo_has(&memo, h1 ? h1 : 1, h2)) dead = 1;
        }
        if (!dead) {
            branches++;
            /* candidates: `first`, then the others by key */
            if (nfr == frcap) {
                frcap = frcap ? 2 * frcap : 1024;
                frame_t *nf = (frame_t *)realloc(fr, frcap * sizeof(frame_t));
                if (!nf) goto out;
                fr = nf;
            }
            frame_t *F = &fr[nfr++];
            F->trail = s.nlin;
            F->cstart = ncand;
            F->cnext = 1;
            F->h1 = h1;
            F->h2 = h2;
            uint64_t want = width ? width : E;
            if (ncand + want + 1 > candcap) {
                candcap = 2 * (ncand + want + 1);
                uint64_t *nc = (uint64_t *)realloc(cand, candcap * 8);
                if (!nc) goto out;
                cand = nc;
            }
            cand[ncand++] = first;
            if (width == 0) {
                /* every other eligible enqueue, by key */
                const uint64_t c0 = ncand;
                for (uint64_t p = 0; p < E; p++) {
                    const uint32_t o = s.byc[p];
                    if (o != first && s.kind[o] == K_ENQ && !s.lin[o]) cand[ncand++] = enq_key(&s, o);
                }
                qsort(cand + c0, ncand - c0, 8, cmp_u64);
                for (uint64_t k = c0; k < ncand; k++) cand[k] = s.byc[(uint32_t)cand[k]];
            } else {
                /* the next width - 1 by key: take them out of the tree in turn;
                   one more found means the branch is cut short */
                const uint64_t c0 = ncand;
                const uint64_t fk = enq_key(&s, first);
                seg_set(&s.tenq, s.posof[first], INF64);
                for (uint32_t w = 1; w <= width; w++) {
                    const uint64_t k = seg_min(&s.tenq, 0, E);
                    if (k == INF64) break;
                    if (w == width) {
                        truncated = 1;
                        break;
                    }
                    cand[ncand++] = s.byc[(uint32_t)k];
                    seg_set(&s.tenq, (uint32_t)k, INF64);
                }
                for (uint64_t k = c0; k < ncand; k++)
                    seg_set(&s.tenq, s.posof[cand[k]], enq_key(&s, (uint32_t)cand[k]));
                seg_set(&s.tenq, s.posof[first], fk);
            }
            F->cn = ncand - F->cstart;
            do_lin(&s, first);
            continue;
        }
        /* dead end: back to the latest branch with an untried candidate */
        if (s.nlin >= info[2]) {
            info[2] = s.nlin;
            info[3] = om;
        }
        if (++backtracks > budget) {
            rc = -1;
            break;
        }
        int resumed = 0;
        while (nfr) {
            frame_t *F = &fr[nfr - 1];
            while (s.nlin > F->trail) undo_lin(&s);
            if (F->cnext < F->cn) {
                do_lin(&s, (uint32_t)cand[F->cstart + F->cnext++]);
                resumed = 1;
                break;
            }
            if (width == 0 && memo_put(&memo, F->h1 ? F->h1 : 1, F->h2)) goto out;
            ncand = F->cstart;
            nfr--;
        }
        if (!resumed) {
            while (s.nlin) undo_lin(&s);
            rc = truncated ? -1 : 0;
            break;
        }
    }
    info[0] = branches;
    info[1] = backtracks;
    if (rc == 1) info[2] = M;

out:
    free(s.kind);
    free(s.C);
    free(s.R);
    free(s.V);
    free(s.byc);
    free(s.posof);
    free(s.csorted);
    free(s.rrank);
    free(s.partner);
    free(s.lin);
    free(s.tret.t);
    free(s.tenq.t);
    free(s.tfull.t);
    free(s.temp.t);
    free(s.qd);
    free(s.qv);
    free(fr);
    free(cand);
    free(keys);
    free(bid);
    free(vk);
    free(vid);
    free(memo.a);
    free(memo.b);
    return rc;
}
