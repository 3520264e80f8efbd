/*
 * graphgen.c -- fast builders for the BFS inputs defined in workloads/__init__.py.
 *
 * Workload generation only (no queue arithmetic).  Produces exactly the
 * graphs the numpy definitions produce (tests compare them on small sizes):
 *   wl_rmat_pairs   R-MAT edge endpoints: for edge e and level l the quadrant
 *                   comes from u = splitmix64(seed, (e << 8) | l) against the
 *                   cumulative thresholds ta <= tab <= tabc;
 *   wl_csr          symmetrise, drop self loops, deduplicate, build CSR with
 *                   uint32 offsets and columns (rows ascending, columns
 *                   ascending within a row);
 *   wl_csr_par      the same, partitioned by row range over threads.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t splitmix64(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

typedef struct {
    uint64_t e0, e1, seed, ta, tab, tabc;
    uint32_t scale;
    uint64_t *src, *dst;
    const uint64_t *perm;  /* optional vertex relabelling */
} rmat_job_t;

static void *rmat_worker(void *p)
{
    rmat_job_t *j = (rmat_job_t *)p;
    for (uint64_t e = j->e0; e < j->e1; e++) {
        uint64_t s = 0, d = 0;
        for (uint32_t l = 0; l < j->scale; l++) {
            uint64_t u = splitmix64(j->seed, (e << 8) | l);
            uint64_t bit = 1ull << (j->scale - 1 - l);
            int right = (u >= j->ta && u < j->tab) || u >= j->tabc;
            int down = u >= j->tab;
            if (down) s |= bit;
            if (right) d |= bit;
        }
        j->src[e] = j->perm ? j->perm[s] : s;
        j->dst[e] = j->perm ? j->perm[d] : d;
    }
    return NULL;
}

int wl_rmat_pairs(uint32_t scale, uint64_t ne, uint64_t seed, uint64_t ta, uint64_t tab,
                  uint64_t tabc, uint64_t *src, uint64_t *dst, uint32_t threads, const uint64_t *perm)
{
    if (threads < 1) threads = 1;
    if (threads > 64) threads = 64;
    pthread_t th[64];
    rmat_job_t jobs[64];
    for (uint32_t t = 0; t < threads; t++) {
        jobs[t].e0 = ne * t / threads;
        jobs[t].e1 = ne * (t + 1) / threads;
        jobs[t].seed = seed;
        jobs[t].ta = ta;
        jobs[t].tab = tab;
        jobs[t].tabc = tabc;
        jobs[t].scale = scale;
        jobs[t].src = src;
        jobs[t].dst = dst;
        jobs[t].perm = perm;
        pthread_create(&th[t], NULL, rmat_worker, &jobs[t]);
    }
    for (uint32_t t = 0; t < threads; t++) pthread_join(th[t], NULL);
    return 0;
}

/* LSD radix sort of 64-bit keys, 16 bits per pass, skipping constant digits. */
static void radix_sort_u64(uint64_t *a, uint64_t n, uint64_t *tmp)
{
    uint64_t *src = a, *dst = tmp;
    uint64_t *count = (uint64_t *)malloc(65536 * sizeof(uint64_t));
    for (int pass = 0; pass < 4; pass++) {
        int shift = 16 * pass;
        memset(count, 0, 65536 * sizeof(uint64_t));
        for (uint64_t i = 0; i < n; i++) count[(src[i] >> shift) & 0xFFFF]++;
        int single = 0;
        for (int d = 0; d < 65536; d++)
            if (count[d] == n) single = 1;
        if (single) continue;
        uint64_t sum = 0;
        for (int d = 0; d < 65536; d++) {
            uint64_t c = count[d];
            count[d] = sum;
            sum += c;
        }
        for (uint64_t i = 0; i < n; i++) dst[count[(src[i] >> shift) & 0xFFFF]++] = src[i];
        uint64_t *t = src;
        src = dst;
        dst = t;
    }
    if (src != a) memcpy(a, src, n * sizeof(uint64_t));
    free(count);
}

/* Returns the number of CSR entries, or -1 on allocation failure / overflow.
 * offsets must hold nv + 1 entries; cols must hold 2 * m entries.           */
int64_t wl_csr(uint64_t nv, uint64_t m, const uint64_t *src, const uint64_t *dst,
               uint32_t *offsets, uint32_t *cols)
{
    uint64_t *key = (uint64_t *)malloc(2 * m * sizeof(uint64_t) + 8);
    uint64_t *tmp = (uint64_t *)malloc(2 * m * sizeof(uint64_t) + 8);
    if (!key || !tmp) { free(key); free(tmp); return -1; }
    uint64_t k = 0;
    for (uint64_t i = 0; i < m; i++) {
        if (src[i] == dst[i]) continue;
        key[k++] = (src[i] << 32) | dst[i];
        key[k++] = (dst[i] << 32) | src[i];
    }
    radix_sort_u64(key, k, tmp);
    free(tmp);
    uint64_t u = 0;
    for (uint64_t i = 0; i < k; i++)
        if (i == 0 || key[i] != key[i - 1]) key[u++] = key[i];
    if (u >= (1ull << 32)) { free(key); return -1; }
    memset(offsets, 0, (nv + 1) * sizeof(uint32_t));
    for (uint64_t i = 0; i < u; i++) offsets[(key[i] >> 32) + 1]++;
    for (uint64_t v = 0; v < nv; v++) offsets[v + 1] += offsets[v];
    for (uint64_t i = 0; i < u; i++) cols[i] = (uint32_t)(key[i] & 0xFFFFFFFFull);
    free(key);
    return (int64_t)u;
}

/* ---- parallel CSR build --------------------------------------------------
 * Keys (row << 32 | col) of both directions are partitioned by row range into
 * one bucket per thread, each bucket is sorted and deduplicated on its own,
 * and the buckets are concatenated.  Same output as wl_csr.                 */
typedef struct {
    uint32_t t, T;
    uint64_t nv, m;
    const uint64_t *src, *dst;
    uint64_t *counts;   /* [T][T]: counts[t * T + b] */
    uint64_t *bucket;   /* all keys, bucket-major */
    uint64_t *bstart;   /* [T + 1] bucket starts */
    uint64_t *tmp;
    uint64_t *uniq;     /* [T] unique counts */
    uint32_t *offsets, *cols;
    uint64_t *ustart;   /* [T + 1] output starts */
    int phase;
} csr_job_t;

static inline uint32_t row_bucket(uint64_t row, uint64_t nv, uint32_t T)
{
    return (uint32_t)(row * T / nv);
}

static void *csr_worker(void *p)
{
    csr_job_t *j = (csr_job_t *)p;
    const uint32_t T = j->T, t = j->t;
    const uint64_t e0 = j->m * t / T, e1 = j->m * (t + 1) / T;
    if (j->phase == 0) {
        uint64_t *c = j->counts + (uint64_t)t * T;
        for (uint32_t b = 0; b < T; b++) c[b] = 0;
        for (uint64_t e = e0; e < e1; e++) {
            if (j->src[e] == j->dst[e]) continue;
            c[row_bucket(j->src[e], j->nv, T)]++;
            c[row_bucket(j->dst[e], j->nv, T)]++;
        }
    } else if (j->phase == 1) {
        uint64_t *pos = (uint64_t *)malloc(T * sizeof(uint64_t));
        for (uint32_t b = 0; b < T; b++) {
            uint64_t o = j->bstart[b];
            for (uint32_t u = 0; u < t; u++) o += j->counts[(uint64_t)u * T + b];
            pos[b] = o;
        }
        for (uint64_t e = e0; e < e1; e++) {
            uint64_t s = j->src[e], d = j->dst[e];
            if (s == d) continue;
            j->bucket[pos[row_bucket(s, j->nv, T)]++] = (s << 32) | d;
            j->bucket[pos[row_bucket(d, j->nv, T)]++] = (d << 32) | s;
        }
        free(pos);
    } else if (j->phase == 2) {
        uint64_t *a = j->bucket + j->bstart[t];
        uint64_t n = j->bstart[t + 1] - j->bstart[t];
        radix_sort_u64(a, n, j->tmp + j->bstart[t]);
        uint64_t u = 0;
        for (uint64_t i = 0; i < n; i++)
            if (i == 0 || a[i] != a[i - 1]) a[u++] = a[i];
        j->uniq[t] = u;
    } else {
        const uint64_t *a = j->bucket + j->bstart[t];
        const uint64_t u = j->uniq[t];
        const uint64_t r0 = (j->nv * t + T - 1) / T;  /* first row of this bucket */
        uint64_t r1 = (j->nv * (t + 1) + T - 1) / T;
        if (r1 > j->nv) r1 = j->nv;
        uint64_t i = 0;
        for (uint64_t r = r0; r < r1; r++) {
            j->offsets[r] = (uint32_t)(j->ustart[t] + i);
            while (i < u && (a[i] >> 32) == r) {
                j->cols[j->ustart[t] + i] = (uint32_t)(a[i] & 0xFFFFFFFFull);
                i++;
            }
        }
    }
    return NULL;
}

static void run_phase(csr_job_t *jobs, uint32_t T, int phase)
{
    pthread_t th[64];
    for (uint32_t t = 0; t < T; t++) {
        jobs[t].phase = phase;
        pthread_create(&th[t], NULL, csr_worker, &jobs[t]);
    }
    for (uint32_t t = 0; t < T; t++) pthread_join(th[t], NULL);
}

int64_t wl_csr_par(uint64_t nv, uint64_t m, const uint64_t *src, const uint64_t *dst,
                   uint32_t *offsets, uint32_t *cols, uint32_t threads)
{
    uint32_t T = threads < 1 ? 1 : (threads > 64 ? 64 : threads);
    if (nv < T) T = 1;
    csr_job_t jobs[64];
    uint64_t *counts = (uint64_t *)calloc((uint64_t)T * T, sizeof(uint64_t));
    uint64_t *bstart = (uint64_t *)calloc(T + 1, sizeof(uint64_t));
    uint64_t *ustart = (uint64_t *)calloc(T + 1, sizeof(uint64_t));
    uint64_t *uniq = (uint64_t *)calloc(T, sizeof(uint64_t));
    uint64_t *bucket = (uint64_t *)malloc(2 * m * sizeof(uint64_t) + 8);
    uint64_t *tmp = (uint64_t *)malloc(2 * m * sizeof(uint64_t) + 8);
    if (!counts || !bstart || !ustart || !uniq || !bucket || !tmp) {
        free(counts); free(bstart); free(ustart); free(uniq); free(bucket); free(tmp);
        return -1;
    }
    for (uint32_t t = 0; t < T; t++) {
        jobs[t].t = t; jobs[t].T = T; jobs[t].nv = nv; jobs[t].m = m;
        jobs[t].src = src; jobs[t].dst = dst; jobs[t].counts = counts;
        jobs[t].bucket = bucket; jobs[t].bstart = bstart; jobs[t].tmp = tmp;
        jobs[t].uniq = uniq; jobs[t].offsets = offsets; jobs[t].cols = cols;
        jobs[t].ustart = ustart;
    }
    run_phase(jobs, T, 0);
    for (uint32_t b = 0; b < T; b++) {
        uint64_t c = 0;
        for (uint32_t t = 0; t < T; t++) c += counts[(uint64_t)t * T + b];
        bstart[b + 1] = bstart[b] + c;
    }
    run_phase(jobs, T, 1);
    run_phase(jobs, T, 2);
    for (uint32_t t = 0; t < T; t++) ustart[t + 1] = ustart[t] + uniq[t];
    int64_t total = (int64_t)ustart[T];
    if (total >= (int64_t)(1ull << 32)) {
        free(counts); free(bstart); free(ustart); free(uniq); free(bucket); free(tmp);
        return -1;
    }
    run_phase(jobs, T, 3);
    offsets[nv] = (uint32_t)total;
    free(counts); free(bstart); free(ustart); free(uniq); free(bucket); free(tmp);
    return total;
}
