/*
 * esq_oracle.c -- plain, slow, obviously correct CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the GPU library.
 *
 * What it computes (Hercher, "On the Sum of Squarefree Integers and a Power
 * of Two", arXiv 2411.01964):
 *
 *   * Erdos' conjecture (Section 1, Conjecture): an odd n > 1 is m + 2^k with
 *     m squarefree.  Following Section 2 (events A_k) and Section 3 (k = 0 is
 *     excluded, so n - 2^k is odd), we look for the least k >= 1 with
 *     m = n - 2^k >= 1 squarefree.  1 counts as squarefree (mu(1) = 1).
 *   * Squarefreeness of an odd m is decided exactly as Section 2 defines the
 *     event A_k: m is squarefree iff no p^2 divides it, p running over the
 *     odd primes (2^2 never divides an odd number).  This file tests every
 *     odd prime p with p*p <= m by plain trial division: no sieve, no
 *     blocking, no shortcut.
 *   * Algorithm 2 (Section 3): per odd n, k = 1, 2, ... until n - 2^k is
 *     squarefree or the search limit is passed.  The limit is
 *     kmax (when kmax > 0) and always 2^k < n (positivity).
 *   * Section 3, "Collecting the results": aggregates over the interval --
 *     per-k counts (Table 4 style), sum of least k, maximum least k -- plus
 *     the record-setters of Table 3 and the list of n with no representation
 *     (Algorithm 2's "no representation found" report).
 *   * Algorithm 1 alone: the squarefree flag of every odd number in
 *     [lo, hi).
 *
 * Readings where the paper is silent (each restated in the design notes):
 *   - ranges are half-open [lo, hi); only odd n >= 3 are examined;
 *   - a record-setter is an n (ascending order inside the call) whose depth
 *     d(n) is strictly larger than the depth of every smaller n of the call,
 *     where d(n) = least k, or "infinity" when no k was found; such an
 *     exception is reported as a record with k = 0 and nothing after it can
 *     be a record;
 *   - exceptions are reported in ascending order.
 *
 * Multi-threading splits the n-range into contiguous chunks; per-chunk
 * results are merged in chunk order (counts add, records keep the entries
 * that beat the running maximum of all earlier chunks, exceptions
 * concatenate).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- primes */

static uint32_t *g_primes;    /* odd primes 3, 5, 7, ... */
static uint64_t *g_psq;       /* their squares */
static size_t g_nprimes;
static uint64_t g_plimit;     /* every odd prime <= g_plimit is present */
static pthread_mutex_t g_plock = PTHREAD_MUTEX_INITIALIZER;

static uint64_t isqrt_u64(uint64_t x)
{
    uint64_t r = 0, bit;
    for (bit = (uint64_t)1 << 62; bit > x; bit >>= 2) {
    }
    for (; bit; bit >>= 2) {
        if (x >= r + bit) {
            x -= r + bit;
            r = (r >> 1) + bit;
        } else {
            r >>= 1;
        }
    }
    return r;
}

/* Sieve of Eratosthenes over 0..limit (one byte per integer). */
int oracle_prepare(uint64_t limit)
{
    int rc = 0;
    pthread_mutex_lock(&g_plock);
    if (g_primes && g_plimit >= limit)
        goto out;
    if (limit < 3)
        limit = 3;
    {
        unsigned char *comp = (unsigned char *)calloc(limit + 1, 1);
        uint32_t *pr;
        uint64_t *sq;
        size_t cnt = 0, i, j;
        if (!comp) {
            rc = -1;
            goto out;
        }
        for (i = 2; i * i <= limit; i++)
            if (!comp[i])
                for (j = i * i; j <= limit; j += i)
                    comp[j] = 1;
        for (i = 3; i <= limit; i += 2)
            cnt += !comp[i];
        pr = (uint32_t *)malloc((cnt + 1) * sizeof(uint32_t));
        sq = (uint64_t *)malloc((cnt + 1) * sizeof(uint64_t));
        if (!pr || !sq) {
            free(comp);
            free(pr);
            free(sq);
            rc = -1;
            goto out;
        }
        cnt = 0;
        for (i = 3; i <= limit; i += 2)
            if (!comp[i]) {
                pr[cnt] = (uint32_t)i;
                sq[cnt] = (uint64_t)i * i;
                cnt++;
            }
        free(comp);
        free(g_primes);
        free(g_psq);
        g_primes = pr;
        g_psq = sq;
        g_nprimes = cnt;
        g_plimit = limit;
    }
out:
    pthread_mutex_unlock(&g_plock);
    return rc;
}

size_t oracle_nprimes(void) { return g_nprimes; }
const uint32_t *oracle_primes(void) { return g_primes; }

/* ------------------------------------------------------- the definitions */

/* m >= 1 odd.  Returns 1 iff no odd prime square divides m.  The caller
 * guarantees that the prime list reaches isqrt(m) (oracle_prepare). */
int oracle_is_squarefree(uint64_t m)
{
    size_t i;
    for (i = 0; i < g_nprimes && g_psq[i] <= m; i++)
        if (m % g_psq[i] == 0)
            return 0;
    return 1;
}

/* Algorithm 2 for one odd n >= 3: least k >= 1 with n - 2^k >= 1 squarefree,
 * trying k while 2^k < n and (kmax == 0 or k <= kmax).  0 = none found. */
unsigned oracle_mink(uint64_t n, unsigned kmax)
{
    unsigned k;
    for (k = 1; k < 64; k++) {
        uint64_t pk = (uint64_t)1 << k;
        if (pk >= n)
            break;
        if (kmax && k > kmax)
            break;
        if (oracle_is_squarefree(n - pk))
            return k;
    }
    return 0;
}

/* ----------------------------------------------------- interval driver */

typedef struct {
    uint64_t n0;          /* first odd n examined (0 if none) */
    uint64_t n_odd;       /* how many odd n were examined */
    uint64_t hist[65];    /* hist[0] = exceptions, hist[k] = n with least k */
    uint64_t ksum;        /* sum of least k over n with a representation */
    uint32_t kmax_seen;   /* largest least k found */
    uint32_t n_records;   /* number of record-setters (may exceed capacity) */
    uint64_t n_exceptions;
} oracle_summary;

typedef struct {
    uint64_t n;
    uint32_t k;     /* 0 = exception (depth "infinity") */
    uint32_t flags; /* k = 0 only: 1 when the search stopped at kmax while a
                       larger k still gave a positive n - 2^k, 0 when every k
                       with 2^k < n was tried */
} oracle_record;

/* Why Algorithm 2 found no representation of n (its "no representation
 * found" report, Section 3): 1 = the limit kmax cut the search short, i.e.
 * the next exponent kmax + 1 still has 2^(kmax+1) < n; 0 = the positivity
 * bound 2^k < n ended it. */
static uint32_t exception_kind(uint64_t n, unsigned kmax)
{
    if (kmax == 0 || kmax >= 63)
        return 0;
    return ((uint64_t)1 << (kmax + 1)) < n ? 1u : 0u;
}

typedef struct {
    /* input */
    uint64_t first_n, count;
    unsigned kmax;
    uint8_t *per_n; /* optional, indexed from the call's first n */
    uint64_t per_n_offset;
    /* output */
    uint64_t hist[65];
    uint64_t ksum;
    uint32_t kmax_seen;
    oracle_record *recs; /* local records of this chunk (<= 65) */
    size_t nrecs;
    uint64_t *exc;
    size_t nexc, exc_cap;
} chunk_t;

static void *chunk_run(void *arg)
{
    chunk_t *c = (chunk_t *)arg;
    uint64_t i;
    unsigned depth_max = 0; /* 0 = nothing seen yet; 65 = "infinity" */
    for (i = 0; i < c->count; i++) {
        uint64_t n = c->first_n + 2 * i;
        unsigned k = oracle_mink(n, c->kmax);
        unsigned depth = k ? k : 65;
        c->hist[k]++;
        c->ksum += k;
        if (k > c->kmax_seen)
            c->kmax_seen = k;
        if (c->per_n)
            c->per_n[c->per_n_offset + i] = (uint8_t)k;
        if (depth > depth_max) {
            c->recs[c->nrecs].n = n;
            c->recs[c->nrecs].k = k;
            c->recs[c->nrecs].flags = k ? 0u : exception_kind(n, c->kmax);
            c->nrecs++;
            depth_max = depth;
        }
        if (k == 0) {
            if (c->nexc < c->exc_cap)
                c->exc[c->nexc] = n;
            c->nexc++;
        }
    }
    return NULL;
}

/*
 * Every odd n in [lo, hi) with n >= 3.  out_per_n (optional) receives
 * n_odd bytes.  records / exceptions receive at most rec_cap / exc_cap
 * entries in ascending n; the summary holds the exact totals.
 * Returns 0, or -1 on allocation failure.
 */
int oracle_verify_range(uint64_t lo, uint64_t hi, unsigned kmax, int nthreads,
                        uint8_t *out_per_n, oracle_summary *sum,
                        oracle_record *records, size_t rec_cap,
                        uint64_t *exceptions, size_t exc_cap)
{
    uint64_t n0, n_odd, per, start;
    chunk_t *ch;
    pthread_t *th;
    int t, nt;
    unsigned run_max = 0;
    size_t nrec = 0, nexc = 0, j, k;

    memset(sum, 0, sizeof(*sum));
    if (lo < 3)
        lo = 3;
    n0 = lo | 1;
    if (hi <= n0)
        return 0;
    n_odd = (hi - n0 + 1) / 2;
    sum->n0 = n0;
    sum->n_odd = n_odd;
    if (oracle_prepare(isqrt_u64(hi)) != 0)
        return -1;

    nt = nthreads > 0 ? nthreads : 1;
    if ((uint64_t)nt > n_odd)
        nt = (int)n_odd;
    ch = (chunk_t *)calloc((size_t)nt, sizeof(chunk_t));
    th = (pthread_t *)calloc((size_t)nt, sizeof(pthread_t));
    if (!ch || !th) {
        free(ch);
        free(th);
        return -1;
    }
    per = n_odd / (uint64_t)nt;
    start = 0;
    for (t = 0; t < nt; t++) {
        uint64_t cnt = per + ((uint64_t)t < n_odd % (uint64_t)nt ? 1 : 0);
        ch[t].first_n = n0 + 2 * start;
        ch[t].count = cnt;
        ch[t].kmax = kmax;
        ch[t].per_n = out_per_n;
        ch[t].per_n_offset = start;
        ch[t].recs = (oracle_record *)calloc(66, sizeof(oracle_record));
        ch[t].exc_cap = exc_cap;
        ch[t].exc = exc_cap ? (uint64_t *)malloc(exc_cap * sizeof(uint64_t)) : NULL;
        start += cnt;
    }
    for (t = 0; t < nt; t++)
        pthread_create(&th[t], NULL, chunk_run, &ch[t]);
    for (t = 0; t < nt; t++)
        pthread_join(th[t], NULL);

    /* merge in chunk order */
    for (t = 0; t < nt; t++) {
        for (k = 0; k < 65; k++)
            sum->hist[k] += ch[t].hist[k];
        sum->ksum += ch[t].ksum;
        if (ch[t].kmax_seen > sum->kmax_seen)
            sum->kmax_seen = ch[t].kmax_seen;
        for (j = 0; j < ch[t].nrecs; j++) {
            unsigned depth = ch[t].recs[j].k ? ch[t].recs[j].k : 65;
            if (depth > run_max) {
                if (nrec < rec_cap) {
                    records[nrec].n = ch[t].recs[j].n;
                    records[nrec].k = ch[t].recs[j].k;
                    records[nrec].flags = ch[t].recs[j].flags;
                }
                nrec++;
                run_max = depth;
            }
        }
        for (j = 0; j < ch[t].nexc && j < ch[t].exc_cap; j++) {
            if (nexc < exc_cap)
                exceptions[nexc] = ch[t].exc[j];
            nexc++;
        }
        free(ch[t].recs);
        free(ch[t].exc);
    }
    sum->n_records = (uint32_t)nrec;
    sum->n_exceptions = sum->hist[0];
    free(ch);
    free(th);
    return 0;
}

/* ------------------------------------------------ Algorithm 1 alone */

typedef struct {
    uint64_t m0;
    uint64_t w_begin, w_end, n_odd;
    uint64_t *bits;
} sieve_chunk_t;

static void *sieve_chunk_run(void *arg)
{
    sieve_chunk_t *c = (sieve_chunk_t *)arg;
    uint64_t w, b;
    for (w = c->w_begin; w < c->w_end; w++) {
        uint64_t word = 0;
        for (b = 0; b < 64; b++) {
            uint64_t i = w * 64 + b;
            if (i >= c->n_odd)
                break;
            if (oracle_is_squarefree(c->m0 + 2 * i))
                word |= (uint64_t)1 << b;
        }
        c->bits[w] = word;
    }
    return NULL;
}

/*
 * Squarefree flag of every odd m in [lo, hi), m >= 1 (Algorithm 1's output).
 * Bit i of the little-endian uint64 words (LSB first) is 1 iff m0 + 2i is
 * squarefree, m0 = first odd >= max(lo, 1).  Bits past the last m are 0.
 * Returns the number of odd m (bits), or -1 on failure.
 */
int64_t oracle_sieve_bits(uint64_t lo, uint64_t hi, int nthreads, uint64_t *bits)
{
    uint64_t m0, n_odd, nw, per;
    int t, nt;
    sieve_chunk_t *ch;
    pthread_t *th;
    if (lo < 1)
        lo = 1;
    m0 = lo | 1;
    if (hi <= m0)
        return 0;
    n_odd = (hi - m0 + 1) / 2;
    if (oracle_prepare(isqrt_u64(hi)) != 0)
        return -1;
    nw = (n_odd + 63) / 64;
    nt = nthreads > 0 ? nthreads : 1;
    if ((uint64_t)nt > nw)
        nt = (int)nw;
    ch = (sieve_chunk_t *)calloc((size_t)nt, sizeof(*ch));
    th = (pthread_t *)calloc((size_t)nt, sizeof(*th));
    if (!ch || !th) {
        free(ch);
        free(th);
        return -1;
    }
    per = (nw + (uint64_t)nt - 1) / (uint64_t)nt;
    for (t = 0; t < nt; t++) {
        ch[t].m0 = m0;
        ch[t].n_odd = n_odd;
        ch[t].bits = bits;
        ch[t].w_begin = per * (uint64_t)t;
        ch[t].w_end = per * (uint64_t)(t + 1) < nw ? per * (uint64_t)(t + 1) : nw;
        if (ch[t].w_begin > nw)
            ch[t].w_begin = nw;
        pthread_create(&th[t], NULL, sieve_chunk_run, &ch[t]);
    }
    for (t = 0; t < nt; t++)
        pthread_join(th[t], NULL);
    free(ch);
    free(th);
    return (int64_t)n_odd;
}

/* ------------------------------------------- many independent n at once */

typedef struct {
    const uint64_t *ns;
    uint8_t *out;
    size_t begin, end;
    unsigned kmax;
} many_chunk_t;

static void *many_run(void *arg)
{
    many_chunk_t *c = (many_chunk_t *)arg;
    size_t i;
    for (i = c->begin; i < c->end; i++)
        c->out[i] = (uint8_t)oracle_mink(c->ns[i], c->kmax);
    return NULL;
}

/* Least k for each of count odd n >= 3 (arbitrary order); 0 = none found. */
int oracle_mink_many(const uint64_t *ns, size_t count, unsigned kmax,
                     int nthreads, uint8_t *out)
{
    uint64_t mx = 3;
    size_t i, per;
    int t, nt;
    many_chunk_t *ch;
    pthread_t *th;
    for (i = 0; i < count; i++)
        if (ns[i] > mx)
            mx = ns[i];
    if (oracle_prepare(isqrt_u64(mx)) != 0)
        return -1;
    nt = nthreads > 0 ? nthreads : 1;
    if ((size_t)nt > count)
        nt = count ? (int)count : 1;
    ch = (many_chunk_t *)calloc((size_t)nt, sizeof(*ch));
    th = (pthread_t *)calloc((size_t)nt, sizeof(*th));
    if (!ch || !th) {
        free(ch);
        free(th);
        return -1;
    }
    per = (count + (size_t)nt - 1) / (size_t)nt;
    for (t = 0; t < nt; t++) {
        ch[t].ns = ns;
        ch[t].out = out;
        ch[t].kmax = kmax;
        ch[t].begin = per * (size_t)t < count ? per * (size_t)t : count;
        ch[t].end = per * (size_t)(t + 1) < count ? per * (size_t)(t + 1) : count;
        pthread_create(&th[t], NULL, many_run, &ch[t]);
    }
    for (t = 0; t < nt; t++)
        pthread_join(th[t], NULL);
    free(ch);
    free(th);
    return 0;
}

/* Squarefree flag for each of count odd m >= 1. */
int oracle_sqf_many(const uint64_t *ms, size_t count, uint8_t *out)
{
    uint64_t mx = 3;
    size_t i;
    for (i = 0; i < count; i++)
        if (ms[i] > mx)
            mx = ms[i];
    if (oracle_prepare(isqrt_u64(mx)) != 0)
        return -1;
    for (i = 0; i < count; i++)
        out[i] = (uint8_t)oracle_is_squarefree(ms[i]);
    return 0;
}
