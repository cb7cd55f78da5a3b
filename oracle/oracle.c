/*
 * CPU oracle for exact multi-pattern matching.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load or run this file.  It shares no
 * code, header, table or helper with the GPU library; both sides only see the
 * same seeded inputs.
 *
 * What is computed (Background, "Multi-Pattern Matching"; Background,
 * "Parallel Failure-Less Aho-Corasick"): for patterns P_0..P_{k-1} (non-empty
 * byte strings) and a text T of n bytes, the match set is
 *
 *     M(T) = { (i, j) : 0 <= i <= n - |P_j|,  T[i .. i+|P_j|) == P_j }
 *
 * reported sorted by (i, j); for a batch of texts, by (text, i, j), with i
 * relative to its own text.  The failure-less walk of the paper (one thread per
 * text byte, walk until mismatch, report every match on the way) reaches
 * exactly this set, so the oracle is the definition itself, not a replay of
 * the walk.
 *
 * Three independent ways to compute M:
 *   ORC_BRUTE     the definition written out: every pattern at every position.
 *   ORC_BUCKETED  the same definition with a sound filter: a pattern can only
 *                 occur at i if its first m = min(min_len, 8) bytes equal
 *                 T[i..i+m); candidates are looked up by those m bytes.
 *   ORC_AC        the textbook Aho-Corasick automaton (goto, failure and output
 *                 functions of Aho & Corasick 1975, cited in Background,
 *                 "Multi-Pattern Matching"), a different algorithm whose
 *                 agreement with ORC_BRUTE pins both.
 * Work is split into ranges of start positions; a range scans up to
 * (longest pattern - 1) bytes past its end, the overlap rule of Background,
 * "Multi-Pattern Matching".
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

enum { ORC_BRUTE = 1, ORC_BUCKETED = 2, ORC_AC = 3 };

/* ------------------------------------------------------------ result lists */

typedef struct {
    uint64_t n, cap;
    uint64_t *pos;
    uint32_t *id;
    uint32_t *tid;
    int oom;
} olist;

static void ol_push(olist *l, uint64_t pos, uint32_t id, uint32_t tid) {
    if (l->oom) return;
    if (l->n == l->cap) {
        uint64_t nc = l->cap ? l->cap * 2 : 64;
        uint64_t *p = realloc(l->pos, nc * sizeof(uint64_t));
        uint32_t *q = realloc(l->id, nc * sizeof(uint32_t));
        uint32_t *r = realloc(l->tid, nc * sizeof(uint32_t));
        if (p) l->pos = p;
        if (q) l->id = q;
        if (r) l->tid = r;
        if (!p || !q || !r) { l->oom = 1; return; }
        l->cap = nc;
    }
    l->pos[l->n] = pos;
    l->id[l->n] = id;
    l->tid[l->n] = tid;
    l->n++;
}

static void ol_free(olist *l) {
    free(l->pos); free(l->id); free(l->tid);
    memset(l, 0, sizeof(*l));
}

/* --------------------------------------------------------------- patterns */

typedef struct {
    const uint8_t *data;
    const uint64_t *off;
    uint32_t k;
    uint64_t min_len, max_len;
} pset;

static inline uint64_t plen(const pset *P, uint32_t j) { return P->off[j + 1] - P->off[j]; }
static inline const uint8_t *pbytes(const pset *P, uint32_t j) { return P->data + P->off[j]; }

/* ----------------------------------------------------- ORC_BUCKETED index */

typedef struct {
    uint32_t m;           /* bytes in the key, 1..8 */
    uint64_t mask;        /* hash table size - 1 */
    uint64_t *key;        /* slot key */
    uint32_t *lo, *hi;    /* slot range in `ids` */
    uint8_t *used;
    uint32_t *ids;        /* pattern ids sorted by (key, id) */
} bindex;

static uint64_t load_key(const uint8_t *p, uint32_t m) {
    uint64_t x = 0;
    memcpy(&x, p, m);
    return x;
}

/* Hash-table index mixing: the 64-bit finalizer (fmix64) of Austin Appleby's
 * published MurmurHash3. */
static inline uint64_t hmix(uint64_t x) {
    x ^= x >> 33; x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return x;
}

/* qsort has no context argument: the key parameters are per thread, since
 * the exhaustive check builds indexes on several threads at once */
static _Thread_local const pset *g_sort_P;
static _Thread_local uint32_t g_sort_m;
static int cmp_key_id(const void *a, const void *b) {
    uint32_t ja = *(const uint32_t *)a, jb = *(const uint32_t *)b;
    uint64_t ka = load_key(pbytes(g_sort_P, ja), g_sort_m);
    uint64_t kb = load_key(pbytes(g_sort_P, jb), g_sort_m);
    if (ka != kb) return ka < kb ? -1 : 1;
    return ja < jb ? -1 : (ja > jb);
}

static int bindex_build(bindex *B, const pset *P) {
    memset(B, 0, sizeof(*B));
    B->m = (uint32_t)(P->min_len < 8 ? P->min_len : 8);
    if (P->k == 0) return 0;
    B->ids = malloc(sizeof(uint32_t) * P->k);
    if (!B->ids) return -1;
    for (uint32_t j = 0; j < P->k; j++) B->ids[j] = j;
    g_sort_P = P; g_sort_m = B->m;
    qsort(B->ids, P->k, sizeof(uint32_t), cmp_key_id);
    uint64_t cap = 16;
    while (cap < 2ull * P->k) cap <<= 1;
    B->mask = cap - 1;
    B->key = calloc(cap, sizeof(uint64_t));
    B->lo = calloc(cap, sizeof(uint32_t));
    B->hi = calloc(cap, sizeof(uint32_t));
    B->used = calloc(cap, 1);
    if (!B->key || !B->lo || !B->hi || !B->used) return -1;
    uint32_t a = 0;
    while (a < P->k) {
        uint64_t key = load_key(pbytes(P, B->ids[a]), B->m);
        uint32_t b = a + 1;
        while (b < P->k && load_key(pbytes(P, B->ids[b]), B->m) == key) b++;
        uint64_t h = hmix(key) & B->mask;
        while (B->used[h]) h = (h + 1) & B->mask;
        B->used[h] = 1; B->key[h] = key; B->lo[h] = a; B->hi[h] = b;
        a = b;
    }
    return 0;
}

static void bindex_free(bindex *B) {
    free(B->key); free(B->lo); free(B->hi); free(B->used); free(B->ids);
    memset(B, 0, sizeof(*B));
}

/* ------------------------------------------------- ORC_AC automaton (1975) */

typedef struct {
    uint32_t n_nodes;
    /* goto function: hash of (state, byte) -> state */
    uint64_t gmask;
    uint64_t *gkey;       /* (state << 8 | byte) + 1, 0 = empty */
    uint32_t *gval;
    /* tree structure for the breadth-first failure computation */
    uint32_t *first_child, *next_sibling;
    uint8_t *in_label;
    uint32_t *fail;       /* failure function f(s) */
    uint32_t *dict;       /* nearest state on the failure chain with output, or 0 */
    uint32_t *out_head;   /* output(s): linked list of pattern ids ending at s */
    uint32_t *out_next;
} acm;

#define AC_NONE 0xffffffffu

static uint32_t ac_goto(const acm *A, uint32_t s, uint8_t c) {
    uint64_t key = (((uint64_t)s << 8) | c) + 1;
    uint64_t h = hmix(key) & A->gmask;
    while (A->gkey[h]) {
        if (A->gkey[h] == key) return A->gval[h];
        h = (h + 1) & A->gmask;
    }
    return AC_NONE;
}

static void ac_set(acm *A, uint32_t s, uint8_t c, uint32_t t) {
    uint64_t key = (((uint64_t)s << 8) | c) + 1;
    uint64_t h = hmix(key) & A->gmask;
    while (A->gkey[h]) h = (h + 1) & A->gmask;
    A->gkey[h] = key; A->gval[h] = t;
}

static int ac_build(acm *A, const pset *P) {
    memset(A, 0, sizeof(*A));
    uint64_t total = P->off[P->k];
    uint64_t maxn = total + 1;
    uint64_t cap = 16;
    while (cap < 2 * maxn) cap <<= 1;
    A->gmask = cap - 1;
    A->gkey = calloc(cap, sizeof(uint64_t));
    A->gval = malloc(cap * sizeof(uint32_t));
    A->first_child = malloc(maxn * sizeof(uint32_t));
    A->next_sibling = malloc(maxn * sizeof(uint32_t));
    A->in_label = malloc(maxn);
    A->fail = malloc(maxn * sizeof(uint32_t));
    A->dict = malloc(maxn * sizeof(uint32_t));
    A->out_head = malloc(maxn * sizeof(uint32_t));
    A->out_next = malloc((P->k + 1) * sizeof(uint32_t));
    if (!A->gkey || !A->gval || !A->first_child || !A->next_sibling || !A->in_label ||
        !A->fail || !A->dict || !A->out_head || !A->out_next)
        return -1;
    A->n_nodes = 1;
    A->first_child[0] = AC_NONE; A->next_sibling[0] = AC_NONE;
    A->out_head[0] = AC_NONE; A->in_label[0] = 0;
    /* goto construction: enter each keyword into the tree */
    for (uint32_t j = 0; j < P->k; j++) {
        uint32_t s = 0;
        const uint8_t *w = pbytes(P, j);
        for (uint64_t d = 0; d < plen(P, j); d++) {
            uint32_t t = ac_goto(A, s, w[d]);
            if (t == AC_NONE) {
                t = A->n_nodes++;
                ac_set(A, s, w[d], t);
                A->first_child[t] = AC_NONE;
                A->out_head[t] = AC_NONE;
                A->in_label[t] = w[d];
                A->next_sibling[t] = A->first_child[s];
                A->first_child[s] = t;
            }
            s = t;
        }
        A->out_next[j] = A->out_head[s];
        A->out_head[s] = j;
    }
    /* failure construction, breadth first */
    uint32_t *queue = malloc(A->n_nodes * sizeof(uint32_t));
    if (!queue) return -1;
    uint32_t qh = 0, qt = 0;
    A->fail[0] = 0; A->dict[0] = 0;
    for (uint32_t s = A->first_child[0]; s != AC_NONE; s = A->next_sibling[s]) {
        A->fail[s] = 0; A->dict[s] = 0;
        queue[qt++] = s;
    }
    while (qh < qt) {
        uint32_t r = queue[qh++];
        for (uint32_t s = A->first_child[r]; s != AC_NONE; s = A->next_sibling[s]) {
            uint8_t a = A->in_label[s];
            uint32_t st = A->fail[r];
            uint32_t g;
            while ((g = ac_goto(A, st, a)) == AC_NONE && st != 0) st = A->fail[st];
            if (g == AC_NONE) g = 0;
            A->fail[s] = g;
            /* output(s) is merged with output(f(s)): keep a link to the next
             * state on the failure chain that has its own outputs */
            A->dict[s] = (A->out_head[g] != AC_NONE) ? g : A->dict[g];
            queue[qt++] = s;
        }
    }
    free(queue);
    return 0;
}

static void ac_free(acm *A) {
    free(A->gkey); free(A->gval); free(A->first_child); free(A->next_sibling);
    free(A->in_label); free(A->fail); free(A->dict); free(A->out_head); free(A->out_next);
    memset(A, 0, sizeof(*A));
}

/* ------------------------------------------------------- per-range matchers */

typedef struct {
    int algo;
    const pset *P;
    const bindex *B;
    const acm *A;
} matcher;

/* Start positions [lo, hi) of text t (length n, id tid) into list L. */
static void match_range(const matcher *M, const uint8_t *t, uint64_t n, uint32_t tid,
                        uint64_t lo, uint64_t hi, olist *L) {
    const pset *P = M->P;
    if (hi > n) hi = n;
    if (lo >= hi || P->k == 0) return;
    if (M->algo == ORC_BRUTE) {
        for (uint64_t i = lo; i < hi; i++)
            for (uint32_t j = 0; j < P->k; j++) {
                uint64_t L_j = plen(P, j);
                if (L_j <= n - i && memcmp(t + i, pbytes(P, j), L_j) == 0) ol_push(L, i, j, tid);
            }
    } else if (M->algo == ORC_BUCKETED) {
        const bindex *B = M->B;
        for (uint64_t i = lo; i < hi; i++) {
            if (B->m > n - i) break; /* every pattern is at least m long */
            uint64_t key = load_key(t + i, B->m);
            uint64_t h = hmix(key) & B->mask;
            while (B->used[h] && B->key[h] != key) h = (h + 1) & B->mask;
            if (!B->used[h]) continue;
            for (uint32_t r = B->lo[h]; r < B->hi[h]; r++) {
                uint32_t j = B->ids[r];
                uint64_t L_j = plen(P, j);
                if (L_j <= n - i && memcmp(t + i, pbytes(P, j), L_j) == 0) ol_push(L, i, j, tid);
            }
        }
    } else {
        const acm *A = M->A;
        uint64_t end = hi + (P->max_len - 1);
        if (end > n) end = n;
        uint64_t first = L->n;
        uint32_t s = 0;
        for (uint64_t i = lo; i < end; i++) {
            uint32_t g;
            while ((g = ac_goto(A, s, t[i])) == AC_NONE && s != 0) s = A->fail[s];
            s = (g == AC_NONE) ? 0 : g;
            for (uint32_t u = (A->out_head[s] != AC_NONE) ? s : A->dict[s]; u != 0; u = A->dict[u])
                for (uint32_t j = A->out_head[u]; j != AC_NONE; j = A->out_next[j]) {
                    uint64_t start = i + 1 - plen(P, j);
                    if (start >= lo && start < hi) ol_push(L, start, j, tid);
                }
        }
        /* AC reports by end position; restore (start, id) order by insertion
         * sort on this range's slice (small per range) */
        for (uint64_t a = first + 1; a < L->n; a++) {
            uint64_t p = L->pos[a]; uint32_t id = L->id[a], tt = L->tid[a];
            uint64_t b = a;
            while (b > first && (L->pos[b - 1] > p || (L->pos[b - 1] == p && L->id[b - 1] > id))) {
                L->pos[b] = L->pos[b - 1]; L->id[b] = L->id[b - 1]; L->tid[b] = L->tid[b - 1];
                b--;
            }
            L->pos[b] = p; L->id[b] = id; L->tid[b] = tt;
        }
    }
}

/* ------------------------------------------------------------ work engine */

typedef struct { uint32_t tid; uint64_t lo, hi; } item;

typedef struct {
    const matcher *M;
    const uint8_t *text;
    const uint64_t *toff;
    item *items;
    olist *lists;
    uint64_t n_items;
    uint64_t next;  /* atomic item cursor */
} job;

static void *worker(void *arg) {
    job *J = arg;
    for (;;) {
        uint64_t r = __atomic_fetch_add(&J->next, 1, __ATOMIC_RELAXED);
        if (r >= J->n_items) break;
        item *it = &J->items[r];
        const uint8_t *t = J->text + J->toff[it->tid];
        uint64_t n = J->toff[it->tid + 1] - J->toff[it->tid];
        match_range(J->M, t, n, it->tid, it->lo, it->hi, &J->lists[r]);
    }
    return NULL;
}

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

typedef struct { olist all; } orc_result;

/*
 * Match every text of a batch (text i = text[toff[i] .. toff[i+1])), start
 * positions restricted to [lo, hi) within each text.  Patterns must be
 * non-empty.  timing[0] = index build seconds, timing[1] = matching seconds.
 * Returns an opaque result or NULL on bad input / out of memory.
 */
void *orc_match(int algo, const uint8_t *text, const uint64_t *toff, uint32_t n_texts,
                const uint8_t *pdata, const uint64_t *poff, uint32_t k,
                uint64_t lo, uint64_t hi, int threads, uint64_t chunk, double *timing) {
    pset P = {pdata, poff, k, UINT64_MAX, 0};
    for (uint32_t j = 0; j < k; j++) {
        uint64_t L = plen(&P, j);
        if (L == 0) return NULL;
        if (L < P.min_len) P.min_len = L;
        if (L > P.max_len) P.max_len = L;
    }
    if (k == 0) P.min_len = 1;
    if (threads < 1) threads = 1;
    if (chunk == 0) chunk = 1 << 20;

    double t0 = now_s();
    bindex B; acm A;
    int have_b = 0, have_a = 0;
    if (algo == ORC_BUCKETED) { if (bindex_build(&B, &P)) { bindex_free(&B); return NULL; } have_b = 1; }
    if (algo == ORC_AC) { if (ac_build(&A, &P)) { ac_free(&A); return NULL; } have_a = 1; }
    double t1 = now_s();
    matcher M = {algo, &P, have_b ? &B : NULL, have_a ? &A : NULL};

    /* split every text's start range into chunks, in output order */
    uint64_t n_items = 0;
    for (uint32_t i = 0; i < n_texts; i++) {
        uint64_t n = toff[i + 1] - toff[i];
        uint64_t a = lo, b = hi < n ? hi : n;
        if (a < b) n_items += (b - a + chunk - 1) / chunk;
    }
    item *items = malloc((n_items ? n_items : 1) * sizeof(item));
    olist *lists = calloc(n_items ? n_items : 1, sizeof(olist));
    orc_result *res = calloc(1, sizeof(orc_result));
    if (!items || !lists || !res) {
        free(items); free(lists); free(res);
        if (have_b) bindex_free(&B);
        if (have_a) ac_free(&A);
        return NULL;
    }
    uint64_t r = 0;
    for (uint32_t i = 0; i < n_texts; i++) {
        uint64_t n = toff[i + 1] - toff[i];
        uint64_t b = hi < n ? hi : n;
        for (uint64_t a = lo; a < b; a += chunk) {
            items[r].tid = i; items[r].lo = a; items[r].hi = (a + chunk < b) ? a + chunk : b;
            r++;
        }
    }
    job J = {&M, text, toff, items, lists, n_items, 0};
    pthread_t *th = malloc(sizeof(pthread_t) * threads);
    int started = 0;
    if (th && threads > 1) {
        for (int q = 0; q < threads - 1; q++)
            if (pthread_create(&th[q], NULL, worker, &J) == 0) started++;
    }
    worker(&J);
    for (int q = 0; q < started; q++) pthread_join(th[q], NULL);
    free(th);
    double t2 = now_s();

    uint64_t total = 0;
    int oom = 0;
    for (uint64_t q = 0; q < n_items; q++) { total += lists[q].n; oom |= lists[q].oom; }
    res->all.n = total;
    res->all.cap = total;
    res->all.pos = malloc((total ? total : 1) * sizeof(uint64_t));
    res->all.id = malloc((total ? total : 1) * sizeof(uint32_t));
    res->all.tid = malloc((total ? total : 1) * sizeof(uint32_t));
    if (oom || !res->all.pos || !res->all.id || !res->all.tid) {
        for (uint64_t q = 0; q < n_items; q++) ol_free(&lists[q]);
        ol_free(&res->all);
        free(res); res = NULL;
    } else {
        uint64_t w = 0;
        for (uint64_t q = 0; q < n_items; q++) {
            if (lists[q].n) {  /* an empty list may hold no buffers at all */
                memcpy(res->all.pos + w, lists[q].pos, lists[q].n * sizeof(uint64_t));
                memcpy(res->all.id + w, lists[q].id, lists[q].n * sizeof(uint32_t));
                memcpy(res->all.tid + w, lists[q].tid, lists[q].n * sizeof(uint32_t));
            }
            w += lists[q].n;
            ol_free(&lists[q]);
        }
    }
    free(items); free(lists);
    if (have_b) bindex_free(&B);
    if (have_a) ac_free(&A);
    if (timing) { timing[0] = t1 - t0; timing[1] = t2 - t1; }
    return res;
}

uint64_t orc_count(const void *h) { return h ? ((const orc_result *)h)->all.n : 0; }

void orc_copy(const void *h, uint64_t *pos, uint32_t *id, uint32_t *tid) {
    const orc_result *R = h;
    if (!R) return;
    if (pos) memcpy(pos, R->all.pos, R->all.n * sizeof(uint64_t));
    if (id) memcpy(id, R->all.id, R->all.n * sizeof(uint32_t));
    if (tid) memcpy(tid, R->all.tid, R->all.n * sizeof(uint32_t));
}

void orc_free(void *h) {
    orc_result *R = h;
    if (!R) return;
    ol_free(&R->all);
    free(R);
}

/* ------------------------------------------------------- exhaustive check */

/*
 * All multisets of 1..max_npat patterns drawn from the strings of length
 * 1..max_plen over the alphabet {0..sigma-1}, against all texts of length
 * 0..max_tlen: compares ORC_BRUTE, ORC_BUCKETED and ORC_AC on every case.
 * Returns the number of disagreeing cases; *n_cases gets the number checked.
 */
typedef struct {
    int sigma, max_plen, max_npat, max_tlen;
    uint8_t (*strs)[8];
    int *slen;
    int n_strs;
    uint64_t *sets;      /* encoded multisets: up to 3 indices, 16 bits each, +1 */
    uint64_t n_sets;
    uint64_t next;
    uint64_t bad, cases;
} ex_job;

static int same(const olist *a, const olist *b) {
    if (a->n != b->n) return 0;
    for (uint64_t i = 0; i < a->n; i++)
        if (a->pos[i] != b->pos[i] || a->id[i] != b->id[i]) return 0;
    return 1;
}

static void *ex_worker(void *arg) {
    ex_job *E = arg;
    uint8_t pdata[64];
    uint64_t poff[8];
    uint8_t text[32];
    uint64_t bad = 0, cases = 0;
    for (;;) {
        uint64_t r = __atomic_fetch_add(&E->next, 1, __ATOMIC_RELAXED);
        if (r >= E->n_sets) break;
        uint64_t code = E->sets[r];
        uint32_t k = 0;
        poff[0] = 0;
        for (int q = 0; q < E->max_npat; q++) {
            uint32_t s = (uint32_t)((code >> (16 * q)) & 0xffff);
            if (!s) break;
            s -= 1;
            memcpy(pdata + poff[k], E->strs[s], E->slen[s]);
            poff[k + 1] = poff[k] + E->slen[s];
            k++;
        }
        pset P = {pdata, poff, k, UINT64_MAX, 0};
        for (uint32_t j = 0; j < k; j++) {
            if (plen(&P, j) < P.min_len) P.min_len = plen(&P, j);
            if (plen(&P, j) > P.max_len) P.max_len = plen(&P, j);
        }
        bindex B; acm A;
        if (bindex_build(&B, &P) || ac_build(&A, &P)) { bad++; bindex_free(&B); ac_free(&A); continue; }
        matcher m1 = {ORC_BRUTE, &P, NULL, NULL};
        matcher m2 = {ORC_BUCKETED, &P, &B, NULL};
        matcher m3 = {ORC_AC, &P, NULL, &A};
        for (int tl = 0; tl <= E->max_tlen; tl++) {
            uint64_t count = 1;
            for (int q = 0; q < tl; q++) count *= E->sigma;
            for (uint64_t c = 0; c < count; c++) {
                uint64_t x = c;
                for (int q = 0; q < tl; q++) { text[q] = (uint8_t)(x % E->sigma); x /= E->sigma; }
                olist l1 = {0}, l2 = {0}, l3 = {0};
                match_range(&m1, text, tl, 0, 0, tl, &l1);
                match_range(&m2, text, tl, 0, 0, tl, &l2);
                match_range(&m3, text, tl, 0, 0, tl, &l3);
                if (!same(&l1, &l2) || !same(&l1, &l3)) bad++;
                cases++;
                ol_free(&l1); ol_free(&l2); ol_free(&l3);
            }
        }
        bindex_free(&B);
        ac_free(&A);
    }
    __atomic_fetch_add(&E->bad, bad, __ATOMIC_RELAXED);
    __atomic_fetch_add(&E->cases, cases, __ATOMIC_RELAXED);
    return NULL;
}

int64_t orc_exhaustive(int sigma, int max_plen, int max_npat, int max_tlen, int threads,
                       uint64_t *n_cases) {
    if (sigma < 1 || sigma > 255 || max_plen < 1 || max_plen > 8 || max_npat < 1 ||
        max_npat > 3 || max_tlen < 0 || max_tlen > 24)
        return -1;
    ex_job E;
    memset(&E, 0, sizeof(E));
    E.sigma = sigma; E.max_plen = max_plen; E.max_npat = max_npat; E.max_tlen = max_tlen;
    uint64_t ns = 0, pw = 1;
    for (int L = 1; L <= max_plen; L++) { pw *= sigma; ns += pw; }
    if (ns > 60000) return -1;
    E.n_strs = (int)ns;
    E.strs = malloc(ns * sizeof(*E.strs));
    E.slen = malloc(ns * sizeof(int));
    int w = 0;
    pw = 1;
    for (int L = 1; L <= max_plen; L++) {
        pw *= sigma;
        for (uint64_t c = 0; c < pw; c++) {
            uint64_t x = c;
            for (int q = L - 1; q >= 0; q--) { E.strs[w][q] = (uint8_t)(x % sigma); x /= sigma; }
            E.slen[w] = L;
            w++;
        }
    }
    /* multisets of 1, 2 or 3 strings as non-decreasing index tuples */
    uint64_t cap = 1024;
    E.sets = malloc(cap * sizeof(uint64_t));
    int S = E.n_strs;
#define PUSH_SET(code_)                                                              \
    do {                                                                             \
        if (E.n_sets == cap) { cap *= 2; E.sets = realloc(E.sets, cap * sizeof(uint64_t)); } \
        E.sets[E.n_sets++] = (code_);                                                \
    } while (0)
    for (int a = 0; a < S; a++) {
        PUSH_SET((uint64_t)(a + 1));
        if (max_npat < 2) continue;
        for (int b = a; b < S; b++) {
            PUSH_SET((uint64_t)(a + 1) | ((uint64_t)(b + 1) << 16));
            if (max_npat < 3) continue;
            for (int c = b; c < S; c++)
                PUSH_SET((uint64_t)(a + 1) | ((uint64_t)(b + 1) << 16) | ((uint64_t)(c + 1) << 32));
        }
    }
#undef PUSH_SET
    if (threads < 1) threads = 1;
    pthread_t *th = malloc(sizeof(pthread_t) * threads);
    int started = 0;
    for (int q = 1; q < threads; q++)
        if (pthread_create(&th[q], NULL, ex_worker, &E) == 0) started++;
    ex_worker(&E);
    for (int q = 1; q <= started; q++) pthread_join(th[q], NULL);
    free(th); free(E.strs); free(E.slen); free(E.sets);
    if (n_cases) *n_cases = E.cases;
    return (int64_t)E.bad;
}
