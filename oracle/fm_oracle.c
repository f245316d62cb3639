/*
 * fm_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE LIBRARY.
 *
 * A plain, slow, obviously correct CPU model of what the FM-index hot path computes,
 * written from "Vectorized Character Counting for Faster Pattern Matching" (Snytsar).
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it. It shares no code, header, table or helper with the GPU library, and the GPU
 * library never loads it.
 *
 * Two layers:
 *   Definitions -- results that have a plain definition, written out directly:
 *     suffix array by sorting suffixes with direct comparison (Background, Eq. 1),
 *     BWT from the suffix array (Eq. 2), Occ by a linear scan and C as the exclusive
 *     prefix sum of the last Occ row (Background, Fig. 1), the SA interval of a
 *     pattern by binary search over the sorted suffixes, and the z-substitution hit set
 *     by enumerating the Hamming ball around a read.
 *   Algorithms -- the paper's procedures in the paper's order:
 *     backward exact match (Listing 1), inexact match restricted to substitutions
 *     (Listing 2), and the D-array lower bound of BWA, which Listing 2 is taken from.
 *
 * Readings of the paper that this file adopts (each is listed in the design notes):
 *   - rows are 0..n (n+1 rows including the '$' row); Occ(c,-1) = 0;
 *   - C has 5 entries and does not count '$'; C[4] = n;
 *   - searches start from the empty-pattern interval (0, n) (the first character c then
 *     gives {C[c]+1, C[c+1]}, the +1 convention of Listing 1, rather than Eq. 3 taken
 *     literally);
 *   - an empty final interval is reported as the canonical miss (k, l) = (1, 0);
 *   - Listing 2: the per-character loop computes its (k, l) into fresh locals from the
 *     parent's interval, every branch is guarded by k <= l, and only the substitution
 *     branches are taken (gap branches are out of scope);
 *   - read symbols outside ACGT (code 4) occur nowhere in R and never equal a base;
 *   - the reverse-complement strand of a read W is W reversed with c -> 3 - c.
 *
 * Symbol codes: A=0, C=1, G=2, T=3; '$' is kept out of band (BWT code 4).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define DOLLAR 4

typedef struct {
    int64_t n;             /* |R| */
    uint8_t *R;            /* copy of the text, n codes */
    uint32_t *SA;          /* n+1 entries */
    uint8_t *BWT;          /* n+1 entries, 0..3 or DOLLAR */
    uint32_t *occ;         /* (n+1)*4 entries: occ[4*k + c] = Occ(c, k) */
    int64_t dollar_row;
    uint64_t C[5];
} oracle_index;

typedef struct {           /* one hit of one read */
    uint32_t read, k, l;
    uint8_t strand, d;
    uint16_t pad;
} oracle_hit;

/* ------------------------------------------------------------------ Eq. (1): SA */

static const uint8_t *cmp_R;
static int64_t cmp_n;

/* Order of the suffixes R[a..n-1]$ and R[b..n-1]$: byte order on the characters, and a
 * suffix that reaches '$' first is smaller, because '$' sorts below every character. */
static int cmp_suffix(const void *pa, const void *pb)
{
    int64_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    int64_t la = cmp_n - a, lb = cmp_n - b;
    int64_t m = la < lb ? la : lb;
    int r = memcmp(cmp_R + a, cmp_R + b, (size_t)m);
    if (r != 0) return r;
    return (la < lb) ? -1 : (la > lb);
}

void oracle_suffix_array(const uint8_t *R, int64_t n, uint32_t *SA)
{
    for (int64_t i = 0; i <= n; i++) SA[i] = (uint32_t)i;
    cmp_R = R;
    cmp_n = n;
    qsort(SA, (size_t)(n + 1), sizeof(uint32_t), cmp_suffix);
}

/* ------------------------------------------------------------------ Eq. (2): BWT */

int64_t oracle_bwt(const uint8_t *R, int64_t n, const uint32_t *SA, uint8_t *BWT)
{
    int64_t dollar_row = -1;
    for (int64_t i = 0; i <= n; i++) {
        if (SA[i] > 0) {
            BWT[i] = R[SA[i] - 1];
        } else {
            BWT[i] = DOLLAR;
            dollar_row = i;
        }
    }
    return dollar_row;
}

/* ------------------------------------------------------------------ Occ and C */

/* Occ(c, k) = number of c in BWT[0..k], by one linear scan over the BWT. */
void oracle_occ_table(const uint8_t *BWT, int64_t n, uint32_t *occ)
{
    uint32_t run[4] = {0, 0, 0, 0};
    for (int64_t k = 0; k <= n; k++) {
        if (BWT[k] < 4) run[BWT[k]]++;
        memcpy(occ + 4 * k, run, sizeof run);
    }
}

static uint32_t occ_at(const oracle_index *x, int c, int64_t k)
{
    if (k < 0) return 0;                 /* Occ(c, -1) = 0 */
    return x->occ[4 * k + c];
}

/* C[c] = occurrences of all characters smaller than c: the exclusive prefix sum of the
 * last Occ row. */
static void c_array(const oracle_index *x, uint64_t C[5])
{
    uint64_t acc = 0;
    for (int c = 0; c < 4; c++) {
        C[c] = acc;
        acc += occ_at(x, c, x->n);
    }
    C[4] = acc;
}

oracle_index *oracle_index_new(const uint8_t *R, int64_t n)
{
    oracle_index *x = calloc(1, sizeof *x);
    if (!x) return NULL;
    x->n = n;
    x->R = malloc((size_t)(n > 0 ? n : 1));
    x->SA = malloc(sizeof(uint32_t) * (size_t)(n + 1));
    x->BWT = malloc((size_t)(n + 1));
    x->occ = malloc(sizeof(uint32_t) * 4 * (size_t)(n + 1));
    if (!x->R || !x->SA || !x->BWT || !x->occ) {
        free(x->R); free(x->SA); free(x->BWT); free(x->occ); free(x);
        return NULL;
    }
    if (n > 0) memcpy(x->R, R, (size_t)n);
    oracle_suffix_array(x->R, n, x->SA);
    x->dollar_row = oracle_bwt(x->R, n, x->SA, x->BWT);
    oracle_occ_table(x->BWT, n, x->occ);
    c_array(x, x->C);
    return x;
}

void oracle_index_free(oracle_index *x)
{
    if (!x) return;
    free(x->R); free(x->SA); free(x->BWT); free(x->occ); free(x);
}

int64_t oracle_index_n(const oracle_index *x) { return x->n; }
int64_t oracle_index_dollar_row(const oracle_index *x) { return x->dollar_row; }
const uint32_t *oracle_index_sa(const oracle_index *x) { return x->SA; }
const uint8_t *oracle_index_bwt(const oracle_index *x) { return x->BWT; }
const uint32_t *oracle_index_occ(const oracle_index *x) { return x->occ; }
void oracle_index_c(const oracle_index *x, uint64_t C[5]) { memcpy(C, x->C, sizeof x->C); }

/* Occ8 for a query (k, l): Occ(c, k-1) for c = A,C,G,T, then Occ(c, l). Queries outside
 * 0 <= k <= n+1, 0 <= l <= n are answered with all-ones words. */
void oracle_occ8(const oracle_index *x, const uint32_t *q, int64_t nq, uint32_t *out)
{
    for (int64_t j = 0; j < nq; j++) {
        int64_t k = q[2 * j], l = q[2 * j + 1];
        uint32_t *o = out + 8 * j;
        if (k > x->n + 1 || l > x->n) {
            for (int c = 0; c < 8; c++) o[c] = 0xFFFFFFFFu;
            continue;
        }
        for (int c = 0; c < 4; c++) {
            o[c] = occ_at(x, c, k - 1);
            o[4 + c] = occ_at(x, c, l);
        }
    }
}

/* ------------------------------------------------------------------ strands */

/* Pattern of strand s for read W: strand 0 is W, strand 1 its reverse complement. */
static void strand_pattern(const uint8_t *W, int64_t m, int s, uint8_t *P)
{
    for (int64_t i = 0; i < m; i++) {
        if (s == 0) {
            P[i] = W[i];
        } else {
            uint8_t c = W[m - 1 - i];
            P[i] = c < 4 ? (uint8_t)(3 - c) : c;
        }
    }
}

/* ------------------------------------------------------------------ definition of the interval */

/* Compare the suffix R[s..n-1]$ with the pattern P[0..m): negative if the suffix is
 * smaller, zero if P is a prefix of the suffix, positive if the suffix is larger. */
static int cmp_suffix_pattern(const oracle_index *x, int64_t s, const uint8_t *P, int64_t m)
{
    for (int64_t j = 0; j < m; j++) {
        if (s + j >= x->n) return -1;            /* the suffix reaches '$' first */
        if (x->R[s + j] != P[j]) return x->R[s + j] < P[j] ? -1 : 1;
    }
    return 0;
}

/* Rows whose suffix starts with P are [k, l], with k = number of suffixes smaller than P
 * and l = k - 1 + (occurrences of P). Both bounds by binary search over the SA. */
static void interval_by_definition(const oracle_index *x, const uint8_t *P, int64_t m,
                                   int64_t *k_out, int64_t *l_out)
{
    int64_t lo = 0, hi = x->n + 1;               /* first row not smaller than P */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (cmp_suffix_pattern(x, x->SA[mid], P, m) < 0) lo = mid + 1; else hi = mid;
    }
    int64_t first = lo;
    hi = x->n + 1;                               /* first row larger than P */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (cmp_suffix_pattern(x, x->SA[mid], P, m) <= 0) lo = mid + 1; else hi = mid;
    }
    *k_out = first;
    *l_out = lo - 1;
}

/* ------------------------------------------------------------------ Listing 1 */

/* Backward exact match: from the empty-pattern interval (0, n), for i = m-1 down to 0
 * with b = P[i]: k <- C(b) + Occ(b, k-1) + 1 and l <- C(b) + Occ(b, l). A non-ACGT
 * symbol occurs nowhere, so its step yields an empty interval (which stays empty). */
static void exact_listing1(const oracle_index *x, const uint8_t *P, int64_t m,
                           int64_t *k_out, int64_t *l_out)
{
    int64_t k = 0, l = x->n;
    for (int64_t i = m - 1; i >= 0; i--) {
        int b = P[i];
        if (b > 3) {
            k = 1;
            l = 0;
            continue;
        }
        k = (int64_t)x->C[b] + occ_at(x, b, k - 1) + 1;
        l = (int64_t)x->C[b] + occ_at(x, b, l);
    }
    *k_out = k;
    *l_out = l;
}

/* Exact search of every read on the requested strands (bit 0: strand 0, bit 1:
 * strand 1). out holds (k, l) pairs, one per read and strand, strand-major within a
 * read. method 0: the definition (binary search); 1: Listing 1. An empty interval is
 * written as the canonical miss (1, 0). */
void oracle_exact(const oracle_index *x, const uint8_t *codes, const uint64_t *offs,
                  int64_t nreads, int strands, int method, uint32_t *out)
{
    int64_t maxm = 0;
    for (int64_t r = 0; r < nreads; r++)
        if ((int64_t)(offs[r + 1] - offs[r]) > maxm) maxm = (int64_t)(offs[r + 1] - offs[r]);
    uint8_t *P = malloc((size_t)(maxm + 1));
    int64_t j = 0;
    for (int64_t r = 0; r < nreads; r++) {
        const uint8_t *W = codes + offs[r];
        int64_t m = (int64_t)(offs[r + 1] - offs[r]);
        for (int s = 0; s < 2; s++) {
            if (!(strands & (1 << s))) continue;
            int64_t k, l;
            strand_pattern(W, m, s, P);
            if (method == 0) interval_by_definition(x, P, m, &k, &l);
            else exact_listing1(x, P, m, &k, &l);
            if (k > l) { k = 1; l = 0; }
            out[2 * j] = (uint32_t)k;
            out[2 * j + 1] = (uint32_t)l;
            j++;
        }
    }
    free(P);
}

/* ------------------------------------------------------------------ D-array (BWA) */

/* Lower bound D[i] on the substitutions needed to place W[0..i] in R. Walks W from left
 * to right with backward search over the index of reverse(R) (prepending W[i] there
 * extends W[0..i-1] to the right in R). When the interval becomes empty, or W[i] is not
 * a base, a difference is certain inside the current segment: count it and restart
 * from the empty-pattern interval. Values saturate at 255. */
void oracle_darray_one(const oracle_index *rev, const uint8_t *W, int64_t m, uint8_t *D)
{
    int64_t k = 0, l = rev->n;
    int z = 0;
    for (int64_t i = 0; i < m; i++) {
        int b = W[i];
        if (b < 4) {
            k = (int64_t)rev->C[b] + occ_at(rev, b, k - 1) + 1;
            l = (int64_t)rev->C[b] + occ_at(rev, b, l);
        }
        if (b > 3 || k > l) {
            z++;
            k = 0;
            l = rev->n;
        }
        D[i] = (uint8_t)(z < 255 ? z : 255);
    }
}

/* D for every read and requested strand; outputs are laid out like the reads (one
 * byte per read position), strand 0 block first, then the strand 1 block. */
void oracle_darray(const oracle_index *rev, const uint8_t *codes, const uint64_t *offs,
                   int64_t nreads, int strands, uint8_t *out)
{
    int64_t total = (int64_t)offs[nreads], maxm = 0;
    for (int64_t r = 0; r < nreads; r++)
        if ((int64_t)(offs[r + 1] - offs[r]) > maxm) maxm = (int64_t)(offs[r + 1] - offs[r]);
    uint8_t *P = malloc((size_t)(maxm + 1));
    int blk = 0;
    for (int s = 0; s < 2; s++) {
        if (!(strands & (1 << s))) continue;
        for (int64_t r = 0; r < nreads; r++) {
            int64_t m = (int64_t)(offs[r + 1] - offs[r]);
            strand_pattern(codes + offs[r], m, s, P);
            oracle_darray_one(rev, P, m, out + (int64_t)blk * total + (int64_t)offs[r]);
        }
        blk++;
    }
    free(P);
}

/* ------------------------------------------------------------------ hit collection */

typedef struct {
    oracle_hit *buf;
    int64_t len, cap;
} hit_list;

static void push_hit(hit_list *h, uint32_t read, uint8_t strand, int64_t k, int64_t l, int d)
{
    if (h->len == h->cap) {
        h->cap = h->cap ? 2 * h->cap : 64;
        h->buf = realloc(h->buf, sizeof(oracle_hit) * (size_t)h->cap);
    }
    oracle_hit *e = &h->buf[h->len++];
    e->read = read;
    e->k = (uint32_t)k;
    e->l = (uint32_t)l;
    e->strand = strand;
    e->d = (uint8_t)d;
    e->pad = 0;
}

static int cmp_hit(const void *pa, const void *pb)
{
    const oracle_hit *a = pa, *b = pb;
    if (a->read != b->read) return a->read < b->read ? -1 : 1;
    if (a->strand != b->strand) return a->strand < b->strand ? -1 : 1;
    if (a->k != b->k) return a->k < b->k ? -1 : 1;
    return 0;
}

/* ------------------------------------------------------------------ Listing 2 */

typedef struct {
    const oracle_index *x;
    const uint8_t *W;
    const uint8_t *D;      /* NULL: no lower bound (the listing's plain z < 0 test) */
    int z0;
    uint32_t read;
    uint8_t strand;
    hit_list *hits;
    uint64_t nodes;        /* calls that reached the per-character loop */
} inex_ctx;

/* InexRecur(W, i, z, k, l), substitution branches only. The bound test is the
 * listing's "z < 0", strengthened to "z < D(i)" when the D-array is used (D(-1) = 0). */
static void inex_recur(inex_ctx *c, int64_t i, int z, int64_t k, int64_t l)
{
    int bound = (c->D && i >= 0) ? c->D[i] : 0;
    if (z < bound) return;
    if (i < 0) {
        push_hit(c->hits, c->read, c->strand, k, l, c->z0 - z);
        return;
    }
    c->nodes++;
    for (int b = 0; b < 4; b++) {
        int64_t kb = (int64_t)c->x->C[b] + occ_at(c->x, b, k - 1) + 1;
        int64_t lb = (int64_t)c->x->C[b] + occ_at(c->x, b, l);
        if (kb <= lb) {
            if (b == c->W[i]) inex_recur(c, i - 1, z, kb, lb);
            else inex_recur(c, i - 1, z - 1, kb, lb);
        }
    }
}

/* ------------------------------------------------------------------ definition of the hit set */

/* Every W' over ACGT of the read's length with Hamming distance d <= z to W (a
 * non-ACGT position always differs) that occurs in R contributes (k(W'), l(W'), d). */
typedef struct {
    const oracle_index *x;
    const uint8_t *P;
    uint8_t *Wp;
    int64_t m;
    uint32_t read;
    uint8_t strand;
    hit_list *hits;
} ball_ctx;

static void ball_recur(ball_ctx *c, int64_t from, int used, int budget)
{
    int64_t k, l;
    int clean = 1;
    for (int64_t i = 0; i < c->m; i++)
        if (c->Wp[i] > 3) clean = 0;             /* N still unresolved: not a word over ACGT */
    if (clean) {
        interval_by_definition(c->x, c->Wp, c->m, &k, &l);
        if (k <= l) push_hit(c->hits, c->read, c->strand, k, l, used);
    }
    if (used == budget) return;
    for (int64_t i = from; i < c->m; i++) {
        uint8_t orig = c->Wp[i];
        for (uint8_t b = 0; b < 4; b++) {
            if (b == orig) continue;
            c->Wp[i] = b;
            ball_recur(c, i + 1, used + 1, budget);
        }
        c->Wp[i] = orig;
        if (orig > 3) return;                    /* an N left unsubstituted cannot match */
    }
}

/* Inexact search of every read on the requested strands with per-read budgets z.
 * method 0: the Hamming-ball definition; 1: Listing 2 (substitutions); 2: Listing 2
 * with the D-array bound (needs rev). Hits are sorted by (read, strand, k). Writes at
 * most cap hits and returns the total number; hit_offs gets nreads+1 CSR offsets and
 * nodes_out (optional) the per-read count of expanded nodes (methods 1 and 2). */
int64_t oracle_inexact(const oracle_index *x, const oracle_index *rev, const uint8_t *codes,
                       const uint64_t *offs, const uint8_t *z, int64_t nreads, int strands,
                       int method, oracle_hit *out, int64_t cap, uint64_t *hit_offs,
                       uint64_t *nodes_out)
{
    hit_list h = {0, 0, 0};
    int64_t maxm = 0;
    for (int64_t r = 0; r < nreads; r++)
        if ((int64_t)(offs[r + 1] - offs[r]) > maxm) maxm = (int64_t)(offs[r + 1] - offs[r]);
    uint8_t *P = malloc((size_t)(maxm + 1));
    uint8_t *Wp = malloc((size_t)(maxm + 1));
    uint8_t *D = malloc((size_t)(maxm + 1));
    for (int64_t r = 0; r < nreads; r++) {
        int64_t m = (int64_t)(offs[r + 1] - offs[r]);
        uint64_t nodes = 0;
        for (int s = 0; s < 2; s++) {
            if (!(strands & (1 << s))) continue;
            strand_pattern(codes + offs[r], m, s, P);
            if (method == 0) {
                ball_ctx b = {x, P, Wp, m, (uint32_t)r, (uint8_t)s, &h};
                memcpy(Wp, P, (size_t)m);
                ball_recur(&b, 0, 0, z[r]);
            } else {
                inex_ctx c = {x, P, NULL, z[r], (uint32_t)r, (uint8_t)s, &h, 0};
                if (method == 2) {
                    oracle_darray_one(rev, P, m, D);
                    c.D = D;
                }
                inex_recur(&c, m - 1, z[r], 0, x->n);
                nodes += c.nodes;
            }
        }
        if (nodes_out) nodes_out[r] = nodes;
    }
    free(P);
    free(Wp);
    free(D);
    if (h.len) qsort(h.buf, (size_t)h.len, sizeof(oracle_hit), cmp_hit);
    int64_t j = 0;
    for (int64_t r = 0; r < nreads; r++) {
        hit_offs[r] = (uint64_t)j;
        while (j < h.len && h.buf[j].read == (uint32_t)r) j++;
    }
    hit_offs[nreads] = (uint64_t)h.len;
    int64_t w = h.len < cap ? h.len : cap;
    if (w > 0) memcpy(out, h.buf, sizeof(oracle_hit) * (size_t)w);
    free(h.buf);
    return h.len;
}

/* ------------------------------------------------------------------ text-only checkers
 * Two computations from the text alone, with no suffix array, BWT, Occ or C, for checks
 * at sizes where the full index above is too large to build. */

/* Rank scan over T = R$: *k = number of suffixes of T smaller than P and *occ = number of
 * positions where P occurs in R. A suffix that reaches '$' while still equal to a prefix
 * of P is smaller than P ('$' sorts first). The interval of P is (k, k + occ - 1). */
void oracle_rank_scan(const uint8_t *R, int64_t n, const uint8_t *P, int64_t m, int64_t *k, int64_t *occ)
{
    int64_t less = 0, eq = 0;
    for (int64_t j = 0; j <= n; j++) {
        const int64_t avail = n - j;
        const int64_t t = avail < m ? avail : m;
        const int r = t ? memcmp(R + j, P, (size_t)t) : 0;
        if (r < 0 || (r == 0 && avail < m)) less++;
        else if (r == 0) eq++;
    }
    *k = less;
    *occ = eq;
}

static int64_t hamming(const uint8_t *a, const uint8_t *b, int64_t m)
{
    int64_t d = 0;
    for (int64_t i = 0; i < m; i++) d += a[i] != b[i];   /* code 4 never equals a text symbol */
    return d;
}

static const uint8_t *win_R;
static int64_t win_m;

static int cmp_window(const void *pa, const void *pb)
{
    return memcmp(win_R + *(const int64_t *)pa, win_R + *(const int64_t *)pb, (size_t)win_m);
}

/* Substitution hit set of one strand pattern P (length m, budget z) by the pigeonhole
 * principle: a window W' of R within Hamming distance z of P agrees with P exactly on at
 * least one of z+1 disjoint pieces of P (pieces are empty when m < z+1, and an empty piece
 * agrees everywhere). Every occurrence of a piece fixes a candidate
 * window; candidates within distance z are kept, identical windows merged, and each
 * distinct W' gets its interval from the rank scan. Writes up to cap (k, l, d) triples,
 * sorted by k, and returns their number. */
int64_t oracle_hits_pigeonhole(const uint8_t *R, int64_t n, const uint8_t *P, int64_t m, int z,
                               uint32_t *out, int64_t cap)
{
    if (m == 0) {
        if (cap > 0) {
            out[0] = 0;
            out[1] = (uint32_t)n;
            out[2] = 0;
        }
        return 1;
    }
    const int parts = z + 1;
    int64_t a[8], b[8];
    for (int i = 0; i < parts; i++) {
        a[i] = m * i / parts;
        b[i] = m * (i + 1) / parts;
    }
    int64_t ncand = 0, ccap = 1024;
    int64_t *cand = malloc(sizeof(int64_t) * (size_t)ccap);
    for (int64_t p = 0; p < n; p++) {
        for (int i = 0; i < parts; i++) {
            const int64_t len = b[i] - a[i];
            const int64_t s = p - a[i];
            if (s < 0 || s + m > n) continue;
            /* an empty piece (m < z + 1) agrees everywhere */
            if (len > 0 && (R[p] != P[a[i]] || memcmp(R + p, P + a[i], (size_t)len) != 0)) continue;
            if (hamming(R + s, P, m) > z) continue;
            if (ncand == ccap) {
                ccap *= 2;
                cand = realloc(cand, sizeof(int64_t) * (size_t)ccap);
            }
            cand[ncand++] = s;
        }
    }
    win_R = R;
    win_m = m;
    if (ncand) qsort(cand, (size_t)ncand, sizeof(int64_t), cmp_window);
    int64_t nh = 0;
    for (int64_t c = 0; c < ncand; c++) {
        if (c > 0 && memcmp(R + cand[c - 1], R + cand[c], (size_t)m) == 0) continue;
        int64_t k, occ;
        oracle_rank_scan(R, n, R + cand[c], m, &k, &occ);
        if (nh < cap) {
            out[3 * nh] = (uint32_t)k;
            out[3 * nh + 1] = (uint32_t)(k + occ - 1);
            out[3 * nh + 2] = (uint32_t)hamming(R + cand[c], P, m);
        }
        nh++;
    }
    free(cand);
    return nh;
}
