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
 *   - Listing 2: every child interval is computed from its parent's (k, l), every branch
 *     that extends the string needs a non-empty interval, and by default only the
 *     substitution branches are taken (the deletion and insertion branches on request);
 *   - read symbols outside ACGT (code 4) occur nowhere in R and never equal a base;
 *   - the reverse-complement strand of a read W is W reversed with c -> 3 - c.
 *
 * Symbol codes: A=0, C=1, G=2, T=3; '$' is kept out of band (BWT code 4).
 */
#include <pthread.h>
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

/* One edge below a node of Listing 2's search tree: the pattern position still to
 * match, the budget left after the edge's cost, and the interval of the string W' built
 * so far (symbols are prepended: backward search). */
typedef struct {
    int64_t i;
    int z;
    int64_t k, l;
} inex_child;

/* A node whose budget is below what its pattern prefix still needs is not expanded: the
 * listing's "z < 0", or "z < D(i)" with the D lower bound (D(-1) = 0). */
static int inex_pruned(const inex_ctx *c, int64_t i, int z)
{
    const int need = (c->D && i >= 0) ? c->D[i] : 0;
    return z < need;
}

/* The edges below node (i, z, k, l). Each symbol b whose extension bW' occurs (its
 * interval by the update of Listing 1 is non-empty) gives a step to position i-1, free
 * when b is W[i] and one substitution otherwise; every child interval is computed from
 * the node's own (k, l). With gaps the listing's two other branches are taken as well:
 * W[i] deleted (position i-1, the node's interval, cost 1) and b inserted before W[i]
 * (position i, the interval of bW', cost 1). Returns the number of edges (at most 9). */
static int inex_children(const inex_ctx *c, int gaps, int64_t i, int z, int64_t k, int64_t l, inex_child *out)
{
    int n = 0;
    if (gaps) out[n++] = (inex_child){i - 1, z - 1, k, l};
    for (int b = 0; b < 4; b++) {
        const int64_t kb = (int64_t)c->x->C[b] + occ_at(c->x, b, k - 1) + 1;
        const int64_t lb = (int64_t)c->x->C[b] + occ_at(c->x, b, l);
        if (kb > lb) continue;
        if (gaps) out[n++] = (inex_child){i, z - 1, kb, lb};
        out[n++] = (inex_child){i - 1, b == c->W[i] ? z : z - 1, kb, lb};
    }
    return n;
}

/* The search below node (i, z, k, l): a node past the pattern's first symbol (i < 0) is a
 * hit of cost z0 - z; any other node not pruned is expanded (counted in c->nodes) and its
 * edges searched. */
static void inex_search(inex_ctx *c, int gaps, int64_t i, int z, int64_t k, int64_t l)
{
    if (inex_pruned(c, i, z)) return;
    if (i < 0) {
        push_hit(c->hits, c->read, c->strand, k, l, c->z0 - z);
        return;
    }
    c->nodes++;
    inex_child ch[9];
    const int n = inex_children(c, gaps, i, z, k, l, ch);
    for (int j = 0; j < n; j++) inex_search(c, gaps, ch[j].i, ch[j].z, ch[j].k, ch[j].l);
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

/* Edit cost of aligning W (m symbols) with W' (mp symbols, codes 0..3) as Listing 2's
 * recursion aligns them: substitutions, deletions of W symbols and insertions of W'
 * symbols cost 1, a non-ACGT W symbol never matches, and no insertion may precede
 * W[0] (the recursion stops once W[0] is consumed). dp holds (m+1)(mp+1) entries:
 * dp[i][j] is the cost of W[0..i) against W'[0..j). */
static int constrained_edit(const uint8_t *W, int64_t m, const uint8_t *Wp, int64_t mp, int *dp)
{
    const int inf = 1 << 28;
    for (int64_t i = 0; i <= m; i++)
        for (int64_t j = 0; j <= mp; j++) {
            int v;
            if (i == 0) v = j == 0 ? 0 : inf;
            else if (j == 0) v = (int)i;
            else {
                v = dp[(i - 1) * (mp + 1) + j] + 1;                                 /* W[i-1] deleted */
                const int ins = dp[i * (mp + 1) + j - 1] + 1;                       /* W'[j-1] inserted */
                const int sub = dp[(i - 1) * (mp + 1) + j - 1] + (W[i - 1] != Wp[j - 1]);
                if (ins < v) v = ins;
                if (sub < v) v = sub;
            }
            dp[i * (mp + 1) + j] = v;
        }
    return dp[m * (mp + 1) + mp];
}

/* Definition of the gapped hit set: every W' over ACGT of length m-z .. m+z whose
 * constrained edit cost d to W is at most z and which occurs in R contributes
 * (k(W'), l(W'), d); the caller keeps the smallest d per interval. */
static void gap_definition(const oracle_index *x, const uint8_t *P, int64_t m, int z, uint32_t read, uint8_t strand,
                           hit_list *h)
{
    const int64_t lo = m - z > 0 ? m - z : 0, hi = m + z;
    uint8_t *Wp = malloc((size_t)hi + 1);
    int *dp = malloc(sizeof(int) * (size_t)(m + 1) * (size_t)(hi + 1));
    for (int64_t L = lo; L <= hi; L++) {
        uint64_t total = 1;
        for (int64_t t = 0; t < L; t++) total *= 4;
        for (uint64_t v = 0; v < total; v++) {
            uint64_t u = v;
            for (int64_t t = 0; t < L; t++) {
                Wp[t] = (uint8_t)(u & 3);
                u >>= 2;
            }
            const int d = constrained_edit(P, m, Wp, L, dp);
            if (d > z) continue;
            int64_t k, l;
            interval_by_definition(x, Wp, L, &k, &l);
            if (k <= l) push_hit(h, read, strand, k, l, d);
        }
    }
    free(Wp);
    free(dp);
}

static int cmp_hit_gap(const void *pa, const void *pb)
{
    const oracle_hit *a = pa, *b = pb;
    if (a->read != b->read) return a->read < b->read ? -1 : 1;
    if (a->strand != b->strand) return a->strand < b->strand ? -1 : 1;
    if (a->k != b->k) return a->k < b->k ? -1 : 1;
    if (a->l != b->l) return a->l < b->l ? -1 : 1;
    return (a->d > b->d) - (a->d < b->d);
}

/* Inexact search of every read on the requested strands with per-read budgets z.
 * method 0: the Hamming-ball definition; 1: Listing 2 (substitutions); 2: Listing 2
 * with the D-array bound (needs rev); 3: Listing 2 with all its branches (deletions and
 * insertions too); 4: method 3 with the D-array bound; 5: the definition of method 3's
 * hit set (small inputs only). Hits are sorted by (read, strand, k), and for methods
 * 3-5 by l too, one per interval with its smallest cost. Writes at most cap hits and
 * returns the total number; hit_offs gets nreads+1 CSR offsets and nodes_out
 * (optional) the per-read count of expanded nodes (methods 1-4). */
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
            } else if (method == 5) {
                gap_definition(x, P, m, z[r], (uint32_t)r, (uint8_t)s, &h);
            } else {
                inex_ctx c = {x, P, NULL, z[r], (uint32_t)r, (uint8_t)s, &h, 0};
                if (method == 2 || method == 4) {
                    oracle_darray_one(rev, P, m, D);
                    c.D = D;
                }
                inex_search(&c, method >= 3, m - 1, z[r], 0, x->n);
                nodes += c.nodes;
            }
        }
        if (nodes_out) nodes_out[r] = nodes;
    }
    free(P);
    free(Wp);
    free(D);
    if (method >= 3) {
        /* one hit per (read, strand, interval): the smallest cost */
        if (h.len) qsort(h.buf, (size_t)h.len, sizeof(oracle_hit), cmp_hit_gap);
        int64_t u = 0;
        for (int64_t e = 0; e < h.len; e++) {
            const oracle_hit *a = &h.buf[e];
            if (u > 0) {
                const oracle_hit *p = &h.buf[u - 1];
                if (p->read == a->read && p->strand == a->strand && p->k == a->k && p->l == a->l) continue;
            }
            h.buf[u++] = *a;
        }
        h.len = u;
    } else if (h.len) {
        qsort(h.buf, (size_t)h.len, sizeof(oracle_hit), cmp_hit);
    }
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

/* ----------------------------------------------------------------- batched scale checkers
 *
 * The rank scan and the pigeonhole checker above take one pass over T per pattern. The
 * functions below give the same results for a whole batch of patterns in a few passes,
 * on host threads, so that texts of billions of symbols can be checked on thousands of
 * reads. They use nothing but T itself: no suffix array, BWT or Occ.
 *
 * Keys: the first KEYLEN symbols of a string as base-5 digits (codes 0..4, first symbol
 * most significant), so keys order like the strings they start. A text position whose
 * suffix has fewer than KEYLEN symbols before '$' has no key and is compared in full.
 */
#define KEYLEN 10
#define NKEYS 9765625            /* 5^10 */

static uint32_t key_of(const uint8_t *s)
{
    uint32_t k = 0;
    for (int i = 0; i < KEYLEN; i++) k = k * 5u + s[i];
    return k;
}

/* Three-way comparison of suffix j of T = R$ with P (length m): -1 when the suffix is
 * smaller ('$' sorts first), 0 when P is a prefix of the suffix (an occurrence), 1 when
 * larger. */
static int suffix_vs(const uint8_t *R, int64_t n, int64_t j, const uint8_t *P, int64_t m)
{
    const int64_t avail = n - j;
    const int64_t t = avail < m ? avail : m;
    const int r = t ? memcmp(R + j, P, (size_t)t) : 0;
    if (r < 0) return -1;
    if (r > 0) return 1;
    return avail < m ? -1 : 0;
}

typedef struct {
    const uint8_t *R;
    int64_t n, lo, hi;          /* text positions [lo, hi) */
    uint32_t *hist;             /* NKEYS counters (pass 1) */
    /* pass 2 */
    const uint8_t *inset;       /* NKEYS flags: some long pattern has this key */
    const uint32_t *bkey;       /* sorted keys of the long patterns */
    const int64_t *border;      /* pattern ids in bkey order */
    int64_t nb;
    const uint8_t *codes;
    const uint64_t *offs;
    int64_t *less, *occ;        /* per pattern, this thread's counts */
} ScanPart;

static void *hist_pass(void *arg)
{
    ScanPart *p = arg;
    const int64_t end = p->n - KEYLEN;        /* last position with a key */
    for (int64_t j = p->lo; j < p->hi && j <= end; j++) p->hist[key_of(p->R + j)]++;
    return NULL;
}

static void *bucket_pass(void *arg)
{
    ScanPart *p = arg;
    const int64_t end = p->n - KEYLEN;
    for (int64_t j = p->lo; j < p->hi && j <= end; j++) {
        const uint32_t k = key_of(p->R + j);
        if (!p->inset[k]) continue;
        int64_t a = 0, b = p->nb;             /* first bucket entry with this key */
        while (a < b) {
            const int64_t mid = (a + b) / 2;
            if (p->bkey[mid] < k) a = mid + 1;
            else b = mid;
        }
        for (int64_t e = a; e < p->nb && p->bkey[e] == k; e++) {
            const int64_t q = p->border[e];
            const int64_t m = (int64_t)(p->offs[q + 1] - p->offs[q]);
            const int c = suffix_vs(p->R, p->n, j, p->codes + p->offs[q], m);
            if (c < 0) p->less[q]++;
            else if (c == 0) p->occ[q]++;
        }
    }
    return NULL;
}

static int cmp_u32_pair(const void *a, const void *b)
{
    const uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : x > y;
}

/* For patterns q = 0..np-1 (codes[offs[q] .. offs[q+1]), codes 0..4): k[q] = number of
 * suffixes of T = R$ smaller than the pattern and occ[q] = number of its occurrences in
 * R -- oracle_rank_scan for every pattern, in two passes over R on `threads` threads.
 * A suffix with a key and a pattern of at least KEYLEN symbols compare by key unless the
 * keys are equal; then, and for shorter patterns or suffixes, the comparison is made in
 * full (shorter patterns P compare against keys through the range of keys that start
 * with P). Returns 0, or -1 when memory runs out. */
int oracle_rank_scan_batch(const uint8_t *R, int64_t n, const uint8_t *codes, const uint64_t *offs, int64_t np,
                           int threads, int64_t *k, int64_t *occ)
{
    if (threads < 1) threads = 1;
    int rc = -1;
    uint64_t *cum = NULL;                       /* cum[key] = text keys below key */
    uint32_t **hist = calloc((size_t)threads, sizeof *hist);
    ScanPart *part = calloc((size_t)threads, sizeof *part);
    pthread_t *tid = calloc((size_t)threads, sizeof *tid);
    uint8_t *inset = NULL;
    uint64_t *kb = NULL;
    uint32_t *bkey = NULL;
    int64_t *border = NULL, *lessv = NULL, *occv = NULL;
    if (!hist || !part || !tid) goto out;
    for (int64_t q = 0; q < np; q++) k[q] = occ[q] = 0;
    const int64_t chunk = (n + threads - 1) / threads;

    /* pass 1: histogram of the text's keys */
    for (int t = 0; t < threads; t++) {
        hist[t] = calloc(NKEYS, sizeof(uint32_t));
        if (!hist[t]) goto out;
        part[t].R = R;
        part[t].n = n;
        part[t].lo = t * chunk;
        part[t].hi = (t + 1) * chunk < n ? (t + 1) * chunk : n;
        part[t].hist = hist[t];
        pthread_create(&tid[t], NULL, hist_pass, &part[t]);
    }
    for (int t = 0; t < threads; t++) pthread_join(tid[t], NULL);
    cum = malloc(sizeof(uint64_t) * (NKEYS + 1));
    if (!cum) goto out;
    cum[0] = 0;
    for (uint32_t key = 0; key < NKEYS; key++) {
        uint64_t s = 0;
        for (int t = 0; t < threads; t++) s += hist[t][key];
        cum[key + 1] = cum[key] + s;
    }

    /* keyed part of each pattern's counts */
    int64_t nlong = 0;
    for (int64_t q = 0; q < np; q++) {
        const uint8_t *P = codes + offs[q];
        const int64_t m = (int64_t)(offs[q + 1] - offs[q]);
        if (m >= KEYLEN) {
            k[q] = (int64_t)cum[key_of(P)];        /* keyed suffixes with a smaller key */
            nlong++;
        } else {
            /* keys starting with P: [P 0..0, P 4..4]; smaller keys are smaller suffixes,
               keys in the range are suffixes that P is a prefix of */
            uint32_t lo = 0, hi = 0;
            for (int i = 0; i < KEYLEN; i++) {
                lo = lo * 5u + (i < m ? P[i] : 0u);
                hi = hi * 5u + (i < m ? P[i] : 4u);
            }
            k[q] = (int64_t)cum[lo];
            occ[q] = (int64_t)(cum[hi + 1] - cum[lo]);
        }
    }

    /* pass 2: keyed suffixes in the bucket of a long pattern, compared in full */
    if (nlong) {
        inset = calloc(NKEYS, 1);
        kb = malloc(sizeof(uint64_t) * (size_t)nlong);
        bkey = malloc(sizeof(uint32_t) * (size_t)nlong);
        border = malloc(sizeof(int64_t) * (size_t)nlong);
        lessv = calloc((size_t)np * (size_t)threads, sizeof(int64_t));
        occv = calloc((size_t)np * (size_t)threads, sizeof(int64_t));
        if (!inset || !kb || !bkey || !border || !lessv || !occv) goto out;
        int64_t e = 0;
        for (int64_t q = 0; q < np; q++) {
            const int64_t m = (int64_t)(offs[q + 1] - offs[q]);
            if (m < KEYLEN) continue;
            const uint32_t key = key_of(codes + offs[q]);
            kb[e++] = ((uint64_t)key << 32) | (uint64_t)q;   /* np < 2^32 */
            inset[key] = 1;
        }
        qsort(kb, (size_t)nlong, sizeof(uint64_t), cmp_u32_pair);
        for (e = 0; e < nlong; e++) {
            bkey[e] = (uint32_t)(kb[e] >> 32);
            border[e] = (int64_t)(kb[e] & 0xFFFFFFFFu);
        }
        for (int t = 0; t < threads; t++) {
            part[t].inset = inset;
            part[t].bkey = bkey;
            part[t].border = border;
            part[t].nb = nlong;
            part[t].codes = codes;
            part[t].offs = offs;
            part[t].less = lessv + (size_t)t * (size_t)np;
            part[t].occ = occv + (size_t)t * (size_t)np;
            pthread_create(&tid[t], NULL, bucket_pass, &part[t]);
        }
        for (int t = 0; t < threads; t++) pthread_join(tid[t], NULL);
        for (int t = 0; t < threads; t++)
            for (int64_t q = 0; q < np; q++) {
                k[q] += lessv[(size_t)t * (size_t)np + q];
                occ[q] += occv[(size_t)t * (size_t)np + q];
            }
    }

    /* suffixes without a key (fewer than KEYLEN symbols before '$'), compared in full */
    for (int64_t j = n - KEYLEN + 1 < 0 ? 0 : n - KEYLEN + 1; j <= n; j++)
        for (int64_t q = 0; q < np; q++) {
            const int c = suffix_vs(R, n, j, codes + offs[q], (int64_t)(offs[q + 1] - offs[q]));
            if (c < 0) k[q]++;
            else if (c == 0) occ[q]++;
        }
    rc = 0;
out:
    if (hist)
        for (int t = 0; t < threads; t++) free(hist[t]);
    free(hist);
    free(part);
    free(tid);
    free(cum);
    free(inset);
    free(kb);
    free(bkey);
    free(border);
    free(lessv);
    free(occv);
    return rc;
}

/* ---- pigeonhole for a batch of patterns */

#define SEEDLEN 12               /* seeds are found by their first 12 symbols, 2 bits each */

typedef struct {
    const uint8_t *R;
    int64_t n, lo, hi;
    const uint64_t *seedbits;    /* 4^12 bits: some seed starts with these 12 symbols */
    const uint64_t *seeds;       /* sorted (key << 32 | seed id) */
    int64_t ns;
    const int64_t *seed_q, *seed_a, *seed_len;   /* per seed: pattern, piece start, piece length */
    const uint8_t *codes;
    const uint64_t *offs;
    const int *z;
    int64_t *cand;               /* (pattern, window start) pairs found by this thread */
    int64_t ncand, ccap;
    int failed;
} SeedPart;

static void *seed_pass(void *arg)
{
    SeedPart *p = arg;
    const int64_t last = p->n - SEEDLEN;
    uint32_t key = 0;
    const uint32_t mask = (1u << (2 * SEEDLEN)) - 1u;
    int64_t j0 = p->lo;
    for (int i = 0; i < SEEDLEN - 1 && j0 + i < p->n; i++) key = (key << 2) | p->R[j0 + i];
    for (int64_t j = j0; j < p->hi && j <= last; j++) {
        key = ((key << 2) | p->R[j + SEEDLEN - 1]) & mask;
        if (!((p->seedbits[key >> 6] >> (key & 63)) & 1u)) continue;
        int64_t a = 0, b = p->ns;
        while (a < b) {
            const int64_t mid = (a + b) / 2;
            if ((p->seeds[mid] >> 32) < key) a = mid + 1;
            else b = mid;
        }
        for (int64_t e = a; e < p->ns && (p->seeds[e] >> 32) == key; e++) {
            const int64_t sd = (int64_t)(p->seeds[e] & 0xFFFFFFFFu);
            const int64_t q = p->seed_q[sd], pa = p->seed_a[sd], len = p->seed_len[sd];
            const uint8_t *P = p->codes + p->offs[q];
            const int64_t m = (int64_t)(p->offs[q + 1] - p->offs[q]);
            const int64_t s = j - pa;
            if (s < 0 || s + m > p->n) continue;
            if (memcmp(p->R + j, P + pa, (size_t)len) != 0) continue;
            if (hamming(p->R + s, P, m) > p->z[q]) continue;
            if (p->ncand == p->ccap) {
                const int64_t nc = p->ccap ? 2 * p->ccap : 1024;
                int64_t *c = realloc(p->cand, sizeof(int64_t) * 2 * (size_t)nc);
                if (!c) {
                    p->failed = 1;
                    return NULL;
                }
                p->cand = c;
                p->ccap = nc;
            }
            p->cand[2 * p->ncand] = q;
            p->cand[2 * p->ncand + 1] = s;
            p->ncand++;
        }
    }
    return NULL;
}

static const uint8_t *pg_R;
static const int64_t *pg_len;   /* window length per pattern */

/* order of candidates: pattern, then window content, then start */
static int cmp_cand(const void *pa, const void *pb)
{
    const int64_t *x = pa, *y = pb;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    const int r = memcmp(pg_R + x[1], pg_R + y[1], (size_t)pg_len[x[0]]);
    if (r) return r;
    return (x[1] > y[1]) - (x[1] < y[1]);
}

/* oracle_hits_pigeonhole for patterns q = 0..np-1 with budgets z[q] <= 7: hits of pattern
 * q go to out[3*hoff[q] .. 3*hoff[q+1]) as (k, l, d) triples sorted by k, for up to cap
 * triples in all; hoff (np + 1 entries) is written even when cap is exceeded. Seeds
 * (pieces of at least SEEDLEN symbols holding no N) are found in one pass over R on
 * `threads` threads; patterns with a shorter piece use oracle_hits_pigeonhole. The
 * distinct windows get their intervals from oracle_rank_scan_batch. Returns the total
 * number of hits, or -1 when memory runs out. */
int64_t oracle_hits_pigeonhole_batch(const uint8_t *R, int64_t n, const uint8_t *codes, const uint64_t *offs,
                                     const int *z, int64_t np, int threads, uint32_t *out, int64_t cap,
                                     int64_t *hoff)
{
    if (threads < 1) threads = 1;
    int64_t total = -1;
    int64_t ns = 0, scap = 0;
    int64_t *seed_q = NULL, *seed_a = NULL, *seed_len = NULL, *wlen = NULL, *cand = NULL, *nh = NULL;
    uint64_t *seeds = NULL, *seedbits = NULL, *woffs = NULL;
    uint8_t *slow = NULL, *wcodes = NULL;
    int64_t *wk = NULL, *wocc = NULL;
    SeedPart *part = calloc((size_t)threads, sizeof *part);
    pthread_t *tid = calloc((size_t)threads, sizeof *tid);
    slow = calloc((size_t)np + 1, 1);
    wlen = malloc(sizeof(int64_t) * ((size_t)np + 1));
    nh = calloc((size_t)np + 1, sizeof(int64_t));
    if (!part || !tid || !slow || !wlen || !nh) goto out;

    for (int64_t q = 0; q < np; q++) {
        const uint8_t *P = codes + offs[q];
        const int64_t m = (int64_t)(offs[q + 1] - offs[q]);
        const int parts = z[q] + 1;
        wlen[q] = m;
        for (int i = 0; i < parts; i++)
            if (m * (i + 1) / parts - m * i / parts < SEEDLEN) slow[q] = 1;
        if (slow[q]) continue;
        for (int i = 0; i < parts; i++) {
            const int64_t a = m * i / parts, b = m * (i + 1) / parts;
            int has_n = 0;
            for (int64_t x = a; x < b; x++) has_n |= P[x] > 3;
            if (has_n) continue;
            if (ns == scap) {
                scap = scap ? 2 * scap : 1024;
                seeds = realloc(seeds, sizeof(uint64_t) * (size_t)scap);
                seed_q = realloc(seed_q, sizeof(int64_t) * (size_t)scap);
                seed_a = realloc(seed_a, sizeof(int64_t) * (size_t)scap);
                seed_len = realloc(seed_len, sizeof(int64_t) * (size_t)scap);
                if (!seeds || !seed_q || !seed_a || !seed_len) goto out;
            }
            uint32_t key = 0;
            for (int x = 0; x < SEEDLEN; x++) key = (key << 2) | P[a + x];
            seeds[ns] = ((uint64_t)key << 32) | (uint64_t)ns;
            seed_q[ns] = q;
            seed_a[ns] = a;
            seed_len[ns] = b - a;
            ns++;
        }
    }
    seedbits = calloc((size_t)1 << (2 * SEEDLEN - 6), sizeof(uint64_t));
    if (!seedbits) goto out;
    if (ns) qsort(seeds, (size_t)ns, sizeof(uint64_t), cmp_u32_pair);
    for (int64_t e = 0; e < ns; e++) {
        const uint32_t key = (uint32_t)(seeds[e] >> 32);
        seedbits[key >> 6] |= 1ull << (key & 63);
    }
    const int64_t chunk = (n + threads - 1) / threads;
    for (int t = 0; t < threads; t++) {
        SeedPart *p = &part[t];
        p->R = R;
        p->n = n;
        p->lo = t * chunk;
        p->hi = (t + 1) * chunk < n ? (t + 1) * chunk : n;
        p->seedbits = seedbits;
        p->seeds = seeds;
        p->ns = ns;
        p->seed_q = seed_q;
        p->seed_a = seed_a;
        p->seed_len = seed_len;
        p->codes = codes;
        p->offs = offs;
        p->z = z;
        pthread_create(&tid[t], NULL, seed_pass, p);
    }
    int64_t nc = 0;
    for (int t = 0; t < threads; t++) {
        pthread_join(tid[t], NULL);
        if (part[t].failed) goto out;
        nc += part[t].ncand;
    }
    cand = malloc(sizeof(int64_t) * 2 * (size_t)(nc ? nc : 1));
    if (!cand) goto out;
    nc = 0;
    for (int t = 0; t < threads; t++) {
        memcpy(cand + 2 * nc, part[t].cand, sizeof(int64_t) * 2 * (size_t)part[t].ncand);
        nc += part[t].ncand;
    }
    pg_R = R;
    pg_len = wlen;
    if (nc) qsort(cand, (size_t)nc, 2 * sizeof(int64_t), cmp_cand);
    /* distinct windows per pattern, in content order */
    int64_t nw = 0;
    for (int64_t c = 0; c < nc; c++) {
        const int64_t q = cand[2 * c], s = cand[2 * c + 1];
        if (c > 0 && cand[2 * c - 2] == q && memcmp(R + cand[2 * c - 1], R + s, (size_t)wlen[q]) == 0) continue;
        cand[2 * nw] = q;
        cand[2 * nw + 1] = s;
        nw++;
    }
    woffs = malloc(sizeof(uint64_t) * ((size_t)nw + 1));
    wk = malloc(sizeof(int64_t) * ((size_t)nw + 1));
    wocc = malloc(sizeof(int64_t) * ((size_t)nw + 1));
    if (!woffs || !wk || !wocc) goto out;
    woffs[0] = 0;
    for (int64_t w = 0; w < nw; w++) woffs[w + 1] = woffs[w] + (uint64_t)wlen[cand[2 * w]];
    wcodes = malloc(woffs[nw] ? woffs[nw] : 1);
    if (!wcodes) goto out;
    for (int64_t w = 0; w < nw; w++) memcpy(wcodes + woffs[w], R + cand[2 * w + 1], (size_t)wlen[cand[2 * w]]);
    if (oracle_rank_scan_batch(R, n, wcodes, woffs, nw, threads, wk, wocc)) goto out;

    /* hits per pattern: the batch's windows, or the per-pattern checker for slow ones */
    for (int64_t w = 0; w < nw; w++) nh[cand[2 * w]]++;
    total = 0;
    int64_t w = 0;
    for (int64_t q = 0; q < np; q++) {
        hoff[q] = total;
        const uint8_t *P = codes + offs[q];
        const int64_t m = wlen[q];
        if (slow[q] || m == 0) {
            uint32_t *dst = total < cap ? out + 3 * total : NULL;
            const int64_t room = total < cap ? cap - total : 0;
            const int64_t h = oracle_hits_pigeonhole(R, n, P, m, z[q], dst, room);
            total += h;
            continue;
        }
        for (; w < nw && cand[2 * w] == q; w++) {
            if (total < cap) {
                out[3 * total] = (uint32_t)wk[w];
                out[3 * total + 1] = (uint32_t)(wk[w] + wocc[w] - 1);
                out[3 * total + 2] = (uint32_t)hamming(R + cand[2 * w + 1], P, m);
            }
            total++;
        }
    }
    hoff[np] = total;
out:
    if (part)
        for (int t = 0; t < threads; t++) free(part[t].cand);
    free(part);
    free(tid);
    free(slow);
    free(wlen);
    free(nh);
    free(seeds);
    free(seed_q);
    free(seed_a);
    free(seed_len);
    free(seedbits);
    free(cand);
    free(woffs);
    free(wcodes);
    free(wk);
    free(wocc);
    return total;
}
