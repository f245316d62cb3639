/*
 * fm.h -- C ABI of libfmocc, an MI355X (gfx950) FM-index engine: the Occ computation
 * over an interleaved 2-bit BWT with checkpoint counts, and the exact and z-mismatch
 * backward searches built on it.
 *
 * Definitions follow "Vectorized Character Counting for Faster Pattern Matching"
 * (Snytsar): the suffix array of R$ (Background, Eq. 1), the BWT derived from it
 * (Eq. 2), Occ(c, k) = number of c in BWT[0..k] and C[c] = number of characters
 * smaller than c (Background, Fig. 1), the backward exact match (Listing 1) and the
 * inexact match (Listing 2, substitution branches).
 *
 * Conventions used by every call:
 *   - Symbol codes: A=0, C=1, G=2, T=3. In reads, any other value (4 is used for N)
 *     occurs nowhere in R and never equals a base.
 *   - R has length n; the index has n+1 rows 0..n; row 0 holds the suffix "$".
 *     n + 1 must be below 2^32.
 *   - An interval (k, l) names rows k..l (inclusive) whose suffix starts with the
 *     pattern; the empty pattern has (0, n). A pattern that does not occur is
 *     reported as the canonical miss (1, 0). Listing 1's update is
 *       k <- C[b] + Occ(b, k-1) + 1,   l <- C[b] + Occ(b, l),   Occ(b, -1) = 0.
 *   - Strand 0 searches the read W; strand 1 searches its reverse complement (W
 *     reversed, c -> 3 - c for c < 4).
 *   - Device pointers are HIP device memory (for example torch tensors' data_ptr());
 *     host pointers are ordinary process memory. The library never keeps a pointer
 *     it is passed beyond the call, except an index that owns its own memory.
 *   - `stream` is a hipStream_t (NULL = the null stream). Calls that take a stream
 *     only enqueue work and return; results are valid once the stream reaches them.
 *   - Return values are FM_OK or an fm_status code; argument errors are detected on
 *     the host before anything is enqueued. Per-read problems are reported per read
 *     in device status words and never fail the whole call.
 */
#ifndef FM_H
#define FM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fm_index fm_index;   /* opaque, immutable after construction except for
                                       its launch tuning; one device */

typedef struct {
    uint32_t k, l;                  /* inclusive row range; miss = (1, 0) */
} fm_interval;

typedef struct {
    uint32_t read;                  /* read number in the batch */
    uint32_t k, l;                  /* interval of one distinct W' */
    uint8_t strand;                 /* 0 = W, 1 = reverse complement */
    uint8_t nmm;                    /* substitutions in W' relative to the strand */
    uint16_t pad;
} fm_hit;                           /* 16 bytes */

enum fm_status {
    FM_OK = 0,
    FM_EINVAL = 1,                  /* bad argument (or, per read, a budget above zmax) */
    FM_EIO = 2,                     /* file could not be read or written */
    FM_EFORMAT = 3,                 /* index file or BWT is malformed */
    FM_ENOMEM = 4,                  /* host or device allocation failed */
    FM_EDEVICE = 5,                 /* a HIP call failed */
    FM_EOVERFLOW = 6,               /* per read: its hits did not fit in hit_cap */
    FM_EBUDGET = 7,                 /* per read: node budget exhausted */
    FM_ERANGE = 8,                  /* size beyond what the index or ABI supports */
    FM_EAGAIN = 9                   /* not finished within the time allowed */
};

/* Search flags. */
enum {
    FM_FWD = 1,                     /* search strand 0 */
    FM_REVCOMP = 2,                 /* search strand 1 */
    FM_BOTH = 3,
    FM_DARRAY = 4,                  /* prune with the D lower bound (needs the reverse index) */
    FM_PLAIN = 16,                  /* use the plain one-thread-per-read-strand kernels */
    FM_STATS = 32,                  /* count Occ queries and bucket fetches into the workspace */
    FM_FULL_RANK = 64,              /* fm_search_exact: no early exit; misses report (rank, rank-1) */
    FM_GAPS = 128,                  /* fm_search_inexact: Listing 2 with its deletion and insertion
                                       branches too (edit differences, not only substitutions) */
    FM_TUNE_KEEP_LAYOUT = 256       /* fm_autotune only: keep the current layout and lanes per
                                       read-strand and time the other settings */
};

/* Load flags. */
enum {
    FM_LOAD_REVERSE = 1,            /* also build/keep the index of reverse(R) */
    FM_LOAD_ALL_LAYOUTS = 2,        /* build the layouts for every supported I */
    FM_LOAD_DEVICE_SORT = 4,        /* fm_index_from_text: sort suffixes on the device (see
                                       fm_bwt_device) instead of the host builder; same index */
    FM_LOAD_LOCATE = 8              /* fm_index_from_text: keep the SA values of every 32nd row,
                                       so that fm_locate works (4 bytes per 32 rows) */
};

#define FM_ZMAX 4                   /* largest per-read mismatch budget */

typedef struct {
    int device;                     /* HIP device ordinal */
    uint32_t occ_interval;          /* checkpoint interval I: 64, 96, 128, 192, 224, 256, 448;
                                       0 for 128 */
    uint32_t flags;                 /* FM_LOAD_* */
    void *dev_buf;                  /* NULL: the index allocates its device memory and frees it
                                       in fm_index_free. Otherwise caller-owned device memory
                                       on `device`, 256-byte aligned, of dev_buf_bytes bytes
                                       (at least fm_index_bytes / fm_index_required_bytes),
                                       into which the index places everything it keeps (its
                                       layouts and SA samples); the caller frees it, and it
                                       must outlive the index. Construction still allocates
                                       transient working memory, freed before it returns. */
    size_t dev_buf_bytes;
} fm_load_opts;

typedef struct {
    uint64_t n;                     /* |R|; rows 0..n */
    uint64_t dollar_row;            /* row whose BWT symbol is '$' */
    uint64_t C[5];                  /* C[4] = n */
    uint64_t rev_dollar_row;        /* same for reverse(R), if present */
    uint64_t rev_C[5];
    uint32_t occ_interval;          /* layout used by the searches */
    uint32_t layouts;               /* built layouts: bits 0..6 = I of 64, 96, 128, 192, 224,
                                       256, 448 */
    uint32_t has_reverse;
    uint32_t sa_sample;             /* 32 when SA samples are kept (fm_locate), else 0 */
    uint64_t device_bytes;          /* device memory the index keeps (in its own allocation, or
                                       in the caller's dev_buf) */
    uint32_t caller_memory;         /* 1 when that memory is the caller's dev_buf */
    uint32_t table_depth;           /* longest strings in the prefix table (see fm_tuning) */
} fm_info;

/* Launch configuration of one operation (see fm_get_tuning). */
typedef struct {
    uint32_t occ_interval;          /* one of the index's layouts (see fm_load_opts) */
    uint32_t lanes;                 /* lanes per read-strand: 1, 2, 4 or 8, at most the bucket's
                                       16-byte chunks (2 for I = 64/96, 4 for 128/192/224,
                                       8 for 256/448) */
    uint32_t depth;                 /* walks: read-strands in flight per lane group, 1 or 2
                                       (the DFS keeps one); FM_OP_LOCATE: rows in flight per
                                       lane, 1, 2 or 4 */
    uint32_t block;                 /* threads per workgroup: 64, 128, 192 or 256 */
    uint32_t waves_per_cu;          /* persistent grid = CUs * waves_per_cu * 64 / block;
                                       0 = as many as fit */
    uint32_t node_budget;           /* inexact: DFS nodes per read-strand before FM_EBUDGET */
    uint32_t order;                 /* substitution search with FM_DARRAY, batched kernels:
                                       1 = the DFS claims read-strands heaviest first,
                                       weighing each by its D bound's slack, sum over i of
                                       max(0, z - D(i)); 0 = in read order (always so with
                                       FM_GAPS). Results are the same either way. */
    uint32_t table_depth;           /* substitution search, one lane per read-strand: a DFS node
                                       whose matched pattern suffix S is shorter than this takes
                                       the intervals of its four children bS from the index's
                                       prefix table (the Listing 1 interval of every string of
                                       length 1..fm_info.table_depth, kept at load time) instead
                                       of an Occ8 over the BWT; 0 = never. At most
                                       fm_info.table_depth. Results are the same either way. */
} fm_tuning;

/* Operations with launch settings of their own. FM_OP_LOCATE (fm_locate: layout, depth
 * and waves_per_cu; lanes are unused) is set by hand, not by fm_autotune. */
enum { FM_OP_EXACT = 0, FM_OP_DARRAY = 1, FM_OP_INEXACT = 2, FM_OP_LOCATE = 3 };

/* ----------------------------------------------------------------- general */

/* Text for a status code; never NULL. */
const char *fm_strerror(int status);

/* ABI version (increases when signatures change). */
int fm_version(void);

/* ----------------------------------------------------------------- construction (host) */

/* BWT of R$ computed by the library's host builder (suffix array by induced sorting,
 * then Eq. 2). text: host, n codes 0..3. bwt: host, n+1 bytes, receives codes 0..3
 * and 4 at the '$' row, which is stored in *dollar_row. FM_EINVAL on a code above 3
 * or n + 1 >= 2^32; FM_ENOMEM when the builder's memory cannot be allocated. */
int fm_bwt_host(const uint8_t *text, uint64_t n, uint8_t *bwt, uint64_t *dollar_row);

/* The same BWT computed on a device: the suffixes of R$ are sorted by prefix doubling
 * (first by their first 21 symbols, then, for the suffixes that still tie, by pairs of
 * ranks of prefixes of length L and 2L, with device radix sorts), and Eq. 2 is applied
 * to the result. text and bwt are host arrays as in fm_bwt_host; the device allocates
 * about 41(n+1) bytes of working memory during the call. FM_EINVAL on a code above 3,
 * FM_ERANGE when n + 1 >= 2^32, FM_ENOMEM when the device memory cannot be allocated. */
int fm_bwt_device(const uint8_t *text, uint64_t n, uint8_t *bwt, uint64_t *dollar_row, int device);

/* The library's 2-bit packing (host): code j of `codes` goes to bits 2(j mod 16) and
 * 2(j mod 16)+1 of words[j / 16], least significant first -- the ordering of the
 * 32-character register in Fig. 2. words: ceil(count/16) entries, fully written (the
 * unused high bits of the last word are 0). Codes above 3 give FM_EINVAL. */
int fm_pack_host(const uint8_t *codes, uint64_t count, uint32_t *words);

/* Writes an index file for text (host, n codes 0..3): header, C, '$' row and the
 * packed BWT of R$ (and of reverse(R)$ when flags has FM_LOAD_REVERSE). */
int fm_index_build_file(const uint8_t *text, uint64_t n, const char *path, uint32_t flags);

/* Builds the index of text (host) in memory and moves it to the device. */
int fm_index_from_text(const uint8_t *text, uint64_t n, const fm_load_opts *opts, fm_index **out);

/* Index from a BWT given directly (host): rows = n+1 codes 0..3 with exactly one 4 for
 * '$'. rev_bwt (nullable) is the BWT of reverse(R)$ with the same number of rows.
 * FM_EFORMAT when a BWT does not hold exactly one '$' or the two disagree in size. */
int fm_index_from_codes(const uint8_t *bwt, uint64_t rows, const uint8_t *rev_bwt,
                        const fm_load_opts *opts, fm_index **out);

/* Loads an index file written by fm_index_build_file: the packed BWT of R$ (Eq. 2) and,
 * if the file has it, of reverse(R)$, with n, C (Background, Fig. 1) and the '$' rows.
 * The file is read and checked on the host before any device work: FM_EIO when it
 * cannot be opened, FM_EFORMAT for a bad magic or version, a truncated or oversized body,
 * sizes that disagree, a checksum (over header and body) that does not match, or C or a
 * '$' row that disagrees with the symbol counts of the packed BWT; FM_EINVAL when
 * FM_LOAD_REVERSE is asked of a file without a reverse index, or dev_buf is given but
 * misaligned, on another device or smaller than fm_index_required_bytes. Files hold no
 * SA samples, so FM_LOAD_LOCATE has no effect here. */
int fm_index_load(const char *path, const fm_load_opts *opts, fm_index **out);

/* Device bytes an index over n symbols keeps when built with opts (fm_index_from_text,
 * _codes or _load): the layouts (the one named by occ_interval, or all of them with
 * FM_LOAD_ALL_LAYOUTS) of R and, with FM_LOAD_REVERSE, of reverse(R); the prefix table
 * of R: for t = 1..T the Listing 1 interval (k, l) of every string of length t over ACGT,
 * 8 bytes each, with T = min(14, floor(log4(n + 1)) - 1) (none when that is below 1); and
 * with FM_LOAD_LOCATE the SA samples of fm_index_from_text (4 bytes per 32 rows); each
 * piece is 256-byte aligned. This is the smallest dev_buf_bytes accepted. Host only; FM_EINVAL
 * for an unsupported occ_interval, FM_ERANGE when n + 1 >= 2^32. */
int fm_index_bytes(uint64_t n, const fm_load_opts *opts, size_t *bytes);

/* fm_index_bytes for the index fm_index_load(path, opts) would create, with n and the
 * presence of a reverse index read from the file's header (FM_LOAD_LOCATE ignored).
 * Reads only the header: FM_EIO, FM_EFORMAT (bad magic or sizes), FM_EINVAL as for
 * fm_index_load. Host only. */
int fm_index_required_bytes(const char *path, const fm_load_opts *opts, size_t *bytes);

int fm_index_info(const fm_index *idx, fm_info *out);

/* Frees the index's device memory; safe on NULL. No call may be in flight on it. */
void fm_index_free(fm_index *idx);

/* ----------------------------------------------------------------- tuning */

/* Current launch configuration of op (FM_OP_*). Defaults are chosen at load time. */
int fm_get_tuning(const fm_index *idx, int op, fm_tuning *out);

/* Sets the launch configuration of op. FM_EINVAL when a value is outside the listed
 * ones or the layout was not built. Not safe concurrently with searches on idx. */
int fm_set_tuning(fm_index *idx, int op, const fm_tuning *t);

/* Times every compiled launch configuration of op (layout, lanes, depth, waves per CU;
 * for the substitution DFS also the claim order and the prefix table on or off) on a
 * sample batch (same arguments as the corresponding search, device buffers owned by the
 * caller, ws sized with the op's workspace call for the sample and hit_cap) and keeps the
 * fastest that
 * reproduces the plain kernel's output bit for bit (a candidate replaces the current
 * choice only when it is at least 1% faster, so settings within timing noise of each
 * other resolve to the one tried first). Synchronises `stream`. If
 * cache_path is non-NULL the choice is looked up there first (key: device
 * architecture, n, read count, total length, zmax, flags) and stored after tuning.
 * With FM_TUNE_KEEP_LAYOUT in flags only the depth, waves per CU, claim order and prefix
 * table are searched, at the current layout and lanes: a coarse tuning on a sample can
 * then be refined on a batch of the real size, where the launch's tail weighs less and
 * the best occupancy can differ.
 * best (nullable) receives the choice; ms (nullable) its time per call. */
int fm_autotune(fm_index *idx, int op, const uint8_t *codes, const uint64_t *offs,
                const uint8_t *z, uint64_t nreads, uint32_t flags, uint32_t zmax,
                void *out_buf, uint64_t hit_cap, uint64_t *hit_offs, uint32_t *status,
                void *ws, size_t ws_bytes, const char *cache_path, void *stream,
                fm_tuning *best, float *ms);

/* ----------------------------------------------------------------- Occ8 */

/* For each query (k, l), 0 <= k <= n+1 and 0 <= l <= n, writes the eight values
 *   Occ(A,k-1) Occ(C,k-1) Occ(G,k-1) Occ(T,k-1) Occ(A,l) Occ(C,l) Occ(G,l) Occ(T,l)
 * -- everything one step of the inexact match consumes (Background). q: device, nq
 * pairs. out: device, 8*nq uint32. A query outside the ranges gets eight 0xFFFFFFFF
 * (no Occ value can be that large). */
int fm_occ8(const fm_index *idx, const fm_interval *q, uint64_t nq, uint32_t *out, void *stream);

/* Diagnostic: the memory system's ceiling for the searches' access pattern. One launch on
 * idx's device (16 waves per compute unit, 4 reads in flight per lane, `rounds` rounds)
 * in which every lane reads random 32-byte blocks of buf[0 .. span): one 32-byte bucket
 * is what an Occ8 reads at I=64 (Background), and a bucket fetch is a read of a random
 * block of the index. Timing the call over a span about the size of the index gives the
 * rate of independent bucket fetches the device can serve there. buf: device, at least
 * span bytes, 16-byte aligned, read only. span: a power of two, at least 4096. rounds:
 * 1..4096. sink: device, one uint32, written only if a lane's sum of the words it read
 * equals a fixed constant (it keeps the loads live). *reads (host) receives the number of
 * 32-byte reads the launch makes. FM_EINVAL for other arguments, FM_EDEVICE if the launch
 * fails. */
int fm_probe_random_reads(const fm_index *idx, const void *buf, uint64_t span, uint32_t rounds,
                          uint32_t *sink, uint64_t *reads, void *stream);

/* ----------------------------------------------------------------- exact search */

/* Workspace bytes fm_search_exact needs (256; also with FM_PLAIN, where ws may be NULL
 * unless FM_STATS is set). With FM_STATS the uint64s at byte offsets 80 and 88 of ws
 * count the search steps that fetched and the buckets they fetched. */
int fm_search_exact_workspace(const fm_index *idx, uint64_t nreads, uint32_t flags, size_t *bytes);

/* Backward exact match (Listing 1) of every read on the strands in flags.
 * codes: device, offs[nreads] bytes (reads concatenated). offs: device, nreads+1
 * uint64 CSR offsets, offs[0] = 0. out: device, one fm_interval per read and strand,
 * out[s_count * r + j] for the j-th requested strand. ws: device workspace (may be
 * NULL with FM_PLAIN and no FM_STATS). An empty read gives (0, n); a miss or a non-ACGT symbol gives
 * (1, 0). Reads may have any length below 2^32.
 * With FM_FULL_RANK the search takes every step of Listing 1 even after the interval is
 * empty, and reports it as it ends: (k, l) with k = the number of suffixes of R$ smaller
 * than the pattern and l = k - 1 + its occurrences, so a miss gives its insertion rank
 * (k, k - 1). A non-ACGT symbol ranks above T (C = n for it, no occurrences). */
int fm_search_exact(const fm_index *idx, const uint8_t *codes, const uint64_t *offs,
                    uint64_t nreads, uint32_t flags, fm_interval *out, void *ws,
                    size_t ws_bytes, void *stream);

/* ----------------------------------------------------------------- D-array */

/* BWA's lower bound D (used by FM_DARRAY): for each read and requested strand, D[i] is
 * the number of disjoint segments of the strand's pattern W[0..i] that do not occur in
 * R, found by a left-to-right walk over the index of reverse(R) that restarts after
 * each failure (values saturate at 255). total_len: host copy of offs[nreads].
 * D: device, s_count * total_len bytes, the strand-0 block first, each laid out like
 * `codes`. Needs FM_LOAD_REVERSE. Runs the plain (one thread per read-strand) walk. */
int fm_darray(const fm_index *idx, const uint8_t *codes, const uint64_t *offs,
              uint64_t nreads, uint64_t total_len, uint32_t flags, uint8_t *D, void *stream);

/* ----------------------------------------------------------------- inexact search */

/* Workspace bytes fm_search_inexact needs for this batch shape. */
int fm_search_inexact_workspace(const fm_index *idx, uint64_t nreads, uint64_t total_len,
                                uint32_t flags, uint32_t zmax, uint64_t hit_cap, size_t *bytes);

/* Inexact match restricted to substitutions (Listing 2): for every read r and
 * requested strand, every W' over ACGT of the read's length with at most z[r]
 * substitutions (non-ACGT positions always count) that occurs in R, reported once
 * as (read, k, l, strand, nmm). With FM_DARRAY the search is pruned with the D bound,
 * which never changes the result.
 * With FM_GAPS the search takes every branch of Listing 2: besides the substitution of
 * pattern symbol i it may skip it (a deletion) or insert any symbol before it, each
 * costing 1; the recursion stops once the first pattern symbol is consumed, so nothing
 * is inserted before it. Every interval reached is reported once, with the smallest
 * number of edits nmm; hits are sorted by (strand, k, l), and the D bound (a lower bound
 * on edits too) still never changes the result. The count at byte offset 8 of ws counts
 * hits before this merging, an upper bound for a retry.
 *   z: device, nreads uint8 budgets; zmax: host, an upper bound on them (<= FM_ZMAX);
 *      a read with z[r] > zmax gets status FM_EINVAL and no hits.
 *   hits: device, hit_cap entries; hit_offs: device, nreads+1 uint64: the hits of
 *      read r are hits[hit_offs[r] .. hit_offs[r+1]) sorted by (strand, k) (and l).
 *   status: device, nreads uint32: FM_OK, FM_EINVAL, FM_ERANGE (read longer than
 *      65535), FM_EOVERFLOW (hits did not fit in hit_cap; the read has no hits
 *      listed) or FM_EBUDGET (node budget reached; no hits listed).
 *   ws: device workspace of at least fm_search_inexact_workspace bytes. After the
 *      call, the uint64 at byte offset 8 of ws holds the total hit count every read
 *      would need (for a retry with a larger hit_cap); with FM_STATS the uint64s at
 *      offsets 64 (expanded DFS nodes, each one Occ8 step), 72 (buckets fetched by
 *      them; a node whose interval is still (0, n) takes its children from C and
 *      fetches none), 80 (D-walk steps that fetched) and 88 (buckets they fetched)
 *      count the work done, 96 the subtrees that idle lanes of the batched DFS took
 *      over from busy ones at the end of the launch (one lane per read-strand; zmax >= 2,
 *      or zmax 1 in batches of fewer than 512 read-strands per compute unit),
 *      and 104 the expanded nodes whose children came from the prefix table (they fetch
 *      no bucket; see fm_tuning.table_depth).
 * Output is deterministic (independent of scheduling, batch order and launch tuning)
 * whenever hit_cap suffices. When it does not, hits beyond the per-read-strand slots
 * compete for hit_cap places in arrival order, so which reads end FM_EOVERFLOW can vary
 * from call to call; every read listed FM_OK still has all its hits, and the required
 * total at byte offset 8 of ws is exact. */
int fm_search_inexact(const fm_index *idx, const uint8_t *codes, const uint64_t *offs,
                      const uint8_t *z, uint64_t nreads, uint32_t flags, uint32_t zmax,
                      fm_hit *hits, uint64_t hit_cap, uint64_t *hit_offs, uint32_t *status,
                      void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): fm_search_inexact with its workspace in
 * a static device array of FM_NOALLOC_WS_BYTES bytes that the library keeps on each device
 * it runs on until the process ends, so the call takes no ws argument and allocates
 * nothing. Arguments, results and errors are fm_search_inexact's, except: FM_ERANGE when
 * the batch's workspace (fm_search_inexact_workspace) exceeds FM_NOALLOC_WS_BYTES (about
 * 140 bytes per read-strand plus 16 per read and 16 per hit_cap entry); FM_EINVAL with
 * FM_STATS (the counts would stay in the array). required (nullable, device, one uint64)
 * receives the total hit count every read would need, as fm_search_inexact leaves it at
 * byte offset 8 of ws. Every call on a device uses that device's one array, which keeps
 * the last call's contents (each call clears what it needs), so calls that overlap on one
 * device -- on different streams, or from different host threads -- race and must not be
 * made; calls on one stream are ordered and safe. */
#define FM_NOALLOC_WS_BYTES (64u << 20)
int fm_search_inexact_noalloc(const fm_index *idx, const uint8_t *codes, const uint64_t *offs,
                              const uint8_t *z, uint64_t nreads, uint32_t flags, uint32_t zmax,
                              fm_hit *hits, uint64_t hit_cap, uint64_t *hit_offs, uint32_t *status,
                              uint64_t *required, void *stream);

/* Both searches of one batch: exactly the results of fm_search_exact(codes, offs, nreads,
 * exact_flags, intervals) and of fm_search_inexact(codes, offs, z, nreads, flags, zmax,
 * hits, hit_cap, hit_offs, status, ws, ws_bytes), bit for bit. When every strand of
 * exact_flags is also searched by the inexact search, the exact intervals come out of
 * its DFS (Listing 2): the branch that matches every symbol is Listing 1's backward
 * search with the same interval updates, so a read-strand's exact interval is its hit
 * with no substitution, or the miss (1, 0) when the DFS ends without one; a read-strand
 * whose DFS stops early (FM_EINVAL, FM_ERANGE, FM_EBUDGET) finishes that branch alone,
 * so its interval is still exact. Otherwise, and with FM_PLAIN, the two searches run one
 * after the other. Arguments and errors are those of the two calls; ws is sized by
 * fm_search_inexact_workspace. exact_flags: FM_FWD/FM_REVCOMP, and FM_FULL_RANK, which
 * also makes the two searches separate (FM_STATS and FM_PLAIN are taken from flags). */
int fm_search_both(const fm_index *idx, const uint8_t *codes, const uint64_t *offs, const uint8_t *z,
                   uint64_t nreads, uint32_t exact_flags, uint32_t flags, uint32_t zmax,
                   fm_interval *intervals, fm_hit *hits, uint64_t hit_cap, uint64_t *hit_offs,
                   uint32_t *status, void *ws, size_t ws_bytes, void *stream);

/* ----------------------------------------------------------------- locate */

/* Workspace bytes fm_locate needs for niv intervals. */
int fm_locate_workspace(const fm_index *idx, uint64_t niv, size_t *bytes);

/* Text positions of the rows of SA intervals (Background, Eq. 4-5): pos holds SA[k_j + t]
 * for every interval j and t = 0 .. l_j - k_j, intervals in order. Only the SA values of
 * rows that are multiples of 32 are kept; any other row k is walked with
 * Psi^-1(i) = C[BWT[i]] + Occ(BWT[i], i) until it reaches a kept row (or the '$' row,
 * whose SA value is 0), and SA[k] is that value plus the number of steps. Needs an index
 * built by fm_index_from_text with FM_LOAD_LOCATE (FM_EINVAL otherwise).
 *   kl: device, niv intervals; interval j is (kl[j*stride], kl[j*stride+1]) as uint32
 *      (stride >= 2: 2 for an fm_interval array; an fm_hit array passes &hits[0].k and
 *      stride 4). Intervals with k > l or l > n hold no rows (misses such as (1, 0)).
 *   offs: device, niv+1 uint64, written: offs[j] = rows of the intervals before j, so the
 *      rows of interval j go to pos[offs[j] ..]; offs[niv] = total rows.
 *   pos: device, pos_cap uint32 (pos_cap <= 2^31). Only the first min(pos_cap, total)
 *      rows are located; call with pos_cap = 0 to size pos from offs[niv] first.
 *   flags: FM_STATS counts the Psi^-1 steps into the uint64 at byte offset 80 of ws.
 *   ws: device workspace of fm_locate_workspace bytes.
 * Uses the forward layout and launch settings of FM_OP_LOCATE. Asynchronous on stream. */
int fm_locate(const fm_index *idx, const uint32_t *kl, uint64_t niv, uint32_t stride, uint64_t *offs,
              uint32_t *pos, uint64_t pos_cap, uint32_t flags, void *ws, size_t ws_bytes, void *stream);

/* ----------------------------------------------------------------- phase timing */

/* Diagnostics. With capacity > 0, every later search call on idx records HIP events on
 * its stream at its phase boundaries (the first `capacity` calls are kept); capacity 0
 * turns this off. Not for concurrent use. A plan captured meanwhile records events of its
 * own instead (fm_plan_phase_times); its replays are not recorded here. */
int fm_phase_timing(fm_index *idx, uint32_t capacity);

/* Waits for the recorded events and writes the milliseconds spent per phase, summed
 * over the recorded calls: ms[0] exact walk, ms[1] D walk, ms[2] DFS kernel, ms[3]
 * compaction; *calls (nullable) gets the number of calls. Clears the record. */
int fm_phase_times(fm_index *idx, float ms[4], uint32_t *calls);

/* ----------------------------------------------------------------- launch graphs */

typedef struct fm_plan fm_plan;

/* Captures one call of an operation into a HIP graph for a fixed batch shape and fixed
 * buffers (all pointers as in the search calls, op = FM_OP_EXACT or FM_OP_INEXACT).
 * Replaying it searches whatever the buffers hold at replay time. Capture runs on an
 * internal stream; nothing is executed. */
int fm_plan_create(const fm_index *idx, int op, const uint8_t *codes, const uint64_t *offs,
                   const uint8_t *z, uint64_t nreads, uint32_t flags, uint32_t zmax,
                   void *out_buf, uint64_t hit_cap, uint64_t *hit_offs, uint32_t *status,
                   void *ws, size_t ws_bytes, fm_plan **out);

/* A plan capturing one fm_search_both call (arguments as there). */
int fm_plan_create_both(const fm_index *idx, const uint8_t *codes, const uint64_t *offs, const uint8_t *z,
                        uint64_t nreads, uint32_t exact_flags, uint32_t flags, uint32_t zmax,
                        fm_interval *intervals, fm_hit *hits, uint64_t hit_cap, uint64_t *hit_offs,
                        uint32_t *status, void *ws, size_t ws_bytes, fm_plan **out);

/* Enqueues one replay of the plan on stream. */
int fm_plan_launch(fm_plan *plan, void *stream);

/* A plan created while the index's phase timing (fm_phase_timing) is on records HIP events
 * of its own at the phase boundaries of every replay, on the stream it is replayed on.
 * This waits for the last replay's events and writes its milliseconds per phase as
 * fm_phase_times does (ms[0] exact walk, ms[1] D walk and claim order, ms[2] DFS kernel,
 * ms[3] compaction; 0 for phases the plan does not have). FM_EINVAL for a plan created
 * without phase timing. A replay still queued when this is called is waited for; the
 * events of earlier replays are overwritten by later ones. */
int fm_plan_phase_times(fm_plan *plan, float ms[4]);

void fm_plan_free(fm_plan *plan);

/* ----------------------------------------------------------------- serving */

/* A request server over fm_search_inexact with continuous batching. Submitted
 * requests (reads with per-read budgets) wait in arrival order. A worker thread keeps
 * up to `lanes` batches on the device at once, each on a stream of its own with an
 * equal share of a device arena allocated at creation. Whenever a lane is idle it
 * admits waiting requests, oldest first, while the batch's memory (fm_server_bytes)
 * still fits the lane's share and the batch stays within max_batch_reads; requests
 * that arrive while batches run therefore join the next batch of the first lane to
 * free up, and their work overlaps with the batches already running. A batch whose
 * hits exceed the reserve is searched again with room for all of them. Each read is
 * searched independently of the rest of its batch, so a request gets the same bytes
 * whatever it is batched with. The index must outlive the server, and its phase
 * timing must stay off while the server runs. */
typedef struct fm_server fm_server;

typedef struct {
    uint32_t lanes;                 /* batches in flight at once, 1..8 */
    uint32_t flags;                 /* search flags for every request: strands, FM_DARRAY */
    uint32_t zmax;                  /* largest budget a request may carry, <= FM_ZMAX */
    uint32_t hit_reserve;           /* hits reserved per read-strand when admitting */
    uint64_t arena_bytes;           /* device memory for batches in flight (split evenly
                                       among lanes; the same again is pinned on the host) */
    uint64_t max_batch_reads;       /* reads per batch; 0 = only memory limits a batch */
    uint64_t ring_bytes;            /* pinned host ring holding the symbols of queued requests
                                       until their upload; 0 = arena_bytes */
} fm_server_opts;

typedef struct {
    uint64_t nreads;
    const fm_hit *hits;             /* host; hits[i].read counts reads within the request */
    uint64_t nhits;
    const uint64_t *hit_offs;       /* host, nreads + 1, as in fm_search_inexact */
    const uint32_t *status;         /* host, nreads, as in fm_search_inexact */
    int error;                      /* FM_OK, or why the request as a whole failed */
    double t_submit, t_launch, t_done;  /* seconds on the server clock: submitted, its batch
                                       launched, results in host memory */
    uint64_t batch;                 /* number of the batch that served it (from 1) */
} fm_result;

typedef struct {
    uint64_t batches, retries, requests_done, reads_done, pending;
    int error;                      /* first device error seen, FM_OK if none */
} fm_server_counts;

/* Device bytes a batch of nreads reads with total_len symbols takes under opts: the
 * inputs, status, hit offsets, search workspace and hit_reserve hits per read-strand,
 * each 256-byte aligned. This is the admission rule. Host only. */
int fm_server_bytes(const fm_server_opts *opts, uint64_t nreads, uint64_t total_len, uint64_t *bytes);

/* Creates the server and starts its worker. FM_EINVAL for options outside the listed
 * ranges (or FM_DARRAY without a reverse index), FM_ENOMEM when the arena or its
 * pinned mirror cannot be allocated. Each lane runs on a stream of its own; a process
 * has few hardware queues (4 by default), and lanes whose streams share a queue with
 * other streams no longer overlap, so create the server before other streams that
 * stay alive. */
int fm_server_create(const fm_index *idx, const fm_server_opts *opts, fm_server **out);

/* Queues a request: codes (host) with nreads+1 nondecreasing offsets (host, codes of
 * read r at offs[r] .. offs[r+1]) and nreads budgets z (host). The data are copied
 * before the call returns (the symbols into the server's pinned ring, waiting while
 * the ring is full of requests not yet uploaded). *ticket names the request.
 * FM_ERANGE if the request alone does not fit a lane or the ring. Thread-safe. */
int fm_server_submit(fm_server *s, const uint8_t *codes, const uint64_t *offs, const uint8_t *z,
                     uint64_t nreads, uint64_t *ticket);

/* Waits up to timeout_s seconds (negative: without limit) for the request to finish
 * and describes its results; the pointers stay valid until fm_server_release.
 * FM_EAGAIN if it is still running, FM_EINVAL for an unknown ticket. Thread-safe. */
int fm_server_wait(fm_server *s, uint64_t ticket, double timeout_s, fm_result *out);

/* Frees a finished request's results. */
int fm_server_release(fm_server *s, uint64_t ticket);

/* Seconds since the server was created (the clock of fm_result's times). */
double fm_server_clock(const fm_server *s);

int fm_server_stats(fm_server *s, fm_server_counts *out);

/* Finishes every queued request, stops the worker and frees the arena; safe on NULL.
 * Results not yet released are freed too. */
void fm_server_free(fm_server *s);

#ifdef __cplusplus
}
#endif

#endif /* FM_H */
