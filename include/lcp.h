/*
 * lcp.h - exact top-k retrieval under longest-common-prefix (LCP) similarity
 * on one AMD Instinct MI355X (gfx950).
 *
 * Problem (section 2.1 of the paper, Definitions "LCP Similarity" and
 * "Top-k LCP Retrieval"): a database of N categorical sequences of fixed
 * length L over an alphabet of V symbols; for a query q of the same length,
 * LCP(q, s) is the number of leading positions where q and s agree, and the
 * answer is the k rows of highest LCP with ties broken by index.  This library
 * breaks ties by the LOWER 0-based row id and lists every answer in rank order
 * (LCP descending, id ascending), so results are bit-identical on every run
 * (section 5.3, Theorem "Determinism").
 *
 * Index: instead of the paper's pointer trie (section 5.2, Algorithms 1-2) the
 * rows are kept in lexicographic order (a trie's leaf order; tokens compared
 * as unsigned integers, position 0 most significant, equal rows by ascending
 * id) together with the adjacent-LCP array A[i] = LCP(T[i-1], T[i]), A[0] = 0.
 * A trie node of depth d is a contiguous range of that order, the prefix
 * bucket of section 6.2.  A query is answered by a batched search for its
 * insertion point (the predecessor search of section 4.2), an outward walk
 * over A that finds the cutoff LCP c at which the answer fills up, and a
 * bounded scan of the rows tied at c for the lowest ids (the range-bounded
 * scan of section 6.2 and Appendix D.1).  A plain full scan is provided as
 * the brute-force path.
 *
 * Conventions for every entry point:
 *   - Device pointers are HIP device allocations on the device that was
 *     current when the index was built; host pointers are ordinary memory.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Query
 *     calls only enqueue work; their outputs are valid once the stream has
 *     been synchronised.  Calls on one stream run in order; calls on
 *     different streams may overlap (each stream gets its own scratch).
 *   - Tokens are uint8 when V <= 256 and uint16 (little-endian) otherwise;
 *     token arrays are row-major [rows][L] with no padding between rows.
 *   - Errors are returned as lcp_status codes and never abort; the message of
 *     the calling thread's last failure is available from lcp_last_error().
 */
#ifndef LCP_H_
#define LCP_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lcp_index lcp_index; /* opaque; owns every device buffer of an index */

typedef enum {
    LCP_OK = 0,
    LCP_EINVAL = -1,   /* an argument is out of its documented range */
    LCP_ENOMEM = -2,   /* a device or pinned-host allocation failed */
    LCP_EDEVICE = -3,  /* a HIP runtime call failed */
    LCP_ERANGE = -4,   /* lcp_index_build found a token >= V */
    LCP_ENOTIMPL = -5  /* the request is valid but not supported by this library */
} lcp_status;

#define LCP_L_MAX 255   /* LCP values are stored in one byte */
#define LCP_K_MAX 1024  /* largest k accepted per query */

/*
 * Build an index over N rows (section 5.2, the sorted-order equivalent of
 * Algorithms 1-2: leaf order of the trie with posting lists in id order).
 * Besides the sorted rows, their ids and the adjacent-LCP array the index
 * keeps the top levels of a 65-ary search tree over the sorted rows, the
 * sorted position where each first-token value starts, for
 * every run of 64 sorted positions the smallest id in it (used to skip most
 * of a long run of rows tied at the cutoff LCP), and the first 8 bytes of
 * every row in id order (the stream the full scan reads).  Device memory:
 * about N * (8 * row_words + 13.06) bytes plus at most 4.4 MB of search
 * tables and 4 * (V + 2) bytes of directory; the first lcp_index_append adds a
 * second copy of the order-dependent arrays (N * (4 * row_words + 5.06) bytes
 * and the tables), with room for a quarter more rows.
 *
 *   tokens : device, [N][L] uint8 (V <= 256) or uint16 (V > 256).  The
 *            index copies them; the caller may free `tokens` after return.
 *   N      : 1 <= N <= 2^31 - 2^16 (positions stay 32-bit).
 *   L      : 1 <= L <= LCP_L_MAX.
 *   V      : 1 <= V <= 65536; every token must be < V.
 *   stream : stream the build runs on; the call synchronises it before it
 *            returns, so the index is ready on return.
 *   out    : receives the new handle (set to NULL on failure).
 *
 * Errors: LCP_EINVAL (bad sizes or NULL pointers), LCP_ERANGE (a token >= V;
 * nothing is kept), LCP_ENOMEM, LCP_EDEVICE.
 */
lcp_status lcp_index_build(const void* tokens, int64_t N, int32_t L, int32_t V, void* stream,
                           lcp_index** out);

/*
 * Index path: exact top-k for Q queries (section 2.1 definition; method of
 * sections 4.2, 5.3 and 6.2 on the sorted order).
 *
 *   queries : device, [Q][L], same token width as the index.  Query tokens
 *             are not checked against V: any value compares as an integer.
 *   Q       : 0 <= Q < 2^31 (Q = 0 is a no-op).
 *   k       : HOST array of Q values, 1 <= k[i] <= LCP_K_MAX.  Read during
 *             the call only.
 *   out_ids, out_lcp : device int32 arrays of sum(k) entries.  Query i owns
 *             entries [off_i, off_i + k[i]) with off_i = k[0] + ... + k[i-1];
 *             they hold its answer in rank order (LCP descending, id
 *             ascending).  When k[i] > N the last k[i] - N entries are -1.
 *
 * Errors: LCP_EINVAL (NULL handle or pointers, Q < 0, k out of range),
 * LCP_ENOMEM, LCP_EDEVICE.  Outputs are unspecified after an error.
 */
lcp_status lcp_topk(const lcp_index* index, const void* queries, int64_t Q, const int32_t* k,
                    int32_t* out_ids, int32_t* out_lcp, void* stream);

/*
 * lcp_topk that also reports, per query, the shape of the work the method did
 * (the quantities section 6.2's range-scan cost is stated in, Theorem "Range
 * Scan Complexity"): the answers are those of lcp_topk, and
 *
 *   stats : device int32 [Q][4], 16-byte aligned; query i gets
 *           stats[4i + 0] = c, the cutoff LCP: the largest d with at least
 *                           min(k, N) rows of LCP >= d,
 *           stats[4i + 1] = n_gt, the rows with LCP > c (all in the answer),
 *           stats[4i + 2] = the rows with LCP exactly c (the tied range the
 *                           lowest ids are taken from),
 *           stats[4i + 3] = the tie selection used: 0 none needed, 1 id walk
 *                           (c = 0), 2 wave minima, 3 bisection on id bits,
 *                           4 pruned by per-64-position minima, 5 sorted list.
 * Errors: those of lcp_topk; LCP_EINVAL for a NULL or misaligned stats.
 */
lcp_status lcp_topk_stats(const lcp_index* index, const void* queries, int64_t Q, const int32_t* k,
                          int32_t* out_ids, int32_t* out_lcp, int32_t* stats, void* stream);

/*
 * Plain path: the same answer as lcp_topk computed by brute force (LCP of every
 * query against all N rows, then per-query top-k; the "full scan" the paper
 * compares against in section 7, Table "TAL range-scan vs full-scan").
 * Arguments, output layout and errors are those of lcp_topk.
 */
lcp_status lcp_scan_topk(const lcp_index* index, const void* queries, int64_t Q, const int32_t* k,
                         int32_t* out_ids, int32_t* out_lcp, void* stream);

/*
 * Prefix-bucket range scan (section 6.2: Definition "Prefix Bucket", Theorem
 * "Range Scan Complexity", Definition "Thermal-Aware Logic"; the range scan of
 * Appendix D.1).  Query i scans only its bucket: the rows whose first `depth`
 * tokens equal its own, a contiguous range of the sorted order.  Its answer is
 * the top-k of that bucket alone, by the section 2.1 order (LCP descending,
 * id ascending), with LCP and ids as in lcp_topk; when the bucket holds fewer
 * than k[i] rows (none, if no row has the query's prefix) the remaining
 * entries are -1.  Whenever the k-th best LCP over all rows is at least
 * `depth`, the answer equals lcp_topk's.
 *
 *   depth  : 0 <= depth <= L; 0 makes the bucket every row (a full scan).
 *   bounds : NULL, or device int32 [Q][2], 8-byte aligned: receives each
 *            query's bucket as sorted positions [lo, hi) (positions of the
 *            sorted order that lcp_index_views exposes); lo == hi for an
 *            empty bucket, at the query's insertion point.
 * Other arguments, the output layout and k's range are those of lcp_topk.
 * The first call at a given depth after a build, append or reserve also lays
 * out what that depth streams (the first two key words of the sorted rows, or
 * one key word of them once depth covers whole words: 8 or 4 bytes a row, held
 * by the index) and waits for the device once.
 * Errors: those of lcp_topk; LCP_EINVAL for depth outside [0, L] or a
 * misaligned bounds.
 */
lcp_status lcp_bucket_scan_topk(const lcp_index* index, const void* queries, int64_t Q, int32_t depth,
                                const int32_t* k, int32_t* out_ids, int32_t* out_lcp, int32_t* bounds,
                                void* stream);

/*
 * Device-side variants for callers that keep k and the output offsets on the
 * device (serving loops, captured graphs): no host staging, no host sync.
 *
 *   k_dev   : device int32 [Q], 1 <= k_dev[i] <= k_max (not re-checked on the
 *             device: a value outside that range yields unspecified output
 *             for that query, never a write outside [off_dev[i], off_dev[i+1])).
 *   off_dev : device int64 [Q+1], off_dev[0] = 0, off_dev[i+1] = off_dev[i] + k_dev[i].
 *   k_max   : host upper bound on every k_dev[i]; 1 <= k_max <= LCP_K_MAX.
 * Other arguments as lcp_topk.
 */
lcp_status lcp_topk_dev(const lcp_index* index, const void* queries, int64_t Q, const int32_t* k_dev,
                        const int64_t* off_dev, int32_t k_max, int32_t* out_ids, int32_t* out_lcp,
                        void* stream);
lcp_status lcp_scan_topk_dev(const lcp_index* index, const void* queries, int64_t Q,
                             const int32_t* k_dev, const int64_t* off_dev, int32_t k_max,
                             int32_t* out_ids, int32_t* out_lcp, void* stream);

/*
 * Allocation-free form of lcp_scan_topk_dev, for callers that cannot allocate
 * device memory during a call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  The scan's working memory
 * (partial top-k lists, per-query limits and fill counts, seed histograms,
 * query key words) lives in one fixed array of LCP_NOALLOC_SCRATCH_BYTES that
 * the library's device code holds on each GPU it runs on until the process
 * ends; the call allocates nothing, creates no events and never synchronises.
 * The first call on a device looks up that array's device address once.
 *
 * Arguments, output layout and answers are those of lcp_scan_topk_dev
 * (bit-identical).  Additional limits:
 *   Q : at most 262,140 per call, and small enough that the scratch holds the
 *       partial lists: about Q * k_max * 16 bytes at the least, plus
 *       Q * (L + W + 35) * 4 bytes, must fit in LCP_NOALLOC_SCRATCH_BYTES
 *       (e.g. Q = 8,192 at k_max = 100 fits).  A larger batch is rejected with
 *       LCP_EINVAL before anything is launched; split it into several calls.
 * Concurrency: every call on one GPU shares that GPU's array (the previous
 * call's contents are overwritten; the values that must start at zero are
 * cleared by the call's first kernel).  Calls whose work overlaps on one GPU,
 * on different streams or from different threads, race on the array and give
 * unspecified answers: issue them on one stream, or order them with events.
 */
#define LCP_NOALLOC_SCRATCH_BYTES (32u << 20)
lcp_status lcp_scan_topk_dev_noalloc(const lcp_index* index, const void* queries, int64_t Q,
                                     const int32_t* k_dev, const int64_t* off_dev, int32_t k_max,
                                     int32_t* out_ids, int32_t* out_lcp, void* stream);

/*
 * Append n rows to an index; they get ids N, N+1, ..., N+n-1.  Afterwards the
 * index is identical (sorted order, adjacent LCP, answers) to one built over
 * the concatenated rows.  The paper lists dynamic insertion as future work
 * (section "Limitations"); this is the sorted-order merge: the new rows are
 * sorted, merged into the sorted order after equal old rows (their ids are
 * larger), the adjacent LCP of old rows is carried over and recomputed only
 * where a new row was inserted, and the search tables and tie summaries are
 * rebuilt for the merged order.  The index keeps two copies of the sorted
 * arrays: the merge writes the copy queries do not read, which becomes the
 * one they read only when every step has succeeded, so on any error the index
 * is unchanged.  Buffers grow with room for a quarter more rows; an append
 * that fits allocates nothing, except the first one and appends of more than
 * 8,192 rows (whose temporaries are allocated per call).
 *
 *   tokens : device, [n][L], same width as the index; every token < V.
 *   n      : 0 <= n, N + n <= 2^31 - 2^16 (n = 0 is a no-op).
 *   stream : the call first synchronises every stream the index has been used
 *            on, then runs on `stream` and synchronises it before returning.
 *            No query may run on the index during the call.
 * A successful append moves the arrays queries read and changes N, so a HIP
 * graph captured before it (lcp_topk_persistent) must not be replayed after
 * it: compare lcp_index_generation before replaying.
 * Errors: LCP_EINVAL, LCP_ERANGE (a token >= V), LCP_ENOMEM, LCP_EDEVICE; the
 * index is unchanged after any of them.
 */
lcp_status lcp_index_append(lcp_index* index, const void* tokens, int64_t n, void* stream);

/*
 * Room for `rows` rows in total (N included) for later appends: the id-order
 * rows, both copies of the sorted arrays and the append temporaries are grown
 * now, so that appends of at most 8,192 rows each, up to that total, allocate
 * nothing (for callers that append from a paced loop).  The arrays queries
 * read may move: the generation advances (see lcp_index_generation).
 *   rows   : 0 <= rows <= 2^31 - 2^16; rows <= N only prepares the second copy.
 *   stream : runs the copies; synchronised before the call returns, as is
 *            every stream the index has been used on.
 * Errors: LCP_EINVAL, LCP_ENOMEM, LCP_EDEVICE (the index stays usable).
 */
lcp_status lcp_index_reserve(lcp_index* index, int64_t rows, void* stream);

/*
 * Graph-capturable form of lcp_topk_dev for batches of uneven size and k:
 * the batch size is read on the device, so a HIP graph captured once replays
 * for any batch up to the capacity of the buffers it was captured with.  The
 * launch has `blocks` workgroups of 4 waves; wave w answers query w, and when
 * the grid has fewer waves than the batch has queries, waves then take
 * further queries from a device work counter (the persistent form).  Answers
 * are those of lcp_topk_dev (bit-identical; which wave answers a query does
 * not reach the output).
 *
 *   q_capacity  : largest batch size any launch of this call (or of a graph
 *                 captured from it) may see; 1 <= q_capacity < 2^31.  The
 *                 queries, k_dev, off_dev and output buffers hold that many.
 *   q_count_dev : device int64, number of queries of this launch
 *                 (0..q_capacity).
 *   k_dev, off_dev, k_max : as lcp_topk_dev (k_max bounds every k of any
 *                 batch replayed through a captured graph).
 *   blocks      : <= 0 picks ceil(q_capacity / 4), one wave per query and no
 *                 work counter; fewer blocks make waves loop over queries.
 * Capture: make one call on the stream first (it sets up the stream's work
 * counter); the call itself then allocates nothing and never synchronises.
 * A graph captured from this call holds the index's arrays and N as they were
 * at capture: after lcp_index_append it must be captured again (see
 * lcp_index_generation).
 */
lcp_status lcp_topk_persistent(const lcp_index* index, const void* queries, int64_t q_capacity,
                               const int64_t* q_count_dev, const int32_t* k_dev, const int64_t* off_dev,
                               int32_t k_max, int32_t* out_ids, int32_t* out_lcp, int32_t blocks, void* stream);

/*
 * Number of changes to what queries read since the build (0 after it): each
 * successful lcp_index_append and lcp_index_reserve, and each
 * lcp_index_set_search that switches the mode, adds one.  A HIP graph captured while it had one value must not be
 * replayed once it has another.  Errors: LCP_EINVAL for a NULL argument.
 */
lcp_status lcp_index_generation(const lcp_index* index, uint64_t* generation);

/*
 * How the index path finds a query's insertion point (both give the same
 * answers; this only changes the work):
 *   mode 0: a static 65-ary search whose top three levels come from
 *          the search tables (each step compares the query with 64 pivots'
 *          first 16 bytes in one coalesced load).
 *   mode 1: the first-token directory, a table of V + 2 sorted positions
 *          giving the range of rows that share the query's first token (the
 *          prefix bucket of depth one, section 6.2, Definitions "Prefix
 *          Bucket" and "Thermal-Aware Logic"); the 65-ary search then runs
 *          over that range on the rows themselves.
 * The build picks the one with fewer dependent steps for rows like the
 * database's (the directory costs one lookup and then the steps over the
 * query's first-token bucket; ties keep the tables); this call overrides it.
 * The call synchronises every stream the index has been used on.
 * Errors: LCP_EINVAL (NULL index, mode not 0 or 1), LCP_EDEVICE.
 */
lcp_status lcp_index_set_search(lcp_index* index, int32_t mode);
/* The search in use (0 or 1).  Errors: LCP_EINVAL for a NULL argument. */
lcp_status lcp_index_search_mode(const lcp_index* index, int32_t* mode);

/* Synchronise every stream the index has been used on, then free it.  NULL is a no-op. */
void lcp_index_free(lcp_index* index);

/* Message of the calling thread's most recent failed call ("" if none).  The
 * pointer stays valid until the thread's next failing call. */
const char* lcp_last_error(void);

/*
 * Introspection (tests, tooling).  Any output pointer may be NULL.
 *   token_bytes : 1 or 2.   row_words : 32-bit words per stored row.
 */
lcp_status lcp_index_info(const lcp_index* index, int64_t* N, int32_t* L, int32_t* V,
                          int32_t* token_bytes, int32_t* row_words);

/*
 * Read-only device views owned by the index (valid until lcp_index_free):
 *   perm        : int32 [N], perm[i] = id of the i-th row in sorted order.
 *   adj_lcp     : uint8 [N], A[i] = LCP(T[i-1], T[i]), A[0] = 0.
 *   sorted_keys : uint32 [N][row_words], sorted rows in key form (tokens
 *                 packed big-end first into 32-bit words, zero padded).
 *   id_keys     : uint32 [N][row_words], the same rows in id order.
 */
lcp_status lcp_index_views(const lcp_index* index, const int32_t** perm, const uint8_t** adj_lcp,
                           const uint32_t** sorted_keys, const uint32_t** id_keys);

/*
 * How lcp_scan_topk would split a batch of Q queries with largest k = k_max:
 *   query_groups : passes over the database (each group streams all rows once)
 *   chunks       : row chunks per pass
 *   seed_rows    : leading rows whose LCP histogram gives every query a
 *                  starting limit before the pass
 * Any output pointer may be NULL.
 */
lcp_status lcp_scan_info(const lcp_index* index, int64_t Q, int32_t k_max, int32_t* query_groups,
                         int32_t* chunks, int64_t* seed_rows);

/*
 * Kernel timing for benchmarks: when enabled, each query call records HIP
 * events on its stream around its main kernel (the fused index-path kernel or
 * the scan kernel).  lcp_kernel_time synchronises those events and returns
 * the summed milliseconds and launch count since the last reset.
 *   which : 0 = index-path kernel, 1 = the scan's main kernel (one pass of
 *           the rows per query group; not the seed-limit kernels before it),
 *           2 = scan merge kernel.
 */
lcp_status lcp_set_kernel_timing(const lcp_index* index, int32_t enable);
lcp_status lcp_kernel_time(const lcp_index* index, int32_t which, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* LCP_H_ */
