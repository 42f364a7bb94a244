/*
 * Plain CPU brute force for exact top-k LCP retrieval.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test-suite (parity at sizes the NumPy
 * oracle is too slow for) and by the benchmark's CPU-baseline leg.  The
 * product library never links or calls it, and it shares no code with the GPU
 * implementation.
 *
 * What it computes, straight from the definitions of section 2.1:
 *   - LCP(q, s) = number of leading positions where q and s carry the same
 *     token, found by comparing token after token (Definition "LCP
 *     Similarity");
 *   - for every query, the k rows of highest LCP, ties going to the lower
 *     0-based id, listed in rank order (LCP descending, id ascending), the
 *     tail padded with (-1, -1) when k > N (Definition "Top-k LCP Retrieval").
 *
 * Selection: rows are visited in ascending id order and kept in a list sorted
 * by rank.  A row enters when the list is not yet full or when its LCP beats
 * the LCP of the last kept row; it is placed after every kept row with an LCP
 * greater than or equal to its own.  Because every earlier row has a smaller
 * id, a row whose LCP only equals the last kept LCP ranks below all of them and
 * never enters a full list.
 *
 * Tokens are 1 byte (token_bytes = 1) or 2 bytes (token_bytes = 2), rows are
 * row-major [N][L], ids are row positions.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline uint32_t tok(const void* base, int64_t row, int32_t L, int32_t j, int32_t tb) {
    if (tb == 1) return ((const uint8_t*)base)[row * L + j];
    return ((const uint16_t*)base)[row * L + j];
}

static int32_t lcp_rows(const void* db, int64_t id, const void* qs, int64_t qi, int32_t L, int32_t tb) {
    int32_t j = 0;
    while (j < L && tok(db, id, L, j, tb) == tok(qs, qi, L, j, tb)) ++j;
    return j;
}

static void one_query(const void* db, int64_t N, int32_t L, int32_t tb, const void* qs, int64_t qi,
                      int32_t k, int32_t* ids, int32_t* lcps) {
    int32_t kept = 0;
    for (int64_t id = 0; id < N; ++id) {
        int32_t l = lcp_rows(db, id, qs, qi, L, tb);
        if (kept == k && l <= lcps[k - 1]) continue;
        /* insertion point: after every kept row with LCP >= l */
        int32_t pos = 0;
        while (pos < kept && lcps[pos] >= l) ++pos;
        int32_t last = (kept < k) ? kept : k - 1;   /* slot that gets overwritten */
        for (int32_t t = last; t > pos; --t) {
            ids[t] = ids[t - 1];
            lcps[t] = lcps[t - 1];
        }
        ids[pos] = (int32_t)id;
        lcps[pos] = l;
        if (kept < k) ++kept;
    }
    for (int32_t t = kept; t < k; ++t) {
        ids[t] = -1;
        lcps[t] = -1;
    }
}

/* Returns 0 on success, -1 on bad arguments. */
int oracle_topk(const void* db, int64_t N, int32_t L, int32_t token_bytes, const void* queries, int64_t Q,
                const int32_t* k, const int64_t* off, int32_t* out_ids, int32_t* out_lcp, int32_t nthreads) {
    if (!db || !queries || !k || !off || !out_ids || !out_lcp) return -1;
    if (N < 1 || L < 1 || Q < 0 || (token_bytes != 1 && token_bytes != 2)) return -1;
    for (int64_t i = 0; i < Q; ++i)
        if (k[i] < 1 || off[i + 1] - off[i] != k[i]) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t i = 0; i < Q; ++i)
        one_query(db, N, L, token_bytes, queries, i, k[i], out_ids + off[i], out_lcp + off[i]);
    return 0;
}

/* Threads an OpenMP parallel region actually gets (1 without OpenMP). */
int oracle_threads(int32_t nthreads) {
#ifdef _OPENMP
    int n = 1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
    return n;
#else
    (void)nthreads;
    return 1;
#endif
}
