// Host-side launchers of the library's kernels (defined next to the kernels).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"

namespace lcpx {

// ---- build
hipError_t launch_pack(const void* tokens, int64_t N, RowGeo g, uint32_t V, int dbits, int Wd, uint32_t* keys,
                       uint32_t* dense, uint32_t* bad, hipStream_t s);
hipError_t launch_varying_bits(const uint32_t* dense, int64_t N, int Wd, uint32_t* vary, hipStream_t s);
int radix_tiles(int64_t N);
size_t radix_counts_words(int64_t N);  // counts + block sums for one radix pass
hipError_t launch_iota(int32_t* p, int64_t N, hipStream_t s);
hipError_t launch_gather_word(const uint32_t* dense, const int32_t* perm, int64_t N, int Wd, int d, uint32_t* keys,
                              hipStream_t s);
hipError_t launch_radix_pass(const uint32_t* keys_in, const int32_t* vals_in, int64_t N, int shift, uint32_t* counts,
                             uint32_t* keys_out, int32_t* vals_out, bool write_keys, hipStream_t s);
hipError_t launch_gather_rows(const uint32_t* keys, const int32_t* perm, int64_t N, int W, uint32_t* sorted,
                              hipStream_t s);
hipError_t launch_adjacent_lcp(const uint32_t* sorted, int64_t N, RowGeo g, uint8_t* A, hipStream_t s);

// ub[j] = number of rows of `sorted` (N rows) that are <= row j of `newrows` (n rows, sorted)
hipError_t launch_upper_bounds(const uint32_t* sorted, int64_t N, const uint32_t* newrows, int64_t n, RowGeo g,
                               int64_t* ub, hipStream_t s);
// merge two sorted row sets (old first on ties); new ids are N + newperm[j];
// the adjacent LCP of old rows is carried over and recomputed where new rows
// were inserted
hipError_t launch_merge_sorted(const uint32_t* sorted, const int32_t* perm, const uint8_t* A, int64_t N,
                               const uint32_t* newrows, const int32_t* newperm, const int64_t* ub, int64_t n, RowGeo g,
                               uint32_t* out_sorted, int32_t* out_perm, uint8_t* out_A, hipStream_t s);
// key-form rows of n token rows (flag set on a token >= V), and their stable
// order by rank (small n)
hipError_t launch_pack_keys(const void* tokens, int64_t n, RowGeo g, uint32_t V, uint32_t* keys, uint32_t* bad,
                            uint32_t mark, hipStream_t s);
// after an append's merge, in one launch: search tables (levels > 0), tie
// summaries and first-token directory of the merged copy (M rows), and plane
// entries [from, plane_entries(M))
hipError_t launch_append_tail(const int32_t* perm, const uint32_t* sorted, int64_t M, RowGeo g, int V,
                              const uint32_t* rows, int64_t from, uint32_t* bmin, uint32_t* dir, uint64_t* plane,
                              int levels, uint4* stab, hipStream_t s);
// rank sort of n <= 8,192 new rows and their upper bounds among the N old sorted rows, one wave per new row
hipError_t launch_rank_ub(const uint32_t* keys, int64_t n, const uint32_t* old_sorted, int64_t N, int W,
                          uint32_t* sorted, int32_t* lperm, int64_t* ub, hipStream_t s);
hipError_t launch_search_tables(const uint32_t* sorted, int64_t N, int W, int levels, uint4* stab,
                                hipStream_t s);

// scan prefix plane: key words 0 (high half) and 1 of each row as one 64-bit
// value, id order, padded with a zero entry to an even length
__host__ __device__ inline int64_t plane_entries(int64_t N) { return (N + 1) & ~(int64_t)1; }
// entries [from, plane_entries(to)) of the plane of rows [0, to)
hipError_t launch_prefix_plane(const uint32_t* rows, int64_t from, int64_t to, int W, uint64_t* plane, hipStream_t s);

// first-token directory: dir[t] = the first sorted position whose first token
// is >= t, for t < V, and dir[V] = dir[V + 1] = N (the prefix buckets of
// depth one)
hipError_t launch_first_token_dir(const uint32_t* sorted, int64_t N, RowGeo g, int V, uint32_t* dir, hipStream_t s);

// tie summaries: smallest id of each run of 64 sorted positions
inline int64_t block_min_entries(int64_t N) { return (N + kWave - 1) / kWave; }
hipError_t launch_block_min(const int32_t* perm, int64_t N, uint32_t* bmin, hipStream_t s);

// ---- queries
// Largest index: positions, and the A window reads up to kAdjPad past the
// end, stay below 2^31, so the query kernels keep positions in 32 bits.
constexpr int64_t kMaxRows = ((int64_t)1 << 31) - ((int64_t)1 << 16);
constexpr int kAdjWindow = 1024;                  // bytes of A one query wave stages in LDS
constexpr size_t kAdjPad = kAdjWindow + 64;       // zero bytes allocated past A[N-1]

// Search tables: the top `levels` levels of the static 65-ary search tree over
// [0, N).  A node with range [lo, hi), n = hi - lo > 64, has pivots
// lo + (i+1)*n/65 (i < 64) and children [lo, p0), [p0+1, p1), ..., [p63+1, hi).
// Level d holds 65^d nodes of 64 entries starting at entry 65^d - 1; an entry
// is the pivot row's first four key words (zero past the row's end).
constexpr int kSearchTableMaxLevels = 3;
int search_table_levels(int64_t N);
int64_t search_table_entries(int levels);  // 65^levels - 1

struct IndexView {
    const uint32_t* sorted;  // [N][W] key form, lexicographic order
    const uint32_t* rows;    // [N][W] key form, id order
    const int32_t* perm;     // [N]
    const uint8_t* A;        // [N] adjacent LCP
    const uint4* stab;       // search tables (may be null when levels == 0)
    const uint32_t* bmin;    // [ceil(N/64)] smallest id of each run of 64 sorted positions
    const uint64_t* plane;   // [plane_entries(N)] (word 0 << 32) | word 1 of each row, id order (the scan's stream)
    const uint32_t* dir;     // null, or [dir_V + 2]: the first sorted position whose first token is >= t
    int dir_V;               // first-token values the directory covers (V)
    int stab_levels;
    int64_t N;
    RowGeo g;
};

struct QueryBatch {
    const void* raw;         // [Q][L] raw tokens (tb bytes each)
    int64_t Q;
    const int32_t* k;        // [Q] device (unused when k_uniform > 0)
    const int64_t* off;      // [Q+1] device (unused when k_uniform > 0)
    int32_t k_uniform;       // > 0: every query has this k and query i starts at (q_base + i) * k
    int64_t q_base;          // absolute index of this slice's first query
    int32_t k_max;
    int32_t* out_ids;
    int32_t* out_lcp;
    // index path only, optional: per query of this batch, 4 int32 at stats + 4 * i:
    // cutoff c, inner-group rows n_gt = |G_{c+1}|, tied rows |G_c| - n_gt, and
    // which tie selection ran (a TiePath value)
    int32_t* stats = nullptr;
};

enum TiePath : int32_t {
    kTieNone = 0,    // the inner group fills the answer (no tied rows taken)
    kTieIdWalk = 1,  // c = 0: ids walked in ascending order
    kTieFew = 2,     // at most 16 ids from at most 512 tied rows: wave minima
    kTieSelect = 3,  // at most 256 ids from at most 512 tied rows: bisection on id bits
    kTiePruned = 4,  // long range: pruned by the per-64-position id minima
    kTieList = 5     // the sorted list over every tied row
};

__device__ __forceinline__ int query_k(const QueryBatch& qb, int64_t qi) {
    return qb.k_uniform > 0 ? qb.k_uniform : qb.k[qi];
}
__device__ __forceinline__ int64_t query_off(const QueryBatch& qb, int64_t qi) {
    return qb.k_uniform > 0 ? (qb.q_base + qi) * (int64_t)qb.k_uniform : qb.off[qi];
}

hipError_t launch_index_query(const IndexView& ix, const QueryBatch& qb, hipStream_t s);
// Device-counted forms: `blocks` blocks of 4 waves; the batch size is read
// from q_count (device).  looping = false: one wave per query, blocks*4 must
// cover every batch size the call may see.  looping = true: waves take
// further queries from `counter` (device), reset by a kernel in the same stream.
hipError_t launch_index_query_persistent(const IndexView& ix, const QueryBatch& qb, const int64_t* q_count,
                                         unsigned long long* counter, int blocks, bool looping, hipStream_t s);

// Full scan.  `part` must hold scan_partial_entries(...) keys.
struct ScanPlan {
    int tq;             // queries per wave (a query group)
    bool hash;          // the group's rows are pre-filtered by hash tables of its queries
    int nr;             // list registers (capacity 64*nr >= k_max)
    int chunks;         // row chunks (one wave each) over [seed_rows, N)
    int qgroups;        // query groups; each streams every row once
    int nparts;         // waves, and partial lists per query: seed_chunks + chunks
    int seed_chunks;    // chunks over the sampled rows (the first waves of a group)
    int64_t seed_rows;  // rows [0, seed_rows) whose LCP histogram sets each query's starting limit
    int seed_parts;     // histogram blocks per query
    int64_t seed_chunk_rows;
    int64_t chunk_rows;
};
// part_budget_bytes bounds the partial lists (Q * nparts * k_max * 8 bytes);
// nparts == 0 in the result means not even one seed chunk and one row chunk
// per query fit in it.
constexpr int64_t kScanPartBudget = (int64_t)256 << 20;
ScanPlan plan_scan(int64_t N, int W, int64_t Q, int32_t k_max, int64_t part_budget_bytes = kScanPartBudget);

// Per-call scratch of the scan, carved from one device allocation.
struct ScanScratch {
    int64_t cap;       // partial-list entries per query (nparts * k_max)
    uint64_t* part;    // [Q][cap]
    uint64_t* gthr;    // [Q] shared limits
    uint32_t* cnt;     // [Q] partial entries appended, one per 128-byte line
    uint32_t* hist;    // [Q][L+1] seed LCP histogram
    uint32_t* qkeys;   // [Q][W] query key words
    size_t words;      // total size in 32-bit words
};
ScanScratch scan_scratch(const ScanPlan& p, int64_t Q, int32_t k_max, const RowGeo& g, uint64_t* base);
size_t scan_partial_entries(const ScanPlan& p, int64_t Q, int32_t k_max, const RowGeo& g);  // in 8-byte units
// ev_scan0/ev_scan1 bracket the main scan kernel, ev_merge1 follows the merge
hipError_t launch_scan(const IndexView& ix, const QueryBatch& qb, const ScanPlan& p, uint64_t* scratch, hipStream_t s,
                       hipEvent_t ev_scan0, hipEvent_t ev_scan1, hipEvent_t ev_merge1);

// Prefix-bucket range scan: one wave per query scans the sorted rows sharing
// its first `depth` tokens.  The plane it streams: bucket_column(depth, g) < 0:
// the first two key words of every sorted row (launch_prefix_plane over the
// sorted copy); otherwise the column of that key word (launch_sorted_column).
// bounds: null, or [Q][2] int32 receiving each query's bucket [lo, hi) in
// sorted positions.
__host__ __device__ inline int64_t column_entries(int64_t N) { return (N + 3) & ~(int64_t)3; }
int bucket_column(int depth, const RowGeo& g);
hipError_t launch_sorted_column(const uint32_t* sorted, int64_t N, int W, int w, uint32_t* col, hipStream_t s);
hipError_t launch_bucket_scan(const IndexView& ix, const void* plane, const QueryBatch& qb, int depth,
                              int32_t* bounds, hipStream_t s);

}  // namespace lcpx
