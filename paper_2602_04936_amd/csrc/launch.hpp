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
hipError_t launch_iota(int32_t* p, int64_t N, hipStream_t s);
hipError_t launch_gather_word(const uint32_t* dense, const int32_t* perm, int64_t N, int Wd, int d, uint32_t* keys,
                              hipStream_t s);
hipError_t launch_radix_pass(const uint32_t* keys_in, const int32_t* vals_in, int64_t N, int shift, uint32_t* counts,
                             uint32_t* keys_out, int32_t* vals_out, bool write_keys, hipStream_t s);
hipError_t launch_gather_rows(const uint32_t* keys, const int32_t* perm, int64_t N, int W, uint32_t* sorted,
                              hipStream_t s);
hipError_t launch_adjacent_lcp(const uint32_t* sorted, int64_t N, RowGeo g, uint8_t* A, hipStream_t s);

// ---- queries
struct IndexView {
    const uint32_t* sorted;  // [N][W] key form, lexicographic order
    const uint32_t* rows;    // [N][W] key form, id order
    const int32_t* perm;     // [N]
    const uint8_t* A;        // [N] adjacent LCP
    int64_t N;
    RowGeo g;
};

struct QueryBatch {
    const void* raw;         // [Q][L] raw tokens (tb bytes each)
    int64_t Q;
    const int32_t* k;        // [Q] device
    const int64_t* off;      // [Q+1] device
    int32_t k_max;
    int32_t* out_ids;
    int32_t* out_lcp;
};

hipError_t launch_index_query(const IndexView& ix, const QueryBatch& qb, hipStream_t s);

// Full scan.  `part` must hold scan_partial_entries(...) keys.
struct ScanPlan {
    int tq;        // queries per wave
    int nr;        // list registers (capacity 64*nr >= k_max)
    int chunks;    // row chunks (grid x)
    int qgroups;   // query groups (grid y), 4*tq queries each
    int64_t chunk_rows;
};
ScanPlan plan_scan(int64_t N, int64_t Q, int32_t k_max);
size_t scan_partial_entries(const ScanPlan& p, int64_t Q, int32_t k_max);
hipError_t launch_scan(const IndexView& ix, const QueryBatch& qb, const ScanPlan& p, uint64_t* part, hipStream_t s,
                       hipEvent_t ev_scan0, hipEvent_t ev_scan1, hipEvent_t ev_merge1);

}  // namespace lcpx
