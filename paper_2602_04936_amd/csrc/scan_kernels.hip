// Plain path: brute-force full scan (LCP of every query against all N rows,
// then per-query top-k), the baseline the paper's range scan is measured
// against (section 7, Table "TAL range-scan vs full-scan").
//
// Grid = (row chunks) x (query groups).  A block's 4 waves stream the same
// row chunk (one row per lane, 4 tiles of 64 rows in flight, ascending ids)
// and each wave serves its own TQ queries, keeping one lane-distributed top-k
// list per query.  Once a list holds k entries, every row still to come has a
// larger id than all of them, so it can only enter with an LCP at least one
// more than the k-th entry's LCP t: the hot loop tests the first t + 1 tokens
// of the row's first key word with one AND and one compare against a
// pre-masked query word, and computes the exact LCP only for rows that pass.
// Each wave writes its per-chunk lists; a second kernel merges the chunks of
// each query.
#include "device.hpp"
#include "launch.hpp"

namespace lcpx {

constexpr int kScanWaves = 4;
constexpr int kScanUnroll = 4;

// Mask and masked query bits that a row's first two key words (as one 64-bit
// value, word 0 high) must match for the row's rank key to beat `lim`
// (kKeyMax: no limit yet).  A row with the same LCP as `lim` beats it only with
// a smaller id, so when every row still to come has an id above lim's
// (id(lim) < next_id) one more token must match.
__device__ __forceinline__ void limit_filter(uint64_t lim, int64_t next_id, uint64_t q01, const RowGeo& g,
                                             uint64_t& msk, uint64_t& qm) {
    if (lim == kKeyMax) {
        msk = 0;  // no limit: every row is a candidate
        qm = 0;
        return;
    }
    const int need = key_lcp(lim) + ((int64_t)(uint32_t)lim < next_id ? 1 : 0);
    const int bits = need * 8 * g.tb;  // leading bits that must match
    if (need > g.L) {
        msk = 0;  // no row can share more than L tokens: nothing enters any more
        qm = 1;
    } else if (bits >= 64) {
        msk = ~0ull;  // both words must match; later words are checked exactly
        qm = q01;
    } else {
        msk = bits == 0 ? 0ull : ~(~0ull >> bits);
        qm = q01 & msk;
    }
}

__global__ void k_fill_u64(uint64_t* __restrict__ p, int64_t n, uint64_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// gthr[q] holds the smallest k-th key any chunk has reached for query q: a row
// whose key is not below it cannot be in q's answer (that k-th key is the
// k-th best of k real rows), so every chunk may skip such rows.  The limit
// only prunes; the merged answer is the unique exact top-k either way.
//
// Code layout: the unrolled hot loop only tests (tile, query) pairs and sets
// a bit for each pair with a candidate lane; a single, non-unrolled slow path
// then serves the flagged pairs, with each query's list and filter in LDS, so
// the kernel stays small enough for the instruction cache.
template <int NR>
struct ScanQueryState {  // per (wave, query), in LDS
    uint64_t list[NR * kWave];
    uint64_t lim;
    uint64_t msk, qm;
    int32_t kk;  // min(k, N)
    int32_t pad_;
};

// Query key words, computed once per launch for every block to copy.
__global__ void k_query_keys(QueryBatch qb, RowGeo g, uint32_t* __restrict__ qkeys) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= qb.Q * g.W) return;
    const int64_t qi = t / g.W;
    qkeys[t] = key_word(qb.raw, qi * g.L, g, (int)(t - qi * g.W));
}

// Rows [row0, row_end) in chunks of chunk_rows; chunk c writes partial list
// part0 + c of each query (nparts lists per query in total).
template <int NR, int TQ>
__global__ __launch_bounds__(kScanWaves * kWave) void k_scan(IndexView ix, QueryBatch qb, const uint32_t* qkeys,
                                                             int64_t row0, int64_t row_end, int64_t chunk_rows,
                                                             int part0, int nparts, uint64_t* __restrict__ part,
                                                             uint64_t* __restrict__ gthr) {
    static_assert(kScanUnroll * TQ <= 64, "one flag bit per (tile, query)");
    extern __shared__ uint64_t s_dyn64[];
    ScanQueryState<NR>* st_all = reinterpret_cast<ScanQueryState<NR>*>(s_dyn64);  // [kScanWaves*TQ]
    uint32_t* s_q = reinterpret_cast<uint32_t*>(st_all + kScanWaves * TQ);       // [kScanWaves*TQ][W]
    const RowGeo g = ix.g;
    const int lane = lane_id();
    const int64_t qblock = (int64_t)blockIdx.y * kScanWaves * TQ;
    for (int idx = threadIdx.x; idx < kScanWaves * TQ * g.W; idx += kScanWaves * kWave)
        s_q[idx] = qblock * g.W + idx < qb.Q * g.W ? qkeys[qblock * g.W + idx] : 0u;
    for (int idx = threadIdx.x; idx < kScanWaves * TQ; idx += kScanWaves * kWave) {
        // query slots past the end of the batch get a filter nothing matches
        const bool real = qblock + idx < qb.Q;
        st_all[idx].lim = kKeyMax;
        st_all[idx].msk = 0;
        st_all[idx].qm = real ? 0 : 1;
        const int ki = real ? query_k(qb, qblock + idx) : 1;
        st_all[idx].kk = (int)((int64_t)ki < ix.N ? (int64_t)ki : ix.N);
    }
    for (int idx = threadIdx.x; idx < kScanWaves * TQ * NR * kWave; idx += kScanWaves * kWave)
        st_all[idx / (NR * kWave)].list[idx % (NR * kWave)] = kKeyMax;
    __syncthreads();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t q0i = qblock + (int64_t)wv * TQ;
    if (q0i >= qb.Q) return;
    const int ntq = (int)(qb.Q - q0i < TQ ? qb.Q - q0i : TQ);
    const int64_t N = ix.N;
    const int W = g.W;
    ScanQueryState<NR>* st = st_all + wv * TQ;
    const uint32_t* qwords = s_q + wv * TQ * W;

    const int64_t r_lo = row0 + (int64_t)blockIdx.x * chunk_rows;
    const int64_t r_hi = r_lo + chunk_rows < row_end ? r_lo + chunk_rows : row_end;
    const int second = W > 1 ? 1 : 0;                 // a one-word row has no second word:
    const uint32_t second_mask = W > 1 ? ~0u : 0u;    // it reads word 0 again and masks it off
    // rows of the next step are requested before the current step is
    // processed, so a step's loads overlap the previous step's compute
    uint32_t na[kScanUnroll], nb[kScanUnroll];
#pragma unroll
    for (int u = 0; u < kScanUnroll; ++u) {
        const int64_t id = r_lo + u * kWave + lane;
        const uint32_t* r = ix.rows + (id < r_hi ? id : r_hi - 1) * W;
        na[u] = r[0];
        nb[u] = r[second];
    }
    int it = 0;
    for (int64_t base = r_lo; base < r_hi; base += kScanUnroll * kWave, ++it) {
        if ((it & 7) == 0) {
            // pick up tighter limits reached by other chunks: lane i reads query
            // i's limit with a plain load (a stale value only prunes less)
            const uint64_t mine = lane < ntq ? gthr[q0i + lane] : kKeyMax;
#pragma unroll 1
            for (int i = 0; i < ntq; ++i) {
                const uint64_t gv = readlane64(mine, i);
                if (gv < st[i].lim) {
                    const uint32_t* q = qwords + i * W;
                    const uint64_t q01 = ((uint64_t)q[0] << 32) | (W >= 2 ? q[1] : 0u);
                    uint64_t msk, qm;
                    limit_filter(gv, base, q01, g, msk, qm);
                    if (lane == 0) {
                        st[i].lim = gv;
                        st[i].msk = msk;
                        st[i].qm = qm;
                    }
                }
            }
        }
        // first two key words of each lane's row (word 0 in the high half)
        uint32_t wa[kScanUnroll], wb[kScanUnroll];
#pragma unroll
        for (int u = 0; u < kScanUnroll; ++u) {
            wa[u] = na[u];
            wb[u] = nb[u];
        }
        if (base + kScanUnroll * kWave < r_hi) {
#pragma unroll
            for (int u = 0; u < kScanUnroll; ++u) {
                const int64_t id = base + (kScanUnroll + u) * kWave + lane;
                const uint32_t* r = ix.rows + (id < r_hi ? id : r_hi - 1) * W;
                na[u] = r[0];
                nb[u] = r[second];
            }
        }
        uint64_t w01[kScanUnroll];
        uint64_t live[kScanUnroll];  // lanes holding a row of this chunk
#pragma unroll
        for (int u = 0; u < kScanUnroll; ++u) {
            w01[u] = ((uint64_t)wa[u] << 32) | (wb[u] & second_mask);
            live[u] = ballot(base + u * kWave + lane < r_hi);
        }
        // filters stay in VGPRs (wave-uniform values): one AND pair and one
        // 64-bit compare per (tile, query)
        uint64_t msk[TQ], qm[TQ];
#pragma unroll
        for (int i = 0; i < TQ; ++i) {
            msk[i] = st[i].msk;
            qm[i] = st[i].qm;
        }
        // hot loop: which (tile, query) pairs have a candidate lane
        uint64_t flagged = 0;
#pragma unroll
        for (int u = 0; u < kScanUnroll; ++u) {
#pragma unroll
            for (int i = 0; i < TQ; ++i)
                if (ballot((w01[u] & msk[i]) == qm[i]) & live[u]) flagged |= 1ull << (u * TQ + i);
        }
        // slow path, one flagged pair at a time (tiles in ascending order)
        while (flagged) {
            const int bit = low_lane(flagged);
            flagged &= flagged - 1;
            const int u = bit / TQ;
            const int i = bit - u * TQ;
            const int64_t id = base + u * kWave + lane;
            const bool act = id < r_hi;
            uint64_t w = w01[0];
#pragma unroll
            for (int uu = 1; uu < kScanUnroll; ++uu) w = u == uu ? w01[uu] : w;
            const uint32_t* q = qwords + i * W;
            const uint64_t q01 = ((uint64_t)q[0] << 32) | (W > 1 ? q[1] : 0u);
            const bool cand = act && (w & st[i].msk) == st[i].qm;
            int lc = -1;
            if (cand) {
                const uint64_t x = w ^ q01;
                if (x >> 32)
                    lc = lcp_from_diff(0, (uint32_t)(x >> 32), g);
                else if ((uint32_t)x)
                    lc = lcp_from_diff(1, (uint32_t)x, g);
                else
                    lc = W > 2 ? lcp_tail(ix.rows + id * W, q, g, 2) : g.L;
            }
            const int kk = st[i].kk;
            const uint64_t lim = st[i].lim;
            const uint64_t key = rank_key(lc, (uint32_t)id);
            WaveList<NR> lst;
#pragma unroll
            for (int r = 0; r < NR; ++r) lst.v[r] = st[i].list[r * kWave + lane];
            lst.offer(key, cand && key < lim, kk);
            const uint64_t kth = lst.get(kk - 1);
            uint64_t nlim = lim;
            if (kth < lim) {
                nlim = kth;
                if (lane == 0) atomicMin((unsigned long long*)(gthr + q0i + i), (unsigned long long)kth);
            }
            uint64_t nm, nq;
            limit_filter(nlim, base + (u + 1) * kWave, q01, g, nm, nq);
#pragma unroll
            for (int r = 0; r < NR; ++r) st[i].list[r * kWave + lane] = lst.v[r];
            if (lane == 0) {
                st[i].lim = nlim;
                st[i].msk = nm;
                st[i].qm = nq;
            }
        }
    }

#pragma unroll 1
    for (int i = 0; i < ntq; ++i) {
        const int kk = st[i].kk;
        uint64_t* dst = part + ((q0i + i) * nparts + part0 + blockIdx.x) * (int64_t)qb.k_max;
        for (int e = lane; e < qb.k_max; e += kWave) dst[e] = e < kk ? st[i].list[e] : kKeyMax;
    }
}

// Merge partial lists [part_lo, part_hi) of each query.  With `limit` set,
// write the k-th smallest merged key (kKeyMax if fewer than k) as the query's
// starting limit instead of emitting the answer.
template <int NR>
__global__ __launch_bounds__(kScanWaves * kWave) void k_scan_merge(QueryBatch qb, int64_t N, int nparts, int part_lo,
                                                                   int part_hi, const uint64_t* __restrict__ part,
                                                                   uint64_t* __restrict__ limit) {
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t qi = (int64_t)blockIdx.x * kScanWaves + wv;
    if (qi >= qb.Q) return;
    const int k = query_k(qb, qi);
    const int m = (int)((int64_t)k < N ? (int64_t)k : N);
    const int64_t total = (int64_t)(part_hi - part_lo) * qb.k_max;
    const uint64_t* src = part + (qi * nparts + part_lo) * (int64_t)qb.k_max;
    WaveList<NR> lst;
    lst.init();
    constexpr int kMergeUnroll = 8;
    for (int64_t b = 0; b < total; b += kMergeUnroll * kWave) {
        uint64_t key[kMergeUnroll];
#pragma unroll
        for (int u = 0; u < kMergeUnroll; ++u) {  // all loads in flight before any is used
            const int64_t t = b + u * kWave + lane;
            const bool act = t < total && (int)(t % qb.k_max) < m;
            key[u] = act ? src[t] : kKeyMax;
        }
#pragma unroll 1
        for (int u = 0; u < kMergeUnroll && b + u * kWave < total; ++u) {  // one copy of the offer code
            uint64_t x = key[0];
#pragma unroll
            for (int uu = 1; uu < kMergeUnroll; ++uu) x = u == uu ? key[uu] : x;
            lst.offer(x, x != kKeyMax, m);
        }
    }
    if (limit) {
        const uint64_t kth = lst.get(m - 1);
        if (lane == 0) limit[qi] = kth;
        return;
    }
    int32_t* oid = qb.out_ids + query_off(qb, qi);
    int32_t* olc = qb.out_lcp + query_off(qb, qi);
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) {
        const int e = rr * kWave + lane;
        if (e < m) {
            oid[e] = key_id(lst.v[rr]);
            olc[e] = key_lcp(lst.v[rr]);
        }
    }
    for (int e = m + lane; e < k; e += kWave) {
        oid[e] = -1;
        olc[e] = -1;
    }
}

static int nr_for(int32_t k_max) { return k_max <= 64 ? 1 : k_max <= 128 ? 2 : k_max <= 256 ? 4 : 16; }

static int tq_for(int nr, int64_t Q) {
    // queries per wave, from the compiled set, no more than the batch needs
    int tq;
    switch (nr) {
        case 1: tq = 8; break;
        case 2: tq = 8; break;
        case 4: tq = 4; break;
        default: tq = 1; break;
    }
    while (tq > 1 && (int64_t)kScanWaves * tq / 2 >= Q) tq = tq > 4 ? 4 : 1;
    return tq;
}

// The first rows are scanned first, in seed chunks whose merged k-th key
// becomes every query's starting limit for the remaining chunks.
constexpr int64_t kChunkMinRows = 2048;
constexpr int64_t kSeedChunkRows = kScanUnroll * kWave;  // one step per seed chunk
constexpr int64_t kSeedRowsMax = 32768;

ScanPlan plan_scan(int64_t N, int64_t Q, int32_t k_max) {
    ScanPlan p;
    p.nr = nr_for(k_max);
    p.tq = tq_for(p.nr, Q);
    const int64_t per_group = (int64_t)kScanWaves * p.tq;
    p.qgroups = (int)((Q + per_group - 1) / per_group);
    const int64_t bytes_per_chunk = Q * (int64_t)k_max * 8;
    const int64_t max_by_mem = bytes_per_chunk > 0 ? ((int64_t)256 << 20) / bytes_per_chunk : 1;
    // seed: up to 1/8 of the rows (at most kSeedRowsMax) in one-step chunks
    p.seed_rows = N / 8 < kSeedRowsMax ? N / 8 : kSeedRowsMax;
    p.seed_chunks = (int)(p.seed_rows / kSeedChunkRows);
    if (p.seed_chunks > max_by_mem / 2) p.seed_chunks = (int)(max_by_mem / 2);
    if (p.seed_chunks < 4) p.seed_chunks = 0;  // too few rows to be worth a seed
    p.seed_rows = p.seed_chunks * kSeedChunkRows;
    const int64_t rest = N - p.seed_rows;
    // main: aim for >= 4096 blocks (16 per CU), chunks of >= kChunkMinRows rows, partials <= 256 MiB
    int64_t chunks = (4096 + p.qgroups - 1) / p.qgroups;
    const int64_t max_by_rows = (rest + kChunkMinRows - 1) / kChunkMinRows;
    if (chunks > max_by_rows) chunks = max_by_rows;
    if (chunks > max_by_mem - p.seed_chunks) chunks = max_by_mem - p.seed_chunks;
    if (chunks > 65535) chunks = 65535;
    if (chunks < 1) chunks = 1;
    const int64_t step = (int64_t)kScanUnroll * kWave;
    int64_t rows = (rest + chunks - 1) / chunks;
    rows = (rows + step - 1) / step * step;
    p.chunk_rows = rows;
    p.chunks = (int)((rest + rows - 1) / rows);
    p.nparts = p.seed_chunks + p.chunks;
    return p;
}

size_t scan_partial_entries(const ScanPlan& p, int64_t Q, int32_t k_max, int W) {
    // per-chunk lists, one shared limit per query, then the query key words
    return (size_t)Q * (size_t)p.nparts * (size_t)k_max + (size_t)Q + ((size_t)Q * W + 1) / 2;
}

template <int NR, int TQ>
static void launch_scan_t(const IndexView& ix, const QueryBatch& qb, const ScanPlan& p, uint64_t* part,
                          hipStream_t s) {
    const size_t shm =
        (size_t)kScanWaves * TQ * (sizeof(ScanQueryState<NR>) + (size_t)ix.g.W * sizeof(uint32_t));
    uint64_t* gthr = part + (size_t)qb.Q * (size_t)p.nparts * (size_t)qb.k_max;
    const uint32_t* qkeys = reinterpret_cast<const uint32_t*>(gthr + qb.Q);
    const dim3 blk(kScanWaves * kWave);
    if (p.seed_chunks > 0) {
        hipLaunchKernelGGL((k_scan<NR, TQ>), dim3((unsigned)p.seed_chunks, (unsigned)p.qgroups), blk, shm, s, ix, qb,
                           qkeys, (int64_t)0, p.seed_rows, kSeedChunkRows, 0, p.nparts, part, gthr);
        hipLaunchKernelGGL((k_scan_merge<NR>), dim3((unsigned)((qb.Q + kScanWaves - 1) / kScanWaves)), blk, 0, s, qb,
                           ix.N, p.nparts, 0, p.seed_chunks, part, gthr);
    }
    hipLaunchKernelGGL((k_scan<NR, TQ>), dim3((unsigned)p.chunks, (unsigned)p.qgroups), blk, shm, s, ix, qb, qkeys,
                       p.seed_rows, ix.N, p.chunk_rows, p.seed_chunks, p.nparts, part, gthr);
}

hipError_t launch_scan(const IndexView& ix, const QueryBatch& qb, const ScanPlan& p, uint64_t* part, hipStream_t s,
                       hipEvent_t ev0, hipEvent_t ev1, hipEvent_t ev2) {
    if (qb.Q <= 0) return hipSuccess;
    if (ev0) hipEventRecord(ev0, s);
    {
        uint64_t* gthr = part + (size_t)qb.Q * (size_t)p.nparts * (size_t)qb.k_max;
        uint32_t* qkeys = reinterpret_cast<uint32_t*>(gthr + qb.Q);
        hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((qb.Q + 255) / 256)), dim3(256), 0, s, gthr, qb.Q, kKeyMax);
        hipLaunchKernelGGL(k_query_keys, dim3((unsigned)((qb.Q * ix.g.W + 255) / 256)), dim3(256), 0, s, qb, ix.g,
                           qkeys);
    }
    switch (p.nr * 100 + p.tq) {
        case 108: launch_scan_t<1, 8>(ix, qb, p, part, s); break;
        case 104: launch_scan_t<1, 4>(ix, qb, p, part, s); break;
        case 101: launch_scan_t<1, 1>(ix, qb, p, part, s); break;
        case 208: launch_scan_t<2, 8>(ix, qb, p, part, s); break;
        case 204: launch_scan_t<2, 4>(ix, qb, p, part, s); break;
        case 201: launch_scan_t<2, 1>(ix, qb, p, part, s); break;
        case 404: launch_scan_t<4, 4>(ix, qb, p, part, s); break;
        case 401: launch_scan_t<4, 1>(ix, qb, p, part, s); break;
        case 1601: launch_scan_t<16, 1>(ix, qb, p, part, s); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev1) hipEventRecord(ev1, s);
    const unsigned grid = (unsigned)((qb.Q + kScanWaves - 1) / kScanWaves);
    const dim3 blk(kScanWaves * kWave);
    switch (p.nr) {
        case 1: hipLaunchKernelGGL((k_scan_merge<1>), dim3(grid), blk, 0, s, qb, ix.N, p.nparts, 0, p.nparts, part,
                                   (uint64_t*)nullptr); break;
        case 2: hipLaunchKernelGGL((k_scan_merge<2>), dim3(grid), blk, 0, s, qb, ix.N, p.nparts, 0, p.nparts, part,
                                   (uint64_t*)nullptr); break;
        case 4: hipLaunchKernelGGL((k_scan_merge<4>), dim3(grid), blk, 0, s, qb, ix.N, p.nparts, 0, p.nparts, part,
                                   (uint64_t*)nullptr); break;
        default: hipLaunchKernelGGL((k_scan_merge<16>), dim3(grid), blk, 0, s, qb, ix.N, p.nparts, 0, p.nparts, part,
                                    (uint64_t*)nullptr); break;
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev2) hipEventRecord(ev2, s);
    return hipSuccess;
}

}  // namespace lcpx
