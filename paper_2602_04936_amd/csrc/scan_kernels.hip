// Plain path: brute-force full scan (LCP of every query against all N rows,
// then per-query top-k), the baseline the paper's range scan is measured
// against (section 7, Table "TAL range-scan vs full-scan").
//
// Grid = (row chunks) x (query groups).  A block's 4 waves stream the same
// row chunk (64 rows per step, one row per lane, in ascending id order) and
// each wave serves its own TQ queries, keeping one lane-distributed top-k
// list per query.  A row can only enter query i's list if its rank key beats
// the current k-th entry, which needs LCP >= that entry's LCP t: the hot loop
// therefore tests only the first min(t, tokens per word) tokens of the row's
// first key word with one AND and one compare against a pre-masked query word,
// and computes the exact LCP only for the rows that pass.  Each wave writes
// its per-chunk lists; a second kernel merges the chunks of each query.
#include "device.hpp"
#include "launch.hpp"

namespace lcpx {

constexpr int kScanWaves = 4;

template <int NR, int TQ>
__global__ __launch_bounds__(kScanWaves * kWave) void k_scan(IndexView ix, QueryBatch qb, int64_t chunk_rows,
                                                             int nparts, uint64_t* __restrict__ part) {
    extern __shared__ uint32_t s_q[];  // [kScanWaves*TQ][W]
    const RowGeo g = ix.g;
    const int lane = lane_id();
    const int64_t qblock = (int64_t)blockIdx.y * kScanWaves * TQ;
    for (int idx = threadIdx.x; idx < kScanWaves * TQ * g.W; idx += kScanWaves * kWave) {
        const int qq = idx / g.W;
        const int w = idx - qq * g.W;
        const int64_t qi = qblock + qq;
        s_q[idx] = qi < qb.Q ? key_word(qb.raw, qi * g.L, g, w) : 0u;
    }
    __syncthreads();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t q0i = qblock + (int64_t)wv * TQ;
    if (q0i >= qb.Q) return;
    const int ntq = (int)(qb.Q - q0i < TQ ? qb.Q - q0i : TQ);
    const int64_t N = ix.N;
    const int tpw = 1 << g.tpw_log2;
    const int tbits = 8 * g.tb;

    WaveList<NR> lst[TQ];
    uint32_t qw0[TQ], msk[TQ], qm[TQ];
    int kk[TQ];
#pragma unroll
    for (int i = 0; i < TQ; ++i) {
        lst[i].init();
        qw0[i] = uniform(s_q[(wv * TQ + i) * g.W]);
        msk[i] = 0u;
        qm[i] = 0u;
        const int ki = i < ntq ? qb.k[q0i + i] : 1;
        kk[i] = (int)((int64_t)ki < N ? (int64_t)ki : N);
    }

    const int64_t r_lo = (int64_t)blockIdx.x * chunk_rows;
    const int64_t r_hi = r_lo + chunk_rows < N ? r_lo + chunk_rows : N;
    for (int64_t base = r_lo; base < r_hi; base += kWave) {
        const int64_t id = base + lane;
        const bool act = id < r_hi;
        const uint32_t w0 = act ? ix.rows[id * g.W] : 0u;
#pragma unroll
        for (int i = 0; i < TQ; ++i) {
            if (i < ntq) {
                const bool cand = act && (w0 & msk[i]) == qm[i];
                if (ballot(cand)) {
                    int lc = -1;
                    if (cand) {
                        const uint32_t x = w0 ^ qw0[i];
                        lc = x ? lcp_from_diff(0, x, g)
                               : lcp_tail(ix.rows + id * g.W, s_q + (wv * TQ + i) * g.W, g, 1);
                    }
                    lst[i].offer(rank_key(lc, (uint32_t)id), cand, kk[i]);
                    const uint64_t th = lst[i].get(kk[i] - 1);
                    const int tl = th == kKeyMax ? 0 : key_lcp(th);
                    msk[i] = tl >= tpw ? 0xFFFFFFFFu : ~(0xFFFFFFFFu >> (tl * tbits));
                    qm[i] = qw0[i] & msk[i];
                }
            }
        }
    }

#pragma unroll
    for (int i = 0; i < TQ; ++i) {
        if (i < ntq) {
            uint64_t* dst = part + ((q0i + i) * nparts + blockIdx.x) * (int64_t)qb.k_max;
#pragma unroll
            for (int rr = 0; rr < NR; ++rr) {
                const int e = rr * kWave + lane;
                if (e < qb.k_max) dst[e] = e < kk[i] ? lst[i].v[rr] : kKeyMax;
            }
        }
    }
}

template <int NR>
__global__ __launch_bounds__(kScanWaves * kWave) void k_scan_merge(QueryBatch qb, int64_t N, int nparts,
                                                                   const uint64_t* __restrict__ part) {
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t qi = (int64_t)blockIdx.x * kScanWaves + wv;
    if (qi >= qb.Q) return;
    const int k = qb.k[qi];
    const int m = (int)((int64_t)k < N ? (int64_t)k : N);
    const int64_t total = (int64_t)nparts * qb.k_max;
    const uint64_t* src = part + qi * total;
    WaveList<NR> lst;
    lst.init();
    for (int64_t b = 0; b < total; b += kWave) {
        const int64_t t = b + lane;
        const bool act = t < total && (int)(t % qb.k_max) < m;
        const uint64_t key = act ? src[t] : kKeyMax;
        lst.offer(key, act && key != kKeyMax, m);
    }
    int32_t* oid = qb.out_ids + qb.off[qi];
    int32_t* olc = qb.out_lcp + qb.off[qi];
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
        case 1: tq = 16; break;
        case 2: tq = 8; break;
        case 4: tq = 4; break;
        default: tq = 1; break;
    }
    while (tq > 1 && (int64_t)kScanWaves * tq / 2 >= Q) tq = tq > 4 ? 4 : 1;
    return tq;
}

ScanPlan plan_scan(int64_t N, int64_t Q, int32_t k_max) {
    ScanPlan p;
    p.nr = nr_for(k_max);
    p.tq = tq_for(p.nr, Q);
    const int64_t per_group = (int64_t)kScanWaves * p.tq;
    p.qgroups = (int)((Q + per_group - 1) / per_group);
    // aim for >= 2048 blocks, chunks of >= 4096 rows, partials <= 256 MiB
    int64_t chunks = (2048 + p.qgroups - 1) / p.qgroups;
    const int64_t max_by_rows = (N + 4095) / 4096;
    if (chunks > max_by_rows) chunks = max_by_rows;
    const int64_t bytes_per_chunk = Q * (int64_t)k_max * 8;
    const int64_t max_by_mem = bytes_per_chunk > 0 ? ((int64_t)256 << 20) / bytes_per_chunk : chunks;
    if (chunks > max_by_mem) chunks = max_by_mem;
    if (chunks > 65535) chunks = 65535;
    if (chunks < 1) chunks = 1;
    int64_t rows = (N + chunks - 1) / chunks;
    rows = (rows + kWave - 1) / kWave * kWave;
    p.chunk_rows = rows;
    p.chunks = (int)((N + rows - 1) / rows);
    return p;
}

size_t scan_partial_entries(const ScanPlan& p, int64_t Q, int32_t k_max) {
    return (size_t)Q * (size_t)p.chunks * (size_t)k_max;
}

template <int NR, int TQ>
static void launch_scan_t(const IndexView& ix, const QueryBatch& qb, const ScanPlan& p, uint64_t* part,
                          hipStream_t s) {
    const size_t shm = (size_t)kScanWaves * TQ * ix.g.W * sizeof(uint32_t);
    hipLaunchKernelGGL((k_scan<NR, TQ>), dim3((unsigned)p.chunks, (unsigned)p.qgroups), dim3(kScanWaves * kWave),
                       shm, s, ix, qb, p.chunk_rows, p.chunks, part);
}

hipError_t launch_scan(const IndexView& ix, const QueryBatch& qb, const ScanPlan& p, uint64_t* part, hipStream_t s,
                       hipEvent_t ev0, hipEvent_t ev1, hipEvent_t ev2) {
    if (qb.Q <= 0) return hipSuccess;
    if (ev0) hipEventRecord(ev0, s);
    switch (p.nr * 100 + p.tq) {
        case 116: launch_scan_t<1, 16>(ix, qb, p, part, s); break;
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
        case 1: hipLaunchKernelGGL((k_scan_merge<1>), dim3(grid), blk, 0, s, qb, ix.N, p.chunks, part); break;
        case 2: hipLaunchKernelGGL((k_scan_merge<2>), dim3(grid), blk, 0, s, qb, ix.N, p.chunks, part); break;
        case 4: hipLaunchKernelGGL((k_scan_merge<4>), dim3(grid), blk, 0, s, qb, ix.N, p.chunks, part); break;
        default: hipLaunchKernelGGL((k_scan_merge<16>), dim3(grid), blk, 0, s, qb, ix.N, p.chunks, part); break;
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev2) hipEventRecord(ev2, s);
    return hipSuccess;
}

}  // namespace lcpx
