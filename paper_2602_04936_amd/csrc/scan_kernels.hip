// Plain path: brute-force full scan (LCP of every query against all N rows,
// then per-query top-k), the baseline the paper's range scan is measured
// against (section 7, Table "TAL range-scan vs full-scan").
//
// The pass streams the 8-byte prefix plane (key words 0 and 1 of every row,
// id order).  Queries are split into groups of TQ; each wave streams one row
// chunk for the TQ queries of its group (16 bytes, two rows, per lane and
// load, the next step's loads in flight while the current step is tested),
// keeping one top-k list per query.  Once a list holds k entries, every row
// still to come has a larger id than all of them, so it can only enter with an
// LCP at least one more than the k-th entry's LCP t: the hot loop tests the
// first t + 1 tokens of the row's first two key words with one 64-bit compare
// (and two ANDs when t + 1 tokens are fewer than 64 bits) against a pre-masked
// query value, and computes the exact LCP only for rows that pass.  Before the
// scan, an LCP histogram of every query against the first rows gives each
// query a starting limit, so most rows fail the filter from the first step
// on.  Each wave appends the entries of its lists that can still be in the
// answer to the query's compact partial list; a second kernel merges them.
#include "device.hpp"
#include "launch.hpp"

namespace lcpx {

constexpr int kScanWaves = 4;
// Each query's fill count sits on its own 128-byte line: every wave of every
// chunk adds to the counts of its queries, and counts sharing a line would
// serialise those atomics in one L2 channel.
constexpr int kCntStride = 32;

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


// Starting limits from the first S rows (ids 0..S-1).  hist[q][d] counts the
// sample rows with LCP exactly d.  With t the largest d such that at least k'
// sample rows have LCP >= d, those k' rows have keys <= rank_key(t, S - 1),
// so the answer's k'-th key is below rank_key(t, S): every answer row beats
// that key, which becomes the query's limit.  Block b counts part b % parts
// of the sample for query b / parts.
constexpr int kSeedThreads = 256;
__global__ __launch_bounds__(kSeedThreads) void k_seed_hist(IndexView ix, const uint32_t* __restrict__ qkeys,
                                                            int64_t S, int parts, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[256];                 // LCP 0..L, L <= 255
    __shared__ uint32_t qw[128];                // key words of one query, W <= 128
    const RowGeo g = ix.g;
    const int lane = lane_id();
    const int64_t qi = (int64_t)blockIdx.x / parts;
    const int part = (int)((int64_t)blockIdx.x - qi * parts);
    for (int i = threadIdx.x; i <= g.L; i += kSeedThreads) h[i] = 0;
    for (int w = threadIdx.x; w < g.W; w += kSeedThreads) qw[w] = qkeys[qi * g.W + w];
    __syncthreads();
    const int64_t per = (S + parts - 1) / parts;
    const int64_t r0 = (int64_t)part * per;
    const int64_t r1 = r0 + per < S ? r0 + per : S;
    for (int64_t base = r0; base < r1; base += kSeedThreads) {
        const int64_t r = base + threadIdx.x;
        const bool act = r < r1;
        int lc = g.L;
        if (act) {
            const uint64_t pw = ix.plane[r];
            const uint32_t x0 = (uint32_t)(pw >> 32) ^ qw[0];
            const uint32_t x1 = g.W > 1 ? (uint32_t)pw ^ qw[1] : 0u;
            if (x0) {
                lc = lcp_from_diff(0, x0, g);
            } else if (x1) {
                lc = lcp_from_diff(1, x1, g);
            } else {
                const uint32_t* row = ix.rows + r * g.W;
                for (int w = 2; w < g.W; ++w) {
                    const uint32_t x = row[w] ^ qw[w];
                    if (x) {
                        lc = lcp_from_diff(w, x, g);
                        break;
                    }
                }
            }
        }
        // rows sharing no token with the query (most of them) in one add,
        // then one LDS add per distinct nonzero LCP value in the wave
        const uint64_t zero = ballot(act && lc == 0);
        if (lane == 0 && zero) atomicAdd(&h[0], (uint32_t)popc64(zero));
        uint64_t pending = ballot(act && lc != 0);
        while (pending) {
            const int v = readlane_i(lc, low_lane(pending));
            const uint64_t same = ballot(((pending >> lane) & 1ull) && lc == v);
            if (lane == low_lane(same)) atomicAdd(&h[v], (uint32_t)popc64(same));
            pending &= ~same;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= g.L; i += kSeedThreads)
        if (h[i]) atomicAdd(hist + qi * (g.L + 1) + i, h[i]);
}

// One wave per query.  Lane i takes d = top - i, so the wave's inclusive
// prefix sum at lane i counts the sample rows with LCP in [d, top] (plus the
// rows above top from earlier passes); the first lane where it reaches k'
// gives the largest d with at least k' sample rows of LCP >= d.  All of a
// pass's histogram loads are in flight at once.
__global__ __launch_bounds__(kScanWaves * kWave) void k_seed_limit(QueryBatch qb, int64_t N, int L, int64_t S,
                                                                   const uint32_t* __restrict__ hist,
                                                                   uint64_t* __restrict__ gthr) {
    const int lane = lane_id();
    const int64_t qi = (int64_t)blockIdx.x * kScanWaves + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (qi >= qb.Q) return;
    const int k = query_k(qb, qi);
    const uint32_t kk = (uint32_t)((int64_t)k < N ? (int64_t)k : N);
    const uint32_t* h = hist + qi * (L + 1);
    uint64_t lim = kKeyMax;
    uint32_t above = 0;  // sample rows with LCP above this pass's top
    for (int top = L; top >= 0; top -= kWave) {
        const int d = top - lane;
        const uint32_t acc = wave_prefix_sum(d >= 0 ? h[d] : 0u) + above;
        const uint64_t ok = ballot(d >= 0 && acc >= kk);
        if (ok) {
            lim = rank_key(top - low_lane(ok), (uint32_t)S);
            break;
        }
        above = readlane(acc, kWave - 1);
    }
    if (lane == 0) gthr[qi] = lim;
}

// gthr[q] holds the smallest k-th key any wave has reached for query q: a row
// whose key is not below it cannot be in q's answer (that k-th key is the
// k-th best of k real rows), so every wave may skip such rows.  The limit
// only prunes; the merged answer is the unique exact top-k either way.

// One launch before the scan: zero the fill counts and histograms (a kernel,
// not a memset, so the sequence can be captured in a graph) and compute the
// query key words once for every block to copy.
__global__ void k_scan_prep(QueryBatch qb, RowGeo g, uint32_t* __restrict__ zero, int64_t nz,
                            uint32_t* __restrict__ qkeys) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nz) zero[t] = 0u;
    if (t < qb.Q * g.W) {
        const int64_t qi = t / g.W;
        qkeys[t] = key_word(qb.raw, qi * g.L, g, (int)(t - qi * g.W));
    }
}

// Per (wave, query) filter state in LDS.
struct ScanFilter {
    uint64_t msk, qm;  // a row passes when (plane & msk) == qm
    uint64_t lim;      // the wave's limit key for the query
    int32_t kk;        // min(k, N)
    int32_t pad_;
};

// Geometry of one scan launch (grid x = qgroups * ceil(nparts / kScanWaves)).
struct ScanGrid {
    int64_t seed_rows;        // rows [0, seed_rows) are the seed sample
    int64_t seed_chunk_rows;  // rows per seed wave
    int64_t chunk_rows;       // rows per main wave, over [seed_rows, N)
    int nparts;               // waves (partial lists) per query group: seed waves first
    int seed_chunks;
    int qgroups;
    int lstride;              // list entries kept per (wave, query): k_max
};

// One wave streams one row chunk of the prefix plane for the TQ queries of its
// block's query group; the block's 4 waves take 4 consecutive chunks.  Each
// lane reads 16 bytes (two rows) per load, kScanU loads per step (512 rows),
// and the next step's loads are in flight while the current step is tested.
// Consecutive blocks (after the XCD remap below) take the same rows for
// different query groups, so a chunk is fetched into one XCD's L2 once.
//
// Code layout: the unrolled hot loop only tests, per query, whether any of the
// step's rows passes its filter (one 64-bit compare per row, and two ANDs
// when the filter keeps part of the 64 bits), and sets one bit per flagged
// query; a single non-unrolled slow path then serves the flagged queries with
// the query's list and filter in LDS.
//
// At the end each wave appends, per query, the entries of its list that do
// not exceed the query's limit to the query's partial list (cap entries at
// part + q * cap, fill count in cnt[q]); the append order does not matter,
// the merge ranks by key.
constexpr int kScanU = 4;                                  // 16-byte loads per lane per step
constexpr int64_t kPairRows = 2 * kWave;                   // rows of one 16-byte load of the wave
constexpr int64_t kScanStepRows = kScanU * kPairRows;      // rows per wave step
constexpr int kGthrEvery = 4;                              // steps between pick-ups of shared limits

template <int NR, int TQ>
__global__ __launch_bounds__(kScanWaves * kWave) void k_scan(IndexView ix, QueryBatch qb,
                                                             const uint32_t* __restrict__ qkeys, ScanGrid sg,
                                                             int64_t cap, uint64_t* __restrict__ part,
                                                             uint32_t* __restrict__ cnt,
                                                             uint64_t* __restrict__ gthr) {
    static_assert(TQ <= 64, "one flag bit per query");
    extern __shared__ uint64_t s_dyn64[];
    const RowGeo g = ix.g;
    const int W = g.W;
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    // blocks are dealt to the 8 XCDs round robin; renumber them so that each
    // XCD holds a contiguous run of logical blocks
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned xcd = b & 7u, q8 = nb >> 3, r8 = nb & 7u;
    const unsigned lb = (xcd < r8 ? xcd * (q8 + 1) : r8 * (q8 + 1) + (xcd - r8) * q8) + (b >> 3);
    const int grp = (int)(lb % (unsigned)sg.qgroups);
    const int pidx = (int)(lb / (unsigned)sg.qgroups) * kScanWaves + wv;
    const int64_t q0i = (int64_t)grp * TQ;
    const int ntq = (int)(qb.Q - q0i < TQ ? qb.Q - q0i : TQ);

    uint32_t* s_q = reinterpret_cast<uint32_t*>(s_dyn64);  // [TQ][W] query words, shared by the block
    const int qwords64 = (TQ * W + 1) / 2;
    ScanFilter* filt = reinterpret_cast<ScanFilter*>(s_dyn64 + qwords64) + wv * TQ;
    uint64_t* lists = s_dyn64 + qwords64 + (size_t)kScanWaves * TQ * (sizeof(ScanFilter) / 8) +
                      (size_t)wv * TQ * sg.lstride;
    for (int t = threadIdx.x; t < TQ * W; t += kScanWaves * kWave)
        s_q[t] = t < ntq * W ? qkeys[q0i * W + t] : 0u;
    __syncthreads();
    if (pidx >= sg.nparts) return;

    const int64_t N = ix.N;
    int64_t r_lo, r_hi;
    if (pidx < sg.seed_chunks) {
        r_lo = (int64_t)pidx * sg.seed_chunk_rows;
        r_hi = r_lo + sg.seed_chunk_rows < sg.seed_rows ? r_lo + sg.seed_chunk_rows : sg.seed_rows;
    } else {
        r_lo = sg.seed_rows + (int64_t)(pidx - sg.seed_chunks) * sg.chunk_rows;
        r_hi = r_lo + sg.chunk_rows < N ? r_lo + sg.chunk_rows : N;
    }
    // pairs of rows [p_lo, p_hi): r_lo is even, and an odd N has a zero entry
    // after its last row; loads past the chunk re-read its last pair.  The
    // first step's loads go out before the filters are set up.
    const uint4* __restrict__ pl = reinterpret_cast<const uint4*>(ix.plane);
    const int64_t p_lo = r_lo >> 1, p_last = ((r_hi + 1) >> 1) - 1;
    uint4 nx[kScanU];
#pragma unroll
    for (int u = 0; u < kScanU; ++u) {
        const int64_t pp = p_lo + u * kWave + lane;
        nx[u] = pl[pp < p_last ? pp : p_last];
    }
    // filters from the starting limits; query slots past the batch get one
    // that nothing matches
    if (lane < TQ) {
        ScanFilter f;
        const bool real = lane < ntq;
        f.lim = real ? gthr[q0i + lane] : kKeyMax;
        const int ki = real ? query_k(qb, q0i + lane) : 1;
        f.kk = (int)((int64_t)ki < N ? (int64_t)ki : N);
        f.pad_ = 0;
        const uint32_t* q = s_q + lane * W;
        const uint64_t q01 = ((uint64_t)q[0] << 32) | (W > 1 ? q[1] : 0u);
        limit_filter(f.lim, r_lo, q01, g, f.msk, f.qm);
        if (!real) {
            f.msk = 0;
            f.qm = 1;
        }
        filt[lane] = f;
    }
    for (int e = lane; e < TQ * sg.lstride; e += kWave) lists[e] = kKeyMax;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // the filters as wave-uniform values (scalar registers), reloaded from
    // LDS only after the slow path or a pick-up of shared limits changed one
    uint64_t fm[TQ], fq[TQ];
    auto load_filters = [&]() {
#pragma unroll
        for (int i = 0; i < TQ; ++i) {
            fm[i] = uniform64(filt[i].msk);
            fq[i] = uniform64(filt[i].qm);
        }
    };
    load_filters();
    int it = 0;
    for (int64_t base = r_lo; base < r_hi; base += kScanStepRows, ++it) {
        if (it > 0 && it % kGthrEvery == 0) {
            // pick up tighter limits reached by other waves: lane i reads query
            // i's limit with a plain load (a stale value only prunes less)
            const uint64_t mine = lane < ntq ? gthr[q0i + lane] : kKeyMax;
#pragma unroll 1
            for (int i = 0; i < ntq; ++i) {
                const uint64_t gv = readlane64(mine, i);
                if (gv < filt[i].lim) {
                    const uint32_t* q = s_q + i * W;
                    const uint64_t q01 = ((uint64_t)q[0] << 32) | (W > 1 ? q[1] : 0u);
                    uint64_t msk, qm;
                    limit_filter(gv, base, q01, g, msk, qm);
                    if (lane == 0) {
                        filt[i].lim = gv;
                        filt[i].msk = msk;
                        filt[i].qm = qm;
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            load_filters();
        }
        // the step's rows, as 64-bit plane values (word 0 high): row
        // base + u * 128 + 2 * lane + h is v[2u + h]
        uint64_t v[2 * kScanU];
#pragma unroll
        for (int u = 0; u < kScanU; ++u) {
            v[2 * u] = ((uint64_t)nx[u].y << 32) | nx[u].x;
            v[2 * u + 1] = ((uint64_t)nx[u].w << 32) | nx[u].z;
        }
        if (base + kScanStepRows < r_hi) {
            const int64_t pn = p_lo + (int64_t)(it + 1) * (kScanU * kWave);
#pragma unroll
            for (int u = 0; u < kScanU; ++u) {
                const int64_t pp = pn + u * kWave + lane;
                nx[u] = pl[pp < p_last ? pp : p_last];
            }
        }
        // hot loop: which queries have a row passing their filter this step.
        // Lanes past the chunk re-read its last pair, so they may flag a
        // query; the slow path drops them.
        uint64_t flagged = 0;
#pragma unroll
        for (int i = 0; i < TQ; ++i) {
            const uint64_t msk = fm[i], qm = fq[i];
            uint64_t any = 0;
            if (msk == ~0ull) {
#pragma unroll
                for (int t = 0; t < 2 * kScanU; ++t) any |= ballot(v[t] == qm);
            } else {
#pragma unroll
                for (int t = 0; t < 2 * kScanU; ++t) any |= ballot((v[t] & msk) == qm);
            }
            flagged |= any ? (1ull << i) : 0ull;
        }
        // slow path, one flagged query at a time, its rows in id order
        const bool any_flagged = flagged != 0;
#pragma unroll 1
        while (flagged) {
            const int i = low_lane(flagged);
            flagged &= flagged - 1;
            const uint32_t* q = s_q + i * W;
            const uint64_t q01 = ((uint64_t)q[0] << 32) | (W > 1 ? q[1] : 0u);
            ScanFilter f = filt[i];
            uint64_t* lp = lists + (size_t)i * sg.lstride;
            WaveList<NR> lst;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const int e = r * kWave + lane;
                lst.v[r] = e < sg.lstride ? lp[e] : kKeyMax;
            }
            bool touched = false;
#pragma unroll 1
            for (int t = 0; t < 2 * kScanU; ++t) {
                uint64_t w = v[0];
#pragma unroll
                for (int tt = 1; tt < 2 * kScanU; ++tt) w = t == tt ? v[tt] : w;
                const int u = t >> 1, h = t & 1;
                const int64_t id = base + u * kPairRows + 2 * lane + h;
                const bool cand = id < r_hi && (w & f.msk) == f.qm;
                if (ballot(cand) == 0) continue;
                touched = true;
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
                const uint64_t key = rank_key(lc, (uint32_t)id);
                lst.offer(key, cand && key < f.lim, f.kk);
                const uint64_t kth = lst.get(f.kk - 1);
                if (kth < f.lim) {
                    f.lim = kth;
                    if (lane == 0) atomicMin((unsigned long long*)(gthr + q0i + i), (unsigned long long)kth);
                }
                // rows still to come: the second row of this pair, or the next pairs
                limit_filter(f.lim, base + u * kPairRows + (h == 0 ? 1 : kPairRows), q01, g, f.msk, f.qm);
            }
            if (touched) {
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const int e = r * kWave + lane;
                    if (e < sg.lstride) lp[e] = lst.v[r];
                }
                if (lane == 0) filt[i] = f;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        if (any_flagged) load_filters();
    }

    // entries above a valid limit cannot be in the answer; each list is
    // ascending, so the kept ones are a prefix.  The wave's own limit is used
    // (the shared one may be tighter, but reading it would cost another round
    // trip; the merge ranks whatever is kept).  Lane i counts query i's and
    // reserves room for them with one atomic for all the wave's queries.
    int mine = 0;
#pragma unroll 1
    for (int i = 0; i < ntq; ++i) {
        const int kk = filt[i].kk;
        const uint64_t keep = filt[i].lim;
        const uint64_t* lp = lists + (size_t)i * sg.lstride;
        int n = 0;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int e = r * kWave + lane;
            const uint64_t x = e < kk ? lp[e] : kKeyMax;
            n += popc64(ballot(x != kKeyMax && x <= keep));
        }
        mine = lane == i ? n : mine;
    }
    uint32_t at = 0;
    if (lane < ntq && mine > 0) at = atomicAdd(cnt + (q0i + lane) * kCntStride, (uint32_t)mine);
#pragma unroll 1
    for (int i = 0; i < ntq; ++i) {
        const int n = readlane_i(mine, i);
        if (n == 0) continue;
        uint64_t* dst = part + (q0i + i) * cap + (uint32_t)readlane_i((int)at, i);
        const uint64_t* lp = lists + (size_t)i * sg.lstride;
        for (int e = lane; e < n; e += kWave) dst[e] = lp[e];
    }
}

// Merge each query's partial list (cnt[q] entries) into its answer.
constexpr int kMergeFew = 16;        // answers at most this many, from at most
constexpr int64_t kMergeFewMax = 4096;  // this many entries: repeated wave minima instead of the list
template <int NR>
__global__ __launch_bounds__(kScanWaves * kWave) void k_scan_merge(QueryBatch qb, int64_t N, int64_t cap,
                                                                   const uint64_t* __restrict__ part,
                                                                   const uint32_t* __restrict__ cnt) {
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t qi = (int64_t)blockIdx.x * kScanWaves + wv;
    if (qi >= qb.Q) return;
    const int k = query_k(qb, qi);
    const int m = (int)((int64_t)k < N ? (int64_t)k : N);
    const int64_t total = (int64_t)cnt[qi * kCntStride];
    const uint64_t* src = part + qi * cap;
    int32_t* oid = qb.out_ids + query_off(qb, qi);
    int32_t* olc = qb.out_lcp + query_off(qb, qi);
    constexpr int kMergeUnroll = 8;
    if (m <= kMergeFew && total <= kMergeFewMax) {
        // few answers: passes over the entries, each lane sorting at most 8
        // keys, then m rounds take the smallest of the lanes' heads (the
        // 64-bit minimum as two 32-bit wave minima: high words, then the low
        // words of the heads with that high word; keys are distinct) and the
        // lane holding it drops it.  The first pass reads 512 entries; each
        // later pass reads 448 and carries the winners so far in the last
        // register of lanes 0..m-1.
        uint64_t mine = kKeyMax;  // lane e keeps the e-th smallest so far
        for (int64_t b = 0; b < total;) {
            const int fresh = b == 0 ? kMergeUnroll : kMergeUnroll - 1;
            uint64_t key[kMergeUnroll];
#pragma unroll
            for (int u = 0; u < kMergeUnroll; ++u) {
                const int64_t t = b + u * kWave + lane;
                key[u] = u < fresh && t < total ? src[t] : kKeyMax;
            }
            if (fresh < kMergeUnroll) key[kMergeUnroll - 1] = mine;
            b += (int64_t)fresh * kWave;
            uint64_t h0 = key[0], h1 = key[1], h2 = key[2], h3 = key[3];
            uint64_t h4 = key[4], h5 = key[5], h6 = key[6], h7 = key[7];
#define LCPX_CE64(x, y)                            \
    {                                              \
        const uint64_t lo_ = x < y ? x : y;        \
        y = x < y ? y : x;                         \
        x = lo_;                                   \
    }
            LCPX_CE64(h0, h1) LCPX_CE64(h2, h3) LCPX_CE64(h4, h5) LCPX_CE64(h6, h7) LCPX_CE64(h0, h2)
            LCPX_CE64(h1, h3) LCPX_CE64(h4, h6) LCPX_CE64(h5, h7) LCPX_CE64(h1, h2) LCPX_CE64(h5, h6)
            LCPX_CE64(h0, h4) LCPX_CE64(h1, h5) LCPX_CE64(h2, h6) LCPX_CE64(h3, h7) LCPX_CE64(h2, h4)
            LCPX_CE64(h3, h5) LCPX_CE64(h1, h2) LCPX_CE64(h3, h4) LCPX_CE64(h5, h6)
#undef LCPX_CE64
            for (int e = 0; e < m; ++e) {
                const uint32_t hh = (uint32_t)(h0 >> 32);
                const uint32_t mh = wave_min_u32(hh);
                const uint32_t ml = wave_min_u32(hh == mh ? (uint32_t)h0 : 0xFFFFFFFFu);
                const uint64_t v = ((uint64_t)mh << 32) | ml;
                if (lane == e) mine = v;
                if (h0 == v && v != kKeyMax) {  // one lane (fewer than m entries leave only kKeyMax)
                    h0 = h1;
                    h1 = h2;
                    h2 = h3;
                    h3 = h4;
                    h4 = h5;
                    h5 = h6;
                    h6 = h7;
                    h7 = kKeyMax;
                }
            }
        }
        if (lane < m) {
            oid[lane] = key_id(mine);
            olc[lane] = key_lcp(mine);
        }
        for (int e = m + lane; e < k; e += kWave) {
            oid[e] = -1;
            olc[e] = -1;
        }
        return;
    }
    WaveList<NR> lst;
    lst.init();
    for (int64_t b = 0; b < total; b += kMergeUnroll * kWave) {
        uint64_t key[kMergeUnroll];
#pragma unroll
        for (int u = 0; u < kMergeUnroll; ++u) {  // all loads in flight before any is used
            const int64_t t = b + u * kWave + lane;
            key[u] = t < total ? src[t] : kKeyMax;
        }
#pragma unroll 1
        for (int u = 0; u < kMergeUnroll && b + u * kWave < total; ++u) {  // one copy of the offer code
            uint64_t x = key[0];
#pragma unroll
            for (int uu = 1; uu < kMergeUnroll; ++uu) x = u == uu ? key[uu] : x;
            lst.offer(x, x != kKeyMax, m);
        }
    }
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

// Bytes of LDS a scan block needs: the query words, then per wave TQ filters
// and TQ lists of k_max entries.
static size_t scan_block_lds(int tq, int32_t k_max, int W) {
    return ((size_t)tq * W * sizeof(uint32_t) + 7) / 8 * 8 +
           (size_t)kScanWaves * tq * (sizeof(ScanFilter) + (size_t)k_max * sizeof(uint64_t));
}
constexpr size_t kScanLdsBudget = 40 << 10;  // per block: at least 4 blocks (16 waves) per CU

// Queries per wave, from the compiled set for the list size: the fewest
// (query slot, row) tests for the batch, then the most queries per wave,
// within the LDS budget (one query per wave always fits).
static int tq_for(int nr, int32_t k_max, int64_t Q, int W) {
    static const int c1[] = {16, 8, 2, 1}, c2[] = {8, 1}, c4[] = {4, 1}, c16[] = {1};
    const int* c = nr == 1 ? c1 : nr == 2 ? c2 : nr == 4 ? c4 : c16;
    const int n = nr == 1 ? 4 : nr == 16 ? 1 : 2;
    int best = 1;
    int64_t best_slots = Q;
    for (int i = n - 1; i >= 0; --i) {  // ascending tq: a larger one wins ties
        const int tq = c[i];
        if (tq > 1 && scan_block_lds(tq, k_max, W) > kScanLdsBudget) continue;
        const int64_t slots = (Q + tq - 1) / tq * tq;
        if (slots <= best_slots) {
            best = tq;
            best_slots = slots;
        }
    }
    return best;
}

// Rows sampled for the starting limits, and the main pass's chunking.
constexpr int64_t kChunkMinRows = 2 * kScanStepRows;
constexpr int64_t kSeedRows = 65536;
constexpr int64_t kScanTargetWaves = 8192;  // 32 per CU

ScanPlan plan_scan(int64_t N, int W, int64_t Q, int32_t k_max, int64_t part_budget_bytes) {
    ScanPlan p;
    p.nr = nr_for(k_max);
    p.tq = tq_for(p.nr, k_max, Q, W);
    p.qgroups = (int)((Q + p.tq - 1) / p.tq);
    // the sample: 65,536 rows, and for batches of at most 1,024 queries up to
    // 1/32 of a larger database (at most 262,144 rows), so that the starting
    // limits stay as tight on large databases (the sample's cost grows with
    // Q times its size)
    int64_t S = kSeedRows;
    if (Q <= 1024) {
        const int64_t big = (N / 32 + kScanStepRows - 1) / kScanStepRows * kScanStepRows;
        S = big > S ? (big < 4 * kSeedRows ? big : 4 * kSeedRows) : S;
    }
    p.seed_rows = N < S ? N : S;
    // seed blocks per query: enough blocks in all to fill the device, but at
    // most 32, since every block adds its counts to the query's histogram
    // with global atomics on the same few addresses
    const int64_t seed_tiles = (p.seed_rows + 255) / 256;
    int64_t parts = Q > 0 ? 4096 / Q : 1;
    if (parts > 32) parts = 32;
    if (parts > seed_tiles) parts = seed_tiles;
    p.seed_parts = (int)(parts < 1 ? 1 : parts);
    const int64_t bytes_per_chunk = Q * (int64_t)k_max * 8;
    const int64_t max_by_mem = bytes_per_chunk > 0 ? part_budget_bytes / bytes_per_chunk : 1;
    if (max_by_mem < 2) {  // one seed chunk and one row chunk per query do not fit
        p.seed_chunks = p.chunks = p.nparts = 0;
        p.seed_chunk_rows = p.chunk_rows = 0;
        return p;
    }
    // sampled rows: one-step waves while the grid stays near the target,
    // fewer and longer ones for many query groups or a tight partial budget
    int64_t sc = (p.seed_rows + kScanStepRows - 1) / kScanStepRows;
    const int64_t by_grid = kScanTargetWaves / 2 / p.qgroups;
    if (sc > by_grid) sc = by_grid;
    if (sc > max_by_mem / 2) sc = max_by_mem / 2;
    if (sc < 1) sc = 1;
    p.seed_chunk_rows = (p.seed_rows + sc - 1) / sc;
    p.seed_chunk_rows = (p.seed_chunk_rows + kScanStepRows - 1) / kScanStepRows * kScanStepRows;
    p.seed_chunks = (int)((p.seed_rows + p.seed_chunk_rows - 1) / p.seed_chunk_rows);
    // main: rows [seed_rows, N); aim for the target wave count, chunks of at
    // least kChunkMinRows rows (whole steps), partials within the budget
    const int64_t rest = N - p.seed_rows;
    if (rest <= 0) {
        p.chunk_rows = kChunkMinRows;
        p.chunks = 0;
    } else {
        int64_t chunks = (kScanTargetWaves + p.qgroups - 1) / p.qgroups;
        const int64_t max_by_rows = (rest + kChunkMinRows - 1) / kChunkMinRows;
        if (chunks > max_by_rows) chunks = max_by_rows;
        if (chunks > max_by_mem - p.seed_chunks) chunks = max_by_mem - p.seed_chunks;
        if (chunks < 1) chunks = 1;
        int64_t rows = (rest + chunks - 1) / chunks;
        rows = (rows + kScanStepRows - 1) / kScanStepRows * kScanStepRows;
        p.chunk_rows = rows;
        p.chunks = (int)((rest + rows - 1) / rows);
    }
    p.nparts = p.seed_chunks + p.chunks;
    return p;
}

ScanScratch scan_scratch(const ScanPlan& p, int64_t Q, int32_t k_max, const RowGeo& g, uint64_t* base) {
    ScanScratch sc;
    sc.cap = (int64_t)p.nparts * k_max;
    sc.part = base;
    sc.gthr = base + (size_t)Q * (size_t)sc.cap;
    uint32_t* u = reinterpret_cast<uint32_t*>(sc.gthr + Q);
    sc.cnt = u;                                // [Q][kCntStride], entry 0 used; zeroed per call
    sc.hist = u + (size_t)Q * kCntStride;      // [Q][L+1] zeroed per call
    sc.qkeys = sc.hist + (size_t)Q * (g.L + 1);  // [Q][W]
    sc.words = ((size_t)Q * (size_t)sc.cap + (size_t)Q) * 2 + (size_t)Q * (kCntStride + (g.L + 1) + g.W);
    return sc;
}

size_t scan_partial_entries(const ScanPlan& p, int64_t Q, int32_t k_max, const RowGeo& g) {
    return (scan_scratch(p, Q, k_max, g, nullptr).words + 1) / 2;
}

template <int NR, int TQ>
static void launch_scan_t(const IndexView& ix, const QueryBatch& qb, const ScanPlan& p, const ScanScratch& sc,
                          int32_t k_max, hipStream_t s) {
    ScanGrid sg;
    sg.seed_rows = p.seed_rows;
    sg.seed_chunk_rows = p.seed_chunk_rows;
    sg.chunk_rows = p.chunk_rows;
    sg.nparts = p.nparts;
    sg.seed_chunks = p.seed_chunks;
    sg.qgroups = p.qgroups;
    sg.lstride = k_max;
    const size_t shm = scan_block_lds(TQ, k_max, ix.g.W);
    const int64_t blocks = (int64_t)p.qgroups * ((p.nparts + kScanWaves - 1) / kScanWaves);
    hipLaunchKernelGGL((k_scan<NR, TQ>), dim3((unsigned)blocks), dim3(kScanWaves * kWave), shm, s, ix, qb, sc.qkeys,
                       sg, sc.cap, sc.part, sc.cnt, sc.gthr);
}

hipError_t launch_scan(const IndexView& ix, const QueryBatch& qb, const ScanPlan& p, uint64_t* scratch, hipStream_t s,
                       hipEvent_t ev0, hipEvent_t ev1, hipEvent_t ev2) {
    if (qb.Q <= 0) return hipSuccess;
    const ScanScratch sc = scan_scratch(p, qb.Q, qb.k_max, ix.g, scratch);
    const int64_t nz = qb.Q * (int64_t)(kCntStride + ix.g.L + 1);  // cnt and hist
    const int64_t nprep = nz > qb.Q * ix.g.W ? nz : qb.Q * ix.g.W;
    hipLaunchKernelGGL(k_scan_prep, dim3((unsigned)((nprep + 255) / 256)), dim3(256), 0, s, qb, ix.g, sc.cnt, nz,
                       sc.qkeys);
    hipLaunchKernelGGL(k_seed_hist, dim3((unsigned)(qb.Q * p.seed_parts)), dim3(kSeedThreads), 0, s, ix, sc.qkeys,
                       p.seed_rows, p.seed_parts, sc.hist);
    hipLaunchKernelGGL(k_seed_limit, dim3((unsigned)((qb.Q + kScanWaves - 1) / kScanWaves)), dim3(kScanWaves * kWave),
                       0, s, qb, ix.N, ix.g.L, p.seed_rows, sc.hist, sc.gthr);
    if (ev0) hipEventRecord(ev0, s);
    switch (p.nr * 100 + p.tq) {
        case 116: launch_scan_t<1, 16>(ix, qb, p, sc, qb.k_max, s); break;
        case 108: launch_scan_t<1, 8>(ix, qb, p, sc, qb.k_max, s); break;
        case 102: launch_scan_t<1, 2>(ix, qb, p, sc, qb.k_max, s); break;
        case 101: launch_scan_t<1, 1>(ix, qb, p, sc, qb.k_max, s); break;
        case 208: launch_scan_t<2, 8>(ix, qb, p, sc, qb.k_max, s); break;
        case 201: launch_scan_t<2, 1>(ix, qb, p, sc, qb.k_max, s); break;
        case 404: launch_scan_t<4, 4>(ix, qb, p, sc, qb.k_max, s); break;
        case 401: launch_scan_t<4, 1>(ix, qb, p, sc, qb.k_max, s); break;
        case 1601: launch_scan_t<16, 1>(ix, qb, p, sc, qb.k_max, s); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev1) hipEventRecord(ev1, s);
    const unsigned grid = (unsigned)((qb.Q + kScanWaves - 1) / kScanWaves);
    const dim3 blk(kScanWaves * kWave);
    switch (p.nr) {
        case 1: hipLaunchKernelGGL((k_scan_merge<1>), dim3(grid), blk, 0, s, qb, ix.N, sc.cap, sc.part, sc.cnt); break;
        case 2: hipLaunchKernelGGL((k_scan_merge<2>), dim3(grid), blk, 0, s, qb, ix.N, sc.cap, sc.part, sc.cnt); break;
        case 4: hipLaunchKernelGGL((k_scan_merge<4>), dim3(grid), blk, 0, s, qb, ix.N, sc.cap, sc.part, sc.cnt); break;
        default:
            hipLaunchKernelGGL((k_scan_merge<16>), dim3(grid), blk, 0, s, qb, ix.N, sc.cap, sc.part, sc.cnt);
            break;
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev2) hipEventRecord(ev2, s);
    return hipSuccess;
}

}  // namespace lcpx
