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


// Starting limits from the first S rows (ids 0..S-1), cut into `parts`
// consecutive id ranges.  hist[q][p][d] counts the rows of part p with LCP
// exactly d.  With t the largest d such that at least k' sample rows have
// LCP >= d, and p* the first part at whose end the sample rows with LCP > t
// plus those of parts 0..p* with LCP == t number at least k', those k' rows
// have keys <= rank_key(t, X - 1), X the end of part p*: the answer's k'-th
// key is below rank_key(t, X), every answer row beats that key, and it
// becomes the query's limit (rows with LCP == t after X need not be looked
// at).  Block b counts part b % parts of the sample for query b / parts.
//
// The 8-byte plane decides every LCP below cmax, the tokens it holds: each
// wave counts its rows with LCP >= d for d = 1..cmax with one ballot per level
// (no per-row histogram updates), and only rows that agree with the query on
// all cmax tokens read the rest of the row and add to the histogram one by one.
constexpr int kSeedThreads = 256;
constexpr int kSeedU = 8;
constexpr int kSeedLevels = 8;  // cmax <= 8 (eight 1-byte tokens in the plane)
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
    const int plane_tokens = (g.W > 1 ? 8 : 4) / g.tb;
    const int cmax = g.L < plane_tokens ? g.L : plane_tokens;
    const uint32_t q0 = qw[0], q1 = g.W > 1 ? qw[1] : 0u;
    uint32_t rows = 0;
    uint32_t ge[kSeedLevels];  // ge[d - 1]: this wave's rows with LCP >= d (wave-uniform)
#pragma unroll
    for (int d = 0; d < kSeedLevels; ++d) ge[d] = 0;
    // kSeedU rows per thread and round, all loads in flight before any is used
    for (int64_t base = r0; base < r1; base += (int64_t)kSeedThreads * kSeedU) {
        uint64_t pw[kSeedU];
#pragma unroll
        for (int u = 0; u < kSeedU; ++u) {
            const int64_t r = base + u * kSeedThreads + threadIdx.x;
            pw[u] = r < r1 ? ix.plane[r] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < kSeedU; ++u) {
            const int64_t r = base + u * kSeedThreads + threadIdx.x;
            const bool act = r < r1;
            const uint32_t x0 = (uint32_t)(pw[u] >> 32) ^ q0, x1 = (uint32_t)pw[u] ^ q1;
            const int lc = x0 ? lcp_from_diff(0, x0, g) : x1 ? lcp_from_diff(1, x1, g) : cmax;
            rows += (uint32_t)popc64(ballot(act));
#pragma unroll
            for (int d = 1; d <= kSeedLevels; ++d)
                if (d <= cmax) ge[d - 1] += (uint32_t)popc64(ballot(act && lc >= d));
            if (act && lc == cmax && g.L > cmax) {  // the rest of the row decides
                const uint32_t* row = ix.rows + r * g.W;
                int full = g.L;
                for (int w = 2; w < g.W; ++w) {
                    const uint32_t x = row[w] ^ qw[w];
                    if (x) {
                        full = lcp_from_diff(w, x, g);
                        break;
                    }
                }
                atomicAdd(&h[full], 1u);
            }
        }
    }
    // exact counts below cmax from the level counts; at cmax itself only when
    // the plane holds the whole row
    if (lane == 0) {
        uint32_t above = rows;
        for (int d = 1; d <= cmax; ++d) {
            const uint32_t cur = ge[d - 1];
            if (above - cur) atomicAdd(&h[d - 1], above - cur);
            above = cur;
        }
        if (g.L == cmax && above) atomicAdd(&h[cmax], above);
    }
    __syncthreads();
    uint32_t* hq = hist + ((size_t)qi * parts + part) * (g.L + 1);  // this block's own histogram
    for (int i = threadIdx.x; i <= g.L; i += kSeedThreads) hq[i] = h[i];
}

// One wave per query.  Lane i takes d = top - i and sums that level over the
// parts, so the wave's inclusive prefix sum at lane i counts the sample rows
// with LCP in [d, top] (plus the rows above top from earlier passes); the
// first lane where it reaches k' gives t.  Then lane p takes part p's rows at
// LCP t, and the first lane where the rows above t plus the prefix sum reach
// k' gives p*.
__global__ __launch_bounds__(kScanWaves * kWave) void k_seed_limit(QueryBatch qb, int64_t N, int L, int64_t S,
                                                                   int parts, const uint32_t* __restrict__ hist,
                                                                   uint64_t* __restrict__ gthr) {
    const int lane = lane_id();
    const int64_t qi = (int64_t)blockIdx.x * kScanWaves + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (qi >= qb.Q) return;
    const int k = query_k(qb, qi);
    const uint32_t kk = (uint32_t)((int64_t)k < N ? (int64_t)k : N);
    const uint32_t* h = hist + qi * (int64_t)parts * (L + 1);
    uint64_t lim = kKeyMax;
    uint32_t above = 0;  // sample rows with LCP above this pass's top
    for (int top = L; top >= 0; top -= kWave) {
        const int d = top - lane;
        uint32_t c = 0;
        if (d >= 0) {
#pragma unroll 8
            for (int p = 0; p < parts; ++p) c += h[(int64_t)p * (L + 1) + d];
        }
        const uint32_t acc = wave_prefix_sum(c) + above;
        const uint64_t ok = ballot(d >= 0 && acc >= kk);
        if (ok) {
            const int i = low_lane(ok);
            const int t = top - i;
            const uint32_t gt = readlane(acc, i) - readlane(c, i);  // sample rows with LCP > t
            const uint32_t ct = lane < parts ? h[(int64_t)lane * (L + 1) + t] : 0u;
            const uint64_t reach = ballot(lane < parts && wave_prefix_sum(ct) + gt >= kk);
            const int64_t per = (S + parts - 1) / parts;
            const int64_t end = (int64_t)(low_lane(reach) + 1) * per;
            lim = rank_key(t, (uint32_t)(end < S ? end : S));
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

// One launch before the scan: zero the fill counts (a kernel, not a memset,
// so the sequence can be captured in a graph) and compute the query key words
// once for every block to copy.
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
// Which rows need a closer look is decided in two ways:
//  - a hash pre-filter (the hashed variants, for large groups): the block puts each
//    query's filter at its starting limit (a looser filter than any the waves
//    reach later) into one of two small hash tables in LDS, one per mask
//    length, keyed by the masked query value; per row and table the hot loop
//    costs one hash, one LDS read and two 64-bit compares however many
//    queries the table holds; each slot also holds the set of queries whose
//    keys fall in it, and a step with a hit tests the queries of the matched
//    slots one by one.  Queries that do not fit (a third mask length, a full
//    slot, no limit) are tested one by one on every step;
//  - one by one: the query's current filter (lane i holds query i's) against
//    the step's rows, one 64-bit compare per row, and two ANDs when the
//    filter keeps part of the 64 bits.
// Both only select candidates: a flagged query's rows are re-tested against
// its current filter in the slow path, which computes exact LCPs and offers
// them to the query's list in LDS.
//
// At the end each wave appends, per query, the entries of its list that do
// not exceed the query's limit to the query's partial list (cap entries at
// part + q * cap, fill count in cnt[q]); the append order does not matter,
// the merge ranks by key.
constexpr int kScanU = 4;                                  // 16-byte loads per lane per step
constexpr int kQwRegs = 4;                                 // query words per thread fetched with the first loads
constexpr int64_t kPairRows = 2 * kWave;                   // rows of one 16-byte load of the wave
constexpr int64_t kScanStepRows = kScanU * kPairRows;      // rows per wave step
constexpr int kGthrEvery = 4;                              // steps between pick-ups of shared limits
constexpr int kHashTables = 2;
constexpr int kHashSlots = 128;                            // two keys each
constexpr uint64_t kHashEmpty = ~0ull;                     // an empty slot's keys (a row equal to it only costs a test)

// Block-shared pre-filter state in LDS.
struct ScanHash {
    uint4 slot[kHashTables][kHashSlots];     // (key0 lo, key0 hi, key1 lo, key1 hi)
    uint64_t qbits[kHashTables][kHashSlots];  // the queries whose key falls in the slot
    uint64_t mask[kHashTables];
    uint64_t left;  // queries tested one by one on every step
    int32_t ntab;
    int32_t pad_;
};

// Shifts and XORs only (full-rate VALU operations; a 32-bit multiply issues
// at a quarter of the rate).
__device__ __forceinline__ uint32_t hash_slot(uint64_t key) {
    uint32_t x = (uint32_t)(key >> 32) ^ (uint32_t)key;
    x ^= x >> 16;
    x ^= x >> 7;
    return x & (kHashSlots - 1);
}

template <int NR, int TQ, bool kHash>
__global__ __launch_bounds__(kScanWaves * kWave) __attribute__((amdgpu_waves_per_eu(NR == 1 ? 6 : 1))) void k_scan(IndexView ix, QueryBatch qb,
                                                             const uint32_t* __restrict__ qkeys, ScanGrid sg,
                                                             int64_t cap, uint64_t* __restrict__ part,
                                                             uint32_t* __restrict__ cnt,
                                                             uint64_t* __restrict__ gthr) {
    static_assert(TQ <= 64, "one lane and one flag bit per query");
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
    const int pidx0 = (int)(lb / (unsigned)sg.qgroups) * kScanWaves;
    const int pidx = pidx0 + wv;
    const int64_t q0i = (int64_t)grp * TQ;
    const int ntq = (int)(qb.Q - q0i < TQ ? qb.Q - q0i : TQ);
    const uint64_t real = ntq >= 64 ? ~0ull : (1ull << ntq) - 1;
    const int64_t N = ix.N;

    // rows of part p: the seed chunks first (sampled rows: their looser
    // filters leave them most of the slow-path work, and in the first blocks
    // dispatched that work overlaps the rest of the pass instead of trailing
    // it), then the main chunks
    auto chunk_rows_of = [&](int p, int64_t& lo, int64_t& hi) {
        if (p < sg.seed_chunks) {
            lo = (int64_t)p * sg.seed_chunk_rows;
            hi = lo + sg.seed_chunk_rows < sg.seed_rows ? lo + sg.seed_chunk_rows : sg.seed_rows;
        } else {
            lo = sg.seed_rows + (int64_t)(p - sg.seed_chunks) * sg.chunk_rows;
            hi = lo + sg.chunk_rows < N ? lo + sg.chunk_rows : N;
        }
    };

    // everything the set-up reads from memory is requested first, in one
    // round trip with the first plane loads: the group's query words (up to
    // kQwRegs per thread here, the rest below), and lane i's query limit and k
    const int nqw = ntq * W;
    uint32_t qwr[kQwRegs];
#pragma unroll
    for (int j = 0; j < kQwRegs; ++j) {
        const int t = j * kScanWaves * kWave + (int)threadIdx.x;
        qwr[j] = t < nqw ? qkeys[q0i * W + t] : 0u;
    }
    // (clamped indices instead of masked loads: no branch, so nothing waits
    // for these before the plane loads go out)
    const bool lane_real = lane < ntq;
    const int lq_idx = lane_real ? lane : 0;
    const uint64_t lim_ld = gthr[q0i + lq_idx];
    int k_ld = qb.k_uniform;
    if (qb.k_uniform <= 0) k_ld = qb.k[q0i + lq_idx];

    // the wave's rows [r_lo, r_hi) as pairs [p_lo, p_last]: r_lo is even, and
    // an odd N has a zero entry after its last row; loads past the chunk
    // re-read its last pair.  The first step's loads go out before any of the
    // set-up below (waves past the last chunk only help set up the block).
    const bool active = pidx < sg.nparts;
    int64_t r_lo = 0, r_hi = 1;  // a wave past the last chunk loads row 0 and leaves after the set-up
    if (active) chunk_rows_of(pidx, r_lo, r_hi);
    const uint4* __restrict__ pl = reinterpret_cast<const uint4*>(ix.plane);
    const int64_t p_lo = r_lo >> 1, p_last = ((r_hi + 1) >> 1) - 1;
    uint4 nx[kScanU];
#pragma unroll
    for (int u = 0; u < kScanU; ++u) {
        const int64_t pp = p_lo + u * kWave + lane;
        nx[u] = pl[pp < p_last ? pp : p_last];
    }
    const uint64_t lim0 = lane_real ? lim_ld : kKeyMax;
    uint64_t published = lim0;  // lane i: query i's limit as this wave last made it shared

    // LDS: [TQ][W] query words, the pre-filter (hashed variants), then per
    // wave [TQ] filters and [TQ][lstride] list entries
    uint32_t* s_q = reinterpret_cast<uint32_t*>(s_dyn64);
    const int qwords64 = (TQ * W + 3) / 4 * 2;  // 16-byte aligned
    ScanHash* hs = reinterpret_cast<ScanHash*>(s_dyn64 + qwords64);
    const int hash64 = kHash ? (int)(sizeof(ScanHash) / 8) : 0;
    ScanFilter* filt = reinterpret_cast<ScanFilter*>(s_dyn64 + qwords64 + hash64) + wv * TQ;
    uint64_t* lists = s_dyn64 + qwords64 + hash64 + (size_t)kScanWaves * TQ * (sizeof(ScanFilter) / 8) +
                      (size_t)wv * TQ * sg.lstride;
#pragma unroll
    for (int j = 0; j < kQwRegs; ++j) {
        const int t = j * kScanWaves * kWave + (int)threadIdx.x;
        if (t < TQ * W) s_q[t] = qwr[j];
    }
    for (int t = kQwRegs * kScanWaves * kWave + (int)threadIdx.x; t < TQ * W; t += kScanWaves * kWave)
        s_q[t] = t < nqw ? qkeys[q0i * W + t] : 0u;
    if constexpr (kHash) {
        for (int t = threadIdx.x; t < kHashTables * kHashSlots; t += kScanWaves * kWave) {
            (&hs->slot[0][0])[t] = make_uint4(~0u, ~0u, ~0u, ~0u);
            (&hs->qbits[0][0])[t] = 0ull;
        }
    }
    __syncthreads();
    if constexpr (kHash) {
        if (wv == 0) {
            // the filters at the starting limits, for the rows from the
            // block's first chunk on (the loosest any of its waves uses)
            uint64_t msk = 0, qm = 1;
            if (lane < ntq) {
                const uint32_t* q = s_q + lane * W;
                const uint64_t q01 = ((uint64_t)q[0] << 32) | (W > 1 ? q[1] : 0u);
                int64_t first = N;  // the block's first row
                for (int j = 0; j < kScanWaves && pidx0 + j < sg.nparts; ++j) {
                    int64_t lo, hi;
                    chunk_rows_of(pidx0 + j, lo, hi);
                    first = lo < first ? lo : first;
                }
                limit_filter(lim0, first, q01, g, msk, qm);
            }
            // up to two mask lengths get a table; a query without a limit
            // (mask 0) or with another mask length is tested one by one
            const bool cand = lane < ntq && msk != 0;
            int tab = -1;
            uint64_t m0 = 0, m1 = 0;
            uint64_t pend = ballot(cand);
            int ntab = 0;
            if (pend) {
                m0 = readlane64(msk, low_lane(pend));
                tab = cand && msk == m0 ? 0 : tab;
                ntab = 1;
                pend &= ~ballot(cand && msk == m0);
                if (pend) {
                    m1 = readlane64(msk, low_lane(pend));
                    tab = cand && msk == m1 ? 1 : tab;
                    ntab = 2;
                }
            }
            // join the slot's query set; the queries already in it give the
            // place: the first key of a slot also fills its second place, a
            // second key then overwrites that place, later ones go one by one
            uint32_t sl = tab >= 0 ? hash_slot(qm) : 0u;
            uint32_t pos = 2;
            if (tab >= 0)
                pos = (uint32_t)popc64(atomicOr((unsigned long long*)&hs->qbits[tab][sl], 1ull << lane));
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (pos == 0) hs->slot[tab][sl] = make_uint4((uint32_t)qm, (uint32_t)(qm >> 32), (uint32_t)qm,
                                                         (uint32_t)(qm >> 32));
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (pos == 1) {
                hs->slot[tab][sl].z = (uint32_t)qm;
                hs->slot[tab][sl].w = (uint32_t)(qm >> 32);
            }
            const uint64_t left = ballot(lane < ntq && pos >= 2);
            if (lane == 0) {
                hs->mask[0] = m0;
                hs->mask[1] = m1;
                hs->ntab = ntab;
                hs->left = left;
            }
        }
        __syncthreads();
    }
    if (!active) return;

    // the wave's filters from the starting limits; query slots past the batch
    // get one that nothing matches
    if (lane < TQ) {
        ScanFilter f;
        const bool is_real = lane < ntq;
        f.lim = lim0;
        const int ncap = N < 0x7fffffff ? (int)N : 0x7fffffff;
        f.kk = is_real ? (k_ld < ncap ? k_ld : ncap) : 1;
        f.pad_ = 0;
        const uint32_t* q = s_q + lane * W;
        const uint64_t q01 = ((uint64_t)q[0] << 32) | (W > 1 ? q[1] : 0u);
        limit_filter(f.lim, r_lo, q01, g, f.msk, f.qm);
        if (!is_real) {
            f.msk = 0;
            f.qm = 1;
        }
        filt[lane] = f;
    }
    for (int e = lane; e < TQ * sg.lstride; e += kWave) lists[e] = kKeyMax;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // lane i holds query i's current filter; reloaded after any change
    uint64_t lm = 0, lq = 1;
    auto load_filters = [&]() {
        if (lane < TQ) {
            lm = filt[lane].msk;
            lq = filt[lane].qm;
        }
    };
    load_filters();
    uint64_t hmask[kHashTables] = {0, 0};
    int ntab = 0;
    uint64_t one_by_one = real;
    if constexpr (kHash) {
        hmask[0] = uniform64(hs->mask[0]);
        hmask[1] = uniform64(hs->mask[1]);
        ntab = (int)uniform((uint32_t)hs->ntab);
        one_by_one = uniform64(hs->left) & real;
    }
    const uint64_t hashed = real & ~one_by_one;

    int it = 0;
    for (int64_t base = r_lo; base < r_hi; base += kScanStepRows, ++it) {
        if (it > 0 && it % kGthrEvery == 0) {
            // publish the limits this wave tightened since the last time, and
            // pick up tighter ones reached by other waves: lane i reads query
            // i's limit with a plain load (a stale value only prunes less)
            if (lane < ntq) {
                const uint64_t mylim = filt[lane].lim;
                if (mylim < published) {
                    atomicMin((unsigned long long*)(gthr + q0i + lane), (unsigned long long)mylim);
                    published = mylim;
                }
            }
            const uint64_t mine = lane < ntq ? gthr[q0i + lane] : kKeyMax;
            bool changed = false;
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
                    changed = true;
                }
            }
            if (changed) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                load_filters();
            }
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
        // which queries have a row passing their filter this step.  Lanes
        // past the chunk re-read its last pair, so they may flag a query; the
        // slow path drops them.
        uint64_t test = one_by_one;
        if constexpr (kHash) {
            uint64_t hitq = 0;
#pragma unroll 1
            for (int t0 = 0; t0 < ntab; ++t0) {
                const uint64_t m = hmask[t0];
                const uint4* tab = hs->slot[t0];
                uint64_t hit = 0;
                if (m == ~0ull) {
#pragma unroll
                    for (int t = 0; t < 2 * kScanU; ++t) {
                        const uint4 e = tab[hash_slot(v[t])];
                        hit |= ballot(v[t] == (((uint64_t)e.y << 32) | e.x));
                        hit |= ballot(v[t] == (((uint64_t)e.w << 32) | e.z));
                    }
                } else {
#pragma unroll
                    for (int t = 0; t < 2 * kScanU; ++t) {
                        const uint64_t key = v[t] & m;
                        const uint4 e = tab[hash_slot(key)];
                        hit |= ballot(key == (((uint64_t)e.y << 32) | e.x));
                        hit |= ballot(key == (((uint64_t)e.w << 32) | e.z));
                    }
                }
                if (hit) {
                    // rare: collect the query sets of the matched slots, so
                    // that only those queries are tested one by one
#pragma unroll 1
                    for (int t = 0; t < 2 * kScanU; ++t) {
                        uint64_t w = v[0];
#pragma unroll
                        for (int tt = 1; tt < 2 * kScanU; ++tt) w = t == tt ? v[tt] : w;
                        const uint64_t key = w & m;
                        const uint32_t sl = hash_slot(key);
                        const uint4 e = tab[sl];
                        const uint64_t k0 = ((uint64_t)e.y << 32) | e.x, k1 = ((uint64_t)e.w << 32) | e.z;
                        const bool match = key == k0 || key == k1;
                        const uint64_t qs = match ? hs->qbits[t0][sl] : 0ull;
                        for (uint64_t mm = ballot(match); mm; mm &= mm - 1) hitq |= readlane64(qs, low_lane(mm));
                    }
                }
            }
            test |= hitq & hashed;
        }
        uint64_t flagged = 0;
#pragma unroll 1
        for (uint64_t todo = test; todo; todo &= todo - 1) {
            const int i = low_lane(todo);
            const uint64_t msk = readlane64(lm, i), qm = readlane64(lq, i);
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
        // slow path, one flagged query at a time, its rows in id order.  A row
        // that agrees with the query on the whole plane needs the row's next
        // words: each lane fetches words 2-3 of its first such row (for any
        // flagged query) once for the step, so that one round trip serves
        // them all; a lane's further such rows read theirs on their own.
        const bool any_flagged = flagged != 0;
        int tail_t = -1;
        uint32_t tw2 = 0, tw3 = 0;
        if (any_flagged && W > 2) {
#pragma unroll 1
            for (uint64_t todo = flagged; todo; todo &= todo - 1) {
                const uint32_t* q = s_q + low_lane(todo) * W;
                const uint64_t q01 = ((uint64_t)q[0] << 32) | q[1];
#pragma unroll
                for (int t = 2 * kScanU - 1; t >= 0; --t)
                    if (v[t] == q01) tail_t = t < tail_t || tail_t < 0 ? t : tail_t;
            }
            if (tail_t >= 0) {
                const int64_t id = base + (tail_t >> 1) * kPairRows + 2 * lane + (tail_t & 1);
                if (id < r_hi) {
                    const uint32_t* rp = ix.rows + id * W;
                    tw2 = rp[2];
                    tw3 = W > 3 ? rp[3] : 0u;
                } else {
                    tail_t = -1;
                }
            }
        }
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
            // the rows with a candidate under the filter at entry (a superset:
            // the filter only tightens below), then only those, in id order
            uint32_t rows_todo = 0;
#pragma unroll
            for (int t = 0; t < 2 * kScanU; ++t) {
                const int64_t id = base + (t >> 1) * kPairRows + 2 * lane + (t & 1);
                rows_todo |= ballot(id < r_hi && (v[t] & f.msk) == f.qm) ? 1u << t : 0u;
            }
            const bool touched = rows_todo != 0;
#pragma unroll 1
            for (; rows_todo; rows_todo &= rows_todo - 1) {
                const int t = __builtin_ctz(rows_todo);
                uint64_t w = v[0];
#pragma unroll
                for (int tt = 1; tt < 2 * kScanU; ++tt) w = t == tt ? v[tt] : w;
                const int u = t >> 1, h = t & 1;
                const int64_t id = base + u * kPairRows + 2 * lane + h;
                const bool cand = id < r_hi && (w & f.msk) == f.qm;
                if (ballot(cand) == 0) continue;
                int lc = -1;
                if (cand) {
                    const uint64_t x = w ^ q01;
                    if (x >> 32)
                        lc = lcp_from_diff(0, (uint32_t)(x >> 32), g);
                    else if ((uint32_t)x)
                        lc = lcp_from_diff(1, (uint32_t)x, g);
                    else if (W <= 2)
                        lc = g.L;
                    else if (t != tail_t)
                        lc = lcp_tail(ix.rows + id * W, q, g, 2);
                    else if (tw2 ^ q[2])
                        lc = lcp_from_diff(2, tw2 ^ q[2], g);
                    else if (W == 3)
                        lc = g.L;
                    else if (tw3 ^ q[3])
                        lc = lcp_from_diff(3, tw3 ^ q[3], g);
                    else
                        lc = W > 4 ? lcp_tail(ix.rows + id * W, q, g, 4) : g.L;
                }
                const uint64_t key = rank_key(lc, (uint32_t)id);
                lst.offer(key, cand && key < f.lim, f.kk);
                const uint64_t kth = lst.get(f.kk - 1);
                if (kth < f.lim) f.lim = kth;
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
    // trip; the merge ranks whatever is kept).  Lane i counts query i's (most
    // lists are empty: the count stops at the first entry not kept) and
    // reserves room for them with one atomic for all the wave's queries.
    int mine = 0;
    if (lane < ntq) {
        const int kk = filt[lane].kk;
        const uint64_t keep = filt[lane].lim;
        const uint64_t* lp = lists + (size_t)lane * sg.lstride;
        for (int e = 0; e < kk; ++e) {
            const uint64_t x = lp[e];
            if (x == kKeyMax || x > keep) break;
            ++mine;
        }
    }
    // limits this wave tightened since it last published them go to the
    // shared ones (waves that start later read them)
    if (lane < ntq) {
        const uint64_t mylim = filt[lane].lim;
        if (mylim < published) atomicMin((unsigned long long*)(gthr + q0i + lane), (unsigned long long)mylim);
    }
    uint32_t at = 0;
    if (lane < ntq && mine > 0) at = atomicAdd(cnt + (q0i + lane) * kCntStride, (uint32_t)mine);
#pragma unroll 1
    for (uint64_t todo = ballot(mine > 0); todo; todo &= todo - 1) {
        const int i = low_lane(todo);
        const int n = readlane_i(mine, i);
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
static size_t scan_block_lds(int tq, bool hash, int32_t k_max, int W) {
    return ((size_t)tq * W * sizeof(uint32_t) + 15) / 16 * 16 + (hash ? sizeof(ScanHash) : 0) +
           (size_t)kScanWaves * tq * (sizeof(ScanFilter) + (size_t)k_max * sizeof(uint64_t));
}
constexpr size_t kScanLdsBudget = 40 << 10;  // per block: at least 4 blocks (16 waves) per CU

// Queries per wave, from the compiled set for the list size and within the
// LDS budget (one query per wave always fits): the least test work per row
// over the query groups, a larger group on ties.  A group tested one query at
// a time costs one compare per real query; a hashed group costs, whatever its
// size, about kHashCost compares (measured on the 2M- and 8M-row hierarchy
// databases: its random LDS reads and its registers, 108 against 75, make the
// hashed variant slower at 32 queries and faster from a few hundred on).
constexpr int kHashCost = 12;
struct ScanShape {
    int tq;
    bool hash;
};
static ScanShape shape_for(int nr, int32_t k_max, int64_t Q, int W) {
    static const ScanShape c1[] = {{64, true}, {32, true}, {16, false}, {8, false}, {2, false}, {1, false}},
                           c2[] = {{16, true}, {8, false}, {1, false}}, c4[] = {{4, false}, {1, false}},
                           c16[] = {{1, false}};
    const ScanShape* c = nr == 1 ? c1 : nr == 2 ? c2 : nr == 4 ? c4 : c16;
    const int n = nr == 1 ? 6 : nr == 2 ? 3 : nr == 4 ? 2 : 1;
    ScanShape best = {1, false};
    int64_t best_cost = Q, best_groups = Q;
    for (int i = n - 1; i >= 0; --i) {  // ascending tq: on equal cost a larger one wins only with fewer groups
        const ScanShape sh = c[i];
        if (sh.tq > 1 && scan_block_lds(sh.tq, sh.hash, k_max, W) > kScanLdsBudget) continue;
        const int64_t groups = (Q + sh.tq - 1) / sh.tq;
        const int64_t cost = groups * (sh.hash ? kHashCost : (Q < sh.tq ? Q : sh.tq));
        if (cost < best_cost || (cost == best_cost && groups < best_groups)) {
            best = sh;
            best_cost = cost;
            best_groups = groups;
        }
    }
    return best;
}

// Rows sampled for the starting limits, and the main pass's chunking.
constexpr int64_t kChunkMinRows = 2 * kScanStepRows;
constexpr int64_t kSeedRows = 65536;
constexpr int64_t kScanTargetWaves = 8192;  // 32 per CU
constexpr int64_t kChunkAlign = kScanStepRows;  // main chunks: whole steps
constexpr int64_t kSeedChunkRows = kScanStepRows;  // sampled rows per wave (while the grid allows)

ScanPlan plan_scan(int64_t N, int W, int64_t Q, int32_t k_max, int64_t part_budget_bytes) {
    ScanPlan p;
    p.nr = nr_for(k_max);
    const ScanShape sh = shape_for(p.nr, k_max, Q, W);
    p.tq = sh.tq;
    p.hash = sh.hash;
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
    // most 64 (the limit kernel gives each part a lane and sums the parts'
    // histograms level by level)
    const int64_t seed_tiles = (p.seed_rows + 255) / 256;
    int64_t parts = Q > 0 ? 4096 / Q : 1;
    if (parts > kWave) parts = kWave;
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
    int64_t sc = (p.seed_rows + kSeedChunkRows - 1) / kSeedChunkRows;
    const int64_t by_grid = kScanTargetWaves / 2 / p.qgroups;
    if (sc > by_grid) sc = by_grid;
    if (sc > max_by_mem / 2) sc = max_by_mem / 2;
    if (sc < 1) sc = 1;
    p.seed_chunk_rows = (p.seed_rows + sc - 1) / sc;
    p.seed_chunk_rows = (p.seed_chunk_rows + kSeedChunkRows - 1) / kSeedChunkRows * kSeedChunkRows;
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
        rows = (rows + kChunkAlign - 1) / kChunkAlign * kChunkAlign;
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
    sc.hist = u + (size_t)Q * kCntStride;      // [Q][seed_parts][L+1], written whole by the seed blocks
    sc.qkeys = sc.hist + (size_t)Q * p.seed_parts * (g.L + 1);  // [Q][W]
    sc.words = ((size_t)Q * (size_t)sc.cap + (size_t)Q) * 2 +
               (size_t)Q * (kCntStride + (size_t)p.seed_parts * (g.L + 1) + g.W);
    return sc;
}

size_t scan_partial_entries(const ScanPlan& p, int64_t Q, int32_t k_max, const RowGeo& g) {
    return (scan_scratch(p, Q, k_max, g, nullptr).words + 1) / 2;
}

template <int NR, int TQ, bool H>
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
    const size_t shm = scan_block_lds(TQ, H, k_max, ix.g.W);
    const int64_t blocks = (int64_t)p.qgroups * ((p.nparts + kScanWaves - 1) / kScanWaves);
    hipLaunchKernelGGL((k_scan<NR, TQ, H>), dim3((unsigned)blocks), dim3(kScanWaves * kWave), shm, s, ix, qb, sc.qkeys,
                       sg, sc.cap, sc.part, sc.cnt, sc.gthr);
}

hipError_t launch_scan(const IndexView& ix, const QueryBatch& qb, const ScanPlan& p, uint64_t* scratch, hipStream_t s,
                       hipEvent_t ev0, hipEvent_t ev1, hipEvent_t ev2) {
    if (qb.Q <= 0) return hipSuccess;
    const ScanScratch sc = scan_scratch(p, qb.Q, qb.k_max, ix.g, scratch);
    const int64_t nz = qb.Q * (int64_t)kCntStride;  // the fill counts
    const int64_t nprep = nz > qb.Q * ix.g.W ? nz : qb.Q * ix.g.W;
    hipLaunchKernelGGL(k_scan_prep, dim3((unsigned)((nprep + 255) / 256)), dim3(256), 0, s, qb, ix.g, sc.cnt, nz,
                       sc.qkeys);
    hipLaunchKernelGGL(k_seed_hist, dim3((unsigned)(qb.Q * p.seed_parts)), dim3(kSeedThreads), 0, s, ix, sc.qkeys,
                       p.seed_rows, p.seed_parts, sc.hist);
    hipLaunchKernelGGL(k_seed_limit, dim3((unsigned)((qb.Q + kScanWaves - 1) / kScanWaves)), dim3(kScanWaves * kWave),
                       0, s, qb, ix.N, ix.g.L, p.seed_rows, p.seed_parts, sc.hist, sc.gthr);
    if (ev0) hipEventRecord(ev0, s);
    switch (p.nr * 1000 + p.tq * 10 + (p.hash ? 1 : 0)) {
        case 1641: launch_scan_t<1, 64, true>(ix, qb, p, sc, qb.k_max, s); break;
        case 1321: launch_scan_t<1, 32, true>(ix, qb, p, sc, qb.k_max, s); break;
        case 1160: launch_scan_t<1, 16, false>(ix, qb, p, sc, qb.k_max, s); break;
        case 1080: launch_scan_t<1, 8, false>(ix, qb, p, sc, qb.k_max, s); break;
        case 1020: launch_scan_t<1, 2, false>(ix, qb, p, sc, qb.k_max, s); break;
        case 1010: launch_scan_t<1, 1, false>(ix, qb, p, sc, qb.k_max, s); break;
        case 2161: launch_scan_t<2, 16, true>(ix, qb, p, sc, qb.k_max, s); break;
        case 2080: launch_scan_t<2, 8, false>(ix, qb, p, sc, qb.k_max, s); break;
        case 2010: launch_scan_t<2, 1, false>(ix, qb, p, sc, qb.k_max, s); break;
        case 4040: launch_scan_t<4, 4, false>(ix, qb, p, sc, qb.k_max, s); break;
        case 4010: launch_scan_t<4, 1, false>(ix, qb, p, sc, qb.k_max, s); break;
        case 16010: launch_scan_t<16, 1, false>(ix, qb, p, sc, qb.k_max, s); break;
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
