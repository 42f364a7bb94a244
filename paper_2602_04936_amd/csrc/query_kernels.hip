// Index path: one wave per query, all steps fused in one kernel.
//
// Notation: T = rows in lexicographic order, A[i] = LCP(T[i-1], T[i]),
// perm[i] = id of T[i], p = insertion point of q (number of rows < q).
//
//  1. Search.  The top-1 LCP problem reduces to predecessor search in the
//     sorted order (section 4.2, Theorem "Query Lower Bound"), and the paper's
//     range scan starts from a binary search for the query prefix (Appendix
//     D.1).  Here each step compares q with 64 evenly spaced pivots at once
//     (one per lane) and keeps the gap that contains q, so the insertion point
//     is found in ceil(log_65(N)) dependent steps instead of log_2(N).  The
//     top levels read the pivots' first four key words from the search tables
//     (one coalesced 1 KB load per step; the first two levels stay in L2) and
//     touch a pivot row only on a tie; the last step reads its at most 64
//     contiguous rows.  The steps also yield lL = LCP(q, T[p-1]) and
//     lR = LCP(q, T[p]).
//  2. Outward walk.  By the strong triangle inequality (section 2.1, Theorem
//     "Ultrametric Property") and sorted order, LCP(q, T[j]) = min(lR,
//     A[p+1..j]) for j >= p and min(lL, A[j+1..p-1]) for j < p: the LCP only
//     falls moving away from p, and the rows with LCP >= d are one contiguous
//     range G_d around p (the prefix bucket of section 6.2, a trie subtree of
//     section 5.1).  Reading A outward level by level gives the cutoff
//     c = max{d : |G_d| >= k'} (k' = min(k, N)), the inner group G_{c+1}
//     (fewer than k' rows, all in the answer) and the range G_c.
//  3. Inner group: LCPs by prefix minimum over A, ranked by (LCP desc, id
//     asc).  When the inner group has at most k rows the paper takes the
//     whole subtree (Appendix D.2, CollectTopKOptimized fast path).
//  4. Tied rows (LCP exactly c): the k' - |G_{c+1}| lowest ids, from a scan of
//     perm over G_c minus G_{c+1} (the range-bounded scan of section 6.2).
//     When c = 0 that range is the whole database; then the ids are walked in
//     ascending order instead, keeping those whose first token differs from
//     q's, which stops after at most k' + 64 probes.
//  5. Emit in rank order; pad with (-1, -1) past N.
#include "device.hpp"
#include "launch.hpp"

namespace lcpx {

constexpr int kQueryWaves = 4;
constexpr int kTieUnroll = 8;
constexpr int kHeldUnroll = 10;  // tied ids held in registers: ranges of at most 640 rows
constexpr int kFewTied = 16;  // tied selections of at most this many ids use repeated wave minima
constexpr int kSelMax = kAdjWindow / 4;  // 32-bit entries of the LDS window the tie selections reuse

// A[j] for the 64 positions j = j0 + dir * lane: from the wave's LDS window
// when the whole chunk lies inside it, else from global memory.  Lanes whose
// position is outside [lo_ok, hi_ok] get -1.
__device__ __forceinline__ int a_lane(const uint8_t* __restrict__ A, const uint8_t* win, int wbase, int j0, int dir,
                                      int lo_ok, int hi_ok) {
    const int lane = lane_id();
    const int j = j0 + dir * lane;
    const int jmin = dir > 0 ? j0 : j0 - (kWave - 1);
    const int jmax = dir > 0 ? j0 + (kWave - 1) : j0;
    const bool in_win = jmin >= wbase && jmax < wbase + kAdjWindow;
    if (j < lo_ok || j > hi_ok) return -1;
    // the window is read through an LDS pointer: a select between the two
    // pointers would otherwise become one generic (flat) load on both paths
    if (in_win) return (int)((const __attribute__((address_space(3))) uint8_t*)win)[j - wbase];
    return (int)A[j];
}

// Inner group G_{c+1} = [in_lo, in_hi) around p, fewer than 128 rows, in rank
// order.  The LCP of T[p+t] is the prefix minimum of lR, A[p+1..p+t]; that of
// T[p-1-t] the prefix minimum of lL, A[p-1..p-t].  Keys (255 - LCP) << 32 | id
// are held in registers (two chunks of 64 per side) until the last A read,
// then compacted into the wave's LDS window; each key's rank is the number of
// keys below it.
__device__ __forceinline__ void inner_by_rank(const IndexView& ix, uint8_t* win, int wbase, int p, int in_lo,
                                              int in_hi, int lL, int lR, int n_gt, int32_t* __restrict__ oid,
                                              int32_t* __restrict__ olc) {
    const int lane = lane_id();
    const int nr = in_hi - p;
    const int nl = p - in_lo;
    uint32_t id[2][2];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
        for (int b = 0; b < 2; ++b) {  // all perm loads in flight first
            const int t = b * kWave + lane;
            const bool act = t < (sd == 0 ? nr : nl);
            id[sd][b] = act ? (uint32_t)ix.perm[sd == 0 ? p + t : p - 1 - t] : 0u;
        }
    uint64_t key[2][2];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
        const int n = sd == 0 ? nr : nl;
        int carry = 255;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int t = b * kWave + lane;
            key[sd][b] = kKeyMax;
            if (b * kWave < n) {
                // right: row p+t needs A[p+t]; left: row p-1-t needs A[p-t]
                const int av = sd == 0 ? a_lane(ix.A, win, wbase, p + b * kWave, +1, p + 1, in_hi - 1)
                                       : a_lane(ix.A, win, wbase, p - b * kWave, -1, in_lo + 1, p - 1);
                const int a = t < n ? (t == 0 ? (sd == 0 ? lR : lL) : av) : 255;
                int v = wave_prefix_min(a);
                v = v < carry ? v : carry;
                carry = readlane_i(v, kWave - 1);
                if (t < n) key[sd][b] = rank_key(v, id[sd][b]);
            }
        }
    }
    uint64_t* s64 = reinterpret_cast<uint64_t*>(win);  // the A window is not read again
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int t = b * kWave + lane;
            if (t < (sd == 0 ? nr : nl)) s64[sd == 0 ? t : nr + t] = key[sd][b];
        }
    const int n2 = (n_gt + 1) & ~1;
    if (lane == 0 && n_gt < n2) s64[n_gt] = kKeyMax;  // pad to whole 16-byte reads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int rank[2][2] = {{0, 0}, {0, 0}};
    const uint4* s4 = reinterpret_cast<const uint4*>(win);
#pragma unroll 2
    for (int j = 0; j < n2 / 2; ++j) {
        const uint4 x = s4[j];
        const uint64_t k0 = ((uint64_t)x.y << 32) | x.x;
        const uint64_t k1 = ((uint64_t)x.w << 32) | x.z;
#pragma unroll
        for (int sd = 0; sd < 2; ++sd)
#pragma unroll
            for (int b = 0; b < 2; ++b) rank[sd][b] += (k0 < key[sd][b]) + (k1 < key[sd][b]);
    }
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
        for (int b = 0; b < 2; ++b)
            if (key[sd][b] != kKeyMax) {
                oid[rank[sd][b]] = key_id(key[sd][b]);
                olc[rank[sd][b]] = key_lcp(key[sd][b]);
            }
}

// The m lowest ids among at most U*64 tied positions, m <= kSelMax, whose ids
// the caller holds in `id` (0xFFFFFFFF past the range end): the m-th
// smallest, tau, by bisection on the id bits from the most significant (the
// ids are distinct, so exactly m of them are <= tau); those m are compacted
// into the wave's LDS window and each is written at its rank, the count of
// selected ids below it.
template <int U>
__device__ __forceinline__ void tied_select(const IndexView& ix, const uint32_t* id, int m, int c,
                                            int32_t* __restrict__ oid, int32_t* __restrict__ olc, uint32_t* sel) {
    const int lane = lane_id();
    const int bits = 32 - __builtin_clz((uint32_t)(ix.N - 1) | 1u);  // ids are < 2^bits
    uint32_t pre = 0;  // the bits of tau above bit b
    int rem = m;       // rank of tau among the ids that share those bits
#pragma unroll 1
    for (int b = bits - 1; b >= 0; --b) {
        const uint32_t want = pre << 1;
        int cnt = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) cnt += popc64(ballot((id[u] >> b) == want));
        if (rem <= cnt) {
            pre = want;
        } else {
            rem -= cnt;
            pre = want | 1u;
        }
    }
    const uint32_t tau = pre;
    int n = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const bool s = id[u] <= tau;
        const uint64_t bal = ballot(s);
        const int pos = n + count_below(bal);
        if (s && pos < kSelMax) sel[pos] = id[u];
        n += popc64(bal);
    }
    const int m4 = (m + 3) & ~3;
    if (m + lane < m4) sel[m + lane] = 0xFFFFFFFFu;  // pad to whole 16-byte reads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    constexpr int kPer = kSelMax / kWave;  // selected ids per lane
    uint32_t v[kPer];
    int rank[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int e = t * kWave + lane;
        v[t] = e < m ? sel[e] : 0u;
        rank[t] = 0;
    }
    const uint4* s4 = reinterpret_cast<const uint4*>(sel);
#pragma unroll 2
    for (int j = 0; j < m4 / 4; ++j) {
        const uint4 x = s4[j];
#pragma unroll
        for (int t = 0; t < kPer; ++t)
            rank[t] += (x.x < v[t]) + (x.y < v[t]) + (x.z < v[t]) + (x.w < v[t]);
    }
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int e = t * kWave + lane;
        if (e < m) {
            oid[rank[t]] = (int32_t)v[t];
            olc[rank[t]] = c;
        }
    }
}

// The m lowest ids among the tied positions [l, in_lo) and [in_hi, r) using
// the per-64-position minima bmin (section 6.2's range scan, pruned).
// Every position lies either in a run of 64 that sits wholly inside one of the
// two ranges (a full block) or in one of the at most four partial runs at
// their ends.  Representatives are the full blocks' minima and the partial
// positions' own ids: all distinct ids of tied rows.  With tau the m-th
// smallest representative, at least m tied ids are <= tau, so every answer is
// <= tau; an answer in a full block makes that block's minimum <= tau, and
// exactly m representatives are <= tau, so at most m full blocks need reading.
// Phase 0 finds tau from the minima, phase 1 reads the selected blocks (their
// indices kept in `sel`, the wave's LDS window, <= kSelMax entries) and the
// partial positions, keeping ids <= tau.
template <int NR>
__device__ __forceinline__ void tied_pruned(const IndexView& ix, int64_t l, int64_t in_lo, int64_t in_hi, int64_t r,
                                         int m, int c, int32_t* __restrict__ oid, int32_t* __restrict__ olc,
                                         uint32_t* sel) {
    const int lane = lane_id();
    const int64_t ss[2] = {l, in_hi};
    const int64_t ee[2] = {in_lo, r};
    int64_t hs[2], te[2], bf[2], nbk[2];
#pragma unroll
    for (int sg = 0; sg < 2; ++sg) {
        const int64_t up = (ss[sg] + kWave - 1) & ~(int64_t)(kWave - 1);
        const int64_t h = ee[sg] < up ? ee[sg] : up;                        // head run [s, h)
        const int64_t dn = ee[sg] & ~(int64_t)(kWave - 1);
        const int64_t t = dn > h ? dn : h;                                  // tail run [t, e)
        hs[sg] = h;
        te[sg] = t;
        bf[sg] = h / kWave;                                                 // full blocks [h/64, t/64)
        nbk[sg] = t / kWave - h / kWave;
    }
    const int64_t nbt = nbk[0] + nbk[1];
    int nsel = 0;
    uint32_t tau = 0xFFFFFFFFu;
    WaveList<NR> lst;
#pragma unroll 1
    for (int ph = 0; ph < 2; ++ph) {
        lst.init();
        uint32_t px[4];
        bool pv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int sg = u >> 1;
            const int64_t a = (u & 1) ? te[sg] : ss[sg];
            const int64_t b = (u & 1) ? ee[sg] : hs[sg];
            const int64_t j = a + lane;
            pv[u] = j < b;
            px[u] = pv[u] ? (uint32_t)ix.perm[j] : 0u;
        }
#pragma unroll 1
        for (int u = 0; u < 4; ++u) {
            uint32_t x = px[0];
            bool v = pv[0];
#pragma unroll
            for (int uu = 1; uu < 4; ++uu) {
                x = u == uu ? px[uu] : x;
                v = u == uu ? pv[uu] : v;
            }
            lst.offer((uint64_t)x, v && x <= tau, m);
        }
        // items: 64 block minima each (phase 0) or one selected block of 64 ids (phase 1)
        const int64_t nit = ph == 0 ? (nbt + kWave - 1) / kWave : (int64_t)nsel;
#pragma unroll 1
        for (int64_t t0 = 0; t0 < nit; t0 += kTieUnroll) {
            uint32_t x[kTieUnroll];
            bool v[kTieUnroll];
#pragma unroll
            for (int u = 0; u < kTieUnroll; ++u) {  // all loads in flight before any is used
                const int64_t t = t0 + u;
                if (ph == 0) {
                    const int64_t vb = t * kWave + lane;
                    v[u] = t < nit && vb < nbt;
                    const int64_t pb = vb < nbk[0] ? bf[0] + vb : bf[1] + (vb - nbk[0]);
                    x[u] = v[u] ? ix.bmin[pb] : 0u;
                } else {
                    v[u] = t < nit;
                    const int64_t blk = v[u] ? (int64_t)sel[t] : 0;
                    x[u] = v[u] ? (uint32_t)ix.perm[blk * kWave + lane] : 0u;
                }
            }
#pragma unroll 1
            for (int u = 0; u < kTieUnroll && t0 + u < nit; ++u) {
                uint32_t xx = x[0];
                bool vv = v[0];
#pragma unroll
                for (int uu = 1; uu < kTieUnroll; ++uu) {
                    xx = u == uu ? x[uu] : xx;
                    vv = u == uu ? v[uu] : vv;
                }
                lst.offer((uint64_t)xx, vv && xx <= tau, m);
            }
        }
        if (ph == 0) {
            const uint64_t tk = lst.get(m - 1);
            tau = tk < 0xFFFFFFFFull ? (uint32_t)tk : 0xFFFFFFFFu;
            nsel = 0;
            for (int64_t b0 = 0; b0 < nbt; b0 += kWave) {
                const int64_t vb = b0 + lane;
                const int64_t pb = vb < nbk[0] ? bf[0] + vb : bf[1] + (vb - nbk[0]);
                const bool hit = vb < nbt && ix.bmin[pb] <= tau;
                const uint64_t bal = ballot(hit);
                const int pos = nsel + count_below(bal);
                if (hit && pos < kSelMax) sel[pos] = (uint32_t)pb;
                nsel += popc64(bal);
            }
            nsel = nsel < kSelMax ? nsel : kSelMax;  // at most m <= kSelMax by the argument above
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) {
        const int e = rr * kWave + lane;
        if (e < m) {
            oid[e] = (int32_t)(uint32_t)lst.v[rr];
            olc[e] = c;
        }
    }
}

template <int NR, int VEC>
__device__ __forceinline__ void index_query_body(const IndexView& ix, const QueryBatch& qb, int64_t qi) {
    extern __shared__ __align__(16) uint32_t s_dyn[];  // [kQueryWaves][W] query words, then [kQueryWaves][kAdjWindow] A bytes
    const RowGeo g = ix.g;
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    uint32_t* q = s_dyn + wv * g.W;
    uint8_t* win = reinterpret_cast<uint8_t*>(s_dyn + kQueryWaves * g.W) + wv * kAdjWindow;
    // the root node of the search tables does not depend on q: its load is
    // issued before the query's and overlaps it
    uint4 root = make_uint4(0u, 0u, 0u, 0u);
    if (ix.stab_levels > 0) root = ix.stab[lane];
    // the wave's own LDS slot: the writes below are seen by its later reads
    for (int w = lane; w < g.W; w += kWave) q[w] = key_word(qb.raw, qi * g.L, g, w);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    const int N = (int)ix.N;  // at most kMaxRows: positions and window offsets fit in 32 bits
    const int k = query_k(qb, qi);
    const int64_t out0 = query_off(qb, qi);
    int32_t* __restrict__ oid = qb.out_ids + out0;
    int32_t* __restrict__ olc = qb.out_lcp + out0;
    const int kp = k < N ? k : N;

    // ---- 1. insertion point and the LCPs of its two neighbours
    // the query's first four key words as two 64-bit halves (zero past the row's end)
    const uint64_t qa = ((uint64_t)q[0] << 32) | (g.W > 1 ? q[1] : 0u);
    const uint64_t qb2 = ((uint64_t)(g.W > 2 ? q[2] : 0u) << 32) | (g.W > 3 ? q[3] : 0u);
    int lo = 0, hi = N;
    int lcp_lo = -1, lcp_hi = -1;  // LCP(q, T[lo-1]), LCP(q, T[hi])
    // with the first-token directory the search starts in the query's bucket:
    // the rows around it have other first tokens, so their LCP with q is 0
    int levels = ix.stab_levels;
    if (ix.dir != nullptr) {
        const uint32_t t0 = q[0] >> (32 - 8 * g.tb);
        const uint32_t t = t0 < (uint32_t)ix.dir_V ? t0 : (uint32_t)ix.dir_V;
        lo = (int)ix.dir[t];
        hi = (int)ix.dir[t + 1];
        lcp_lo = 0;
        lcp_hi = 0;
        levels = 0;
    }
    int p;
    int lL, lR;
    int wbase;
    int depth = 0;
    int node = 0, level_start = 0;  // table node and the entry where its level starts
    for (;;) {
        const int n = hi - lo;
        if (n <= kWave) {
            // last step: the rows [lo, hi) are contiguous; the A window around
            // lo (p is within 64 of it) is fetched in the same round trip
            wbase = lo - kAdjWindow / 2;
            wbase = wbase < 0 ? 0 : wbase & ~15;
            const uint4 av = *reinterpret_cast<const uint4*>(ix.A + wbase + 16 * lane);
            const bool act = lane < n;
            int lc;
            bool less;
            // the wave's first row address is uniform; lanes add lane * W
            const uint32_t* rows = ix.sorted + (int64_t)lo * g.W;
            compare_row<VEC>(act ? rows + __umul24((unsigned)lane, (unsigned)g.W) : ix.sorted, q, g, act, lc, less);
            *reinterpret_cast<uint4*>(win + 16 * lane) = av;
            const int cnt = popc64(ballot(less));
            p = lo + cnt;
            lL = cnt > 0 ? readlane_i(lc, cnt - 1) : lcp_lo;
            lR = cnt < n ? readlane_i(lc, cnt) : lcp_hi;
            break;
        }
        // lane i's pivot is row lo + (i + 1) * n / 65, computed in 32 bits as
        // lo + (i + 1) * a + (i + 1) * b / 65 with n = 65 a + b; only the rare
        // paths that read pivot rows need it per lane, the chosen child's
        // bounds below come from the (uniform) count
        const int a65 = (int)((uint32_t)n / (kWave + 1));
        const int b65 = n - (kWave + 1) * a65;
        int lc;
        bool less;
        if (depth < levels) {
            // pivot's first four key words from the table (one coalesced load)
            const uint4 e = depth == 0 ? root : ix.stab[level_start + node * kWave + lane];
            const uint64_t ka = ((uint64_t)e.x << 32) | e.y;
            const uint64_t kb = ((uint64_t)e.z << 32) | e.w;
            // first differing 64-bit half by selects (no per-lane branches)
            const uint64_t xa = ka ^ qa, xb = kb ^ qb2;
            const bool da = xa != 0;
            lc = (int)(((da ? 0 : 64) + __clzll((long long)(da ? xa : xb))) >> g.bits_log2);
            less = da ? ka < qa : kb < qb2;
            const bool tie = !da && xb == 0;
            if (ballot(tie)) {  // a pivot ties on the first four words: compare the rest of its row
                if (tie) {
                    lc = g.L;
                    less = false;
                    const int pos = lo + (lane + 1) * a65 + (int)((uint32_t)((lane + 1) * b65) / (kWave + 1));
                    const uint32_t* row = ix.sorted + (int64_t)pos * g.W;
                    for (int w = 4; w < g.W; ++w) {
                        const uint32_t rw = row[w];
                        if (rw != q[w]) {
                            lc = lcp_from_diff(w, rw ^ q[w], g);
                            less = rw < q[w];
                            break;
                        }
                    }
                }
            }
        } else {
            const int pos = lo + (lane + 1) * a65 + (int)((uint32_t)((lane + 1) * b65) / (kWave + 1));
            compare_row<VEC>(ix.sorted + (int64_t)pos * g.W, q, g, true, lc, less);
        }
        const int cnt = popc64(ballot(less));  // pivots below q form a prefix of the lanes
        const int lo0 = lo;
        if (cnt > 0) {  // just above pivot cnt - 1
            lo = lo0 + cnt * a65 + (int)((uint32_t)(cnt * b65) / (kWave + 1)) + 1;
            lcp_lo = readlane_i(lc, cnt - 1);
        }
        if (cnt < kWave) {  // up to pivot cnt
            hi = lo0 + (cnt + 1) * a65 + (int)((uint32_t)((cnt + 1) * b65) / (kWave + 1));
            lcp_hi = readlane_i(lc, cnt);
        }
        if (depth < levels) {
            node = node * (kWave + 1) + cnt;
            level_start = level_start * (kWave + 1) + kWave;
            ++depth;
        }
    }

    // ---- 2. walk outward level by level: group [l, r) = G_lev
    int l = p, r = p;
    int vr = p < N ? lR : -1;  // LCP(q, T[r]), -1 past the end
    int vl = p > 0 ? lL : -1;  // LCP(q, T[l-1]), -1 before the start
    int lev = vr > vl ? vr : vl;
    int in_lo = p, in_hi = p;  // G_{c+1}
    int c;
    for (;;) {
        if (lev <= 0) {
            l = 0;
            r = N;
            c = 0;
            break;
        }
        if (vr >= lev) {  // T[r] is in: extend to the first j > r with A[j] < lev
            for (int j0 = r + 1;; j0 += kWave) {
                const int a = a_lane(ix.A, win, wbase, j0, +1, 1, N - 1);  // -1 past the end stops
                const uint64_t stop = ballot(a < lev);
                if (stop) {
                    const int f = low_lane(stop);
                    r = j0 + f;
                    vr = readlane_i(a, f);
                    break;
                }
            }
        }
        if (vl >= lev) {  // T[l-1] is in: extend down to the first i <= l-1 with A[i] < lev
            for (int i0 = l - 1;; i0 -= kWave) {
                const int a = a_lane(ix.A, win, wbase, i0, -1, 1, N - 1);  // -1 at i < 1 stops
                const uint64_t stop = ballot(a < lev);
                if (stop) {
                    const int f = low_lane(stop);
                    const int ii = i0 - f;
                    if (ii >= 1) {
                        l = ii;
                        vl = readlane_i(a, f);
                    } else {
                        l = 0;
                        vl = -1;
                    }
                    break;
                }
            }
        }
        if (r - l >= kp) {
            c = lev;
            break;
        }
        in_lo = l;
        in_hi = r;
        lev = vr > vl ? vr : vl;
    }
    const int n_gt = (int)(in_hi - in_lo);
    const int m = kp - n_gt;

    // ids of a short tied range are requested now, so that their round trip
    // overlaps the inner group's
    const int tnl = in_lo - l;
    const int tn = tnl + (r - in_hi);
    const bool held = m > 0 && c > 0 && m <= kSelMax && tn <= kHeldUnroll * kWave;
    const bool few = held && m <= kFewTied && tn <= kTieUnroll * kWave;
    uint32_t tid[kHeldUnroll];
    {
        // positions fit in 32 bits (N < 2^31); t < tnl picks the left part
        const int tnl32 = tnl, tn32 = held ? tn : 0;
        const uint32_t lb = (uint32_t)l, rb = (uint32_t)in_hi - (uint32_t)tnl32;
#pragma unroll
        for (int u = 0; u < kHeldUnroll; ++u) {
            const int t = u * kWave + lane;
            const uint32_t j = (t < tnl32 ? lb : rb) + (uint32_t)t;
            tid[u] = t < tn32 ? (uint32_t)ix.perm[j] : 0xFFFFFFFFu;  // above every id
        }
    }

    // ---- 3. inner group G_{c+1}, ranked by (LCP desc, id asc)
    if constexpr (NR <= 2) {
        // at most 127 rows (k <= 128): all keys in registers while A is read,
        // then into the LDS window, each written at its rank (the count of
        // keys below it; keys are distinct since ids are)
        if (n_gt > 0) inner_by_rank(ix, win, wbase, p, in_lo, in_hi, lL, lR, n_gt, oid, olc);
    } else if (n_gt > 0) {
        WaveList<NR> inner;
        inner.init();
        int carry = 255;
        const int64_t nr = in_hi - p;
        for (int64_t b = 0; b < nr; b += kWave) {
            const int64_t t = b + lane;
            const bool act = t < nr;
            const int64_t j = p + t;
            const int av = a_lane(ix.A, win, wbase, p + b, +1, p + 1, in_hi - 1);
            const int a = act ? (t == 0 ? lR : av) : 255;
            int v = wave_prefix_min(a);
            v = v < carry ? v : carry;
            carry = readlane_i(v, kWave - 1);
            const uint32_t id = act ? (uint32_t)ix.perm[j] : 0u;
            inner.offer(rank_key(v, id), act, NR * kWave);
        }
        carry = 255;
        const int64_t nl = p - in_lo;
        for (int64_t b = 0; b < nl; b += kWave) {
            const int64_t t = b + lane;
            const bool act = t < nl;
            const int64_t j = p - 1 - t;
            // the LCP of T[j] with q needs A[j+1]
            const int av = a_lane(ix.A, win, wbase, p - b, -1, in_lo + 1, p - 1);
            const int a = act ? (t == 0 ? lL : av) : 255;
            int v = wave_prefix_min(a);
            v = v < carry ? v : carry;
            carry = readlane_i(v, kWave - 1);
            const uint32_t id = act ? (uint32_t)ix.perm[j] : 0u;
            inner.offer(rank_key(v, id), act, NR * kWave);
        }
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
            const int e = rr * kWave + lane;
            if (e < n_gt) {
                oid[e] = key_id(inner.v[rr]);
                olc[e] = key_lcp(inner.v[rr]);
            }
        }
    }

    if (qb.stats != nullptr) {
        const bool pruned = m <= kSelMax && (in_lo - l) + (r - in_hi) >= kWave * 4 * (m > 8 ? m : 8);
        const int path = m <= 0   ? kTieNone
                         : c == 0 ? kTieIdWalk
                         : few    ? kTieFew
                         : held   ? kTieSelect
                         : pruned ? kTiePruned
                                  : kTieList;
        if (lane == 0) *reinterpret_cast<int4*>(qb.stats + 4 * qi) = make_int4(c, n_gt, tn, path);
    }

    // ---- 4. the m lowest ids among rows with LCP exactly c
    if (m > 0) {
        if (c == 0) {
            const uint32_t q0 = q[0];
            const int drop = 32 - 8 * g.tb;
            int got = 0;
            for (int b = 0; got < m && b < N; b += kWave) {
                const int id = b + lane;
                const bool hit = id < N && ((ix.rows[(int64_t)id * g.W] ^ q0) >> drop) != 0u;
                const uint64_t bal = ballot(hit);
                const int rank = got + count_below(bal);
                if (hit && rank < m) {
                    oid[n_gt + rank] = (int32_t)id;
                    olc[n_gt + rank] = 0;
                }
                got += popc64(bal);
            }
        } else if (few) {
            // small case: each lane sorts its (at most 8) tied ids, then m
            // rounds take the wave minimum of the lanes' smallest remaining id
            // and the lane holding it drops that id
            uint32_t h0 = tid[0], h1 = tid[1], h2 = tid[2], h3 = tid[3], h4 = tid[4], h5 = tid[5], h6 = tid[6],
                     h7 = tid[7];
#define LCPX_CE(x, y)                              \
    {                                              \
        const uint32_t lo_ = x < y ? x : y;        \
        y = x < y ? y : x;                         \
        x = lo_;                                   \
    }
            LCPX_CE(h0, h1) LCPX_CE(h2, h3) LCPX_CE(h4, h5) LCPX_CE(h6, h7) LCPX_CE(h0, h2) LCPX_CE(h1, h3)
            LCPX_CE(h4, h6) LCPX_CE(h5, h7) LCPX_CE(h1, h2) LCPX_CE(h5, h6) LCPX_CE(h0, h4) LCPX_CE(h1, h5)
            LCPX_CE(h2, h6) LCPX_CE(h3, h7) LCPX_CE(h2, h4) LCPX_CE(h3, h5) LCPX_CE(h1, h2) LCPX_CE(h3, h4)
            LCPX_CE(h5, h6)
#undef LCPX_CE
            uint32_t mine = 0xFFFFFFFFu;  // lane e keeps the e-th smallest
            for (int e = 0; e < m; ++e) {
                const uint32_t v = wave_min_u32(h0);
                // lane e takes v: one lane write instead of a compare and a select
                asm("v_writelane_b32 %0, %1, m0" : "+v"(mine) : "s"(v), "{m0}"(e));
                if (h0 == v) {  // one lane: the ids are distinct
                    h0 = h1;
                    h1 = h2;
                    h2 = h3;
                    h3 = h4;
                    h4 = h5;
                    h5 = h6;
                    h6 = h7;
                    h7 = 0xFFFFFFFFu;
                }
            }
            if (lane < m) {
                oid[n_gt + lane] = (int32_t)mine;
                olc[n_gt + lane] = c;
            }
        } else if (held) {
            tied_select<kHeldUnroll>(ix, tid, m, c, oid + n_gt, olc + n_gt, reinterpret_cast<uint32_t*>(win));
        } else if (m <= kSelMax && (in_lo - l) + (r - in_hi) >= kWave * 4 * (m > 8 ? m : 8)) {
            tied_pruned<NR>(ix, l, in_lo, in_hi, r, m, c, oid + n_gt, olc + n_gt, reinterpret_cast<uint32_t*>(win));
        } else {
            WaveList<NR> tied;
            tied.init();
            const int64_t nleft = in_lo - l;
            const int64_t tn = nleft + (r - in_hi);
            for (int64_t b = 0; b < tn; b += kTieUnroll * kWave) {
                uint32_t id[kTieUnroll];
#pragma unroll
                for (int u = 0; u < kTieUnroll; ++u) {  // all loads in flight before any is used
                    const int64_t t = b + u * kWave + lane;
                    const int64_t j = t < nleft ? l + t : in_hi + (t - nleft);
                    id[u] = t < tn ? (uint32_t)ix.perm[j] : 0u;
                }
#pragma unroll 1
                for (int u = 0; u < kTieUnroll && b + u * kWave < tn; ++u) {  // one copy of the offer code
                    uint32_t x = id[0];
#pragma unroll
                    for (int uu = 1; uu < kTieUnroll; ++uu) x = u == uu ? id[uu] : x;
                    tied.offer((uint64_t)x, b + u * kWave + lane < tn, m);
                }
            }
#pragma unroll
            for (int rr = 0; rr < NR; ++rr) {
                const int e = rr * kWave + lane;
                if (e < m) {
                    oid[n_gt + e] = (int32_t)(uint32_t)tied.v[rr];
                    olc[n_gt + e] = c;
                }
            }
        }
    }

    // ---- 5. padding when k > N
    for (int e = kp + lane; e < k; e += kWave) {
        oid[e] = -1;
        olc[e] = -1;
    }
}

// Registers: with one list register (k <= 64) the cap lets 8 waves fit per
// SIMD, so a whole 8,192-query batch is resident at once; two or four list
// registers (k <= 256) would spill under that cap, so those variants allow 6
// waves per SIMD instead.  Large lists (k > 256) keep their registers.
template <int NR, int VEC>
__device__ __forceinline__ void one_query_per_wave(const IndexView& ix, const QueryBatch& qb) {
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t qi = (int64_t)blockIdx.x * kQueryWaves + wv;
    if (qi < qb.Q) index_query_body<NR, VEC>(ix, qb, qi);
}

// Persistent form: a grid that fills the GPU once; each wave takes the next
// query from a device counter (reset to 0 before the launch) until the batch
// size read from device memory is reached.  Queries of uneven cost balance
// themselves; the order in which waves take them never reaches the output.
// Persistent form: wave w of the grid first answers query w, then (only when
// the grid has fewer waves than the batch has queries) takes further queries
// nwaves, nwaves + 1, ... from the device work counter.  A grid of one wave
// per query of the capacity therefore needs no atomics at all.
template <int NR, int VEC>
__device__ __forceinline__ void queries_from_counter(const IndexView& ix, const QueryBatch& qb, const int64_t* q_count,
                                                     unsigned long long* counter) {
    const int64_t Q = *q_count;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t nwaves = (int64_t)gridDim.x * kQueryWaves;
    int64_t qi = (int64_t)blockIdx.x * kQueryWaves + wv;
#pragma unroll 1
    while (qi < Q) {
        index_query_body<NR, VEC>(ix, qb, qi);
        if (nwaves >= Q) break;
        unsigned long long got = 0;
        if (lane_id() == 0) got = atomicAdd(counter, 1ull);
        qi = nwaves + (int64_t)readlane64(got, 0);
    }
}

constexpr int waves_per_simd(int nr) { return nr == 1 ? 8 : 6; }

template <int NR, int VEC>
__global__ __launch_bounds__(kQueryWaves * kWave) __attribute__((amdgpu_waves_per_eu(waves_per_simd(NR), 8))) void
k_index_query(IndexView ix, QueryBatch qb) {
    one_query_per_wave<NR, VEC>(ix, qb);
}

template <int VEC>
__global__ __launch_bounds__(kQueryWaves * kWave) void k_index_query_wide(IndexView ix, QueryBatch qb) {
    one_query_per_wave<16, VEC>(ix, qb);
}

template <int NR, int VEC>
__global__ __launch_bounds__(kQueryWaves * kWave) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_index_query_persistent(
    IndexView ix, QueryBatch qb, const int64_t* q_count, unsigned long long* counter) {
    queries_from_counter<NR, VEC>(ix, qb, q_count, counter);
}

// One wave per query of the capacity; waves past the device-side batch size
// leave at once.
template <int NR, int VEC>
__global__ __launch_bounds__(kQueryWaves * kWave) __attribute__((amdgpu_waves_per_eu(waves_per_simd(NR), 8))) void
k_index_query_counted(IndexView ix, QueryBatch qb, const int64_t* q_count) {
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t qi = (int64_t)blockIdx.x * kQueryWaves + wv;
    if (qi < *q_count) index_query_body<NR, VEC>(ix, qb, qi);
}

template <int VEC>
__global__ __launch_bounds__(kQueryWaves * kWave) void k_index_query_counted_wide(IndexView ix, QueryBatch qb,
                                                                                 const int64_t* q_count) {
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t qi = (int64_t)blockIdx.x * kQueryWaves + wv;
    if (qi < *q_count) index_query_body<16, VEC>(ix, qb, qi);
}

template <int VEC>
__global__ __launch_bounds__(kQueryWaves * kWave) void k_index_query_persistent_wide(IndexView ix, QueryBatch qb,
                                                                                    const int64_t* q_count,
                                                                                    unsigned long long* counter) {
    queries_from_counter<16, VEC>(ix, qb, q_count, counter);
}

__global__ void k_reset_counter(unsigned long long* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0ull;
}

template <int NR>
static hipError_t launch_nr(const IndexView& ix, const QueryBatch& qb, hipStream_t s) {
    const unsigned grid = (unsigned)((qb.Q + kQueryWaves - 1) / kQueryWaves);
    const size_t shm = (size_t)kQueryWaves * (ix.g.W * sizeof(uint32_t) + kAdjWindow);
    const dim3 blk(kQueryWaves * kWave);
    if constexpr (NR == 16) {
        if (ix.g.W % 4 == 0)
            hipLaunchKernelGGL((k_index_query_wide<4>), dim3(grid), blk, shm, s, ix, qb);
        else if (ix.g.W % 2 == 0)
            hipLaunchKernelGGL((k_index_query_wide<2>), dim3(grid), blk, shm, s, ix, qb);
        else
            hipLaunchKernelGGL((k_index_query_wide<1>), dim3(grid), blk, shm, s, ix, qb);
    } else {
        if (ix.g.W % 4 == 0)
            hipLaunchKernelGGL((k_index_query<NR, 4>), dim3(grid), blk, shm, s, ix, qb);
        else if (ix.g.W % 2 == 0)
            hipLaunchKernelGGL((k_index_query<NR, 2>), dim3(grid), blk, shm, s, ix, qb);
        else
            hipLaunchKernelGGL((k_index_query<NR, 1>), dim3(grid), blk, shm, s, ix, qb);
    }
    return hipGetLastError();
}

template <int NR>
static hipError_t launch_persistent_nr(const IndexView& ix, const QueryBatch& qb, const int64_t* q_count,
                                       unsigned long long* counter, int blocks, bool looping, hipStream_t s) {
    const size_t shm = (size_t)kQueryWaves * (ix.g.W * sizeof(uint32_t) + kAdjWindow);
    const dim3 blk(kQueryWaves * kWave);
    const dim3 grid((unsigned)blocks);
    const int vec = ix.g.W % 4 == 0 ? 4 : ix.g.W % 2 == 0 ? 2 : 1;
    if (!looping) {
        if constexpr (NR == 16) {
            if (vec == 4) hipLaunchKernelGGL((k_index_query_counted_wide<4>), grid, blk, shm, s, ix, qb, q_count);
            else if (vec == 2) hipLaunchKernelGGL((k_index_query_counted_wide<2>), grid, blk, shm, s, ix, qb, q_count);
            else hipLaunchKernelGGL((k_index_query_counted_wide<1>), grid, blk, shm, s, ix, qb, q_count);
        } else {
            if (vec == 4) hipLaunchKernelGGL((k_index_query_counted<NR, 4>), grid, blk, shm, s, ix, qb, q_count);
            else if (vec == 2) hipLaunchKernelGGL((k_index_query_counted<NR, 2>), grid, blk, shm, s, ix, qb, q_count);
            else hipLaunchKernelGGL((k_index_query_counted<NR, 1>), grid, blk, shm, s, ix, qb, q_count);
        }
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, counter);
    if constexpr (NR == 16) {
        if (vec == 4)
            hipLaunchKernelGGL((k_index_query_persistent_wide<4>), grid, blk, shm, s, ix, qb, q_count, counter);
        else if (vec == 2)
            hipLaunchKernelGGL((k_index_query_persistent_wide<2>), grid, blk, shm, s, ix, qb, q_count, counter);
        else
            hipLaunchKernelGGL((k_index_query_persistent_wide<1>), grid, blk, shm, s, ix, qb, q_count, counter);
    } else {
        if (vec == 4)
            hipLaunchKernelGGL((k_index_query_persistent<NR, 4>), grid, blk, shm, s, ix, qb, q_count, counter);
        else if (vec == 2)
            hipLaunchKernelGGL((k_index_query_persistent<NR, 2>), grid, blk, shm, s, ix, qb, q_count, counter);
        else
            hipLaunchKernelGGL((k_index_query_persistent<NR, 1>), grid, blk, shm, s, ix, qb, q_count, counter);
    }
    return hipGetLastError();
}

hipError_t launch_index_query_persistent(const IndexView& ix, const QueryBatch& qb, const int64_t* q_count,
                                         unsigned long long* counter, int blocks, bool looping, hipStream_t s) {
    if (qb.k_max <= 64) return launch_persistent_nr<1>(ix, qb, q_count, counter, blocks, looping, s);
    if (qb.k_max <= 128) return launch_persistent_nr<2>(ix, qb, q_count, counter, blocks, looping, s);
    if (qb.k_max <= 256) return launch_persistent_nr<4>(ix, qb, q_count, counter, blocks, looping, s);
    return launch_persistent_nr<16>(ix, qb, q_count, counter, blocks, looping, s);
}

hipError_t launch_index_query(const IndexView& ix, const QueryBatch& qb, hipStream_t s) {
    if (qb.Q <= 0) return hipSuccess;
    if (qb.k_max <= 64) return launch_nr<1>(ix, qb, s);
    if (qb.k_max <= 128) return launch_nr<2>(ix, qb, s);
    if (qb.k_max <= 256) return launch_nr<4>(ix, qb, s);
    return launch_nr<16>(ix, qb, s);
}

}  // namespace lcpx
