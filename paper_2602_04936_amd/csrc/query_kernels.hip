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
//     (one coalesced 1 KB load per step, resident in L2) and touch a
//     pivot row only on a tie; the last step reads its at most 64 contiguous
//     rows.  The steps also yield lL = LCP(q, T[p-1]) and lR = LCP(q, T[p]).
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
constexpr int kFewTied = 16;  // tied selections of at most this many ids use repeated wave minima

// A[j] for the 64 positions j = j0 + dir * lane: from the wave's LDS window
// when the whole chunk lies inside it, else from global memory.  Lanes whose
// position is outside [lo_ok, hi_ok] get -1.
__device__ __forceinline__ int a_lane(const uint8_t* __restrict__ A, const uint8_t* win, int64_t wbase, int64_t j0,
                                      int dir, int64_t lo_ok, int64_t hi_ok) {
    const int lane = lane_id();
    const int64_t j = j0 + dir * lane;
    const int64_t jmin = dir > 0 ? j0 : j0 - (kWave - 1);
    const int64_t jmax = dir > 0 ? j0 + (kWave - 1) : j0;
    const bool in_win = jmin >= wbase && jmax < wbase + kAdjWindow;
    if (j < lo_ok || j > hi_ok) return -1;
    return in_win ? (int)win[j - wbase] : (int)A[j];
}

template <int NR, int VEC>
__device__ __forceinline__ void index_query_body(const IndexView& ix, const QueryBatch& qb) {
    extern __shared__ uint32_t s_dyn[];  // [kQueryWaves][W] query words, then [kQueryWaves][kAdjWindow] A bytes
    const RowGeo g = ix.g;
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t qi = (int64_t)blockIdx.x * kQueryWaves + wv;
    const bool live = qi < qb.Q;
    uint32_t* q = s_dyn + wv * g.W;
    uint8_t* win = reinterpret_cast<uint8_t*>(s_dyn + kQueryWaves * g.W) + wv * kAdjWindow;
    if (live)
        for (int w = lane; w < g.W; w += kWave) q[w] = key_word(qb.raw, qi * g.L, g, w);
    __syncthreads();
    if (!live) return;

    const int64_t N = ix.N;
    const int k = query_k(qb, qi);
    const int64_t out0 = query_off(qb, qi);
    int32_t* __restrict__ oid = qb.out_ids + out0;
    int32_t* __restrict__ olc = qb.out_lcp + out0;
    const int kp = (int)((int64_t)k < N ? (int64_t)k : N);

    // ---- 1. insertion point and the LCPs of its two neighbours
    // the query's first four key words as two 64-bit halves (zero past the row's end)
    const uint64_t qa = ((uint64_t)q[0] << 32) | (g.W > 1 ? q[1] : 0u);
    const uint64_t qb2 = ((uint64_t)(g.W > 2 ? q[2] : 0u) << 32) | (g.W > 3 ? q[3] : 0u);
    int64_t lo = 0, hi = N;
    int lcp_lo = -1, lcp_hi = -1;  // LCP(q, T[lo-1]), LCP(q, T[hi])
    int64_t p;
    int lL, lR;
    int64_t wbase;
    int depth = 0;
    int64_t node = 0, level_start = 0;  // table node and the entry where its level starts
    for (;;) {
        const int64_t n = hi - lo;
        if (n <= kWave) {
            // last step: the rows [lo, hi) are contiguous; the A window around
            // lo (p is within 64 of it) is fetched in the same round trip
            wbase = lo - kAdjWindow / 2;
            wbase = wbase < 0 ? 0 : wbase & ~(int64_t)15;
            const uint4 av = *reinterpret_cast<const uint4*>(ix.A + wbase + 16 * lane);
            const bool act = lane < n;
            int lc;
            bool less;
            compare_row<VEC>(ix.sorted + (act ? lo + lane : 0) * g.W, q, g, act, lc, less);
            *reinterpret_cast<uint4*>(win + 16 * lane) = av;
            const int cnt = popc64(ballot(less));
            p = lo + cnt;
            lL = cnt > 0 ? readlane_i(lc, cnt - 1) : lcp_lo;
            lR = cnt < n ? readlane_i(lc, cnt) : lcp_hi;
            break;
        }
        const int64_t pos = lo + ((int64_t)(lane + 1) * n) / (kWave + 1);
        int lc;
        bool less;
        if (depth < ix.stab_levels) {
            // pivot's first four key words from the table (one coalesced load)
            const uint4 e = ix.stab[level_start + node * kWave + lane];
            const uint64_t ka = ((uint64_t)e.x << 32) | e.y;
            const uint64_t kb = ((uint64_t)e.z << 32) | e.w;
            if (ka != qa) {
                lc = (int)(__clzll((long long)(ka ^ qa)) >> g.bits_log2);
                less = ka < qa;
            } else if (kb != qb2) {
                lc = (int)((64 + __clzll((long long)(kb ^ qb2))) >> g.bits_log2);
                less = kb < qb2;
            } else {  // tie on the first four words: compare the rest of the row
                lc = g.L;
                less = false;
                const uint32_t* row = ix.sorted + pos * g.W;
                for (int w = 4; w < g.W; ++w) {
                    const uint32_t rw = row[w];
                    if (rw != q[w]) {
                        lc = lcp_from_diff(w, rw ^ q[w], g);
                        less = rw < q[w];
                        break;
                    }
                }
            }
        } else {
            compare_row<VEC>(ix.sorted + pos * g.W, q, g, true, lc, less);
        }
        const int cnt = popc64(ballot(less));  // pivots below q form a prefix of the lanes
        if (cnt > 0) {
            lo = readlane_i64(pos, cnt - 1) + 1;
            lcp_lo = readlane_i(lc, cnt - 1);
        }
        if (cnt < kWave) {
            hi = readlane_i64(pos, cnt);
            lcp_hi = readlane_i(lc, cnt);
        }
        if (depth < ix.stab_levels) {
            node = node * (kWave + 1) + cnt;
            level_start = level_start * (kWave + 1) + kWave;
            ++depth;
        }
    }

    // ---- 2. walk outward level by level: group [l, r) = G_lev
    int64_t l = p, r = p;
    int vr = p < N ? lR : -1;  // LCP(q, T[r]), -1 past the end
    int vl = p > 0 ? lL : -1;  // LCP(q, T[l-1]), -1 before the start
    int lev = vr > vl ? vr : vl;
    int64_t in_lo = p, in_hi = p;  // G_{c+1}
    int c;
    for (;;) {
        if (lev <= 0) {
            l = 0;
            r = N;
            c = 0;
            break;
        }
        if (vr >= lev) {  // T[r] is in: extend to the first j > r with A[j] < lev
            for (int64_t j0 = r + 1;; j0 += kWave) {
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
            for (int64_t i0 = l - 1;; i0 -= kWave) {
                const int a = a_lane(ix.A, win, wbase, i0, -1, 1, N - 1);  // -1 at i < 1 stops
                const uint64_t stop = ballot(a < lev);
                if (stop) {
                    const int f = low_lane(stop);
                    const int64_t ii = i0 - f;
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

    // ---- 3. inner group G_{c+1}, ranked by (LCP desc, id asc)
    if (n_gt > 0) {
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

    // ---- 4. the m lowest ids among rows with LCP exactly c
    if (m > 0) {
        if (c == 0) {
            const uint32_t q0 = q[0];
            const int drop = 32 - 8 * g.tb;
            int got = 0;
            for (int64_t b = 0; got < m && b < N; b += kWave) {
                const int64_t id = b + lane;
                const bool hit = id < N && ((ix.rows[id * g.W] ^ q0) >> drop) != 0u;
                const uint64_t bal = ballot(hit);
                const int rank = got + count_below(bal);
                if (hit && rank < m) {
                    oid[n_gt + rank] = (int32_t)id;
                    olc[n_gt + rank] = 0;
                }
                got += popc64(bal);
            }
        } else if (m <= kFewTied && (r - l) - n_gt <= kTieUnroll * kWave) {
            // small case: every tied id in registers, then m rounds of "take the
            // wave minimum and remove it"
            const int64_t nleft = in_lo - l;
            const int64_t tn = nleft + (r - in_hi);
            uint32_t id[kTieUnroll];
#pragma unroll
            for (int u = 0; u < kTieUnroll; ++u) {
                const int64_t t = u * kWave + lane;
                const int64_t j = t < nleft ? l + t : in_hi + (t - nleft);
                id[u] = t < tn ? (uint32_t)ix.perm[j] : 0xFFFFFFFFu;
            }
            uint32_t mine = 0xFFFFFFFFu;  // lane e keeps the e-th smallest
            for (int e = 0; e < m; ++e) {
                uint32_t v = id[0];
#pragma unroll
                for (int u = 1; u < kTieUnroll; ++u) v = id[u] < v ? id[u] : v;
                v = wave_min_u32(v);
                if (lane == e) mine = v;
#pragma unroll
                for (int u = 0; u < kTieUnroll; ++u) id[u] = id[u] == v ? 0xFFFFFFFFu : id[u];
            }
            if (lane < m) {
                oid[n_gt + lane] = (int32_t)mine;
                olc[n_gt + lane] = c;
            }
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

// Small lists: registers are capped so that 8 waves fit per SIMD and a whole
// 8,192-query batch is resident at once.  Large lists (k > 256) keep their
// registers instead.
template <int NR, int VEC>
__global__ __launch_bounds__(kQueryWaves * kWave) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_index_query(
    IndexView ix, QueryBatch qb) {
    index_query_body<NR, VEC>(ix, qb);
}

template <int VEC>
__global__ __launch_bounds__(kQueryWaves * kWave) void k_index_query_wide(IndexView ix, QueryBatch qb) {
    index_query_body<16, VEC>(ix, qb);
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

hipError_t launch_index_query(const IndexView& ix, const QueryBatch& qb, hipStream_t s) {
    if (qb.Q <= 0) return hipSuccess;
    if (qb.k_max <= 64) return launch_nr<1>(ix, qb, s);
    if (qb.k_max <= 128) return launch_nr<2>(ix, qb, s);
    if (qb.k_max <= 256) return launch_nr<4>(ix, qb, s);
    return launch_nr<16>(ix, qb, s);
}

}  // namespace lcpx
