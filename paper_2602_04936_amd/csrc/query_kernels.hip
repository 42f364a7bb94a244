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
//     step also yields lL = LCP(q, T[p-1]) and lR = LCP(q, T[p]).
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

template <int NR, int VEC>
__global__ __launch_bounds__(kQueryWaves * kWave) void k_index_query(IndexView ix, QueryBatch qb) {
    extern __shared__ uint32_t s_q[];  // [kQueryWaves][W] query key words
    const RowGeo g = ix.g;
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t qi = (int64_t)blockIdx.x * kQueryWaves + wv;
    const bool live = qi < qb.Q;
    uint32_t* q = s_q + wv * g.W;
    if (live)
        for (int w = lane; w < g.W; w += kWave) q[w] = key_word(qb.raw, qi * g.L, g, w);
    __syncthreads();
    if (!live) return;

    const int64_t N = ix.N;
    const int k = qb.k[qi];
    const int64_t out0 = qb.off[qi];
    int32_t* __restrict__ oid = qb.out_ids + out0;
    int32_t* __restrict__ olc = qb.out_lcp + out0;
    const int kp = (int)((int64_t)k < N ? (int64_t)k : N);

    // ---- 1. insertion point and the LCPs of its two neighbours
    int64_t lo = 0, hi = N;
    int lcp_lo = -1, lcp_hi = -1;  // LCP(q, T[lo-1]), LCP(q, T[hi])
    int64_t p;
    int lL, lR;
    for (;;) {
        const int64_t n = hi - lo;
        int64_t pos;
        bool act;
        if (n <= kWave) {
            pos = lo + lane;
            act = lane < n;
        } else {
            pos = lo + ((int64_t)(lane + 1) * n) / (kWave + 1);
            act = true;
        }
        int lc;
        bool less;
        compare_row<VEC>(ix.sorted + (act ? pos : 0) * g.W, q, g, act, lc, less);
        const int cnt = popc64(ballot(less));  // pivots below q form a prefix of the lanes
        if (n <= kWave) {
            p = lo + cnt;
            lL = cnt > 0 ? readlane_i(lc, cnt - 1) : lcp_lo;
            lR = cnt < n ? readlane_i(lc, cnt) : lcp_hi;
            break;
        }
        if (cnt > 0) {
            lo = readlane_i64(pos, cnt - 1) + 1;
            lcp_lo = readlane_i(lc, cnt - 1);
        }
        if (cnt < kWave) {
            hi = readlane_i64(pos, cnt);
            lcp_hi = readlane_i(lc, cnt);
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
                const int64_t j = j0 + lane;
                const int a = j < N ? (int)ix.A[j] : -1;
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
                const int64_t i = i0 - lane;
                const int a = i >= 1 ? (int)ix.A[i] : -1;
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
            const int a = act ? (t == 0 ? lR : (int)ix.A[j]) : 255;
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
            const int a = act ? (t == 0 ? lL : (int)ix.A[j + 1]) : 255;
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
        } else {
            WaveList<NR> tied;
            tied.init();
            const int64_t nleft = in_lo - l;
            const int64_t tn = nleft + (r - in_hi);
            for (int64_t b = 0; b < tn; b += kWave) {
                const int64_t t = b + lane;
                const bool act = t < tn;
                const int64_t j = t < nleft ? l + t : in_hi + (t - nleft);
                const uint32_t id = act ? (uint32_t)ix.perm[j] : 0u;
                tied.offer((uint64_t)id, act, m);
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

template <int NR>
static hipError_t launch_nr(const IndexView& ix, const QueryBatch& qb, hipStream_t s) {
    const unsigned grid = (unsigned)((qb.Q + kQueryWaves - 1) / kQueryWaves);
    const size_t shm = (size_t)kQueryWaves * ix.g.W * sizeof(uint32_t);
    const dim3 blk(kQueryWaves * kWave);
    if (ix.g.W % 4 == 0)
        hipLaunchKernelGGL((k_index_query<NR, 4>), dim3(grid), blk, shm, s, ix, qb);
    else if (ix.g.W % 2 == 0)
        hipLaunchKernelGGL((k_index_query<NR, 2>), dim3(grid), blk, shm, s, ix, qb);
    else
        hipLaunchKernelGGL((k_index_query<NR, 1>), dim3(grid), blk, shm, s, ix, qb);
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
