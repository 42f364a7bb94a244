// Prefix-bucket range scan (section 6.2: Definition "Prefix Bucket",
// Theorem "Range Scan Complexity", Definition "Thermal-Aware Logic"; the range
// scan of Appendix D.1).
//
// Each query finds the range of sorted positions whose rows share its first d
// tokens (a prefix bucket is contiguous in the sorted order) and scans only
// that range: the LCP of every row in it, and the k best rows by (LCP
// descending, id ascending).  One wave per query.  The rows are streamed from
// a plane of the sorted order, coalesced: while the prefix ends inside key
// word 0, the first two key words of each row (8 bytes a row); once it covers
// whole words, which every row of the bucket shares with the query, only the
// next word, from a column of that word (4 bytes a row).  The full row is
// read only where the streamed words equal the query's, and the row's id only
// where the row can still enter the answer.
#include "device.hpp"
#include "launch.hpp"

namespace lcpx {

namespace {

constexpr int kBucketWaves = 4;     // waves (queries) per block
constexpr int kBucketUnroll = 1;    // 16-byte plane loads per lane and step (pair plane)
constexpr int kColUnroll = 1;       // the same for a column plane
constexpr int kBucketMaxW = (255 * 2 + 3) / 4;  // key words of the longest row: 255 two-byte tokens

// Order of the first d tokens of a row against the query's: nw whole key words,
// then the top bits `mask` of word nw (mask == 0: none).
__device__ __forceinline__ int cmp_prefix(const uint32_t* __restrict__ row, const uint32_t* q, int nw, uint32_t mask) {
    for (int w = 0; w < nw; ++w) {
        const uint32_t r = row[w], t = q[w];
        if (r != t) return r < t ? -1 : 1;
    }
    if (mask) {
        const uint32_t r = row[nw] & mask, t = q[nw] & mask;
        if (r != t) return r < t ? -1 : 1;
    }
    return 0;
}

// Both ends of the bucket at once: lanes 0-31 find the first sorted position
// whose row's d-prefix is >= the query's (lo), lanes 32-63 the first whose
// prefix is > it (hi).  Each half runs a 32-ary search over [0, N): per step
// its lanes probe the last position of 32 equal segments of the half's range
// and keep the segment where its predicate turns.
__device__ __forceinline__ void bucket_bounds(const uint32_t* __restrict__ sorted, int W, const uint32_t* q, int nw,
                                              uint32_t mask, int64_t N, int64_t& lo, int64_t& hi) {
    constexpr int kHalf = kWave / 2;
    const int lane = lane_id();
    const bool upper = lane >= kHalf;
    const int j = lane & (kHalf - 1);
    int64_t a = 0, b = N;  // the half's range: its answer lies in [a, b]
    while (ballot(a < b)) {
        const int64_t s = (b - a + kHalf - 1) / kHalf;
        const int64_t p = a + (int64_t)(j + 1) * s - 1;
        const bool valid = a < b && p < b;
        const int c = valid ? cmp_prefix(sorted + p * W, q, nw, mask) : 1;
        const bool before = valid && (upper ? c <= 0 : c < 0);
        const uint64_t bal = ballot(before);
        const int64_t cnt = popc64(upper ? bal >> kHalf : bal & ((1ull << kHalf) - 1));
        if (a < b) {
            const int64_t nb = a + (cnt + 1) * s - 1;
            a += cnt * s;
            b = nb < b ? nb : b;
        }
    }
    lo = readlane_i64(a, 0);
    hi = readlane_i64(a, kHalf);
}

// Column plane: key word w of every sorted row, zero-padded to a multiple of 4 rows.
__global__ void k_sorted_column(const uint32_t* __restrict__ sorted, int64_t N, int W, int w,
                                uint32_t* __restrict__ col) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < column_entries(N)) col[p] = p < N ? sorted[p * W + w] : 0u;
}

// kCol == false: `plane` is the pair plane (key words 0 and 1 of each sorted
// row, 8 bytes a row).  kCol == true: `plane` is the column of key word cw,
// and every row of the bucket shares words 0 .. cw-1 with the query.
// With one list register (k <= 64) the kernel is held to 64 VGPRs, so that 8
// waves fit per SIMD and a whole 8,192-query batch is resident at once.
template <int NR, bool kCol>
__global__ __launch_bounds__(kBucketWaves * kWave) __attribute__((amdgpu_waves_per_eu(NR == 1 ? 8 : 1))) void
k_bucket_scan(IndexView ix, const void* __restrict__ plane, int cw, QueryBatch qb, int depth,
              int32_t* __restrict__ bounds) {
    __shared__ uint32_t s_q[kBucketWaves][kBucketMaxW];
    const RowGeo g = ix.g;
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t qi = (int64_t)blockIdx.x * kBucketWaves + wv;
    if (qi >= qb.Q) return;  // whole waves: every wave only uses its own LDS row
    uint32_t* q = s_q[wv];
    for (int w = lane; w < g.W; w += kWave) q[w] = key_word(qb.raw, qi * g.L, g, w);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // ---- 1. the bucket: sorted positions [lo, hi) of the rows sharing q's first `depth` tokens
    int64_t lo = 0, hi = ix.N;
    if (depth > 0) {
        const int nw = depth >> g.tpw_log2;
        const int rem = depth & ((1 << g.tpw_log2) - 1);
        const uint32_t mask = rem ? ~0u << (32 - (rem << g.bits_log2)) : 0u;
        bucket_bounds(ix.sorted, g.W, q, nw, mask, ix.N, lo, hi);
    }
    if (bounds && lane == 0) {
        bounds[2 * qi] = (int32_t)lo;
        bounds[2 * qi + 1] = (int32_t)hi;
    }

    // ---- 2. scan it: LCP of every row, the k best keys kept in a wave list.
    // Each lane takes kRows adjacent rows per 16-byte load; a step is
    // kU loads per lane, and the next step's loads are issued
    // before this step's rows are compared.  The range is widened to whole
    // loads ([lo, hi) rounded out to multiples of kRows lies inside the plane,
    // whose entry count is such a multiple); rows outside [lo, hi) are masked.
    constexpr int kRows = kCol ? 4 : 2;
    const int k = query_k(qb, qi);
    const uint64_t qp = kCol ? (uint64_t)q[cw] : ((uint64_t)q[0] << 32) | (g.W > 1 ? q[1] : 0u);
    const int lcp_base = kCol ? cw << g.tpw_log2 : 0;  // tokens before the streamed words
    const int tail_from = kCol ? cw + 1 : 2;          // first key word not streamed
    WaveList<NR> list;
    list.init();
    uint64_t thr = kKeyMax;  // the k-th smallest key so far
    const int64_t a0 = lo & ~(int64_t)(kRows - 1);
    const int64_t hend = (hi + kRows - 1) & ~(int64_t)(kRows - 1);
    constexpr int kU = kCol ? kColUnroll : kBucketUnroll;
    constexpr int kStep = kU * kRows * kWave;
    auto load_rows = [&](int64_t b, int u) -> uint4 {
        int64_t p = b + (u * kWave + lane) * kRows;
        p = p < hend ? p : hend - kRows;
        if constexpr (kCol)
            return *reinterpret_cast<const uint4*>(static_cast<const uint32_t*>(plane) + p);
        else
            return *reinterpret_cast<const uint4*>(static_cast<const uint64_t*>(plane) + p);
    };
    auto row_lcp = [&](uint64_t v, int64_t p) -> int {
        const uint64_t x = v ^ qp;
        int lcp;
        if constexpr (kCol)
            lcp = x ? lcp_base + (__clz((int)(uint32_t)x) >> g.bits_log2) : g.L;
        else
            lcp = x ? (int)(__clzll((long long)x) >> g.bits_log2) : g.L;
        if (x == 0 && tail_from < g.W && p < hi) lcp = lcp_tail(ix.sorted + p * g.W, q, g, tail_from);
        return lcp;
    };
    auto scan_step = [&](const uint4 (&buf)[kU], int64_t base) {
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t p0 = base + (u * kWave + lane) * kRows;
            uint64_t v[kRows];
            if constexpr (kCol) {
                v[0] = buf[u].x;
                v[1] = buf[u].y;
                v[2] = buf[u].z;
                v[3] = buf[u].w;
            } else {
                v[0] = ((uint64_t)buf[u].y << 32) | buf[u].x;
                v[1] = ((uint64_t)buf[u].w << 32) | buf[u].z;
            }
            int lcp[kRows];
            bool c[kRows];
            bool any = false;
            // a row enters only with an LCP of at least the k-th key's (its id decides a tie)
            const int tl = thr == kKeyMax ? -1 : key_lcp(thr);
#pragma unroll
            for (int r = 0; r < kRows; ++r) {
                lcp[r] = row_lcp(v[r], p0 + r);
                c[r] = p0 + r >= lo && p0 + r < hi && lcp[r] >= tl;
                any = any || c[r];
            }
            if (ballot(any)) {
#pragma unroll
                for (int r = 0; r < kRows; ++r) {
                    const uint32_t id = c[r] ? (uint32_t)ix.perm[p0 + r] : 0u;
                    list.offer(rank_key(lcp[r], id), c[r], k);
                }
                thr = list.get(k - 1);
            }
        }
    };
    // two register sets in turn: one step's loads are in flight while the
    // other's rows are compared, with no copy between them
    uint4 ba[kU], bb[kU];
    if (lo < hi) {
#pragma unroll
        for (int u = 0; u < kU; ++u) ba[u] = load_rows(a0, u);
    }
    for (int64_t base = a0; base < hi;) {
#pragma unroll
        for (int u = 0; u < kU; ++u) bb[u] = load_rows(base + kStep, u);
        scan_step(ba, base);
        base += kStep;
        if (base >= hi) break;
#pragma unroll
        for (int u = 0; u < kU; ++u) ba[u] = load_rows(base + kStep, u);
        scan_step(bb, base);
        base += kStep;
    }

    // ---- 3. emit in rank order; entries past the bucket's size are (-1, -1)
    const int64_t out0 = query_off(qb, qi);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int e = r * kWave + lane;
        if (e < k) {
            const uint64_t key = list.v[r];
            qb.out_ids[out0 + e] = key == kKeyMax ? -1 : key_id(key);
            qb.out_lcp[out0 + e] = key == kKeyMax ? -1 : key_lcp(key);
        }
    }
}

template <int NR, bool kCol>
hipError_t launch_bucket_t(const IndexView& ix, const void* plane, int cw, const QueryBatch& qb, int depth,
                           int32_t* bounds, hipStream_t s) {
    const int64_t blocks = (qb.Q + kBucketWaves - 1) / kBucketWaves;
    hipLaunchKernelGGL((k_bucket_scan<NR, kCol>), dim3((unsigned)blocks), dim3(kBucketWaves * kWave), 0, s, ix, plane,
                       cw, qb, depth, bounds);
    return hipGetLastError();
}

template <bool kCol>
hipError_t launch_bucket_k(const IndexView& ix, const void* plane, int cw, const QueryBatch& qb, int depth,
                           int32_t* bounds, hipStream_t s) {
    if (qb.k_max <= 64) return launch_bucket_t<1, kCol>(ix, plane, cw, qb, depth, bounds, s);
    if (qb.k_max <= 128) return launch_bucket_t<2, kCol>(ix, plane, cw, qb, depth, bounds, s);
    if (qb.k_max <= 256) return launch_bucket_t<4, kCol>(ix, plane, cw, qb, depth, bounds, s);
    return launch_bucket_t<16, kCol>(ix, plane, cw, qb, depth, bounds, s);
}

}  // namespace

int bucket_column(int depth, const RowGeo& g) {
    if (depth < (1 << g.tpw_log2)) return -1;
    const int w = depth >> g.tpw_log2;
    return w < g.W ? w : g.W - 1;
}

hipError_t launch_sorted_column(const uint32_t* sorted, int64_t N, int W, int w, uint32_t* col, hipStream_t s) {
    const int64_t n = column_entries(N);
    hipLaunchKernelGGL(k_sorted_column, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, sorted, N, W, w, col);
    return hipGetLastError();
}

hipError_t launch_bucket_scan(const IndexView& ix, const void* plane, const QueryBatch& qb, int depth,
                              int32_t* bounds, hipStream_t s) {
    if (qb.Q <= 0) return hipSuccess;
    const int cw = bucket_column(depth, ix.g);
    if (cw >= 0) return launch_bucket_k<true>(ix, plane, cw, qb, depth, bounds, s);
    return launch_bucket_k<false>(ix, plane, 0, qb, depth, bounds, s);
}

}  // namespace lcpx
