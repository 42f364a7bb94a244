// Index construction: pack + validate, stable LSD radix sort, row gather,
// adjacent LCP.
//
// The paper builds a pointer trie whose leaves, read left to right with each
// leaf's posting list in insertion order, give the rows in lexicographic order
// with equal rows by id (section 5.2, Algorithms 1-2).  Here that order is
// produced directly: a stable least-significant-digit radix sort of row ids
// keyed on a dense bit packing of each row (ceil(log2 V) bits per token,
// position 0 most significant), starting from the identity permutation so that
// equal rows keep ascending ids.  The adjacent-LCP array then stores, for each
// sorted position, the depth of the deepest trie node shared with the previous
// row; any trie node of depth d is the contiguous range where it stays >= d.
#include "device.hpp"
#include "launch.hpp"

namespace lcpx {

// ------------------------------------------------------------ pack/validate

// One thread per (row, key word): key-form row in id order + token range check
// (a token >= V raises *bad to at least `mark`).
__global__ void k_pack_keys(const void* __restrict__ tokens, int64_t N, RowGeo g, uint32_t V,
                            uint32_t* __restrict__ keys, uint32_t* __restrict__ bad, uint32_t mark) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * g.W) return;
    const int64_t row = t / g.W;
    const int w = (int)(t - row * g.W);
    const int tpw = 1 << g.tpw_log2;
    const int bits = 8 * g.tb;
    uint32_t x = 0;
    bool out_of_range = false;
    for (int j = 0; j < tpw; ++j) {
        const int pos = w * tpw + j;
        uint32_t v = 0;
        if (pos < g.L) {
            v = raw_token(tokens, row * g.L + pos, g.tb);
            out_of_range |= v >= V;
        }
        x |= v << (32 - bits * (j + 1));
    }
    keys[t] = x;
    if (out_of_range) atomicMax(bad, mark);
}

// One thread per (row, dense word): tokens at `dbits` bits each, concatenated
// most significant first into a bit string, cut into 32-bit words.
__global__ void k_pack_dense(const void* __restrict__ tokens, int64_t N, RowGeo g, int dbits, int Wd,
                             uint32_t* __restrict__ dense) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * Wd) return;
    const int64_t row = t / Wd;
    const int d = (int)(t - row * Wd);
    const int first = (32 * d) / dbits;
    int last = (32 * d + 31) / dbits;
    if (last > g.L - 1) last = g.L - 1;
    uint32_t x = 0;
    for (int j = first; j <= last; ++j) {
        const uint64_t v = raw_token(tokens, row * g.L + j, g.tb);
        const int sh = 32 - (j * dbits - 32 * d) - dbits;  // left shift inside this word
        x |= sh >= 0 ? (uint32_t)(v << sh) : (uint32_t)(v >> (-sh));
    }
    dense[t] = x;
}

// OR over rows of (word ^ word of row 0): the bits that vary in each dense
// word.  The grid has Wd * gx blocks of 256 threads, so the grid stride is a
// multiple of Wd and every thread reads one fixed word position d of the flat
// [N][Wd] array with coalesced loads.
__global__ __launch_bounds__(256) void k_varying_bits(const uint32_t* __restrict__ dense, int64_t N, int Wd,
                                                       uint32_t* __restrict__ vary) {
    __shared__ uint32_t acc_d[128];
    for (int i = threadIdx.x; i < Wd; i += 256) acc_d[i] = 0;
    __syncthreads();
    const int64_t tid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * 256;
    const int d = (int)(tid % Wd);
    const uint32_t ref = dense[d];
    uint32_t acc = 0;
    for (int64_t e = tid; e < N * Wd; e += stride) acc |= dense[e] ^ ref;
    if (acc) atomicOr(&acc_d[d], acc);  // OR is order independent
    __syncthreads();
    for (int i = threadIdx.x; i < Wd; i += 256)
        if (acc_d[i]) atomicOr(&vary[i], acc_d[i]);
}

__global__ void k_iota(int32_t* __restrict__ p, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) p[i] = (int32_t)i;
}

__global__ void k_gather_word(const uint32_t* __restrict__ dense, const int32_t* __restrict__ perm, int64_t N,
                              int Wd, int d, uint32_t* __restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) keys[i] = dense[(int64_t)perm[i] * Wd + d];
}

// ------------------------------------------------------------ radix pass
//
// Tile of kTile = 256 threads x 16 items.  Histogram, exclusive scan over
// (digit, tile) in digit-major order, then a stable scatter: inside a tile
// the items are ranked in index order (wave by wave, and inside a wave item
// slot by item slot, lanes in ascending order), so equal digits keep their
// relative order.

constexpr int kRadixThreads = 256;
constexpr int kRadixItems = 16;
constexpr int kTile = kRadixThreads * kRadixItems;   // 4096
constexpr int kWaveSpan = kWave * kRadixItems;        // 1024 items per wave

__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(const uint32_t* __restrict__ keys, int64_t N, int shift,
                                                               uint32_t* __restrict__ counts, int ntiles) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int j = 0; j < kRadixItems; ++j) {
        const int64_t i = base + (int64_t)j * kRadixThreads + threadIdx.x;
        if (i < N) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of the (digit, tile) counts: per-block sums, a scan of the
// block sums by one block, then each block scans its span and adds its base.
constexpr int kScanSpan = 4096;  // elements per block (256 threads x 16)

__device__ __forceinline__ uint32_t block_exclusive_256(uint32_t v, uint32_t* wave_tot, uint32_t& total) {
    // exclusive prefix of v over the 256 threads of the block; total = block sum
    const int lane = lane_id();
    const int wv = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t o = __shfl_up(x, d);
        if (lane >= d) x += o;
    }
    if (lane == kWave - 1) wave_tot[wv] = x;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
    for (int w = 0; w < 4; ++w) {
        const uint32_t t = wave_tot[w];
        if (w < wv) before += t;
        total += t;
    }
    __syncthreads();
    return before + x - v;
}

__global__ __launch_bounds__(256) void k_span_sums(const uint32_t* __restrict__ a, int64_t n,
                                                   uint32_t* __restrict__ sums) {
    __shared__ uint32_t wt[4];
    const int64_t base = (int64_t)blockIdx.x * kScanSpan;
    uint32_t s = 0;
    for (int j = 0; j < kScanSpan / 256; ++j) {
        const int64_t i = base + (int64_t)j * 256 + threadIdx.x;
        if (i < n) s += a[i];
    }
    uint32_t total;
    block_exclusive_256(s, wt, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// exclusive scan of nb block sums (one block; nb <= 1024 * 64)
__global__ __launch_bounds__(1024) void k_scan_sums(uint32_t* __restrict__ sums, int nb) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int per = (nb + 1023) / 1024;
    const int lo = t * per;
    const int hi = lo + per < nb ? lo + per : nb;
    uint32_t s = 0;
    for (int i = lo; i < hi; ++i) s += sums[i];
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const uint32_t v = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = t > 0 ? part[t - 1] : 0u;
    for (int i = lo; i < hi; ++i) {
        const uint32_t v = sums[i];
        sums[i] = run;
        run += v;
    }
}

__global__ __launch_bounds__(256) void k_span_scan(uint32_t* __restrict__ a, int64_t n,
                                                   const uint32_t* __restrict__ sums) {
    __shared__ uint32_t wt[4];
    // thread t owns 16 consecutive elements of the span
    const int64_t i0 = (int64_t)blockIdx.x * kScanSpan + (int64_t)threadIdx.x * 16;
    uint32_t v[16];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        v[j] = i0 + j < n ? a[i0 + j] : 0u;
        s += v[j];
    }
    uint32_t total;
    uint32_t run = sums[blockIdx.x] + block_exclusive_256(s, wt, total);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (i0 + j < n) a[i0 + j] = run;
        run += v[j];
    }
}

__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(const uint32_t* __restrict__ keys_in,
                                                                  const int32_t* __restrict__ vals_in, int64_t N,
                                                                  int shift, const uint32_t* __restrict__ offsets,
                                                                  int ntiles, uint32_t* __restrict__ keys_out,
                                                                  int32_t* __restrict__ vals_out, int write_keys) {
    __shared__ uint32_t cnt[4][256];
    const int lane = lane_id();
    const int wv = threadIdx.x >> 6;
    for (int b = threadIdx.x; b < 4 * 256; b += kRadixThreads) (&cnt[0][0])[b] = 0;
    __syncthreads();

    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)wv * kWaveSpan;
    uint32_t key[kRadixItems];
    int32_t val[kRadixItems];
    uint32_t dig[kRadixItems];
    uint32_t pos[kRadixItems];
#pragma unroll
    for (int j = 0; j < kRadixItems; ++j) {
        const int64_t i = base + (int64_t)j * kWave + lane;
        const bool ok = i < N;
        key[j] = ok ? keys_in[i] : 0u;
        val[j] = ok ? vals_in[i] : 0;
        dig[j] = (key[j] >> shift) & 255u;
        // lanes holding the same digit: intersect the ballots of its 8 bits
        uint64_t peers = ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dig[j] >> b) & 1u;
            const uint64_t m = ballot(ok && bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t before = ok ? cnt[wv][dig[j]] : 0u;
        pos[j] = before + (uint32_t)count_below(peers);
        if (ok && low_lane(peers) == lane) cnt[wv][dig[j]] = before + (uint32_t)popc64(peers);
        if (!ok) dig[j] = 256;  // marks an empty slot
    }
    __syncthreads();
    // per digit: exclusive prefix over the 4 waves, plus the tile's global offset
    {
        const int d = threadIdx.x;
        uint32_t run = offsets[(int64_t)d * ntiles + blockIdx.x];
        for (int w = 0; w < 4; ++w) {
            uint32_t c = cnt[w][d];
            cnt[w][d] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kRadixItems; ++j) {
        if (dig[j] < 256) {
            const uint32_t dst = cnt[wv][dig[j]] + pos[j];
            if ((int64_t)dst < N) {  // always true when the counts agree; never write out of bounds
                if (write_keys) keys_out[dst] = key[j];
                vals_out[dst] = val[j];
            }
        }
    }
}

// ------------------------------------------------------------ rows, A

__global__ void k_gather_rows(const uint32_t* __restrict__ keys, const int32_t* __restrict__ perm, int64_t N, int W,
                              uint32_t* __restrict__ sorted) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * W) return;
    const int64_t i = t / W;
    const int w = (int)(t - i * W);
    sorted[t] = keys[(int64_t)perm[i] * W + w];
}

__global__ void k_adjacent_lcp(const uint32_t* __restrict__ sorted, int64_t N, RowGeo g, uint8_t* __restrict__ A) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    if (i == 0) {
        A[0] = 0;
        return;
    }
    const uint32_t* a = sorted + (i - 1) * g.W;
    const uint32_t* b = a + g.W;
    int l = g.L;
    for (int w = 0; w < g.W; ++w) {
        const uint32_t x = a[w] ^ b[w];
        if (x) {
            l = lcp_from_diff(w, x, g);
            break;
        }
    }
    A[i] = (uint8_t)l;
}

static inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

// ------------------------------------------------------------ search tables

int search_table_levels(int64_t N) {
    int levels = 0;
    int64_t m = N;  // typical node size at the next level
    while (levels < kSearchTableMaxLevels && m > kWave) {
        ++levels;
        m /= kWave + 1;
    }
    return levels;
}

int64_t search_table_entries(int levels) {
    int64_t p = 1;
    for (int d = 0; d < levels; ++d) p *= kWave + 1;
    return p - 1;
}

// One thread per table entry: walk the node's path from the root (the same
// integer arithmetic as the query's search), then store its pivot's first four
// key words (zero past the row's end).  Entries of nodes the search never
// reaches are zero.
// Scan prefix plane: the first two key words of every row as one 64-bit value
// (word 0 in the high half), id order, so the full scan streams 8 bytes per
// row instead of the whole row.  An odd N gets one zero entry after the last
// row, so the plane is read as whole 16-byte pairs of rows.
// Entries [from, plane_entries(to)) are written (an append fills in its new rows).
__global__ void k_prefix_plane(const uint32_t* __restrict__ rows, int64_t from, int64_t to, int W,
                               uint64_t* __restrict__ plane) {
    const int64_t i = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= plane_entries(to)) return;
    plane[i] = i < to ? ((uint64_t)rows[i * W] << 32) | (W > 1 ? rows[i * W + 1] : 0u) : 0ull;
}

// First-token directory (the prefix buckets of depth one, section 6.2): one
// thread per token value, a binary search over the sorted rows' first tokens.
__global__ void k_first_token_dir(const uint32_t* __restrict__ sorted, int64_t N, int W, int tb, int V,
                                  uint32_t* __restrict__ dir) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > V + 1) return;
    int64_t lo = 0, hi = N;
    if (t >= V) lo = N;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if ((int64_t)(sorted[mid * W] >> (32 - 8 * tb)) < t)
            lo = mid + 1;
        else
            hi = mid;
    }
    dir[t] = (uint32_t)lo;
}

// Tie summaries: bmin[b] = the smallest id among sorted positions
// [64b, min(64b + 64, N)).  One wave per block of positions.
__global__ void k_block_min(const int32_t* __restrict__ perm, int64_t N, uint32_t* __restrict__ bmin) {
    const int64_t nb = (N + kWave - 1) / kWave;
    const int64_t b = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (b >= nb) return;  // whole waves leave together
    const int64_t j = b * kWave + lane_id();
    const uint32_t v = wave_min_u32(j < N ? (uint32_t)perm[j] : 0xFFFFFFFFu);
    if (lane_id() == 0) bmin[b] = v;
}

__device__ __forceinline__ void search_table_entry(int64_t t, const uint32_t* __restrict__ sorted, int64_t N, int W,
                                                   int levels, uint4* __restrict__ stab) {
    int64_t total = 1;
    for (int d = 0; d < levels; ++d) total *= kWave + 1;
    if (t >= total - 1) return;
    int d = 0;
    int64_t level_start = 0, level_nodes = 1;
    while (t >= level_start + level_nodes * kWave) {
        level_start += level_nodes * kWave;
        level_nodes *= kWave + 1;
        ++d;
    }
    const int64_t local = t - level_start;
    const int64_t node = local / kWave;
    const int i = (int)(local - node * kWave);
    int64_t lo = 0, hi = N;
    int64_t rest = node, div = level_nodes / (kWave + 1);
    bool reachable = true;
    for (int e = 0; e < d; ++e) {  // digits of `node` in base 65, most significant first
        const int64_t n = hi - lo;
        if (n <= kWave) {
            reachable = false;
            break;
        }
        const int c = (int)(rest / div);
        rest -= (int64_t)c * div;
        div /= kWave + 1;
        const int64_t left = c > 0 ? lo + ((int64_t)c * n) / (kWave + 1) + 1 : lo;
        const int64_t right = c < kWave ? lo + ((int64_t)(c + 1) * n) / (kWave + 1) : hi;
        lo = left;
        hi = right;
    }
    uint4 key = make_uint4(0u, 0u, 0u, 0u);
    if (reachable && hi - lo > kWave) {
        const int64_t pos = lo + ((int64_t)(i + 1) * (hi - lo)) / (kWave + 1);
        const uint32_t* r = sorted + pos * W;
        key.x = r[0];
        key.y = W > 1 ? r[1] : 0u;
        key.z = W > 2 ? r[2] : 0u;
        key.w = W > 3 ? r[3] : 0u;
    }
    stab[t] = key;
}

__global__ void k_search_tables(const uint32_t* __restrict__ sorted, int64_t N, int W, int levels,
                                uint4* __restrict__ stab) {
    search_table_entry((int64_t)blockIdx.x * blockDim.x + threadIdx.x, sorted, N, W, levels, stab);
}

// ------------------------------------------------------------ append (merge)

// -1, 0, +1: order of two key-form rows
__device__ __forceinline__ int compare_rows(const uint32_t* a, const uint32_t* b, int W) {
    for (int w = 0; w < W; ++w)
        if (a[w] != b[w]) return a[w] < b[w] ? -1 : 1;
    return 0;
}

// One thread per new row: binary search for the number of old rows <= it
// (old rows equal to a new row come first: they have smaller ids).
__global__ void k_upper_bounds(const uint32_t* __restrict__ sorted, int64_t N, const uint32_t* __restrict__ newrows,
                               int64_t n, int W, int64_t* __restrict__ ub) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint32_t* x = newrows + j * W;
    int64_t lo = 0, hi = N;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (compare_rows(sorted + mid * W, x, W) <= 0)
            lo = mid + 1;
        else
            hi = mid;
    }
    ub[j] = lo;
}

// Small appends, one wave per new row j (n <= kRankSortMax):
//  - its rank among the new rows: #{i : row i < row j, or row i == row j and
//    i < j}, 64 rows per ballot, their leading 64 bits compared first and the
//    remaining words only where those agree (a stable sort by rank);
//  - its upper bound among the old sorted rows (the number of old rows <= it;
//    old rows equal to it come first: they have smaller ids) by a 65-ary
//    search: 64 lanes compare 64 pivots per step, ceil(log65 N) steps;
//  - the row, its local id and its upper bound written at its rank.
__device__ __forceinline__ int compare_tail(const uint32_t* a, const uint32_t* b, int from, int W) {
    for (int w = from; w < W; ++w)
        if (a[w] != b[w]) return a[w] < b[w] ? -1 : 1;
    return 0;
}

constexpr int kRankUbWaves = 4;
constexpr int kRankUnroll = 8;
__global__ __launch_bounds__(kRankUbWaves * kWave) void k_rank_ub(const uint32_t* __restrict__ keys, int64_t n,
                                                                  const uint32_t* __restrict__ old_sorted,
                                                                  int64_t N, int W, uint32_t* __restrict__ sorted,
                                                                  int32_t* __restrict__ lperm,
                                                                  int64_t* __restrict__ ub) {
    const int lane = lane_id();
    const int64_t j = (int64_t)blockIdx.x * kRankUbWaves + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (j >= n) return;  // whole waves leave together
    const uint32_t* mine = keys + j * W;
    const uint64_t pj = ((uint64_t)mine[0] << 32) | (W > 1 ? mine[1] : 0u);
    // rank: kRankUnroll groups of 64 rows per round, all loads in flight first
    int64_t rank = 0;
    for (int64_t b = 0; b < n; b += (int64_t)kRankUnroll * kWave) {
        uint64_t pv[kRankUnroll];
#pragma unroll
        for (int u = 0; u < kRankUnroll; ++u) {
            const int64_t i = b + u * kWave + lane;
            const uint32_t* o = keys + (i < n ? i : 0) * W;
            pv[u] = ((uint64_t)o[0] << 32) | (W > 1 ? o[1] : 0u);
        }
#pragma unroll
        for (int u = 0; u < kRankUnroll; ++u) {
            const int64_t i = b + u * kWave + lane;
            const bool act = i < n;
            int c = pv[u] < pj ? -1 : pv[u] > pj ? 1 : 0;
            if (act && c == 0 && i != j && W > 2) c = compare_tail(keys + i * W, mine, 2, W);
            rank += popc64(ballot(act && (c < 0 || (c == 0 && i < j))));
        }
    }
    // upper bound among the old rows
    int64_t lo = 0, hi = N;
    while (hi - lo > kWave) {
        const int64_t len = hi - lo;
        const int64_t a65 = len / (kWave + 1), b65 = len - (kWave + 1) * a65;
        const int64_t pos = lo + (lane + 1) * a65 + ((lane + 1) * b65) / (kWave + 1);
        const uint32_t* o = old_sorted + pos * W;
        const uint64_t po = ((uint64_t)o[0] << 32) | (W > 1 ? o[1] : 0u);
        int c = po < pj ? -1 : po > pj ? 1 : 0;
        if (c == 0 && W > 2) c = compare_tail(o, mine, 2, W);
        const int cnt = popc64(ballot(c <= 0));  // pivots <= the row: a prefix of the lanes
        const int64_t lo0 = lo;
        if (cnt > 0) lo = lo0 + cnt * a65 + (cnt * b65) / (kWave + 1) + 1;
        if (cnt < kWave) hi = lo0 + (cnt + 1) * a65 + ((cnt + 1) * b65) / (kWave + 1);
    }
    {
        const int64_t pos = lo + lane;
        int c = 1;
        if (pos < hi) {
            const uint32_t* o = old_sorted + pos * W;
            const uint64_t po = ((uint64_t)o[0] << 32) | (W > 1 ? o[1] : 0u);
            c = po < pj ? -1 : po > pj ? 1 : 0;
            if (c == 0 && W > 2) c = compare_tail(o, mine, 2, W);
        }
        lo += popc64(ballot(pos < hi && c <= 0));
    }
    for (int w = lane; w < W; w += kWave) sorted[rank * W + w] = mine[w];
    if (lane == 0) {
        lperm[rank] = (int32_t)j;
        ub[rank] = lo;
    }
}

__device__ __forceinline__ int row_lcp(const uint32_t* a, const uint32_t* b, const RowGeo& g) {
    for (int w = 0; w < g.W; ++w) {
        const uint32_t x = a[w] ^ b[w];
        if (x) return lcp_from_diff(w, x, g);
    }
    return g.L;
}

// The merge of the new rows into a sorted copy, in one launch by block
// ranges.  Blocks [0, nb_old) move the old rows: old row i moves right by the
// number of new rows placed before it (those with ub <= i; ub is
// non-decreasing along the sorted new rows), one thread per row finds that
// shift and the block copies its rows word by word; the row's id goes along,
// and its adjacent LCP too unless a new row now precedes it.  The next nb_new
// blocks place sorted new row j at ub[j] + j, one thread per (row, word).
// The rest compute the adjacent LCP at and
// right after each new row from the source rows themselves (the merged
// neighbours of new row j at P = ub[j] + j are new row j - 1 when it has the
// same upper bound, else old row ub[j] - 1, and new row j + 1 when it has the
// same upper bound, else old row ub[j]), so no block reads another's output.
constexpr int kMergeThreads = 256;
__global__ __launch_bounds__(kMergeThreads) void k_merge_fused(
    const uint32_t* __restrict__ sorted, const int32_t* __restrict__ perm, const uint8_t* __restrict__ A, int64_t N,
    const uint32_t* __restrict__ newrows, const int32_t* __restrict__ newperm, const int64_t* __restrict__ ub,
    int64_t n, RowGeo g, uint32_t* __restrict__ out_sorted, int32_t* __restrict__ out_perm,
    uint8_t* __restrict__ out_A, unsigned nb_old, unsigned nb_new) {
    __shared__ int64_t shift[kMergeThreads];
    const int W = g.W;
    const unsigned b = blockIdx.x;
    if (b < nb_old) {
        const int64_t i0 = (int64_t)b * kMergeThreads;
        const int64_t i = i0 + threadIdx.x;
        int64_t lo = 0;
        if (i < N) {
            int64_t hi = n;
            while (lo < hi) {
                const int64_t mid = lo + (hi - lo) / 2;
                if (ub[mid] <= i)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            out_perm[i + lo] = perm[i];
            if (!(lo > 0 && ub[lo - 1] == i)) out_A[i + lo] = A[i];  // else a new row precedes it
        }
        shift[threadIdx.x] = lo;
        __syncthreads();
        const int64_t rows = N - i0 < kMergeThreads ? N - i0 : kMergeThreads;
        for (int64_t t = threadIdx.x; t < rows * W; t += kMergeThreads) {
            const int64_t r = t / W;
            const int64_t w = t - r * W;
            out_sorted[(i0 + r + shift[r]) * W + w] = sorted[i0 * W + t];
        }
        return;
    }
    if (b < nb_old + nb_new) {
        const int64_t t = (int64_t)(b - nb_old) * kMergeThreads + threadIdx.x;
        if (t >= n * W) return;
        const int64_t j = t / W;
        const int64_t w = t - j * W;
        const int64_t dst = ub[j] + j;
        out_sorted[dst * W + w] = newrows[t];
        if (w == 0) out_perm[dst] = (int32_t)(N + newperm[j]);
        return;
    }
    const int64_t j = (int64_t)(b - nb_old - nb_new) * kMergeThreads + threadIdx.x;
    if (j >= n) return;
    const int64_t u = ub[j];
    const int64_t P = u + j;
    const uint32_t* row = newrows + j * W;
    const uint32_t* pred = j > 0 && ub[j - 1] == u ? newrows + (j - 1) * W : u > 0 ? sorted + (u - 1) * W : nullptr;
    out_A[P] = pred ? (uint8_t)row_lcp(pred, row, g) : 0;
    const uint32_t* succ = j + 1 < n && ub[j + 1] == u ? newrows + (j + 1) * W : u < N ? sorted + u * W : nullptr;
    if (succ) out_A[P + 1] = (uint8_t)row_lcp(row, succ, g);
}

// ------------------------------------------------------------ launchers

hipError_t launch_upper_bounds(const uint32_t* sorted, int64_t N, const uint32_t* newrows, int64_t n, RowGeo g,
                               int64_t* ub, hipStream_t s) {
    hipLaunchKernelGGL(k_upper_bounds, dim3(blocks_for(n, 256)), dim3(256), 0, s, sorted, N, newrows, n, g.W, ub);
    return hipGetLastError();
}

hipError_t launch_merge_sorted(const uint32_t* sorted, const int32_t* perm, const uint8_t* A, int64_t N,
                               const uint32_t* newrows, const int32_t* newperm, const int64_t* ub, int64_t n, RowGeo g,
                               uint32_t* out_sorted, int32_t* out_perm, uint8_t* out_A, hipStream_t s) {
    const int W = g.W;
    const unsigned nb_old = blocks_for(N, kMergeThreads), nb_new = blocks_for(n * W, kMergeThreads);
    const unsigned nb_seam = blocks_for(n, kMergeThreads);
    hipLaunchKernelGGL(k_merge_fused, dim3(nb_old + nb_new + nb_seam), dim3(kMergeThreads), 0, s, sorted, perm, A, N,
                       newrows, newperm, ub, n, g, out_sorted, out_perm, out_A, nb_old, nb_new);
    return hipGetLastError();
}

hipError_t launch_first_token_dir(const uint32_t* sorted, int64_t N, RowGeo g, int V, uint32_t* dir, hipStream_t s) {
    hipLaunchKernelGGL(k_first_token_dir, dim3(blocks_for((int64_t)V + 2, 256)), dim3(256), 0, s, sorted, N, g.W, g.tb,
                       V, dir);
    return hipGetLastError();
}

// The order-dependent summaries of a merged copy and the new rows' plane
// entries in one launch: blocks [0, nb) take the tie summaries (a wave per 64
// positions), the next nd blocks the first-token directory, the rest the plane.
__global__ void k_append_tail(const int32_t* __restrict__ perm, const uint32_t* __restrict__ sorted, int64_t M,
                              RowGeo g, int V, const uint32_t* __restrict__ rows, int64_t from,
                              uint32_t* __restrict__ bmin, uint32_t* __restrict__ dir, uint64_t* __restrict__ plane,
                              int levels, uint4* __restrict__ stab, unsigned ns, unsigned nb, unsigned nd) {
    if (blockIdx.x < ns) {
        search_table_entry((int64_t)blockIdx.x * blockDim.x + threadIdx.x, sorted, M, g.W, levels, stab);
        return;
    }
    const unsigned b = blockIdx.x - ns;
    if (b < nb) {
        const int64_t blk = (int64_t)b * (blockDim.x / kWave) + (threadIdx.x / kWave);
        if (blk >= (M + kWave - 1) / kWave) return;  // whole waves leave together
        const int64_t j = blk * kWave + lane_id();
        const uint32_t v = wave_min_u32(j < M ? (uint32_t)perm[j] : 0xFFFFFFFFu);
        if (lane_id() == 0) bmin[blk] = v;
        return;
    }
    if (b < nb + nd) {
        const int64_t t = (int64_t)(b - nb) * blockDim.x + threadIdx.x;
        if (t > V + 1) return;
        int64_t lo = 0, hi = M;
        if (t >= V) lo = M;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if ((int64_t)(sorted[mid * g.W] >> (32 - 8 * g.tb)) < t)
                lo = mid + 1;
            else
                hi = mid;
        }
        dir[t] = (uint32_t)lo;
        return;
    }
    const int64_t i = from + (int64_t)(b - nb - nd) * blockDim.x + threadIdx.x;
    if (i >= plane_entries(M)) return;
    plane[i] = i < M ? ((uint64_t)rows[i * g.W] << 32) | (g.W > 1 ? rows[i * g.W + 1] : 0u) : 0ull;
}

hipError_t launch_append_tail(const int32_t* perm, const uint32_t* sorted, int64_t M, RowGeo g, int V,
                              const uint32_t* rows, int64_t from, uint32_t* bmin, uint32_t* dir, uint64_t* plane,
                              int levels, uint4* stab, hipStream_t s) {
    const int64_t nst = levels > 0 ? search_table_entries(levels) : 0;
    const unsigned ns = nst > 0 ? blocks_for(nst, 256) : 0u;
    const unsigned nb = blocks_for(block_min_entries(M), 256 / kWave);
    const unsigned nd = blocks_for((int64_t)V + 2, 256);
    const int64_t np = plane_entries(M) - from;
    const unsigned npb = np > 0 ? blocks_for(np, 256) : 0u;
    hipLaunchKernelGGL(k_append_tail, dim3(ns + nb + nd + npb), dim3(256), 0, s, perm, sorted, M, g, V, rows, from, bmin,
                       dir, plane, levels, stab, ns, nb, nd);
    return hipGetLastError();
}

hipError_t launch_rank_ub(const uint32_t* keys, int64_t n, const uint32_t* old_sorted, int64_t N, int W,
                          uint32_t* sorted, int32_t* lperm, int64_t* ub, hipStream_t s) {
    hipLaunchKernelGGL(k_rank_ub, dim3(blocks_for(n, kRankUbWaves)), dim3(kRankUbWaves * kWave), 0, s, keys, n,
                       old_sorted, N, W, sorted, lperm, ub);
    return hipGetLastError();
}

hipError_t launch_pack_keys(const void* tokens, int64_t n, RowGeo g, uint32_t V, uint32_t* keys, uint32_t* bad,
                            uint32_t mark, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_keys, dim3(blocks_for(n * g.W, 256)), dim3(256), 0, s, tokens, n, g, V, keys, bad, mark);
    return hipGetLastError();
}

hipError_t launch_prefix_plane(const uint32_t* rows, int64_t from, int64_t to, int W, uint64_t* plane, hipStream_t s) {
    const int64_t n = plane_entries(to) - from;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_prefix_plane, dim3(blocks_for(n, 256)), dim3(256), 0, s, rows, from, to, W, plane);
    return hipGetLastError();
}

hipError_t launch_block_min(const int32_t* perm, int64_t N, uint32_t* bmin, hipStream_t s) {
    const int64_t nb = block_min_entries(N);
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_block_min, dim3(blocks_for(nb, 4)), dim3(256), 0, s, perm, N, bmin);
    return hipGetLastError();
}

hipError_t launch_search_tables(const uint32_t* sorted, int64_t N, int W, int levels, uint4* stab,
                                hipStream_t s) {
    const int64_t n = search_table_entries(levels);
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_search_tables, dim3(blocks_for(n, 256)), dim3(256), 0, s, sorted, N, W, levels, stab);
    return hipGetLastError();
}


hipError_t launch_pack(const void* tokens, int64_t N, RowGeo g, uint32_t V, int dbits, int Wd, uint32_t* keys,
                       uint32_t* dense, uint32_t* bad, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_keys, dim3(blocks_for(N * g.W, 256)), dim3(256), 0, s, tokens, N, g, V, keys, bad, 1u);
    hipLaunchKernelGGL(k_pack_dense, dim3(blocks_for(N * Wd, 256)), dim3(256), 0, s, tokens, N, g, dbits, Wd, dense);
    return hipGetLastError();
}

hipError_t launch_varying_bits(const uint32_t* dense, int64_t N, int Wd, uint32_t* vary, hipStream_t s) {
    // Wd <= 128; grid = Wd * gx blocks keeps the grid stride a multiple of Wd
    int64_t gx = (N + 255) / 256;
    if (gx > 2048 / Wd + 1) gx = 2048 / Wd + 1;
    hipLaunchKernelGGL(k_varying_bits, dim3((unsigned)(gx * Wd)), dim3(256), 0, s, dense, N, Wd, vary);
    return hipGetLastError();
}

int radix_tiles(int64_t N) { return (int)((N + kTile - 1) / kTile); }

size_t radix_counts_words(int64_t N) {
    const int64_t n = (int64_t)radix_tiles(N) * 256;
    return (size_t)(n + (n + kScanSpan - 1) / kScanSpan);
}

hipError_t launch_iota(int32_t* p, int64_t N, hipStream_t s) {
    hipLaunchKernelGGL(k_iota, dim3(blocks_for(N, 256)), dim3(256), 0, s, p, N);
    return hipGetLastError();
}

hipError_t launch_gather_word(const uint32_t* dense, const int32_t* perm, int64_t N, int Wd, int d, uint32_t* keys,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_gather_word, dim3(blocks_for(N, 256)), dim3(256), 0, s, dense, perm, N, Wd, d, keys);
    return hipGetLastError();
}

hipError_t launch_radix_pass(const uint32_t* keys_in, const int32_t* vals_in, int64_t N, int shift, uint32_t* counts,
                             uint32_t* keys_out, int32_t* vals_out, bool write_keys, hipStream_t s) {
    const int nt = radix_tiles(N);
    hipLaunchKernelGGL(k_radix_hist, dim3(nt), dim3(kRadixThreads), 0, s, keys_in, N, shift, counts, nt);
    const int64_t n = (int64_t)nt * 256;
    const int nb = (int)((n + kScanSpan - 1) / kScanSpan);
    uint32_t* sums = counts + n;  // the counts buffer has room for the block sums
    hipLaunchKernelGGL(k_span_sums, dim3(nb), dim3(256), 0, s, counts, n, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, sums, nb);
    hipLaunchKernelGGL(k_span_scan, dim3(nb), dim3(256), 0, s, counts, n, sums);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nt), dim3(kRadixThreads), 0, s, keys_in, vals_in, N, shift, counts, nt,
                       keys_out, vals_out, write_keys ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_gather_rows(const uint32_t* keys, const int32_t* perm, int64_t N, int W, uint32_t* sorted,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_gather_rows, dim3(blocks_for(N * W, 256)), dim3(256), 0, s, keys, perm, N, W, sorted);
    return hipGetLastError();
}

hipError_t launch_adjacent_lcp(const uint32_t* sorted, int64_t N, RowGeo g, uint8_t* A, hipStream_t s) {
    hipLaunchKernelGGL(k_adjacent_lcp, dim3(blocks_for(N, 256)), dim3(256), 0, s, sorted, N, g, A);
    return hipGetLastError();
}

}  // namespace lcpx
