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

// One thread per (row, key word): key-form row in id order + token range check.
__global__ void k_pack_keys(const void* __restrict__ tokens, int64_t N, RowGeo g, uint32_t V,
                            uint32_t* __restrict__ keys, uint32_t* __restrict__ bad) {
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
    if (out_of_range) atomicOr(bad, 1u);
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

// OR over rows of (word ^ word of row 0): the bits that vary in each dense word.
__global__ void k_varying_bits(const uint32_t* __restrict__ dense, int64_t N, int Wd, uint32_t* __restrict__ vary) {
    const int d = blockIdx.y;
    uint32_t ref = dense[d];
    uint32_t acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        acc |= dense[i * Wd + d] ^ ref;
    // wave OR reduction, then one atomic per wave (OR is order independent)
    for (int off = 32; off > 0; off >>= 1) acc |= __shfl_xor(acc, off);
    if (lane_id() == 0 && acc) atomicOr(&vary[d], acc);
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

// Exclusive scan of n values by one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan_exclusive(uint32_t* __restrict__ a, int64_t n) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (n + 1023) / 1024;
    const int64_t lo = t * per;
    const int64_t hi = lo + per < n ? lo + per : n;
    uint32_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += a[i];
    part[t] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the 1024 partial sums
    for (int d = 1; d < 1024; d <<= 1) {
        uint32_t v = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = t > 0 ? part[t - 1] : 0u;
    for (int64_t i = lo; i < hi; ++i) {
        uint32_t v = a[i];
        a[i] = run;
        run += v;
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

// ------------------------------------------------------------ launchers

static inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

hipError_t launch_pack(const void* tokens, int64_t N, RowGeo g, uint32_t V, int dbits, int Wd, uint32_t* keys,
                       uint32_t* dense, uint32_t* bad, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_keys, dim3(blocks_for(N * g.W, 256)), dim3(256), 0, s, tokens, N, g, V, keys, bad);
    hipLaunchKernelGGL(k_pack_dense, dim3(blocks_for(N * Wd, 256)), dim3(256), 0, s, tokens, N, g, dbits, Wd, dense);
    return hipGetLastError();
}

hipError_t launch_varying_bits(const uint32_t* dense, int64_t N, int Wd, uint32_t* vary, hipStream_t s) {
    unsigned gx = blocks_for(N, 256);
    if (gx > 1024) gx = 1024;
    hipLaunchKernelGGL(k_varying_bits, dim3(gx, (unsigned)Wd), dim3(256), 0, s, dense, N, Wd, vary);
    return hipGetLastError();
}

int radix_tiles(int64_t N) { return (int)((N + kTile - 1) / kTile); }

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
    hipLaunchKernelGGL(k_scan_exclusive, dim3(1), dim3(1024), 0, s, counts, (int64_t)nt * 256);
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
