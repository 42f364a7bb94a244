// Device helpers shared by the index-build, index-query and scan kernels.
//
// Wave64 primitives for CDNA4 (gfx950), the "key form" of a row, and a
// lane-distributed sorted list of 64-bit keys used for every exact top-k
// selection in the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lcpx {

constexpr int kWave = 64;
constexpr uint64_t kKeyMax = ~0ull;

// ---------------------------------------------------------------- wave ops

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int popc64(uint64_t m) { return __popcll(m); }

// index of the lowest set bit of a non-zero mask
__device__ __forceinline__ int low_lane(uint64_t m) { return __ffsll((unsigned long long)m) - 1; }

// number of set bits of m in lanes below the calling lane
__device__ __forceinline__ int count_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ int readlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
    uint32_t lo = readlane((uint32_t)v, l);
    uint32_t hi = readlane((uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ int64_t readlane_i64(int64_t v, int l) {
    return (int64_t)readlane64((uint64_t)v, l);
}
__device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
// a value every lane holds alike, as a scalar
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    return ((uint64_t)uniform((uint32_t)(v >> 32)) << 32) | uniform((uint32_t)v);
}

// value of lane (lane - 1); lane 0 receives its own value
__device__ __forceinline__ uint32_t from_lower_lane(uint32_t v) {
    int src = lane_id() - 1;
    src = src < 0 ? 0 : src;
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}
__device__ __forceinline__ uint64_t from_lower_lane64(uint64_t v) {
    return ((uint64_t)from_lower_lane((uint32_t)(v >> 32)) << 32) | from_lower_lane((uint32_t)v);
}

// DPP lane-permutation controls used below (all stay within the wave)
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr3 = 0x113, kDppRowShr4 = 0x114,
              kDppRowShr8 = 0x118;
constexpr int kDppQuadSwap1 = 0xB1, kDppQuadSwap2 = 0x4E;  // quad_perm 1,0,3,2 and 2,3,0,1
constexpr int kDppRowHalfMirror = 0x141, kDppRowMirror = 0x140;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

// v combined with the value of another lane chosen by a DPP control; lanes
// the control or the row/bank masks leave out take `ident`, the operation's
// identity, so the combining min or add folds into one DPP instruction
#define LCPX_DPP(ident, v, ctrl, rmask, bmask) __builtin_amdgcn_update_dpp((ident), (v), (ctrl), (rmask), (bmask), false)

// inclusive prefix minimum over the wave's lanes (call with all lanes
// active): shifts by 1, 2 and 3 within each row of 16 lanes (from the
// original values), then by 4 and 8 for the upper banks, then lane 15 of
// each row into the next row and lane 31 into the upper half
__device__ __forceinline__ int wave_prefix_min(int v) {
    constexpr int I = 0x7FFFFFFF;
    const int x = v;
    v = min(v, LCPX_DPP(I, x, kDppRowShr1, 0xF, 0xF));
    v = min(v, LCPX_DPP(I, x, kDppRowShr2, 0xF, 0xF));
    v = min(v, LCPX_DPP(I, x, kDppRowShr3, 0xF, 0xF));
    v = min(v, LCPX_DPP(I, v, kDppRowShr4, 0xF, 0xE));
    v = min(v, LCPX_DPP(I, v, kDppRowShr8, 0xF, 0xC));
    v = min(v, LCPX_DPP(I, v, kDppRowBcast15, 0xA, 0xF));
    v = min(v, LCPX_DPP(I, v, kDppRowBcast31, 0xC, 0xF));
    return v;
}

// inclusive prefix sum over the wave's lanes (call with all lanes active):
// the same shift pattern as the prefix minimum, with 0 for lanes left out
__device__ __forceinline__ uint32_t wave_prefix_sum(uint32_t v) {
    const int x = (int)v;
    int s = x;
    s += LCPX_DPP(0, x, kDppRowShr1, 0xF, 0xF);
    s += LCPX_DPP(0, x, kDppRowShr2, 0xF, 0xF);
    s += LCPX_DPP(0, x, kDppRowShr3, 0xF, 0xF);
    s += LCPX_DPP(0, s, kDppRowShr4, 0xF, 0xE);
    s += LCPX_DPP(0, s, kDppRowShr8, 0xF, 0xC);
    s += LCPX_DPP(0, s, kDppRowBcast15, 0xA, 0xF);
    s += LCPX_DPP(0, s, kDppRowBcast31, 0xC, 0xF);
    return (uint32_t)s;
}

// minimum over the wave's lanes, as a scalar (call with all lanes active).
// Swapping neighbours, swapping pairs, mirroring each half row and mirroring
// the row leave every lane with its row's minimum; lane 15 of each row then
// goes into the next row and lane 31 into the upper half, so lane 63 holds
// the minimum of all 64.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
    constexpr int I = -1;  // 0xFFFFFFFF
    v = min(v, (uint32_t)LCPX_DPP(I, (int)v, kDppQuadSwap1, 0xF, 0xF));
    v = min(v, (uint32_t)LCPX_DPP(I, (int)v, kDppQuadSwap2, 0xF, 0xF));
    v = min(v, (uint32_t)LCPX_DPP(I, (int)v, kDppRowHalfMirror, 0xF, 0xF));
    v = min(v, (uint32_t)LCPX_DPP(I, (int)v, kDppRowMirror, 0xF, 0xF));
    v = min(v, (uint32_t)LCPX_DPP(I, (int)v, kDppRowBcast15, 0xA, 0xF));
    v = min(v, (uint32_t)LCPX_DPP(I, (int)v, kDppRowBcast31, 0xC, 0xF));
    return readlane(v, kWave - 1);
}
#undef LCPX_DPP

// ---------------------------------------------------------------- rows
//
// Key form: a row of L tokens of `tb` bytes is stored as W = ceil(L*tb/4)
// 32-bit words, tokens packed big-end first (token j of word w sits in bits
// [32 - 8*tb*(j+1), 32 - 8*tb*j)), the tail of the last word zero.  Then
//   - lexicographic order of rows == unsigned order of the word sequences,
//   - the first differing word w and x = a[w] ^ b[w] give
//     LCP = w * tokens_per_word + clz(x) / token_bits.

struct RowGeo {
    int L;          // tokens per row
    int W;          // words per row
    int tb;         // bytes per token (1 or 2)
    int tpw_log2;   // log2(tokens per word): 2 for 1-byte tokens, 1 for 2-byte
    int bits_log2;  // log2(bits per token): 3 or 4
};

__host__ __device__ inline RowGeo make_geo(int L, int tb) {
    RowGeo g;
    g.L = L;
    g.tb = tb;
    g.W = (L * tb + 3) / 4;
    g.tpw_log2 = tb == 1 ? 2 : 1;
    g.bits_log2 = tb == 1 ? 3 : 4;
    return g;
}

__device__ __forceinline__ uint32_t raw_token(const void* base, int64_t idx, int tb) {
    return tb == 1 ? (uint32_t)((const uint8_t*)base)[idx] : (uint32_t)((const uint16_t*)base)[idx];
}

// Key word w of the row starting at token index `row0` of a raw token array.
__device__ __forceinline__ uint32_t key_word(const void* raw, int64_t row0, const RowGeo& g, int w) {
    const int tpw = 1 << g.tpw_log2;
    const int bits = 8 * g.tb;
    uint32_t x = 0;
    for (int t = 0; t < tpw; ++t) {
        int j = w * tpw + t;
        uint32_t v = j < g.L ? raw_token(raw, row0 + j, g.tb) : 0u;
        x |= v << (32 - bits * (t + 1));
    }
    return x;
}

__device__ __forceinline__ int lcp_from_diff(int word, uint32_t x, const RowGeo& g) {
    return (word << g.tpw_log2) + (__clz((int)x) >> g.bits_log2);
}

// Per-lane LCP and order of a stored row against a query held in LDS.
// Lanes with act == false return lcp = -1, less = false; their `row` must
// still point at a stored row (any), since every lane loads each word group.
// Within a group the first differing word is picked with selects, not
// per-lane branches; the loop leaves as soon as every active lane has found
// its first differing word.  W is a multiple of VEC.
template <int VEC>
__device__ __forceinline__ void compare_row(const uint32_t* __restrict__ row, const uint32_t* q, const RowGeo& g,
                                            bool act, int& lcp, bool& less) {
    int fw = -1;
    uint32_t fx = 0;
    bool lt = false;
    bool open = act;
    for (int w = 0; w < g.W; w += VEC) {
        uint32_t r[VEC];
        if constexpr (VEC == 4) {
            const uint4 v = *reinterpret_cast<const uint4*>(row + w);
            r[0] = v.x; r[1] = v.y; r[2] = v.z; r[3] = v.w;
        } else if constexpr (VEC == 2) {
            const uint2 v = *reinterpret_cast<const uint2*>(row + w);
            r[0] = v.x; r[1] = v.y;
        } else {
            r[0] = row[w];
        }
        int gw = -1;  // first differing word of this group (scanned from the last)
        uint32_t gx = 0;
        bool glt = false;
#pragma unroll
        for (int j = VEC - 1; j >= 0; --j) {
            const uint32_t qq = q[w + j];
            const uint32_t x = r[j] ^ qq;
            const bool d = x != 0u;
            gw = d ? w + j : gw;
            gx = d ? x : gx;
            glt = d ? r[j] < qq : glt;
        }
        const bool take = open && gw >= 0;
        fw = take ? gw : fw;
        fx = take ? gx : fx;
        lt = take ? glt : lt;
        open = open && gw < 0;
        if (ballot(open) == 0) break;
    }
    lcp = act ? (fw < 0 ? g.L : lcp_from_diff(fw, fx, g)) : -1;
    less = act && fw >= 0 && lt;
}

// Same, starting after a known-equal first word (used by the scan's slow path).
__device__ __forceinline__ int lcp_tail(const uint32_t* __restrict__ row, const uint32_t* q, const RowGeo& g,
                                        int from_word) {
    for (int w = from_word; w < g.W; ++w) {
        uint32_t x = row[w] ^ q[w];
        if (x) return lcp_from_diff(w, x, g);
    }
    return g.L;
}

// ---------------------------------------------------------------- keys
//
// Rank key of a (row id, LCP) pair: smaller key = better rank.
__device__ __forceinline__ uint64_t rank_key(int lcp, uint32_t id) {
    return ((uint64_t)(uint32_t)(255 - lcp) << 32) | id;
}
__device__ __forceinline__ int key_lcp(uint64_t k) { return 255 - (int)(k >> 32); }
__device__ __forceinline__ int key_id(uint64_t k) { return (int)(uint32_t)k; }

// ---------------------------------------------------------------- wave sorting

__device__ __forceinline__ uint64_t xor_lane64(uint64_t v, int mask) {
    const int src = lane_id() ^ mask;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t reverse_lanes64(uint64_t v) { return xor_lane64(v, kWave - 1); }

// Ascending bitonic sort of one key per lane.
__device__ __forceinline__ uint64_t wave_sort64(uint64_t x) {
    const int lane = lane_id();
#pragma unroll
    for (int size = 2; size <= kWave; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const uint64_t y = xor_lane64(x, stride);
            const bool keep_min = ((lane & stride) == 0) == ((lane & size) == 0);
            x = keep_min ? (x < y ? x : y) : (x > y ? x : y);
        }
    }
    return x;
}

// Sort a bitonic sequence held one key per lane into ascending order.
__device__ __forceinline__ uint64_t wave_bitonic_clean64(uint64_t x) {
    const int lane = lane_id();
#pragma unroll
    for (int stride = kWave / 2; stride > 0; stride >>= 1) {
        const uint64_t y = xor_lane64(x, stride);
        x = (lane & stride) == 0 ? (x < y ? x : y) : (x > y ? x : y);
    }
    return x;
}

// ---------------------------------------------------------------- sorted list
//
// Ascending list of up to 64*NR keys spread over the wave: entry e lives in
// register e / 64 of lane e % 64.  Unused entries hold kKeyMax.
template <int NR>
struct WaveList {
    uint64_t v[NR];

    __device__ __forceinline__ void init() {
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = kKeyMax;
    }

    // entry e (wave-uniform e)
    __device__ __forceinline__ uint64_t get(int e) const {
        uint64_t out = kKeyMax;
        const int rr = e >> 6;
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if (r == rr) out = readlane64(v[r], e & 63);
        return out;
    }

    // insert one wave-uniform key at its rank; the last entry falls off
    __device__ __forceinline__ void insert(uint64_t key) {
        const int lane = lane_id();
        int pos = 0;
#pragma unroll
        for (int r = 0; r < NR; ++r) pos += popc64(ballot(v[r] < key));
#pragma unroll
        for (int r = NR - 1; r >= 0; --r) {
            uint64_t prev = from_lower_lane64(v[r]);
            if (r > 0) {
                uint64_t carry = readlane64(v[r - 1], 63);
                if (lane == 0) prev = carry;
            }
            const int e = r * 64 + lane;
            v[r] = e > pos ? prev : (e == pos ? key : v[r]);
        }
    }

    // Merge one ascending key per lane into the list (64*NR smallest kept):
    // register by register, the bitonic split of (list register, reversed
    // carry) keeps the 64 smaller keys and carries the 64 larger ones on.
    __device__ __forceinline__ void merge_sorted(uint64_t sorted) {
        uint64_t carry = sorted;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const uint64_t rc = reverse_lanes64(carry);
            const uint64_t lo = v[r] < rc ? v[r] : rc;
            const uint64_t hi = v[r] < rc ? rc : v[r];
            v[r] = wave_bitonic_clean64(lo);
            if (r + 1 < NR) carry = wave_bitonic_clean64(hi);
        }
    }

    // Offer every lane's key where `pass` holds; afterwards entries [0, m)
    // are the m smallest keys among the previous entries and the offers.
    // Few offers are inserted one by one, many are sorted and merged at once.
    __device__ __forceinline__ void offer(uint64_t key, bool pass, int m) {
        const int lane = lane_id();
        uint64_t thr = get(m - 1);
        pass = pass && key < thr;
        uint64_t bal = ballot(pass);
        if (popc64(bal) > 6) {
            merge_sorted(wave_sort64(pass ? key : kKeyMax));
            return;
        }
        while (bal) {
            const int src = low_lane(bal);
            insert(readlane64(key, src));
            thr = get(m - 1);
            pass = pass && lane != src && key < thr;
            bal = ballot(pass);
        }
    }
};

}  // namespace lcpx
