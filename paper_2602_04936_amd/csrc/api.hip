// C-ABI of the library (declared in include/lcp.h): argument checks, device
// buffers, per-stream scratch and the orchestration of the build and query
// kernels.  Every step of the computation runs in the HIP kernels; this file
// only moves sizes, pointers and the host-side k[] array.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/lcp.h"
#include "launch.hpp"

using namespace lcpx;

namespace {

thread_local std::string g_err;

lcp_status fail(lcp_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
lcp_status fail(lcp_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                                 \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess)                                                                         \
            return fail(e_ == hipErrorOutOfMemory ? LCP_ENOMEM : LCP_EDEVICE, "%s: %s (%s:%d)", #expr, \
                        hipGetErrorString(e_), __FILE__, __LINE__);                                   \
    } while (0)

// Pinned staging slot for a host k[] array; reused once its copy has run.
struct Slot {
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};

struct StreamCtx {
    hipStream_t stream = nullptr;
    Slot slots[4];
    int next = 0;
    void* d_kbuf = nullptr;  // [off: Q+1 int64][k: Q int32]
    size_t cap_q = 0;
    uint64_t* d_part = nullptr;
    size_t cap_part = 0;
    unsigned long long* d_counter = nullptr;  // persistent launches' work counter
};

struct TimedLaunch {
    int which;
    hipEvent_t a, b;
};

// One copy of the arrays that depend on the sorted order.  An index keeps two:
// queries read the active one, and an append merges into the other and then
// makes it active, so a failed append leaves the index as it was.
struct SortedCopy {
    int64_t cap = 0;             // rows it can hold
    uint32_t* sorted = nullptr;  // [cap][W] key form, lexicographic order
    int32_t* perm = nullptr;     // [cap]
    uint8_t* A = nullptr;        // [cap + kAdjPad]: fixed-size windows near the end stay inside
    uint32_t* bmin = nullptr;    // [block_min_entries(cap)]
    uint4* stab = nullptr;       // [search_table_entries(search_table_levels(cap))], NULL with no levels
    uint32_t* dir = nullptr;     // [V + 2] first-token directory
    void release() {
        if (dir) hipFree(dir);
        if (sorted) hipFree(sorted);
        if (perm) hipFree(perm);
        if (A) hipFree(A);
        if (bmin) hipFree(bmin);
        if (stab) hipFree(stab);
        *this = SortedCopy();
    }
};

// Device temporaries of small appends, kept between calls.
struct AppendScratch {
    int64_t cap = 0;               // new rows they can hold
    uint32_t* sorted = nullptr;    // [cap][W] new rows in sorted order
    int32_t* lperm = nullptr;      // [cap] local ids in sorted order
    int64_t* ub = nullptr;         // [cap] old rows <= each sorted new row
    uint32_t* flag = nullptr;      // device: the last append (by epoch) that saw a token >= V
    uint32_t* flag_host = nullptr;  // pinned copy of it
    uint32_t epoch = 0;            // appends so far that used the flag
    void release() {
        if (sorted) hipFree(sorted);
        if (lperm) hipFree(lperm);
        if (ub) hipFree(ub);
        if (flag) hipFree(flag);
        if (flag_host) hipHostFree(flag_host);
        *this = AppendScratch();
    }
};

}  // namespace

struct lcp_index {
    int device = 0;
    int cus = 0;  // compute units of the device
    int64_t N = 0;
    int32_t L = 0, V = 0;
    RowGeo g{};
    int64_t rows_cap = 0;          // rows d_rows and d_plane can hold
    uint32_t* d_rows = nullptr;    // [rows_cap][W] id order, key form
    uint64_t* d_plane = nullptr;   // [plane_entries(rows_cap)] the scan's prefix plane
    SortedCopy cp[2];
    int cur = 0;                   // the copy queries read
    int stab_levels = 0;
    int search_mode = 0;           // 0: 65-ary search tables, 1: first-token directory
    uint64_t generation = 0;       // changes of what queries read: appends, search-mode switches
    AppendScratch app;
    // The bucket scan's planes of the sorted order, built by the first call
    // that needs one after each change of generation: the first two key words
    // of every sorted row, and columns of single key words.
    mutable uint64_t* d_splane = nullptr;
    mutable int64_t splane_cap = 0;
    mutable uint64_t splane_gen = ~0ull;
    mutable std::vector<uint32_t*> d_col;  // [W], null until used
    mutable uint64_t col_gen = ~0ull;

    mutable std::mutex mu;
    mutable std::unordered_map<hipStream_t, StreamCtx*> ctx;
    mutable bool timing = false;
    mutable std::vector<TimedLaunch> timed;
    mutable std::vector<hipEvent_t> event_pool;
    mutable double acc_ms[3] = {0, 0, 0};
    mutable int64_t acc_n[3] = {0, 0, 0};

    IndexView view() const {
        IndexView v;
        const SortedCopy& c = cp[cur];
        v.sorted = c.sorted;
        v.rows = d_rows;
        v.perm = c.perm;
        v.A = c.A;
        v.stab = c.stab;
        v.stab_levels = stab_levels;
        v.bmin = c.bmin;
        v.plane = d_plane;
        v.dir = search_mode == 1 ? c.dir : nullptr;
        v.dir_V = V;
        v.N = N;
        v.g = g;
        return v;
    }
};

namespace {

void free_ctx(StreamCtx* c) {
    for (auto& s : c->slots) {
        if (s.done) hipEventDestroy(s.done);
        if (s.host) hipHostFree(s.host);
    }
    if (c->d_kbuf) hipFree(c->d_kbuf);
    if (c->d_part) hipFree(c->d_part);
    if (c->d_counter) hipFree(c->d_counter);
    delete c;
}

// caller holds idx->mu
lcp_status get_ctx(const lcp_index* idx, hipStream_t s, StreamCtx** out) {
    auto it = idx->ctx.find(s);
    if (it != idx->ctx.end()) {
        *out = it->second;
        return LCP_OK;
    }
    StreamCtx* c = new StreamCtx();
    c->stream = s;
    for (auto& sl : c->slots) {
        hipError_t e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            free_ctx(c);
            return fail(LCP_EDEVICE, "hipEventCreate: %s", hipGetErrorString(e));
        }
    }
    idx->ctx[s] = c;
    *out = c;
    return LCP_OK;
}

lcp_status ensure_q(StreamCtx* c, size_t Q) {
    if (Q <= c->cap_q) return LCP_OK;
    size_t cap = std::max<size_t>(Q, 2 * c->cap_q);
    HIP_TRY(hipStreamSynchronize(c->stream));  // earlier calls may still read the old buffer
    if (c->d_kbuf) hipFree(c->d_kbuf);
    c->d_kbuf = nullptr;
    c->cap_q = 0;
    HIP_TRY(hipMalloc(&c->d_kbuf, (cap + 1) * sizeof(int64_t) + cap * sizeof(int32_t)));
    c->cap_q = cap;
    return LCP_OK;
}

lcp_status ensure_part(StreamCtx* c, size_t entries) {
    if (entries <= c->cap_part) return LCP_OK;
    size_t cap = std::max(entries, c->cap_part + c->cap_part / 2);
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (c->d_part) hipFree(c->d_part);
    c->d_part = nullptr;
    c->cap_part = 0;
    HIP_TRY(hipMalloc(&c->d_part, cap * sizeof(uint64_t)));
    c->cap_part = cap;
    return LCP_OK;
}

hipEvent_t take_event(const lcp_index* idx) {
    if (!idx->event_pool.empty()) {
        hipEvent_t e = idx->event_pool.back();
        idx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Copy host k[] and its exclusive prefix sum to the stream's device buffers.
lcp_status stage_k(StreamCtx* c, int64_t Q, const int32_t* k) {
    lcp_status st = ensure_q(c, (size_t)Q);
    if (st != LCP_OK) return st;
    // staging and device buffer share the layout [off: Q+1 int64][k: Q int32] of this call
    const size_t bytes = (size_t)(Q + 1) * sizeof(int64_t) + (size_t)Q * sizeof(int32_t);
    Slot& sl = c->slots[c->next];
    c->next = (c->next + 1) % 4;
    if (sl.pending) {
        HIP_TRY(hipEventSynchronize(sl.done));
        sl.pending = false;
    }
    if (sl.cap < bytes) {
        if (sl.host) hipHostFree(sl.host);
        sl.host = nullptr;
        sl.cap = 0;
        HIP_TRY(hipHostMalloc(&sl.host, bytes, hipHostMallocDefault));
        sl.cap = bytes;
    }
    int64_t* off = reinterpret_cast<int64_t*>(sl.host);
    int32_t* kk = reinterpret_cast<int32_t*>(off + Q + 1);
    off[0] = 0;
    for (int64_t i = 0; i < Q; ++i) off[i + 1] = off[i] + k[i];
    std::memcpy(kk, k, (size_t)Q * sizeof(int32_t));
    // one copy: the device buffer has the same [off][k] layout as the staging slot
    HIP_TRY(hipMemcpyAsync(c->d_kbuf, off, bytes, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipEventRecord(sl.done, c->stream));
    sl.pending = true;
    return LCP_OK;
}

const int64_t* kbuf_off(const StreamCtx* c) { return static_cast<const int64_t*>(c->d_kbuf); }
const int32_t* kbuf_k(const StreamCtx* c, int64_t Q) {
    return reinterpret_cast<const int32_t*>(static_cast<const int64_t*>(c->d_kbuf) + Q + 1);
}

lcp_status check_query_args(const lcp_index* idx, const void* queries, int64_t Q, const void* out_ids,
                            const void* out_lcp) {
    if (!idx) return fail(LCP_EINVAL, "index is NULL");
    if (Q < 0 || Q > INT32_MAX) return fail(LCP_EINVAL, "Q = %lld is outside [0, 2^31)", (long long)Q);
    if (Q > 0 && (!queries || !out_ids || !out_lcp)) return fail(LCP_EINVAL, "NULL queries or output pointer");
    return LCP_OK;
}

enum class Path { Index, Scan, Bucket };

// Queries per launch: the index kernel's grid is Q/4 blocks; the scan's grid y
// is Q/(4*tq) <= 65535 query groups.
constexpr int64_t kSliceIndex = 1 << 20;
constexpr int64_t kSliceScan = 65535 * 4;

// The bucket scan's sorted prefix plane for the current generation; the
// first call after a change builds it and waits for it, so that calls on
// other streams find it complete.  Caller holds idx->mu.
lcp_status ensure_sorted_plane(const lcp_index* idx, hipStream_t s) {
    if (idx->splane_gen == idx->generation) return LCP_OK;
    HIP_TRY(hipDeviceSynchronize());  // calls on other streams may still read the old plane
    const int64_t need = plane_entries(idx->N);
    if (need > idx->splane_cap) {
        if (idx->d_splane) hipFree(idx->d_splane);
        idx->d_splane = nullptr;
        idx->splane_cap = 0;
        HIP_TRY(hipMalloc(&idx->d_splane, (size_t)need * sizeof(uint64_t)));
        idx->splane_cap = need;
    }
    HIP_TRY(launch_prefix_plane(idx->cp[idx->cur].sorted, 0, idx->N, idx->g.W, idx->d_splane, s));
    HIP_TRY(hipStreamSynchronize(s));
    idx->splane_gen = idx->generation;
    return LCP_OK;
}

// The bucket scan's column of key word w for the current generation (built
// and waited for on first use, as the pair plane).  Caller holds idx->mu.
lcp_status ensure_sorted_column(const lcp_index* idx, int w, hipStream_t s) {
    if (idx->col_gen != idx->generation) {
        HIP_TRY(hipDeviceSynchronize());  // calls on other streams may still read the old columns
        for (uint32_t*& c : idx->d_col) {
            if (c) hipFree(c);
            c = nullptr;
        }
        idx->d_col.assign(idx->g.W, nullptr);
        idx->col_gen = idx->generation;
    }
    if (idx->d_col[w]) return LCP_OK;
    uint32_t* col = nullptr;
    HIP_TRY(hipMalloc(&col, (size_t)column_entries(idx->N) * sizeof(uint32_t)));
    hipError_t e = launch_sorted_column(idx->cp[idx->cur].sorted, idx->N, idx->g.W, w, col, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        hipFree(col);
        return fail(LCP_EDEVICE, "sorted column: %s", hipGetErrorString(e));
    }
    idx->d_col[w] = col;
    return LCP_OK;
}

lcp_status run_dev(const lcp_index* idx, Path path, const void* queries, int64_t Q, const int32_t* k_dev,
                   const int64_t* off_dev, int32_t k_uniform, int32_t k_max, int32_t* out_ids, int32_t* out_lcp,
                   hipStream_t s, StreamCtx* c, int32_t* stats = nullptr, int32_t depth = 0) {
    HIP_TRY(hipSetDevice(idx->device));
    const IndexView ix = idx->view();
    const size_t row_bytes = (size_t)idx->L * idx->g.tb;
    const int64_t slice = path == Path::Scan ? kSliceScan : kSliceIndex;
    const void* bucket_plane = nullptr;
    if (path == Path::Bucket) {
        const int cw = bucket_column(depth, idx->g);
        lcp_status st = cw < 0 ? ensure_sorted_plane(idx, s) : ensure_sorted_column(idx, cw, s);
        if (st != LCP_OK) return st;
        bucket_plane = cw < 0 ? static_cast<const void*>(idx->d_splane) : static_cast<const void*>(idx->d_col[cw]);
    }
    for (int64_t q0 = 0; q0 < Q; q0 += slice) {
        QueryBatch qb;
        qb.raw = static_cast<const uint8_t*>(queries) + (size_t)q0 * row_bytes;
        qb.Q = std::min(slice, Q - q0);
        qb.k = k_dev ? k_dev + q0 : nullptr;
        qb.off = off_dev ? off_dev + q0 : nullptr;
        qb.k_uniform = k_uniform;
        qb.q_base = q0;
        qb.k_max = k_max;
        qb.out_ids = out_ids;  // offsets are absolute
        qb.out_lcp = out_lcp;
        qb.stats = stats && path == Path::Index ? stats + 4 * q0 : nullptr;
        hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
        if (idx->timing && path != Path::Bucket) {
            int need = path == Path::Index ? 2 : 3;
            for (int i = 0; i < need; ++i) ev[i] = take_event(idx);
        }
        if (path == Path::Bucket) {
            // the bucket bounds travel in `stats` as [Q][2]
            HIP_TRY(launch_bucket_scan(ix, bucket_plane, qb, depth, stats ? stats + 2 * q0 : nullptr, s));
        } else if (path == Path::Index) {
            if (ev[0]) HIP_TRY(hipEventRecord(ev[0], s));
            HIP_TRY(launch_index_query(ix, qb, s));
            if (ev[1]) {
                HIP_TRY(hipEventRecord(ev[1], s));
                idx->timed.push_back({0, ev[0], ev[1]});
            }
        } else {
            const ScanPlan plan = plan_scan(idx->N, idx->g.W, qb.Q, k_max);
            lcp_status st = ensure_part(c, scan_partial_entries(plan, qb.Q, k_max, idx->g));
            if (st != LCP_OK) return st;
            HIP_TRY(launch_scan(ix, qb, plan, c->d_part, s, ev[0], ev[1], ev[2]));
            if (ev[0] && ev[1] && ev[2]) {
                // the merge interval starts where the scan interval ends
                idx->timed.push_back({1, ev[0], ev[1]});
                idx->timed.push_back({2, ev[1], ev[2]});
            }
        }
    }
    return LCP_OK;
}

lcp_status query_host(const lcp_index* idx, Path path, const void* queries, int64_t Q, const int32_t* k,
                      int32_t* out_ids, int32_t* out_lcp, void* stream, int32_t* stats = nullptr,
                      int32_t depth = 0) {
    lcp_status st = check_query_args(idx, queries, Q, out_ids, out_lcp);
    if (st != LCP_OK) return st;
    if (Q == 0) return LCP_OK;
    if (!k) return fail(LCP_EINVAL, "k is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(idx->mu);
    HIP_TRY(hipSetDevice(idx->device));
    StreamCtx* c = nullptr;
    st = get_ctx(idx, s, &c);
    if (st != LCP_OK) return st;
    // branch-free pass (vectorised): range and uniformity of k
    const int32_t k0 = k[0];
    int32_t kmin = k0, kmax = k0, diff = 0;
    for (int64_t i = 0; i < Q; ++i) {
        const int32_t v = k[i];
        kmin = v < kmin ? v : kmin;
        kmax = v > kmax ? v : kmax;
        diff |= v ^ k0;
    }
    if (kmin < 1 || kmax > LCP_K_MAX) {
        for (int64_t i = 0; i < Q; ++i)
            if (k[i] < 1 || k[i] > LCP_K_MAX)
                return fail(LCP_EINVAL, "k[%lld] = %d is outside [1, %d]", (long long)i, k[i], LCP_K_MAX);
    }
    if (diff == 0)  // one k for all: offsets are i * k, nothing to copy
        return run_dev(idx, path, queries, Q, nullptr, nullptr, k[0], kmax, out_ids, out_lcp, s, c, stats, depth);
    st = stage_k(c, Q, k);
    if (st != LCP_OK) return st;
    return run_dev(idx, path, queries, Q, kbuf_k(c, Q), kbuf_off(c), 0, kmax, out_ids, out_lcp, s, c, stats,
                   depth);
}

// Fixed scratch of the allocation-free full scan: one copy per device,
// allocated with the library's device code and held until the process ends.
// Host code never passes `scratch` itself to a kernel (on the host the name
// only stands for the symbol): its device address comes from
// hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kNoAllocScratchBytes = LCP_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint64_t scratch[kNoAllocScratchBytes / sizeof(uint64_t)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint64_t* g_scratch_ptr[kMaxDevices] = {};

// caller has made `dev` current
lcp_status scratch_on_device(int dev, uint64_t** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(LCP_EDEVICE, "device %d is beyond the scratch table", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(LCP_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<uint64_t*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return LCP_OK;
}

lcp_status query_dev(const lcp_index* idx, Path path, const void* queries, int64_t Q, const int32_t* k_dev,
                     const int64_t* off_dev, int32_t k_max, int32_t* out_ids, int32_t* out_lcp, void* stream) {
    lcp_status st = check_query_args(idx, queries, Q, out_ids, out_lcp);
    if (st != LCP_OK) return st;
    if (Q == 0) return LCP_OK;
    if (!k_dev || !off_dev) return fail(LCP_EINVAL, "NULL k_dev or off_dev");
    if (k_max < 1 || k_max > LCP_K_MAX) return fail(LCP_EINVAL, "k_max = %d is outside [1, %d]", k_max, LCP_K_MAX);
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(idx->mu);
    StreamCtx* c = nullptr;
    st = get_ctx(idx, s, &c);
    if (st != LCP_OK) return st;
    return run_dev(idx, path, queries, Q, k_dev, off_dev, 0, k_max, out_ids, out_lcp, s, c);
}

struct BuildTemps {
    uint32_t* dense = nullptr;
    uint32_t* keys[2] = {nullptr, nullptr};
    int32_t* vals[2] = {nullptr, nullptr};
    uint32_t* counts = nullptr;
    uint32_t* flags = nullptr;  // [0] = bad token, [1..Wd] = varying bits
    ~BuildTemps() {
        if (dense) hipFree(dense);
        for (int i = 0; i < 2; ++i) {
            if (keys[i]) hipFree(keys[i]);
            if (vals[i]) hipFree(vals[i]);
        }
        if (counts) hipFree(counts);
        if (flags) hipFree(flags);
    }
};

void destroy_index(lcp_index* idx) {
    if (!idx) return;
    for (auto& kv : idx->ctx) {
        hipStreamSynchronize(kv.first);
        free_ctx(kv.second);
    }
    idx->ctx.clear();
    for (auto& t : idx->timed) {
        hipEventDestroy(t.a);
        hipEventDestroy(t.b);
    }
    for (auto e : idx->event_pool) hipEventDestroy(e);
    if (idx->d_rows) hipFree(idx->d_rows);
    if (idx->d_plane) hipFree(idx->d_plane);
    if (idx->d_splane) hipFree(idx->d_splane);
    for (uint32_t* c : idx->d_col)
        if (c) hipFree(c);
    idx->cp[0].release();
    idx->cp[1].release();
    idx->app.release();
    delete idx;
}

// Key-form rows (id order) of n raw token rows and their stable lexicographic
// order (perm over local ids 0..n-1).  LCP_ERANGE if a token is >= V.
lcp_status sort_rows(const void* tokens, int64_t n, const RowGeo& g, int32_t V, hipStream_t s, uint32_t* keys_out,
                     int32_t* perm_out) {
    int dbits = 1;
    while ((1 << dbits) < V && dbits < 16) ++dbits;
    const int Wd = (g.L * dbits + 31) / 32;
    BuildTemps t;
    HIP_TRY(hipMalloc(&t.dense, (size_t)n * Wd * sizeof(uint32_t)));
    HIP_TRY(hipMalloc(&t.flags, (size_t)(1 + Wd) * sizeof(uint32_t)));
    HIP_TRY(hipMemsetAsync(t.flags, 0, (size_t)(1 + Wd) * sizeof(uint32_t), s));
    HIP_TRY(launch_pack(tokens, n, g, (uint32_t)V, dbits, Wd, keys_out, t.dense, t.flags, s));
    HIP_TRY(launch_varying_bits(t.dense, n, Wd, t.flags + 1, s));
    std::vector<uint32_t> flags(1 + Wd);
    HIP_TRY(hipMemcpyAsync(flags.data(), t.flags, flags.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (flags[0]) return fail(LCP_ERANGE, "a token is >= V = %d", V);

    // stable LSD radix sort of ids by the dense key: last word first, low digit first
    HIP_TRY(hipMalloc(&t.counts, radix_counts_words(n) * sizeof(uint32_t)));
    for (int b = 0; b < 2; ++b) {
        HIP_TRY(hipMalloc(&t.keys[b], (size_t)n * sizeof(uint32_t)));
        HIP_TRY(hipMalloc(&t.vals[b], (size_t)n * sizeof(int32_t)));
    }
    int cur = 0;
    HIP_TRY(launch_iota(t.vals[cur], n, s));
    for (int d = Wd - 1; d >= 0; --d) {
        const uint32_t vary = flags[1 + d];
        if (!vary) continue;
        HIP_TRY(launch_gather_word(t.dense, t.vals[cur], n, Wd, d, t.keys[cur], s));
        int last_digit = -1;
        for (int dg = 0; dg < 4; ++dg)
            if ((vary >> (8 * dg)) & 0xFFu) last_digit = dg;
        for (int dg = 0; dg < 4; ++dg) {
            if (!((vary >> (8 * dg)) & 0xFFu)) continue;
            HIP_TRY(launch_radix_pass(t.keys[cur], t.vals[cur], n, 8 * dg, t.counts, t.keys[cur ^ 1],
                                      t.vals[cur ^ 1], dg != last_digit, s));
            cur ^= 1;
        }
    }
    HIP_TRY(hipMemcpyAsync(perm_out, t.vals[cur], (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));  // the temporaries are freed on return
    return LCP_OK;
}

// Dependent search steps of the 65-ary search over n rows (down to at most 64
// rows, then the last step).
int search_steps(double n) {
    int s = 1;
    while (n > kWave) {
        n /= kWave + 1;
        ++s;
    }
    return s;
}

// Whether the first-token directory beats the search tables as the top of the
// search, by dependent steps: the directory costs one lookup and then the
// steps over the query's bucket (size weighted by rows, as queries drawn like
// the rows see it); the tables cost their levels and the steps below them.
// A tie keeps the tables, whose steps read one coalesced line instead of 64
// rows.
bool directory_pays(const std::vector<uint32_t>& dir, int64_t N, int levels) {
    double sq = 0;
    for (size_t t = 0; t + 1 < dir.size(); ++t) {
        const double b = (double)dir[t + 1] - (double)dir[t];
        sq += b * b;
    }
    const double bucket = sq / (double)N;
    double below = (double)N;
    for (int d = 0; d < levels; ++d) below /= kWave + 1;
    return 1 + search_steps(bucket) < levels + search_steps(below);
}

// Allocate a sorted copy for `cap` rows (nothing is kept on failure).
lcp_status alloc_copy(SortedCopy& c, int64_t cap, int W, int V, hipStream_t s) {
    SortedCopy n;
    n.cap = cap;
    hipError_t e = hipMalloc(&n.sorted, (size_t)cap * W * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&n.perm, (size_t)cap * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&n.A, (size_t)cap + kAdjPad);
    if (e == hipSuccess) e = hipMalloc(&n.bmin, (size_t)block_min_entries(cap) * sizeof(uint32_t));
    const int levels = search_table_levels(cap);
    if (e == hipSuccess && levels > 0) e = hipMalloc(&n.stab, (size_t)search_table_entries(levels) * sizeof(uint4));
    if (e == hipSuccess) e = hipMalloc(&n.dir, ((size_t)V + 2) * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemsetAsync(n.A, 0, (size_t)cap + kAdjPad, s);
    if (e != hipSuccess) {
        n.release();
        return fail(e == hipErrorOutOfMemory ? LCP_ENOMEM : LCP_EDEVICE, "allocating the sorted arrays for %lld rows: %s",
                    (long long)cap, hipGetErrorString(e));
    }
    c = n;
    return LCP_OK;
}

// A, search tables and tie summaries of copy `c` holding N sorted rows
lcp_status derive_copy(const lcp_index* idx, SortedCopy& c, int64_t N, hipStream_t s) {
    HIP_TRY(launch_adjacent_lcp(c.sorted, N, idx->g, c.A, s));
    const int levels = search_table_levels(N);
    if (levels > 0) HIP_TRY(launch_search_tables(c.sorted, N, idx->g.W, levels, c.stab, s));
    HIP_TRY(launch_block_min(c.perm, N, c.bmin, s));
    HIP_TRY(launch_first_token_dir(c.sorted, N, idx->g, idx->V, c.dir, s));
    return LCP_OK;
}

lcp_status build_into(lcp_index* idx, const void* tokens, hipStream_t s) {
    const int64_t N = idx->N;
    const int W = idx->g.W;
    HIP_TRY(hipMalloc(&idx->d_rows, (size_t)N * W * sizeof(uint32_t)));
    HIP_TRY(hipMalloc(&idx->d_plane, (size_t)plane_entries(N) * sizeof(uint64_t)));
    idx->rows_cap = N;
    lcp_status st = alloc_copy(idx->cp[0], N, W, idx->V, s);
    if (st != LCP_OK) return st;
    SortedCopy& c = idx->cp[0];
    st = sort_rows(tokens, N, idx->g, idx->V, s, idx->d_rows, c.perm);
    if (st != LCP_OK) return st;
    HIP_TRY(launch_gather_rows(idx->d_rows, c.perm, N, W, c.sorted, s));
    st = derive_copy(idx, c, N, s);
    if (st != LCP_OK) return st;
    HIP_TRY(launch_prefix_plane(idx->d_rows, 0, N, W, idx->d_plane, s));
    idx->stab_levels = search_table_levels(N);
    std::vector<uint32_t> dir((size_t)idx->V + 2);
    HIP_TRY(hipMemcpyAsync(dir.data(), c.dir, dir.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    idx->search_mode = directory_pays(dir, N, idx->stab_levels) ? 1 : 0;
    return LCP_OK;
}

// Capacity after growth: room for a quarter more rows, so that a stream of
// appends reallocates rarely.
int64_t grown(int64_t need) {
    const int64_t g = need + need / 4 + 1024;
    return g < kMaxRows ? g : kMaxRows;
}

// Appends of at most this many rows sort them by rank in one kernel and keep
// their temporaries between calls; larger ones take the radix sort.
constexpr int64_t kRankSortMax = 8192;

// Make `c` hold `cap` rows, keeping its first N rows' arrays.
lcp_status grow_copy(lcp_index* idx, SortedCopy& c, int64_t cap, int64_t N, hipStream_t s) {
    if (c.cap >= cap) return LCP_OK;
    SortedCopy n;
    lcp_status st = alloc_copy(n, cap, idx->g.W, idx->V, s);
    if (st != LCP_OK) return st;
    hipError_t e = hipSuccess;
    if (c.sorted && N > 0) {
        e = hipMemcpyAsync(n.sorted, c.sorted, (size_t)N * idx->g.W * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(n.perm, c.perm, (size_t)N * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(n.A, c.A, (size_t)N, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(n.bmin, c.bmin, (size_t)block_min_entries(N) * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        const int levels = search_table_levels(N);
        if (e == hipSuccess && levels > 0)
            e = hipMemcpyAsync(n.stab, c.stab, (size_t)search_table_entries(levels) * sizeof(uint4),
                               hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(n.dir, c.dir, ((size_t)idx->V + 2) * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        n.release();
        return fail(LCP_EDEVICE, "copying the sorted arrays: %s", hipGetErrorString(e));
    }
    c.release();
    c = n;
    return LCP_OK;
}

// Room for `rows` rows in the id-order rows and plane, both sorted copies and
// the append temporaries, so that appends up to that size allocate nothing.
lcp_status reserve_into(lcp_index* idx, int64_t rows, hipStream_t s) {
    for (auto& kv : idx->ctx) HIP_TRY(hipStreamSynchronize(kv.first));
    const int64_t N = idx->N;
    const int W = idx->g.W;
    if (idx->rows_cap < rows) {
        uint32_t* nr = nullptr;
        uint64_t* np = nullptr;
        hipError_t e = hipMalloc(&nr, (size_t)rows * W * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMalloc(&np, (size_t)plane_entries(rows) * sizeof(uint64_t));
        if (e == hipSuccess) e = hipMemcpyAsync(nr, idx->d_rows, (size_t)N * W * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(np, idx->d_plane, (size_t)plane_entries(N) * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            if (nr) hipFree(nr);
            if (np) hipFree(np);
            return fail(e == hipErrorOutOfMemory ? LCP_ENOMEM : LCP_EDEVICE, "growing the rows: %s",
                        hipGetErrorString(e));
        }
        hipFree(idx->d_rows);
        hipFree(idx->d_plane);
        idx->d_rows = nr;
        idx->d_plane = np;
        idx->rows_cap = rows;
    }
    lcp_status st = grow_copy(idx, idx->cp[idx->cur], rows, N, s);
    if (st != LCP_OK) return st;
    st = grow_copy(idx, idx->cp[idx->cur ^ 1], rows, 0, s);
    if (st != LCP_OK) return st;
    AppendScratch& a = idx->app;
    if (!a.flag) {
        HIP_TRY(hipMalloc(&a.flag, sizeof(uint32_t)));
        HIP_TRY(hipHostMalloc(&a.flag_host, sizeof(uint32_t), hipHostMallocDefault));
        HIP_TRY(hipMemsetAsync(a.flag, 0, sizeof(uint32_t), s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    if (a.cap < kRankSortMax) {
        HIP_TRY(hipMalloc(&a.sorted, (size_t)kRankSortMax * W * sizeof(uint32_t)));
        HIP_TRY(hipMalloc(&a.lperm, (size_t)kRankSortMax * sizeof(int32_t)));
        HIP_TRY(hipMalloc(&a.ub, (size_t)kRankSortMax * sizeof(int64_t)));
        a.cap = kRankSortMax;
    }
    idx->generation += 1;  // the active arrays may have moved
    return LCP_OK;
}

// Rows with ids N..N+n-1: the result equals a build over the concatenation.
// The new rows are packed into the id-order rows after the old ones (and the
// plane after the old entries), sorted, placed into the inactive sorted copy
// together with the old rows (old first on equality: smaller ids), and the
// adjacent LCP is copied for old rows and recomputed only where a new row was
// inserted; the tie summaries and search tables of the merged order follow.
// Nothing the queries read changes until every step has succeeded.
lcp_status append_into(lcp_index* idx, const void* tokens, int64_t n, hipStream_t s) {
    for (auto& kv : idx->ctx) HIP_TRY(hipStreamSynchronize(kv.first));  // no query may still read the index
    const int64_t N = idx->N;
    const int64_t M = N + n;
    const int W = idx->g.W;
    const RowGeo g = idx->g;

    // id-order rows and plane: in place when they have room, else new buffers
    // that replace the old ones only on success
    uint32_t* rows = idx->d_rows;
    uint64_t* plane = idx->d_plane;
    int64_t rows_cap = idx->rows_cap;
    struct Fresh {
        uint32_t* rows = nullptr;
        uint64_t* plane = nullptr;
        ~Fresh() {
            if (rows) hipFree(rows);
            if (plane) hipFree(plane);
        }
    } fresh;
    if (rows_cap < M) {
        rows_cap = grown(M);
        HIP_TRY(hipMalloc(&fresh.rows, (size_t)rows_cap * W * sizeof(uint32_t)));
        HIP_TRY(hipMalloc(&fresh.plane, (size_t)plane_entries(rows_cap) * sizeof(uint64_t)));
        HIP_TRY(hipMemcpyAsync(fresh.rows, idx->d_rows, (size_t)N * W * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(fresh.plane, idx->d_plane, (size_t)plane_entries(N) * sizeof(uint64_t),
                               hipMemcpyDeviceToDevice, s));
        rows = fresh.rows;
        plane = fresh.plane;
    }
    SortedCopy& src = idx->cp[idx->cur];
    SortedCopy& dst = idx->cp[idx->cur ^ 1];
    if (dst.cap < M) {
        dst.release();
        lcp_status st = alloc_copy(dst, grown(M), W, idx->V, s);
        if (st != LCP_OK) return st;
    }
    uint32_t* newkeys = rows + (size_t)N * W;  // the new rows, key form, id order

    uint32_t* nsorted;
    int32_t* nperm;
    int64_t* ub;
    struct Big {
        uint32_t* sorted = nullptr;
        int32_t* perm = nullptr;
        int64_t* ub = nullptr;
        ~Big() {
            if (sorted) hipFree(sorted);
            if (perm) hipFree(perm);
            if (ub) hipFree(ub);
        }
    } big;
    AppendScratch& a = idx->app;
    if (!a.flag) {
        HIP_TRY(hipMalloc(&a.flag, sizeof(uint32_t)));
        HIP_TRY(hipHostMalloc(&a.flag_host, sizeof(uint32_t), hipHostMallocDefault));
        HIP_TRY(hipMemsetAsync(a.flag, 0, sizeof(uint32_t), s));
    }
    const uint32_t epoch = ++a.epoch;  // a bad token raises the flag to this epoch: no clearing between appends
    if (n <= kRankSortMax) {
        if (a.cap < n) {
            if (a.sorted) hipFree(a.sorted);
            if (a.lperm) hipFree(a.lperm);
            if (a.ub) hipFree(a.ub);
            a.sorted = nullptr;
            a.lperm = nullptr;
            a.ub = nullptr;
            a.cap = 0;
            HIP_TRY(hipMalloc(&a.sorted, (size_t)kRankSortMax * W * sizeof(uint32_t)));
            HIP_TRY(hipMalloc(&a.lperm, (size_t)kRankSortMax * sizeof(int32_t)));
            HIP_TRY(hipMalloc(&a.ub, (size_t)kRankSortMax * sizeof(int64_t)));
            a.cap = kRankSortMax;
        }
        HIP_TRY(launch_pack_keys(tokens, n, g, (uint32_t)idx->V, newkeys, a.flag, epoch, s));
        HIP_TRY(launch_rank_ub(newkeys, n, src.sorted, N, W, a.sorted, a.lperm, a.ub, s));
        nsorted = a.sorted;
        nperm = a.lperm;
        ub = a.ub;
    } else {
        HIP_TRY(hipMalloc(&big.sorted, (size_t)n * W * sizeof(uint32_t)));
        HIP_TRY(hipMalloc(&big.perm, (size_t)n * sizeof(int32_t)));
        HIP_TRY(hipMalloc(&big.ub, (size_t)n * sizeof(int64_t)));
        lcp_status st = sort_rows(tokens, n, g, idx->V, s, newkeys, big.perm);
        if (st != LCP_OK) return st;  // index unchanged
        HIP_TRY(launch_gather_rows(newkeys, big.perm, n, W, big.sorted, s));  // validated by sort_rows
        nsorted = big.sorted;
        nperm = big.perm;
        ub = big.ub;
    }
    if (n > kRankSortMax) HIP_TRY(launch_upper_bounds(src.sorted, N, nsorted, n, g, ub, s));
    HIP_TRY(launch_merge_sorted(src.sorted, src.perm, src.A, N, nsorted, nperm, ub, n, g, dst.sorted, dst.perm,
                                dst.A, s));
    const int levels = search_table_levels(M);
    HIP_TRY(launch_append_tail(dst.perm, dst.sorted, M, g, idx->V, rows, N, dst.bmin, dst.dir, plane, levels, dst.stab,
                               s));
    HIP_TRY(hipMemcpyAsync(a.flag_host, a.flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (*a.flag_host == epoch) return fail(LCP_ERANGE, "a token is >= V = %d", idx->V);  // index unchanged

    // commit
    if (fresh.rows) {
        std::swap(idx->d_rows, fresh.rows);
        std::swap(idx->d_plane, fresh.plane);
        idx->rows_cap = rows_cap;
    }
    idx->cur ^= 1;
    idx->N = M;
    idx->stab_levels = levels;
    idx->generation += 1;
    return LCP_OK;
}

}  // namespace

extern "C" {

lcp_status lcp_index_build(const void* tokens, int64_t N, int32_t L, int32_t V, void* stream, lcp_index** out) {
    if (!out) return fail(LCP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!tokens) return fail(LCP_EINVAL, "tokens is NULL");
    if (N < 1 || N > kMaxRows) return fail(LCP_EINVAL, "N = %lld is outside [1, 2^31 - 2^16]", (long long)N);
    if (L < 1 || L > LCP_L_MAX) return fail(LCP_EINVAL, "L = %d is outside [1, %d]", L, LCP_L_MAX);
    if (V < 1 || V > 65536) return fail(LCP_EINVAL, "V = %d is outside [1, 65536]", V);
    lcp_index* idx = new lcp_index();
    hipError_t e = hipGetDevice(&idx->device);
    if (e != hipSuccess) {
        delete idx;
        return fail(LCP_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    }
    if (hipDeviceGetAttribute(&idx->cus, hipDeviceAttributeMultiprocessorCount, idx->device) != hipSuccess)
        idx->cus = 256;
    idx->N = N;
    idx->L = L;
    idx->V = V;
    idx->g = make_geo(L, V <= 256 ? 1 : 2);
    lcp_status st = build_into(idx, tokens, static_cast<hipStream_t>(stream));
    if (st != LCP_OK) {
        std::string msg = g_err;
        hipStreamSynchronize(static_cast<hipStream_t>(stream));
        destroy_index(idx);
        g_err = msg;
        return st;
    }
    *out = idx;
    return LCP_OK;
}

lcp_status lcp_topk(const lcp_index* index, const void* queries, int64_t Q, const int32_t* k, int32_t* out_ids,
                    int32_t* out_lcp, void* stream) {
    return query_host(index, Path::Index, queries, Q, k, out_ids, out_lcp, stream);
}

lcp_status lcp_topk_stats(const lcp_index* index, const void* queries, int64_t Q, const int32_t* k,
                          int32_t* out_ids, int32_t* out_lcp, int32_t* stats, void* stream) {
    if (Q > 0 && !stats) return fail(LCP_EINVAL, "stats is NULL");
    if (reinterpret_cast<uintptr_t>(stats) % 16 != 0) return fail(LCP_EINVAL, "stats is not 16-byte aligned");
    return query_host(index, Path::Index, queries, Q, k, out_ids, out_lcp, stream, stats);
}

lcp_status lcp_scan_topk(const lcp_index* index, const void* queries, int64_t Q, const int32_t* k,
                         int32_t* out_ids, int32_t* out_lcp, void* stream) {
    return query_host(index, Path::Scan, queries, Q, k, out_ids, out_lcp, stream);
}

lcp_status lcp_bucket_scan_topk(const lcp_index* index, const void* queries, int64_t Q, int32_t depth,
                                const int32_t* k, int32_t* out_ids, int32_t* out_lcp, int32_t* bounds,
                                void* stream) {
    if (index && (depth < 0 || depth > index->L))
        return fail(LCP_EINVAL, "depth = %d is outside [0, L = %d]", depth, index->L);
    if (reinterpret_cast<uintptr_t>(bounds) % 8 != 0) return fail(LCP_EINVAL, "bounds is not 8-byte aligned");
    return query_host(index, Path::Bucket, queries, Q, k, out_ids, out_lcp, stream, bounds, depth);
}

lcp_status lcp_topk_dev(const lcp_index* index, const void* queries, int64_t Q, const int32_t* k_dev,
                        const int64_t* off_dev, int32_t k_max, int32_t* out_ids, int32_t* out_lcp, void* stream) {
    return query_dev(index, Path::Index, queries, Q, k_dev, off_dev, k_max, out_ids, out_lcp, stream);
}

lcp_status lcp_scan_topk_dev(const lcp_index* index, const void* queries, int64_t Q, const int32_t* k_dev,
                             const int64_t* off_dev, int32_t k_max, int32_t* out_ids, int32_t* out_lcp,
                             void* stream) {
    return query_dev(index, Path::Scan, queries, Q, k_dev, off_dev, k_max, out_ids, out_lcp, stream);
}

lcp_status lcp_scan_topk_dev_noalloc(const lcp_index* idx, const void* queries, int64_t Q, const int32_t* k_dev,
                                     const int64_t* off_dev, int32_t k_max, int32_t* out_ids, int32_t* out_lcp,
                                     void* stream) {
    lcp_status st = check_query_args(idx, queries, Q, out_ids, out_lcp);
    if (st != LCP_OK) return st;
    if (Q == 0) return LCP_OK;
    if (!k_dev || !off_dev) return fail(LCP_EINVAL, "NULL k_dev or off_dev");
    if (k_max < 1 || k_max > LCP_K_MAX) return fail(LCP_EINVAL, "k_max = %d is outside [1, %d]", k_max, LCP_K_MAX);
    if (Q > kSliceScan)
        return fail(LCP_EINVAL, "Q = %lld is above %lld, the largest batch of one allocation-free scan",
                    (long long)Q, (long long)kSliceScan);
    // everything but the partial lists, then the partial lists in what is left
    const ScanPlan probe = plan_scan(idx->N, idx->g.W, Q, k_max, 0);
    const size_t fixed = scan_partial_entries(probe, Q, k_max, idx->g) * sizeof(uint64_t);
    const int64_t left = fixed < kNoAllocScratchBytes ? (int64_t)(kNoAllocScratchBytes - fixed) : 0;
    const ScanPlan plan = plan_scan(idx->N, idx->g.W, Q, k_max, left);
    if (plan.nparts == 0 ||
        scan_partial_entries(plan, Q, k_max, idx->g) * sizeof(uint64_t) > kNoAllocScratchBytes)
        return fail(LCP_EINVAL,
                    "Q = %lld queries with k_max = %d need more than the %zu bytes of fixed scratch "
                    "(at least %lld bytes); split the batch",
                    (long long)Q, k_max, kNoAllocScratchBytes,
                    (long long)(fixed + (size_t)Q * (size_t)k_max * 16));
    HIP_TRY(hipSetDevice(idx->device));
    uint64_t* ptr = nullptr;
    st = scratch_on_device(idx->device, &ptr);
    if (st != LCP_OK) return st;
    QueryBatch qb;
    qb.raw = queries;
    qb.Q = Q;
    qb.k = k_dev;
    qb.off = off_dev;
    qb.k_uniform = 0;
    qb.q_base = 0;
    qb.k_max = k_max;
    qb.out_ids = out_ids;
    qb.out_lcp = out_lcp;
    HIP_TRY(launch_scan(idx->view(), qb, plan, ptr, static_cast<hipStream_t>(stream), nullptr, nullptr, nullptr));
    return LCP_OK;
}

lcp_status lcp_topk_persistent(const lcp_index* idx, const void* queries, int64_t q_capacity,
                               const int64_t* q_count_dev, const int32_t* k_dev, const int64_t* off_dev, int32_t k_max,
                               int32_t* out_ids, int32_t* out_lcp, int32_t blocks, void* stream) {
    if (!idx) return fail(LCP_EINVAL, "index is NULL");
    if (q_capacity < 1 || q_capacity > INT32_MAX)
        return fail(LCP_EINVAL, "q_capacity = %lld is outside [1, 2^31)", (long long)q_capacity);
    if (!queries || !q_count_dev || !k_dev || !off_dev || !out_ids || !out_lcp)
        return fail(LCP_EINVAL, "NULL device pointer");
    if (k_max < 1 || k_max > LCP_K_MAX) return fail(LCP_EINVAL, "k_max = %d is outside [1, %d]", k_max, LCP_K_MAX);
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(idx->mu);
    StreamCtx* c = nullptr;
    lcp_status st = get_ctx(idx, s, &c);
    if (st != LCP_OK) return st;
    if (!c->d_counter) HIP_TRY(hipMalloc(&c->d_counter, sizeof(unsigned long long)));
    // blocks <= 0: one wave per query of the capacity
    const int64_t cover = (q_capacity + 3) / 4;
    const int b = blocks > 0 ? blocks : (int)cover;
    const bool looping = (int64_t)b < cover;
    QueryBatch qb;
    qb.raw = queries;
    qb.Q = 0;  // read on the device
    qb.k = k_dev;
    qb.off = off_dev;
    qb.k_uniform = 0;
    qb.q_base = 0;
    qb.k_max = k_max;
    qb.out_ids = out_ids;
    qb.out_lcp = out_lcp;
    HIP_TRY(launch_index_query_persistent(idx->view(), qb, q_count_dev, c->d_counter, b, looping, s));
    return LCP_OK;
}

lcp_status lcp_index_append(lcp_index* index, const void* tokens, int64_t n, void* stream) {
    if (!index) return fail(LCP_EINVAL, "index is NULL");
    if (n == 0) return LCP_OK;
    if (!tokens) return fail(LCP_EINVAL, "tokens is NULL");
    if (n < 0 || index->N + n > kMaxRows)
        return fail(LCP_EINVAL, "n = %lld would take N past 2^31 - 2^16", (long long)n);
    std::lock_guard<std::mutex> lk(index->mu);
    HIP_TRY(hipSetDevice(index->device));
    return append_into(index, tokens, n, static_cast<hipStream_t>(stream));
}

void lcp_index_free(lcp_index* index) { destroy_index(index); }

const char* lcp_last_error(void) { return g_err.c_str(); }

lcp_status lcp_index_info(const lcp_index* idx, int64_t* N, int32_t* L, int32_t* V, int32_t* token_bytes,
                          int32_t* row_words) {
    if (!idx) return fail(LCP_EINVAL, "index is NULL");
    if (N) *N = idx->N;
    if (L) *L = idx->L;
    if (V) *V = idx->V;
    if (token_bytes) *token_bytes = idx->g.tb;
    if (row_words) *row_words = idx->g.W;
    return LCP_OK;
}

lcp_status lcp_index_views(const lcp_index* idx, const int32_t** perm, const uint8_t** adj_lcp,
                           const uint32_t** sorted_keys, const uint32_t** id_keys) {
    if (!idx) return fail(LCP_EINVAL, "index is NULL");
    const SortedCopy& c = idx->cp[idx->cur];
    if (perm) *perm = c.perm;
    if (adj_lcp) *adj_lcp = c.A;
    if (sorted_keys) *sorted_keys = c.sorted;
    if (id_keys) *id_keys = idx->d_rows;
    return LCP_OK;
}

lcp_status lcp_index_reserve(lcp_index* idx, int64_t rows, void* stream) {
    if (!idx) return fail(LCP_EINVAL, "index is NULL");
    if (rows < 0 || rows > kMaxRows) return fail(LCP_EINVAL, "rows = %lld is outside [0, 2^31 - 2^16]", (long long)rows);
    std::lock_guard<std::mutex> lk(idx->mu);
    HIP_TRY(hipSetDevice(idx->device));
    if (rows <= idx->N) rows = idx->N;
    return reserve_into(idx, rows, static_cast<hipStream_t>(stream));
}

lcp_status lcp_index_set_search(lcp_index* idx, int32_t mode) {
    if (!idx) return fail(LCP_EINVAL, "index is NULL");
    if (mode != 0 && mode != 1) return fail(LCP_EINVAL, "search mode %d is not 0 or 1", mode);
    std::lock_guard<std::mutex> lk(idx->mu);
    for (auto& kv : idx->ctx) HIP_TRY(hipStreamSynchronize(kv.first));
    if (idx->search_mode != mode) idx->generation += 1;  // captured graphs hold the old view
    idx->search_mode = mode;
    return LCP_OK;
}

lcp_status lcp_index_search_mode(const lcp_index* idx, int32_t* mode) {
    if (!idx || !mode) return fail(LCP_EINVAL, "NULL index or output pointer");
    std::lock_guard<std::mutex> lk(idx->mu);
    *mode = idx->search_mode;
    return LCP_OK;
}

lcp_status lcp_index_generation(const lcp_index* idx, uint64_t* generation) {
    if (!idx || !generation) return fail(LCP_EINVAL, "NULL index or output pointer");
    std::lock_guard<std::mutex> lk(idx->mu);
    *generation = idx->generation;
    return LCP_OK;
}

lcp_status lcp_scan_info(const lcp_index* idx, int64_t Q, int32_t k_max, int32_t* query_groups, int32_t* chunks,
                         int64_t* seed_rows) {
    if (!idx) return fail(LCP_EINVAL, "index is NULL");
    if (Q < 1 || k_max < 1 || k_max > LCP_K_MAX) return fail(LCP_EINVAL, "Q or k_max out of range");
    const ScanPlan p = plan_scan(idx->N, idx->g.W, std::min<int64_t>(Q, kSliceScan), k_max);
    if (query_groups) *query_groups = p.qgroups;
    if (chunks) *chunks = p.chunks;
    if (seed_rows) *seed_rows = p.seed_rows;
    return LCP_OK;
}

lcp_status lcp_set_kernel_timing(const lcp_index* idx, int32_t enable) {
    if (!idx) return fail(LCP_EINVAL, "index is NULL");
    std::lock_guard<std::mutex> lk(idx->mu);
    idx->timing = enable != 0;
    return LCP_OK;
}

lcp_status lcp_kernel_time(const lcp_index* idx, int32_t which, double* total_ms, int64_t* launches) {
    if (!idx) return fail(LCP_EINVAL, "index is NULL");
    if (which < 0 || which > 2) return fail(LCP_EINVAL, "which = %d is outside [0, 2]", which);
    std::lock_guard<std::mutex> lk(idx->mu);
    // fold every recorded interval into the accumulators; events are recycled
    std::vector<hipEvent_t> freed;
    for (auto& t : idx->timed) {
        HIP_TRY(hipEventSynchronize(t.b));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, t.a, t.b));
        idx->acc_ms[t.which] += ms;
        idx->acc_n[t.which] += 1;
        freed.push_back(t.a);
        freed.push_back(t.b);
    }
    idx->timed.clear();
    std::sort(freed.begin(), freed.end());
    freed.erase(std::unique(freed.begin(), freed.end()), freed.end());
    for (auto e : freed) idx->event_pool.push_back(e);
    if (total_ms) *total_ms = idx->acc_ms[which];
    if (launches) *launches = idx->acc_n[which];
    // reading resets the accumulator that was read
    idx->acc_ms[which] = 0;
    idx->acc_n[which] = 0;
    return LCP_OK;
}

}  // extern "C"
