// C ABI of libifgp (declared in include/ifgp.h): argument checking, handle
// lifecycle, host<->device staging of edge lists, the allocator hook, error
// strings and hop timing.  Every device step is a kernel in graph.hip,
// primitives.hip or ffp.hip.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <unordered_map>

#include "internal.h"

namespace ifgp {

namespace {
thread_local std::string g_last_error;

struct AllocHook {
    void *(*alloc)(size_t, void *, void *) = nullptr;
    void (*free)(void *, void *, void *) = nullptr;
    void *ctx = nullptr;
} g_hook;
}  // namespace

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

namespace {
// Default allocator: a caching allocator over hipMalloc.  Freed blocks are
// kept per (device, stream) and handed out again only to allocations on the
// same stream, which are ordered after every earlier use of the block on that
// stream (the release is stream-ordered, as with torch's caching allocator).
// A block's device is the one it was allocated on, whichever is current when
// it is released.
// A request reuses the smallest cached block of at least its size and at most
// twice its size; when hipMalloc fails, the whole cache is released and the
// allocation retried.
class BlockCache {
  public:
    void *get(size_t bytes, hipStream_t s) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return nullptr;
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto &fl = free_[{dev, s}];
            auto it = fl.lower_bound(bytes);
            if (it != fl.end() && it->first <= 2 * bytes) {
                void *p = it->second;
                fl.erase(it);
                return p;
            }
        }
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            release_all();
            if (hipMalloc(&p, bytes) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
        }
        std::lock_guard<std::mutex> lk(mu_);
        size_[p] = {bytes, dev};
        return p;
    }
    void put(void *p, hipStream_t s) {
        std::lock_guard<std::mutex> lk(mu_);
        const auto it = size_.find(p);
        if (it == size_.end()) return;  // not a block of this cache
        free_[{it->second.second, s}].insert({it->second.first, p});
    }
    // hipFree every cached block (implicitly synchronises the device).
    void release_all() {
        std::lock_guard<std::mutex> lk(mu_);
        for (auto &kv : free_)
            for (auto &blk : kv.second) {
                (void)hipFree(blk.second);
                size_.erase(blk.second);
            }
        free_.clear();
    }

  private:
    std::mutex mu_;
    std::map<std::pair<int, hipStream_t>, std::multimap<size_t, void *>> free_;
    std::unordered_map<void *, std::pair<size_t, int>> size_;  // bytes, device
};

BlockCache &cache() {
    static BlockCache *c = new BlockCache();  // never destroyed: outlives static handles
    return *c;
}

void cache_free(void *p, void *stream, void *) { cache().put(p, (hipStream_t)stream); }

// Size classes: 512-byte steps below 1 MiB, 2 MiB steps above.
size_t size_class(size_t n) {
    const size_t step = n < (1u << 20) ? 512 : (2u << 20);
    return (n + step - 1) / step * step;
}
}  // namespace

void release_cached_blocks() { cache().release_all(); }

namespace {
std::atomic<int64_t> g_grid_x{GRID_X_BLOCKS};
}  // namespace

int64_t grid_x_blocks() { return g_grid_x.load(std::memory_order_relaxed); }

void *raw_alloc(size_t bytes, hipStream_t s, FreeFn *free_fn, void **ctx) {
    if (g_hook.alloc) {
        *free_fn = g_hook.free;
        *ctx = g_hook.ctx;
        return g_hook.alloc(bytes, (void *)s, g_hook.ctx);
    }
    void *p = cache().get(size_class(bytes), s);
    *free_fn = cache_free;
    *ctx = nullptr;
    return p;
}

void raw_free(void *p, hipStream_t s, FreeFn free_fn, void *ctx) {
    if (p && free_fn) free_fn(p, (void *)s, ctx);
}

ifgp_status alloc(Buf &b, size_t bytes, hipStream_t s) {
    // a block being replaced is released on the stream of the call replacing
    // it: calls on a handle are ordered, so every earlier use of the block
    // comes before that stream's later work
    if (b.p) b.s = s;
    b.reset();
    const size_t n = bytes < 256 ? 256 : ((bytes + 255) / 256) * 256;
    FreeFn fn = nullptr;
    void *ctx = nullptr;
    void *p = raw_alloc(n, s, &fn, &ctx);
    if (!p) {
        set_error("device allocation of %zu bytes failed", n);
        return IFGP_E_OOM;
    }
    b.p = p;
    b.bytes = n;
    b.s = s;
    b.free_fn = fn;
    b.ctx = ctx;
    return IFGP_OK;
}

ifgp_status ensure(Buf &b, size_t bytes, hipStream_t s) {
    if (b.p && b.bytes >= bytes) return IFGP_OK;
    return alloc(b, bytes, s);
}

namespace {

constexpr int64_t MAX_N = 2147483646;  // ids fit int32 with one spare value
// From this many edges a build runs its few oversized buckets on the side stream.
constexpr int64_t BUILD_SIDE_MIN_EDGES = 1 << 19;

ifgp_params resolve(const ifgp_params *p) {
    ifgp_params q;
    ifgp_default_params(&q);
    return p ? *p : q;
}

// Device copies of the edge arrays (or the caller's pointers if already there).
struct Edges {
    Buf sbuf, dbuf;
    const int64_t *src = nullptr, *dst = nullptr;
};

ifgp_status stage_edges(const int64_t *src, const int64_t *dst, int64_t E, int on_device,
                        hipStream_t s, Edges &e) {
    if (E == 0) return IFGP_OK;
    if (on_device) {
        e.src = src;
        e.dst = dst;
        return IFGP_OK;
    }
    IFGP_TRY(alloc(e.sbuf, sizeof(int64_t) * E, s));
    IFGP_TRY(alloc(e.dbuf, sizeof(int64_t) * E, s));
    IFGP_HIP(hipMemcpyAsync(e.sbuf.p, src, sizeof(int64_t) * E, hipMemcpyHostToDevice, s));
    IFGP_HIP(hipMemcpyAsync(e.dbuf.p, dst, sizeof(int64_t) * E, hipMemcpyHostToDevice, s));
    e.src = e.sbuf.as<int64_t>();
    e.dst = e.dbuf.as<int64_t>();
    return IFGP_OK;
}

ifgp_status check_handle(ifgp_graph_t g) {
    if (!g) {
        set_error("NULL graph handle");
        return IFGP_E_INVALID;
    }
    return IFGP_OK;
}

ifgp_status use_device(ifgp_graph_t g) {
    IFGP_HIP(hipSetDevice(g->device));
    return IFGP_OK;
}

// One whole embedding on g; on failure g is left with no job in progress.
// `noalloc` runs it in the device's static scratch array (random input only).
ifgp_status run_job(ifgp_graph_t g, double tau, int32_t K, int32_t d, uint64_t seed,
                    const float *X, const ifgp_params &p, float *out, hipStream_t s,
                    bool noalloc = false) {
    ifgp_status st = noalloc ? job_begin_noalloc(g, tau, K, d, seed, p, out, s)
                             : job_begin(g, tau, K, d, seed, X, p, out, s);
    while (st == IFGP_OK && !g->job.done) {
        ifgp_graph_s *one = g;
        st = jobs_step(&one, 1, s);
    }
    if (st != IFGP_OK) g->job = Job{};
    else g->job.active = false;
    return st;
}

}  // namespace
}  // namespace ifgp

using namespace ifgp;

extern "C" {

IFGP_API ifgp_status ifgp_default_params(ifgp_params *p) {
    if (!p) {
        set_error("NULL params");
        return IFGP_E_INVALID;
    }
    p->alpha = 1.0;
    p->theta = 0.1;
    p->eps = 1e-3;
    p->znorm_ddof = 0;
    p->storage = IFGP_F32;
    return IFGP_OK;
}

IFGP_API ifgp_status ifgp_build_graph(const int64_t *src, const int64_t *dst, int64_t num_edges, int64_t N,
                             int edges_on_device, void *hip_stream, ifgp_graph_t *out) {
    if (!out || N < 1 || N > MAX_N || num_edges < 0 || (num_edges > 0 && (!src || !dst))) {
        set_error("ifgp_build_graph: need out != NULL, 1 <= N <= %lld, num_edges >= 0 and "
                  "edge arrays",
                  (long long)MAX_N);
        return IFGP_E_INVALID;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    ifgp_graph_s *h = new (std::nothrow) ifgp_graph_s();
    if (!h) {
        set_error("host allocation failed");
        return IFGP_E_OOM;
    }
    auto fail = [&](ifgp_status st) {
        (void)ifgp_destroy(h);
        return st;
    };
    const hipError_t de = hipGetDevice(&h->device);
    if (de != hipSuccess) {
        set_error("hipGetDevice: %s", hipGetErrorString(de));
        return fail(IFGP_E_DEVICE);
    }
    h->stream = s;
    Edges e;
    ifgp_status st = stage_edges(src, dst, num_edges, edges_on_device, s, e);
    if (st != IFGP_OK) return fail(st);
    if (num_edges >= BUILD_SIDE_MIN_EDGES) {
        st = ensure_side_stream(h);
        if (st != IFGP_OK) return fail(st);
    }
    st = build_graph_device(e.src, e.dst, num_edges, N, s, h->aux, h->ev_fork, h->ev_join, h->g);
    if (st != IFGP_OK) return fail(st);
    *out = h;
    return IFGP_OK;
}

IFGP_API ifgp_status ifgp_embed(ifgp_graph_t g, double tau, int32_t K, int32_t d, uint64_t seed,
                       const ifgp_params *p, float *out, void *hip_stream) {
    IFGP_TRY(check_handle(g));
    IFGP_TRY(use_device(g));
    hipStream_t s = (hipStream_t)hip_stream;
    g->stream = s;
    return run_job(g, tau, K, d, seed, nullptr, resolve(p), out, s);
}

IFGP_API ifgp_status ifgp_embed_noalloc(ifgp_graph_t g, double tau, int32_t K, int32_t d,
                                        uint64_t seed, const ifgp_params *p, float *out,
                                        void *hip_stream) {
    IFGP_TRY(check_handle(g));
    IFGP_TRY(use_device(g));
    hipStream_t s = (hipStream_t)hip_stream;
    g->stream = s;
    return run_job(g, tau, K, d, seed, nullptr, resolve(p), out, s, true);
}

IFGP_API ifgp_status ifgp_embed_x(ifgp_graph_t g, double tau, int32_t K, int32_t d, const float *X,
                         const ifgp_params *p, float *out, void *hip_stream) {
    IFGP_TRY(check_handle(g));
    if (!X) {
        set_error("NULL X");
        return IFGP_E_INVALID;
    }
    IFGP_TRY(use_device(g));
    hipStream_t s = (hipStream_t)hip_stream;
    g->stream = s;
    return run_job(g, tau, K, d, 0, X, resolve(p), out, s);
}

IFGP_API ifgp_status ifgp_gaussian_input(int64_t N, int32_t d, uint64_t seed, int32_t dtype, void *out,
                                void *hip_stream) {
    if (N < 0 || d < 1 || (N > 0 && !out) || dtype_bytes(dtype) == 0) {
        set_error("ifgp_gaussian_input: need N >= 0, d >= 1, a known dtype and out");
        return IFGP_E_INVALID;
    }
    return gaussian_input_device(N, d, seed, dtype, out, (hipStream_t)hip_stream);
}

IFGP_API ifgp_status ifgp_stream_add(ifgp_graph_t g, const int64_t *src, const int64_t *dst,
                            int64_t num_edges, int64_t new_N, int edges_on_device,
                            void *hip_stream) {
    IFGP_TRY(check_handle(g));
    if (num_edges < 0 || new_N < g->g.N || new_N > MAX_N || (num_edges > 0 && (!src || !dst))) {
        set_error("ifgp_stream_add: need num_edges >= 0, N <= new_N <= %lld and edge arrays",
                  (long long)MAX_N);
        return IFGP_E_INVALID;
    }
    if (g->job.active && !g->job.done) {
        set_error("ifgp_stream_add: the graph has an unfinished job");
        return IFGP_E_STATE;
    }
    IFGP_TRY(use_device(g));
    hipStream_t s = (hipStream_t)hip_stream;
    Edges e;
    IFGP_TRY(stage_edges(src, dst, num_edges, edges_on_device, s, e));
    IFGP_TRY(ensure_colidx(g->g, s));
    GraphData fresh;
    IFGP_TRY(merge_graph_device(g->g, e.src, e.dst, num_edges, new_N, s, fresh));
    // commit: nothing below can fail
    g->stream = s;
    g->g = std::move(fresh);
    g->sc.valid = false;
    g->job = Job{};
    return IFGP_OK;
}

IFGP_API ifgp_status ifgp_embed_batch(ifgp_graph_t *gs, int32_t n, const double *tau, const int32_t *K,
                             const int32_t *d, const uint64_t *seed, const ifgp_params *p,
                             float **outs, void *hip_stream) {
    if (n < 0 || (n > 0 && (!gs || !tau || !K || !d || !seed || !outs))) {
        set_error("ifgp_embed_batch: bad arguments");
        return IFGP_E_INVALID;
    }
    for (int i = 0; i < n; ++i) {
        IFGP_TRY(check_handle(gs[i]));
        for (int k = 0; k < i; ++k)
            if (gs[k] == gs[i]) {
                set_error("ifgp_embed_batch: handle listed twice");
                return IFGP_E_INVALID;
            }
    }
    hipStream_t s = (hipStream_t)hip_stream;
    // a failure leaves none of the graphs with a job in progress
    auto fail = [&](ifgp_status st) {
        for (int i = 0; i < n; ++i) gs[i]->job = Job{};
        return st;
    };
    for (int i = 0; i < n; ++i) {
        ifgp_status st = use_device(gs[i]);
        if (st == IFGP_OK) {
            gs[i]->stream = s;
            st = job_begin(gs[i], tau[i], K[i], d[i], seed[i], nullptr, resolve(p), outs[i], s);
        }
        if (st != IFGP_OK) return fail(st);
    }
    for (;;) {
        bool more = false;
        for (int i = 0; i < n; ++i) more |= !gs[i]->job.done;
        if (!more) break;
        const ifgp_status st = jobs_step(gs, n, s);
        if (st != IFGP_OK) return fail(st);
    }
    for (int i = 0; i < n; ++i) gs[i]->job.active = false;
    return IFGP_OK;
}

IFGP_API ifgp_status ifgp_job_begin(ifgp_graph_t g, double tau, int32_t K, int32_t d, uint64_t seed,
                           const ifgp_params *p, float *out, void *hip_stream) {
    IFGP_TRY(check_handle(g));
    IFGP_TRY(use_device(g));
    hipStream_t s = (hipStream_t)hip_stream;
    g->stream = s;
    return job_begin(g, tau, K, d, seed, nullptr, resolve(p), out, s);
}

IFGP_API ifgp_status ifgp_job_step(ifgp_graph_t *gs, int32_t n, int32_t *done_flags, void *hip_stream) {
    if (n < 0 || (n > 0 && !gs)) {
        set_error("ifgp_job_step: bad arguments");
        return IFGP_E_INVALID;
    }
    for (int i = 0; i < n; ++i) {
        IFGP_TRY(check_handle(gs[i]));
        if (!gs[i]->job.active) {
            set_error("ifgp_job_step: graph %d has no job", i);
            return IFGP_E_STATE;
        }
        for (int k = 0; k < i; ++k)
            if (gs[k] == gs[i]) {
                set_error("ifgp_job_step: handle listed twice");
                return IFGP_E_INVALID;
            }
    }
    hipStream_t s = (hipStream_t)hip_stream;
    if (n > 0) IFGP_TRY(use_device(gs[0]));
    for (int i = 0; i < n; ++i) gs[i]->stream = s;
    IFGP_TRY(jobs_step(gs, n, s));
    if (done_flags)
        for (int i = 0; i < n; ++i) done_flags[i] = gs[i]->job.done ? 1 : 0;
    return IFGP_OK;
}

IFGP_API ifgp_status ifgp_graph_info(ifgp_graph_t g, int64_t *N, int64_t *nnz, int64_t *self_loops_dropped,
                            int64_t *dups_dropped) {
    IFGP_TRY(check_handle(g));
    if (N) *N = g->g.N;
    if (nnz) *nnz = g->g.nnz;
    if (self_loops_dropped) *self_loops_dropped = g->g.self_loops;
    if (dups_dropped) *dups_dropped = g->g.dups;
    return IFGP_OK;
}

IFGP_API ifgp_status ifgp_plan_info(ifgp_graph_t g, int64_t *hub_rows, int64_t *medium_rows,
                                    int64_t *hop_blocks, int32_t *max_degree) {
    IFGP_TRY(check_handle(g));
    if (hub_rows) *hub_rows = g->g.n_hub;
    if (medium_rows) *medium_rows = g->g.n_med;
    if (hop_blocks) *hop_blocks = ifgp::hop_blocks(g->g, 64, IFGP_BF16);  // BF16, width 64
    if (max_degree) *max_degree = g->g.max_deg;
    return IFGP_OK;
}

IFGP_API ifgp_status ifgp_export_csr(ifgp_graph_t g, int64_t *rowptr, int32_t *colidx, int32_t *deg) {
    IFGP_TRY(check_handle(g));
    IFGP_TRY(use_device(g));
    hipStream_t s = g->stream;
    if (colidx) IFGP_TRY(ensure_colidx(g->g, s));
    const GraphData &G = g->g;
    if (rowptr)
        IFGP_HIP(hipMemcpyAsync(rowptr, G.rowptr.p, sizeof(int64_t) * (G.N + 1),
                                hipMemcpyDeviceToHost, s));
    if (colidx && G.nnz > 0)
        IFGP_HIP(hipMemcpyAsync(colidx, G.colidx.p, sizeof(int32_t) * G.nnz,
                                hipMemcpyDeviceToHost, s));
    if (deg)
        IFGP_HIP(hipMemcpyAsync(deg, G.deg.p, sizeof(int32_t) * G.N, hipMemcpyDeviceToHost, s));
    IFGP_HIP(hipStreamSynchronize(s));
    return IFGP_OK;
}

IFGP_API ifgp_status ifgp_export_scales(ifgp_graph_t g, double tau, double eps, double *s_host) {
    IFGP_TRY(check_handle(g));
    if (!s_host || !std::isfinite(tau) || !(eps > 0)) {
        set_error("ifgp_export_scales: need s_host, finite tau and eps > 0");
        return IFGP_E_INVALID;
    }
    IFGP_TRY(use_device(g));
    IFGP_TRY(ensure_scales(g, tau, eps, g->stream));
    return scales_to_host(g, s_host, g->stream);
}

IFGP_API ifgp_status ifgp_footprint_bytes(int64_t N, int64_t nnz, int32_t d, int32_t storage,
                                 int64_t *bytes) {
    const size_t b = dtype_bytes(storage);
    if (!bytes || N < 1 || nnz < 0 || d < 1 || d > 256 || b == 0 || storage == IFGP_F64) {
        set_error("ifgp_footprint_bytes: bad arguments");
        return IFGP_E_INVALID;
    }
    const int64_t Dp = padded_width(d);
    // resident graph: canonical CSR + degrees + plan (perm, iperm, relabelled CSR);
    // until the first export or merge after a build, the build's survivors
    // (4 bytes per edge end, at most nnz as counted here when nnz = 2E) and
    // bucket starts (at most 8 (N + 1)) stand in for the canonical colidx
    int64_t total = 2 * (8 * (N + 1) + 4 * nnz) + 4 * N * 3 + 8 * (N + 1);
    // scales: FP64 s, FP32 s and (s, sqrt(D_tau), r, 0) as float4
    total += 8 * N + 4 * N + 16 * N;
    // two feature buffers, block statistics (bounded by the row classes:
    // hub rows <= nnz / HUB_DEGREE, medium rows <= nnz / MED_DEGREE), coefficients
    const int64_t light = std::max<int64_t>(LIGHT_TARGET_BLOCKS, ceil_div(N, light_rows_per_block(1)));
    const int64_t blocks = nnz / HUB_DEGREE + ceil_div(nnz / MED_DEGREE, MED_ROWS_PER_BLOCK) +
                           light + 2;
    total += 2 * N * Dp * (int64_t)b + 16 * Dp * blocks + 8 * Dp;
    *bytes = total;
    return IFGP_OK;
}

IFGP_API ifgp_status ifgp_set_allocator(void *(*alloc_fn)(size_t, void *, void *),
                               void (*free_fn)(void *, void *, void *), void *ctx) {
    if ((alloc_fn == nullptr) != (free_fn == nullptr)) {
        set_error("ifgp_set_allocator: give both callbacks or neither");
        return IFGP_E_INVALID;
    }
    g_hook.alloc = alloc_fn;
    g_hook.free = free_fn;
    g_hook.ctx = alloc_fn ? ctx : nullptr;
    return IFGP_OK;
}

IFGP_API ifgp_status ifgp_empty_cache(void) {
    release_cached_blocks();
    return IFGP_OK;
}

IFGP_API ifgp_status ifgp_debug_grid_x(int64_t max_x_blocks, int64_t *previous) {
    if (max_x_blocks < 0) {
        set_error("ifgp_debug_grid_x: max_x_blocks must be >= 0");
        return IFGP_E_INVALID;
    }
    const int64_t prev = g_grid_x.exchange(max_x_blocks ? max_x_blocks : GRID_X_BLOCKS);
    if (previous) *previous = prev;
    return IFGP_OK;
}

IFGP_API ifgp_status ifgp_debug_hop_depth(int32_t depth, int32_t *previous) {
    if (depth < -1 || depth > 2) {
        set_error("ifgp_debug_hop_depth: depth must be -1, 0, 1 or 2");
        return IFGP_E_INVALID;
    }
    const int prev = force_hop_depth(depth);
    if (previous) *previous = prev;
    return IFGP_OK;
}

IFGP_API ifgp_status ifgp_timing_enable(ifgp_graph_t g, int enable) {
    IFGP_TRY(check_handle(g));
    g->timing = enable != 0;
    return IFGP_OK;
}

IFGP_API ifgp_status ifgp_timing_read(ifgp_graph_t g, int64_t *hop_launches, double *hop_ms) {
    IFGP_TRY(check_handle(g));
    IFGP_TRY(use_device(g));
    double total = 0.0;
    int64_t count = 0;
    ifgp_status st = IFGP_OK;
    for (auto &pr : g->events) {
        if (st == IFGP_OK && pr.first && pr.second) {
            float ms = 0.f;
            if (hipEventSynchronize(pr.second) != hipSuccess ||
                hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess) {
                set_error("hipEventElapsedTime failed");
                st = IFGP_E_DEVICE;
            } else {
                total += ms;
                ++count;
            }
        }
        if (pr.first) (void)hipEventDestroy(pr.first);
        if (pr.second) (void)hipEventDestroy(pr.second);
    }
    g->events.clear();
    if (hop_launches) *hop_launches = count;
    if (hop_ms) *hop_ms = total;
    return st;
}

IFGP_API ifgp_status ifgp_destroy(ifgp_graph_t g) {
    if (!g) return IFGP_OK;
    (void)hipSetDevice(g->device);
    for (auto &pr : g->events) {
        if (pr.first) (void)hipEventDestroy(pr.first);
        if (pr.second) (void)hipEventDestroy(pr.second);
    }
    if (g->ev_fork) (void)hipEventDestroy(g->ev_fork);
    if (g->ev_join) (void)hipEventDestroy(g->ev_join);
    delete g;   // the auxiliary stream is shared and stays
    return IFGP_OK;
}

IFGP_API const char *ifgp_last_error(void) { return g_last_error.c_str(); }

IFGP_API const char *ifgp_version(void) { return "ifgp 0.1.0 (gfx950)"; }

}  // extern "C"
