// Declarations shared between the libifgp translation units.
#pragma once

#include <vector>

#include "common.h"

namespace ifgp {

// ---- primitives.hip
template <typename In>
ifgp_status exclusive_scan(const In *in, int64_t *out, int64_t n, int64_t *total, hipStream_t s);
ifgp_status fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s);
// Stable sort of n keys by their bits [lo, hi) (bits at and above hi must be
// zero), 8 bits per pass, RADIX_TILE keys per block; a and b are both n
// long; on return *sorted is whichever of them holds the result.  If
// first_hist is given it holds the first pass's counts,
// first_hist[digit * tiles + tile] for digit (key >> lo) & 255, and serves
// as the histogram buffer (256 * tiles entries).
constexpr int RADIX_TILE = 4096;
ifgp_status radix_sort_u64(uint64_t *a, uint64_t *b, int64_t n, int lo, int hi, hipStream_t s,
                           uint64_t **sorted, int64_t *first_hist = nullptr);
// The same for the 2E keys of E edge pairs (edge_keys below), made from the
// pairs by the first pass itself (a and b are both 2E long; first_hist, the
// first pass's counts, is required): the first pass reads the edge lists
// instead of keys that were written out before.
ifgp_status radix_sort_pairs(const int64_t *src, const int64_t *dst, int64_t E, int64_t N, int B,
                             uint64_t *a, uint64_t *b, int lo, int hi, hipStream_t s,
                             uint64_t **sorted, int64_t *first_hist);

// Keys of edge pair (u, v) with B-bit ids: (u << B | v) and (v << B | u); for
// a self loop or an id outside [0, N), two sentinels N << B.
__device__ __forceinline__ void edge_keys(int64_t u, int64_t v, int64_t N, int B, uint64_t &k0,
                                          uint64_t &k1) {
    if (u < 0 || u >= N || v < 0 || v >= N || u == v) {
        k0 = k1 = (uint64_t)N << B;
    } else {
        k0 = ((uint64_t)u << B) | (uint64_t)v;
        k1 = ((uint64_t)v << B) | (uint64_t)u;
    }
}

// Row classes of the hop kernel, by degree.  Rows are kept in descending-
// degree order, so each class is a contiguous range of internal rows.
// The defaults can be overridden at compile time (-DIFGP_HUB_DEGREE=...).
#ifndef IFGP_HUB_DEGREE
#define IFGP_HUB_DEGREE 4096
#endif
#ifndef IFGP_MED_DEGREE
#define IFGP_MED_DEGREE 128
#endif
#ifndef IFGP_LIGHT_ROWS
#define IFGP_LIGHT_ROWS 256
#endif
constexpr int64_t HUB_DEGREE = IFGP_HUB_DEGREE;  // >= : one 256-thread block per row
constexpr int64_t MED_DEGREE = IFGP_MED_DEGREE;  // >= : one wave per row
constexpr int MED_ROWS_PER_BLOCK = 4;
// Light rows per block: at most IFGP_LIGHT_ROWS (or one pass of the block,
// 4 waves of rpw rows each, if that is larger); fewer for small graphs, so
// that a hop still launches about LIGHT_TARGET_BLOCKS blocks.
constexpr int64_t LIGHT_TARGET_BLOCKS = 4096;
constexpr int light_rows_per_block(int rpw) {
    return IFGP_LIGHT_ROWS > 4 * rpw ? IFGP_LIGHT_ROWS : 4 * rpw;
}
inline int light_rows_for(int64_t n_light, int rpw) {
    const int pass = 4 * rpw, max_passes = light_rows_per_block(rpw) / pass;
    int64_t passes = (n_light + LIGHT_TARGET_BLOCKS * pass - 1) / (LIGHT_TARGET_BLOCKS * pass);
    if (passes < 1) passes = 1;
    if (passes > max_passes) passes = max_passes;
    return (int)passes * pass;
}

// Canonical graph plus the execution plan of the hop kernel.
struct GraphData {
    int64_t N = 0, nnz = 0;
    int64_t self_loops = 0, dups = 0;   // totals over every edge ever added
    int32_t max_deg = 0;
    // canonical CSR over original ids, columns ascending
    Buf rowptr;   // int64 N+1
    Buf colidx;   // int32 nnz; after a fresh build, empty until ensure_colidx
    Buf deg;      // int32 N
    // a fresh build's survivors until the canonical colidx is made: per
    // bucket of 2^tcol_s rows, from tcol[bst[b]], local keys (row in the
    // bucket << tcol_B | column) in row order
    Buf tcol;     // uint32, 2E
    Buf bst;      // int64, buckets + 1
    int tcol_B = 0, tcol_s = 0;
    // plan: internal row k holds node perm[k]; rows sorted by degree,
    // descending (ties by id); the CSR relabelled into that order
    Buf perm;     // int32 N
    Buf iperm;    // int32 N (node -> internal row)
    Buf irowptr;  // int64 N+1
    Buf icolidx;  // int32 nnz, internal ids
    int64_t n_hub = 0, n_med = 0;
};

// Per-(tau, eps) node quantities in internal order.
struct Scales {
    bool valid = false;
    double tau = 0, eps = 0;
    Buf s64;       // double N: (D_tau)^{-1/2}
    Buf s32;       // float N: s64 rounded, gathered to form r
    Buf nodeinfo;  // float4 N: (s, sqrt(D_tau), sum_{j in N(i)} s_j, 0)
    Buf stab;      // float: s per bucket of internal ids of one degree (-1: mixed)
};

struct Workspace {
    Buf feat[2];    // N x Dp storage elements each
    Buf partials;   // double2 [hop blocks][Dp]
    Buf ab;         // float [2][Dp]: per-column scale a = 1/sigma and shift b = -mu/sigma
};

// The device memory one embedding works in, as plain pointers: the handle's
// own buffers (Scales, Workspace) or a carved-up region of the library's
// static scratch array (the allocation-free entry point).
struct EmbedMem {
    double *s64 = nullptr;
    float *s32 = nullptr;
    float4 *node = nullptr;
    float *stab = nullptr;
    void *feat[2] = {nullptr, nullptr};
    double2 *partials = nullptr;
    float *ab = nullptr;
};

struct Job {
    bool active = false;
    int32_t K = 0, d = 0, Dp = 0, hop = 0;
    int32_t storage = IFGP_F32;
    double alpha = 1, theta = 0.1;
    int32_t ddof = 0;
    int cur = 0;      // which feat buffer holds the current hop's input
    float *out = nullptr;
    bool done = false;
    bool noalloc = false;   // runs in the static scratch array: no events, no side stream
};

}  // namespace ifgp

struct ifgp_graph_s {
    int device = 0;
    hipStream_t stream = nullptr;   // stream of the most recent call
    hipStream_t aux = nullptr;      // library-owned stream (shared per device) for independent work
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    ifgp::GraphData g;
    ifgp::Scales sc;
    ifgp::Workspace ws;
    ifgp::EmbedMem mem;             // what the current job's kernels read and write
    ifgp::Job job;
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
};

namespace ifgp {

// ---- api.hip
void release_cached_blocks();

// ---- graph.hip
// Build the canonical CSR and plan from edges already in device memory.  If
// aux is given, part of the work runs there, forked from and joined back to
// s with the two events.
ifgp_status build_graph_device(const int64_t *src, const int64_t *dst, int64_t E, int64_t N,
                               hipStream_t s, hipStream_t aux, hipEvent_t ev_fork,
                               hipEvent_t ev_join, GraphData &out);
// Make the canonical colidx of a fresh build from its survivors, on stream s
// (no-op once made); releases the survivors.
ifgp_status ensure_colidx(GraphData &g, hipStream_t s);
// Merge device edges into `in`, producing `out` (in is left unchanged; its
// canonical colidx must be made).
ifgp_status merge_graph_device(const GraphData &in, const int64_t *src, const int64_t *dst,
                               int64_t E, int64_t new_N, hipStream_t s, GraphData &out);

// ---- ffp.hip
// The library's side stream of h's device (shared, created on first use)
// and h's fork/join events.
ifgp_status ensure_side_stream(ifgp_graph_s *h);
ifgp_status ensure_scales(ifgp_graph_s *h, double tau, double eps, hipStream_t s);
ifgp_status job_begin(ifgp_graph_s *h, double tau, int32_t K, int32_t d, uint64_t seed,
                      const float *X, const ifgp_params &p, float *out, hipStream_t s);
// As job_begin (random input only) with every buffer carved out of the
// device's static scratch array: no allocation, no side stream, no events.
// IFGP_E_INVALID if the embedding needs more than NOALLOC_SCRATCH_BYTES.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
ifgp_status job_begin_noalloc(ifgp_graph_s *h, double tau, int32_t K, int32_t d, uint64_t seed,
                              const ifgp_params &p, float *out, hipStream_t s);
// Advance every listed job by one hop (one launch per storage/width class).
ifgp_status jobs_step(ifgp_graph_s **hs, int n, hipStream_t s);
int64_t hop_blocks(const GraphData &g, int Dp, int storage);
// Force the gather depth of every later 2-byte-storage hop (0 normal, 1
// shallow, 2 deep; -1 = per graph); returns the previous setting.
int force_hop_depth(int depth);
int light_rows(const GraphData &g, int Dp, int storage);
ifgp_status gaussian_input_device(int64_t N, int32_t d, uint64_t seed, int32_t dtype, void *out,
                                  hipStream_t s);
ifgp_status scales_to_host(ifgp_graph_s *h, double *s_host, hipStream_t s);

}  // namespace ifgp
