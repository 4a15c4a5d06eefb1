// Graph construction on the device: the adjacency of Sec. II (undirected,
// unweighted, A in {0,1}) from an edge list, as a canonical CSR, plus the
// execution plan the hop kernel runs on.
//
//   ingest     validate ids, emit both orientations of every pair as a 64-bit
//              key (row << B) | col, self-loops as a sentinel past every row
//   sort       stable LSD radix sort of the keys (primitives.hip)
//   unique     keep the first of each run of equal keys, drop sentinels
//   CSR        rowptr by binary search of each row's first key, colidx from the
//              low bits, degree = row length
//   plan       node order by descending degree (ties by id) and the CSR
//              relabelled into it: the hop kernel then sees degree-homogeneous
//              waves, the heavy rows first, and the most gathered rows packed
//              together
//   merge      (stream_add) resident keys and increment keys merged by rank,
//              duplicates dropped, CSR and plan rebuilt
#include "internal.h"

namespace ifgp {
namespace {

constexpr int T256 = 256;

__device__ __forceinline__ int64_t block_sum_i64(int64_t v) {
    __shared__ int64_t red[T256 / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t t = 0;
#pragma unroll
    for (int i = 0; i < T256 / 64; ++i) t += red[i];
    __syncthreads();
    return t;
}

// counters[0] = self-loop pairs, counters[1] = 1 if any id is out of range
__global__ __launch_bounds__(T256) void ingest_kernel(const int64_t *__restrict__ src,
                                                      const int64_t *__restrict__ dst, int64_t E,
                                                      int64_t N, int B,
                                                      uint64_t *__restrict__ keys,
                                                      int64_t *__restrict__ counters) {
    const int64_t e = (int64_t)blockIdx.x * T256 + threadIdx.x;
    int64_t loop = 0, bad = 0;
    if (e < E) {
        const int64_t u = src[e], v = dst[e];
        const uint64_t sent = (uint64_t)N << B;
        if (u < 0 || u >= N || v < 0 || v >= N) {
            bad = 1;
            keys[2 * e] = sent;
            keys[2 * e + 1] = sent;
        } else if (u == v) {
            loop = 1;
            keys[2 * e] = sent;
            keys[2 * e + 1] = sent;
        } else {
            keys[2 * e] = ((uint64_t)u << B) | (uint64_t)v;
            keys[2 * e + 1] = ((uint64_t)v << B) | (uint64_t)u;
        }
    }
    loop = block_sum_i64(loop);
    bad = block_sum_i64(bad);
    if (threadIdx.x == 0) {
        if (loop) atomicAdd((unsigned long long *)&counters[0], (unsigned long long)loop);
        if (bad) atomicOr((unsigned long long *)&counters[1], 1ull);
    }
}

// flag[i] = 1 for the first key of each run of equal keys whose row is < N
__global__ void unique_flags_kernel(const uint64_t *__restrict__ k, int64_t n, int B, int64_t N,
                                    uint8_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t x = k[i];
    const bool first = (i == 0) || (k[i - 1] != x);
    flag[i] = (first && (int64_t)(x >> B) < N) ? 1 : 0;
}

__global__ void compact_kernel(const uint64_t *__restrict__ k, const uint8_t *__restrict__ flag,
                               const int64_t *__restrict__ pos, int64_t n,
                               uint64_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flag[i]) out[pos[i]] = k[i];
}

// rowptr[r] = first index p with ukeys[p] >= (r << B), r = 0..N
__global__ void rowptr_kernel(const uint64_t *__restrict__ uk, int64_t nnz, int B, int64_t N,
                              int64_t *__restrict__ rowptr) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > N) return;
    const uint64_t target = (uint64_t)r << B;
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (uk[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    rowptr[r] = lo;
}

__global__ void colidx_kernel(const uint64_t *__restrict__ uk, int64_t nnz, uint64_t mask,
                              int32_t *__restrict__ colidx) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) colidx[p] = (int32_t)(uk[p] & mask);
}

// deg and the statistics the plan needs: stats[0] = max degree,
// stats[1] = rows with deg >= HUB_DEGREE, stats[2] = rows with deg >= MED_DEGREE
__global__ __launch_bounds__(T256) void degree_kernel(const int64_t *__restrict__ rowptr,
                                                      int64_t N, int32_t *__restrict__ deg,
                                                      int64_t *__restrict__ stats) {
    const int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x;
    int64_t dg = 0;
    if (i < N) {
        dg = rowptr[i + 1] - rowptr[i];
        deg[i] = (int32_t)dg;
    }
    int64_t mx = dg;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off, 64));
    __shared__ int64_t red[T256 / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = max(max(red[0], red[1]), max(red[2], red[3]));
    __syncthreads();
    const int64_t hub = block_sum_i64(dg >= HUB_DEGREE ? 1 : 0);
    const int64_t med = block_sum_i64(dg >= MED_DEGREE ? 1 : 0);
    if (threadIdx.x == 0) {
        atomicMax((unsigned long long *)&stats[0], (unsigned long long)mx);
        if (hub) atomicAdd((unsigned long long *)&stats[1], (unsigned long long)hub);
        if (med) atomicAdd((unsigned long long *)&stats[2], (unsigned long long)med);
    }
}

// key = (max_deg - deg) << B | node: ascending key = descending degree, ties by id
__global__ void order_keys_kernel(const int32_t *__restrict__ deg, int64_t N, int32_t max_deg,
                                  int B, uint64_t *__restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) keys[i] = ((uint64_t)(max_deg - deg[i]) << B) | (uint64_t)i;
}

__global__ void perm_kernel(const uint64_t *__restrict__ keys, int64_t N, uint64_t mask,
                            const int32_t *__restrict__ deg, int32_t *__restrict__ perm,
                            int32_t *__restrict__ iperm, int32_t *__restrict__ ideg) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int32_t node = (int32_t)(keys[k] & mask);
    perm[k] = node;
    iperm[node] = (int32_t)k;
    ideg[k] = deg[node];
}

// One thread per stored entry p of the canonical CSR (unique key (i, j)):
// its place in the relabelled CSR is irowptr[iperm[i]] + (p - rowptr[i]) and
// its column becomes iperm[j].  Entries are independent, so many lookups are
// in flight at once.
__global__ void relabel_kernel(const uint64_t *__restrict__ uk, int64_t nnz, int B,
                               const int64_t *__restrict__ rowptr,
                               const int32_t *__restrict__ iperm,
                               const int64_t *__restrict__ irowptr,
                               int32_t *__restrict__ icolidx) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    const uint64_t key = uk[p];
    const int64_t i = (int64_t)(key >> B);
    const int64_t j = (int64_t)(key & (((uint64_t)1 << B) - 1));
    icolidx[irowptr[iperm[i]] + (p - rowptr[i])] = iperm[j];
}

// keys of a canonical CSR, packed with B bits per id: (row << B) | col
__global__ __launch_bounds__(T256) void csr_keys_kernel(const int64_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ colidx,
                                                        int64_t N, int B,
                                                        uint64_t *__restrict__ keys) {
    const int64_t r = (int64_t)blockIdx.x * (T256 / 16) + (threadIdx.x >> 4);
    const int l = threadIdx.x & 15;
    if (r >= N) return;
    for (int64_t t = rowptr[r] + l; t < rowptr[r + 1]; t += 16)
        keys[t] = ((uint64_t)r << B) | (uint64_t)(uint32_t)colidx[t];
}

// Stable merge by rank: a[i] goes to i + #{b < a[i]}, b[j] to j + #{a <= b[j]}.
__global__ void merge_rank_kernel(const uint64_t *__restrict__ a, int64_t na,
                                  const uint64_t *__restrict__ b, int64_t nb,
                                  uint64_t *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < na) {
        const uint64_t x = a[t];
        int64_t lo = 0, hi = nb;
        while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            if (b[mid] < x) lo = mid + 1;
            else hi = mid;
        }
        out[t + lo] = x;
    } else if (t < na + nb) {
        const int64_t j = t - na;
        const uint64_t x = b[j];
        int64_t lo = 0, hi = na;
        while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            if (a[mid] <= x) lo = mid + 1;
            else hi = mid;
        }
        out[j + lo] = x;
    }
}

inline unsigned grid1(int64_t n, int t = T256) { return (unsigned)ceil_div(n, t); }

ifgp_status copy_d2h_sync(void *h, const void *d, size_t bytes, hipStream_t s) {
    IFGP_HIP(hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, s));
    IFGP_HIP(hipStreamSynchronize(s));
    return IFGP_OK;
}

// Keys of E pairs -> 2E keys; reports self-loop pairs, fails on bad ids.
ifgp_status ingest(const int64_t *src, const int64_t *dst, int64_t E, int64_t N, int B,
                   hipStream_t s, Buf &keys, int64_t &loops) {
    IFGP_TRY(alloc(keys, sizeof(uint64_t) * 2 * E, s));
    Buf cnt;
    IFGP_TRY(alloc(cnt, sizeof(int64_t) * 2, s));
    IFGP_TRY(fill_i64(cnt.as<int64_t>(), 2, 0, s));
    if (E > 0) {
        ingest_kernel<<<grid1(E), T256, 0, s>>>(src, dst, E, N, B, keys.as<uint64_t>(),
                                                cnt.as<int64_t>());
        IFGP_LAUNCHED();
    }
    int64_t h[2] = {0, 0};
    IFGP_TRY(copy_d2h_sync(h, cnt.p, sizeof(h), s));
    if (h[1]) {
        set_error("edge list holds a node id outside [0, %lld)", (long long)N);
        return IFGP_E_RANGE;
    }
    loops = h[0];
    return IFGP_OK;
}

// Sorted keys (n of them, some may repeat or be sentinels) -> unique keys.
ifgp_status unique_keys(const uint64_t *k, int64_t n, int B, int64_t N, hipStream_t s, Buf &uk,
                        int64_t &nu) {
    Buf flag, pos, tot;
    IFGP_TRY(alloc(flag, n, s));
    IFGP_TRY(alloc(pos, sizeof(int64_t) * n, s));
    IFGP_TRY(alloc(tot, sizeof(int64_t), s));
    if (n > 0) {
        unique_flags_kernel<<<grid1(n), T256, 0, s>>>(k, n, B, N, flag.as<uint8_t>());
        IFGP_LAUNCHED();
    }
    IFGP_TRY(exclusive_scan<uint8_t>(flag.as<uint8_t>(), pos.as<int64_t>(), n, tot.as<int64_t>(),
                                     s));
    IFGP_TRY(copy_d2h_sync(&nu, tot.p, sizeof(int64_t), s));
    IFGP_TRY(alloc(uk, sizeof(uint64_t) * nu, s));
    if (n > 0) {
        compact_kernel<<<grid1(n), T256, 0, s>>>(k, flag.as<uint8_t>(), pos.as<int64_t>(), n,
                                                 uk.as<uint64_t>());
        IFGP_LAUNCHED();
    }
    return IFGP_OK;
}

// Unique sorted keys -> canonical CSR + plan.
ifgp_status csr_and_plan(const uint64_t *uk, int64_t nnz, int B, int64_t N, hipStream_t s,
                         GraphData &g) {
    g.N = N;
    g.nnz = nnz;
    IFGP_TRY(alloc(g.rowptr, sizeof(int64_t) * (N + 1), s));
    IFGP_TRY(alloc(g.colidx, sizeof(int32_t) * nnz, s));
    IFGP_TRY(alloc(g.deg, sizeof(int32_t) * N, s));
    rowptr_kernel<<<grid1(N + 1), T256, 0, s>>>(uk, nnz, B, N, g.rowptr.as<int64_t>());
    IFGP_LAUNCHED();
    if (nnz > 0) {
        colidx_kernel<<<grid1(nnz), T256, 0, s>>>(uk, nnz, ((uint64_t)1 << B) - 1,
                                                  g.colidx.as<int32_t>());
        IFGP_LAUNCHED();
    }
    Buf stats;
    IFGP_TRY(alloc(stats, sizeof(int64_t) * 3, s));
    IFGP_TRY(fill_i64(stats.as<int64_t>(), 3, 0, s));
    degree_kernel<<<grid1(N), T256, 0, s>>>(g.rowptr.as<int64_t>(), N, g.deg.as<int32_t>(),
                                            stats.as<int64_t>());
    IFGP_LAUNCHED();
    int64_t st[3];
    IFGP_TRY(copy_d2h_sync(st, stats.p, sizeof(st), s));
    g.max_deg = (int32_t)st[0];
    g.n_hub = st[1];
    g.n_med = st[2] - st[1];

    // node order by descending degree
    const int dbits = bit_width((uint64_t)g.max_deg);
    Buf ka, kb;
    IFGP_TRY(alloc(ka, sizeof(uint64_t) * N, s));
    IFGP_TRY(alloc(kb, sizeof(uint64_t) * N, s));
    order_keys_kernel<<<grid1(N), T256, 0, s>>>(g.deg.as<int32_t>(), N, g.max_deg, B,
                                                ka.as<uint64_t>());
    IFGP_LAUNCHED();
    uint64_t *sorted = nullptr;
    IFGP_TRY(radix_sort_u64(ka.as<uint64_t>(), kb.as<uint64_t>(), N, B + dbits, s, &sorted));
    IFGP_TRY(alloc(g.perm, sizeof(int32_t) * N, s));
    IFGP_TRY(alloc(g.iperm, sizeof(int32_t) * N, s));
    Buf ideg;
    IFGP_TRY(alloc(ideg, sizeof(int32_t) * N, s));
    perm_kernel<<<grid1(N), T256, 0, s>>>(sorted, N, ((uint64_t)1 << B) - 1, g.deg.as<int32_t>(),
                                          g.perm.as<int32_t>(), g.iperm.as<int32_t>(),
                                          ideg.as<int32_t>());
    IFGP_LAUNCHED();
    IFGP_TRY(alloc(g.irowptr, sizeof(int64_t) * (N + 1), s));
    IFGP_TRY(exclusive_scan<int32_t>(ideg.as<int32_t>(), g.irowptr.as<int64_t>(), N,
                                     g.irowptr.as<int64_t>() + N, s));
    IFGP_TRY(alloc(g.icolidx, sizeof(int32_t) * nnz, s));
    if (nnz > 0) {
        relabel_kernel<<<grid1(nnz), T256, 0, s>>>(uk, nnz, B, g.rowptr.as<int64_t>(),
                                                   g.iperm.as<int32_t>(), g.irowptr.as<int64_t>(),
                                                   g.icolidx.as<int32_t>());
        IFGP_LAUNCHED();
    }
    return IFGP_OK;
}

}  // namespace

ifgp_status build_graph_device(const int64_t *src, const int64_t *dst, int64_t E, int64_t N,
                               hipStream_t s, GraphData &out) {
    const int B = bit_width((uint64_t)N);  // holds 0..N (N is the sentinel row)
    Buf keys;
    int64_t loops = 0;
    IFGP_TRY(ingest(src, dst, E, N, B, s, keys, loops));
    Buf tmp;
    IFGP_TRY(alloc(tmp, sizeof(uint64_t) * 2 * E, s));
    uint64_t *sorted = nullptr;
    IFGP_TRY(radix_sort_u64(keys.as<uint64_t>(), tmp.as<uint64_t>(), 2 * E, 2 * B, s, &sorted));
    Buf uk;
    int64_t nnz = 0;
    IFGP_TRY(unique_keys(sorted, 2 * E, B, N, s, uk, nnz));
    keys.reset();
    tmp.reset();
    GraphData g;
    IFGP_TRY(csr_and_plan(uk.as<uint64_t>(), nnz, B, N, s, g));
    g.self_loops = loops;
    g.dups = (E - loops) - nnz / 2;
    out = std::move(g);
    return IFGP_OK;
}

ifgp_status merge_graph_device(const GraphData &in, const int64_t *src, const int64_t *dst,
                               int64_t E, int64_t new_N, hipStream_t s, GraphData &out) {
    const int B = bit_width((uint64_t)new_N);
    // increment: keys, sort, unique
    Buf keys;
    int64_t loops = 0;
    IFGP_TRY(ingest(src, dst, E, new_N, B, s, keys, loops));
    Buf tmp;
    IFGP_TRY(alloc(tmp, sizeof(uint64_t) * 2 * E, s));
    uint64_t *sorted = nullptr;
    IFGP_TRY(radix_sort_u64(keys.as<uint64_t>(), tmp.as<uint64_t>(), 2 * E, 2 * B, s, &sorted));
    Buf inc;
    int64_t ninc = 0;
    IFGP_TRY(unique_keys(sorted, 2 * E, B, new_N, s, inc, ninc));
    keys.reset();
    tmp.reset();
    // resident keys repacked with B bits (row-major order is unchanged)
    Buf res;
    IFGP_TRY(alloc(res, sizeof(uint64_t) * in.nnz, s));
    if (in.N > 0) {
        csr_keys_kernel<<<grid1(in.N, 16), T256, 0, s>>>(in.rowptr.as<int64_t>(),
                                                         in.colidx.as<int32_t>(), in.N, B,
                                                         res.as<uint64_t>());
        IFGP_LAUNCHED();
    }
    Buf merged;
    const int64_t nm = in.nnz + ninc;
    IFGP_TRY(alloc(merged, sizeof(uint64_t) * nm, s));
    if (nm > 0) {
        merge_rank_kernel<<<grid1(nm), T256, 0, s>>>(res.as<uint64_t>(), in.nnz,
                                                     inc.as<uint64_t>(), ninc,
                                                     merged.as<uint64_t>());
        IFGP_LAUNCHED();
    }
    res.reset();
    inc.reset();
    Buf uk;
    int64_t nnz = 0;
    IFGP_TRY(unique_keys(merged.as<uint64_t>(), nm, B, new_N, s, uk, nnz));
    merged.reset();
    GraphData g;
    IFGP_TRY(csr_and_plan(uk.as<uint64_t>(), nnz, B, new_N, s, g));
    g.self_loops = in.self_loops + loops;
    // pairs of this increment that added no new edge
    g.dups = in.dups + (E - loops) - (nnz - in.nnz) / 2;
    out = std::move(g);
    return IFGP_OK;
}

}  // namespace ifgp
