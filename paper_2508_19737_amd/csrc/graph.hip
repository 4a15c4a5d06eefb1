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
#include <algorithm>

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

// Deduplication of sorted keys in tiles of UQ_ITEMS consecutive keys per
// thread: key i is kept iff it differs from key i-1 and its row is < N (self
// loops and padding carry row N).
constexpr int UQ_ITEMS = 8;
constexpr int UQ_TILE = T256 * UQ_ITEMS;

__device__ __forceinline__ bool keep_key(const uint64_t *__restrict__ k, int64_t i, int B,
                                         int64_t N) {
    const uint64_t x = k[i];
    return (i == 0 || k[i - 1] != x) && (int64_t)(x >> B) < N;
}

// Tile t holds keys [t*UQ_TILE, (t+1)*UQ_TILE); round q of the tile gives
// thread j key t*UQ_TILE + q*T256 + j, so loads and stores are coalesced.
__global__ __launch_bounds__(T256) void unique_count_kernel(const uint64_t *__restrict__ k,
                                                            int64_t n, int B, int64_t N,
                                                            int64_t *__restrict__ bcount) {
    const int64_t base = (int64_t)blockIdx.x * UQ_TILE + threadIdx.x;
    int64_t c = 0;
#pragma unroll
    for (int q = 0; q < UQ_ITEMS; ++q) {
        const int64_t i = base + (int64_t)q * T256;
        if (i < n && keep_key(k, i, B, N)) ++c;
    }
    c = block_sum_i64(c);
    if (threadIdx.x == 0) bcount[blockIdx.x] = c;
}

__global__ __launch_bounds__(T256) void unique_write_kernel(const uint64_t *__restrict__ k,
                                                            int64_t n, int B, int64_t N,
                                                            const int64_t *__restrict__ boff,
                                                            uint64_t *__restrict__ out) {
    __shared__ int wcount[UQ_ITEMS][T256 / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * UQ_TILE + threadIdx.x;
    const uint64_t lt = __lanemask_lt();
    bool keep[UQ_ITEMS];
    uint64_t key[UQ_ITEMS];
    int below[UQ_ITEMS];
#pragma unroll
    for (int q = 0; q < UQ_ITEMS; ++q) {
        const int64_t i = base + (int64_t)q * T256;
        keep[q] = i < n && keep_key(k, i, B, N);
        key[q] = keep[q] ? k[i] : 0;
        const uint64_t m = __ballot(keep[q]);
        below[q] = __popcll(m & lt);
        if (lane == 0) wcount[q][w] = __popcll(m);
    }
    __syncthreads();
    // kept keys before (round q, wave w): all earlier rounds, then earlier waves
    int64_t pos = boff[blockIdx.x];
#pragma unroll
    for (int q = 0; q < UQ_ITEMS; ++q) {
        int before = 0, round = 0;
#pragma unroll
        for (int ww = 0; ww < T256 / 64; ++ww) {
            before += ww < w ? wcount[q][ww] : 0;
            round += wcount[q][ww];
        }
        if (keep[q]) out[pos + before + below[q]] = key[q];
        pos += round;
    }
}

// rowptr[r] = first index p with ukeys[p] >= (r << B), r = 0..N
__global__ void rowptr_kernel(const uint64_t *__restrict__ uk, const int64_t *__restrict__ nnz_d,
                              int B, int64_t N, int64_t *__restrict__ rowptr) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > N) return;
    const uint64_t target = (uint64_t)r << B;
    int64_t lo = 0, hi = *nnz_d;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (uk[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    rowptr[r] = lo;
}

__global__ void colidx_kernel(const uint64_t *__restrict__ uk, const int64_t *__restrict__ nnz_d,
                              int64_t bound, uint64_t mask, int32_t *__restrict__ colidx) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < bound && p < *nnz_d) colidx[p] = (int32_t)(uk[p] & mask);
}

// deg and the statistics the plan needs: stats[0] = max degree,
// stats[1] = rows with deg >= HUB_DEGREE, stats[2] = rows with deg >= MED_DEGREE.
// Grid-stride over rows, so that few blocks meet at the atomics.
__global__ __launch_bounds__(T256) void degree_kernel(const int64_t *__restrict__ rowptr,
                                                      int64_t N, int32_t *__restrict__ deg,
                                                      int64_t *__restrict__ stats) {
    int64_t mx = 0, hub = 0, med = 0;
    for (int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * T256) {
        const int64_t dg = rowptr[i + 1] - rowptr[i];
        deg[i] = (int32_t)dg;
        mx = dg > mx ? dg : mx;
        hub += dg >= HUB_DEGREE;
        med += dg >= MED_DEGREE;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t o = __shfl_xor(mx, off, 64);
        mx = o > mx ? o : mx;
    }
    __shared__ int64_t red[T256 / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = red[0];
#pragma unroll
    for (int i = 1; i < T256 / 64; ++i) mx = red[i] > mx ? red[i] : mx;
    __syncthreads();
    hub = block_sum_i64(hub);
    med = block_sum_i64(med);
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
// b holds *nb_d valid keys out of nb_bound; output slots past na + *nb_d get
// the sentinel, so the whole output stays sorted.
__global__ void merge_rank_kernel(const uint64_t *__restrict__ a, int64_t na,
                                  const uint64_t *__restrict__ b, const int64_t *__restrict__ nb_d,
                                  int64_t nb_bound, uint64_t sentinel,
                                  uint64_t *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nb = *nb_d;
    if (t < na) {
        const uint64_t x = a[t];
        int64_t lo = 0, hi = nb;
        while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            if (b[mid] < x) lo = mid + 1;
            else hi = mid;
        }
        out[t + lo] = x;
    } else if (t < na + nb_bound) {
        const int64_t j = t - na;
        if (j < nb) {
            const uint64_t x = b[j];
            int64_t lo = 0, hi = na;
            while (lo < hi) {
                const int64_t mid = lo + ((hi - lo) >> 1);
                if (a[mid] <= x) lo = mid + 1;
                else hi = mid;
            }
            out[j + lo] = x;
        } else {
            out[t] = sentinel;
        }
    }
}

inline unsigned grid1(int64_t n, int t = T256) { return (unsigned)ceil_div(n, t); }

ifgp_status copy_d2h_sync(void *h, const void *d, size_t bytes, hipStream_t s) {
    IFGP_HIP(hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, s));
    IFGP_HIP(hipStreamSynchronize(s));
    return IFGP_OK;
}

// Device counters of one build, read back by the single host synchronisation.
enum { C_LOOPS = 0, C_BAD, C_NNZ, C_MAXDEG, C_HUB, C_MED, C_COUNT };

// Keys of E pairs -> 2E keys; self-loop pairs and bad ids counted on the device.
ifgp_status ingest(const int64_t *src, const int64_t *dst, int64_t E, int64_t N, int B,
                   hipStream_t s, Buf &keys, int64_t *ctr) {
    IFGP_TRY(alloc(keys, sizeof(uint64_t) * 2 * E, s));
    if (E > 0) {
        ingest_kernel<<<grid1(E), T256, 0, s>>>(src, dst, E, N, B, keys.as<uint64_t>(),
                                                ctr + C_LOOPS);
        IFGP_LAUNCHED();
    }
    return IFGP_OK;
}

// n sorted keys (repeats and sentinels allowed) -> unique keys; the count goes
// to *nu_d on the device; uk is allocated for the upper bound n.
ifgp_status unique_keys(const uint64_t *k, int64_t n, int B, int64_t N, hipStream_t s, Buf &uk,
                        int64_t *nu_d) {
    IFGP_TRY(alloc(uk, sizeof(uint64_t) * n, s));
    const int64_t nb = ceil_div(n, UQ_TILE);
    Buf bc;
    IFGP_TRY(alloc(bc, sizeof(int64_t) * (nb + 1), s));
    if (n > 0) {
        unique_count_kernel<<<(unsigned)nb, T256, 0, s>>>(k, n, B, N, bc.as<int64_t>());
        IFGP_LAUNCHED();
    }
    IFGP_TRY(exclusive_scan<int64_t>(bc.as<int64_t>(), bc.as<int64_t>(), nb, nu_d, s));
    if (n > 0) {
        unique_write_kernel<<<(unsigned)nb, T256, 0, s>>>(k, n, B, N, bc.as<int64_t>(),
                                                          uk.as<uint64_t>());
        IFGP_LAUNCHED();
    }
    return IFGP_OK;
}

// Unique sorted keys (count on the device, at most bound) -> canonical CSR
// and plan.  The one host synchronisation of a build happens here.
ifgp_status csr_and_plan(const uint64_t *uk, int64_t bound, int B, int64_t N, hipStream_t s,
                         int64_t *ctr, GraphData &g) {
    g.N = N;
    IFGP_TRY(alloc(g.rowptr, sizeof(int64_t) * (N + 1), s));
    IFGP_TRY(alloc(g.colidx, sizeof(int32_t) * bound, s));
    IFGP_TRY(alloc(g.deg, sizeof(int32_t) * N, s));
    rowptr_kernel<<<grid1(N + 1), T256, 0, s>>>(uk, ctr + C_NNZ, B, N, g.rowptr.as<int64_t>());
    IFGP_LAUNCHED();
    if (bound > 0) {
        colidx_kernel<<<grid1(bound), T256, 0, s>>>(uk, ctr + C_NNZ, bound,
                                                    ((uint64_t)1 << B) - 1,
                                                    g.colidx.as<int32_t>());
        IFGP_LAUNCHED();
    }
    const unsigned dgrid = (unsigned)std::min<int64_t>(grid1(N), 1024);
    degree_kernel<<<dgrid, T256, 0, s>>>(g.rowptr.as<int64_t>(), N, g.deg.as<int32_t>(),
                                         ctr + C_MAXDEG);
    IFGP_LAUNCHED();
    int64_t h[C_COUNT];
    IFGP_TRY(copy_d2h_sync(h, ctr, sizeof(h), s));
    if (h[C_BAD]) {
        set_error("edge list holds a node id outside [0, %lld)", (long long)N);
        return IFGP_E_RANGE;
    }
    const int64_t nnz = h[C_NNZ];
    g.nnz = nnz;
    g.self_loops = h[C_LOOPS];
    g.max_deg = (int32_t)h[C_MAXDEG];
    g.n_hub = h[C_HUB];
    g.n_med = h[C_MED] - h[C_HUB];

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
    Buf ctr;
    IFGP_TRY(alloc(ctr, sizeof(int64_t) * C_COUNT, s));
    IFGP_TRY(fill_i64(ctr.as<int64_t>(), C_COUNT, 0, s));
    Buf keys;
    IFGP_TRY(ingest(src, dst, E, N, B, s, keys, ctr.as<int64_t>()));
    Buf tmp;
    IFGP_TRY(alloc(tmp, sizeof(uint64_t) * 2 * E, s));
    uint64_t *sorted = nullptr;
    IFGP_TRY(radix_sort_u64(keys.as<uint64_t>(), tmp.as<uint64_t>(), 2 * E, 2 * B, s, &sorted));
    Buf uk;
    IFGP_TRY(unique_keys(sorted, 2 * E, B, N, s, uk, ctr.as<int64_t>() + C_NNZ));
    keys.reset();
    tmp.reset();
    GraphData g;
    IFGP_TRY(csr_and_plan(uk.as<uint64_t>(), 2 * E, B, N, s, ctr.as<int64_t>(), g));
    g.dups = (E - g.self_loops) - g.nnz / 2;
    out = std::move(g);
    return IFGP_OK;
}

ifgp_status merge_graph_device(const GraphData &in, const int64_t *src, const int64_t *dst,
                               int64_t E, int64_t new_N, hipStream_t s, GraphData &out) {
    const int B = bit_width((uint64_t)new_N);
    Buf ctr, cinc;
    IFGP_TRY(alloc(ctr, sizeof(int64_t) * C_COUNT, s));
    IFGP_TRY(fill_i64(ctr.as<int64_t>(), C_COUNT, 0, s));
    IFGP_TRY(alloc(cinc, sizeof(int64_t), s));
    // increment: keys, sort, unique (count of unique increment keys in cinc)
    Buf keys;
    IFGP_TRY(ingest(src, dst, E, new_N, B, s, keys, ctr.as<int64_t>()));
    Buf tmp;
    IFGP_TRY(alloc(tmp, sizeof(uint64_t) * 2 * E, s));
    uint64_t *sorted = nullptr;
    IFGP_TRY(radix_sort_u64(keys.as<uint64_t>(), tmp.as<uint64_t>(), 2 * E, 2 * B, s, &sorted));
    Buf inc;
    IFGP_TRY(unique_keys(sorted, 2 * E, B, new_N, s, inc, cinc.as<int64_t>()));
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
    const int64_t nm = in.nnz + 2 * E;   // upper bound; unused slots hold the sentinel
    IFGP_TRY(alloc(merged, sizeof(uint64_t) * nm, s));
    if (nm > 0) {
        merge_rank_kernel<<<grid1(nm), T256, 0, s>>>(res.as<uint64_t>(), in.nnz,
                                                     inc.as<uint64_t>(), cinc.as<int64_t>(),
                                                     2 * E, (uint64_t)new_N << B,
                                                     merged.as<uint64_t>());
        IFGP_LAUNCHED();
    }
    res.reset();
    inc.reset();
    Buf uk;
    IFGP_TRY(unique_keys(merged.as<uint64_t>(), nm, B, new_N, s, uk, ctr.as<int64_t>() + C_NNZ));
    merged.reset();
    GraphData g;
    IFGP_TRY(csr_and_plan(uk.as<uint64_t>(), nm, B, new_N, s, ctr.as<int64_t>(), g));
    g.self_loops += in.self_loops;
    // pairs of this increment that added no new edge
    g.dups = in.dups + (E - (g.self_loops - in.self_loops)) - (g.nnz - in.nnz) / 2;
    out = std::move(g);
    return IFGP_OK;
}

}  // namespace ifgp
