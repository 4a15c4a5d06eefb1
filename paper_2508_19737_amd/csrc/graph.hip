// Graph construction on the device: the adjacency of Sec. II (undirected,
// unweighted, A in {0,1}) from an edge list, as a canonical CSR, plus the
// execution plan the hop kernel runs on.
//
//   ingest     validate ids, emit both orientations of every pair as a 64-bit
//              key (row << B) | col, self-loops as a sentinel past every row
//   bucket     stable LSD radix passes (primitives.hip) over the high bits of
//              the row only, so keys are grouped in buckets of 2^s rows
//   per bucket one block sorts the bucket by (row, col) in LDS, keeps the
//              first of each run of equal keys, drops sentinels, and writes
//              the survivors' columns and its rows' degrees
//   CSR        rowptr = prefix sum of the degrees
//   plan       node order by descending degree (ties by id) and the CSR
//              relabelled into it: the hop kernel then sees degree-homogeneous
//              waves, the heavy rows first, and the most gathered rows packed
//              together; the columns move to their CSR place in the same pass
//   merge      (stream_add) resident keys and increment keys merged by rank,
//              duplicates dropped, CSR and plan rebuilt
#include <algorithm>

#include "internal.h"
#include "wave_match.h"

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

// counters[0] = self-loop pairs, counters[1] = 1 if any id is out of range.
// Edge e's keys (edge_keys) go to keys[2e], keys[2e + 1] unless keys is null.
// Block t takes the RADIX_TILE / 2 edges whose keys form radix tile t; with
// hist != nullptr it also writes the tile's counts of the digit
// (key >> hist_shift) & 255 to hist[digit * ntiles + t] (the first pass of
// radix_sort_u64 or radix_sort_pairs).
constexpr int INGEST_EDGES = RADIX_TILE / 2;
__global__ __launch_bounds__(T256) void ingest_kernel(const int64_t *__restrict__ src,
                                                      const int64_t *__restrict__ dst, int64_t E,
                                                      int64_t N, int B,
                                                      uint64_t *__restrict__ keys,
                                                      int64_t *__restrict__ counters,
                                                      int64_t *__restrict__ hist, int hist_shift,
                                                      int64_t ntiles) {
    __shared__ int cnt[T256 / 64][256];
    const int tid = threadIdx.x, w = tid >> 6;
    if (hist) {
        for (int i = tid; i < (T256 / 64) * 256; i += T256) (&cnt[0][0])[i] = 0;
        __syncthreads();
    }
    int64_t loop = 0, bad = 0;
#pragma unroll 4
    for (int r = 0; r < INGEST_EDGES / T256; ++r) {
        const int64_t e = (int64_t)blockIdx.x * INGEST_EDGES + r * T256 + tid;
        if (e < E) {
            const int64_t u = src[e], v = dst[e];
            uint64_t k0, k1;
            edge_keys(u, v, N, B, k0, k1);
            if (u < 0 || u >= N || v < 0 || v >= N) bad = 1;
            else if (u == v) ++loop;
            if (keys) {
                keys[2 * e] = k0;
                keys[2 * e + 1] = k1;
            }
            if (hist) {
                atomicAdd(&cnt[w][(unsigned)(k0 >> hist_shift) & 255u], 1);
                atomicAdd(&cnt[w][(unsigned)(k1 >> hist_shift) & 255u], 1);
            }
        }
    }
    if (hist) {
        __syncthreads();
        int t = 0;
#pragma unroll
        for (int ww = 0; ww < T256 / 64; ++ww) t += cnt[ww][tid];
        hist[(int64_t)tid * ntiles + blockIdx.x] = t;
    }
    loop = block_sum_i64(loop);
    bad = block_sum_i64(bad);
    if (threadIdx.x == 0) {
        if (loop) atomicAdd((unsigned long long *)&counters[0], (unsigned long long)loop);
        if (bad) atomicOr((unsigned long long *)&counters[1], 1ull);
    }
}

// key = (top - deg) << B | node with top >= every degree: ascending key =
// descending degree, ties by id
__global__ void order_keys_kernel(const int32_t *__restrict__ deg, int64_t N, int32_t top, int B,
                                  uint64_t *__restrict__ keys) {
    const int64_t i = block_index() * blockDim.x + threadIdx.x;
    if (i < N) keys[i] = ((uint64_t)(top - deg[i]) << B) | (uint64_t)i;
}

__global__ void perm_kernel(const uint64_t *__restrict__ keys, int64_t N, uint64_t mask,
                            const int32_t *__restrict__ deg, int32_t *__restrict__ perm,
                            int32_t *__restrict__ iperm, int32_t *__restrict__ ideg) {
    const int64_t k = block_index() * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int32_t node = (int32_t)(keys[k] & mask);
    perm[k] = node;
    iperm[node] = (int32_t)k;
    ideg[k] = deg[node];
}

// keys of a canonical CSR, packed with B bits per id: (row << B) | col
__global__ __launch_bounds__(T256) void csr_keys_kernel(const int64_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ colidx,
                                                        int64_t N, int B,
                                                        uint64_t *__restrict__ keys) {
    const int64_t r = block_index() * (T256 / 16) + (threadIdx.x >> 4);
    const int l = threadIdx.x & 15;
    if (r >= N) return;
    for (int64_t t = rowptr[r] + l; t < rowptr[r + 1]; t += 16)
        keys[t] = ((uint64_t)r << B) | (uint64_t)(uint32_t)colidx[t];
}

// ---------------------------------------------------------------- bucketed build
// A fresh build sorts the keys only by the high bits of their row (bucket =
// row >> s, 2^s consecutive rows per bucket), which takes few device-wide
// radix passes; one block then sorts, deduplicates and counts each bucket.
// Inside a bucket a key is ((row mod 2^s) << B) | col, which fits 32 bits.
constexpr int BK_THREADS = 512;               // bucket_csr_kernel: three blocks per CU
constexpr int BK_KPL = 16;                    // keys per lane in one LDS pass
constexpr int BK_CAP = BK_THREADS * BK_KPL;   // largest bucket of bucket_csr_kernel
constexpr int BK_BIG_THREADS = 1024;          // bucket_big_kernel: one block per CU
constexpr int BK_BIG_KPL = 24;
constexpr int BK_SMAX = 9;                    // at most 512 rows per bucket
constexpr int BK_BINS = 256;
constexpr uint32_t BK_NONE = 0xFFFFFFFFu;     // self loop or bad id; above every real key
constexpr int64_t BK_BIG_BLOCKS = 64;         // blocks striding over the oversized buckets

template <int THREADS, int KPL>
struct BucketLds {
    static_assert(THREADS >= BK_BINS && THREADS % 64 == 0, "one thread per digit");
    static constexpr int threads = THREADS, waves = THREADS / 64, kpl = KPL, cap = THREADS * KPL;
    uint32_t a[cap];
    int cnt[waves][BK_BINS];
    int dstart[BK_BINS + 1];
    int wsum[waves];
    int64_t gpos[BK_BINS];
    int64_t wsum64[BK_BINS / 64];
    int64_t rstart[1 << BK_SMAX];
    int64_t rend[1 << BK_SMAX];
    int64_t red[3][waves];
};

// Stable in-place sort of sh.a[0, rounds * threads) by the digit
// (a >> shift) & 255 (callers pad with BK_NONE, which sorts last).  Keys
// other than BK_NONE are below 2^top, so where top - shift < 8 the digits
// are told apart by their low top - shift + 1 bits (BK_NONE's bit
// top - shift is set, every other key's clear).  Wave w ranks the keys at
// [w*rounds*64, (w+1)*rounds*64), so key order is (wave, round, lane).  On
// return sh.dstart[g] is where digit g starts (sh.dstart[256] = rounds *
// threads).  Begins and ends with a block barrier; all lanes active.
template <typename Lds>
__device__ __forceinline__ void lds_digit_pass(Lds &sh, int rounds, int shift, int top) {
    const int bits = top - shift < 8 ? top - shift + 1 : 8;
    constexpr int KPL = Lds::kpl;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int base = w * rounds * 64 + lane;
    const uint64_t lt = __lanemask_lt();
    for (int i = lane; i < BK_BINS; i += 64) sh.cnt[w][i] = 0;
    __syncthreads();
    uint32_t key[KPL];
    uint32_t rank2[KPL / 2];  // two 16-bit ranks per register (ranks < cap)
    static_assert(Lds::cap <= 65536 && KPL % 2 == 0, "ranks are packed in 16 bits");
#pragma unroll
    for (int r = 0; r < KPL; ++r) key[r] = r < rounds ? sh.a[base + r * 64] : 0;
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        if (r % 2 == 0) rank2[r / 2] = 0;
        if (r < rounds) {  // uniform over the block
            const unsigned g = (key[r] >> shift) & (BK_BINS - 1);
            const uint64_t m = match_digit8(g, true, bits);
            const int below = __popcll(m & lt);
            const int c = sh.cnt[w][g];
            // the leader's write follows every lane's read of this wave
            if (below == 0) sh.cnt[w][g] = c + __popcll(m);
            rank2[r / 2] |= (uint32_t)(c + below) << (16 * (r % 2));
        }
    }
    __syncthreads();
    int total = 0, inc = 0;
    if (tid < BK_BINS) {
        for (int ww = 0; ww < Lds::waves; ++ww) {
            const int t = sh.cnt[ww][tid];
            sh.cnt[ww][tid] = total;
            total += t;
        }
        inc = total;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(inc, off, 64);
            if (lane >= off) inc += t;
        }
        if (lane == 63) sh.wsum[w] = inc;
    }
    __syncthreads();
    if (tid < BK_BINS) {
        int woff = 0;
        for (int ww = 0; ww < w; ++ww) woff += sh.wsum[ww];
        sh.dstart[tid] = woff + inc - total;
    }
    if (tid == 0) sh.dstart[BK_BINS] = rounds * Lds::threads;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        if (r < rounds) {
            const unsigned g = (key[r] >> shift) & (BK_BINS - 1);
            const int rank = (rank2[r / 2] >> (16 * (r % 2))) & 0xFFFF;
            sh.a[sh.dstart[g] + sh.cnt[w][g] + rank] = key[r];
        }
    }
    __syncthreads();
}

// Exclusive scan of sh.gpos[0, 256) in place (every thread calls it).
template <typename Lds>
__device__ __forceinline__ void scan_gpos(Lds &sh) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int64_t v = 0, inc = 0;
    if (tid < BK_BINS) {
        v = sh.gpos[tid];
        inc = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t t = __shfl_up(inc, off, 64);
            if (lane >= off) inc += t;
        }
        if (lane == 63) sh.wsum64[w] = inc;
    }
    __syncthreads();
    if (tid < BK_BINS) {
        int64_t woff = 0;
        for (int ww = 0; ww < w; ++ww) woff += sh.wsum64[ww];
        sh.gpos[tid] = woff + inc - v;
    }
    __syncthreads();
}

// Survivors of the sorted local keys src[0, n) (LDS or global): the first of
// each run of equal keys, sentinels dropped.  They go to out[] in order, as
// local keys (row in the bucket << B | column); row r of the bucket owns
// survivors [rstart[r], rend[r]).  Every thread calls it.
template <typename Lds, typename P>
__device__ __forceinline__ void bucket_survivors(Lds &sh, P src, int64_t n, int B,
                                                 uint32_t *__restrict__ out) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t lt = __lanemask_lt();
    int64_t kept = 0;
    for (int64_t c = 0; c < n; c += Lds::threads) {
        const int64_t i = c + tid;
        uint32_t k = BK_NONE, prev = BK_NONE, next = BK_NONE;
        if (i < n) {
            k = src[i];
            if (i > 0) prev = src[i - 1];
            if (i + 1 < n) next = src[i + 1];
        }
        const bool valid = k != BK_NONE;
        const bool keep = valid && (i == 0 || prev != k);
        const uint32_t row = valid ? k >> B : 0;
        const bool first = valid && (i == 0 || (prev >> B) != row);
        const bool last = valid && (next == BK_NONE || (next >> B) != row);
        const uint64_t m = __ballot(keep);
        if (lane == 0) sh.wsum[w] = __popcll(m);
        __syncthreads();
        int before = 0, total = 0;
        for (int ww = 0; ww < Lds::waves; ++ww) {
            before += ww < w ? sh.wsum[ww] : 0;
            total += sh.wsum[ww];
        }
        const int64_t pos = kept + before + __popcll(m & lt);
        if (keep) out[pos] = k;
        if (first) sh.rstart[row] = pos;
        if (last) sh.rend[row] = pos + (keep ? 1 : 0);
        kept += total;
        __syncthreads();
    }
}

// bstart[b] = first key of bucket b (keys sorted by row >> s); bstart[nbk] = n.
__global__ void bucket_bounds_kernel(const uint64_t *__restrict__ keys, int64_t n, int B, int s,
                                     int64_t nbk, int64_t *__restrict__ bstart) {
    const int64_t b = block_index() * blockDim.x + threadIdx.x;
    if (b > nbk) return;
    if (b == nbk) {
        bstart[b] = n;
        return;
    }
    const uint64_t target = ((uint64_t)b << s) << B;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (keys[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    bstart[b] = lo;
}

__device__ __forceinline__ uint32_t local_key(uint64_t k, int64_t N, int B, int s) {
    const int64_t row = (int64_t)(k >> B);
    return row >= N ? BK_NONE
                    : (uint32_t)((((uint64_t)row & (((uint64_t)1 << s) - 1)) << B) |
                                 (k & (((uint64_t)1 << B) - 1)));
}

// Degrees of bucket b's rows from sh.rstart/rend, and the block's part of
// the statistics: the largest degree and the counts of hub and medium rows
// (summed into stats[0..2] by atomics).  Every thread calls it.
template <typename Lds>
__device__ __forceinline__ void bucket_degrees(Lds &sh, int64_t b, int s, int64_t N,
                                               int32_t *__restrict__ deg,
                                               int64_t *__restrict__ stats) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int64_t mx = 0, hub = 0, med = 0;
    for (int r = tid; r < (1 << s); r += Lds::threads) {
        const int64_t node = (b << s) + r;
        if (node < N) {
            const int64_t d = sh.rend[r] - sh.rstart[r];
            deg[node] = (int32_t)d;
            mx = d > mx ? d : mx;
            hub += d >= HUB_DEGREE;
            med += d >= MED_DEGREE;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t o = __shfl_xor(mx, off, 64);
        mx = o > mx ? o : mx;
        hub += __shfl_xor(hub, off, 64);
        med += __shfl_xor(med, off, 64);
    }
    if (lane == 0) {
        sh.red[0][w] = mx;
        sh.red[1][w] = hub;
        sh.red[2][w] = med;
    }
    __syncthreads();
    if (tid == 0) {
        for (int ww = 1; ww < Lds::waves; ++ww) {
            mx = sh.red[0][ww] > mx ? sh.red[0][ww] : mx;
            hub += sh.red[1][ww];
            med += sh.red[2][ww];
        }
        if (mx) atomicMax((unsigned long long *)&stats[0], (unsigned long long)mx);
        if (hub) atomicAdd((unsigned long long *)&stats[1], (unsigned long long)hub);
        if (med) atomicAdd((unsigned long long *)&stats[2], (unsigned long long)med);
    }
}

// Buckets with more than BK_CAP keys, appended to big[] (in no particular
// order: each is handled on its own).  *nbig counts them.
__global__ void bucket_big_list_kernel(const int64_t *__restrict__ bstart, int64_t nbk,
                                       int64_t *__restrict__ big, int64_t *__restrict__ nbig) {
    const int64_t b = block_index() * blockDim.x + threadIdx.x;
    if (b < nbk && bstart[b + 1] - bstart[b] > BK_CAP)
        big[atomicAdd((unsigned long long *)nbig, 1ull)] = b;
}

// One block per bucket of at most BK_CAP keys (larger ones are left to
// bucket_big_kernel): sort its keys by (row, col) in LDS, drop repeats and
// self loops, write the survivors' local keys to tcol[bstart[b] ...] in order
// and the degrees of the bucket's rows.
__global__ __launch_bounds__(BK_THREADS) __attribute__((amdgpu_waves_per_eu(6))) void bucket_csr_kernel(
    const uint64_t *__restrict__ keys, const int64_t *__restrict__ bstart, int64_t N, int B,
    int s, int64_t nbk, uint32_t *__restrict__ tcol, int32_t *__restrict__ deg,
    int64_t *__restrict__ stats) {
    __shared__ BucketLds<BK_THREADS, BK_KPL> sh;
    const int tid = threadIdx.x;
    const int64_t b = block_index();
    if (b >= nbk) return;
    const int64_t bs = bstart[b], n64 = bstart[b + 1] - bs;
    if (n64 > BK_CAP) return;
    const int n = (int)n64;
    for (int r = tid; r < (1 << s); r += BK_THREADS) {
        sh.rstart[r] = 0;
        sh.rend[r] = 0;
    }
    const int rounds = (n + BK_THREADS - 1) / BK_THREADS;  // padded with BK_NONE
    constexpr int H = BK_KPL / 2;  // two batches of independent loads
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        uint64_t k[H];
#pragma unroll
        for (int r = 0; r < H; ++r) {
            const int i = (h * H + r) * BK_THREADS + tid;
            k[r] = i < n ? keys[bs + i] : 0;
        }
#pragma unroll
        for (int r = 0; r < H; ++r) {
            const int i = (h * H + r) * BK_THREADS + tid;
            if (h * H + r < rounds) sh.a[i] = i < n ? local_key(k[r], N, B, s) : BK_NONE;
        }
    }
    if (rounds > 0)
        for (int shift = 0; shift < s + B; shift += 8) lds_digit_pass(sh, rounds, shift, s + B);
    bucket_survivors(sh, sh.a, n, B, tcol + bs);
    bucket_degrees(sh, b, s, N, deg, stats);
}

// The buckets listed in big[0, *nbig), a few blocks striding over the list,
// one block per CU with most of its LDS: a bucket that fits that LDS
// is handled as in bucket_csr_kernel; a larger one is sorted chunk by chunk
// through global memory, in its own range of `scratch` (8 bytes per key:
// room for two 32-bit copies).
__global__ __launch_bounds__(BK_BIG_THREADS) void bucket_big_kernel(
    const uint64_t *__restrict__ keys, uint64_t *__restrict__ scratch,
    const int64_t *__restrict__ bstart, const int64_t *__restrict__ big,
    const int64_t *__restrict__ nbig, int64_t N, int B, int s, uint32_t *__restrict__ tcol,
    int32_t *__restrict__ deg, int64_t *__restrict__ stats) {
    using Lds = BucketLds<BK_BIG_THREADS, BK_BIG_KPL>;
    __shared__ Lds sh;
    constexpr int CAP = Lds::cap, T = Lds::threads;
    const int tid = threadIdx.x;
    const int64_t count = *nbig;
    for (int64_t q = blockIdx.x; q < count; q += gridDim.x) {
        const int64_t b = big[q];
        const int64_t bs = bstart[b], n = bstart[b + 1] - bs;
        for (int r = tid; r < (1 << s); r += T) {
            sh.rstart[r] = 0;
            sh.rend[r] = 0;
        }
        if (n <= CAP) {  // wholly in LDS
            const int rounds = (int)((n + T - 1) / T);
            for (int i = tid; i < rounds * T; i += T)
                sh.a[i] = i < n ? local_key(keys[bs + i], N, B, s) : BK_NONE;
            for (int shift = 0; shift < s + B; shift += 8) lds_digit_pass(sh, rounds, shift, s + B);
            bucket_survivors(sh, sh.a, n, B, tcol + bs);
            bucket_degrees(sh, b, s, N, deg, stats);
            __syncthreads();
            continue;
        }
        uint32_t *x = reinterpret_cast<uint32_t *>(scratch + bs), *y = x + n;
        for (int64_t i = tid; i < n; i += T) x[i] = local_key(keys[bs + i], N, B, s);
        for (int shift = 0; shift < s + B; shift += 8) {
            for (int i = tid; i < BK_BINS; i += T) sh.gpos[i] = 0;
            __syncthreads();
            for (int64_t i = tid; i < n; i += T)
                atomicAdd((unsigned long long *)&sh.gpos[(x[i] >> shift) & (BK_BINS - 1)], 1ull);
            __syncthreads();
            scan_gpos(sh);
            for (int64_t c0 = 0; c0 < n; c0 += CAP) {
                const int m = (int)(n - c0 < CAP ? n - c0 : CAP);
                const int rounds = (m + T - 1) / T, pad = rounds * T - m;
                // padding (BK_NONE, digit 255) sorts after every key of the chunk
                for (int i = tid; i < rounds * T; i += T)
                    sh.a[i] = i < m ? x[c0 + i] : BK_NONE;
                lds_digit_pass(sh, rounds, shift, s + B);
                for (int i = tid; i < m; i += T) {
                    const uint32_t k = sh.a[i];
                    const unsigned g = (k >> shift) & (BK_BINS - 1);
                    y[sh.gpos[g] + (i - sh.dstart[g])] = k;
                }
                __syncthreads();
                if (tid < BK_BINS)
                    sh.gpos[tid] += sh.dstart[tid + 1] - sh.dstart[tid] - (tid == BK_BINS - 1 ? pad : 0);
                __syncthreads();
            }
            uint32_t *t = x;
            x = y;
            y = t;
        }
        __syncthreads();
        bucket_survivors(sh, x, n, B, tcol + bs);
        bucket_degrees(sh, b, s, N, deg, stats);
        __syncthreads();
    }
}

// One block per bucket, after the plan: each survivor (local key: row in the
// bucket << B | column, in row order) is placed in the relabelled CSR: entry q
// of row i goes to irowptr[iperm[i]] + q, column iperm[j].
constexpr int FN_THREADS = 256;
constexpr int FN_ITEMS = 8;  // entries per thread in flight
__global__ __launch_bounds__(FN_THREADS) void bucket_finish_kernel(
    const uint32_t *__restrict__ tcol, const int64_t *__restrict__ bstart,
    const int64_t *__restrict__ rowptr, const int32_t *__restrict__ iperm,
    const int64_t *__restrict__ irowptr, int64_t N, int B, int s,
    int32_t *__restrict__ icolidx) {
    __shared__ int64_t dst[1 << BK_SMAX];  // per row: its first place minus its first entry
    const int64_t b = block_index(), r0 = b << s;
    if (r0 >= N) return;  // also every block past the last bucket
    const int nr = (int)((N - r0) < ((int64_t)1 << s) ? (N - r0) : ((int64_t)1 << s));
    const int64_t p0 = rowptr[r0], cnt = rowptr[r0 + nr] - p0;
    for (int r = threadIdx.x; r < nr; r += FN_THREADS)
        dst[r] = irowptr[iperm[r0 + r]] - (rowptr[r0 + r] - p0);
    __syncthreads();
    const uint32_t *src = tcol + bstart[b];
    const uint32_t cmask = (1u << B) - 1u;
    for (int64_t q0 = 0; q0 < cnt; q0 += FN_THREADS * FN_ITEMS) {
        uint32_t k[FN_ITEMS];
        int32_t v[FN_ITEMS];
#pragma unroll
        for (int it = 0; it < FN_ITEMS; ++it) {
            const int64_t q = q0 + it * FN_THREADS + threadIdx.x;
            k[it] = q < cnt ? src[q] : 0u;
        }
#pragma unroll
        for (int it = 0; it < FN_ITEMS; ++it) {
            const int64_t q = q0 + it * FN_THREADS + threadIdx.x;
            if (q < cnt) v[it] = iperm[k[it] & cmask];
        }
#pragma unroll
        for (int it = 0; it < FN_ITEMS; ++it) {
            const int64_t q = q0 + it * FN_THREADS + threadIdx.x;
            if (q < cnt) icolidx[dst[k[it] >> B] + q] = v[it];
        }
    }
}

// The canonical colidx from a build's survivors (one block per bucket): the
// bucket's entries, in row order, from tcol[bstart[b] ...] to
// colidx[rowptr[b << s] ...], columns only.
__global__ void canonical_colidx_kernel(const uint32_t *__restrict__ tcol,
                                        const int64_t *__restrict__ bstart,
                                        const int64_t *__restrict__ rowptr, int64_t N, int B,
                                        int s, int32_t *__restrict__ colidx) {
    const int64_t b = block_index(), r0 = b << s;
    if (r0 >= N) return;
    const int64_t r1 = (N - r0) < ((int64_t)1 << s) ? N : r0 + ((int64_t)1 << s);
    const int64_t p0 = rowptr[r0], cnt = rowptr[r1] - p0;
    const uint32_t *src = tcol + bstart[b];
    const uint32_t cmask = (1u << B) - 1u;
    for (int64_t q = threadIdx.x; q < cnt; q += blockDim.x) colidx[p0 + q] = (int32_t)(src[q] & cmask);
}

inline dim3 grid1(int64_t n, int t = T256) { return grid_for(ceil_div(n, t)); }

ifgp_status copy_d2h_sync(void *h, const void *d, size_t bytes, hipStream_t s) {
    IFGP_HIP(hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, s));
    IFGP_HIP(hipStreamSynchronize(s));
    return IFGP_OK;
}

// Device counters of one build, read back by the single host synchronisation.
enum { C_LOOPS = 0, C_BAD, C_NNZ, C_MAXDEG, C_HUB, C_MED, C_COUNT };

// Page-locked host slots for the counters, one set per host thread (kept for
// the thread's life), so that their copy is asynchronous.
ifgp_status pinned_counters(int64_t **out) {
    thread_local int64_t *slots = nullptr;
    if (!slots) IFGP_HIP(hipHostMalloc((void **)&slots, sizeof(int64_t) * C_COUNT, 0));
    *out = slots;
    return IFGP_OK;
}

// Keys of E pairs -> 2E keys at keys[0, 2E) (none written if keys is null);
// self-loop pairs and bad ids counted on the device; with hist, the first
// radix pass's tile counts of the digit at hist_shift (see ingest_kernel).
ifgp_status ingest_to(const int64_t *src, const int64_t *dst, int64_t E, int64_t N, int B,
                      hipStream_t s, uint64_t *keys, int64_t *ctr, int64_t *hist = nullptr,
                      int hist_shift = 0) {
    if (E > 0) {
        const int64_t ntiles = ceil_div(2 * E, (int64_t)RADIX_TILE);
        ingest_kernel<<<(unsigned)ceil_div(E, (int64_t)INGEST_EDGES), T256, 0, s>>>(
            src, dst, E, N, B, keys, ctr + C_LOOPS, hist, hist_shift, ntiles);
        IFGP_LAUNCHED();
    }
    return IFGP_OK;
}

// Counters (host copy) -> GraphData fields.
ifgp_status apply_counters(const int64_t *h, int64_t N, GraphData &g) {
    if (h[C_BAD]) {
        set_error("edge list holds a node id outside [0, %lld)", (long long)N);
        return IFGP_E_RANGE;
    }
    g.nnz = h[C_NNZ];
    g.self_loops = h[C_LOOPS];
    g.max_deg = (int32_t)h[C_MAXDEG];
    g.n_hub = h[C_HUB];
    g.n_med = h[C_MED] - h[C_HUB];
    return IFGP_OK;
}

// The one host synchronisation of a build: counters -> GraphData fields.
ifgp_status read_counters(const int64_t *ctr, int64_t N, hipStream_t s, GraphData &g) {
    int64_t h[C_COUNT];
    IFGP_TRY(copy_d2h_sync(h, ctr, sizeof(h), s));
    return apply_counters(h, N, g);
}

// Node order by descending degree (ties by id): perm, iperm and the
// relabelled row pointers irowptr.  Degrees are below 2^dbits.  The keys
// (2^dbits - 1 - deg) << B | node start in id order, so a stable sort of
// the degree bits alone leaves equal degrees in id order.
ifgp_status plan_order(int B, int dbits, hipStream_t s, GraphData &g) {
    const int64_t N = g.N;
    Buf ka, kb;
    IFGP_TRY(alloc(ka, sizeof(uint64_t) * N, s));
    IFGP_TRY(alloc(kb, sizeof(uint64_t) * N, s));
    order_keys_kernel<<<grid1(N), T256, 0, s>>>(g.deg.as<int32_t>(), N,
                                                (int32_t)(((int64_t)1 << dbits) - 1), B,
                                                ka.as<uint64_t>());
    IFGP_LAUNCHED();
    uint64_t *sorted = nullptr;
    IFGP_TRY(radix_sort_u64(ka.as<uint64_t>(), kb.as<uint64_t>(), N, B, B + dbits, s, &sorted));
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
    return IFGP_OK;
}

// Rows per bucket of a fresh build: 2^s, with s as large as the 32-bit
// local key and the row tables allow while the average bucket stays at half
// of what one block sorts in LDS.
int bucket_bits(int64_t N, int64_t nkeys, int B) {
    int s = std::min(std::min(BK_SMAX, B), 32 - B);
    while (s > 0 && (double)nkeys * (double)((int64_t)1 << s) > (BK_CAP / 2) * (double)N) --s;
    return s;
}

}  // namespace

namespace {

// The bucketed build from n keys (row << B | column, sentinel row N allowed)
// sorted by the rows' high bits (rows per bucket 2^sb) into one of the two
// n-key buffers keys and tmp (`sorted`; the other is scratch); ctr holds what
// the keys' making counted (self loops, bad ids).  Buckets sorted,
// deduplicated and counted in LDS; rowptr, counters, plan, relabelled CSR.
ifgp_status bucket_build(Buf &keys, Buf &tmp, uint64_t *sorted, int64_t n, int64_t N, int B,
                         int sb, Buf &ctr, hipStream_t s, hipStream_t aux, hipEvent_t ev_fork,
                         hipEvent_t ev_join, GraphData &g) {
    uint64_t *other = sorted == keys.as<uint64_t>() ? tmp.as<uint64_t>() : keys.as<uint64_t>();
    const int64_t nbk = (N >> sb) + 1;
    g.N = N;
    Buf &bst = g.bst, &tcol = g.tcol;
    IFGP_TRY(alloc(bst, sizeof(int64_t) * (nbk + 1), s));
    IFGP_TRY(alloc(tcol, sizeof(uint32_t) * n, s));
    g.tcol_B = B;
    g.tcol_s = sb;
    IFGP_TRY(alloc(g.deg, sizeof(int32_t) * N, s));
    bucket_bounds_kernel<<<grid1(nbk + 1), T256, 0, s>>>(sorted, n, B, sb, nbk,
                                                          bst.as<int64_t>());
    IFGP_LAUNCHED();
    Buf big;
    IFGP_TRY(alloc(big, sizeof(int64_t) * (nbk + 1), s));
    int64_t *nbig = big.as<int64_t>() + nbk;
    IFGP_TRY(fill_i64(nbig, 1, 0, s));
    bucket_big_list_kernel<<<grid1(nbk), T256, 0, s>>>(bst.as<int64_t>(), nbk, big.as<int64_t>(),
                                                        nbig);
    IFGP_LAUNCHED();
    // The few oversized buckets take long on one block each.  They go first,
    // on the caller's stream, and the many small buckets beside them on the
    // side stream, so that the long blocks are placed before the short ones
    // fill the device.
    const bool side = aux != nullptr;
    if (side) {
        IFGP_HIP(hipEventRecord(ev_fork, s));
        IFGP_HIP(hipStreamWaitEvent(aux, ev_fork, 0));
    }
    bucket_big_kernel<<<(unsigned)BK_BIG_BLOCKS, BK_BIG_THREADS, 0, s>>>(
        sorted, other, bst.as<int64_t>(), big.as<int64_t>(), nbig, N, B, sb, tcol.as<uint32_t>(),
        g.deg.as<int32_t>(), ctr.as<int64_t>() + C_MAXDEG);
    hipError_t le = hipGetLastError();
    if (le == hipSuccess) {
        bucket_csr_kernel<<<grid_for(nbk), BK_THREADS, 0, side ? aux : s>>>(
            sorted, bst.as<int64_t>(), N, B, sb, nbk, tcol.as<uint32_t>(), g.deg.as<int32_t>(),
            ctr.as<int64_t>() + C_MAXDEG);
        le = hipGetLastError();
    }
    if (side) {  // joined before anything can return, so no buffer is released early
        IFGP_HIP(hipEventRecord(ev_join, aux));
        IFGP_HIP(hipStreamWaitEvent(s, ev_join, 0));
    }
    IFGP_HIP(le);
    keys.reset();
    tmp.reset();
    IFGP_TRY(alloc(g.rowptr, sizeof(int64_t) * (N + 1), s));
    IFGP_TRY(exclusive_scan<int32_t>(g.deg.as<int32_t>(), g.rowptr.as<int64_t>(), N,
                                     g.rowptr.as<int64_t>() + N, s));
    IFGP_HIP(hipMemcpyAsync(ctr.as<int64_t>() + C_NNZ, g.rowptr.as<int64_t>() + N,
                            sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    if (ev_fork) {
        // The plan needs only the degrees: it is queued before the host waits
        // for the counters (with a degree bound), so the device keeps working
        // while the host reads them.
        int64_t *hc = nullptr;
        IFGP_TRY(pinned_counters(&hc));
        IFGP_HIP(hipMemcpyAsync(hc, ctr.as<int64_t>(), sizeof(int64_t) * C_COUNT,
                                hipMemcpyDeviceToHost, s));
        IFGP_HIP(hipEventRecord(ev_fork, s));
        IFGP_TRY(plan_order(B, bit_width((uint64_t)std::min<int64_t>(N - 1, n)), s, g));
        IFGP_HIP(hipEventSynchronize(ev_fork));
        IFGP_TRY(apply_counters(hc, N, g));
    } else {
        IFGP_TRY(read_counters(ctr.as<int64_t>(), N, s, g));
        IFGP_TRY(plan_order(B, bit_width((uint64_t)g.max_deg), s, g));
    }
    // the canonical colidx waits for its first use (ensure_colidx); the
    // survivors stay in g.tcol until then
    IFGP_TRY(alloc(g.icolidx, sizeof(int32_t) * g.nnz, s));
    if (g.nnz > 0) {
        bucket_finish_kernel<<<grid_for(nbk), FN_THREADS, 0, s>>>(
            tcol.as<uint32_t>(), bst.as<int64_t>(), g.rowptr.as<int64_t>(), g.iperm.as<int32_t>(),
            g.irowptr.as<int64_t>(), N, B, sb, g.icolidx.as<int32_t>());
        IFGP_LAUNCHED();
    }
    return IFGP_OK;
}

}  // namespace

ifgp_status build_graph_device(const int64_t *src, const int64_t *dst, int64_t E, int64_t N,
                               hipStream_t s, hipStream_t aux, hipEvent_t ev_fork,
                               hipEvent_t ev_join, GraphData &out) {
    const int B = bit_width((uint64_t)N);  // holds 0..N (N is the sentinel row)
    Buf ctr;
    IFGP_TRY(alloc(ctr, sizeof(int64_t) * C_COUNT, s));
    IFGP_TRY(fill_i64(ctr.as<int64_t>(), C_COUNT, 0, s));
    const int64_t n = 2 * E;
    const int sb = bucket_bits(N, n, B);
    Buf keys, tmp;
    IFGP_TRY(alloc(keys, sizeof(uint64_t) * n, s));
    IFGP_TRY(alloc(tmp, sizeof(uint64_t) * n, s));
    uint64_t *sorted = keys.as<uint64_t>();
    if (B + sb < 2 * B && n > 1) {
        // the first radix pass's histogram taken from the edge lists (ids
        // checked, loops counted), and the pass itself making the keys from
        // them: no key array is written and read back in between
        Buf hist;
        IFGP_TRY(alloc(hist, sizeof(int64_t) * 256 * ceil_div(n, (int64_t)RADIX_TILE), s));
        IFGP_TRY(ingest_to(src, dst, E, N, B, s, nullptr, ctr.as<int64_t>(), hist.as<int64_t>(),
                           B + sb));
        IFGP_TRY(radix_sort_pairs(src, dst, E, N, B, keys.as<uint64_t>(), tmp.as<uint64_t>(),
                                  B + sb, 2 * B, s, &sorted, hist.as<int64_t>()));
    } else {
        IFGP_TRY(ingest_to(src, dst, E, N, B, s, keys.as<uint64_t>(), ctr.as<int64_t>()));
    }
    GraphData g;
    IFGP_TRY(bucket_build(keys, tmp, sorted, n, N, B, sb, ctr, s, aux, ev_fork, ev_join, g));
    g.dups = (E - g.self_loops) - g.nnz / 2;
    out = std::move(g);
    return IFGP_OK;
}

ifgp_status ensure_colidx(GraphData &g, hipStream_t s) {
    if (!g.tcol.p) return IFGP_OK;
    Buf colidx;
    IFGP_TRY(alloc(colidx, sizeof(int32_t) * g.nnz, s));
    if (g.nnz > 0) {
        canonical_colidx_kernel<<<grid_for((g.N >> g.tcol_s) + 1), T256, 0, s>>>(
            g.tcol.as<uint32_t>(), g.bst.as<int64_t>(), g.rowptr.as<int64_t>(), g.N, g.tcol_B,
            g.tcol_s, colidx.as<int32_t>());
        IFGP_LAUNCHED();
    }
    g.colidx = std::move(colidx);
    g.tcol.s = s;  // released after the kernel above, on its stream
    g.bst.s = s;
    g.tcol.reset();
    g.bst.reset();
    return IFGP_OK;
}

ifgp_status merge_graph_device(const GraphData &in, const int64_t *src, const int64_t *dst,
                               int64_t E, int64_t new_N, hipStream_t s, GraphData &out) {
    const int B = bit_width((uint64_t)new_N);
    Buf ctr;
    IFGP_TRY(alloc(ctr, sizeof(int64_t) * C_COUNT, s));
    IFGP_TRY(fill_i64(ctr.as<int64_t>(), C_COUNT, 0, s));
    // the resident entries (repacked with B bits) and the increment's keys in
    // one array, then the bucketed build as for a fresh graph: repeats of
    // resident edges are dropped with the other duplicates
    const int64_t n = in.nnz + 2 * E;
    const int sb = bucket_bits(new_N, n, B);
    Buf keys;
    IFGP_TRY(alloc(keys, sizeof(uint64_t) * n, s));
    if (in.N > 0 && in.nnz > 0) {
        csr_keys_kernel<<<grid1(in.N, 16), T256, 0, s>>>(in.rowptr.as<int64_t>(),
                                                         in.colidx.as<int32_t>(), in.N, B,
                                                         keys.as<uint64_t>());
        IFGP_LAUNCHED();
    }
    IFGP_TRY(ingest_to(src, dst, E, new_N, B, s, keys.as<uint64_t>() + in.nnz, ctr.as<int64_t>()));
    Buf tmp;
    IFGP_TRY(alloc(tmp, sizeof(uint64_t) * n, s));
    uint64_t *sorted = nullptr;
    IFGP_TRY(radix_sort_u64(keys.as<uint64_t>(), tmp.as<uint64_t>(), n, B + sb, 2 * B, s, &sorted));
    GraphData g;
    IFGP_TRY(bucket_build(keys, tmp, sorted, n, new_N, B, sb, ctr, s, nullptr, nullptr, nullptr, g));
    g.self_loops += in.self_loops;
    // pairs of this increment that added no new edge
    g.dups = in.dups + (E - (g.self_loops - in.self_loops)) - (g.nnz - in.nnz) / 2;
    out = std::move(g);
    return IFGP_OK;
}

}  // namespace ifgp
