// Device-wide building blocks for the graph build: exclusive prefix sums and
// a stable least-significant-digit radix sort of 64-bit keys.
//
// Both are written for wave64: block = 4 waves of 64 lanes; the radix sort
// ranks keys inside a wave with 64-bit ballots (lanes holding the same digit
// are found by matching the digit bit by bit), so no LDS atomics contend when
// many keys share a digit.
#include "internal.h"
#include "wave_match.h"

namespace ifgp {

// ------------------------------------------------------------------ scan
namespace {
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ __forceinline__ int64_t wave_incl_scan(int64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int64_t t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

// Exclusive prefix of v over the block (256 threads) and the block total.
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t &total) {
    __shared__ int64_t wsum[SCAN_THREADS / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int64_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < SCAN_THREADS / 64; ++i) {
        if (i < w) off += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
}

template <typename In>
__global__ __launch_bounds__(SCAN_THREADS) void scan_reduce_kernel(const In *__restrict__ in,
                                                                   int64_t n,
                                                                   int64_t *__restrict__ bsum) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + k;
        if (i < n) s += (int64_t)in[i];
    }
    int64_t tot;
    block_excl_scan(s, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// out[i] = boff[block] + sum of in[j] for block-local j < i.  `in` may alias
// `out` (each thread reads its items before anything is written).
template <typename In>
__global__ __launch_bounds__(SCAN_THREADS) void scan_down_kernel(const In *in, int64_t *out,
                                                                 int64_t n, const int64_t *boff,
                                                                 int64_t *total) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + k;
        v[k] = i < n ? (int64_t)in[i] : 0;
        s += v[k];
    }
    int64_t tot;
    const int64_t b0 = boff ? boff[blockIdx.x] : 0;
    int64_t pre = block_excl_scan(s, tot) + b0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = pre;
        pre += v[k];
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = b0 + tot;
}

__global__ void fill_i64_kernel(int64_t *p, int64_t n, int64_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
}  // namespace

template <typename In>
ifgp_status exclusive_scan(const In *in, int64_t *out, int64_t n, int64_t *total, hipStream_t s) {
    if (n <= 0) {
        if (total) {
            fill_i64_kernel<<<1, 64, 0, s>>>(total, 1, 0);
            IFGP_LAUNCHED();
        }
        return IFGP_OK;
    }
    const int64_t nb = ceil_div(n, SCAN_TILE);
    if (nb == 1) {
        scan_down_kernel<In><<<1, SCAN_THREADS, 0, s>>>(in, out, n, nullptr, total);
        IFGP_LAUNCHED();
        return IFGP_OK;
    }
    Buf bsum;
    IFGP_TRY(alloc(bsum, sizeof(int64_t) * nb, s));
    scan_reduce_kernel<In><<<nb, SCAN_THREADS, 0, s>>>(in, n, bsum.as<int64_t>());
    IFGP_LAUNCHED();
    IFGP_TRY(exclusive_scan<int64_t>(bsum.as<int64_t>(), bsum.as<int64_t>(), nb, nullptr, s));
    scan_down_kernel<In><<<nb, SCAN_THREADS, 0, s>>>(in, out, n, bsum.as<int64_t>(), total);
    IFGP_LAUNCHED();
    return IFGP_OK;
}

template ifgp_status exclusive_scan<int32_t>(const int32_t *, int64_t *, int64_t, int64_t *,
                                             hipStream_t);
template ifgp_status exclusive_scan<int64_t>(const int64_t *, int64_t *, int64_t, int64_t *,
                                             hipStream_t);
template ifgp_status exclusive_scan<uint8_t>(const uint8_t *, int64_t *, int64_t, int64_t *,
                                             hipStream_t);

ifgp_status fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s) {
    if (n <= 0) return IFGP_OK;
    fill_i64_kernel<<<ceil_div(n, 256), 256, 0, s>>>(p, n, v);
    IFGP_LAUNCHED();
    return IFGP_OK;
}

// ------------------------------------------------------------------ radix sort
namespace {
constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / 64;
constexpr int RS_ROUNDS = 16;                       // keys per lane
constexpr int RS_WAVE_TILE = 64 * RS_ROUNDS;        // 1024 keys per wave
constexpr int RS_TILE = RS_WAVES * RS_WAVE_TILE;    // 4096 keys per block
constexpr int RS_BITS = 8;  // the digit of match_digit8
constexpr int RS_BINS = 1 << RS_BITS;

// Per-block digit counts, digit-major: hist[digit * nb + block].
__global__ __launch_bounds__(RS_THREADS) void radix_hist_kernel(const uint64_t *__restrict__ keys,
                                                                int64_t n, int shift,
                                                                int64_t *__restrict__ hist,
                                                                int64_t nb) {
    __shared__ int cnt[RS_WAVES][RS_BINS];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int i = tid; i < RS_WAVES * RS_BINS; i += RS_THREADS) (&cnt[0][0])[i] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * RS_TILE + (int64_t)w * RS_WAVE_TILE;
    uint64_t key[RS_ROUNDS];
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const int64_t idx = t0 + r * 64 + lane;
        key[r] = idx < n ? keys[idx] : 0;
    }
    // Counting needs no ranks: LDS atomics into the wave's own counters (lanes
    // hitting one digit serialise inside the instruction, which is cheap even
    // for the few-valued top digit).
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r) {
        if (t0 + r * 64 + lane < n)
            atomicAdd(&cnt[w][(unsigned)(key[r] >> shift) & (RS_BINS - 1)], 1);
    }
    __syncthreads();
    int64_t tot = 0;
#pragma unroll
    for (int ww = 0; ww < RS_WAVES; ++ww) tot += cnt[ww][tid];
    hist[(int64_t)tid * nb + blockIdx.x] = tot;
}

// Stable scatter.  Key order within the block is (wave, round, lane).  The
// tile is first placed in LDS in digit order, then each digit's run is
// written to its global range by consecutive threads (coalesced stores).
// Keys read from `in`, or (PAIRS) made from edge pairs: key i is edge_keys of
// pair i / 2, the first (i even) or the second.
struct PairKeys {
    const int64_t *src, *dst;
    int64_t N;
    int B;
};

template <bool PAIRS>
__global__ __launch_bounds__(RS_THREADS) void radix_scatter_kernel(
    const uint64_t *__restrict__ in, PairKeys pk, uint64_t *__restrict__ out, int64_t n, int shift,
    const int64_t *__restrict__ offs, int64_t nb) {
    __shared__ int cnt[RS_WAVES][RS_BINS];
    __shared__ int tstart[RS_BINS];
    __shared__ int wsum[RS_WAVES];
    __shared__ int64_t gbase[RS_BINS];
    __shared__ uint64_t lkeys[RS_TILE];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int i = tid; i < RS_WAVES * RS_BINS; i += RS_THREADS) (&cnt[0][0])[i] = 0;
    gbase[tid] = offs[(int64_t)tid * nb + blockIdx.x];
    __syncthreads();
    const int64_t tile0 = (int64_t)blockIdx.x * RS_TILE;
    const int64_t t0 = tile0 + (int64_t)w * RS_WAVE_TILE;
    const uint64_t lt = __lanemask_lt();
    uint64_t key[RS_ROUNDS];
    int rank[RS_ROUNDS];
    if constexpr (PAIRS) {
        // every round's pair loaded before any key is made (the loads in
        // flight together); lanes 2k and 2k + 1 read the same pair
        int64_t u[RS_ROUNDS], v[RS_ROUNDS];
#pragma unroll
        for (int r = 0; r < RS_ROUNDS; ++r) {
            const int64_t idx = t0 + r * 64 + lane;
            u[r] = idx < n ? pk.src[idx >> 1] : 0;
            v[r] = idx < n ? pk.dst[idx >> 1] : 0;
        }
#pragma unroll
        for (int r = 0; r < RS_ROUNDS; ++r) {
            uint64_t k0, k1;
            edge_keys(u[r], v[r], pk.N, pk.B, k0, k1);
            key[r] = (lane & 1) ? k1 : k0;
        }
    } else {
#pragma unroll
        for (int r = 0; r < RS_ROUNDS; ++r) {
            const int64_t idx = t0 + r * 64 + lane;
            key[r] = idx < n ? in[idx] : 0;
        }
    }
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const bool valid = t0 + r * 64 + lane < n;
        const unsigned g = (unsigned)(key[r] >> shift) & (RS_BINS - 1);
        const uint64_t m = match_digit8(g, valid);
        const int below = __popcll(m & lt);
        int c = 0;
        if (valid) c = cnt[w][g];
        // The leader's write depends on the value all lanes just read, so the
        // read of this wave completes before the write is issued.
        if (valid && below == 0) cnt[w][g] = c + __popcll(m);
        rank[r] = valid ? c + below : -1;
    }
    __syncthreads();
    // per digit (one per thread): offsets of the waves, and the tile total
    int total = 0;
#pragma unroll
    for (int ww = 0; ww < RS_WAVES; ++ww) {
        const int t = cnt[ww][tid];
        cnt[ww][tid] = total;
        total += t;
    }
    // exclusive scan of the 256 digit totals -> tile-local start of each digit
    int inc = total;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(inc, off, 64);
        if (lane >= off) inc += t;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int woff = 0;
#pragma unroll
    for (int ww = 0; ww < RS_WAVES; ++ww)
        if (ww < w) woff += wsum[ww];
    tstart[tid] = woff + inc - total;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r) {
        if (rank[r] >= 0) {
            const unsigned g = (unsigned)(key[r] >> shift) & (RS_BINS - 1);
            lkeys[tstart[g] + cnt[w][g] + rank[r]] = key[r];
        }
    }
    __syncthreads();
    const int tile_n = (int)(n - tile0 < RS_TILE ? n - tile0 : RS_TILE);
    for (int i = tid; i < tile_n; i += RS_THREADS) {
        const uint64_t k = lkeys[i];
        const unsigned g = (unsigned)(k >> shift) & (RS_BINS - 1);
        out[gbase[g] + (i - tstart[g])] = k;
    }
}
}  // namespace

namespace {
// The passes over bits [lo, hi) of keys in src (the first pass's counts
// already in hist if have_first), ping-ponging with dst.
ifgp_status radix_passes(uint64_t *src, uint64_t *dst, int64_t n, int lo, int hi, hipStream_t s,
                         uint64_t **sorted, int64_t *hist, bool have_first) {
    const int64_t nb = ceil_div(n, RS_TILE);
    for (int shift = lo; shift < hi; shift += RS_BITS) {
        if (!(have_first && shift == lo)) {
            radix_hist_kernel<<<nb, RS_THREADS, 0, s>>>(src, n, shift, hist, nb);
            IFGP_LAUNCHED();
        }
        IFGP_TRY(exclusive_scan<int64_t>(hist, hist, RS_BINS * nb, nullptr, s));
        radix_scatter_kernel<false><<<nb, RS_THREADS, 0, s>>>(src, PairKeys{}, dst, n, shift, hist,
                                                              nb);
        IFGP_LAUNCHED();
        std::swap(src, dst);
    }
    *sorted = src;
    return IFGP_OK;
}
}  // namespace

ifgp_status radix_sort_u64(uint64_t *a, uint64_t *b, int64_t n, int lo, int hi, hipStream_t s,
                           uint64_t **sorted, int64_t *first_hist) {
    static_assert(RS_TILE == RADIX_TILE, "tile of the fused first histogram");
    *sorted = a;
    if (n <= 1 || hi <= lo) return IFGP_OK;
    Buf own;
    int64_t *hist = first_hist;
    if (!hist) {
        IFGP_TRY(alloc(own, sizeof(int64_t) * RS_BINS * ceil_div(n, RS_TILE), s));
        hist = own.as<int64_t>();
    }
    return radix_passes(a, b, n, lo, hi, s, sorted, hist, first_hist != nullptr);
}

ifgp_status radix_sort_pairs(const int64_t *src, const int64_t *dst, int64_t E, int64_t N, int B,
                             uint64_t *a, uint64_t *b, int lo, int hi, hipStream_t s,
                             uint64_t **sorted, int64_t *first_hist) {
    const int64_t n = 2 * E, nb = ceil_div(n, RS_TILE);
    *sorted = a;
    if (n < 1 || hi <= lo || !first_hist) {
        set_error("radix_sort_pairs: needs keys, a bit range and the first pass's counts");
        return IFGP_E_INVALID;
    }
    // the first pass: keys made from the pairs, scattered into a
    IFGP_TRY(exclusive_scan<int64_t>(first_hist, first_hist, RS_BINS * nb, nullptr, s));
    radix_scatter_kernel<true><<<nb, RS_THREADS, 0, s>>>(nullptr, PairKeys{src, dst, N, B}, a, n, lo,
                                                         first_hist, nb);
    IFGP_LAUNCHED();
    if (lo + RS_BITS >= hi) return IFGP_OK;
    return radix_passes(a, b, n, lo + RS_BITS, hi, s, sorted, first_hist, false);
}

}  // namespace ifgp
