// InfraredGP's feed-forward propagation on gfx950.
//
// Layer l (Eq. (4)) with the filter of Eq. (3):
//     Y = theta Zn + alpha S A S Zn,   T = tanh(Y),   Z^(l) = ZNorm(T)
// where S = D_tau^{-1/2} (Eq. (1)) and Zn = Z^(l-1).
//
// Storage between hops.  Row i of the feature buffer holds W_i = s_i T_i
// (s_i = (D_tau)_ii^{-1/2}) rounded to the storage type, and ZNorm is applied
// lazily by the next hop through per-column a_c = 1/sigma_c, b_c = -mu_c/sigma_c
// (Zn = a T + b).  Then
//     sum_j s_j Zn_j = a (sum_j W_j) + b r_i,     r_i = sum_{j in N(i)} s_j,
// so a hop gathers W rows and adds them, with no per-neighbour multiply and no
// per-neighbour scale load; the self term uses T_i = W_i sqrt((D_tau)_ii).
// Z^(0) is stored the same way (W = s X) with a = 1, b = 0.
//
// Column statistics (mu, sigma of T, Eq. (4)) are gathered in FP64 from the
// values actually stored, per block, then reduced in a fixed order by a
// finalize kernel: results are deterministic run to run.
//
// Kernel geometry (wave64): a row of D storage elements is read as 16-byte
// vectors by LPR = D / (16 / sizeof(T)) lanes.  Rows are in descending-degree
// order (plan built with the graph), split into three classes:
//   hub     deg >= 4096  one 256-thread block per row
//   medium  deg >= 128   one wave per row (subgroups split the neighbours)
//   light   the rest     one LPR-lane subgroup per row, 256 rows per block
// Heavy rows come first in the grid, so long blocks start early.
#include <cmath>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <mutex>
#include <type_traits>

#include "internal.h"

namespace ifgp {
namespace {

constexpr int THREADS = 256;
constexpr int WAVES = THREADS / 64;
// Neighbour rows in flight per lane: 16-byte loads of 4-byte storage cover
// half as many columns as those of 2-byte storage, so they get twice the
// depth.  For 2-byte storage the depth is chosen per graph (hop_depth): a
// feature matrix that stays in cache gathers more rows at a time, one far
// beyond the Infinity Cache with rows of 64 columns or more fewer (measured
// per hop at width 64: 200k nodes 91 us with 8 rows, 83 us with 16; 1M nodes
// 387 us with 8, 397 with 16, 425 with 4; 2M nodes 0.788 ms with 8, 0.777 ms
// with 4).
#ifndef IFGP_HOP_UNROLL_2B
#define IFGP_HOP_UNROLL_2B 8
#endif
#ifndef IFGP_HOP_UNROLL_2B_SHALLOW
#define IFGP_HOP_UNROLL_2B_SHALLOW 4
#endif
#ifndef IFGP_HOP_UNROLL_2B_DEEP
#define IFGP_HOP_UNROLL_2B_DEEP 16
#endif
enum HopDepth { DEPTH_NORMAL = 0, DEPTH_SHALLOW = 1, DEPTH_DEEP = 2 };
#ifndef IFGP_HOP_UNROLL_4B
#define IFGP_HOP_UNROLL_4B 16
#endif

template <typename T, int D, int DEPTH = DEPTH_NORMAL> struct Cfg {
    static constexpr int U = sizeof(T) == 4                         ? IFGP_HOP_UNROLL_4B
                             : (DEPTH == DEPTH_SHALLOW && D >= 64) ? IFGP_HOP_UNROLL_2B_SHALLOW
                             : DEPTH == DEPTH_DEEP                 ? IFGP_HOP_UNROLL_2B_DEEP
                                                                   : IFGP_HOP_UNROLL_2B;
    static constexpr int EPL = 16 / (int)sizeof(T);   // elements per lane
    static constexpr int LPR = D / EPL;               // lanes per row
    static constexpr int RPW = 64 / LPR;              // rows (subgroups) per wave
    static constexpr int QI = (U + LPR - 1) / LPR;    // index loads per lane per chunk
    static constexpr int LIGHT_ROWS = light_rows_per_block(RPW);
    static_assert(LPR >= 1 && LPR <= 64 && (64 % LPR) == 0, "unsupported width");
    static_assert(LIGHT_ROWS % (WAVES * RPW) == 0, "light block shape");
};

// ---------------------------------------------------------------- pack/unpack
__device__ __forceinline__ uint4 ld16(const void *p) { return *reinterpret_cast<const uint4 *>(p); }
__device__ __forceinline__ void st16(void *p, const uint4 &v) { *reinterpret_cast<uint4 *>(p) = v; }
// Streaming store (non-temporal hint): a hop's output rows are not read again
// within the hop, so they should not displace the rows being gathered.
typedef unsigned int v4u_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void st16_stream(void *p, const uint4 &v) {
    const v4u_t x = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(x, reinterpret_cast<v4u_t *>(p));
}

template <typename T> __device__ __forceinline__ void unpack(const uint4 &r, float *f);
template <> __device__ __forceinline__ void unpack<float>(const uint4 &r, float *f) {
    f[0] = __uint_as_float(r.x);
    f[1] = __uint_as_float(r.y);
    f[2] = __uint_as_float(r.z);
    f[3] = __uint_as_float(r.w);
}
template <> __device__ __forceinline__ void unpack<bf16_t>(const uint4 &r, float *f) {
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f[2 * i] = __uint_as_float(w[i] << 16);
        f[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
    }
}
template <> __device__ __forceinline__ void unpack<f16_t>(const uint4 &r, float *f) {
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f[2 * i] = (float)__builtin_bit_cast(f16_t, (uint16_t)(w[i] & 0xffffu));
        f[2 * i + 1] = (float)__builtin_bit_cast(f16_t, (uint16_t)(w[i] >> 16));
    }
}

// Round f to T; `back` receives the float value of what is stored.
template <typename T> __device__ __forceinline__ uint4 pack(const float *f, float *back);
template <> __device__ __forceinline__ uint4 pack<float>(const float *f, float *back) {
#pragma unroll
    for (int i = 0; i < 4; ++i) back[i] = f[i];
    return make_uint4(__float_as_uint(f[0]), __float_as_uint(f[1]), __float_as_uint(f[2]),
                      __float_as_uint(f[3]));
}
template <> __device__ __forceinline__ uint4 pack<bf16_t>(const float *f, float *back) {
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t lo = from_f32<bf16_t>(f[2 * i]).x, hi = from_f32<bf16_t>(f[2 * i + 1]).x;
        back[2 * i] = __uint_as_float(lo << 16);
        back[2 * i + 1] = __uint_as_float(hi << 16);
        w[i] = lo | (hi << 16);
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}
template <> __device__ __forceinline__ uint4 pack<f16_t>(const float *f, float *back) {
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const f16_t a = (f16_t)f[2 * i], b = (f16_t)f[2 * i + 1];
        back[2 * i] = (float)a;
        back[2 * i + 1] = (float)b;
        w[i] = (uint32_t)__builtin_bit_cast(uint16_t, a) |
               ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// An FP64 value in a storage type: FP32 and FP16 are rounded once, straight
// from FP64 (to nearest, ties to even); BF16 through FP32 (two roundings).
template <typename T> __device__ __forceinline__ T cvt_from_f64(double v) {
    return from_f32<T>((float)v);
}
template <> __device__ __forceinline__ f16_t cvt_from_f64<f16_t>(double v) { return (f16_t)v; }

// ---------------------------------------------------------------- Philox / Box-Muller
// Full 64 x 64 -> 128-bit product from four 32 x 32 -> 64-bit multiply-adds
// (each a single v_mad_u64_u32), the partial products shared by both halves.
__device__ __forceinline__ void mulhilo64(uint64_t a, uint64_t b, uint64_t &hi, uint64_t &lo) {
    const uint32_t al = (uint32_t)a, ah = (uint32_t)(a >> 32);
    const uint32_t bl = (uint32_t)b, bh = (uint32_t)(b >> 32);
    const uint64_t p0 = (uint64_t)al * bl;
    const uint64_t t = (uint64_t)al * bh + (p0 >> 32);
    const uint64_t u = (uint64_t)ah * bl + (uint32_t)t;
    lo = (u << 32) | (uint32_t)p0;
    hi = (uint64_t)ah * bh + (t >> 32) + (u >> 32);
}

// a ^ b ^ c with one three-input bitwise instruction per 32-bit half (truth
// table 0x96 is the odd-parity function of the three inputs)
__device__ __forceinline__ uint64_t xor3(uint64_t a, uint64_t b, uint64_t c) {
    const uint32_t lo = __builtin_amdgcn_bitop3_b32((uint32_t)a, (uint32_t)b, (uint32_t)c, 0x96);
    const uint32_t hi = __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), (uint32_t)(b >> 32),
                                                    (uint32_t)(c >> 32), 0x96);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ void philox4x64_10(uint64_t &c0, uint64_t &c1, uint64_t &c2,
                                              uint64_t &c3, uint64_t k0, uint64_t k1) {
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, c0, hi0, lo0);
        mulhilo64(M1, c2, hi1, lo1);
        const uint64_t n0 = xor3(hi1, c1, k0), n2 = xor3(hi0, c3, k1);
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
}

// Z^(0)[i, 4q .. 4q+3] in FP64 (see ifgp_embed in ifgp.h for the rule): one
// Philox4x64-10 block, two Box-Muller pairs (cos and sin of each).
__device__ __forceinline__ void gaussian4(uint64_t seed, int64_t i, int64_t q, int d, double *z) {
    uint64_t c0 = (uint64_t)i + 1, c1 = (uint64_t)q, c2 = 0, c3 = 0;
    philox4x64_10(c0, c1, c2, c3, seed, 0);
    const uint64_t w[4] = {c0, c1, c2, c3};
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const double ua = ((double)(w[2 * p] >> 11) + 0.5) * 0x1p-53;
        const double ub = ((double)(w[2 * p + 1] >> 11) + 0.5) * 0x1p-53;
        const double r = sqrt(-2.0 * log(ua));
        double sn, cs;
        sincos(2.0 * M_PI * ub, &sn, &cs);
        z[2 * p] = (r * cs) / sqrt((double)d);
        z[2 * p + 1] = (r * sn) / sqrt((double)d);
    }
}

// The same four entries for 2-byte storage, whose rounding (2^-8 or 2^-11)
// is far coarser than FP32 arithmetic's: the uniforms are formed from the
// words' top 23 bits, u = ((w >> 41) + 0.5) 2^-23 (exact in FP32, inside
// (0, 1)), and Box-Muller uses the hardware's FP32 instructions: log2
// (ln u = log2 u * ln 2), square root, and sine and cosine of a fraction of
// a turn (sin(2 pi u) taken as the turn u).
__device__ __forceinline__ void gaussian4_f32(uint64_t seed, int64_t i, int64_t q, int d, float *z) {
    uint64_t c0 = (uint64_t)i + 1, c1 = (uint64_t)q, c2 = 0, c3 = 0;
    philox4x64_10(c0, c1, c2, c3, seed, 0);
    const uint64_t w[4] = {c0, c1, c2, c3};
    const float inv = 1.0f / sqrtf((float)d);
    constexpr float kMinus2Ln2 = -1.3862943611198906f;  // -2 ln 2
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const float ua = ((float)(uint32_t)(w[2 * p] >> 41) + 0.5f) * 0x1p-23f;
        const float ub = ((float)(uint32_t)(w[2 * p + 1] >> 41) + 0.5f) * 0x1p-23f;
        const float r = __builtin_amdgcn_sqrtf(kMinus2Ln2 * __builtin_amdgcn_logf(ua)) * inv;
        z[2 * p] = r * __builtin_amdgcn_cosf(ub);
        z[2 * p + 1] = r * __builtin_amdgcn_sinf(ub);
    }
}

// ---------------------------------------------------------------- small kernels
template <typename T>
__global__ void gaussian_kernel(int64_t N, int d, uint64_t seed, T *out) {
    const int64_t nq = (d + 3) / 4;
    const int64_t t = block_index() * blockDim.x + threadIdx.x;
    if (t >= N * nq) return;
    const int64_t i = t / nq, q = t - i * nq;
    double z[4];
    gaussian4(seed, i, q, d, z);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t c = 4 * q + j;
        if (c < d) {
            if constexpr (std::is_same<T, double>::value) out[i * d + c] = z[j];
            else out[i * d + c] = cvt_from_f64<T>(z[j]);
        }
    }
}

// W0[k, c] = s_k Z^(0)[perm[k], c] for c < d, 0 in the padding columns; one
// thread per group of four columns.
template <typename T, int D>
__global__ void noise_kernel(int64_t N, int d, uint64_t seed, const int32_t *__restrict__ perm,
                             const double *__restrict__ s64, T *__restrict__ W) {
    constexpr int NQ = D / 4;
    const int64_t t = block_index() * blockDim.x + threadIdx.x;
    if (t >= N * NQ) return;
    const int64_t k = t / NQ;
    const int q = (int)(t % NQ);
    const double sk = s64[k];
    if constexpr (sizeof(T) == 2) {
        float z[4] = {0.f, 0.f, 0.f, 0.f};
        if (4 * q < d) gaussian4_f32(seed, perm[k], q, d, z);
        const float skf = (float)sk;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = 4 * q + j;
            W[k * D + c] = from_f32<T>(c < d ? skf * z[j] : 0.f);
        }
    } else {
        double z[4] = {0.0, 0.0, 0.0, 0.0};
        if (4 * q < d) gaussian4(seed, perm[k], q, d, z);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = 4 * q + j;
            W[k * D + c] = cvt_from_f64<T>(c < d ? sk * z[j] : 0.0);
        }
    }
}

// W0[k, c] = s_k X[perm[k], c] for a caller-supplied X.
template <typename T, int D>
__global__ void prep_x_kernel(int64_t N, int d, const float *__restrict__ X,
                              const int32_t *__restrict__ perm, const double *__restrict__ s64,
                              T *__restrict__ W) {
    const int64_t t = block_index() * blockDim.x + threadIdx.x;
    if (t >= N * D) return;
    const int64_t k = t / D;
    const int c = (int)(t % D);
    double v = 0.0;
    if (c < d) v = s64[k] * (double)X[(int64_t)perm[k] * d + c];
    W[t] = cvt_from_f64<T>(v);
}

__global__ void ab_identity_kernel(float *ab, int D) {
    const int c = threadIdx.x;
    if (c < D) {
        ab[c] = 1.0f;
        ab[D + c] = 0.0f;
    }
}

// (D_tau)_ii: Eq. (1) for tau <= 0, literal; deg + tau for tau > 0.
__device__ __forceinline__ double dtau_of(double deg, double tau, double eps) {
    if (tau > 0) return deg + tau;
    const double at = fabs(tau), m = deg - eps;
    return deg - (at < m ? at : m);
}

__global__ void scales_kernel(int64_t N, const int64_t *__restrict__ irowptr, double tau,
                              double eps, double *__restrict__ s64, float *__restrict__ s32) {
    const int64_t k = block_index() * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const double dt = dtau_of((double)(irowptr[k + 1] - irowptr[k]), tau, eps);
    const double sk = 1.0 / sqrt(dt);
    s64[k] = sk;
    s32[k] = (float)sk;
}

// r_k = sum of s over row k's neighbours (FP32 copies of s, summed in FP64).
// Rows are in descending-degree order: the first n_heavy rows get one wave
// each, the rest NI_LANES lanes each; every lane keeps NI_DEPTH independent
// loads in flight and the lanes of a row combine by a fixed butterfly
// (deterministic order).
//
// A neighbour's s comes from a table in LDS where it can.  Internal ids are
// sorted by degree and s depends on the degree alone, so s is constant over
// long runs of ids: the table holds, for each bucket of 2^sh consecutive ids,
// the bucket's s if all its ids have one degree and -1 otherwise (s > 0), and
// only entries in mixed buckets gather s from memory.  The mixed buckets are
// those of the few high-degree nodes, whose ids are low and whose s values
// stay in L2; a random 4-byte gather from the whole N-long table would move
// a 128-byte line.  The values are the same either way, so the sums are too.
// Below NI_TABLE_MIN_NODES the whole FP32 s fits in L2 and the table is not
// built.
constexpr int NI_LANES = 8;
constexpr int NI_DEPTH = 4;
constexpr int NI_TABLE = 4096;      // buckets (16 KB of LDS)
constexpr int64_t NI_GRID = 1024;   // blocks striding over the row groups (4 per CU: room for the
                                    // random input, which runs beside them)
constexpr int64_t NI_TABLE_MIN_NODES = int64_t(1) << 19;

int ni_shift(int64_t N) {
    int sh = 0;
    while (ceil_div(N, (int64_t)1 << sh) > NI_TABLE) ++sh;
    return sh;
}

// Bucket k covers internal ids [k 2^sh, min((k+1) 2^sh, N)); degrees are
// non-increasing in the id, so equal degrees at both ends mean one degree.
__global__ void s_table_kernel(int64_t N, int sh, int64_t nbk, const int64_t *__restrict__ irowptr,
                               const float *__restrict__ s32, float *__restrict__ tab) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nbk) return;
    const int64_t lo = k << sh, hi = ((k + 1) << sh < N ? (k + 1) << sh : N) - 1;
    const int64_t dlo = irowptr[lo + 1] - irowptr[lo], dhi = irowptr[hi + 1] - irowptr[hi];
    tab[k] = dlo == dhi ? s32[lo] : -1.0f;
}

template <int LANES, bool TABLE>
__device__ __forceinline__ double row_neighbour_sum(const int32_t *__restrict__ icolidx,
                                                    const float *__restrict__ s32,
                                                    const float *lt, int sh, int64_t beg,
                                                    int64_t end, int l) {
    double r = 0.0;
    for (int64_t e0 = beg + l; e0 < end; e0 += (int64_t)LANES * NI_DEPTH) {
        int32_t j[NI_DEPTH];
#pragma unroll
        for (int q = 0; q < NI_DEPTH; ++q) {
            const int64_t e = e0 + (int64_t)q * LANES;
            j[q] = e < end ? icolidx[e] : -1;
        }
        float v[NI_DEPTH];
        if constexpr (TABLE) {
#pragma unroll
            for (int q = 0; q < NI_DEPTH; ++q) v[q] = j[q] >= 0 ? lt[j[q] >> sh] : 0.f;
#pragma unroll
            for (int q = 0; q < NI_DEPTH; ++q)
                if (v[q] < 0.f) v[q] = s32[j[q]];
        } else {
#pragma unroll
            for (int q = 0; q < NI_DEPTH; ++q) v[q] = j[q] >= 0 ? s32[j[q]] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < NI_DEPTH; ++q) r += (double)v[q];
    }
#pragma unroll
    for (int off = LANES / 2; off > 0; off >>= 1) r += __shfl_xor(r, off, LANES);
    return r;
}

// Row groups: heavy_groups of THREADS/64 heavy rows, then groups of
// THREADS/NI_LANES light rows; with the table each block loads it once and
// strides over the groups, without it a block takes one group.
template <bool TABLE>
__global__ __launch_bounds__(THREADS) void nodeinfo_kernel(int64_t N, int64_t n_heavy,
                                                           int64_t heavy_groups, int64_t groups,
                                                           const int64_t *__restrict__ irowptr,
                                                           const int32_t *__restrict__ icolidx,
                                                           const double *__restrict__ s64,
                                                           const float *__restrict__ s32,
                                                           const float *__restrict__ tab,
                                                           int ntab, int sh, double tau,
                                                           double eps,
                                                           float4 *__restrict__ info) {
    __shared__ float lt[TABLE ? NI_TABLE : 1];
    if constexpr (TABLE) {
        for (int i = threadIdx.x; i < ntab; i += THREADS) lt[i] = tab[i];
        __syncthreads();
    }
    for (int64_t grp = blockIdx.x; grp < groups; grp += gridDim.x) {
        int64_t k;
        int l;
        double r;
        if (grp < heavy_groups) {
            k = grp * (THREADS / 64) + threadIdx.x / 64;
            l = threadIdx.x % 64;
            if (k >= n_heavy) continue;   // the whole wave
            r = row_neighbour_sum<64, TABLE>(icolidx, s32, lt, sh, irowptr[k], irowptr[k + 1], l);
        } else {
            k = n_heavy + (grp - heavy_groups) * (THREADS / NI_LANES) + threadIdx.x / NI_LANES;
            l = threadIdx.x % NI_LANES;
            if (k >= N) continue;         // the whole subgroup
            r = row_neighbour_sum<NI_LANES, TABLE>(icolidx, s32, lt, sh, irowptr[k], irowptr[k + 1],
                                                   l);
        }
        if (l == 0) {
            const double dt = dtau_of((double)(irowptr[k + 1] - irowptr[k]), tau, eps);
            info[k] = make_float4((float)s64[k], (float)sqrt(dt), (float)r, 0.0f);
        }
    }
}

__global__ void perm_scales_kernel(int64_t N, const int32_t *__restrict__ perm,
                                   const double *__restrict__ s64, double *__restrict__ out) {
    const int64_t k = block_index() * blockDim.x + threadIdx.x;
    if (k < N) out[perm[k]] = s64[k];
}

// ---------------------------------------------------------------- the hop
struct HopArgs {
    const int64_t *rowptr;   // internal CSR
    const int32_t *colidx;
    const void *Win;         // N x D storage, W of the previous hop
    void *Wout;
    const float4 *node;      // (s, sqrt(D_tau), r, 0)
    const float *ab;         // a[D], b[D] of the previous hop's ZNorm
    double2 *partials;       // [D][blocks] (sum T, sum T^2), column-major
    int64_t N, n_hub, n_med;
    int64_t blk_hub_end, blk_med_end, blocks;
    int light_rows;          // rows per light block (a multiple of 4 * RPW)
    float alpha, theta;
};

// Gather-add W rows of neighbours e in [first, end) visited in chunks of U
// starting every `step`: acc[e] += sum W[j, sl*EPL + e].
template <typename T, int D, int DEPTH>
__device__ __forceinline__ void gather_add(const int32_t *__restrict__ colidx,
                                           const char *__restrict__ Win, int64_t first,
                                           int64_t end, int64_t step, int sl, int lane_base,
                                           float *acc) {
    using C = Cfg<T, D, DEPTH>;
    constexpr int EPL = C::EPL, LPR = C::LPR, QI = C::QI, U = C::U;
    const int64_t col_off = (int64_t)sl * EPL * (int64_t)sizeof(T);
    for (int64_t e0 = first; e0 < end; e0 += step) {
        int32_t idx[QI];
#pragma unroll
        for (int q = 0; q < QI; ++q) {
            const int slot = q * LPR + sl;
            const int64_t e = e0 + slot;
            idx[q] = (slot < U && e < end) ? colidx[e] : -1;
        }
        uint4 raw[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            int j;
            if constexpr (LPR == 1) j = idx[k];
            else j = __shfl(idx[k / LPR], lane_base + (k % LPR), 64);
            if (j >= 0) raw[k] = ld16(Win + (int64_t)j * (D * (int64_t)sizeof(T)) + col_off);
            else raw[k] = make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            float f[EPL];
            unpack<T>(raw[k], f);
#pragma unroll
            for (int e = 0; e < EPL; ++e) acc[e] += f[e];
        }
    }
}

// Finish row r from its neighbour sum: tanh, store W = s T, add the stored
// T to the column statistics.
template <typename T, int D>
__device__ __forceinline__ void row_finish(const HopArgs &a, int64_t r, int sl, const float *acc,
                                           const float *av, const float *bv, double *ssum,
                                           double *ssq) {
    using C = Cfg<T, D>;
    constexpr int EPL = C::EPL;
    const float4 nd = a.node[r];
    const int64_t off = (r * D + (int64_t)sl * EPL) * (int64_t)sizeof(T);
    float xin[EPL];
    unpack<T>(ld16((const char *)a.Win + off), xin);
    float wnew[EPL], back[EPL];
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
        const float tprev = xin[e] * nd.y;                  // T_i of the previous hop
        const float zself = fmaf(av[e], tprev, bv[e]);      // Zn_i
        const float agg = fmaf(av[e], acc[e], bv[e] * nd.z); // sum_j s_j Zn_j
        const float y = fmaf(a.theta, zself, a.alpha * nd.x * agg);
        wnew[e] = nd.x * tanhf(y);
    }
    st16_stream((char *)a.Wout + off, pack<T>(wnew, back));
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
        const double t = (double)back[e] * (double)nd.y;  // stored T_i (float product, exact in FP64)
        ssum[e] += t;
        ssq[e] += t * t;
    }
}

template <typename T, int D, int DEPTH>
__device__ __forceinline__ void hop_block(const HopArgs &a, int64_t blk) {
    using C = Cfg<T, D, DEPTH>;
    constexpr int EPL = C::EPL, LPR = C::LPR, RPW = C::RPW, U = C::U;
    __shared__ float lds_acc[WAVES][D];
    __shared__ double2 lds_st[WAVES][D];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int g = lane / LPR, sl = lane % LPR, lane_base = lane - sl;
    const char *Win = (const char *)a.Win;

    float av[EPL], bv[EPL];
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
        av[e] = a.ab[sl * EPL + e];
        bv[e] = a.ab[D + sl * EPL + e];
    }
    double ssum[EPL], ssq[EPL];
#pragma unroll
    for (int e = 0; e < EPL; ++e) ssum[e] = ssq[e] = 0.0;

    if (blk < a.blk_hub_end) {
        // hub: the whole block on one row
        const int64_t r = blk;
        float acc[EPL];
#pragma unroll
        for (int e = 0; e < EPL; ++e) acc[e] = 0.f;
        const int64_t beg = a.rowptr[r], end = a.rowptr[r + 1];
        gather_add<T, D, DEPTH>(a.colidx, Win, beg + (int64_t)(w * RPW + g) * U, end,
                         (int64_t)WAVES * RPW * U, sl, lane_base, acc);
#pragma unroll
        for (int off = LPR; off < 64; off <<= 1)
#pragma unroll
            for (int e = 0; e < EPL; ++e) acc[e] += __shfl_xor(acc[e], off, 64);
        if (g == 0)
#pragma unroll
            for (int e = 0; e < EPL; ++e) lds_acc[w][sl * EPL + e] = acc[e];
        __syncthreads();
        if (w == 0 && g == 0) {
#pragma unroll
            for (int e = 0; e < EPL; ++e) {
                const int c = sl * EPL + e;
                acc[e] = ((lds_acc[0][c] + lds_acc[1][c]) + lds_acc[2][c]) + lds_acc[3][c];
            }
            row_finish<T, D>(a, r, sl, acc, av, bv, ssum, ssq);
        }
    } else if (blk < a.blk_med_end) {
        // medium: one wave per row
        const int64_t r = a.n_hub + (blk - a.blk_hub_end) * MED_ROWS_PER_BLOCK + w;
        if (r < a.n_hub + a.n_med) {
            float acc[EPL];
#pragma unroll
            for (int e = 0; e < EPL; ++e) acc[e] = 0.f;
            const int64_t beg = a.rowptr[r], end = a.rowptr[r + 1];
            gather_add<T, D, DEPTH>(a.colidx, Win, beg + (int64_t)g * U, end, (int64_t)RPW * U, sl,
                             lane_base, acc);
#pragma unroll
            for (int off = LPR; off < 64; off <<= 1)
#pragma unroll
                for (int e = 0; e < EPL; ++e) acc[e] += __shfl_xor(acc[e], off, 64);
            if (g == 0) row_finish<T, D>(a, r, sl, acc, av, bv, ssum, ssq);
        }
    } else {
        // light: one LPR-lane subgroup per row
        const int64_t row0 = a.n_hub + a.n_med + (blk - a.blk_med_end) * (int64_t)a.light_rows;
        const int passes = a.light_rows / (WAVES * RPW);
        for (int p = 0; p < passes; ++p) {
            const int64_t r = row0 + (int64_t)p * WAVES * RPW + w * RPW + g;
            if (r < a.N) {
                float acc[EPL];
#pragma unroll
                for (int e = 0; e < EPL; ++e) acc[e] = 0.f;
                gather_add<T, D, DEPTH>(a.colidx, Win, a.rowptr[r], a.rowptr[r + 1], (int64_t)U, sl,
                                 lane_base, acc);
                row_finish<T, D>(a, r, sl, acc, av, bv, ssum, ssq);
            }
        }
    }

    // block statistics: subgroups (butterfly), then waves in order
#pragma unroll
    for (int off = LPR; off < 64; off <<= 1)
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
            ssum[e] += __shfl_xor(ssum[e], off, 64);
            ssq[e] += __shfl_xor(ssq[e], off, 64);
        }
    if (g == 0)
#pragma unroll
        for (int e = 0; e < EPL; ++e) lds_st[w][sl * EPL + e] = make_double2(ssum[e], ssq[e]);
    __syncthreads();
    if (tid < D) {
        double2 t = lds_st[0][tid];
#pragma unroll
        for (int ww = 1; ww < WAVES; ++ww) {
            t.x += lds_st[ww][tid].x;
            t.y += lds_st[ww][tid].y;
        }
        a.partials[(int64_t)tid * a.blocks + blk] = t;
    }
}

template <typename T, int D, int DEPTH>
__global__ __launch_bounds__(THREADS) void hop_kernel(const HopArgs a) {
    const int64_t blk = block_index();
    if (blk >= a.blocks) return;
    hop_block<T, D, DEPTH>(a, blk);
}

// Many graphs in one launch; the table travels as a kernel argument (no
// device allocation, no host synchronisation).  Graph gi owns blocks
// [start[gi], start[gi+1]).
constexpr int MAX_BATCH = 24;
struct HopBatch {
    HopArgs a[MAX_BATCH];
    int64_t start[MAX_BATCH + 1];
    int n;
};
static_assert(sizeof(HopBatch) <= 3584, "batch table must fit the kernel argument segment");

template <typename T, int D, int DEPTH>
__global__ __launch_bounds__(THREADS) void hop_batch_kernel(const HopBatch bt) {
    const int64_t b = block_index();
    if (b >= bt.start[bt.n]) return;
    int gi = 0;
    while (gi + 1 < bt.n && bt.start[gi + 1] <= b) ++gi;
    hop_block<T, D, DEPTH>(bt.a[gi], b - bt.start[gi]);
}

// mu, sigma per column from the block partials (fixed order), then
// a = 1/sigma, b = -mu/sigma; a column of zero spread gives a = b = 0.
struct FinArgs {
    const double2 *partials;
    int64_t blocks, N;
    int D, ddof;
    float *ab;
};

constexpr int FIN_THREADS = 1024;

__device__ __forceinline__ void finalize_column(const FinArgs &f, int c) {
    __shared__ double rs[FIN_THREADS / 64], rq[FIN_THREADS / 64];
    double s = 0.0, q = 0.0;
    const double2 *col = f.partials + (int64_t)c * f.blocks;
    for (int64_t b = threadIdx.x; b < f.blocks; b += FIN_THREADS) {
        const double2 p = col[b];
        s += p.x;
        q += p.y;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        s += __shfl_xor(s, off, 64);
        q += __shfl_xor(q, off, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        rs[w] = s;
        rq[w] = q;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s = 0.0;
        q = 0.0;
        for (int i = 0; i < FIN_THREADS / 64; ++i) {
            s += rs[i];
            q += rq[i];
        }
        const double n = (double)f.N;
        const double mu = s / n;
        const double den = n - (double)f.ddof;
        // s*mu rounded on its own (no fused multiply-add), so that one row, or
        // identical rows summed exactly, give a variance of exactly zero
        double var = 0.0;
        if (den > 0) {
#pragma clang fp contract(off)
            const double smu = s * mu;
            var = (q - smu) / den;
        }
        float a = 0.f, b = 0.f;
        if (var > 0) {
            const double sd = sqrt(var);
            a = (float)(1.0 / sd);
            b = (float)(-mu / sd);
        }
        f.ab[c] = a;
        f.ab[f.D + c] = b;
    }
}

__global__ __launch_bounds__(FIN_THREADS) void finalize_kernel(const FinArgs f) {
    finalize_column(f, blockIdx.x);
}

struct FinBatch {
    FinArgs f[MAX_BATCH];
};
static_assert(sizeof(FinBatch) <= 3584, "batch table must fit the kernel argument segment");

// grid = (D, graphs)
__global__ __launch_bounds__(FIN_THREADS) void finalize_batch_kernel(const FinBatch fb) {
    const FinArgs &f = fb.f[blockIdx.y];
    if ((int)blockIdx.x < f.D) finalize_column(f, blockIdx.x);
}

// Four consecutive storage elements as floats (8- or 16-byte load).
template <typename T> __device__ __forceinline__ void load4(const T *p, float *f);
template <> __device__ __forceinline__ void load4<float>(const float *p, float *f) {
    const float4 v = *reinterpret_cast<const float4 *>(p);
    f[0] = v.x;
    f[1] = v.y;
    f[2] = v.z;
    f[3] = v.w;
}
template <> __device__ __forceinline__ void load4<bf16_t>(const bf16_t *p, float *f) {
    const uint2 v = *reinterpret_cast<const uint2 *>(p);
    f[0] = __uint_as_float(v.x << 16);
    f[1] = __uint_as_float(v.x & 0xffff0000u);
    f[2] = __uint_as_float(v.y << 16);
    f[3] = __uint_as_float(v.y & 0xffff0000u);
}
template <> __device__ __forceinline__ void load4<f16_t>(const f16_t *p, float *f) {
    const uint2 v = *reinterpret_cast<const uint2 *>(p);
    f[0] = (float)__builtin_bit_cast(f16_t, (uint16_t)(v.x & 0xffffu));
    f[1] = (float)__builtin_bit_cast(f16_t, (uint16_t)(v.x >> 16));
    f[2] = (float)__builtin_bit_cast(f16_t, (uint16_t)(v.y & 0xffffu));
    f[3] = (float)__builtin_bit_cast(f16_t, (uint16_t)(v.y >> 16));
}

// out[perm[k], c] = sigma(a_c T_k,c + b_c), c < d; one thread per four columns.
template <typename T, int D>
__global__ __launch_bounds__(THREADS) void epilogue_kernel(int64_t N, int d,
                                                           const void *__restrict__ Wv,
                                                           const float4 *__restrict__ node,
                                                           const float *__restrict__ ab,
                                                           const int32_t *__restrict__ perm,
                                                           float *__restrict__ out) {
    constexpr int NQ = D / 4;
    const int64_t gl = block_index() * THREADS + threadIdx.x;
    const int64_t k = gl / NQ;
    const int c0 = (int)(gl % NQ) * 4;
    if (k >= N || c0 >= d) return;
    float t[4];
    load4<T>((const T *)Wv + k * D + c0, t);
    const float sq = node[k].y;
    float z[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float x = fmaf(ab[c0 + e], t[e] * sq, ab[D + c0 + e]);
        z[e] = 1.0f / (1.0f + expf(-x));
    }
    float *o = out + (int64_t)perm[k] * d + c0;
    if ((d & 3) == 0) {  // streaming store: the output is not read again here
        typedef float f4v_t __attribute__((ext_vector_type(4)));
        const f4v_t v = {z[0], z[1], z[2], z[3]};
        __builtin_nontemporal_store(v, reinterpret_cast<f4v_t *>(o));
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (c0 + e < d) o[e] = z[e];
    }
}

// ---------------------------------------------------------------- host side


#define IFGP_WIDTHS(T, Dp, CALL)                                  \
    switch (Dp) {                                                 \
    case 8: return CALL(T, 8);                                    \
    case 16: return CALL(T, 16);                                  \
    case 32: return CALL(T, 32);                                  \
    case 64: return CALL(T, 64);                                  \
    case 128: return CALL(T, 128);                                \
    case 256: return CALL(T, 256);                                \
    default: break;                                               \
    }

#define IFGP_DISPATCH(storage, Dp, CALL)                          \
    do {                                                          \
        switch (storage) {                                        \
        case IFGP_F32: IFGP_WIDTHS(float, Dp, CALL) break;        \
        case IFGP_BF16: IFGP_WIDTHS(bf16_t, Dp, CALL) break;      \
        case IFGP_F16: IFGP_WIDTHS(f16_t, Dp, CALL) break;        \
        default: break;                                           \
        }                                                         \
    } while (0)

HopArgs make_hop_args(ifgp_graph_s *h) {
    const GraphData &g = h->g;
    const Job &j = h->job;
    HopArgs a{};
    a.rowptr = g.irowptr.as<int64_t>();
    a.colidx = g.icolidx.as<int32_t>();
    a.Win = h->mem.feat[j.cur];
    a.Wout = h->mem.feat[1 - j.cur];
    a.node = h->mem.node;
    a.ab = h->mem.ab;
    a.partials = h->mem.partials;
    a.N = g.N;
    a.n_hub = g.n_hub;
    a.n_med = g.n_med;
    a.blk_hub_end = g.n_hub;
    a.blk_med_end = g.n_hub + ceil_div(g.n_med, MED_ROWS_PER_BLOCK);
    a.blocks = hop_blocks(g, j.Dp, j.storage);
    a.light_rows = light_rows(g, j.Dp, j.storage);
    a.alpha = (float)j.alpha;
    a.theta = (float)j.theta;
    return a;
}

FinArgs make_fin_args(ifgp_graph_s *h) {
    FinArgs f{};
    f.partials = h->mem.partials;
    f.blocks = hop_blocks(h->g, h->job.Dp, h->job.storage);
    f.N = h->g.N;
    f.D = h->job.Dp;
    f.ddof = h->job.ddof;
    f.ab = h->mem.ab;
    return f;
}

// The gather depth of a graph's hops (see Cfg): 2-byte feature matrices of
// at most 32 MiB gather deep, those of 224 MiB or more with rows of 64
// columns or more shallow.  It depends on the graph only, so a graph's
// result is the same alone and in any batch.
constexpr int64_t DEEP_MAX_BYTES = (int64_t)32 << 20;
constexpr int64_t SHALLOW_MIN_BYTES = (int64_t)224 << 20;
// A depth forced by ifgp_debug_hop_depth (-1: chosen per graph as below).
std::atomic<int> g_forced_depth{-1};

int hop_depth(const GraphData &g, int Dp, int storage) {
    if (dtype_bytes(storage) != 2) return DEPTH_NORMAL;
    const int forced = g_forced_depth.load(std::memory_order_relaxed);
    if (forced >= 0) return forced;
    const int64_t bytes = g.N * (int64_t)Dp * 2;
    if (Dp >= 64 && bytes >= SHALLOW_MIN_BYTES) return DEPTH_SHALLOW;
    if (bytes <= DEEP_MAX_BYTES) return DEPTH_DEEP;
    return DEPTH_NORMAL;
}

// Variants other than the normal depth exist only for 2-byte storage (and
// the shallow one for widths >= 64), where they differ.
template <typename T, int D>
ifgp_status hop_launch(const HopArgs &a, int depth, hipStream_t s) {
    if constexpr (sizeof(T) == 2) {
        if constexpr (D >= 64)
            if (depth == DEPTH_SHALLOW) {
                hop_kernel<T, D, DEPTH_SHALLOW><<<grid_for(a.blocks), THREADS, 0, s>>>(a);
                return IFGP_OK;
            }
        if (depth == DEPTH_DEEP) {
            hop_kernel<T, D, DEPTH_DEEP><<<grid_for(a.blocks), THREADS, 0, s>>>(a);
            return IFGP_OK;
        }
    }
    hop_kernel<T, D, DEPTH_NORMAL><<<grid_for(a.blocks), THREADS, 0, s>>>(a);
    return IFGP_OK;
}

template <typename T, int D>
ifgp_status hop_batch_launch(const HopBatch &bt, int64_t total_blocks, int depth,
                             hipStream_t s) {
    if constexpr (sizeof(T) == 2) {
        if constexpr (D >= 64)
            if (depth == DEPTH_SHALLOW) {
                hop_batch_kernel<T, D, DEPTH_SHALLOW><<<grid_for(total_blocks), THREADS, 0, s>>>(bt);
                return IFGP_OK;
            }
        if (depth == DEPTH_DEEP) {
            hop_batch_kernel<T, D, DEPTH_DEEP><<<grid_for(total_blocks), THREADS, 0, s>>>(bt);
            return IFGP_OK;
        }
    }
    hop_batch_kernel<T, D, DEPTH_NORMAL><<<grid_for(total_blocks), THREADS, 0, s>>>(bt);
    return IFGP_OK;
}

ifgp_status launch_hop(const HopArgs &a, int storage, int Dp, int depth, hipStream_t s) {
#define HOP_CALL(T, D) hop_launch<T, D>(a, depth, s)
    IFGP_DISPATCH(storage, Dp, HOP_CALL);
#undef HOP_CALL
    set_error("unsupported storage/width");
    return IFGP_E_INVALID;
}

ifgp_status launch_hop_batch(const HopBatch &bt, int64_t total_blocks, int storage, int Dp,
                             int depth, hipStream_t s) {
#define HOPB_CALL(T, D) hop_batch_launch<T, D>(bt, total_blocks, depth, s)
    IFGP_DISPATCH(storage, Dp, HOPB_CALL);
#undef HOPB_CALL
    set_error("unsupported storage/width");
    return IFGP_E_INVALID;
}

ifgp_status launch_noise(ifgp_graph_s *h, uint64_t seed, const float *X, hipStream_t s) {
    const Job &j = h->job;
    const int64_t n = h->g.N * j.Dp;
    const dim3 grid = grid_for(ceil_div(n, THREADS));
    const dim3 grid4 = grid_for(ceil_div(n / 4, THREADS));
    void *W = h->mem.feat[0];
    const int32_t *perm = h->g.perm.as<int32_t>();
    const double *s64 = h->mem.s64;
    const int64_t N = h->g.N;
    const int d = j.d;
#define NOISE_CALL(T, D)                                                                        \
    (X ? (prep_x_kernel<T, D><<<grid, THREADS, 0, s>>>(N, d, X, perm, s64, (T *)W), IFGP_OK)    \
       : (noise_kernel<T, D><<<grid4, THREADS, 0, s>>>(N, d, seed, perm, s64, (T *)W), IFGP_OK))
    IFGP_DISPATCH(j.storage, j.Dp, NOISE_CALL);
#undef NOISE_CALL
    set_error("unsupported storage/width");
    return IFGP_E_INVALID;
}

ifgp_status launch_epilogue(ifgp_graph_s *h, hipStream_t s) {
    const Job &j = h->job;
    const int64_t N = h->g.N;
    const void *W = h->mem.feat[j.cur];
    const float4 *node = h->mem.node;
    const float *ab = h->mem.ab;
    const int32_t *perm = h->g.perm.as<int32_t>();
    float *out = j.out;
    const int d = j.d;
#define EPI_CALL(T, D)                                                                          \
    (epilogue_kernel<T, D><<<grid_for(ceil_div(N * (D / 4), THREADS)), THREADS, 0, s>>>(        \
         N, d, W, node, ab, perm, out),                                                         \
     IFGP_OK)
    IFGP_DISPATCH(j.storage, j.Dp, EPI_CALL);
#undef EPI_CALL
    set_error("unsupported storage/width");
    return IFGP_E_INVALID;
}

ifgp_status validate_params(const ifgp_params &p) {
    if (!std::isfinite(p.alpha) || !std::isfinite(p.theta) || !(p.eps > 0) ||
        !std::isfinite(p.eps)) {
        set_error("alpha and theta must be finite and eps > 0");
        return IFGP_E_INVALID;
    }
    if (p.znorm_ddof != 0 && p.znorm_ddof != 1) {
        set_error("znorm_ddof must be 0 or 1");
        return IFGP_E_INVALID;
    }
    if (p.storage != IFGP_F32 && p.storage != IFGP_BF16 && p.storage != IFGP_F16) {
        set_error("storage must be IFGP_F32, IFGP_BF16 or IFGP_F16");
        return IFGP_E_INVALID;
    }
    return IFGP_OK;
}

ifgp_status record_event(ifgp_graph_s *h, hipStream_t s, bool start) {
    if (!h->timing || h->job.noalloc) return IFGP_OK;
    hipEvent_t ev;
    IFGP_HIP(hipEventCreate(&ev));
    IFGP_HIP(hipEventRecord(ev, s));
    if (start) h->events.push_back({ev, nullptr});
    else h->events.back().second = ev;
    return IFGP_OK;
}

}  // namespace

namespace {
int rows_per_wave(int Dp, int storage) { return 1024 / ((int)dtype_bytes(storage) * Dp); }
}  // namespace

int light_rows(const GraphData &g, int Dp, int storage) {
    return light_rows_for(g.N - g.n_hub - g.n_med, rows_per_wave(Dp, storage));
}

int64_t hop_blocks(const GraphData &g, int Dp, int storage) {
    const int64_t n_light = g.N - g.n_hub - g.n_med;
    return g.n_hub + ceil_div(g.n_med, MED_ROWS_PER_BLOCK) +
           ceil_div(n_light, light_rows(g, Dp, storage));
}

ifgp_status gaussian_input_device(int64_t N, int32_t d, uint64_t seed, int32_t dtype, void *out,
                                  hipStream_t s) {
    const int64_t n = N * ((d + 3) / 4);
    if (n == 0) return IFGP_OK;
    const dim3 grid = grid_for(ceil_div(n, THREADS));
    switch (dtype) {
    case IFGP_F64: gaussian_kernel<double><<<grid, THREADS, 0, s>>>(N, d, seed, (double *)out); break;
    case IFGP_F32: gaussian_kernel<float><<<grid, THREADS, 0, s>>>(N, d, seed, (float *)out); break;
    case IFGP_BF16: gaussian_kernel<bf16_t><<<grid, THREADS, 0, s>>>(N, d, seed, (bf16_t *)out); break;
    case IFGP_F16: gaussian_kernel<f16_t><<<grid, THREADS, 0, s>>>(N, d, seed, (f16_t *)out); break;
    default: set_error("unsupported dtype"); return IFGP_E_INVALID;
    }
    IFGP_LAUNCHED();
    return IFGP_OK;
}

namespace {
// s in FP64 and FP32 (cheap) into m.s64, m.s32; the node info (the neighbour
// sums r) follows from them.
ifgp_status launch_scales(const GraphData &g, const EmbedMem &m, double tau, double eps,
                          hipStream_t s) {
    scales_kernel<<<grid_for(ceil_div(g.N, THREADS)), THREADS, 0, s>>>(
        g.N, g.irowptr.as<int64_t>(), tau, eps, m.s64, m.s32);
    IFGP_LAUNCHED();
    return IFGP_OK;
}

ifgp_status launch_nodeinfo(const GraphData &g, const EmbedMem &m, double tau, double eps,
                            hipStream_t s) {
    const int64_t n_heavy = g.n_hub + g.n_med;
    const int64_t heavy_groups = ceil_div(n_heavy, THREADS / 64);
    const int64_t groups = heavy_groups + ceil_div(g.N - n_heavy, THREADS / NI_LANES);
    if (g.N >= NI_TABLE_MIN_NODES) {
        const int sh = ni_shift(g.N);
        const int64_t ntab = ceil_div(g.N, (int64_t)1 << sh);
        s_table_kernel<<<(unsigned)ceil_div(ntab, THREADS), THREADS, 0, s>>>(
            g.N, sh, ntab, g.irowptr.as<int64_t>(), m.s32, m.stab);
        IFGP_LAUNCHED();
        nodeinfo_kernel<true><<<(unsigned)std::min<int64_t>(groups, NI_GRID), THREADS, 0, s>>>(
            g.N, n_heavy, heavy_groups, groups, g.irowptr.as<int64_t>(), g.icolidx.as<int32_t>(),
            m.s64, m.s32, m.stab, (int)ntab, sh, tau, eps, m.node);
    } else {
        // one block per group (N < 2^19: at most 2^17 groups)
        nodeinfo_kernel<false><<<(unsigned)groups, THREADS, 0, s>>>(
            g.N, n_heavy, heavy_groups, groups, g.irowptr.as<int64_t>(), g.icolidx.as<int32_t>(),
            m.s64, m.s32, nullptr, 0, 0, tau, eps, m.node);
    }
    IFGP_LAUNCHED();
    return IFGP_OK;
}

// The handle's cached scales: buffers sized for the graph (invalid until
// their node info is launched).
ifgp_status ensure_scale_bufs(ifgp_graph_s *h, hipStream_t s) {
    Scales &sc = h->sc;
    const int64_t N = h->g.N;
    sc.valid = false;
    IFGP_TRY(ensure(sc.s64, sizeof(double) * N, s));
    IFGP_TRY(ensure(sc.s32, sizeof(float) * N, s));
    IFGP_TRY(ensure(sc.nodeinfo, sizeof(float4) * N, s));
    if (N >= NI_TABLE_MIN_NODES) IFGP_TRY(ensure(sc.stab, sizeof(float) * NI_TABLE, s));
    return IFGP_OK;
}

EmbedMem scale_view(const Scales &sc) {
    EmbedMem m;
    m.s64 = sc.s64.as<double>();
    m.s32 = sc.s32.as<float>();
    m.node = sc.nodeinfo.as<float4>();
    m.stab = sc.stab.as<float>();
    return m;
}

void mark_scales(Scales &sc, double tau, double eps) {
    sc.tau = tau;
    sc.eps = eps;
    sc.valid = true;
}

bool scales_cached(const ifgp_graph_s *h, double tau, double eps) {
    return h->sc.valid && h->sc.tau == tau && h->sc.eps == eps;
}

// Independent kernels overlap on a library-owned stream, one per device,
// created once and kept for the life of the process; the fork and join
// events belong to the handle.
std::mutex g_aux_mu;
hipStream_t g_aux[64] = {};

ifgp_status ensure_aux(ifgp_graph_s *h) {
    if (!h->aux) {
        if (h->device < 0 || h->device >= 64) {
            set_error("device index out of range");
            return IFGP_E_DEVICE;
        }
        std::lock_guard<std::mutex> lk(g_aux_mu);
        if (!g_aux[h->device])
            IFGP_HIP(hipStreamCreateWithFlags(&g_aux[h->device], hipStreamNonBlocking));
        h->aux = g_aux[h->device];
    }
    if (!h->ev_fork) IFGP_HIP(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
    if (!h->ev_join) IFGP_HIP(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
    return IFGP_OK;
}

// Below this many nodes the random input and the neighbour sums are short
// and run one after the other on the caller's stream.
constexpr int64_t OVERLAP_MIN_NODES = 65536;
}  // namespace

ifgp_status ensure_side_stream(ifgp_graph_s *h) { return ensure_aux(h); }

int force_hop_depth(int depth) { return g_forced_depth.exchange(depth); }

ifgp_status ensure_scales(ifgp_graph_s *h, double tau, double eps, hipStream_t s) {
    if (scales_cached(h, tau, eps)) return IFGP_OK;
    if (h->job.active && !h->job.done && !h->job.noalloc) {
        // the unfinished job's hops read the cached node info
        set_error("the graph has an unfinished job with other scales");
        return IFGP_E_STATE;
    }
    IFGP_TRY(ensure_scale_bufs(h, s));
    const EmbedMem m = scale_view(h->sc);
    IFGP_TRY(launch_scales(h->g, m, tau, eps, s));
    IFGP_TRY(launch_nodeinfo(h->g, m, tau, eps, s));
    mark_scales(h->sc, tau, eps);
    return IFGP_OK;
}

ifgp_status scales_to_host(ifgp_graph_s *h, double *s_host, hipStream_t s) {
    const int64_t N = h->g.N;
    Buf tmp;
    IFGP_TRY(alloc(tmp, sizeof(double) * N, s));
    perm_scales_kernel<<<grid_for(ceil_div(N, THREADS)), THREADS, 0, s>>>(
        N, h->g.perm.as<int32_t>(), h->sc.s64.as<double>(), tmp.as<double>());
    IFGP_LAUNCHED();
    IFGP_HIP(hipMemcpyAsync(s_host, tmp.p, sizeof(double) * N, hipMemcpyDeviceToHost, s));
    IFGP_HIP(hipStreamSynchronize(s));
    return IFGP_OK;
}

// Device memory that only the allocation-free entry point uses
// (NOALLOC_SCRATCH_BYTES).  Each device holds its own copy for the life of the
// process.  Host code never uses this name as an address: it reaches the
// array only through the pointer hipGetSymbolAddress returns for the current
// device (scratch_address below).
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
ifgp_status check_job_args(double tau, int32_t K, int32_t d, const ifgp_params &p, float *out) {
    IFGP_TRY(validate_params(p));
    if (!std::isfinite(tau)) {
        set_error("tau must be finite");
        return IFGP_E_INVALID;
    }
    if (K < 0 || d < 1 || d > 256 || !out) {
        set_error("need K >= 0, 1 <= d <= 256 and an output buffer");
        return IFGP_E_INVALID;
    }
    return IFGP_OK;
}

// Launch the start of a job whose buffers are in h->mem: the scales if
// fresh_scales (their node info may overlap the random input on the side
// stream when `overlap`), Z^(0), a = 1, b = 0, and at K = 0 the output.
ifgp_status job_start(ifgp_graph_s *h, bool fresh_scales, bool overlap, double tau, int32_t K,
                      int32_t d, uint64_t seed, const float *X, const ifgp_params &p, float *out,
                      hipStream_t s) {
    const GraphData &g = h->g;
    Job &j = h->job;
    j.K = K;
    j.d = d;
    j.Dp = padded_width(d);
    j.hop = 0;
    j.storage = p.storage;
    j.alpha = p.alpha;
    j.theta = p.theta;
    j.ddof = p.znorm_ddof;
    j.cur = 0;
    j.out = out;
    if (fresh_scales) IFGP_TRY(launch_scales(g, h->mem, tau, p.eps, s));
    if (fresh_scales && overlap && !X && g.N >= OVERLAP_MIN_NODES) {
        // The random input needs only s; it is arithmetic-bound while the
        // neighbour sums are gather-bound, so run them side by side.
        IFGP_TRY(ensure_aux(h));
        IFGP_HIP(hipEventRecord(h->ev_fork, s));
        IFGP_HIP(hipStreamWaitEvent(h->aux, h->ev_fork, 0));
        IFGP_TRY(launch_noise(h, seed, X, h->aux));
        IFGP_LAUNCHED();
        IFGP_HIP(hipEventRecord(h->ev_join, h->aux));
        IFGP_TRY(launch_nodeinfo(g, h->mem, tau, p.eps, s));
        IFGP_HIP(hipStreamWaitEvent(s, h->ev_join, 0));
    } else {
        if (fresh_scales) IFGP_TRY(launch_nodeinfo(g, h->mem, tau, p.eps, s));
        IFGP_TRY(launch_noise(h, seed, X, s));
        IFGP_LAUNCHED();
    }
    ab_identity_kernel<<<1, THREADS, 0, s>>>(h->mem.ab, j.Dp);
    IFGP_LAUNCHED();
    j.active = true;
    if (K == 0) {
        IFGP_TRY(launch_epilogue(h, s));
        IFGP_LAUNCHED();
        j.done = true;
    }
    return IFGP_OK;
}

// The allocation-free embedding's buffers, carved in this order out of the
// static array, each starting on a 256-byte boundary.
struct ScratchLayout {
    size_t s64, s32, node, stab, feat0, feat1, partials, ab, total;
};

ScratchLayout scratch_layout(int64_t N, int Dp, int storage, int64_t blocks) {
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    ScratchLayout L{};
    size_t o = 0;
    L.s64 = o;      o += up(sizeof(double) * N);
    L.s32 = o;      o += up(sizeof(float) * N);
    L.node = o;     o += up(sizeof(float4) * N);
    L.stab = o;     o += up(sizeof(float) * NI_TABLE);
    const size_t fb = up((size_t)N * Dp * dtype_bytes(storage));
    L.feat0 = o;    o += fb;
    L.feat1 = o;    o += fb;
    L.partials = o; o += up(sizeof(double2) * Dp * blocks);
    L.ab = o;       o += up(sizeof(float) * 2 * Dp);
    L.total = o;
    return L;
}

std::mutex g_scratch_mu;
void *g_scratch_dev[64] = {};

// The scratch array's address on `device`, which must be current.
ifgp_status scratch_address(int device, unsigned char **out) {
    if (device < 0 || device >= 64) {
        set_error("device index out of range");
        return IFGP_E_DEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void *ptr = nullptr;
        IFGP_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) {
            set_error("hipGetSymbolAddress returned no address for the scratch array");
            return IFGP_E_DEVICE;
        }
        g_scratch_dev[device] = ptr;
    }
    *out = static_cast<unsigned char *>(g_scratch_dev[device]);
    return IFGP_OK;
}
}  // namespace

ifgp_status job_begin(ifgp_graph_s *h, double tau, int32_t K, int32_t d, uint64_t seed,
                      const float *X, const ifgp_params &p, float *out, hipStream_t s) {
    IFGP_TRY(check_job_args(tau, K, d, p, out));
    const int Dp = padded_width(d);
    h->job = Job{};
    const bool fresh_scales = !scales_cached(h, tau, p.eps);
    if (fresh_scales) IFGP_TRY(ensure_scale_bufs(h, s));
    const GraphData &g = h->g;
    const size_t fb = (size_t)g.N * Dp * dtype_bytes(p.storage);
    IFGP_TRY(ensure(h->ws.feat[0], fb, s));
    IFGP_TRY(ensure(h->ws.feat[1], fb, s));
    IFGP_TRY(ensure(h->ws.partials, sizeof(double2) * Dp * hop_blocks(g, Dp, p.storage), s));
    IFGP_TRY(ensure(h->ws.ab, sizeof(float) * 2 * Dp, s));
    EmbedMem m = scale_view(h->sc);
    m.feat[0] = h->ws.feat[0].p;
    m.feat[1] = h->ws.feat[1].p;
    m.partials = h->ws.partials.as<double2>();
    m.ab = h->ws.ab.as<float>();
    h->mem = m;
    IFGP_TRY(job_start(h, fresh_scales, true, tau, K, d, seed, X, p, out, s));
    if (fresh_scales) mark_scales(h->sc, tau, p.eps);
    return IFGP_OK;
}

ifgp_status job_begin_noalloc(ifgp_graph_s *h, double tau, int32_t K, int32_t d, uint64_t seed,
                              const ifgp_params &p, float *out, hipStream_t s) {
    IFGP_TRY(check_job_args(tau, K, d, p, out));
    const int Dp = padded_width(d);
    const GraphData &g = h->g;
    const ScratchLayout L = scratch_layout(g.N, Dp, p.storage, hop_blocks(g, Dp, p.storage));
    if (L.total > NOALLOC_SCRATCH_BYTES) {
        set_error("ifgp_embed_noalloc: N = %lld at width %d in this storage needs %zu bytes of "
                  "scratch, above the limit of %zu",
                  (long long)g.N, Dp, L.total, NOALLOC_SCRATCH_BYTES);
        return IFGP_E_INVALID;
    }
    unsigned char *base = nullptr;
    IFGP_TRY(scratch_address(h->device, &base));
    h->job = Job{};
    EmbedMem m;
    m.s64 = reinterpret_cast<double *>(base + L.s64);
    m.s32 = reinterpret_cast<float *>(base + L.s32);
    m.node = reinterpret_cast<float4 *>(base + L.node);
    m.stab = reinterpret_cast<float *>(base + L.stab);
    m.feat[0] = base + L.feat0;
    m.feat[1] = base + L.feat1;
    m.partials = reinterpret_cast<double2 *>(base + L.partials);
    m.ab = reinterpret_cast<float *>(base + L.ab);
    h->mem = m;
    h->job.noalloc = true;
    // the scales are recomputed into the scratch array; the handle's cached
    // ones are neither read nor touched
    return job_start(h, true, false, tau, K, d, seed, nullptr, p, out, s);
}

ifgp_status jobs_step(ifgp_graph_s **hs, int n, hipStream_t s) {
    // Group unfinished jobs by (storage, width, gather depth); one hop launch
    // and one finalize launch per group.  A graph's gather depth depends on
    // the graph only, so its result is the same alone and in any batch.
    struct Group {
        int storage, Dp, depth;
        std::vector<ifgp_graph_s *> members;
    };
    std::vector<Group> groups;
    for (int i = 0; i < n; ++i) {
        ifgp_graph_s *h = hs[i];
        if (!h->job.active || h->job.done) continue;
        const int dep = hop_depth(h->g, h->job.Dp, h->job.storage);
        Group *gp = nullptr;
        for (auto &G : groups)
            if (G.storage == h->job.storage && G.Dp == h->job.Dp && G.depth == dep) gp = &G;
        if (!gp) {
            groups.push_back({h->job.storage, h->job.Dp, dep, {}});
            gp = &groups.back();
        }
        gp->members.push_back(h);
    }
    for (auto &G : groups) {
        if (G.members.size() == 1) {
            ifgp_graph_s *h = G.members[0];
            const HopArgs a = make_hop_args(h);
            IFGP_TRY(record_event(h, s, true));
            IFGP_TRY(launch_hop(a, G.storage, G.Dp, G.depth, s));
            IFGP_LAUNCHED();
            IFGP_TRY(record_event(h, s, false));
            const FinArgs f = make_fin_args(h);
            finalize_kernel<<<(unsigned)G.Dp, FIN_THREADS, 0, s>>>(f);
            IFGP_LAUNCHED();
        } else {
            const int m = (int)G.members.size();
            for (int b0 = 0; b0 < m; b0 += MAX_BATCH) {
                const int nb = std::min(MAX_BATCH, m - b0);
                HopBatch bt{};
                FinBatch fb{};
                bt.n = nb;
                bt.start[0] = 0;
                for (int i = 0; i < nb; ++i) {
                    bt.a[i] = make_hop_args(G.members[b0 + i]);
                    fb.f[i] = make_fin_args(G.members[b0 + i]);
                    bt.start[i + 1] = bt.start[i] + bt.a[i].blocks;
                }
                for (int i = 0; i < nb; ++i) IFGP_TRY(record_event(G.members[b0 + i], s, true));
                IFGP_TRY(launch_hop_batch(bt, bt.start[nb], G.storage, G.Dp, G.depth, s));
                IFGP_LAUNCHED();
                for (int i = 0; i < nb; ++i) IFGP_TRY(record_event(G.members[b0 + i], s, false));
                finalize_batch_kernel<<<dim3((unsigned)G.Dp, (unsigned)nb), FIN_THREADS, 0, s>>>(fb);
                IFGP_LAUNCHED();
            }
        }
        for (auto *h : G.members) {
            Job &j = h->job;
            j.cur = 1 - j.cur;
            j.hop += 1;
            if (j.hop >= j.K) {
                IFGP_TRY(launch_epilogue(h, s));
                IFGP_LAUNCHED();
                j.done = true;
            }
        }
    }
    return IFGP_OK;
}

}  // namespace ifgp
