// Internal helpers shared by the libifgp translation units: error reporting,
// device buffers drawn from the allocator hook, storage-type traits.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <utility>

#include "ifgp.h"

namespace ifgp {

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);

#define IFGP_TRY(expr)                                   \
    do {                                                 \
        ifgp_status _st = (expr);                        \
        if (_st != IFGP_OK) return _st;                  \
    } while (0)

#define IFGP_HIP(expr)                                                                      \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess) {                                                             \
            ::ifgp::set_error("%s: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__,     \
                              __LINE__);                                                    \
            return IFGP_E_DEVICE;                                                           \
        }                                                                                   \
    } while (0)

// Check the launch that was just enqueued.
#define IFGP_LAUNCHED() IFGP_HIP(hipGetLastError())

// ---------------------------------------------------------------- memory
// Release function of the allocator that produced a block: every buffer frees
// through the allocator it came from, even if the hook changes meanwhile.
using FreeFn = void (*)(void *, void *, void *);
void *raw_alloc(size_t bytes, hipStream_t s, FreeFn *free_fn, void **ctx);
void raw_free(void *p, hipStream_t s, FreeFn free_fn, void *ctx);

// Owning device buffer; memory comes from the allocator hook (default: the
// device's stream-ordered memory pool).
struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
    hipStream_t s = nullptr;
    FreeFn free_fn = nullptr;
    void *ctx = nullptr;

    Buf() = default;
    Buf(const Buf &) = delete;
    Buf &operator=(const Buf &) = delete;
    Buf(Buf &&o) noexcept { swap(o); }
    Buf &operator=(Buf &&o) noexcept {
        if (this != &o) {
            reset();
            swap(o);
        }
        return *this;
    }
    ~Buf() { reset(); }

    void swap(Buf &o) noexcept {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
        std::swap(s, o.s);
        std::swap(free_fn, o.free_fn);
        std::swap(ctx, o.ctx);
    }
    void reset() {
        if (p) raw_free(p, s, free_fn, ctx);
        p = nullptr;
        bytes = 0;
        free_fn = nullptr;
        ctx = nullptr;
    }
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

// Allocate `bytes` (at least 256 so that empty arrays still have an address).
ifgp_status alloc(Buf &b, size_t bytes, hipStream_t s);
// Keep b if it already holds >= bytes, else reallocate.
ifgp_status ensure(Buf &b, size_t bytes, hipStream_t s);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------- grids
// A launch holds at most 2^32 - 1 work items per grid dimension, which a
// kernel with one thread per entry of an N x d matrix, or one block per few
// rows, passes on graphs that still fit in device memory.  Such kernels take
// their grid from grid_for: at most grid_x_blocks() blocks in x (2^21, so
// that blocks of up to 1024 threads stay below 2^31 work items), the rest in
// y, and x widened so that y stays below 65536.  The kernel reads its linear
// block index from block_index(); the blocks past the requested count (at the
// end of the last y row) must leave at once.
constexpr int64_t GRID_X_BLOCKS = int64_t(1) << 21;
int64_t grid_x_blocks();  // GRID_X_BLOCKS unless lowered by ifgp_debug_grid_x
inline dim3 grid_for(int64_t blocks) {
    int64_t x = grid_x_blocks();
    if (blocks <= x) return dim3((unsigned)blocks);
    const int64_t xmin = ceil_div(blocks, 65535);
    if (x < xmin) x = xmin;
    return dim3((unsigned)x, (unsigned)ceil_div(blocks, x));
}
__device__ __forceinline__ int64_t block_index() {
    return (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
}

// ---------------------------------------------------------------- storage types
struct bf16_t {
    uint16_t x;
};
using f16_t = _Float16;

__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(f16_t v) { return (float)v; }
__device__ __forceinline__ float to_f32(bf16_t v) { return __uint_as_float(((uint32_t)v.x) << 16); }

template <typename T> __device__ __forceinline__ T from_f32(float v);
template <> __device__ __forceinline__ float from_f32<float>(float v) { return v; }
template <> __device__ __forceinline__ f16_t from_f32<f16_t>(float v) { return (f16_t)v; }
// Round to nearest even; NaN stays NaN.
template <> __device__ __forceinline__ bf16_t from_f32<bf16_t>(float v) {
    uint32_t u = __float_as_uint(v);
    bf16_t r;
    if ((u & 0x7fffffffu) > 0x7f800000u) {
        r.x = (uint16_t)((u >> 16) | 0x40u);
    } else {
        u += 0x7fffu + ((u >> 16) & 1u);
        r.x = (uint16_t)(u >> 16);
    }
    return r;
}

inline size_t dtype_bytes(int dt) {
    switch (dt) {
    case IFGP_F32: return 4;
    case IFGP_BF16: return 2;
    case IFGP_F16: return 2;
    case IFGP_F64: return 8;
    default: return 0;
    }
}

// Padded feature width: the smallest supported kernel width >= d.
inline int padded_width(int d) {
    static const int widths[] = {8, 16, 32, 64, 128, 256};
    for (int w : widths)
        if (d <= w) return w;
    return 0;
}

// Bits needed to hold the value v (v >= 1 -> floor(log2 v) + 1).
inline int bit_width(uint64_t v) {
    int b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

}  // namespace ifgp
