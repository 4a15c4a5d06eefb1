// BIRCH, the clustering step that turns the FFP's embeddings into a
// K-agnostic partition (Sec. III, Algorithm 1 final step; Algorithm 2 fits it
// partially for streaming).  The algorithm is that of Zhang, Ramakrishnan &
// Livny (SIGMOD 1996) in the configuration the paper runs: no preset number
// of clusters, radius threshold, one branching factor for every node.
//
//   host    the CF-tree.  Insertion is sequential by definition (each point
//           descends the tree the previous points left), and one insertion
//           touches at most B entries per level, so it stays on the host in
//           FP64 (rules in ifgp.h).
//   device  labelling: every point against every leaf-entry centroid, a
//           dense N x M x d contraction with an argmin, on the FP64 matrix
//           cores (the same precision as the tree's own decisions).
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <utility>
#include <vector>

#include "internal.h"

namespace ifgp {
namespace {

constexpr int NB = 16;  // entries per block of the coordinate-major centroid copy
typedef double v4_t __attribute__((ext_vector_type(4)));

struct BNode {
    bool leaf = true;
    std::vector<int64_t> n;   // per entry: points
    std::vector<double> ls;   // per entry: linear sum (d)
    std::vector<double> ss;   // per entry: sum of squared norms
    std::vector<double> c;    // per entry: centroid ls / n (d)
    std::vector<double> cn;   // per entry: |centroid|^2
    std::vector<double> ct;   // the centroids again in blocks of NB entries, coordinate-major
                              // inside a block: entry k, coordinate j at
                              // ct[((k / NB) * d + j) * NB + k % NB]
    int cap = 0;              // entries ct has room for (B + 1 rounded up to a block)
    std::vector<BNode *> child;
    BNode *prev_leaf = nullptr, *next_leaf = nullptr;
    int size() const { return (int)n.size(); }
};

inline double dot(const double *a, const double *b, int d) {
    double s = 0.0;
    for (int k = 0; k < d; ++k) s += a[k] * b[k];
    return s;
}

// c_k . p for the NB entries of one block at once (the block is NB * d
// contiguous doubles, coordinate-major): every entry's sum runs over the
// coordinates in order, exactly as dot() (separate multiply and add, no fused
// multiply-add), so the result is the same to the last bit; the entries only
// share the vector lanes.
__attribute__((always_inline)) inline void dots_block(const double *blk, const double *p, int d,
                                                      double *out) {
    v4_t s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int j = 0; j < d; ++j) {
        const double *r = blk + (size_t)j * NB;
        v4_t c0, c1, c2, c3;
        std::memcpy(&c0, r, sizeof(v4_t));
        std::memcpy(&c1, r + 4, sizeof(v4_t));
        std::memcpy(&c2, r + 8, sizeof(v4_t));
        std::memcpy(&c3, r + 12, sizeof(v4_t));
        const v4_t pj = p[j];
        s0 = s0 + c0 * pj;
        s1 = s1 + c1 * pj;
        s2 = s2 + c2 * pj;
        s3 = s3 + c3 * pj;
    }
    std::memcpy(out, &s0, sizeof(v4_t));
    std::memcpy(out + 4, &s1, sizeof(v4_t));
    std::memcpy(out + 8, &s2, sizeof(v4_t));
    std::memcpy(out + 12, &s3, sizeof(v4_t));
}

__attribute__((always_inline)) inline int nearest_body(const double *ct, const double *cn, int m,
                                                       const double *p, int d) {
    double dots[NB];
    int best = 0;
    double bd = 0.0;
    for (int k0 = 0; k0 < m; k0 += NB) {
        dots_block(ct + (size_t)k0 * d, p, d, dots);
        const int e = m - k0 < NB ? m - k0 : NB;
        for (int l = 0; l < e; ++l) {
            const double dk = cn[k0 + l] - 2.0 * dots[l];
            if (k0 + l == 0 || dk < bd) {
                bd = dk;
                best = k0 + l;
            }
        }
    }
    return best;
}

// c_k . p for every entry k < m (out has room for m rounded up to NB).
__attribute__((always_inline)) inline void dots_body(const double *ct, int m, const double *p,
                                                     int d, double *out) {
    for (int k0 = 0; k0 < m; k0 += NB) dots_block(ct + (size_t)k0 * d, p, d, out + k0);
}

__attribute__((target("avx2"))) int nearest_avx2(const double *ct, const double *cn, int m,
                                                 const double *p, int d) {
    return nearest_body(ct, cn, m, p, d);
}
__attribute__((target("avx2"))) void dots_avx2(const double *ct, int m, const double *p, int d,
                                               double *out) {
    dots_body(ct, m, p, d, out);
}
int nearest_base(const double *ct, const double *cn, int m, const double *p, int d) {
    return nearest_body(ct, cn, m, p, d);
}
void dots_base(const double *ct, int m, const double *p, int d, double *out) {
    dots_body(ct, m, p, d, out);
}

using nearest_fn = int (*)(const double *, const double *, int, const double *, int);
using dots_fn = void (*)(const double *, int, const double *, int, double *);
bool use_avx2() {
    static const bool yes = __builtin_cpu_supports("avx2");  // known by the first call
    return yes;
}


}  // namespace
}  // namespace ifgp

struct ifgp_birch_s {
    int d = 0;
    double T = 0;
    int B = 0;
    std::vector<std::unique_ptr<ifgp::BNode>> pool;
    ifgp::BNode *root = nullptr, *first_leaf = nullptr;
    int64_t points = 0;
    int height = 0;
    int64_t clusters = 0;
    // device copy of the leaf centroids (M x Dp, zero padded) and their norms
    ifgp::Buf centers;
    int Dp = 0;
    bool dirty = true;
    int device = -1;
    bool broken = false;  // a host allocation failed part-way through an insertion
};

namespace ifgp {
namespace {

BNode *new_node(ifgp_birch_s *t, bool leaf) {
    t->pool.emplace_back(new BNode());
    BNode *x = t->pool.back().get();
    x->leaf = leaf;
    x->cap = (t->B + 1 + NB - 1) / NB * NB;
    x->ct.assign((size_t)x->cap * t->d, 0.0);
    // room for B + 1 entries up front: appends never reallocate
    x->n.reserve(t->B + 1);
    x->ls.reserve((size_t)(t->B + 1) * t->d);
    x->ss.reserve(t->B + 1);
    x->c.reserve((size_t)(t->B + 1) * t->d);
    x->cn.reserve(t->B + 1);
    x->child.reserve(t->B + 1);
    return x;
}

// Entry k's centroid and its squared norm from its CF.
void refresh(BNode *x, int k, int d) {
    double *c = &x->c[(size_t)k * d];
    const double *ls = &x->ls[(size_t)k * d];
    const double nk = (double)x->n[k];
    for (int j = 0; j < d; ++j) c[j] = ls[j] / nk;
    double *blk = &x->ct[(size_t)(k / NB) * NB * d + k % NB];
    for (int j = 0; j < d; ++j) blk[(size_t)j * NB] = c[j];
    x->cn[k] = dot(c, c, d);
}

void append(BNode *x, int d, int64_t n, const double *ls, double ss, BNode *child) {
    x->n.push_back(n);
    x->ls.insert(x->ls.end(), ls, ls + d);
    x->ss.push_back(ss);
    x->c.resize(x->c.size() + d);
    x->cn.push_back(0.0);
    x->child.push_back(child);
    refresh(x, x->size() - 1, d);
}

// CF of a whole node (its entries summed in order).
void summary(const BNode *x, int d, int64_t &n, std::vector<double> &ls, double &ss) {
    n = 0;
    ss = 0.0;
    ls.assign(d, 0.0);
    for (int k = 0; k < x->size(); ++k) {
        n += x->n[k];
        for (int j = 0; j < d; ++j) ls[j] += x->ls[(size_t)k * d + j];
        ss += x->ss[k];
    }
}

// Ask for the blocks the next nearest() will read, all at once.
inline void prefetch_node(const BNode *x, int d) {
    const char *a = (const char *)x->ct.data();
    const size_t bytes = (size_t)((x->size() + NB - 1) / NB) * NB * d * sizeof(double);
    for (size_t o = 0; o < bytes; o += 64) __builtin_prefetch(a + o);
    const char *c = (const char *)x->cn.data();
    for (size_t o = 0; o < x->cn.size() * sizeof(double); o += 64) __builtin_prefetch(c + o);
}

// The entry whose centroid is nearest to p (first on ties), by
// |c_k|^2 - 2 c_k . p.
int nearest(const BNode *x, const double *p, int d) {
    static const nearest_fn impl = use_avx2() ? nearest_avx2 : nearest_base;
    return impl(x->ct.data(), x->cn.data(), x->size(), p, d);
}

// Split x around its farthest pair of centroids; a and b replace x (in the
// leaf order too).
std::pair<BNode *, BNode *> split(ifgp_birch_s *t, BNode *x) {
    const int d = t->d, k = x->size();
    static const dots_fn dots = use_avx2() ? dots_avx2 : dots_base;
    std::vector<double> up((size_t)k * k, 0.0);  // squared distances, i < j
    std::vector<double> row((size_t)x->cap);
    int p = 0, q = 1;
    double far = -1.0;
    for (int i = 0; i < k; ++i) {
        dots(x->ct.data(), k, &x->c[(size_t)i * d], d, row.data());  // c_j . c_i, all j
        for (int j = i + 1; j < k; ++j) {
            double v = (x->cn[i] + x->cn[j]) - 2.0 * row[j];
            if (v < 0.0) v = 0.0;
            up[(size_t)i * k + j] = v;
            if (v > far) {
                far = v;
                p = i;
                q = j;
            }
        }
    }
    auto dist = [&](int i, int j) {
        return i == j ? 0.0 : (i < j ? up[(size_t)i * k + j] : up[(size_t)j * k + i]);
    };
    BNode *a = new_node(t, x->leaf), *b = new_node(t, x->leaf);
    for (int i = 0; i < k; ++i) {
        const bool to_a = i == p || dist(p, i) < dist(q, i);
        append(to_a ? a : b, d, x->n[i], &x->ls[(size_t)i * d], x->ss[i], x->child[i]);
    }
    if (x->leaf) {
        a->prev_leaf = x->prev_leaf;
        a->next_leaf = b;
        b->prev_leaf = a;
        b->next_leaf = x->next_leaf;
        if (x->prev_leaf) x->prev_leaf->next_leaf = a;
        else t->first_leaf = a;
        if (x->next_leaf) x->next_leaf->prev_leaf = b;
    }
    *x = BNode();  // x is out of the tree: drop its storage (the pool keeps the shell)
    return {a, b};
}

// Insert point p (|p|^2 = pp) below x; true if x now holds more than B entries.
bool insert(ifgp_birch_s *t, BNode *x, const double *p, double pp, std::vector<double> &tmp) {
    const int d = t->d;
    if (x->size() == 0) {
        append(x, d, 1, p, pp, nullptr);
        return false;
    }
    const int k = nearest(x, p, d);
    if (!x->leaf) {
        BNode *ch = x->child[k];
        if (insert(t, ch, p, pp, tmp)) {
            auto ab = split(t, ch);
            int64_t n;
            double ss;
            summary(ab.first, d, n, tmp, ss);
            x->n[k] = n;
            std::memcpy(&x->ls[(size_t)k * d], tmp.data(), sizeof(double) * d);
            x->ss[k] = ss;
            x->child[k] = ab.first;
            refresh(x, k, d);
            summary(ab.second, d, n, tmp, ss);
            append(x, d, n, tmp.data(), ss, ab.second);
            return x->size() > t->B;
        }
        x->n[k] += 1;
        for (int j = 0; j < d; ++j) x->ls[(size_t)k * d + j] += p[j];
        x->ss[k] += pp;
        refresh(x, k, d);
        return false;
    }
    // leaf: absorb if the radius stays within the threshold
    const int64_t n1 = x->n[k] + 1;
    tmp.resize(2 * (size_t)d);
    double *ls1 = tmp.data(), *c1 = tmp.data() + d;
    for (int j = 0; j < d; ++j) ls1[j] = x->ls[(size_t)k * d + j] + p[j];
    const double ss1 = x->ss[k] + pp;
    for (int j = 0; j < d; ++j) c1[j] = ls1[j] / (double)n1;
    if (ss1 / (double)n1 - dot(c1, c1, d) <= t->T * t->T) {
        x->n[k] = n1;
        std::memcpy(&x->ls[(size_t)k * d], ls1, sizeof(double) * d);
        x->ss[k] = ss1;
        refresh(x, k, d);
        return false;
    }
    append(x, d, 1, p, pp, nullptr);
    return x->size() > t->B;
}

void insert_point(ifgp_birch_s *t, const double *p, std::vector<double> &tmp) {
    const double pp = dot(p, p, t->d);
    if (insert(t, t->root, p, pp, tmp)) {
        auto ab = split(t, t->root);
        BNode *r = new_node(t, false);
        int64_t n;
        double ss;
        summary(ab.first, t->d, n, tmp, ss);
        append(r, t->d, n, tmp.data(), ss, ab.first);
        summary(ab.second, t->d, n, tmp, ss);
        append(r, t->d, n, tmp.data(), ss, ab.second);
        t->root = r;
        ++t->height;
    }
    ++t->points;
}

int64_t count_clusters(const ifgp_birch_s *t) {
    int64_t m = 0;
    for (const BNode *l = t->first_leaf; l; l = l->next_leaf) m += l->size();
    return m;
}

// ---------------------------------------------------------------- labelling
// Distances of points to centroids are a dense contraction, done on the FP64
// matrix cores: v_mfma_f64_16x16x4f64 multiplies a 16 x 4 block A (16 points,
// 4 coordinates) by a 4 x 16 block B (4 coordinates, 16 centroids).  Lane l
// holds A[l % 16][l / 16] and B[l / 16][l % 16]; the 16 x 16 result D[i][j]
// is in lane j + 16 (i % 4), slot i / 4 (checked on the device).
//
// One wave takes 16 * RB points (RB blocks of 16 rows, their coordinates in
// registers for the whole run) and streams every centroid block's B
// fragments from memory, the next block's while the current one multiplies.
// Each lane keeps the best centroid of its column for each of its rows;
// the 16 lanes of a row group agree at the end (first index on ties).
// Centroids are stored on the device as fragments: for block cb of 16
// centroids and coordinate step s, 64 doubles in lane order; the centroid
// count is padded to a multiple of 16 with zero centroids of norm +inf.
typedef double d4_t __attribute__((ext_vector_type(4)));
constexpr int LW = 4;  // waves per block
constexpr int64_t LABEL_SPARE = 2;  // zero blocks stored after the last centroid block

template <int Dp, int RB>
__global__ __launch_bounds__(64 * LW) void birch_label_kernel(const float *__restrict__ Z,
                                                              int64_t n, int d,
                                                              const double *__restrict__ F,
                                                              const double *__restrict__ cn,
                                                              int64_t nblk,
                                                              int32_t *__restrict__ labels) {
    constexpr int S = Dp / 4;
    const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
    const int64_t p0 = (block_index() * LW + (threadIdx.x >> 6)) * (16 * RB);
    if (p0 >= n) return;  // the whole wave (and every block past the last)
    double a[RB][S];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int64_t p = p0 + 16 * rb + col;
            const int k = 4 * s + grp;
            a[rb][s] = (p < n && k < d) ? (double)Z[p * d + k] : 0.0;
        }
    double best[RB][4];
    int32_t bi[RB][4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            best[rb][r] = __builtin_inf();
            bi[rb][r] = 0;
        }
    // Two register sets take turns: while one block multiplies, the next is
    // loading into the other (unrolled by two, so the loads a block waits
    // for are always the older ones).  The spare blocks keep the loads one
    // and two blocks ahead in bounds, and an odd block count ends on a spare
    // block, whose +inf distances never win: the loop body has no branch.
    double bA[S], bB[S], nA, nB;
    auto load = [&](double *bf, double &nr, int64_t cb) {
#pragma unroll
        for (int s = 0; s < S; ++s) bf[s] = F[(cb * S + s) * 64 + lane];
        nr = cn[cb * 16 + col];
        __builtin_amdgcn_sched_barrier(0);  // issued here, not sunk to their use
    };
    auto step = [&](const double *bf, double nrm, int64_t cb) {
        const int32_t c = (int32_t)(cb * 16 + col);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < S; ++s)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb][s], bf[s], acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double dist = nrm - 2.0 * acc[r];
                if (dist < best[rb][r]) {
                    best[rb][r] = dist;
                    bi[rb][r] = c;
                }
            }
        }
    };
    load(bA, nA, 0);
    for (int64_t cb = 0; cb < nblk; cb += 2) {
        load(bB, nB, cb + 1);
        step(bA, nA, cb);
        load(bA, nA, cb + 2);
        step(bB, nB, cb + 1);
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double v = best[rb][r];
            int32_t i = bi[rb][r];
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                const double ov = __shfl_xor(v, off, 64);
                const int32_t oi = __shfl_xor(i, off, 64);
                if (ov < v || (ov == v && oi < i)) {
                    v = ov;
                    i = oi;
                }
            }
            const int64_t p = p0 + 16 * rb + 4 * r + grp;
            if (col == 0 && p < n) labels[p] = i;
        }
}

int padded_dim(int d) {
    int p = 8;
    while (p < d) p <<= 1;
    return p;
}

ifgp_status upload_centers(ifgp_birch_s *t, hipStream_t s) {
    if (!t->dirty) return IFGP_OK;
    const int d = t->d, Dp = padded_dim(d), S = Dp / 4;
    // two spare blocks (zero centroids of norm +inf) after the last: the
    // kernel loads a block or two ahead without bounds checks
    const int64_t M = t->clusters, Mp = (ceil_div(M, (int64_t)16) + LABEL_SPARE) * 16;
    std::vector<double> h((size_t)Mp * Dp + (size_t)Mp, 0.0);
    double *frag = h.data(), *nrm = h.data() + (size_t)Mp * Dp;
    for (int64_t m = M; m < Mp; ++m) nrm[m] = INFINITY;
    int64_t m = 0;
    for (const BNode *l = t->first_leaf; l; l = l->next_leaf)
        for (int k = 0; k < l->size(); ++k, ++m) {
            const int64_t cb = m / 16, col = m % 16;
            for (int j = 0; j < d; ++j)  // coordinate j = 4 s + grp -> lane col + 16 grp
                frag[((size_t)cb * S + j / 4) * 64 + col + 16 * (j % 4)] = l->c[(size_t)k * d + j];
            nrm[m] = l->cn[k];
        }
    IFGP_TRY(ensure(t->centers, sizeof(double) * h.size(), s));
    IFGP_HIP(hipMemcpyAsync(t->centers.p, h.data(), sizeof(double) * h.size(),
                            hipMemcpyHostToDevice, s));
    IFGP_HIP(hipStreamSynchronize(s));  // h is pageable and goes out of scope
    t->Dp = Dp;
    t->dirty = false;
    return IFGP_OK;
}

}  // namespace

ifgp_status partial_fit(ifgp_birch_t b, const float *Z, int64_t n, int Z_on_device,
                        void *hip_stream);
}  // namespace ifgp

using namespace ifgp;

extern "C" {

IFGP_API ifgp_status ifgp_birch_create(int32_t d, double threshold, int32_t branching_factor,
                                       ifgp_birch_t *out) {
    if (!out || d < 1 || d > 1024 || !(threshold >= 0.0) || !std::isfinite(threshold) ||
        branching_factor < 2 || branching_factor > 1024) {
        set_error("ifgp_birch_create: need out, 1 <= d <= 1024, finite threshold >= 0 and "
                  "2 <= branching_factor <= 1024");
        return IFGP_E_INVALID;
    }
    ifgp_birch_s *t = new (std::nothrow) ifgp_birch_s();
    if (!t) {
        set_error("host allocation failed");
        return IFGP_E_OOM;
    }
    t->d = d;
    t->T = threshold;
    t->B = branching_factor;
    try {
        t->root = new_node(t, true);
    } catch (const std::bad_alloc &) {
        delete t;
        set_error("host allocation failed");
        return IFGP_E_OOM;
    }
    t->first_leaf = t->root;
    t->height = 1;
    *out = t;
    return IFGP_OK;
}

IFGP_API ifgp_status ifgp_birch_partial_fit(ifgp_birch_t b, const float *Z, int64_t n,
                                            int Z_on_device, void *hip_stream) {
    if (!b || n < 0 || (n > 0 && !Z)) {
        set_error("ifgp_birch_partial_fit: need a tree, n >= 0 and Z");
        return IFGP_E_INVALID;
    }
    if (b->broken) {
        set_error("ifgp_birch_partial_fit: an earlier call ran out of host memory; the tree is unusable");
        return IFGP_E_STATE;
    }
    if (n == 0) return IFGP_OK;
    try {
        return partial_fit(b, Z, n, Z_on_device, hip_stream);
    } catch (const std::bad_alloc &) {
        b->broken = true;
        set_error("host allocation failed; the tree is unusable (destroy it)");
        return IFGP_E_OOM;
    }
}
}  // extern "C"

namespace ifgp {
ifgp_status partial_fit(ifgp_birch_t b, const float *Z, int64_t n, int Z_on_device,
                        void *hip_stream) {
    const int d = b->d;
    std::vector<float> host;
    const float *src = Z;
    if (Z_on_device) {
        host.resize((size_t)n * d);
        const hipStream_t s = (hipStream_t)hip_stream;
        IFGP_HIP(hipMemcpyAsync(host.data(), Z, sizeof(float) * host.size(),
                                hipMemcpyDeviceToHost, s));
        IFGP_HIP(hipStreamSynchronize(s));
        src = host.data();
    }
    std::vector<double> p(d), tmp;
    for (int64_t i = 0; i < n; ++i) {
        for (int j = 0; j < d; ++j) p[j] = (double)src[(size_t)i * d + j];
        insert_point(b, p.data(), tmp);
    }
    b->clusters = count_clusters(b);
    b->dirty = true;
    return IFGP_OK;
}
}  // namespace ifgp

extern "C" {

IFGP_API ifgp_status ifgp_birch_info(ifgp_birch_t b, int64_t *n_points, int64_t *n_clusters,
                                     int32_t *height) {
    if (!b) {
        set_error("ifgp_birch_info: NULL tree");
        return IFGP_E_INVALID;
    }
    if (n_points) *n_points = b->points;
    if (n_clusters) *n_clusters = b->clusters;
    if (height) *height = b->height;
    return IFGP_OK;
}

IFGP_API ifgp_status ifgp_birch_centers(ifgp_birch_t b, double *centers) {
    if (!b || (b->clusters > 0 && !centers)) {
        set_error("ifgp_birch_centers: need a tree and an output array");
        return IFGP_E_INVALID;
    }
    if (b->broken) {
        set_error("ifgp_birch_centers: an earlier call ran out of host memory; the tree is unusable");
        return IFGP_E_STATE;
    }
    int64_t m = 0;
    for (const BNode *l = b->first_leaf; l; l = l->next_leaf) {
        std::memcpy(centers + (size_t)m * b->d, l->c.data(), sizeof(double) * l->c.size());
        m += l->size();
    }
    return IFGP_OK;
}

IFGP_API ifgp_status ifgp_birch_predict(ifgp_birch_t b, const float *Z, int64_t n,
                                        int32_t *labels, void *hip_stream) {
    if (!b || n < 0 || (n > 0 && (!Z || !labels))) {
        set_error("ifgp_birch_predict: need a tree, n >= 0, Z and labels");
        return IFGP_E_INVALID;
    }
    if (b->clusters == 0 || b->broken) {
        set_error(b->broken ? "ifgp_birch_predict: an earlier call ran out of host memory"
                            : "ifgp_birch_predict: the tree holds no points");
        return IFGP_E_STATE;
    }
    if (n == 0) return IFGP_OK;
    int dev = 0;
    IFGP_HIP(hipGetDevice(&dev));
    if (b->device != dev) {  // the device copy belongs to one device
        b->centers.reset();
        b->device = dev;
        b->dirty = true;
    }
    const hipStream_t s = (hipStream_t)hip_stream;
    try {
        IFGP_TRY(upload_centers(b, s));
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return IFGP_E_OOM;
    }
    const int64_t nblk = ceil_div(b->clusters, (int64_t)16);
    const double *F = b->centers.as<double>();
    const double *cn = F + (nblk + LABEL_SPARE) * 16 * b->Dp;
#define IFGP_LABEL(DP, RB)                                                                  \
    birch_label_kernel<DP, RB><<<grid_for(ceil_div(n, (int64_t)16 * RB * LW)), 64 * LW, 0, s>>>( \
        Z, n, b->d, F, cn, nblk, labels)
    switch (b->Dp) {
    // one row block per wave: more waves in flight beat more independent
    // chains per wave (measured for d = 8 ... 64)
    case 8: IFGP_LABEL(8, 1); break;
    case 16: IFGP_LABEL(16, 1); break;
    case 32: IFGP_LABEL(32, 1); break;
    case 64: IFGP_LABEL(64, 1); break;
    default:
        set_error("ifgp_birch_predict: device labelling supports d <= 64");
        return IFGP_E_INVALID;
    }
#undef IFGP_LABEL
    IFGP_LAUNCHED();
    return IFGP_OK;
}

IFGP_API ifgp_status ifgp_birch_destroy(ifgp_birch_t b) {
    if (!b) return IFGP_OK;
    if (b->device >= 0) (void)hipSetDevice(b->device);
    delete b;
    return IFGP_OK;
}

}  // extern "C"
