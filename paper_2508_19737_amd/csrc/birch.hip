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
//           dense N x M x d contraction with an argmin, in FP64 (the same
//           precision as the tree's own decisions).  On gfx950 FP64 vector
//           FMA runs at the FP64 matrix-core rate, so a plain register/LDS
//           tiled kernel reaches the same peak without MFMA.
#include <cmath>
#include <cstring>
#include <memory>
#include <utility>
#include <vector>

#include "internal.h"

namespace ifgp {
namespace {

struct BNode {
    bool leaf = true;
    std::vector<int64_t> n;   // per entry: points
    std::vector<double> ls;   // per entry: linear sum (d)
    std::vector<double> ss;   // per entry: sum of squared norms
    std::vector<double> c;    // per entry: centroid ls / n (d)
    std::vector<double> cn;   // per entry: |centroid|^2
    std::vector<BNode *> child;
    BNode *prev_leaf = nullptr, *next_leaf = nullptr;
    int size() const { return (int)n.size(); }
};

inline double dot(const double *a, const double *b, int d) {
    double s = 0.0;
    for (int k = 0; k < d; ++k) s += a[k] * b[k];
    return s;
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
};

namespace ifgp {
namespace {

BNode *new_node(ifgp_birch_s *t, bool leaf) {
    t->pool.emplace_back(new BNode());
    BNode *x = t->pool.back().get();
    x->leaf = leaf;
    return x;
}

// Entry k's centroid and its squared norm from its CF.
void refresh(BNode *x, int k, int d) {
    double *c = &x->c[(size_t)k * d];
    const double *ls = &x->ls[(size_t)k * d];
    const double nk = (double)x->n[k];
    for (int j = 0; j < d; ++j) c[j] = ls[j] / nk;
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

int nearest(const BNode *x, const double *p, int d) {
    int best = 0;
    double bd = 0.0;
    for (int k = 0; k < x->size(); ++k) {
        const double dk = x->cn[k] - 2.0 * dot(&x->c[(size_t)k * d], p, d);
        if (k == 0 || dk < bd) {
            bd = dk;
            best = k;
        }
    }
    return best;
}

// Split x around its farthest pair of centroids; a and b replace x (in the
// leaf order too).
std::pair<BNode *, BNode *> split(ifgp_birch_s *t, BNode *x) {
    const int d = t->d, k = x->size();
    std::vector<double> up((size_t)k * k, 0.0);  // squared distances, i < j
    int p = 0, q = 1;
    double far = -1.0;
    for (int i = 0; i < k; ++i)
        for (int j = i + 1; j < k; ++j) {
            double v = (x->cn[i] + x->cn[j]) - 2.0 * dot(&x->c[(size_t)i * d], &x->c[(size_t)j * d], d);
            if (v < 0.0) v = 0.0;
            up[(size_t)i * k + j] = v;
            if (v > far) {
                far = v;
                p = i;
                q = j;
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
// One thread per point, its coordinates in registers (FP64); the centroids
// pass through LDS in tiles of CT (read as broadcasts: every lane reads the
// same centroid).  Centroids are stored zero padded to Dp columns, points are
// read for their d columns only.
constexpr int PT = 256;
constexpr int CT = 64;

template <int Dp>
__global__ __launch_bounds__(PT) void birch_label_kernel(const float *__restrict__ Z, int64_t n,
                                                         int d, const double *__restrict__ C,
                                                         const double *__restrict__ cn,
                                                         int64_t M, int32_t *__restrict__ labels) {
    __shared__ double tile[CT][Dp];
    __shared__ double tnorm[CT];
    const int64_t i = (int64_t)blockIdx.x * PT + threadIdx.x;
    const bool live = i < n;
    double z[Dp];
#pragma unroll
    for (int k = 0; k < Dp; ++k) z[k] = (live && k < d) ? (double)Z[i * d + k] : 0.0;
    double best = 0.0;
    int64_t bi = 0;
    for (int64_t c0 = 0; c0 < M; c0 += CT) {
        const int m = (int)(M - c0 < CT ? M - c0 : CT);
        __syncthreads();
        for (int e = threadIdx.x; e < m * Dp; e += PT) tile[e / Dp][e % Dp] = C[c0 * Dp + e];
        for (int e = threadIdx.x; e < m; e += PT) tnorm[e] = cn[c0 + e];
        __syncthreads();
        for (int j = 0; j < m; ++j) {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};  // four chains: k mod 4
#pragma unroll
            for (int k = 0; k < Dp; ++k) acc[k % 4] = fma(z[k], tile[j][k], acc[k % 4]);
            const double dj = tnorm[j] - 2.0 * ((acc[0] + acc[1]) + (acc[2] + acc[3]));
            if ((c0 == 0 && j == 0) || dj < best) {
                best = dj;
                bi = c0 + j;
            }
        }
    }
    if (live) labels[i] = (int32_t)bi;
}

int padded_dim(int d) {
    int p = 8;
    while (p < d) p <<= 1;
    return p;
}

ifgp_status upload_centers(ifgp_birch_s *t, hipStream_t s) {
    if (!t->dirty) return IFGP_OK;
    const int d = t->d, Dp = padded_dim(d);
    const int64_t M = t->clusters;
    std::vector<double> h((size_t)M * Dp + (size_t)M, 0.0);
    int64_t m = 0;
    for (const BNode *l = t->first_leaf; l; l = l->next_leaf)
        for (int k = 0; k < l->size(); ++k, ++m) {
            std::memcpy(&h[(size_t)m * Dp], &l->c[(size_t)k * d], sizeof(double) * d);
            h[(size_t)M * Dp + m] = l->cn[k];
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
    t->root = new_node(t, true);
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
    if (n == 0) return IFGP_OK;
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
    if (b->clusters == 0) {
        set_error("ifgp_birch_predict: the tree holds no points");
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
    IFGP_TRY(upload_centers(b, s));
    const double *C = b->centers.as<double>();
    const double *cn = C + b->clusters * b->Dp;
    const unsigned grid = (unsigned)ceil_div(n, (int64_t)PT);
    switch (b->Dp) {
    case 8: birch_label_kernel<8><<<grid, PT, 0, s>>>(Z, n, b->d, C, cn, b->clusters, labels); break;
    case 16: birch_label_kernel<16><<<grid, PT, 0, s>>>(Z, n, b->d, C, cn, b->clusters, labels); break;
    case 32: birch_label_kernel<32><<<grid, PT, 0, s>>>(Z, n, b->d, C, cn, b->clusters, labels); break;
    case 64: birch_label_kernel<64><<<grid, PT, 0, s>>>(Z, n, b->d, C, cn, b->clusters, labels); break;
    default:
        set_error("ifgp_birch_predict: device labelling supports d <= 64");
        return IFGP_E_INVALID;
    }
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
