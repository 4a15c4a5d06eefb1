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
#include <algorithm>
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
    std::vector<int32_t> id;  // per entry: the leaf entry's identity (-1 in inner nodes); it
                              // stays with the entry when a split moves it to another leaf
    std::vector<uint64_t> key;  // per leaf entry: twin_key of its centroid and norm
    BNode *prev_leaf = nullptr, *next_leaf = nullptr;
    int size() const { return (int)n.size(); }
};

inline double dot(const double *a, const double *b, int d) {
    double s = 0.0;
    for (int k = 0; k < d; ++k) s += a[k] * b[k];
    return s;
}

// A hash of an entry's centroid and norm bits: four independent streams over
// the coordinates (short dependency chains), then mixed as in the splitmix64
// finaliser (Steele, Lea & Flood 2014).  Equal keys are only candidates: a
// lookup compares the bits themselves.
uint64_t twin_key(const double *c, int d, double cn) {
    constexpr uint64_t M = 0xBF58476D1CE4E5B9ull, G = 0x9E3779B97F4A7C15ull;
    uint64_t h[4] = {G, 2 * G + 1, 3 * G, 4 * G + 1};
    int k = 0;
    for (; k + 4 <= d; k += 4)
        for (int j = 0; j < 4; ++j) {
            uint64_t w;
            std::memcpy(&w, &c[k + j], sizeof w);
            h[j] = (h[j] ^ w) * M;
        }
    for (; k < d; ++k) {
        uint64_t w;
        std::memcpy(&w, &c[k], sizeof w);
        h[k & 3] = (h[k & 3] ^ w) * M;
    }
    uint64_t w;
    std::memcpy(&w, &cn, sizeof w);
    uint64_t x = (h[0] ^ (h[1] << 17 | h[1] >> 47) ^ (h[2] << 31 | h[2] >> 33) ^
                  (h[3] << 47 | h[3] >> 17) ^ w) * M;
    x ^= x >> 31;
    x *= 0x94D049BB133111EBull;
    return x ^ (x >> 29);
}


// c_k . p for the NB entries of one block at once (the block is NB * d
// contiguous doubles, coordinate-major): every entry's sum runs over the
// coordinates in order, exactly as dot() (separate multiply and add, no fused
// multiply-add), so the result is the same to the last bit; the entries only
// share the vector lanes.
__attribute__((always_inline)) inline void dots_block(const double *blk, const double *p, int d,
                                                      double *out) {
#pragma clang fp contract(off)
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

// The same for two consecutive blocks (2 NB entries): eight independent sums
// per coordinate instead of four, so that the additions' latency, not their
// count, no longer sets the pace; each entry's sum is still taken over the
// coordinates in order.
__attribute__((always_inline)) inline void dots_block2(const double *blk, const double *p, int d,
                                                       double *out) {
#pragma clang fp contract(off)
    v4_t s[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) s[q] = 0.0;
    const double *blk1 = blk + (size_t)NB * d;
    for (int j = 0; j < d; ++j) {
        const double *r0 = blk + (size_t)j * NB, *r1 = blk1 + (size_t)j * NB;
        const v4_t pj = p[j];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v4_t c0, c1;
            std::memcpy(&c0, r0 + 4 * q, sizeof(v4_t));
            std::memcpy(&c1, r1 + 4 * q, sizeof(v4_t));
            s[q] = s[q] + c0 * pj;
            s[4 + q] = s[4 + q] + c1 * pj;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        std::memcpy(out + 4 * q, &s[q], sizeof(v4_t));
        std::memcpy(out + NB + 4 * q, &s[4 + q], sizeof(v4_t));
    }
}

// c_k . p for the entries [k0, k0 + 2 NB) (the second block only if k0 + NB
// < m: blocks are allocated whole, so a block with an entry is readable).
__attribute__((always_inline)) inline void dots_pair(const double *ct, int m, int k0,
                                                     const double *p, int d, double *out) {
    if (k0 + NB < m) dots_block2(ct + (size_t)k0 * d, p, d, out);
    else dots_block(ct + (size_t)k0 * d, p, d, out);
}

__attribute__((always_inline)) inline int nearest_body(const double *ct, const double *cn, int m,
                                                       const double *p, int d) {
    double dots[2 * NB];
    int best = 0;
    double bd = 0.0;
    for (int k0 = 0; k0 < m; k0 += 2 * NB) {
        dots_pair(ct, m, k0, p, d, dots);
        const int e = m - k0 < 2 * NB ? m - k0 : 2 * NB;
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

// c_k . p for every entry k < m (out has room for m rounded up to 2 NB).
__attribute__((always_inline)) inline void dots_body(const double *ct, int m, const double *p,
                                                     int d, double *out) {
    double two[2 * NB];
    for (int k0 = 0; k0 < m; k0 += 2 * NB) {
        dots_pair(ct, m, k0, p, d, two);
        const int e = m - k0 < 2 * NB ? m - k0 : 2 * NB;
        std::memcpy(out + k0, two, sizeof(double) * e);
    }
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

// Leaf entries whose centroids and stored norms are equal bit for bit (BIRCH
// leaves such twins when equal rows descend to different leaves) are at the
// same distance from every point, in any precision.  They form a twin group:
// the FP32 passes see one member of each group (its representative; the
// others have norm +inf there), and a point nearest to a group takes the
// group's first entry in leaf order, as the FP64 rule does.
struct TwinGroups {
    struct Group {
        uint64_t key = 0;
        int32_t rep = -1;    // the member the FP32 passes see
        int32_t fresh = 0;   // members that joined in the current update
        int32_t size = 0;
        int32_t head = -1;   // first member; the rest follow through next
        int32_t mpos = -1;   // position in multi, -1 if fewer than two members
    };
    std::vector<Group> g;
    std::vector<int32_t> spare;            // group numbers free for reuse
    std::vector<int32_t> of, next, prev;   // per identity: its group (-1 before it joins one)
                                           // and its neighbours in the group's list
    std::vector<int32_t> multi;            // groups of two or more members
    // groups by key: open addressing, linear probing, capacity a power of two
    // (slot group -1 = empty); keys of different centroids may be equal, so a
    // lookup compares the centroids too
    std::vector<uint64_t> hkey;
    std::vector<int32_t> hgrp;
    size_t used = 0;

    void clear() {
        g.clear(); spare.clear(); of.clear(); next.clear(); prev.clear(); multi.clear();
        hkey.clear(); hgrp.clear();
        used = 0;
    }
    void resize(size_t nid) {
        of.resize(nid, -1);
        next.resize(nid, -1);
        prev.resize(nid, -1);
    }
    int32_t make(uint64_t key) {
        int32_t gi;
        if (!spare.empty()) {
            gi = spare.back();
            spare.pop_back();
        } else {
            gi = (int32_t)g.size();
            g.emplace_back();
        }
        g[gi] = Group();
        g[gi].key = key;
        insert_key(key, gi);
        return gi;
    }
    void drop(int32_t gi) {
        erase_key(g[gi].key, gi);
        g[gi].rep = -1;
        spare.push_back(gi);
    }
    void add(int32_t gi, int32_t id) {
        Group &G = g[gi];
        next[id] = G.head;
        prev[id] = -1;
        if (G.head >= 0) prev[G.head] = id;
        G.head = id;
        of[id] = gi;
        if (++G.size == 2) {
            G.mpos = (int32_t)multi.size();
            multi.push_back(gi);
        }
    }
    void remove(int32_t gi, int32_t id) {
        Group &G = g[gi];
        if (prev[id] >= 0) next[prev[id]] = next[id];
        else G.head = next[id];
        if (next[id] >= 0) prev[next[id]] = prev[id];
        of[id] = next[id] = prev[id] = -1;
        if (--G.size == 1) {
            const int32_t last = multi.back();
            multi[G.mpos] = last;
            g[last].mpos = G.mpos;
            multi.pop_back();
            G.mpos = -1;
        }
    }
    void insert_key(uint64_t key, int32_t gi) {
        if (2 * (used + 1) > hgrp.size()) {
            std::vector<uint64_t> ok;
            std::vector<int32_t> og;
            ok.swap(hkey);
            og.swap(hgrp);
            const size_t cap = std::max<size_t>(1024, og.size() * 2);
            hkey.assign(cap, 0);
            hgrp.assign(cap, -1);
            used = 0;
            for (size_t i = 0; i < og.size(); ++i)
                if (og[i] >= 0) insert_key(ok[i], og[i]);
        }
        const size_t mask = hgrp.size() - 1;
        size_t i = key & mask;
        while (hgrp[i] >= 0) i = (i + 1) & mask;
        hkey[i] = key;
        hgrp[i] = gi;
        ++used;
    }
    // removal with backward shift: a later slot moves into the hole unless its
    // home lies cyclically in (hole, slot]
    void erase_key(uint64_t key, int32_t gi) {
        const size_t mask = hgrp.size() - 1;
        size_t i = key & mask;
        while (hgrp[i] != gi) i = (i + 1) & mask;
        size_t j = i;
        for (;;) {
            j = (j + 1) & mask;
            if (hgrp[j] < 0) break;
            const size_t k = hkey[j] & mask;
            const bool stays = i <= j ? (i < k && k <= j) : (i < k || k <= j);
            if (stays) continue;
            hkey[i] = hkey[j];
            hgrp[i] = hgrp[j];
            i = j;
        }
        hgrp[i] = -1;
        --used;
    }
};

// Device state of ifgp_birch_predict_update: the centroids in slots by entry
// identity (an entry keeps its slot while splits move it through the leaf
// order), what is known of every point labelled so far, and work lists.
struct LabelState {
    Buf f32, f64;          // slot fragments: block cb (identities 16 cb ... 16 cb + 15),
                           // coordinate step s: 64 values in lane order
    Buf cn32, cn64;        // |c|^2 per slot, +inf in unused slots (and, in FP32, for the
                           // members of a twin group other than its representative)
    int64_t cap_blk = 0;   // blocks the slot arrays hold
    Buf gidx;              // int32 per identity: leaf-order index of its twin group's first entry
    Buf chg;               // uint8 per identity: 0 unchanged since the last update; 1 new or
                           // changed; 2 changed while its old centroid stays in unchanged twins
    Buf cmp;               // the entries new in this update, packed: FP32 fragments (blocks
                           // of 16), FP32 norms, identities
    int64_t cmp_blk = 0;   // blocks cmp holds
    Buf raw;               // the entries as uploaded: FP64 centroids, norms, identities, flags
    Buf best_id;           // int32 per point: its entry, by identity
    Buf best32;            // float per point: FP32 distance to that entry, NaN if not known
    Buf second32;          // float per point: a lower bound on its FP32 distance to every
                           // other twin group (valid where best32 is known)
    Buf lists;             // [3][cap_pts]: points to redo in FP32 (int32; later the points
                           // left to the full FP64 pass), points for the FP64 rule (int32),
                           // their candidate thresholds (float)
    Buf ncand, cand;       // per point for the FP64 rule: candidates found, the first ones
    Buf counters;          // int32 [2]: the two lists' lengths
    Buf part;              // per (point, chunk of entries): a pass's partial result
    int64_t cap_pts = 0, n_prev = 0;
    bool slots_valid = false;
    void *stage = nullptr;  // pinned host staging of an upload
    size_t stage_bytes = 0;
    int32_t *hcount = nullptr;  // pinned: the lists' lengths, read back between passes
    int64_t last_counts[4] = {0, 0, 0, 0};  // the last update: points sent to the FP32 pass
                                            // and to the FP64 rule, twin groups new in it,
                                            // points left to the full FP64 pass
    TwinGroups twins;
    // host work arrays of an upload, kept between updates
    std::vector<int32_t> h_idx;             // per identity: its leaf-order index
    std::vector<const BNode *> h_leaf;      // per leaf-order index: the leaf holding the entry
    std::vector<int32_t> h_pos;             // ... and its position there
    std::vector<int32_t> h_changed, h_touched, h_orphan, h_order, h_kept;
    LabelState() = default;
    LabelState(const LabelState &) = delete;
    LabelState &operator=(const LabelState &) = delete;
    ~LabelState() {
        if (stage) (void)hipHostFree(stage);
        if (hcount) (void)hipHostFree(hcount);
    }
    // Drop every device buffer (each released on stream s if given, else on
    // the stream it was allocated on) and what is known of entries and rows.
    void reset(hipStream_t s = nullptr, bool on_s = false) {
        Buf *all[] = {&f32, &f64, &cn32, &cn64, &gidx, &chg, &cmp, &raw, &best_id, &best32,
                      &second32, &lists, &counters, &part, &ncand, &cand};
        for (Buf *x : all) {
            if (on_s) x->s = s;
            x->reset();
        }
        cap_blk = cmp_blk = cap_pts = n_prev = 0;
        slots_valid = false;
        twins.clear();
    }
};
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
    // leaf entries are numbered 0, 1, ... as they are created (they are never
    // removed); chg[id] marks those created, or whose centroid changed, since
    // the last ifgp_birch_predict_update; chg_list lists them
    int32_t next_id = 0;
    std::vector<uint8_t> chg;
    std::vector<int32_t> chg_list;
    ifgp::LabelState ls;  // device state of ifgp_birch_predict_update
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
    x->id.reserve(t->B + 1);
    x->key.reserve(t->B + 1);
    return x;
}

// Entry k's centroid x->c[k] is in place and cn is its squared norm: the
// coordinate-major copy, the norm and (in a leaf) the twin key follow.
void store_centroid(BNode *x, int k, int d, double cn) {
    const double *c = &x->c[(size_t)k * d];
    double *blk = &x->ct[(size_t)(k / NB) * NB * d + k % NB];
    for (int j = 0; j < d; ++j) blk[(size_t)j * NB] = c[j];
    x->cn[k] = cn;
    if (x->leaf) x->key[k] = twin_key(c, d, cn);
}

// Entry k's centroid and its squared norm from its CF.
void refresh(BNode *x, int k, int d) {
    double *c = &x->c[(size_t)k * d];
    const double *ls = &x->ls[(size_t)k * d];
    const double nk = (double)x->n[k];
    for (int j = 0; j < d; ++j) c[j] = ls[j] / nk;
    store_centroid(x, k, d, dot(c, c, d));
}

void append(BNode *x, int d, int64_t n, const double *ls, double ss, BNode *child,
            int32_t id = -1) {
    x->id.push_back(id);
    x->key.push_back(0);
    x->n.push_back(n);
    x->ls.insert(x->ls.end(), ls, ls + d);
    x->ss.push_back(ss);
    x->c.resize(x->c.size() + d);
    x->cn.push_back(0.0);
    x->child.push_back(child);
    refresh(x, x->size() - 1, d);
}

// Entry i of x appended to y as it is: its CF, identity and child, and the
// centroid, norm and twin key refresh made from that CF (a split moves
// entries without changing them).
void move_entry(BNode *y, const BNode *x, int i, int d) {
    const double *ls = &x->ls[(size_t)i * d], *c = &x->c[(size_t)i * d];
    y->id.push_back(x->id[i]);
    y->key.push_back(x->key[i]);
    y->n.push_back(x->n[i]);
    y->ls.insert(y->ls.end(), ls, ls + d);
    y->ss.push_back(x->ss[i]);
    y->c.insert(y->c.end(), c, c + d);
    y->cn.push_back(x->cn[i]);
    y->child.push_back(x->child[i]);
    const int k = y->size() - 1;
    double *blk = &y->ct[(size_t)(k / NB) * NB * d + k % NB];
    for (int j = 0; j < d; ++j) blk[(size_t)j * NB] = c[j];
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
        move_entry(to_a ? a : b, x, i, d);
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

// A leaf entry's centroid changed (or the entry is new).
void mark_changed(ifgp_birch_s *t, int32_t id) {
    if (!t->chg[(size_t)id]) {
        t->chg[(size_t)id] = 1;
        t->chg_list.push_back(id);
    }
}

int32_t new_entry_id(ifgp_birch_s *t) {
    const int32_t id = t->next_id++;
    t->chg.push_back(0);
    mark_changed(t, id);
    return id;
}

// Insert point p (|p|^2 = pp) below x; true if x now holds more than B entries.
bool insert(ifgp_birch_s *t, BNode *x, const double *p, double pp, std::vector<double> &tmp) {
    const int d = t->d;
    if (x->size() == 0) {
        append(x, d, 1, p, pp, nullptr, new_entry_id(t));
        return false;
    }
    const int k = nearest(x, p, d);
    if (!x->leaf) {
        BNode *ch = x->child[k];
        // entry k takes p before the descent (the update does not depend on
        // it, and a split below rewrites the entry from its two halves), so
        // that its refresh overlaps the child's search
        x->n[k] += 1;
        for (int j = 0; j < d; ++j) x->ls[(size_t)k * d + j] += p[j];
        x->ss[k] += pp;
        refresh(x, k, d);
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
        return false;
    }
    // leaf: absorb if the radius stays within the threshold
    const int64_t n1 = x->n[k] + 1;
    tmp.resize(2 * (size_t)d);
    double *ls1 = tmp.data(), *c1 = tmp.data() + d;
    for (int j = 0; j < d; ++j) ls1[j] = x->ls[(size_t)k * d + j] + p[j];
    const double ss1 = x->ss[k] + pp;
    for (int j = 0; j < d; ++j) c1[j] = ls1[j] / (double)n1;
    const double cn1 = dot(c1, c1, d);
    if (ss1 / (double)n1 - cn1 <= t->T * t->T) {
        // the absorbed CF's centroid and norm are c1 and cn1, the values
        // refresh would compute again from it
        x->n[k] = n1;
        std::memcpy(&x->ls[(size_t)k * d], ls1, sizeof(double) * d);
        x->ss[k] = ss1;
        std::memcpy(&x->c[(size_t)k * d], c1, sizeof(double) * d);
        store_centroid(x, k, d, cn1);
        mark_changed(t, x->id[k]);
        return false;
    }
    append(x, d, 1, p, pp, nullptr, new_entry_id(t));
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


// ---------------------------------------------------------------- labelling by update
// ifgp_birch_predict_update gives the labels ifgp_birch_predict gives, for
// Algorithm 2's pattern of use: the rows labelled by the previous call keep
// their values and new rows follow them, while the tree changed in between
// only where points were inserted.
//
// Distances are first taken in FP32 on the matrix cores (v_mfma_f32_16x16x4f32,
// twice the FP64 rate) with a bound beta on their difference from the FP64
// values the FP64 kernel would compare (beta below).  A point's nearest entry
// is decided in FP32 when the runner-up is more than 2 beta further away:
// then the FP64 order is the same.  Otherwise (ties, near ties) the point is
// labelled by the FP64 kernel's rule, first index in leaf order on ties, over
// its candidates: the entries within 2 beta of the FP32 nearest in FP32 (no
// other entry can be nearer in FP64), or over every entry when there are more
// than LABEL_CAND of them.
//
// Twin entries (centroid and norm equal bit for bit) tie exactly for every
// point; the FP32 passes see one of each twin group, and a point that ends
// nearest to a group gets the group's first leaf-order index, which is what
// the FP64 rule picks among them.  Exact ties of that kind, frequent on
// embeddings with repeated rows, therefore need no FP64 pass.
//
// A point labelled before whose nearest entry did not change keeps it against
// every centroid that was there before (they and the point are as they were),
// so it is compared only with the twin groups new since the last update,
// under the same rule.  Each point also keeps a lower bound on its FP32
// distance to every other group, so a point whose nearest entry moved is
// settled against the new groups and that bound.  A point is labelled again
// from scratch only when its FP32 distances are unknown (it went through the
// full FP64 pass) or its old centroid survives in unchanged twins.
//
// Each pass gives a wave 64 points (four row tiles sharing every centroid
// block it loads) and one chunk of the entry blocks, sized so that a pass
// runs about four waves per SIMD; a second kernel merges the chunks' best and
// second distances per point and decides.
//
// Entries sit in slots by identity, so the device copy of the tree changes
// only where entries changed; labels map identities to leaf-order indices at
// the end.
typedef float f4_t __attribute__((ext_vector_type(4)));

// FP32 MFMA lane layout (checked on the device): lane l, slot r of the
// 16 x 16 result holds D[4 (l / 16) + r][l % 16]; the operands are laid out as
// for the FP64 instruction above.

// (best, second, id) with dist added, b <= sc kept: the new second is the
// median of the three (one v_med3_f32), the new best their minimum.  A NaN
// distance (only from NaN coordinates) leaves b and bi as they were and sc at
// one of b, sc or NaN: never above the true second, so no row is decided on
// its account.
__device__ __forceinline__ void best2_insert(float dist, int32_t id, float &b, float &sc,
                                             int32_t &bi) {
    bi = dist < b ? id : bi;
    sc = __builtin_amdgcn_fmed3f(b, sc, dist);
    b = fminf(b, dist);
}

// (best, second, id) of the 16 lanes of each lane group, combined; ties put
// the second equal to the best.
__device__ __forceinline__ void best2_reduce(float &b, float &sc, int32_t &bi) {
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
        const float ob = __shfl_xor(b, off, 64), os = __shfl_xor(sc, off, 64);
        const int32_t oi = __shfl_xor(bi, off, 64);
        if (b <= ob) {
            sc = fminf(sc, ob);
        } else {
            sc = fminf(os, b);
            b = ob;
            bi = oi;
        }
    }
}

// beta for a point of norm xn (an upper bound): |dist32 - dist64| over every
// entry, centroid norms at most cmax.  dist32 = fl(|c|^2_32 - 2 x.c_32):
// |c|^2 rounded once (2^-24 C^2), the centroid's coordinates rounded once and
// d products and additions in the accumulation (counted twice, in case the
// matrix core rounds differently from round-to-nearest: 2 (d + 3) 2^-24 |x| C
// for x.c, times 2), the final subtraction (2^-24 (C^2 + 2 |x| C)); the FP64
// value's own error is far below.
#ifndef IFGP_LABEL_TOL_SCALE
#define IFGP_LABEL_TOL_SCALE 1.0f  // > 1 sends more rows to the FP64 pass (never fewer than needed)
#endif
__device__ __forceinline__ float label_beta(float xn, float cmax, int d) {
    const float c = cmax, e = 0x1p-24f;
    return (e * (2.f * c * c + (4.f * d + 14.f) * xn * c)) * 1.001f * IFGP_LABEL_TOL_SCALE + 1e-30f;
}

template <int S>
__device__ __forceinline__ void load_row(const float *__restrict__ Z, int d, int64_t p, int grp,
                                         float *a) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int k = 4 * s + grp;
        a[s] = (p >= 0 && k < d) ? Z[p * d + k] : 0.f;
    }
}

// |x| of point p in FP32 (rounding well inside the 1e-4 margin label_beta's
// callers add)
__device__ __forceinline__ float row_norm(const float *__restrict__ Z, int d, int64_t p) {
    float sq = 0.f;
    for (int k = 0; k < d; ++k) sq += Z[p * d + k] * Z[p * d + k];
    return sqrtf(sq);
}

// One pass's result for a point over one chunk of entries.
struct Part32 {
    float b, sc;  // best and second FP32 distance (equal on a tie)
    int32_t id;   // the best entry's identity
};
struct Part64 {
    double dist;  // best FP64 distance
    int32_t gx;   // leaf-order index of the best entry's twin group
    int32_t id;   // the best entry's identity
};

__device__ __forceinline__ void merge32(Part32 &acc, const Part32 &o) {
    if (o.b < acc.b) {
        acc.sc = fminf(acc.b, o.sc);
        acc.b = o.b;
        acc.id = o.id;
    } else {
        acc.sc = fminf(acc.sc, o.b);
    }
}

// Appends v to list (length *count) for the lanes where take is set, with one
// atomic per wave; returns the position written (-1 where take is not set).
__device__ __forceinline__ int32_t wave_append(bool take, int32_t v, int32_t *__restrict__ list,
                                               int32_t *__restrict__ count) {
    const uint64_t mask = __ballot(take);
    if (mask == 0) return -1;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(count, (int32_t)__popcll(mask));
    base = __shfl(base, leader, 64);
    if (!take) return -1;
    const int32_t at = base + (int32_t)__popcll(mask & ((1ull << lane) - 1));
    list[at] = v;
    return at;
}

// FP32 pass of RT row tiles (16 points each, coordinates in registers) over
// the entry blocks [cb0, cb1) (fragments F, norms cn, identities ids, or
// identity = slot if ids is null): per lane, tile and result slot the best
// and second distance and the best identity.  Blocks are taken two at a time
// (the next pair loading while one multiplies): cb1 - cb0 is even, or cb1 is
// the last block and the one after it a spare block of +inf norms; every
// block that is loaded lies below cb1 + 2.
template <int S, int RT>
__device__ __forceinline__ void pass32(const float (&a)[RT][S], const float *__restrict__ F,
                                       const float *__restrict__ cn,
                                       const int32_t *__restrict__ ids, int64_t cb0, int64_t cb1,
                                       int lane, float (&b)[RT][4], float (&sc)[RT][4],
                                       int32_t (&bi)[RT][4]) {
    const int col = lane & 15;
    float bA[S], bB[S], nA, nB;
    int32_t iA, iB;
    auto load = [&](float *bf, float &nr, int32_t &id, int64_t cb) {
#pragma unroll
        for (int s = 0; s < S; ++s) bf[s] = F[(cb * S + s) * 64 + lane];
        nr = cn[cb * 16 + col];
        id = ids ? ids[cb * 16 + col] : (int32_t)(cb * 16 + col);
        __builtin_amdgcn_sched_barrier(0);
    };
    // the row tiles' products interleaved (RT independent accumulations in
    // flight), each tile's sum still over s in order
    auto step = [&](const float *bf, float nrm, int32_t id) {
        f4_t acc[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) acc[t] = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int t = 0; t < RT; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][s], bf[s], acc[t], 0, 0, 0);
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                best2_insert(nrm - 2.f * acc[t][r], id, b[t][r], sc[t][r], bi[t][r]);
    };
    load(bA, nA, iA, cb0);
    for (int64_t cb = cb0; cb < cb1; cb += 2) {
        load(bB, nB, iB, cb + 1);
        step(bA, nA, iA);
        load(bA, nA, iA, cb + 2);
        step(bB, nB, iB);
    }
}

// Points rows[q] (q if rows is null), q < count, 16 RT per wave, against one
// chunk of cpc entry blocks each (cpc even): wave w takes chunk ch =
// w / groups (blocks [cpc ch, ...) below nblk) and row group w % groups, and
// writes each point's Part32 of that chunk to part[q * chunks + ch].  Waves
// that run together share a chunk, which the XCD's L2 then holds for all.
template <int Dp, int RT>
__global__ __launch_bounds__(64 * LW) void label_part32_kernel(
    const float *__restrict__ Z, int d, const int32_t *__restrict__ rows, int64_t count,
    const float *__restrict__ F, const float *__restrict__ cn, const int32_t *__restrict__ ids,
    int64_t nblk, int64_t groups, int64_t chunks, int64_t cpc, Part32 *__restrict__ part) {
    constexpr int S = Dp / 4;
    const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
    const int64_t w = block_index() * LW + (threadIdx.x >> 6);
    const int64_t ch = w / groups, q0 = (w % groups) * 16 * RT;
    if (ch >= chunks || q0 >= count) return;
    float a[RT][S];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        const int64_t q = q0 + 16 * t + col;
        load_row<S>(Z, d, q < count ? (rows ? rows[q] : q) : -1, grp, a[t]);
    }
    float b[RT][4], sc[RT][4];
    int32_t bi[RT][4];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            b[t][r] = sc[t][r] = __builtin_inff();
            bi[t][r] = -1;
        }
    const int64_t cb0 = ch * cpc, cb1 = cb0 + cpc < nblk ? cb0 + cpc : nblk;
    pass32<S, RT>(a, F, cn, ids, cb0, cb1, lane, b, sc, bi);
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            best2_reduce(b[t][r], sc[t][r], bi[t][r]);
            const int64_t q = q0 + 16 * t + 4 * grp + r;
            if (col == 0 && q < count) part[q * chunks + ch] = Part32{b[t][r], sc[t][r], bi[t][r]};
        }
}

// Old points [0, n_old) after their pass against the twin groups new in this
// update (chunks partial results each; none if there were none).  Every
// other group is as it was when the point was last decided in FP32, so it
// lies at least second32 away (the point's old entry, if unchanged, at
// best32).  Such a point keeps its entry, or moves to a new group, when the
// choice has a margin above 2 beta; so does a point whose entry changed
// (chg 1), over the new groups and second32.  Every other point (FP32
// distances unknown, or its old centroid still present in unchanged twins:
// chg 2) goes to the FP32 list.
__global__ void label_pick_changed_kernel(const float *__restrict__ Z, int d, int64_t n_old,
                                          int64_t chunks, const Part32 *__restrict__ part,
                                          const uint8_t *__restrict__ chg, float cmax,
                                          int32_t *__restrict__ best_id,
                                          float *__restrict__ best32,
                                          float *__restrict__ second32,
                                          int32_t *__restrict__ redo,
                                          int32_t *__restrict__ nredo) {
    const int64_t p = block_index() * blockDim.x + threadIdx.x;
    if (p >= n_old) return;
    Part32 r{__builtin_inff(), __builtin_inff(), -1};
    for (int64_t ch = 0; ch < chunks; ++ch) merge32(r, part[p * chunks + ch]);
    const int32_t bo = best_id[p];
    const float dold = best32[p], sold = second32[p];
    const float tol = 2.f * label_beta(row_norm(Z, d, p) * 1.0001f, cmax, d);
    bool decided = false;
    if (!__builtin_isnan(dold) && bo >= 0) {
        const uint8_t cg = chg[bo];
        if (cg == 0 && dold <= r.b) {
            if (r.b - dold > tol) {                            // the old entry stays
                second32[p] = fminf(sold, r.b);
                decided = true;
            }
        } else if (cg == 0) {
            // a new group wins (second32 is below dold where the old entry won
            // over a closer FP32 runner-up in FP64)
            const float rest = fminf(r.sc, fminf(dold, sold));
            if (rest - r.b > tol) {
                best_id[p] = r.id;
                best32[p] = r.b;
                second32[p] = rest;
                decided = true;
            }
        } else if (cg == 1 && fminf(r.sc, sold) - r.b > tol) { // the entry moved: a new group wins
            best_id[p] = r.id;
            best32[p] = r.b;
            second32[p] = fminf(r.sc, sold);
            decided = true;
        }
    }
    wave_append(!decided, (int32_t)p, redo, nredo);
}

// Appends the new points [n_old, n) to the FP32 list.
__global__ void label_push_kernel(int64_t n_old, int64_t n, int32_t *__restrict__ list,
                                  int32_t *__restrict__ count) {
    const int64_t p = n_old + block_index() * blockDim.x + threadIdx.x;
    if (p < n) wave_append(true, (int32_t)p, list, count);
}

// Points list[q], q < count, after their FP32 pass against every slot:
// decided when the runner-up is more than 2 beta further away, else sent to
// the FP64 list with the FP32 distance below which its candidates for the
// FP64 rule lie (thr64: best + 3 beta, so that the sum's rounding still
// leaves it above best + 2 beta).
__global__ void label_pick32_kernel(const float *__restrict__ Z, int d,
                                    const int32_t *__restrict__ list, int64_t count,
                                    int64_t chunks, const Part32 *__restrict__ part, float cmax,
                                    int32_t *__restrict__ best_id, float *__restrict__ best32,
                                    float *__restrict__ second32, int32_t *__restrict__ list64,
                                    float *__restrict__ thr64, int32_t *__restrict__ n64) {
    const int64_t q = block_index() * blockDim.x + threadIdx.x;
    if (q >= count) return;
    Part32 r{__builtin_inff(), __builtin_inff(), -1};
    for (int64_t ch = 0; ch < chunks; ++ch) merge32(r, part[q * chunks + ch]);
    const int32_t p = list[q];
    const float tol = 2.f * label_beta(row_norm(Z, d, p) * 1.0001f, cmax, d);
    const bool decided = r.sc - r.b > tol;
    if (decided) {
        best_id[p] = r.id;
        best32[p] = r.b;
        second32[p] = r.sc;
    }
    const int32_t at = wave_append(!decided, p, list64, n64);
    if (at >= 0) thr64[at] = r.b + 1.5f * tol;
}

// The FP64 rule over candidates.  An entry can be a point's nearest in FP64
// only if its FP32 distance is within 2 beta of the FP32 nearest (each FP32
// distance lies within beta of the FP64 one), so those entries are the
// point's candidates; the others are further in FP64 than the FP32 nearest.
constexpr int LABEL_CAND = 8;  // candidates kept per point; more send it to the full FP64 pass
struct Cand {
    int32_t id;   // slot (identity) of a twin group's representative
    float d32;    // its FP32 distance
};

// Points rows[q], q < count, 16 per wave, against one chunk of cpc slot
// blocks each in FP32 (representatives only; wave w takes chunk w / groups,
// row group w % groups): every entry (slot below nid) at most thr[q] away is
// counted in ncand[q], and the first LABEL_CAND are kept in cand[q].
template <int Dp>
__global__ __launch_bounds__(64 * LW) void label_cand_kernel(
    const float *__restrict__ Z, int d, const int32_t *__restrict__ rows, int64_t count,
    const float *__restrict__ thr, const float *__restrict__ F, const float *__restrict__ cn,
    int64_t nid, int64_t nblk, int64_t groups, int64_t chunks, int64_t cpc,
    int32_t *__restrict__ ncand, Cand *__restrict__ cand) {
    constexpr int S = Dp / 4;
    const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
    const int64_t w = block_index() * LW + (threadIdx.x >> 6);
    const int64_t ch = w / groups, q0 = (w % groups) * 16;
    if (ch >= chunks || q0 >= count) return;
    float a[S];
    load_row<S>(Z, d, q0 + col < count ? rows[q0 + col] : -1, grp, a);
    float t[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t q = q0 + 4 * grp + r;
        t[r] = q < count ? thr[q] : -__builtin_inff();
    }
    const int64_t cb0 = ch * cpc, cb1 = cb0 + cpc < nblk ? cb0 + cpc : nblk;
    for (int64_t cb = cb0; cb < cb1; ++cb) {
        float bf[S];
#pragma unroll
        for (int s = 0; s < S; ++s) bf[s] = F[(cb * S + s) * 64 + lane];
        const float nrm = cn[cb * 16 + col];
        f4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < S; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], bf[s], acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float dist = nrm - 2.f * acc[r];
            if (dist <= t[r] && cb * 16 + col < nid) {
                const int64_t q = q0 + 4 * grp + r;
                const int32_t k = atomicAdd(&ncand[q], 1);
                if (k < LABEL_CAND) cand[q * LABEL_CAND + k] = Cand{(int32_t)(cb * 16 + col), dist};
            }
        }
    }
}

// Points rows[q], q < count, 16 per wave, labelled by the FP64 rule over
// their candidates (at most LABEL_CAND; points with more go to the list
// full).  The FP64 distance of point j to its candidate is the diagonal
// element D[j][j] of a product whose column j holds point j's candidate:
// the same sum, in the same order, as in the FP64 kernel.  The FP32
// distances stay known: the winner's, and below every other group the least
// of the other candidates' and thr[q].
template <int Dp>
__global__ __launch_bounds__(64 * LW) void label_cand64_kernel(
    const float *__restrict__ Z, int d, const int32_t *__restrict__ rows, int64_t count,
    const float *__restrict__ thr, const int32_t *__restrict__ ncand,
    const Cand *__restrict__ cand, const double *__restrict__ F, const double *__restrict__ cn,
    const int32_t *__restrict__ gidx, int32_t *__restrict__ best_id, float *__restrict__ best32,
    float *__restrict__ second32, int32_t *__restrict__ full, int32_t *__restrict__ nfull) {
    constexpr int S = Dp / 4;
    const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
    const int64_t q0 = (block_index() * LW + (threadIdx.x >> 6)) * 16;
    if (q0 >= count) return;
    const int64_t q = q0 + col;  // the point of this lane's row and column
    const bool live = q < count;
    const int64_t p = live ? rows[q] : -1;
    double a[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int k = 4 * s + grp;
        a[s] = (p >= 0 && k < d) ? (double)Z[p * d + k] : 0.0;
    }
    const int nc = live ? ncand[q] : 0;
    const int use = nc > LABEL_CAND ? 0 : nc;
    // D[j][j] is in lane j + 16 (j % 4), slot j / 4
    const bool diag = (col & 3) == grp;
    double bd = __builtin_inf();
    int32_t bx = INT32_MAX, bc = -1;
    for (int c = 0; c < LABEL_CAND; ++c) {
        const int32_t id = c < use ? cand[q * LABEL_CAND + c].id : -1;
        double bf[S];
#pragma unroll
        for (int s = 0; s < S; ++s)
            bf[s] = id >= 0 ? F[((int64_t)(id / 16) * S + s) * 64 + id % 16 + 16 * grp] : 0.0;
        d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < S; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], bf[s], acc, 0, 0, 0);
        const int slot = col >> 2;
        const double v = slot == 0 ? acc[0] : slot == 1 ? acc[1] : slot == 2 ? acc[2] : acc[3];
        if (diag && id >= 0) {
            const double dist = cn[id] - 2.0 * v;
            const int32_t gx = gidx[id];
            if (dist < bd || (dist == bd && gx < bx)) {
                bd = dist;
                bx = gx;
                bc = c;
            }
        }
    }
    if (!(diag && live)) return;
    const bool decided = bc >= 0;
    if (decided) {
        float won = 0.f, rest = thr[q];
        for (int c = 0; c < use; ++c) {
            const Cand e = cand[q * LABEL_CAND + c];
            if (c == bc) won = e.d32;
            else rest = fminf(rest, e.d32);
        }
        best_id[p] = cand[q * LABEL_CAND + bc].id;
        best32[p] = won;
        second32[p] = rest;
    }
    wave_append(!decided, (int32_t)p, full, nfull);
}

// Points rows[q], q < count, 16 per wave, against one chunk of cpc slot
// blocks each in FP64, as the FP64 kernel compares them (nearest, then first
// in leaf order; a twin group's members share its first entry's index gx):
// wave w takes chunk ch = w / groups (blocks [cpc ch, ...) below nblk) and row
// group w % groups.
template <int Dp>
__global__ __launch_bounds__(64 * LW) void label_part64_kernel(
    const float *__restrict__ Z, int d, const int32_t *__restrict__ rows, int64_t count,
    const double *__restrict__ F, const double *__restrict__ cn, const int32_t *__restrict__ gidx,
    int64_t nid, int64_t nblk, int64_t groups, int64_t chunks, int64_t cpc,
    Part64 *__restrict__ part) {
    constexpr int S = Dp / 4;
    const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
    const int64_t w = block_index() * LW + (threadIdx.x >> 6);
    const int64_t ch = w / groups, q0 = (w % groups) * 16;
    if (ch >= chunks || q0 >= count) return;
    const int64_t p = q0 + col < count ? rows[q0 + col] : -1;
    double a[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int k = 4 * s + grp;
        a[s] = (p >= 0 && k < d) ? (double)Z[p * d + k] : 0.0;
    }
    double best[4];
    int32_t bi[4], bx[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        best[r] = __builtin_inf();
        bi[r] = -1;
        bx[r] = INT32_MAX;
    }
    const int64_t cb0 = ch * cpc, cb1 = cb0 + cpc < nblk ? cb0 + cpc : nblk;
    for (int64_t cb = cb0; cb < cb1; ++cb) {
        double bf[S];
#pragma unroll
        for (int s = 0; s < S; ++s) bf[s] = F[(cb * S + s) * 64 + lane];
        const double nrm = cn[cb * 16 + col];
        const int64_t c64 = cb * 16 + col;
        const int32_t cx = c64 < nid ? gidx[c64] : INT32_MAX;  // unused slots sort last
        d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < S; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], bf[s], acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double dist = nrm - 2.0 * acc[r];
            const bool take = dist < best[r] || (dist == best[r] && cx < bx[r]);
            best[r] = take ? dist : best[r];
            bi[r] = take ? (int32_t)c64 : bi[r];
            bx[r] = take ? cx : bx[r];
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        double v = best[r];
        int32_t i = bi[r], x = bx[r];
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const double ov = __shfl_xor(v, off, 64);
            const int32_t oi = __shfl_xor(i, off, 64), ox = __shfl_xor(x, off, 64);
            const bool take = ov < v || (ov == v && ox < x);
            v = take ? ov : v;
            i = take ? oi : i;
            x = take ? ox : x;
        }
        // FP64 result layout: D[i][j] in lane j + 16 (i % 4), slot i / 4
        const int64_t q = q0 + 4 * r + grp;
        if (col == 0 && q < count) part[q * chunks + ch] = Part64{v, x, i};
    }
}

// Points list[q], q < count, labelled from their FP64 partial results; their
// FP32 distance is left unknown, so a later update labels them afresh.
__global__ void label_pick64_kernel(const int32_t *__restrict__ list, int64_t count,
                                    int64_t chunks, const Part64 *__restrict__ part,
                                    int32_t *__restrict__ best_id, float *__restrict__ best32) {
    const int64_t q = block_index() * blockDim.x + threadIdx.x;
    if (q >= count) return;
    Part64 r{__builtin_inf(), INT32_MAX, -1};
    for (int64_t ch = 0; ch < chunks; ++ch) {
        const Part64 o = part[q * chunks + ch];
        if (o.dist < r.dist || (o.dist == r.dist && o.gx < r.gx)) r = o;
    }
    const int32_t p = list[q];
    best_id[p] = r.id;
    best32[p] = __builtin_nanf("");
}

__global__ void label_map_kernel(int64_t n, const int32_t *__restrict__ best_id,
                                 const int32_t *__restrict__ gidx, int32_t *__restrict__ labels) {
    const int64_t p = block_index() * blockDim.x + threadIdx.x;
    if (p < n) {
        const int32_t e = best_id[p];
        labels[p] = e >= 0 ? gidx[e] : -1;   // -1 only for rows with no finite distance
    }
}

// The uploaded entries (centroid FP64 m x d, norms, identities, flags: 1 for
// a twin group's representative) into their slots (FP64 and FP32 fragments
// and norms; FP32 norm +inf for the other twins), the first m_pack of them
// also into the packed FP32 array, whose blocks are padded to m_pack_pad
// entries with zero coordinates and norm +inf.  One thread per (entry,
// coordinate) over max(m, m_pack_pad) entries.
__global__ void label_scatter_kernel(int64_t m, int64_t m_pack, int64_t m_pack_pad, int64_t total,
                                     int d, int S, const double *__restrict__ c,
                                     const double *__restrict__ nrm,
                                     const int32_t *__restrict__ ids,
                                     const uint8_t *__restrict__ rep, double *__restrict__ f64,
                                     float *__restrict__ f32, double *__restrict__ cn64,
                                     float *__restrict__ cn32, float *__restrict__ pf,
                                     float *__restrict__ pcn, int32_t *__restrict__ pid) {
    const int Dp = 4 * S;
    const int64_t t = block_index() * blockDim.x + threadIdx.x;
    if (t >= total * Dp) return;
    const int64_t q = t / Dp;
    const int j = (int)(t % Dp);
    const int64_t po = ((q / 16) * S + j / 4) * 64 + q % 16 + 16 * (j % 4);
    if (q < m) {
        const int64_t id = ids[q], cb = id / 16, ccol = id % 16;
        const int64_t so = (cb * S + j / 4) * 64 + ccol + 16 * (j % 4);
        const double v = j < d ? c[q * d + j] : 0.0;
        f64[so] = v;
        f32[so] = (float)v;
        if (q < m_pack) pf[po] = (float)v;
        if (j == 0) {
            cn64[id] = nrm[q];
            cn32[id] = rep[q] ? (float)nrm[q] : __builtin_inff();
            if (q < m_pack) {
                pcn[q] = (float)nrm[q];
                pid[q] = (int32_t)id;
            }
        }
    }
    if (q >= m_pack && q < m_pack_pad) {
        pf[po] = 0.f;
        if (j == 0) {
            pcn[q] = __builtin_inff();
            pid[q] = 0;
        }
    }
}

template <typename T>
__global__ void label_fill_kernel(T *__restrict__ p, int64_t n, T v) {
    const int64_t i = block_index() * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Device copy of b->d-dimensional fragments for nblk slot blocks plus the
// spare ones: grown (old contents kept, new slots empty) when the tree has
// more entries than the arrays hold.
ifgp_status ensure_slots(ifgp_birch_s *b, int64_t nblk, hipStream_t s) {
    LabelState &L = b->ls;
    const int Dp = b->Dp, S = Dp / 4;
    const int64_t need = nblk + LABEL_SPARE;
    if (need <= L.cap_blk) return IFGP_OK;
    const int64_t cap = std::max<int64_t>(need, L.cap_blk * 3 / 2 + 64);
    Buf f32, f64, cn32, cn64;
    IFGP_TRY(alloc(f32, sizeof(float) * cap * S * 64, s));
    IFGP_TRY(alloc(f64, sizeof(double) * cap * S * 64, s));
    IFGP_TRY(alloc(cn32, sizeof(float) * cap * 16, s));
    IFGP_TRY(alloc(cn64, sizeof(double) * cap * 16, s));
    const int64_t old = L.cap_blk;
    if (old > 0) {
        IFGP_HIP(hipMemcpyAsync(f32.p, L.f32.p, sizeof(float) * old * S * 64, hipMemcpyDeviceToDevice, s));
        IFGP_HIP(hipMemcpyAsync(f64.p, L.f64.p, sizeof(double) * old * S * 64, hipMemcpyDeviceToDevice, s));
        IFGP_HIP(hipMemcpyAsync(cn32.p, L.cn32.p, sizeof(float) * old * 16, hipMemcpyDeviceToDevice, s));
        IFGP_HIP(hipMemcpyAsync(cn64.p, L.cn64.p, sizeof(double) * old * 16, hipMemcpyDeviceToDevice, s));
    }
    const int64_t nf = (cap - old) * S * 64, nc = (cap - old) * 16;
    label_fill_kernel<float><<<grid_for(ceil_div(nf, 256)), 256, 0, s>>>(f32.as<float>() + old * S * 64, nf, 0.f);
    label_fill_kernel<double><<<grid_for(ceil_div(nf, 256)), 256, 0, s>>>(f64.as<double>() + old * S * 64, nf, 0.0);
    label_fill_kernel<float><<<grid_for(ceil_div(nc, 256)), 256, 0, s>>>(cn32.as<float>() + old * 16, nc, __builtin_inff());
    label_fill_kernel<double><<<grid_for(ceil_div(nc, 256)), 256, 0, s>>>(cn64.as<double>() + old * 16, nc, __builtin_inf());
    IFGP_LAUNCHED();
    L.f32 = std::move(f32);
    L.f64 = std::move(f64);
    L.cn32 = std::move(cn32);
    L.cn64 = std::move(cn64);
    L.cap_blk = cap;
    return IFGP_OK;
}

// What an upload sent: m entries, the first m_pack of them new in this update
// (twin groups none of whose members was there before) and packed for the
// pass over old points; the largest centroid norm.
struct Upload {
    int64_t m = 0, m_pack = 0;
    double cmax = 0.0;
};

// Host walk of the leaves (identities -> leaf-order indices, the largest
// centroid norm), the twin groups brought up to date with the entries changed
// since the last update (all of them if the slots are not filled yet), and
// the upload: per identity its group's first leaf-order index and whether it
// changed; per uploaded entry its centroid, norm, identity and whether it
// represents its group.  Staged in pinned memory, copied to the device, then
// scattered into place.
ifgp_status upload_changes(ifgp_birch_s *b, hipStream_t s, Upload *up) {
    LabelState &L = b->ls;
    TwinGroups &T = L.twins;
    const int d = b->d, Dp = b->Dp, S = Dp / 4;
    const int64_t nid = b->next_id;
    const bool all = !L.slots_valid;
    const size_t o_chg = sizeof(int32_t) * (size_t)nid;
    const size_t o_c0 = (o_chg + (size_t)nid + 7) / 8 * 8;
    // leaf-order index per identity; the entry behind each index (written in
    // leaf order), read back only for the entries that need their centroid
    std::vector<int32_t> &idx = L.h_idx;
    idx.resize((size_t)nid);
    L.h_leaf.resize((size_t)nid);
    L.h_pos.resize((size_t)nid);
    double mx = 0.0;
    int64_t k = 0;
    for (const BNode *l = b->first_leaf; l; l = l->next_leaf)
        for (int e = 0; e < l->size(); ++e, ++k) {
            idx[l->id[e]] = (int32_t)k;
            L.h_leaf[k] = l;
            L.h_pos[k] = e;
            mx = std::max(mx, l->cn[e]);
        }
    struct At {
        const BNode *leaf;
        int e;
    };
    auto at = [&](int32_t id) {
        const int32_t q = idx[id];
        return At{L.h_leaf[q], L.h_pos[q]};
    };
    std::vector<int32_t> &changed = L.h_changed;
    if (all) {
        T.clear();
        changed.resize((size_t)nid);
        for (int32_t i = 0; i < (int32_t)nid; ++i) changed[i] = i;
    } else {
        changed.assign(b->chg_list.begin(), b->chg_list.end());
    }
    auto is_chg = [&](int32_t id) { return all || b->chg[(size_t)id] != 0; };
    T.resize((size_t)nid);
    // the changed entries leave their groups
    std::vector<int32_t> &orphan = L.h_orphan;
    orphan.clear();
    L.h_kept.clear();
    for (int32_t id : changed) {
        const int32_t gi = T.of[id];
        if (gi < 0) continue;
        T.remove(gi, id);
        TwinGroups::Group &G = T.g[gi];
        if (G.size == 0) {
            T.drop(gi);
            continue;
        }
        for (int32_t x = G.head; x >= 0; x = T.next[x])
            if (!is_chg(x)) {
                L.h_kept.push_back(id);  // its old centroid stays in unchanged twins
                break;
            }
        if (G.rep == id) {
            G.rep = -1;
            orphan.push_back(gi);
        }
    }
    // ... and join the groups of their current centroids
    std::vector<int32_t> &touched = L.h_touched;
    touched.clear();
    for (int32_t id : changed) {
        const At a = at(id);
        const double *c = &a.leaf->c[(size_t)a.e * d];
        const double cn = a.leaf->cn[a.e];
        const uint64_t kid = a.leaf->key[a.e];
        int32_t gi = -1;
        if (!T.hgrp.empty()) {
            const size_t mask = T.hgrp.size() - 1;
            for (size_t i = kid & mask; T.hgrp[i] >= 0; i = (i + 1) & mask) {
                if (T.hkey[i] != kid) continue;
                const At o = at(T.g[T.hgrp[i]].head);
                if (std::memcmp(&o.leaf->cn[o.e], &cn, sizeof cn) == 0 &&
                    std::memcmp(&o.leaf->c[(size_t)o.e * d], c, sizeof(double) * d) == 0) {
                    gi = T.hgrp[i];
                    break;
                }
            }
        }
        if (gi < 0) gi = T.make(kid);
        T.add(gi, id);
        if (T.g[gi].fresh++ == 0) touched.push_back(gi);
    }
    // representatives (an unchanged member where there is one: then only its
    // FP32 norm changes on the device), and the upload order: representatives
    // of the groups new in this update, the other changed entries, then the
    // unchanged members that became representatives
    std::vector<int32_t> &order = L.h_order;
    order.clear();
    std::vector<int32_t> promoted;
    auto choose = [&](TwinGroups::Group &G) {
        for (int32_t x = G.head; x >= 0; x = T.next[x])
            if (!is_chg(x)) {
                G.rep = x;
                promoted.push_back(x);
                return;
            }
        G.rep = G.head;
    };
    for (int32_t gi : touched) {
        TwinGroups::Group &G = T.g[gi];
        if (G.rep < 0) choose(G);
        if (G.fresh == G.size) order.push_back(G.rep);
    }
    for (int32_t gi : orphan) {
        TwinGroups::Group &G = T.g[gi];
        if (G.rep < 0 && G.size > 0) choose(G);
    }
    const int64_t m_pack = (int64_t)order.size();
    for (int32_t id : changed) {
        const TwinGroups::Group &G = T.g[T.of[id]];
        if (!(G.rep == id && G.fresh == G.size)) order.push_back(id);
    }
    for (int32_t gi : touched) T.g[gi].fresh = 0;
    order.insert(order.end(), promoted.begin(), promoted.end());
    const int64_t m = (int64_t)order.size();
    const int64_t m_pack_pad = (ceil_div(m_pack, (int64_t)16) + LABEL_SPARE) * 16;
    // staging layout: gidx (nid int32), chg (nid bytes, padded to 8), centroids
    // (m x d doubles), norms (m doubles), identities (m int32), flags (m bytes)
    const size_t o_c = o_c0;
    const size_t o_n = o_c + sizeof(double) * (size_t)m * d;
    const size_t o_id = o_n + sizeof(double) * (size_t)m;
    const size_t o_rep = o_id + sizeof(int32_t) * (size_t)m;
    const size_t bytes = o_rep + (size_t)m + 8;
    if (L.stage_bytes < bytes) {
        if (L.stage) IFGP_HIP(hipHostFree(L.stage));
        L.stage = nullptr;
        L.stage_bytes = 0;
        const size_t cap = bytes + bytes / 2;
        IFGP_HIP(hipHostMalloc(&L.stage, cap, 0));
        L.stage_bytes = cap;
    }
    char *h = static_cast<char *>(L.stage);
    int32_t *gx = reinterpret_cast<int32_t *>(h);
    uint8_t *chg = reinterpret_cast<uint8_t *>(h + o_chg);
    double *c = reinterpret_cast<double *>(h + o_c), *nrm = reinterpret_cast<double *>(h + o_n);
    int32_t *ids = reinterpret_cast<int32_t *>(h + o_id);
    uint8_t *rep = reinterpret_cast<uint8_t *>(h + o_rep);
    std::memcpy(gx, idx.data(), sizeof(int32_t) * (size_t)nid);
    for (int32_t gi : T.multi) {
        int32_t first = INT32_MAX;
        for (int32_t x = T.g[gi].head; x >= 0; x = T.next[x]) first = std::min(first, idx[x]);
        for (int32_t x = T.g[gi].head; x >= 0; x = T.next[x]) gx[x] = first;
    }
    for (int64_t i = 0; i < nid; ++i) chg[i] = is_chg((int32_t)i) ? 1 : 0;
    for (int32_t id : L.h_kept) chg[id] = 2;
    for (int64_t q = 0; q < m; ++q) {
        const int32_t id = order[q];
        const At a = at(id);
        std::memcpy(c + (size_t)q * d, &a.leaf->c[(size_t)a.e * d], sizeof(double) * d);
        nrm[q] = a.leaf->cn[a.e];
        ids[q] = id;
        rep[q] = T.g[T.of[id]].rep == id ? 1 : 0;
    }
    for (int32_t id : b->chg_list) b->chg[(size_t)id] = 0;
    b->chg_list.clear();
    IFGP_TRY(ensure_slots(b, ceil_div(nid, (int64_t)16), s));
    IFGP_TRY(ensure(L.raw, bytes, s));
    IFGP_TRY(ensure(L.gidx, sizeof(int32_t) * (size_t)nid, s));
    IFGP_TRY(ensure(L.chg, (size_t)nid, s));
    const size_t cmp_bytes = (sizeof(float) * Dp + sizeof(float) + sizeof(int32_t)) * (size_t)m_pack_pad;
    IFGP_TRY(ensure(L.cmp, cmp_bytes, s));
    L.cmp_blk = m_pack_pad / 16;
    IFGP_HIP(hipMemcpyAsync(L.raw.p, h, bytes, hipMemcpyHostToDevice, s));
    const char *r = static_cast<const char *>(L.raw.p);
    IFGP_HIP(hipMemcpyAsync(L.gidx.p, r, sizeof(int32_t) * (size_t)nid, hipMemcpyDeviceToDevice, s));
    IFGP_HIP(hipMemcpyAsync(L.chg.p, r + o_chg, (size_t)nid, hipMemcpyDeviceToDevice, s));
    float *pf = L.cmp.as<float>();
    float *pcn = pf + (size_t)m_pack_pad * Dp;
    int32_t *pid = reinterpret_cast<int32_t *>(pcn + m_pack_pad);
    const int64_t total = std::max(m, m_pack_pad);
    label_scatter_kernel<<<grid_for(ceil_div(total * Dp, 256)), 256, 0, s>>>(
        m, m_pack, m_pack_pad, total, d, S, reinterpret_cast<const double *>(r + o_c),
        reinterpret_cast<const double *>(r + o_n), reinterpret_cast<const int32_t *>(r + o_id),
        reinterpret_cast<const uint8_t *>(r + o_rep), L.f64.as<double>(), L.f32.as<float>(),
        L.cn64.as<double>(), L.cn32.as<float>(), pf, pcn, pid);
    IFGP_LAUNCHED();
    // the staging memory is reused by the next update: wait for the copy
    IFGP_HIP(hipStreamSynchronize(s));
    L.slots_valid = true;
    up->m = m;
    up->m_pack = m_pack;
    up->cmax = std::sqrt(mx);
    return IFGP_OK;
}

constexpr int64_t LABEL_WAVES = 4096;  // waves a pass aims for: four per SIMD
constexpr int LABEL_RT = 4;            // row tiles of 16 points per wave in the FP32 passes

// Chunks of an even number of entry blocks (at least 8) for a pass over nblk
// blocks, so that `groups` row groups times the chunks come to about
// LABEL_WAVES waves.
void label_chunks(int64_t groups, int64_t nblk, int64_t *chunks, int64_t *cpc) {
    const int64_t want = std::max<int64_t>(1, ceil_div(LABEL_WAVES, std::max<int64_t>(groups, 1)));
    int64_t c = std::max<int64_t>(8, ceil_div(std::max<int64_t>(nblk, 1), want));
    c += c & 1;
    *cpc = c;
    *chunks = std::max<int64_t>(1, ceil_div(nblk, c));
}

// The list lengths, read back between passes (the next pass is sized by them).
ifgp_status read_counts(LabelState &L, hipStream_t s) {
    IFGP_HIP(hipMemcpyAsync(L.hcount, L.counters.p, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, s));
    IFGP_HIP(hipStreamSynchronize(s));
    return IFGP_OK;
}

// The passes of an update: old points against the new entries, the FP32
// list against every slot, the FP64 list against every slot; then labels.
template <int Dp>
ifgp_status label_passes(ifgp_birch_s *b, const float *Z, int64_t n, int64_t n_old,
                         const Upload &up, int32_t *labels, hipStream_t s) {
    LabelState &L = b->ls;
    const int d = b->d;
    const int64_t nid = b->next_id, nblk = ceil_div(nid, (int64_t)16);
    int32_t *cnt = L.counters.as<int32_t>();
    int32_t *list32 = L.lists.as<int32_t>(), *list64 = list32 + L.cap_pts;
    float *thr64 = reinterpret_cast<float *>(list32 + 2 * L.cap_pts);
    int32_t *best_id = L.best_id.as<int32_t>();
    float *best32 = L.best32.as<float>();
    // nearest entry in FP32 within 2 beta of the FP64 one: cmax bounds every |c|
    const float cm = (float)(up.cmax * (1.0 + 1e-6)) + 1e-30f;
    label_fill_kernel<int32_t><<<1, 64, 0, s>>>(cnt, 2, 0);
    IFGP_LAUNCHED();
    if (n_old > 0) {
        int64_t chunks = 0, cpc = 0;
        const int64_t pblk = ceil_div(up.m_pack, (int64_t)16);
        if (pblk > 0) {
            const int64_t groups = ceil_div(n_old, (int64_t)16 * LABEL_RT);
            label_chunks(groups, pblk, &chunks, &cpc);
            IFGP_TRY(ensure(L.part, sizeof(Part32) * (size_t)(n_old * chunks), s));
            const float *pf = L.cmp.as<float>();
            const float *pcn = pf + (size_t)L.cmp_blk * 16 * Dp;
            const int32_t *pid = reinterpret_cast<const int32_t *>(pcn + L.cmp_blk * 16);
            label_part32_kernel<Dp, LABEL_RT>
                <<<grid_for(ceil_div(groups * chunks, (int64_t)LW)), 64 * LW, 0, s>>>(
                    Z, d, nullptr, n_old, pf, pcn, pid, pblk, groups, chunks, cpc,
                    L.part.as<Part32>());
            IFGP_LAUNCHED();
        }
        label_pick_changed_kernel<<<grid_for(ceil_div(n_old, (int64_t)256)), 256, 0, s>>>(
            Z, d, n_old, chunks, L.part.as<Part32>(), L.chg.as<uint8_t>(), cm, best_id, best32,
            L.second32.as<float>(), list32, cnt);
        IFGP_LAUNCHED();
    }
    if (n > n_old) {
        label_push_kernel<<<grid_for(ceil_div(n - n_old, (int64_t)256)), 256, 0, s>>>(n_old, n,
                                                                                      list32, cnt);
        IFGP_LAUNCHED();
    }
    IFGP_TRY(read_counts(L, s));
    const int64_t n32 = L.hcount[0];
    if (n32 > 0) {
        int64_t chunks = 0, cpc = 0;
        const int64_t groups = ceil_div(n32, (int64_t)16 * LABEL_RT);
        label_chunks(groups, nblk, &chunks, &cpc);
        IFGP_TRY(ensure(L.part, sizeof(Part32) * (size_t)(n32 * chunks), s));
        label_part32_kernel<Dp, LABEL_RT>
            <<<grid_for(ceil_div(groups * chunks, (int64_t)LW)), 64 * LW, 0, s>>>(
                Z, d, list32, n32, L.f32.as<float>(), L.cn32.as<float>(), nullptr, nblk, groups,
                chunks, cpc, L.part.as<Part32>());
        IFGP_LAUNCHED();
        label_pick32_kernel<<<grid_for(ceil_div(n32, (int64_t)256)), 256, 0, s>>>(
            Z, d, list32, n32, chunks, L.part.as<Part32>(), cm, best_id, best32,
            L.second32.as<float>(), list64, thr64, cnt + 1);
        IFGP_LAUNCHED();
        IFGP_TRY(read_counts(L, s));
    }
    const int64_t n64 = n32 > 0 ? L.hcount[1] : 0;
    int64_t nfull = 0;
    if (n64 > 0) {
        // the FP64 rule over each point's candidates
        IFGP_TRY(ensure(L.ncand, sizeof(int32_t) * (size_t)n64, s));
        IFGP_TRY(ensure(L.cand, sizeof(Cand) * (size_t)(n64 * LABEL_CAND), s));
        int32_t *ncand = L.ncand.as<int32_t>();
        Cand *cand = L.cand.as<Cand>();
        label_fill_kernel<int32_t><<<grid_for(ceil_div(n64, (int64_t)256)), 256, 0, s>>>(ncand, n64, 0);
        label_fill_kernel<int32_t><<<1, 64, 0, s>>>(cnt, 1, 0);  // the full list reuses list32
        IFGP_LAUNCHED();
        int64_t chunks = 0, cpc = 0;
        const int64_t groups = ceil_div(n64, (int64_t)16);
        label_chunks(groups, nblk, &chunks, &cpc);
        label_cand_kernel<Dp><<<grid_for(ceil_div(groups * chunks, (int64_t)LW)), 64 * LW, 0, s>>>(
            Z, d, list64, n64, thr64, L.f32.as<float>(), L.cn32.as<float>(), nid, nblk, groups,
            chunks, cpc, ncand, cand);
        IFGP_LAUNCHED();
        label_cand64_kernel<Dp><<<grid_for(ceil_div(groups, (int64_t)LW)), 64 * LW, 0, s>>>(
            Z, d, list64, n64, thr64, ncand, cand, L.f64.as<double>(), L.cn64.as<double>(),
            L.gidx.as<int32_t>(), best_id, best32, L.second32.as<float>(), list32, cnt);
        IFGP_LAUNCHED();
        IFGP_TRY(read_counts(L, s));
        nfull = L.hcount[0];
    }
    if (nfull > 0) {
        // the full FP64 pass for points with too many candidates
        int64_t chunks = 0, cpc = 0;
        const int64_t groups = ceil_div(nfull, (int64_t)16);
        label_chunks(groups, nblk, &chunks, &cpc);
        IFGP_TRY(ensure(L.part, sizeof(Part64) * (size_t)(nfull * chunks), s));
        label_part64_kernel<Dp><<<grid_for(ceil_div(groups * chunks, (int64_t)LW)), 64 * LW, 0, s>>>(
            Z, d, list32, nfull, L.f64.as<double>(), L.cn64.as<double>(), L.gidx.as<int32_t>(), nid,
            nblk, groups, chunks, cpc, L.part.as<Part64>());
        IFGP_LAUNCHED();
        label_pick64_kernel<<<grid_for(ceil_div(nfull, (int64_t)256)), 256, 0, s>>>(
            list32, nfull, chunks, L.part.as<Part64>(), best_id, best32);
        IFGP_LAUNCHED();
    }
    L.last_counts[0] = n32;
    L.last_counts[1] = n64;
    L.last_counts[2] = up.m_pack;
    L.last_counts[3] = nfull;
    label_map_kernel<<<grid_for(ceil_div(n, (int64_t)256)), 256, 0, s>>>(n, best_id,
                                                                         L.gidx.as<int32_t>(), labels);
    IFGP_LAUNCHED();
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

namespace ifgp {
// The device copies (centroids, label state) belong to the device they were
// made on: when the current device is another, they are dropped (each block
// goes back to its own device's cache) and made again on this one.
ifgp_status use_current_device(ifgp_birch_s *b) {
    int dev = 0;
    IFGP_HIP(hipGetDevice(&dev));
    if (b->device != dev) {
        b->centers.reset();
        b->ls.reset();
        b->device = dev;
        b->dirty = true;
    }
    return IFGP_OK;
}

// The update itself (ifgp_birch_predict_update checks the arguments and, on
// any failure here, drops the label state).  Rows [0, L.n_prev) were labelled
// by the previous update.
ifgp_status predict_update(ifgp_birch_s *b, const float *Z, int64_t n, int32_t *labels,
                           hipStream_t s) {
    LabelState &L = b->ls;
    const int64_t n_old = L.n_prev;
    Upload up;
    IFGP_TRY(upload_changes(b, s, &up));
    if (n > L.cap_pts) {
        const int64_t cap = std::max<int64_t>(n, L.cap_pts * 3 / 2);
        Buf bid, b32, s32, lists;
        IFGP_TRY(alloc(bid, sizeof(int32_t) * cap, s));
        IFGP_TRY(alloc(b32, sizeof(float) * cap, s));
        IFGP_TRY(alloc(s32, sizeof(float) * cap, s));
        IFGP_TRY(alloc(lists, sizeof(int32_t) * 3 * cap, s));
        if (n_old > 0) {
            IFGP_HIP(hipMemcpyAsync(bid.p, L.best_id.p, sizeof(int32_t) * n_old, hipMemcpyDeviceToDevice, s));
            IFGP_HIP(hipMemcpyAsync(b32.p, L.best32.p, sizeof(float) * n_old, hipMemcpyDeviceToDevice, s));
            IFGP_HIP(hipMemcpyAsync(s32.p, L.second32.p, sizeof(float) * n_old, hipMemcpyDeviceToDevice, s));
        }
        L.best_id = std::move(bid);
        L.best32 = std::move(b32);
        L.second32 = std::move(s32);
        L.lists = std::move(lists);
        L.cap_pts = cap;
    }
    IFGP_TRY(ensure(L.counters, sizeof(int32_t) * 2, s));
    if (!L.hcount) IFGP_HIP(hipHostMalloc(reinterpret_cast<void **>(&L.hcount), 64, 0));
    switch (b->Dp) {
    case 8: return label_passes<8>(b, Z, n, n_old, up, labels, s);
    case 16: return label_passes<16>(b, Z, n, n_old, up, labels, s);
    case 32: return label_passes<32>(b, Z, n, n_old, up, labels, s);
    case 64: return label_passes<64>(b, Z, n, n_old, up, labels, s);
    default:
        set_error("ifgp_birch_predict_update: device labelling supports d <= 64");
        return IFGP_E_INVALID;
    }
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
    IFGP_TRY(use_current_device(b));
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

IFGP_API ifgp_status ifgp_birch_predict_update(ifgp_birch_t b, const float *Z, int64_t n,
                                               int32_t *labels, void *hip_stream) {
    if (!b || n < 0 || (n > 0 && (!Z || !labels))) {
        set_error("ifgp_birch_predict_update: need a tree, n >= 0, Z and labels");
        return IFGP_E_INVALID;
    }
    if (b->clusters == 0 || b->broken) {
        set_error(b->broken ? "ifgp_birch_predict_update: an earlier call ran out of host memory"
                            : "ifgp_birch_predict_update: the tree holds no points");
        return IFGP_E_STATE;
    }
    if (padded_dim(b->d) > 64) {
        set_error("ifgp_birch_predict_update: device labelling supports d <= 64");
        return IFGP_E_INVALID;
    }
    if (n > INT32_MAX) {
        set_error("ifgp_birch_predict_update: n must be below 2^31");
        return IFGP_E_INVALID;
    }
    if (n == 0) return IFGP_OK;
    IFGP_TRY(use_current_device(b));
    LabelState &L = b->ls;
    b->Dp = padded_dim(b->d);
    if (n < L.n_prev) L.n_prev = 0;  // not the rows labelled before: start over
    ifgp_status st = IFGP_OK;
    try {
        st = predict_update(b, Z, n, labels, (hipStream_t)hip_stream);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        st = IFGP_E_OOM;
    }
    if (st != IFGP_OK) {
        // the upload may have taken the tree's changes without the device or
        // the points' state following them, and a failed allocation leaves
        // its buffer empty: the label state is dropped (released after this
        // call's work on its stream), and the next update allocates it
        // again, uploads every entry and labels every point
        L.reset((hipStream_t)hip_stream, true);
        return st;
    }
    L.n_prev = n;
    return IFGP_OK;
}

IFGP_API ifgp_status ifgp_birch_update_stats(ifgp_birch_t b, int64_t *new_entries,
                                             int64_t *fp32_rows, int64_t *fp64_rows,
                                             int64_t *fp64_full_rows) {
    if (!b) {
        set_error("ifgp_birch_update_stats: need a tree");
        return IFGP_E_INVALID;
    }
    if (new_entries) *new_entries = b->ls.last_counts[2];
    if (fp32_rows) *fp32_rows = b->ls.last_counts[0];
    if (fp64_rows) *fp64_rows = b->ls.last_counts[1];
    if (fp64_full_rows) *fp64_full_rows = b->ls.last_counts[3];
    return IFGP_OK;
}

IFGP_API ifgp_status ifgp_birch_destroy(ifgp_birch_t b) {
    if (!b) return IFGP_OK;
    if (b->device >= 0) (void)hipSetDevice(b->device);
    delete b;
    return IFGP_OK;
}

}  // extern "C"
