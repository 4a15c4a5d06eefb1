/*
 * ifgp.h -- C ABI of libifgp, InfraredGP's training-free feed-forward
 * propagation (FFP) on AMD Instinct MI355X (gfx950).
 *
 * What is computed (Qin, Li, Cui & Pei, "InfraredGP: Efficient Graph
 * Partitioning via Spectral Graph Neural Networks with Negative Corrections",
 * arXiv 2508.19737):
 *
 *   A        symmetric 0/1 adjacency of an undirected, unweighted graph
 *            (Sec. II, problem statement)
 *   D_tau    degree correction: Eq. (1) for tau <= 0, D + tau I for tau > 0
 *            (Sec. I)
 *   Z^(0)    N x d random input with entries ~ N(0, 1/d) (Sec. III-A, before
 *            Eq. (4); Algorithm 1, noise step)
 *   hop      phi * Z = theta Z + alpha D_tau^{-1/2} A D_tau^{-1/2} Z
 *            (Eq. (3); Eq. (2) gives the general (alpha, theta) form)
 *   layer    Z^(l) = ZNorm(tanh(phi * Z^(l-1))), ZNorm = column z-score
 *            (Eq. (4))
 *   output   Z~ = sigma(Z^(K)) (Eq. (4); Algorithm 1 up to the clustering
 *            step, whose BIRCH calls follow at the end of this header)
 *
 * K is the number of hops (the paper's number of GNN layers L).
 *
 * Conventions for every call:
 *   - Functions return ifgp_status; nothing aborts and no C++ exception
 *     crosses this boundary.  On a non-OK status ifgp_last_error() gives a
 *     message (per calling thread).
 *   - "device" pointers are HIP device memory of the current device; "host"
 *     pointers are ordinary host memory.  All device work is enqueued on the
 *     `hip_stream` argument (NULL = the legacy default stream) and is complete
 *     once that stream is synchronised; calls that must learn a size (graph
 *     build, stream_add, export) synchronise it themselves.
 *   - A graph handle owns all device memory it allocated (through the
 *     allocator hook, see ifgp_set_allocator; by default the library's
 *     caching allocator) and releases it stream-ordered: a block that a call
 *     replaces on the stream of that call (calls on one handle must be
 *     ordered, so its earlier uses come first), the rest on the stream each
 *     block was allocated on.  Work that uses a handle on other
 *     streams must be complete before ifgp_stream_add or ifgp_destroy on it.
 *     A handle is not thread-safe; distinct handles may be used from
 *     distinct threads.
 *   - Node ids are 0 .. N-1 and N must be below 2^31 - 1.
 */
#ifndef IFGP_H
#define IFGP_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define IFGP_API __attribute__((visibility("default")))
#else
#define IFGP_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ifgp_graph_s *ifgp_graph_t;

typedef enum {
    IFGP_OK = 0,
    IFGP_E_INVALID = -1, /* bad argument (size, pointer, dtype, parameter) */
    IFGP_E_RANGE = -2,   /* a node id outside [0, N) */
    IFGP_E_OOM = -3,     /* the allocator returned NULL */
    IFGP_E_DEVICE = -4,  /* a HIP runtime call failed */
    IFGP_E_STATE = -5    /* call not valid in the handle's current state */
} ifgp_status;

typedef enum {
    IFGP_F32 = 0,  /* float32 */
    IFGP_BF16 = 1, /* bfloat16 (storage only) */
    IFGP_F16 = 2,  /* IEEE half (storage only) */
    IFGP_F64 = 3   /* float64 (only ifgp_gaussian_input accepts it) */
} ifgp_dtype;

/*
 * Filter and normalisation parameters.
 *   alpha, theta  filter of Eq. (2)/(3); InfraredGP uses (1, 0.1) (Sec. III-A)
 *   eps           the small positive value of Eq. (1); 0.001 in the paper
 *   znorm_ddof    ZNorm standard deviation divisor N - ddof (0 or 1); 0 is the
 *                 plain standard deviation of the column entries (Eq. (4))
 *   storage       ifgp_dtype in which node features are kept in HBM between
 *                 hops (F32, BF16 or F16); accumulation is always FP32 and the
 *                 D_tau scales are always computed in FP64
 */
typedef struct {
    double alpha;
    double theta;
    double eps;
    int32_t znorm_ddof;
    int32_t storage;
} ifgp_params;

/* Fill *p with the paper's settings: alpha 1, theta 0.1, eps 0.001, ddof 0,
 * storage FP32.  Returns IFGP_E_INVALID if p is NULL. */
IFGP_API ifgp_status ifgp_default_params(ifgp_params *p);

/*
 * Build a graph handle from an edge list (Sec. II: undirected, unweighted;
 * Algorithm 1 input (V, E)).
 *   src, dst        num_edges node ids each (int64), host memory if
 *                   edges_on_device == 0, device memory otherwise; copied, so
 *                   the caller may free them on return
 *   N               number of nodes, 1 <= N < 2^31 - 1
 *   out             receives the new handle (unchanged on error)
 * Every pair is an undirected edge: (u, v) and (v, u) are the same edge, a pair
 * listed more than once is one edge, and u == v is dropped (A in {0,1}, simple
 * graph); both are counted (ifgp_graph_info).  The graph is kept in HBM as a
 * CSR with strictly ascending column indices per row.
 * Errors: IFGP_E_INVALID (N out of range, num_edges < 0, NULL pointers),
 * IFGP_E_RANGE (an id outside [0, N); no handle is created), IFGP_E_OOM,
 * IFGP_E_DEVICE.  Synchronises hip_stream.
 */
IFGP_API ifgp_status ifgp_build_graph(const int64_t *src, const int64_t *dst, int64_t num_edges,
                             int64_t N, int edges_on_device, void *hip_stream,
                             ifgp_graph_t *out);

/*
 * One FFP (Algorithm 1 from the D_tau step to the final sigmoid).
 *   tau     degree correction; tau <= 0 uses Eq. (1), tau > 0 uses D + tau I
 *   K       number of hops, K >= 0 (K = 0 returns sigma(Z^(0)))
 *   d       embedding dimension, 1 <= d <= 256
 *   seed    Z^(0)[i, c] is a pure function of (seed, i, c): with q = c / 4,
 *           the Philox4x64-10 block (Salmon et al., SC'11) with key (seed, 0)
 *           and counter (i + 1, q, 0, 0) gives words w0..w3, each mapped to
 *           u = ((w >> 11) + 0.5) 2^-53; Box-Muller (Box & Muller 1958) on
 *           (u0, u1) gives columns 4q, 4q+1 as r cos(phi), r sin(phi) with
 *           r = sqrt(-2 ln u0), phi = 2 pi u1, and on (u2, u3) columns 4q+2,
 *           4q+3; every value is divided by sqrt(d).  This is evaluated
 *           in FP64 for FP32 storage; for 2-byte storage (BF16, FP16), whose
 *           rounding dwarfs FP32's, the uniforms are formed from the top 23
 *           bits, u = ((w >> 41) + 0.5) 2^-23, and the transform runs in FP32
 *   p       parameters, NULL = ifgp_default_params
 *   out     device, N x d FP32, row-major, caller-owned; row i is node i
 * Errors: IFGP_E_INVALID (d, K, tau not finite, params), IFGP_E_OOM,
 * IFGP_E_DEVICE.  Does not synchronise.
 */
IFGP_API ifgp_status ifgp_embed(ifgp_graph_t g, double tau, int32_t K, int32_t d, uint64_t seed,
                       const ifgp_params *p, float *out, void *hip_stream);

/*
 * ifgp_embed for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops and harnesses that forbid hipMalloc): same
 * arguments, same result, bit for bit.  Instead of the handle's buffers, the
 * call works in a static device array of 64 MiB that the library holds on
 * each device it runs on until the process ends: scales, two feature
 * matrices, column statistics.  It calls no allocator (neither hipMalloc nor
 * the allocator hook), creates no stream or event, and enqueues everything
 * on hip_stream; hop timing (ifgp_timing_enable) does not apply to it.
 * Limit: 28 N + 16 KiB + 2 N Dp b + 16 Dp (hop blocks) + 8 Dp bytes, each
 * part rounded up to 256, must fit in 64 MiB (Dp = d padded to 8, 16, 32,
 * 64, 128 or 256; b = 2 for BF16/FP16 storage, 4 for FP32): e.g. N up to
 * about 220,000 at d = 64 in BF16, 115,000 in FP32.  Larger graphs return
 * IFGP_E_INVALID before any work is enqueued.
 * The array is shared: calls whose work overlaps on one device (other
 * streams, other threads) race and give undefined results; calls ordered on
 * one stream are safe, since each call rewrites every byte it reads.
 * The handle's cached scales are neither used nor changed.
 * Errors: as ifgp_embed (IFGP_E_OOM excepted).  Does not synchronise.
 */
IFGP_API ifgp_status ifgp_embed_noalloc(ifgp_graph_t g, double tau, int32_t K, int32_t d,
                                        uint64_t seed, const ifgp_params *p, float *out,
                                        void *hip_stream);

/* As ifgp_embed with a caller-supplied Z^(0): X is device FP32 N x d
 * row-major (row i is node i).  It is read before the call's first hop: the
 * first hop's input row s_i X[i] is formed in FP64 and rounded to the storage
 * type (once for FP32 and FP16, through FP32 for BF16). */
IFGP_API ifgp_status ifgp_embed_x(ifgp_graph_t g, double tau, int32_t K, int32_t d, const float *X,
                         const ifgp_params *p, float *out, void *hip_stream);

/*
 * The random input alone: out[i, c] = Z^(0)[i, c] for 0 <= i < N, 0 <= c < d,
 * by the rule given at ifgp_embed (in FP64), rounded to `dtype` (F64, F32,
 * BF16 or F16): once for F32 and F16, through FP32 for BF16.  out is device
 * memory, N x d row-major.  Errors: IFGP_E_INVALID.
 */
IFGP_API ifgp_status ifgp_gaussian_input(int64_t N, int32_t d, uint64_t seed, int32_t dtype, void *out,
                                void *hip_stream);

/*
 * Merge an edge increment into the graph (Algorithm 2, topology merge and
 * D_tau update).  new_N >= the current N; new_N == N is the emerging-edge
 * model (nodes fixed), new_N > N adds isolated nodes N .. new_N - 1 before the
 * increment's edges are merged.  Edge semantics as ifgp_build_graph.  After
 * the call the graph equals ifgp_build_graph of the union of all edges so far.
 * Strong guarantee: on any error the graph is unchanged.
 * Errors: IFGP_E_INVALID, IFGP_E_RANGE, IFGP_E_OOM, IFGP_E_DEVICE.
 * Synchronises hip_stream.
 */
IFGP_API ifgp_status ifgp_stream_add(ifgp_graph_t g, const int64_t *src, const int64_t *dst,
                            int64_t num_edges, int64_t new_N, int edges_on_device,
                            void *hip_stream);

/*
 * Embed several graphs together: every hop of every graph runs in one
 * launch per (storage, padded width, gather depth) class, so small graphs
 * share the device (the gather depth, the neighbour rows a lane keeps in
 * flight, follows from the graph's feature-matrix size alone).
 * Arrays have n entries; outs[k] is graph k's device N_k x d_k FP32 output.
 * The result for each graph is identical to ifgp_embed on that graph alone.
 * A handle may appear at most once.  Errors as ifgp_embed.
 */
IFGP_API ifgp_status ifgp_embed_batch(ifgp_graph_t *gs, int32_t n, const double *tau, const int32_t *K,
                             const int32_t *d, const uint64_t *seed, const ifgp_params *p,
                             float **outs, void *hip_stream);

/*
 * Stepwise embedding, for serving loops that admit graphs between hops.
 * ifgp_job_begin prepares Z^(0) of graph g (arguments as ifgp_embed) and
 * sets its hop counter to 0; ifgp_job_step advances every listed graph with
 * an unfinished job by one hop, batched as in ifgp_embed_batch, and writes
 * the output of each job that reaches its K; *done_flags (host, n entries,
 * may be NULL) receives 1 for jobs finished by this call or earlier.
 * A job's result equals ifgp_embed with the same arguments.
 * Errors: IFGP_E_STATE (ifgp_job_step on a handle without a job), others as
 * ifgp_embed.
 */
IFGP_API ifgp_status ifgp_job_begin(ifgp_graph_t g, double tau, int32_t K, int32_t d, uint64_t seed,
                           const ifgp_params *p, float *out, void *hip_stream);
IFGP_API ifgp_status ifgp_job_step(ifgp_graph_t *gs, int32_t n, int32_t *done_flags, void *hip_stream);

/* Sizes and counters: any output pointer may be NULL. */
IFGP_API ifgp_status ifgp_graph_info(ifgp_graph_t g, int64_t *N, int64_t *nnz,
                            int64_t *self_loops_dropped, int64_t *dups_dropped);

/* The execution plan of the hop kernel: rows with at least 4096 neighbours
 * (one 256-thread block each, by default), rows with 128 to 4095 (one wave
 * each, by default), the number of thread blocks one hop launches (BF16
 * storage, width 64), and the largest degree.  Any output pointer may be
 * NULL. */
IFGP_API ifgp_status ifgp_plan_info(ifgp_graph_t g, int64_t *hub_rows, int64_t *medium_rows,
                                    int64_t *hop_blocks, int32_t *max_degree);

/* Copy the CSR to host memory: rowptr N+1 entries, colidx nnz entries (ascending
 * within each row), deg N entries.  Synchronises the stream of the last call.
 * A fresh build leaves the canonical colidx unmade (the hop runs on the
 * relabelled copy); the first export of colidx, or the first ifgp_stream_add,
 * makes it on the device (4 nnz bytes) and releases the build's survivors
 * (4 bytes per edge end), so it can fail with IFGP_E_OOM. */
IFGP_API ifgp_status ifgp_export_csr(ifgp_graph_t g, int64_t *rowptr, int32_t *colidx, int32_t *deg);

/* Copy s_i = (D_tau)_ii^{-1/2} in FP64 for node i = 0 .. N-1 to host memory
 * (Eq. (1) / D + tau I, then the inverse square root). */
IFGP_API ifgp_status ifgp_export_scales(ifgp_graph_t g, double tau, double eps, double *s_host);

/* Device bytes a graph with N nodes and nnz stored entries needs resident for
 * embeddings of width d in `storage` (graph, scales, features, statistics).
 * Until the first export or merge after a build, the graph holds 4 bytes per
 * edge end (2E) in place of the canonical colidx's 4 nnz: pass nnz = 2E for
 * an upper bound that also covers that state. */
IFGP_API ifgp_status ifgp_footprint_bytes(int64_t N, int64_t nnz, int32_t d, int32_t storage,
                                 int64_t *bytes);

/*
 * Route every later device allocation of the library through alloc/free
 * (both non-NULL), or back to the library's caching allocator (both NULL):
 * hipMalloc'd blocks kept per (device, stream) after release and reused only
 * by later allocations on the same stream.  Each block is released through
 * the allocator that produced it, so the hook may change at any time.  alloc(bytes, stream,
 * ctx) returns device memory usable on `stream` or NULL; free(ptr, stream,
 * ctx) releases it after the work already enqueued on `stream`, which may
 * differ from the stream it was allocated on (a hook that cannot order the
 * release on `stream` synchronises it first).  Process-wide; keep the
 * callbacks alive while any block they produced exists.
 */
IFGP_API ifgp_status ifgp_set_allocator(void *(*alloc)(size_t, void *, void *),
                               void (*free_fn)(void *, void *, void *), void *ctx);

/* Return the cached free blocks of the library's own allocator to the device
 * (hipFree; synchronises the device).  Blocks in use are not affected. */
IFGP_API ifgp_status ifgp_empty_cache(void);

/*
 * Kernel timing: while enabled on a handle, each hop launch of that handle is
 * bracketed by HIP events on its stream.  ifgp_timing_read synchronises those
 * events and returns the number of hop launches and their summed duration in
 * milliseconds since the last read, then clears them.
 */
IFGP_API ifgp_status ifgp_timing_enable(ifgp_graph_t g, int enable);
IFGP_API ifgp_status ifgp_timing_read(ifgp_graph_t g, int64_t *hop_launches, double *hop_ms);

/*
 * Test hook for the grids of the kernels that can pass a launch's 2^32
 * work items per dimension (one thread per matrix entry, one block per few
 * rows, on graphs of several hundred million nodes): such grids put at most
 * max_x_blocks blocks in x and continue in y.  Lowering it lets small inputs
 * take the two-dimensional path.  max_x_blocks = 0 restores the default
 * (2^21); negative values are rejected (IFGP_E_INVALID).  *previous (may be
 * NULL) receives the value in force before the call.  Process-wide; results
 * do not depend on it.  Not for use while other threads launch work.
 */
IFGP_API ifgp_status ifgp_debug_grid_x(int64_t max_x_blocks, int64_t *previous);

/*
 * Test hook for the hop kernel's gather depth (the neighbour rows each lane
 * keeps in flight), which is otherwise chosen per graph from the size of its
 * feature matrix (2-byte storage only; FP32 storage has one depth):
 *   -1  per graph (the default): 16 rows if the matrix fits in 32 MiB, 4 if it
 *       reaches 224 MiB with rows of 64 or more columns, 8 otherwise
 *    0  8 rows      1  4 rows (rows of 64 or more columns; narrower rows use 8)
 *    2  16 rows
 * Results of a hop may differ between depths only in the order of the FP32
 * additions.  *previous (may be NULL) receives the setting in force before
 * the call.  Other values: IFGP_E_INVALID.  Process-wide; not for use while
 * other threads launch work.
 */
IFGP_API ifgp_status ifgp_debug_hop_depth(int32_t depth, int32_t *previous);

/* Release the handle and all its device memory (NULL is accepted). */
IFGP_API ifgp_status ifgp_destroy(ifgp_graph_t g);

/* Message for the calling thread's last non-OK status ("" if none). */
IFGP_API const char *ifgp_last_error(void);

/* Library version string. */
IFGP_API const char *ifgp_version(void);

/* ------------------------------------------------------------------ BIRCH
 * The clustering step that turns embeddings into a K-agnostic partition
 * (Sec. III, Algorithm 1 final step; Algorithm 2 fits it partially, to the
 * embeddings of newly added nodes, for streaming): BIRCH (Zhang,
 * Ramakrishnan & Livny, SIGMOD 1996) with no preset number of clusters, the
 * configuration the paper runs (Sec. IV).
 *
 *   CF        (n, LS, SS) per entry: count, linear sum, sum of squared norms;
 *             centroid LS/n, squared radius SS/n - |LS/n|^2
 *   tree      at most B entries per node (leaves too); inner entries
 *             summarise their child
 *   insert    descend to the entry with the nearest centroid (first on
 *             ties); in the leaf the nearest entry absorbs the point if its
 *             radius stays <= threshold, else the point is a new entry; an
 *             overfull node splits around its farthest pair of centroids
 *             (first pair p < q in row-major order; entries strictly nearer
 *             to p join p's node, p always does); a root split adds a level
 *   clusters  the leaf entries, in leaf order (left to right)
 *   labels    index of the nearest leaf-entry centroid (first on ties)
 *
 * All CF arithmetic is FP64.  Distances are compared as |c|^2 - 2 x.c.
 * Insertion is sequential (each point sees the tree the previous ones left)
 * and runs on the host; labelling is a dense N x M contraction and runs on
 * the device.  A BIRCH handle is not thread-safe.
 */
typedef struct ifgp_birch_s *ifgp_birch_t;

/* New empty tree for d-dimensional points.  threshold >= 0 (radius),
 * 2 <= branching_factor <= 1024, 1 <= d <= 1024.  IFGP_E_INVALID otherwise. */
IFGP_API ifgp_status ifgp_birch_create(int32_t d, double threshold, int32_t branching_factor,
                                       ifgp_birch_t *out);

/* Insert n points, in row order: Z is n x d row-major FP32 (device memory if
 * Z_on_device, else host).  A device Z is copied to the host on hip_stream,
 * which is synchronised.  If host memory runs out part-way (IFGP_E_OOM) the
 * tree is left unusable: later partial_fit, centers and predict calls return
 * IFGP_E_STATE; info and destroy still work. */
IFGP_API ifgp_status ifgp_birch_partial_fit(ifgp_birch_t b, const float *Z, int64_t n,
                                            int Z_on_device, void *hip_stream);

/* Points inserted so far, number of clusters (leaf entries), tree height. */
IFGP_API ifgp_status ifgp_birch_info(ifgp_birch_t b, int64_t *n_points, int64_t *n_clusters,
                                     int32_t *height);

/* Cluster centroids in leaf order into host memory, n_clusters x d, FP64. */
IFGP_API ifgp_status ifgp_birch_centers(ifgp_birch_t b, double *centers);

/* labels[i] = index of the nearest cluster centroid to row i of Z (device,
 * n x d FP32, d <= 64); labels is device int32 n.  Needs at least one
 * cluster (IFGP_E_STATE otherwise).  The centroids are uploaded (and
 * hip_stream synchronised) on first use after a change of the tree. */
IFGP_API ifgp_status ifgp_birch_predict(ifgp_birch_t b, const float *Z, int64_t n,
                                        int32_t *labels, void *hip_stream);

/*
 * The labels ifgp_birch_predict gives (bit for bit), for Algorithm 2's use:
 * between calls on one tree the rows labelled by the previous call keep their
 * values and new rows follow them (rows 0 .. m-1 of Z hold what they held in
 * the previous call, m = that call's n <= n; n < m starts over).  The call
 * compares each old row only with the cluster centroids created or changed
 * since the previous call (its nearest entry is otherwise unchanged; if that
 * entry moved, a bound on the row's second-nearest distance kept from before
 * stands for the unchanged ones); distances are taken in FP32 on the
 * matrix cores with a rigorous bound on their difference from the FP64 ones,
 * and rows whose nearest and second-nearest entries lie within that bound are
 * labelled in FP64 by ifgp_birch_predict's rule (first index on ties), over
 * the entries within twice the bound of the FP32 nearest (up to 8; all
 * entries for rows with more).
 * Entries whose centroids and norms are equal bit for bit (twins, which tie
 * exactly for every row) count once in FP32, and a row nearest to them gets
 * the first of them in leaf order, as ifgp_birch_predict gives.  The
 * centroids and what is known of each row stay in device memory held by the
 * tree (about 24 bytes per row, 12 Dp per cluster, Dp = d rounded up to 8,
 * 16, 32 or 64, up to 16 bytes per row and entry chunk for a pass's partial
 * results, and 68 bytes per row left to the FP64 rule).  The call
 * synchronises hip_stream (after the upload of the changed centroids, and
 * before each pass, whose size it reads back).
 * Z: device, n x d FP32, d <= 64; labels: device int32 n.  Errors as
 * ifgp_birch_predict, plus IFGP_E_INVALID for n >= 2^31.  A call that fails
 * part-way (IFGP_E_OOM, IFGP_E_DEVICE) leaves labels undefined and drops what
 * the tree kept for updates: the next call uploads every centroid again and
 * labels all of its rows in full.
 */
IFGP_API ifgp_status ifgp_birch_predict_update(ifgp_birch_t b, const float *Z, int64_t n,
                                               int32_t *labels, void *hip_stream);

/*
 * What the last ifgp_birch_predict_update did (host values; any pointer may
 * be NULL): new_entries = twin groups new since the call before (the entries
 * old rows were compared with), fp32_rows = rows labelled against every
 * entry in FP32 (new rows and old ones not settled by that comparison),
 * fp64_rows = rows of those left to the FP64 rule (ties and near ties),
 * fp64_full_rows = rows of those with more than 8 candidates, compared in
 * FP64 with every entry.  IFGP_E_INVALID for a NULL tree.
 */
IFGP_API ifgp_status ifgp_birch_update_stats(ifgp_birch_t b, int64_t *new_entries,
                                             int64_t *fp32_rows, int64_t *fp64_rows,
                                             int64_t *fp64_full_rows);

/* Release the tree and its device copy (NULL is accepted). */
IFGP_API ifgp_status ifgp_birch_destroy(ifgp_birch_t b);

#ifdef __cplusplus
}
#endif
#endif /* IFGP_H */
