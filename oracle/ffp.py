"""FP64 sparse oracle of InfraredGP's FFP (test infrastructure only).

Each function states the passage of the paper it follows.  Notation: N nodes,
A the symmetric 0/1 adjacency, deg its row sums, tau the degree correction,
K the number of hops (the paper's L, number of GNN layers), d the embedding
dimension, (alpha, theta) the filter parameters of Eq. (2).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

ALPHA = 1.0      # Eq. (2)/(3): InfraredGP's low-pass filter uses (alpha, theta) = (1, 0.1)
THETA = 0.1
EPS = 1e-3       # Eq. (1): the paper sets epsilon to 0.001


# ---------------------------------------------------------------------------
# Graph (Sec. II problem statement: undirected, unweighted, A in {0,1}^{NxN})
# ---------------------------------------------------------------------------
def canonical_csr(src, dst, N):
    """Adjacency of the undirected simple graph on the listed pairs.

    A_ij = A_ji = 1 iff (i, j) or (j, i) is listed and i != j (Sec. II: A is
    symmetric with 0/1 entries; a self-loop is not an edge of a simple graph,
    and a pair listed twice is still one edge).  Returned as CSR with
    strictly ascending column indices in every row:
      rowptr int64 (N+1), colidx int64 (nnz), plus counts of dropped
      self-loop pairs and dropped duplicate undirected pairs.
    Raises ValueError for ids outside [0, N).
    """
    src = np.asarray(src, dtype=np.int64).ravel()
    dst = np.asarray(dst, dtype=np.int64).ravel()
    if src.shape != dst.shape:
        raise ValueError("src/dst length mismatch")
    if N < 0:
        raise ValueError("N must be >= 0")
    if src.size and (min(src.min(), dst.min()) < 0 or max(src.max(), dst.max()) >= N):
        raise ValueError("node id out of range")
    loop = src == dst
    u, v = src[~loop], dst[~loop]
    und = np.unique(np.minimum(u, v) * np.int64(max(N, 1)) + np.maximum(u, v))
    dups = int(u.size - und.size)
    a = und // max(N, 1)
    b = und % max(N, 1)
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    A = sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(N, N))
    A.sum_duplicates()
    A.sort_indices()
    A.data[:] = 1.0
    rowptr = A.indptr.astype(np.int64)
    colidx = A.indices.astype(np.int64)
    return rowptr, colidx, int(loop.sum()), dups


def degrees(rowptr):
    """deg_i = sum_j A_ij (Sec. I, degree diagonal matrix D)."""
    return np.diff(np.asarray(rowptr, dtype=np.int64))


def adjacency(rowptr, colidx, N):
    """scipy CSR of A with unit entries."""
    return sp.csr_matrix((np.ones(len(colidx)), np.asarray(colidx), np.asarray(rowptr)),
                         shape=(N, N))


# ---------------------------------------------------------------------------
# Degree correction (Sec. I and Eq. (1))
# ---------------------------------------------------------------------------
def dtau(deg, tau, eps=EPS):
    """Diagonal of D_tau in FP64.

    tau > 0: D_tau = D + tau I (the degree-corrected Laplacian of Sec. I).
    tau <= 0: Eq. (1), evaluated literally, (D_tau)_ii = deg_i - min(|tau|, deg_i - eps).
    At tau = 0 this is deg_i for deg_i >= 1 and eps for an isolated node, which
    keeps D_tau^{-1/2} finite where D^{-1/2} is not.
    """
    deg = np.asarray(deg, dtype=np.float64)
    if tau > 0:
        return deg + float(tau)
    return deg - np.minimum(abs(float(tau)), deg - eps)


def scales(deg, tau, eps=EPS):
    """s_i = (D_tau)_ii^{-1/2}, the symmetric normalisation of Eq. (3)."""
    return 1.0 / np.sqrt(dtau(deg, tau, eps))


# ---------------------------------------------------------------------------
# Random input Z^(0) ~ N(0, 1/d) (Sec. III-A before Eq. (4); Algorithm 1)
# ---------------------------------------------------------------------------
# Philox4x64-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy
# as 1, 2, 3", SC'11): a 4x64-bit counter and a 2x64-bit key, ten rounds.
_PHILOX_M0 = np.uint64(0xD2E7470EE14C6C93)
_PHILOX_M1 = np.uint64(0xCA5A826395121157)
_PHILOX_W0 = np.uint64(0x9E3779B97F4A7C15)
_PHILOX_W1 = np.uint64(0xBB67AE8584CAA73B)
_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo64(a, b):
    """(high, low) 64-bit halves of the 128-bit product a*b, elementwise."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _MASK32, a >> _S32
    b_lo, b_hi = b & _MASK32, b >> _S32
    p0 = a_lo * b_lo
    p1 = a_lo * b_hi
    p2 = a_hi * b_lo
    p3 = a_hi * b_hi
    mid = (p0 >> _S32) + (p1 & _MASK32) + (p2 & _MASK32)
    hi = p3 + (p1 >> _S32) + (p2 >> _S32) + (mid >> _S32)
    lo = a * b
    return hi, lo


def philox4x64_10(c0, c1, c2, c3, k0, k1):
    """Philox4x64 with ten rounds; arrays of counters, scalar key words."""
    with np.errstate(over="ignore"):
        c0 = np.asarray(c0, dtype=np.uint64)
        c1 = np.asarray(c1, dtype=np.uint64)
        c2 = np.asarray(c2, dtype=np.uint64)
        c3 = np.asarray(c3, dtype=np.uint64)
        k0 = np.uint64(k0)
        k1 = np.uint64(k1)
        for r in range(10):
            if r:
                k0 = np.uint64(k0 + _PHILOX_W0)
                k1 = np.uint64(k1 + _PHILOX_W1)
            hi0, lo0 = _mulhilo64(_PHILOX_M0, c0)
            hi1, lo1 = _mulhilo64(_PHILOX_M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def uniform53(o):
    """Map a 64-bit word to the open interval (0, 1): ((o >> 11) + 0.5) 2^-53."""
    return ((np.asarray(o, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53


def gaussian_input(N, d, seed, rows=None, cols=None):
    """Z^(0)[i, c] ~ N(0, 1/d), variance 1/d (standard deviation d^{-1/2}).

    Entry (i, c) is a pure function of (seed, i, c).  With q = c // 4, the
    Philox4x64-10 block with key (seed, 0) and counter (i + 1, q, 0, 0) gives
    words o0..o3 and uniforms u_k = uniform53(o_k).  The Box-Muller transform
    (Box & Muller 1958) of the pair (u0, u1), r = sqrt(-2 ln u0),
    phi = 2 pi u1, gives columns 4q (r cos phi) and 4q+1 (r sin phi); the pair
    (u2, u3) gives columns 4q+2 and 4q+3 the same way.  Each value is scaled
    by d^{-1/2}.  `rows`/`cols` select a sub-block (default all).  Parity with
    the paper's own random draw is unpinned: the paper does not name its
    generator.
    """
    rows = np.arange(N, dtype=np.uint64) if rows is None else np.asarray(rows, dtype=np.uint64)
    cols = np.arange(d, dtype=np.uint64) if cols is None else np.asarray(cols, dtype=np.uint64)
    ii, cc = np.meshgrid(rows, cols, indexing="ij")
    q = cc // np.uint64(4)
    j = (cc % np.uint64(4)).astype(np.int64)
    with np.errstate(over="ignore"):
        o0, o1, o2, o3 = philox4x64_10(ii + np.uint64(1), q, np.zeros_like(ii), np.zeros_like(ii),
                                       np.uint64(seed), 0)
    first = j < 2
    ua = uniform53(np.where(first, o0, o2))
    ub = uniform53(np.where(first, o1, o3))
    r = np.sqrt(-2.0 * np.log(ua))
    phi = 2.0 * np.pi * ub
    z = np.where(j % 2 == 0, r * np.cos(phi), r * np.sin(phi))
    return z / np.sqrt(float(d))


# ---------------------------------------------------------------------------
# One layer (Eqs. (2)-(4))
# ---------------------------------------------------------------------------
def conv(A, s, Z, alpha=ALPHA, theta=THETA):
    """Spatial form of the filter, Eq. (3) with general (alpha, theta):
    phi * Z = theta Z + alpha D_tau^{-1/2} A D_tau^{-1/2} Z.
    (With (alpha, theta) = (1, 0.1) this is Eq. (3) exactly; Eq. (2) gives
    phi(L) = (theta + alpha) I - alpha L_tau = theta I + alpha (I - L_tau).)"""
    s = np.asarray(s, dtype=np.float64)[:, None]
    return theta * Z + alpha * (s * (A @ (s * Z)))


def znorm(T, ddof=0):
    """Column-wise z-score, Eq. (4): (x - mean(x)) / std(x) per column.

    std uses divisor N - ddof (ddof = 0 is the plain definition of the standard
    deviation of the entries).  A column whose std is zero (or N - ddof <= 0)
    becomes all zeros.
    """
    n = T.shape[0]
    mu = T.mean(axis=0)
    C = T - mu
    if n - ddof <= 0:
        return np.zeros_like(T)
    sd = np.sqrt((C * C).sum(axis=0) / (n - ddof))
    out = np.zeros_like(T)
    nz = sd > 0
    out[:, nz] = C[:, nz] / sd[nz]
    return out


def sigmoid(x):
    """sigma(x) = (1 + e^{-x})^{-1}, Eq. (4)."""
    return 1.0 / (1.0 + np.exp(-x))


def layer(A, s, Z, alpha=ALPHA, theta=THETA, ddof=0):
    """Z^(l) = ZNorm(tanh(phi * Z^(l-1))), Eq. (4)."""
    return znorm(np.tanh(conv(A, s, Z, alpha, theta)), ddof)


def ffp_from_input(rowptr, colidx, N, tau, K, X, alpha=ALPHA, theta=THETA, eps=EPS, ddof=0):
    """Algorithm 1 from D_tau up to the embedding: Z^(0) = X, K layers of
    Eq. (4), then Z~ = sigma(Z^(K)).  FP64 throughout."""
    X = np.asarray(X, dtype=np.float64)
    A = adjacency(rowptr, colidx, N)
    s = scales(degrees(rowptr), tau, eps)
    Z = X
    for _ in range(int(K)):
        Z = layer(A, s, Z, alpha, theta, ddof)
    return sigmoid(Z)


def embed(src, dst, N, tau, K, d, seed, alpha=ALPHA, theta=THETA, eps=EPS, ddof=0):
    """Algorithm 1 steps up to the final sigmoid, from an edge list."""
    rowptr, colidx, _, _ = canonical_csr(src, dst, N)
    X = gaussian_input(N, d, seed)
    return ffp_from_input(rowptr, colidx, N, tau, K, X, alpha, theta, eps, ddof)


def rel_frobenius(got, ref):
    """||got - ref||_F / ||ref||_F in FP64."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
