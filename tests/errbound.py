"""Per-element tolerance for comparing the HIP path's embedding with the FP64
oracle, derived from the arithmetic of the HIP path.  Test infrastructure.

The HIP path keeps each hop's features in the storage type (FP32, BF16 or
FP16) as W_j = s_j T_j, s_j = (D_tau)_jj^{-1/2}, and applies ZNorm lazily
(Zn = a T + b with a = 1/sigma, b = -mu/sigma of the previous hop):

    acc_i = sum_j W_j                          FP32, summed as the kernel does
    agg_i = a acc_i + b r_i,  r_i = sum_j s_j
    y_i   = theta (a T_i + b) + alpha s_i agg_i
    W_i'  = s_i tanh(y_i) rounded to the storage type
    mu, sigma of the stored T' in FP64 give the next (a, b); the output is
    sigma(a T + b) after the last hop (Eq. (3), (4)).

Rounding a value to the storage type is a deterministic function of that
value.  So this module follows the trajectory of the same formulas in FP64
with every stored row rounded to the storage type, exactly as the type
rounds (the reference), and bounds how far the HIP path can be from it:

  * the first hop's input, the caller's FP32 X times s formed in FP64 and
    rounded to the storage type (once for FP32 and FP16, through FP32 for
    BF16), is reproduced bit for bit;
  * a stored value equals the reference's whenever the HIP path's FP32 value
    before rounding is closer to the reference's FP64 value than that value is
    to the nearest rounding boundary (midpoint of the storage grid): then both
    round to the same representable number.  Otherwise (rare for 2-byte
    storage, usual for FP32) the stored value may differ by the FP32 error
    plus one unit in the last place;
  * what remains is FP32 arithmetic: the neighbour sum (every term passes
    through h_i additions, by the kernel's row classes: `sum_depth`), the
    product and fused multiply-add roundings, tanhf and expf (FN_ULPS each),
    and the statistics' FP64 sums;
  * these deviations propagate one layer at a time, with tanh's slope taken
    as its maximum over the interval of uncertainty and sigma reduced by its
    own error bound in every denominator.

The reference differs from the FP64 oracle by the effect of the storage
rounding (reported by the tests, and held to the usual relative Frobenius
tolerances); the HIP path must match the reference to within the bound, which
is at the level of FP32 arithmetic error, so a row summed wrongly, a
neighbour dropped or a column misplaced exceeds it by orders of magnitude.

Everything is column-local (the statistics are per column), so the check can
run on a few sampled columns of a large graph; `width` is the embedding's
width, which sets the kernel's lane geometry."""
import numpy as np

from oracle import ffp

E32 = 2.0 ** -24
FN_ULPS = 4        # assumed accuracy of the device tanhf and expf, in FP32 ulps (<= 2^-23 |x| each)
# storage grids: significand bits p (with the leading one), smallest normal exponent
GRID = {"f32": (24, -126), "bf16": (8, -126), "f16": (11, -14)}


def grid_round(v, storage):
    """v (FP64) rounded to nearest, ties to even, on the storage type's grid;
    also the grid spacing there and the distance from v to the nearest
    rounding boundary (midpoint between neighbouring grid values)."""
    p, emin = GRID[storage]
    v = np.asarray(v, dtype=np.float64)
    _, e = np.frexp(v)                     # |v| in [2^(e-1), 2^e)
    lead = np.maximum(e - 1, emin)
    ulp = np.ldexp(1.0, lead - (p - 1))
    q = v / ulp
    r = np.round(q) * ulp                  # numpy rounds half to even
    frac = q - np.floor(q)
    dist = np.minimum(np.abs(frac - 0.5), 1.5 - np.abs(frac - 0.5)) * ulp
    # just above a power of two the grid below is twice as fine: its
    # boundary sits a quarter of this spacing under the power of two
    dist = np.minimum(dist, np.abs(v) - np.ldexp(1.0, lead) + ulp / 4)
    return r, ulp, np.maximum(dist, 0.0)


def sum_depth(deg, width, storage):
    """Additions a neighbour row's value passes through in the kernel's sum
    for a row of deg neighbours.  A light row (< 128 neighbours) is summed by
    one lane group in sequence; a medium row (< 4096) by the RPW lane groups
    of one wave, each over its share in sequence, then a butterfly over the
    groups; a hub row by the 4 RPW groups of a 256-thread block, then the
    butterfly, then three additions over the waves.  RPW = 64 / LPR groups per
    wave, LPR = (padded width) / (16 bytes / storage bytes) lanes per row."""
    Dp = next(w for w in (8, 16, 32, 64, 128, 256) if width <= w)
    epl = 16 // (4 if storage == "f32" else 2)
    rpw = max(64 // (Dp // epl), 1)
    lg = int(np.log2(rpw))
    deg = np.asarray(deg, dtype=np.int64)
    light = np.maximum(deg - 1, 0)
    medium = -(-deg // rpw) - 1 + lg
    hub = -(-deg // (4 * rpw)) - 1 + lg + 3
    return np.where(deg >= 4096, hub, np.where(deg >= 128, medium, light))


def gamma(h):
    """|FP32 sum - exact| <= gamma(h) sum |terms| when every term passes
    through at most h additions."""
    h = np.asarray(h, dtype=np.float64)
    return h * E32 / (1 - h * E32)


def tanh_slope(y, e):
    """Largest tanh' = 1 - tanh^2 on [y - e, y + e]."""
    t = np.tanh(np.maximum(np.abs(y) - e, 0.0))
    return 1.0 - t * t


def reference_and_bound(rowptr, colidx, N, tau, K, X, storage, width=None, alpha=1.0,
                        theta=0.1, eps=1e-3, ddof=0, plant=None, with_bound=True):
    """(reference output, per-element bound on |HIP path - reference|) for K
    hops from the caller-supplied input X (N x c float32 values: the columns
    to check).  Raises ValueError where the bound stops meaning anything (a
    column's spread below twice its own error bound); with_bound=False gives
    the reference alone (bound None).  `plant(hop, ctx)` may overwrite rows of
    ctx["W"], the hop's stored rows (ctx also holds y, agg, a, b, s, A): the
    planted-mistake tests use it to build a wrong reference."""
    X = np.asarray(X, dtype=np.float32).astype(np.float64)
    width = X.shape[1] if width is None else width
    A = ffp.adjacency(rowptr, colidx, N)
    deg = ffp.degrees(rowptr)
    s = ffp.scales(deg, tau, eps)                     # FP64, as the device computes them
    sqd = np.sqrt(ffp.dtau(deg, tau, eps)).astype(np.float32).astype(np.float64)[:, None]
    s_ = s[:, None]
    r = np.asarray(A @ s)[:, None]
    g_acc = gamma(sum_depth(deg, width, storage))[:, None]
    n = float(N)

    # the stored input, reproduced exactly: s x formed in FP64 and rounded to
    # the storage type, once for FP32 and FP16, through FP32 for BF16
    v0 = s_ * X
    if storage == "bf16":
        v0 = v0.astype(np.float32).astype(np.float64)
    W, _, _ = grid_round(v0, storage)
    nu = np.zeros_like(W)               # |W_gpu - W_ref| bound: zero where provably equal
    a = np.ones((1, X.shape[1]))        # reference (a, b); the first hop's are exact
    b = np.zeros((1, X.shape[1]))
    da = np.zeros_like(a)               # bounds on |a_gpu - a|, |b_gpu - b|
    db = np.zeros_like(b)
    for hop in range(int(K)):
        W_prev = W
        T = W / s_                                      # the reference's T of the stored rows
        Tabs = np.abs(T) + nu / s_
        Zn = a * T + b
        agg = a * np.asarray(A @ W) + b * r
        y = theta * Zn + alpha * s_ * agg
        # uncertainty of the normalised input row and of the neighbour sum
        G = da * Tabs + np.abs(a) * nu / s_ + db
        sumW = np.asarray(A @ (np.abs(W) + nu))
        amax = np.abs(a) + da
        bmax = np.abs(b) + db
        d_agg = (amax * (np.asarray(A @ nu) + g_acc * sumW) + da * sumW + db * r
                 + bmax * 2 * E32 * r + E32 * (amax * sumW + 2 * bmax * r))
        d_self = G + amax * Tabs * 3 * E32 + E32 * (np.abs(Zn) + G)
        E = (theta * d_self + alpha * s_ * d_agg
             + E32 * (2 * theta * (np.abs(Zn) + G) + 4 * alpha * s_ * (np.abs(agg) + d_agg)))
        Tn = np.tanh(y)
        v = s_ * Tn                                     # value before rounding to storage
        P = s_ * (tanh_slope(y, E) * E + 2 * FN_ULPS * E32 * np.abs(Tn)) + 2 * E32 * np.abs(v)
        W, ulp, dist = grid_round(v, storage)
        nu = np.where(dist > P, 0.0, P + ulp)
        if plant is not None:
            plant(hop, {"W": W, "y": y, "agg": agg, "a": a, "b": b, "s": s, "A": A,
                        "Zn": Zn, "Wprev": W_prev, "theta": theta, "alpha": alpha,
                        "storage": storage})
        # statistics of the stored T (= W times the FP32 sqrt(D_tau)) in FP64
        Ts = W * sqd
        mu = Ts.mean(axis=0, keepdims=True)
        sd = np.sqrt(((Ts - mu) ** 2).sum(axis=0, keepdims=True) / (n - ddof))
        dev = nu * sqd
        M = dev.mean(axis=0, keepdims=True) + 1e-13 * np.abs(Ts).mean(axis=0, keepdims=True)
        S = np.sqrt((dev * dev).mean(axis=0, keepdims=True) * n / (n - ddof)) + 1e-13 * sd
        if not with_bound:
            S = M = np.zeros_like(sd)
        elif not np.all(sd > 2 * S):
            raise ValueError("bound lost: a column's spread is below twice its error bound")
        lo = sd - S
        a = 1.0 / sd
        b = -mu / sd
        da = S / (sd * lo) + E32 / lo
        db = M / lo + np.abs(mu) * S / (sd * lo) + 2 * E32 * (np.abs(b) + M / lo)
    T = W / s_
    Tabs = np.abs(T) + nu / s_
    x = a * T + b
    G = da * Tabs + np.abs(a) * nu / s_ + db
    dx = G + (np.abs(a) + da) * Tabs * 3 * E32 + E32 * (np.abs(x) + G)
    ref = ffp.sigmoid(x)
    if not with_bound:
        return ref, None
    bound = dx / 4.0 + 2 * (FN_ULPS + 2) * E32
    return ref, bound


def row_classes(deg):
    """Masks of the hop kernel's row classes: hub (>= 4096 neighbours, one
    256-thread block per row), medium (>= 128, one wave), light (the rest)."""
    deg = np.asarray(deg)
    return {"hub": deg >= 4096, "medium": (deg >= 128) & (deg < 4096), "light": deg < 128}
