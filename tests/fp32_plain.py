"""Eq. (3)-(4) evaluated directly in FP32 on the CPU (NumPy/SciPy float32):
a precision comparator, not a reference.  Where this plain FP32 evaluation
already misses the FP64 oracle by more than the FP32 target, no FP32
arithmetic is expected to meet it, and the HIP path is held to doing no worse.

    Y = theta Z + alpha S A S Z     (float32 sparse product, Eq. (3))
    T = tanh(Y)
    Z = (T - mean) / std            (float32 column statistics, Eq. (4))
    output sigma(Z)
"""
import numpy as np
import scipy.sparse as sp

from oracle import ffp


def ffp_fp32(rowptr, colidx, N, tau, K, X, alpha=1.0, theta=0.1, eps=1e-3):
    rowptr = np.asarray(rowptr, dtype=np.int64)
    s = ffp.scales(np.diff(rowptr), tau, eps).astype(np.float32)[:, None]
    A = sp.csr_matrix((np.ones(len(colidx), np.float32), np.asarray(colidx), rowptr),
                      shape=(N, N))
    a32, t32 = np.float32(alpha), np.float32(theta)
    Z = np.asarray(X, dtype=np.float32)
    for _ in range(int(K)):
        Y = t32 * Z + a32 * (s * (A @ (s * Z)).astype(np.float32))
        T = np.tanh(Y).astype(np.float32)
        mu = T.mean(axis=0, dtype=np.float32)
        sd = T.std(axis=0, dtype=np.float32)
        Z = np.where(sd > 0, (T - mu) / np.where(sd > 0, sd, 1), 0).astype(np.float32)
    return (1.0 / (1.0 + np.exp(-Z))).astype(np.float32)
