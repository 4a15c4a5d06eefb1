"""Dense brute force for tiny graphs (test infrastructure only).

Builds L_tau as a dense matrix and takes the route through its
eigendecomposition that Sec. II and Eq. (2) describe, so that the sparse
spatial form of the oracle (Eq. (3)) can be checked against the spectral
definition it is derived from.
"""
from __future__ import annotations

import numpy as np

from . import ffp


def dense_adjacency(rowptr, colidx, N):
    A = np.zeros((N, N))
    for i in range(N):
        A[i, colidx[rowptr[i]:rowptr[i + 1]]] = 1.0
    return A


def laplacian_tau(A, tau, eps=ffp.EPS):
    """L_tau = I - D_tau^{-1/2} A D_tau^{-1/2} (Sec. I), D_tau by Eq. (1) for
    tau <= 0 and D + tau I for tau > 0."""
    deg = A.sum(axis=1)
    s = 1.0 / np.sqrt(ffp.dtau(deg, tau, eps))
    return np.eye(A.shape[0]) - (s[:, None] * A) * s[None, :]


def normalized_laplacian(A):
    """L = I - D^{-1/2} A D^{-1/2} (Sec. I), for graphs without isolated nodes."""
    deg = A.sum(axis=1)
    s = 1.0 / np.sqrt(deg)
    return np.eye(A.shape[0]) - (s[:, None] * A) * s[None, :]


def eig(L):
    """Eigenvalues ascending and orthonormal eigenvectors (L = U Lambda U^T)."""
    lam, U = np.linalg.eigh(L)
    return lam, U


def filter_response(lam, alpha=ffp.ALPHA, theta=ffp.THETA):
    """phi(lambda) = (theta + alpha) - alpha lambda, Eq. (2)."""
    return (theta + alpha) - alpha * lam


def spectral_conv(L, Z, alpha=ffp.ALPHA, theta=ffp.THETA, power=1):
    """U phi(Lambda)^power U^T Z: the graph convolution of Sec. II with the
    kernel of Eq. (2), applied `power` times in the spectral domain."""
    lam, U = eig(L)
    h = filter_response(lam, alpha, theta) ** power
    return U @ (h[:, None] * (U.T @ Z))


def spectral_ffp(A, tau, K, X, alpha=ffp.ALPHA, theta=ffp.THETA, eps=ffp.EPS, ddof=0):
    """Eq. (4) with every convolution taken through the eigendecomposition of
    L_tau instead of the spatial form: sigma(Z^(K))."""
    L = laplacian_tau(A, tau, eps)
    Z = np.asarray(X, dtype=np.float64)
    for _ in range(int(K)):
        Z = ffp.znorm(np.tanh(spectral_conv(L, Z, alpha, theta)), ddof)
    return ffp.sigmoid(Z)


def gershgorin_interval(A, tau, eps=ffp.EPS):
    """Theorem 1 applied to I - D_tau^{-1} A (similar to L_tau): every
    eigenvalue lies in [1 - max r_i, 1 + max r_i], r_i = deg_i / (D_tau)_ii."""
    deg = A.sum(axis=1)
    r = deg / ffp.dtau(deg, tau, eps)
    return 1.0 - r.max(), 1.0 + r.max()
