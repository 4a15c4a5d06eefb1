"""BIRCH clustering, the K-agnostic module InfraredGP feeds its embeddings to.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper obtains a partition by fitting BIRCH (Zhang, Ramakrishnan & Livny,
SIGMOD 1996) to the embeddings (Sec. III, Alg. 1 final step) and, for
streaming, by partially fitting it to the embeddings of newly added nodes
(Alg. 2); it uses scikit-learn's implementation with no preset number of
clusters (Sec. IV).  This module states that algorithm plainly, in FP64:

* a clustering feature CF = (n, LS, SS): number of points, their linear sum
  and the sum of their squared norms; the centroid is LS / n and the squared
  radius SS / n - |LS / n|^2 (mean squared distance to the centroid);
* the CF-tree: every node holds at most B entries (the branching factor,
  leaves included); an inner entry summarises its child's entries;
* inserting a point: from the root, follow the entry whose centroid is
  nearest to the point (Euclidean; the first one on ties) down to a leaf.  In
  the leaf the nearest entry absorbs the point if the absorbed entry's radius
  stays within the threshold T; otherwise the point becomes a new entry.  On
  the way back every entry on the path adds the point to its CF;
* a node with more than B entries splits: the two entries with the farthest
  centroids (the first such pair (p, q), p < q, in row-major order; squared
  distances |c_p|^2 + |c_q|^2 - 2 c_p.c_q, at least 0) seed two new nodes;
  every entry strictly nearer to the first seed joins it, the others join the
  second, and the first seed always stays in the first node; in the parent
  the entry of the old node is replaced by the first new node's summary and
  the second is appended (which may overflow the parent in turn); a split of
  the root adds a new root above the two halves;
* the result: the leaf entries in leaf order (left to right) are the
  clusters; each point's label is the index of the nearest leaf-entry
  centroid.

Distances are compared as |c|^2 - 2 x.c (the point's own norm is common to
every candidate).  Pinned against scikit-learn's Birch (a library
implementation of the same algorithm) by the CPU tests.
"""
from __future__ import annotations

import numpy as np


class _Node:
    __slots__ = ("leaf", "n", "ls", "ss", "child", "next_leaf")

    def __init__(self, leaf: bool, d: int):
        self.leaf = leaf
        self.n = []          # per entry: count (int)
        self.ls = np.zeros((0, d))  # per entry: linear sum
        self.ss = []         # per entry: sum of squared norms
        self.child = []      # per entry: child node (inner nodes)
        self.next_leaf = None

    def centroids(self):
        return self.ls / np.asarray(self.n, dtype=np.float64)[:, None]

    def nearest(self, x):
        c = self.centroids()
        dist = np.einsum("ij,ij->i", c, c) - 2.0 * (c @ x)
        return int(np.argmin(dist))

    def append(self, n, ls, ss, child=None):
        self.n.append(n)
        self.ls = np.vstack([self.ls, ls[None, :]])
        self.ss.append(ss)
        self.child.append(child)


def _summary(node):
    return sum(node.n), node.ls.sum(axis=0), float(sum(node.ss))


class Birch:
    """BIRCH with threshold T and branching factor B (see the module text)."""

    def __init__(self, threshold: float, branching_factor: int = 50):
        if branching_factor < 2:
            raise ValueError("branching factor must be at least 2")
        self.T = float(threshold)
        self.B = int(branching_factor)
        self.root = None
        self.first_leaf = None
        self.d = None

    # -- insertion ---------------------------------------------------------
    def partial_fit(self, X):
        X = np.asarray(X, dtype=np.float64)
        if self.root is None:
            self.d = X.shape[1]
            self.root = _Node(True, self.d)
            self.first_leaf = self.root
        for x in X:
            if self._insert(self.root, x):
                a, b = self._split(self.root)
                root = _Node(False, self.d)
                root.append(*_summary(a), a)
                root.append(*_summary(b), b)
                self.root = root
        return self

    def fit(self, X):
        self.root = None
        return self.partial_fit(X)

    def _insert(self, node, x):
        """Insert x below node; True if node now holds more than B entries."""
        if not node.n:
            node.append(1, x, float(x @ x))
            return False
        k = node.nearest(x)
        if not node.leaf:
            child = node.child[k]
            if self._insert(child, x):
                a, b = self._split(child)
                node.n[k], node.ls[k], node.ss[k] = _summary(a)
                node.child[k] = a
                node.append(*_summary(b), b)
                return len(node.n) > self.B
            node.n[k] += 1
            node.ls[k] = node.ls[k] + x
            node.ss[k] += float(x @ x)
            return False
        n = node.n[k] + 1
        ls = node.ls[k] + x
        ss = node.ss[k] + float(x @ x)
        c = ls / n
        if ss / n - float(c @ c) <= self.T * self.T:
            node.n[k], node.ls[k], node.ss[k] = n, ls, ss
            return False
        node.append(1, x, float(x @ x))
        return len(node.n) > self.B

    def _split(self, node):
        """Split node in two by the farthest pair of entry centroids; the two
        new nodes take node's place in the leaf order."""
        c = node.centroids()
        nrm = np.einsum("ij,ij->i", c, c)
        up = np.triu(np.maximum(nrm[:, None] + nrm[None, :] - 2.0 * (c @ c.T), 0.0), 1)
        dist = up + up.T          # squared distances, exactly symmetric, zero diagonal
        p, q = np.unravel_index(int(np.argmax(up)), up.shape)
        to_a = dist[p] < dist[q]
        to_a[p] = True
        a, b = _Node(node.leaf, self.d), _Node(node.leaf, self.d)
        for i in range(len(node.n)):
            (a if to_a[i] else b).append(node.n[i], node.ls[i], node.ss[i], node.child[i])
        if node.leaf:
            self._replace_leaf(node, a, b)
        return a, b

    def _replace_leaf(self, old, a, b):
        a.next_leaf, b.next_leaf = b, old.next_leaf
        if self.first_leaf is old:
            self.first_leaf = a
            return
        prev = self.first_leaf
        while prev.next_leaf is not old:
            prev = prev.next_leaf
        prev.next_leaf = a

    # -- result ------------------------------------------------------------
    def centers(self):
        """Leaf-entry centroids in leaf order (M x d)."""
        out = []
        leaf = self.first_leaf
        while leaf is not None:
            if leaf.n:
                out.append(leaf.centroids())
            leaf = leaf.next_leaf
        return np.vstack(out) if out else np.zeros((0, self.d))

    def predict(self, X):
        """Index of the nearest leaf-entry centroid for every row of X."""
        return predict(X, self.centers())


def predict(X, centers):
    """argmin_m |c_m|^2 - 2 x.c_m per row of X (first index on ties)."""
    X = np.asarray(X, dtype=np.float64)
    nrm = np.einsum("ij,ij->i", centers, centers)
    out = np.empty(X.shape[0], dtype=np.int64)
    for a in range(0, X.shape[0], 4096):
        dist = nrm[None, :] - 2.0 * (X[a:a + 4096] @ centers.T)
        out[a:a + 4096] = np.argmin(dist, axis=1)
    return out


def reduced_distances(X, centers):
    """|c_m|^2 - 2 x.c_m for every row of X and every center (for checking a
    label against the best alternative)."""
    X = np.asarray(X, dtype=np.float64)
    nrm = np.einsum("ij,ij->i", centers, centers)
    return nrm[None, :] - 2.0 * (X @ centers.T)
