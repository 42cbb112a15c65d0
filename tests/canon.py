"""Helpers that compare mode blocks and coarse quantities of two hierarchies.

Retained modes are unique only up to an orthogonal change of basis inside each
eigencluster (a sign for a simple eigenvalue), so coarse DOFs of two
hierarchies built from the same level differ by a block-diagonal orthogonal
map.  _canon puts every cluster of a mode block in one basis fixed by the
block alone, so that quantities can be compared after that map.
"""
import numpy as np
import scipy.sparse as sp


def _csr(ex):
    n = len(ex["rowptr"]) - 1
    return sp.csr_matrix((ex["val"], ex["col"], ex["rowptr"]), shape=(n, n))


def _canon(Z, mu, nw, tol=1e-7):
    """Orthogonal k x k transform putting each eigencluster of Z in a canonical basis."""
    k = Z.shape[1]
    Q = np.zeros((k, k))
    d = np.sqrt(np.arange(nw) + 2.0)
    c0 = 0
    while c0 < k:
        c1 = c0 + 1
        while c1 < k and mu[c1] - mu[c1 - 1] <= tol * max(1.0, abs(mu[c1])):
            c1 += 1
        W = Z[:, c0:c1]
        K = W.T @ (d[:, None] * W)
        _, U = np.linalg.eigh(K)
        Wc = W @ U
        gvec = np.sin(1.0 + 0.7 * np.arange(nw))          # generic, so no sign ties
        for j in range(c1 - c0):
            if gvec @ Wc[:, j] < 0:
                U[:, j] *= -1
        Q[c0:c1, c0:c1] = U
        c0 = c1
    return Q


def _gpu_Z_blocks(ex, nw_list):
    out, off = [], 0
    for nw, k in zip(nw_list, ex["k"]):
        out.append(ex["Z"][off:off + nw * k].reshape(nw, k))
        off += nw * k
    return out
