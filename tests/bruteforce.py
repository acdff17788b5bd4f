"""Brute-force references that pin the oracle: the elimination game on a
dense boolean matrix and dense LAPACK Cholesky (numpy).  Tiny inputs only."""
import numpy as np


def dense_lower(n, colptr, rowidx, values=None):
    A = np.zeros((n, n), dtype=np.float64 if values is not None else bool)
    c = np.repeat(np.arange(n), np.diff(colptr))
    A[rowidx, c] = values if values is not None else True
    A[c, rowidx] = values if values is not None else True
    return A


def elimination_game(G):
    """Pattern of L for the symmetric boolean pattern G (diagonal ignored).

    Eliminating vertex j connects all its later neighbours pairwise; the
    column pattern of L is the set of later neighbours at elimination time.
    Returns (parent, cols) with cols[j] the sorted rows i > j of L[:, j].
    """
    G = np.array(G, dtype=bool)
    n = G.shape[0]
    np.fill_diagonal(G, False)
    parent = np.full(n, -1)
    cols = []
    for j in range(n):
        nz = np.nonzero(G[j + 1:, j])[0] + j + 1
        cols.append(nz)
        if nz.size:
            parent[j] = nz[0]
            G[np.ix_(nz, nz)] = True
            np.fill_diagonal(G, False)
    return parent, cols


def permuted_dense(n, colptr, rowidx, values, perm):
    A = dense_lower(n, colptr, rowidx, values)
    return A[np.ix_(perm, perm)]
