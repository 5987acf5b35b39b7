"""Dense matrices of the CCMF grid operators built by explicit index loops from
the paper's definitions (Sec. 2.2, Sec. 3.1), used to pin the oracle."""

import itertools
import math

import numpy as np
import scipy.linalg

def _lin(dims, i, j, k):
    n1, n2, n3 = dims
    return ((i % n1) * n2 + (j % n2)) * n3 + (k % n3)


def _voxels(dims):
    return itertools.product(range(dims[0]), range(dims[1]), range(dims[2]))


def dense_div_minus(dims):
    """div^- as a dense N x 3N matrix, from the face-flux balance of
    eq:theory_CCMF_mass_conservation with v_x[i,j,k] = v[i+1/2,j,k] etc."""
    n = int(np.prod(dims))
    D = np.zeros((n, 3 * n))
    for (i, j, k) in _voxels(dims):
        row = _lin(dims, i, j, k)
        # v[i+1/2] - v[i-1/2] + v[j+1/2] - v[j-1/2] + v[k+1/2] - v[k-1/2]
        D[row, 0 * n + _lin(dims, i, j, k)] += 1
        D[row, 0 * n + _lin(dims, i - 1, j, k)] -= 1
        D[row, 1 * n + _lin(dims, i, j, k)] += 1
        D[row, 1 * n + _lin(dims, i, j - 1, k)] -= 1
        D[row, 2 * n + _lin(dims, i, j, k)] += 1
        D[row, 2 * n + _lin(dims, i, j, k - 1)] -= 1
    return D


def dense_grad_plus(dims):
    n = int(np.prod(dims))
    G = np.zeros((3 * n, n))
    for (i, j, k) in _voxels(dims):
        x = _lin(dims, i, j, k)
        for c, (di, dj, dk) in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
            G[c * n + x, _lin(dims, i + di, j + dj, k + dk)] += 1
            G[c * n + x, x] -= 1
    return G


def dense_shift_back(dims):
    n = int(np.prod(dims))
    S = np.zeros((3 * n, 3 * n))
    for (i, j, k) in _voxels(dims):
        x = _lin(dims, i, j, k)
        S[0 * n + x, 0 * n + _lin(dims, i - 1, j, k)] = 1
        S[1 * n + x, 1 * n + _lin(dims, i, j - 1, k)] = 1
        S[2 * n + x, 2 * n + _lin(dims, i, j, k - 1)] = 1
    return S


def dense_A(dims):
    n3 = 3 * int(np.prod(dims))
    return np.vstack([np.eye(n3), dense_shift_back(dims)]) / math.sqrt(2.0)


def dense_proj_K(w, xibar, dims):
    """Projection onto K = {xi : A* xi - xibar in range(grad^+)} by dense linear
    algebra: K = {xi : M xi = b} with the rows of M spanning the complement."""
    n = int(np.prod(dims))
    A = dense_A(dims)
    G = dense_grad_plus(dims)
    Q = scipy.linalg.null_space(G.T)           # complement of range(grad^+)
    M = Q.T @ A.T
    xbar = np.concatenate([np.full(n, xibar[c]) for c in range(3)])
    b = Q.T @ xbar
    wf = w.ravel()
    return wf - np.linalg.pinv(M) @ (M @ wf - b)
