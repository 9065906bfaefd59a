"""FP64 reference for the differentiable RWR (TEST INFRASTRUCTURE ONLY).

Edge weights are learned through RWR (Appendix F, Eq. 9): every entry e = (i, j)
of the symmetrised adjacency has features f_e, and

    z_e = theta . f_e,   w_e = softplus(z_e) = log(1 + exp(z_e)),
    W_ij = w_e / S_j,    S_j = sum of w over column j   (column-normalised),
    r^0 = e_s,   r^{k+1} = c W r^k + (1 - c) e_s,   k = 0 .. K-1.

The gradient of a loss L(r^K) with respect to theta follows the chain rule
backwards through the iteration (reverse-mode, adjoint vectors g^k = dL/dr^k):

    g^k = c W^T g^{k+1},          dL/dW_ij += c g^{k+1}_i r^k_j,
    dL/dw_ij = (dL/dW_ij - sum_i' dL/dW_i'j W_i'j) / S_j,
    dL/dz_e = dL/dw_e * sigmoid(z_e),   dL/dtheta = sum_e dL/dz_e f_e.

Plain numpy in FP64, one iteration at a time; scipy's CSR product is the
matrix-vector step.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def edge_rows(rp: np.ndarray) -> np.ndarray:
    """Row index of every entry of a CSR pattern."""
    return np.repeat(np.arange(len(rp) - 1), np.diff(rp))


def weights(n: int, rp, col, feats, theta):
    """z, w, S and the column-normalised values W (all FP64)."""
    z = feats.astype(np.float64) @ np.asarray(theta, np.float64)
    w = np.logaddexp(0.0, z)
    S = np.bincount(col, weights=w, minlength=n)
    W = w / S[col]
    return z, w, S, W


def rwr_iterates(n: int, rp, col, W, seed: int, c: float, K: int):
    """[r^0, ..., r^K] in FP64."""
    A = sp.csr_matrix((W, col, rp), shape=(n, n))
    r = np.zeros(n)
    r[seed] = 1.0
    out = [r]
    for _ in range(K):
        r = c * (A @ r)
        r[seed] += 1.0 - c
        out.append(r)
    return out


def loss_of(rK, targets) -> float:
    """The benchmark's loss: minus the summed log scores of the target nodes."""
    return float(-np.sum(np.log(rK[np.asarray(targets)])))


def loss_and_grad(n: int, rp, col, feats, theta, seed: int, targets, c: float, K: int):
    """(loss, dL/dtheta, r^K) for L = -sum_t log r^K_t, all in FP64."""
    z, w, S, W = weights(n, rp, col, feats, theta)
    rs = rwr_iterates(n, rp, col, W, seed, c, K)
    loss = loss_of(rs[K], targets)
    g = np.zeros(n)
    np.add.at(g, np.asarray(targets), -1.0 / rs[K][np.asarray(targets)])
    return (loss,) + backward(n, rp, col, feats, z, S, W, rs, g, c)[:1] + (rs[K],)


def backward(n: int, rp, col, feats, z, S, W, rs, gK, c: float):
    """Adjoint pass from g^K = dL/dr^K: (dL/dtheta, dL/dW per entry, g^0)."""
    K = len(rs) - 1
    rows = edge_rows(rp)
    At = sp.csr_matrix((W, col, rp), shape=(n, n)).T.tocsr()
    G = np.zeros(len(col))
    g = gK.astype(np.float64)
    for k in range(K - 1, -1, -1):
        G += g[rows] * rs[k][col]        # uses g^{k+1} and r^k
        g = c * (At @ g)                 # g^k
    dW = c * G
    colsum = np.bincount(col, weights=dW * W, minlength=n)
    dw = (dW - colsum[col]) / S[col]
    dz = dw / (1.0 + np.exp(-z))
    dtheta = feats.astype(np.float64).T @ dz
    return dtheta, dW, g
