"""Pins of the FP64 differentiable-RWR reference (oracle/rwr_grad.py): the
gradient against central finite differences of the loss (which use only the
forward), the forward against the C oracle's RWR, the adjoint against
differences in single matrix entries, and a case whose exact gradient is 0."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import rwr_grad as rg

C, K = 0.85, 30


def problem(scale=10, ef=8, seed=31):
    g = gg.rmat(scale, ef, seed=seed)
    n, _, rp, col, _ = gg.rwr_matrix(g)
    feats = gg.normal_f32(len(col) * 4, seed + 1).reshape(len(col), 4)
    s = int(gg.rwr_seeds(g, 1, seed + 2)[0])
    theta = np.array([0.4, -0.3, 0.2, 0.1])
    # 16 targets among the nodes the walk reaches
    z, w, S, W = rg.weights(n, rp, col, feats, theta)
    rK = rg.rwr_iterates(n, rp, col, W, s, C, K)[K]
    reach = np.nonzero(rK > 1e-12)[0]
    targets = reach[gg.random_permutation(len(reach), seed + 3)[:16]]
    return n, rp, col, feats, theta, s, targets


def test_gradient_matches_central_differences():
    n, rp, col, feats, theta, s, targets = problem()
    loss, grad, _ = rg.loss_and_grad(n, rp, col, feats, theta, s, targets, C, K)
    for d in range(4):
        h = 1e-5
        tp, tm = theta.copy(), theta.copy()
        tp[d] += h
        tm[d] -= h
        lp = rg.loss_of(rg.rwr_iterates(n, rp, col, rg.weights(n, rp, col, feats, tp)[3], s, C, K)[K], targets)
        lm = rg.loss_of(rg.rwr_iterates(n, rp, col, rg.weights(n, rp, col, feats, tm)[3], s, C, K)[K], targets)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[d]) <= 1e-6 * max(1.0, abs(fd)), (d, fd, grad[d])


def test_forward_matches_the_c_oracle():
    n, rp, col, feats, theta, s, _ = problem(scale=9)
    W32 = rg.weights(n, rp, col, feats, theta)[3].astype(np.float32)
    mine = rg.rwr_iterates(n, rp, col, W32.astype(np.float64), s, C, K)[K]
    R, _, _ = oracle.rwr((n, n, rp, col, W32), [s], C, 0.0, K)
    assert np.allclose(mine, R[:, 0], rtol=0, atol=1e-14)


def test_adjoint_against_single_entry_differences():
    # dL/dW_e from the adjoint against moving one matrix entry (no normalisation)
    n, rp, col, feats, theta, s, targets = problem(scale=8, ef=6)
    z, w, S, W = rg.weights(n, rp, col, feats, theta)
    rs = rg.rwr_iterates(n, rp, col, W, s, C, K)
    gK = np.zeros(n)
    np.add.at(gK, targets, -1.0 / rs[K][targets])
    _, dW, _ = rg.backward(n, rp, col, feats, z, S, W, rs, gK, C)
    for e in gg.uniform_int(12, len(col), 99):
        h = 1e-6
        Wp, Wm = W.copy(), W.copy()
        Wp[e] += h
        Wm[e] -= h
        fd = (rg.loss_of(rg.rwr_iterates(n, rp, col, Wp, s, C, K)[K], targets)
              - rg.loss_of(rg.rwr_iterates(n, rp, col, Wm, s, C, K)[K], targets)) / (2 * h)
        assert abs(fd - dW[e]) <= 1e-6 * max(1.0, abs(fd)), (e, fd, dW[e])


def test_one_entry_per_column_gives_zero_gradient():
    # a perfect matching: every column holds one entry, so W = 1 whatever the
    # weights, and the loss does not depend on theta
    n = 64
    src = np.arange(0, n, 2)
    g = gg.from_edges(n, src, src + 1)
    n, _, rp, col, _ = gg.rwr_matrix(g)
    feats = gg.normal_f32(len(col) * 4, 5).reshape(len(col), 4)
    loss, grad, rK = rg.loss_and_grad(n, rp, col, feats, np.array([1.0, -2.0, 0.5, 3.0]), 4, [4, 5], C, K)
    assert np.all(grad == 0.0)
    # the walk stays on the pair {4, 5}: a_{k+2} = c^2 a_k + (1 - c), a_0 = 1,
    # so after an even K, r_4 = c^K + (1 - c) sum_{m < K/2} c^{2m}
    a = C ** K + (1 - C) * sum(C ** (2 * m) for m in range(K // 2))
    assert abs(rK[4] - a) <= 1e-15
    assert abs(rK[4] + rK[5] - 1.0) <= 1e-15


def test_repeated_targets_count_twice():
    n, rp, col, feats, theta, s, targets = problem(scale=8, ef=6)
    l1, g1, _ = rg.loss_and_grad(n, rp, col, feats, theta, s, list(targets[:3]), C, K)
    l2, g2, _ = rg.loss_and_grad(n, rp, col, feats, theta, s, list(targets[:3]) * 2, C, K)
    assert abs(l2 - 2 * l1) <= 1e-12 * abs(l1)
    assert np.allclose(g2, 2 * g1, rtol=1e-12, atol=0)
