"""Pins of the oracle's power iterations (Appendix F): closed forms, exact
linear solves on tiny graphs, and the invariants of each iteration."""
import numpy as np
import pytest

import graphgen as gg
import oracle


# ---------------------------------------------------------------- PageRank
def _google_solve(n, src, dst, c):
    """p* from (I - c G) p = (1-c)/n 1 with G = column-stochastic transition
    matrix, dangling columns replaced by 1/n (built here from the edge list)."""
    A = np.zeros((n, n))
    A[src, dst] = 1.0
    G = np.zeros((n, n))
    for u in range(n):
        d = A[u].sum()
        G[:, u] = A[u] / d if d > 0 else 1.0 / n
    return np.linalg.solve(np.eye(n) - c * G, np.full(n, (1 - c) / n))


def test_pagerank_cycle_is_uniform_every_iteration():
    n = 17  # n - 1 = 16: every 1/(n-1) exact
    g = gg.from_edges(n, np.arange(n), (np.arange(n) + 1) % n)
    for k in (1, 2, 7):
        p, it, res = oracle.pagerank(gg.pagerank_matrix(g), 0.85, 0.0, k)
        assert it == k
        assert np.allclose(p, 1.0 / n, rtol=0, atol=1e-16)


def test_pagerank_complete_graph_uniform():
    n = 9
    s, d = np.meshgrid(np.arange(n), np.arange(n))
    m = s != d
    g = gg.from_edges(n, s[m], d[m])
    p, _, _ = oracle.pagerank(gg.pagerank_matrix(g), 0.85, 0.0, 5)
    assert np.allclose(p, 1.0 / n, atol=1e-16)


@pytest.mark.parametrize("L", [1, 4, 31])
def test_pagerank_star_closed_form(L):
    c = 0.85
    n = L + 1
    leaves = np.arange(1, n)
    g = gg.from_edges(n, np.concatenate([np.zeros(L, int), leaves]), np.concatenate([leaves, np.zeros(L, int)]))
    p, it, res = oracle.pagerank(gg.pagerank_matrix(g), c, 1e-15, 5000)
    pc = (1 + c * L) / ((L + 1) * (1 + c))
    pl = (L + c) / (L * (L + 1) * (1 + c))
    # fl32(1/L) values make the matrix only approximately stochastic
    assert abs(p[0] - pc) < 1e-7 and np.allclose(p[1:], pl, atol=1e-7)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_pagerank_tiny_graphs_exact_solve(seed):
    rng = np.random.default_rng(seed)
    n = 12
    m = rng.integers(5, 40)
    src, dst = rng.integers(0, n, m), rng.integers(0, n, m)
    # power-of-two out-degrees are impossible to force; use FP64 tolerance of
    # the fl32(1/d) values instead
    g = gg.from_edges(n, src, dst)
    assert (np.bincount(g.src, minlength=n) == 0).any() or seed != 0  # seed 0 has dangling nodes
    p, it, _ = oracle.pagerank(gg.pagerank_matrix(g), 0.85, 1e-15, 5000)
    ref = _google_solve(n, g.src, g.dst, 0.85)
    assert np.allclose(p, ref, atol=2e-7)
    assert abs(p.sum() - 1.0) < 1e-6


def test_pagerank_mass_and_contraction():
    g = gg.rmat(8, 6, seed=5)
    M = gg.pagerank_matrix(g)
    c = 0.85
    pstar, _, _ = oracle.pagerank(M, c, 1e-15, 10000)
    for k in (1, 3, 10, 30):
        p, _, res = oracle.pagerank(M, c, 0.0, k)
        assert abs(p.sum() - 1.0) < 1e-6
        assert np.abs(p - pstar).sum() <= 2 * c ** k + 1e-9
    p1, _, r1 = oracle.pagerank(M, c, 0.0, 11)
    p0, _, _ = oracle.pagerank(M, c, 0.0, 10)
    assert abs(r1[-1] - np.abs(p1 - p0).sum()) < 1e-15


def test_pagerank_stops_at_tolerance():
    g = gg.rmat(8, 6, seed=6)
    p, it, res = oracle.pagerank(gg.pagerank_matrix(g), 0.85, 1e-6, 1000)
    assert res[-1] <= 1e-6 and (it == 1 or res[-2] > 1e-6)


# -------------------------------------------------------------------- HITS
def test_hits_complete_bipartite():
    s_nodes, t_nodes = np.arange(0, 3), np.arange(3, 8)
    S, T = np.meshgrid(s_nodes, t_nodes)
    n = 10  # nodes 8, 9 isolated
    g = gg.from_edges(n, S.ravel(), T.ravel())
    x, it, res = oracle.hits(gg.hits_matrix(g), 0.0, 3)
    a, h = x[:n], x[n:]
    assert np.allclose(a[t_nodes], 1 / 5, atol=1e-16) and np.allclose(np.delete(a, t_nodes), 0)
    assert np.allclose(h[s_nodes], 1 / 3, atol=1e-16) and np.allclose(np.delete(h, s_nodes), 0)


def test_hits_matches_svd():
    rng = np.random.default_rng(4)
    n = 15
    g = gg.from_edges(n, rng.integers(0, n, 60), rng.integers(0, n, 60))
    A = np.zeros((n, n))
    A[g.src, g.dst] = 1
    U, sv, Vt = np.linalg.svd(A)
    assert sv[0] > 1.2 * sv[1]
    x, it, res = oracle.hits(gg.hits_matrix(g), 1e-14, 5000)
    a, h = x[:n], x[n:]
    v1, u1 = np.abs(Vt[0]), np.abs(U[:, 0])
    assert np.allclose(a, v1 / v1.sum(), atol=1e-10)
    assert np.allclose(h, u1 / u1.sum(), atol=1e-10)


def test_hits_halves_sum_to_one():
    g = gg.rmat(8, 8, seed=9)
    n = g.n
    for k in (1, 2, 5):
        x, _, _ = oracle.hits(gg.hits_matrix(g), 0.0, k)
        assert abs(x[:n].sum() - 1) < 1e-12 and abs(x[n:].sum() - 1) < 1e-12


def test_hits_rejects_empty_graph():
    g = gg.from_edges(4, [], [])
    with pytest.raises(ValueError):
        oracle.hits(gg.hits_matrix(g), 0.0, 2)


# --------------------------------------------------------------------- RWR
def test_rwr_directed_cycle_closed_form():
    n, c, s = 10, 0.85, 3
    # W = shift: column i holds a single 1 in row i+1
    rp = np.arange(n + 1, dtype=np.int64)
    col = ((np.arange(n) - 1) % n).astype(np.int32)
    W = (n, n, rp, col, np.ones(n, np.float32))
    R, it, res = oracle.rwr(W, np.array([s]), c, 1e-16, 2000)
    k = np.arange(n)
    ref = (1 - c) * c ** k / (1 - c ** n)
    assert np.allclose(R[(s + k) % n, 0], ref, atol=1e-15)


def test_rwr_exact_solve_and_mass():
    rng = np.random.default_rng(8)
    n = 14
    g = gg.from_edges(n, rng.integers(0, n, 30), rng.integers(0, n, 30))
    Wc = gg.rwr_matrix(g)
    Wd = np.zeros((n, n))
    Wd[np.repeat(np.arange(n), np.diff(Wc[2])), Wc[3]] = Wc[4]
    deg = np.bincount(np.concatenate([g.src, g.dst]), minlength=n)
    seeds = np.nonzero(deg > 0)[0][:3].astype(np.int32)
    c = 0.85
    R, it, res = oracle.rwr(Wc, seeds, c, 1e-15, 5000)
    for q, s in enumerate(seeds):
        e = np.zeros(n)
        e[s] = 1
        ref = np.linalg.solve(np.eye(n) - c * Wd, (1 - c) * e)
        assert np.allclose(R[:, q], ref, atol=1e-12)
    for k in (1, 2, 6):
        Rk, _, resk = oracle.rwr(Wc, seeds, c, 0.0, k)
        assert np.allclose(Rk.sum(axis=0), 1.0, atol=1e-6)
        assert np.all(resk[-1] <= 2 * c ** k + 1e-7)
