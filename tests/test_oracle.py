"""Pins of the CPU oracle against brute force, closed forms, certificates and
the paper's worked example.  CPU only."""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
from paper_1812_04070_amd import gen
from tests import pins

INF = oracle.INF
HERE = os.path.dirname(os.path.abspath(__file__))


def _g(n, edges, w=None, directed=False):
    return gen.from_edges(n, edges, w, directed=directed)


# ------------------------------------------------------------ exhaustive ----

def test_exhaustive_5_vertex_graphs():
    """All 1,024 labelled simple graphs on 5 vertices: BFS and SSSP against
    Floyd-Warshall from every source, core numbers against subset enumeration."""
    rng = np.random.default_rng(5)
    count = 0
    for edges in pins.all_graphs(5):
        w = rng.integers(1, 10, size=len(edges)) if edges else None
        g = _g(5, edges, w if edges else [])
        if g.weights is None:
            g.weights = np.zeros(0, dtype=np.uint32)
        for s in range(5):
            d = oracle.bfs(5, g.offsets, g.indices, s)
            assert np.array_equal(d, pins.fw_depth(5, g.offsets, g.indices, s))
            x = oracle.sssp_dijkstra(5, g.offsets, g.indices, g.weights, s)
            assert np.array_equal(x.astype(np.uint64), pins.fw_dist(5, g.offsets, g.indices, g.weights, s))
            y = oracle.sssp_bellman_ford(5, g.offsets, g.indices, g.weights, s)
            assert np.array_equal(x, y)
        c = oracle.kcore_bz(5, g.offsets, g.indices)
        assert np.array_equal(c, pins.brute_core(5, g.offsets, g.indices))
        assert np.array_equal(c, oracle.kcore_peel(5, g.offsets, g.indices))
        count += 1
    assert count == 1024


@pytest.mark.parametrize("seed", range(12))
def test_random_small_graphs(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 15))
    p = float(rng.uniform(0.1, 0.6))
    g = gen.random_graph(n, p, seed=seed, weights=(1, 20))
    if g.weights is None:
        g.weights = np.zeros(0, dtype=np.uint32)
    for s in range(n):
        assert np.array_equal(oracle.bfs(n, g.offsets, g.indices, s), pins.fw_depth(n, g.offsets, g.indices, s))
        x = oracle.sssp_dijkstra(n, g.offsets, g.indices, g.weights, s)
        assert np.array_equal(x.astype(np.uint64), pins.fw_dist(n, g.offsets, g.indices, g.weights, s))
        assert np.array_equal(x, oracle.sssp_bellman_ford(n, g.offsets, g.indices, g.weights, s))
        assert np.array_equal(x, oracle.sssp_rounds(n, g.offsets, g.indices, g.weights, s)[0])
    if n <= 12:
        assert np.array_equal(oracle.kcore_g(g), pins.brute_core(n, g.offsets, g.indices))
    pins.kcore_certificate(n, g.offsets, g.indices, oracle.kcore_g(g))


@pytest.mark.parametrize("seed", range(8))
def test_random_small_digraphs(seed):
    """Directed: core numbers with degree = in + out against subset enumeration;
    PageRank against the dense Google-matrix power iteration."""
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(2, 12))
    g = gen.random_graph(n, float(rng.uniform(0.1, 0.5)), seed=seed, directed=True)
    c = oracle.kcore_g(g)
    assert np.array_equal(c, pins.brute_core(n, g.offsets, g.indices, g.in_offsets, g.in_indices))
    assert np.array_equal(c, oracle.kcore_peel(n, g.offsets, g.indices, g.in_offsets, g.in_indices))
    x = oracle.pagerank_g(g, 0.85, 20)
    xd, G = pins.pagerank_dense(n, g.offsets, g.in_offsets, g.in_indices, 0.85, 20)
    np.testing.assert_allclose(x, xd, rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------- closed forms ----

def test_path_cycle_star_complete():
    n = 9
    path = _g(n, [(i, i + 1) for i in range(n - 1)], [1] * (n - 1))
    assert np.array_equal(oracle.bfs_g(path, 0), np.arange(n))
    assert np.array_equal(oracle.bfs_g(path, 4), np.abs(np.arange(n) - 4))
    assert np.array_equal(oracle.kcore_g(path), np.ones(n))
    cyc = _g(n, [(i, (i + 1) % n) for i in range(n)], [2] * n)
    exp = np.minimum(np.arange(n), n - np.arange(n))
    assert np.array_equal(oracle.bfs_g(cyc, 0), exp)
    assert np.array_equal(oracle.sssp_g(cyc, 0), 2 * exp)
    assert np.array_equal(oracle.kcore_g(cyc), np.full(n, 2))
    star = _g(n, [(0, i) for i in range(1, n)], list(range(1, n)))
    assert np.array_equal(oracle.bfs_g(star, 0), np.r_[0, np.ones(n - 1)])
    assert np.array_equal(oracle.bfs_g(star, 3), np.r_[1, np.full(n - 1, 2)] - np.eye(n, dtype=int)[3] * 2)
    assert np.array_equal(oracle.sssp_g(star, 0), np.arange(n))
    assert np.array_equal(oracle.kcore_g(star), np.ones(n))
    for k in range(1, 8):
        kn = _g(k, [(i, j) for i in range(k) for j in range(i + 1, k)])
        assert np.array_equal(oracle.kcore_g(kn), np.full(k, k - 1))
    # isolated vertices: depth -1, distance inf, core 0
    iso = _g(4, [(0, 1)], [3])
    assert np.array_equal(oracle.bfs_g(iso, 0), [0, 1, -1, -1])
    assert np.array_equal(oracle.sssp_g(iso, 0), [0, 3, INF, INF])
    assert np.array_equal(oracle.kcore_g(iso), [1, 1, 0, 0])


def test_grid_without_deletions():
    """Full grid from corner 0: depth = Manhattan distance r + c; unit weights
    give the same SSSP; every vertex has core number 2."""
    side = 37
    g = gen.grid(side, 0.0, seed=1)
    r, c = np.divmod(np.arange(side * side), side)
    assert np.array_equal(oracle.bfs_g(g, 0), r + c)
    g.weights = np.ones(g.m, dtype=np.uint32)
    assert np.array_equal(oracle.sssp_g(g, 0), (r + c).astype(np.uint32))
    assert np.array_equal(oracle.kcore_g(g), np.full(side * side, 2))


def test_pagerank_closed_forms():
    n = 7
    # directed cycle: every vertex receives exactly one unit of flow -> 1/n forever
    cyc = _g(n, [(i, (i + 1) % n) for i in range(n)], directed=True)
    np.testing.assert_allclose(oracle.pagerank_g(cyc), np.full(n, 1 / n), rtol=0, atol=1e-16)
    # edgeless graph: all vertices dangle -> 1/n forever
    empty = _g(n, [], directed=True)
    np.testing.assert_allclose(oracle.pagerank_g(empty), np.full(n, 1 / n), rtol=0, atol=1e-16)
    # in-star after one iteration: leaves -> centre 0, the centre dangles
    d = 0.85
    star = _g(n, [(i, 0) for i in range(1, n)], directed=True)
    x1 = oracle.pagerank_g(star, d, 1)
    centre = (1 - d) / n + d * ((n - 1) / n + 1 / n ** 2)
    leaf = (1 - d) / n + d / n ** 2
    np.testing.assert_allclose(x1, np.r_[centre, np.full(n - 1, leaf)], rtol=1e-15)
    # zero iterations: the uniform start vector
    np.testing.assert_allclose(oracle.pagerank_g(star, d, 0), np.full(n, 1 / n))


def test_pagerank_converges_to_eigenvector():
    """Run to convergence and compare with numpy's eigenvector of the Google matrix."""
    g = gen.random_graph(11, 0.25, seed=3, directed=True)
    x = oracle.pagerank_g(g, 0.85, 400)
    _, G = pins.pagerank_dense(g.n, g.offsets, g.in_offsets, g.in_indices, 0.85, 0)
    np.testing.assert_allclose(x, pins.pagerank_stationary(G), rtol=1e-10)


def test_pagerank_invariants_rmat():
    g = gen.rmat(12, seed=4, directed=True)
    x = oracle.pagerank_g(g)
    assert abs(x.sum() - 1.0) < 1e-12
    assert np.all(x >= (1 - 0.85) / g.n - 1e-18)


# ---------------------------------------------------- the worked example ----

def _load_example():
    edges, w, facts = [], [], {}
    for line in open(os.path.join(HERE, "golden", "sssp_worked_example.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0] == "e":
            edges.append((ord(tok[1]) - 97, ord(tok[2]) - 97))
            w.append(int(tok[3]))
        else:
            facts[tok[0]] = tok[1:]
    return edges, w, facts


def test_worked_example_rounds():
    edges, w, facts = _load_example()
    g = _g(9, edges, w)
    V = lambda s: ord(s) - 97
    # iteration 1 from a: b=5, d=1 and nothing else
    d1, u1, _ = oracle.sssp_rounds(9, g.offsets, g.indices, g.weights, 0, max_rounds=1)
    for kv in facts["iter1_updates"]:
        k, v = kv.split("=")
        assert d1[V(k)] == int(v)
    assert sorted(np.nonzero(u1 == 1)[0].tolist()) == sorted(V(x.split("=")[0]) for x in facts["iter1_updates"])
    # iteration 2: active {b, d} -> next {c, e}
    d2, u2, _ = oracle.sssp_rounds(9, g.offsets, g.indices, g.weights, 0, max_rounds=2)
    assert sorted(np.nonzero(u2 == 1)[0]) == sorted(V(x) for x in facts["iter2_active"])
    assert sorted(np.nonzero(u2 == 2)[0]) == sorted(V(x) for x in facts["iter2_next"])
    # iteration 3: {b, f, g, h, i}; ballot words over a-d and e-i
    d3, u3, _ = oracle.sssp_rounds(9, g.offsets, g.indices, g.weights, 0, max_rounds=3)
    nxt = np.nonzero(u3 == 3)[0].tolist()
    assert nxt == [V(x) for x in facts["iter3_next"]]
    bits = "".join("1" if u3[v] == 3 else "0" for v in range(9))
    assert bits[:4] == facts["ballot_word_a_d"][0]
    assert bits[4:] == facts["ballot_word_e_i"][0]
    # b updated in iterations 1 and 3
    assert d1[V("b")] > d3[V("b")] and u3[V("b")] == 3
    # converged: nothing changes in iteration 4; final distances are the shortest paths
    d, u, rounds = oracle.sssp_rounds(9, g.offsets, g.indices, g.weights, 0)
    assert rounds == 3
    assert np.array_equal(d, oracle.sssp_g(g, 0))
    assert np.array_equal(d.astype(np.uint64), pins.fw_dist(9, g.offsets, g.indices, g.weights, 0))
    deg = np.diff(g.offsets)
    assert deg[V("c")] == int(facts["c_degree"][0]) and deg[V("e")] == int(facts["e_degree"][0])


# --------------------------------------------- certificates at real size ----

def test_certificates_rmat16():
    g = gen.workload_graph("rmat16")
    s = gen.max_degree_vertex(g)
    d = oracle.bfs_g(g, s)
    pins.bfs_certificate(g.n, g.offsets, g.indices, s, d)
    x = oracle.sssp_g(g, s)
    pins.sssp_certificate(g.n, g.offsets, g.indices, g.weights, s, x)
    assert np.array_equal(x, oracle.sssp_bellman_ford(g.n, g.offsets, g.indices, g.weights, s))
    c = oracle.kcore_g(g)
    pins.kcore_certificate_fast(g.n, g.offsets, g.indices, c)
    assert np.array_equal(c, oracle.kcore_peel(g.n, g.offsets, g.indices))
    # unit weights reduce SSSP to BFS
    g1 = gen.Graph(n=g.n, offsets=g.offsets, indices=g.indices, weights=np.ones(g.m, dtype=np.uint32))
    x1 = oracle.sssp_g(g1, s)
    assert np.array_equal(np.where(x1 == INF, -1, x1.astype(np.int64)), d)


def test_scipy_cross_check():
    sp = pytest.importorskip("scipy.sparse")
    csg = pytest.importorskip("scipy.sparse.csgraph")
    g = gen.rmat(11, seed=9, weights=(1, 64))
    s = gen.max_degree_vertex(g)
    A = sp.csr_matrix((g.weights.astype(np.float64), g.indices, g.offsets), shape=(g.n, g.n))
    ref = csg.dijkstra(A, indices=s)
    x = oracle.sssp_g(g, s)
    assert np.array_equal(np.where(np.isinf(ref), INF, ref).astype(np.uint32), x)
    B = sp.csr_matrix((np.ones(g.m), g.indices, g.offsets), shape=(g.n, g.n))
    hop = csg.shortest_path(B, unweighted=True, indices=s)
    assert np.array_equal(np.where(np.isinf(hop), -1, hop).astype(np.int32), oracle.bfs_g(g, s))


def test_networkx_cross_check():
    nx = pytest.importorskip("networkx")
    g = gen.rmat(10, seed=4, directed=True)
    G = nx.DiGraph()
    G.add_nodes_from(range(g.n))
    src = np.repeat(np.arange(g.n), np.diff(g.offsets))
    G.add_edges_from(zip(src.tolist(), g.indices.tolist()))
    ref = nx.core_number(G)
    assert np.array_equal(oracle.kcore_g(g), np.array([ref[v] for v in range(g.n)]))
    gu = gen.rmat(10, seed=5)
    H = nx.Graph()
    H.add_nodes_from(range(gu.n))
    su = np.repeat(np.arange(gu.n), np.diff(gu.offsets))
    H.add_edges_from(zip(su.tolist(), gu.indices.tolist()))
    ref = nx.core_number(H)
    assert np.array_equal(oracle.kcore_g(gu), np.array([ref[v] for v in range(gu.n)]))


# ---------------------------------------- fixed-k k-core and components ----

def test_exhaustive_5_vertex_member_and_wcc():
    """All 1,024 graphs on 5 vertices: k-core membership for k = 0..5 against
    subset enumeration, and component labels against the transitive closure."""
    for edges in pins.all_graphs(5):
        g = _g(5, edges)
        for k in range(6):
            assert np.array_equal(oracle.kcore_member(5, g.offsets, g.indices, k),
                                  pins.brute_kcore_member(5, g.offsets, g.indices, k)), (edges, k)
        assert np.array_equal(oracle.wcc(5, g.offsets, g.indices), pins.closure_min_label(5, g.offsets, g.indices))


@pytest.mark.parametrize("seed", range(6))
def test_member_and_wcc_random_digraphs(seed):
    """Directed graphs (degree = in + out; components ignore direction)."""
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(3, 12))
    g = gen.random_graph(n, float(rng.uniform(0.1, 0.4)), seed=seed, directed=True)
    for k in range(0, 7):
        assert np.array_equal(oracle.kcore_member_g(g, k),
                              pins.brute_kcore_member(n, g.offsets, g.indices, k, g.in_offsets, g.in_indices))
    assert np.array_equal(oracle.wcc_g(g), pins.closure_min_label(n, g.offsets, g.indices))


def test_member_and_wcc_closed_forms():
    # K_6: every vertex has degree 5 -> in the k-core exactly for k <= 5
    kn = _g(6, [(i, j) for i in range(6) for j in range(i + 1, 6)])
    for k in range(8):
        assert np.array_equal(oracle.kcore_member(6, kn.offsets, kn.indices, k), np.full(6, int(k <= 5)))
    # cycle: the 2-core is the whole cycle, the 3-core empty; a pendant path
    # hanging off it is peeled away for k = 2
    cyc = _g(7, [(0, 1), (1, 2), (2, 3), (3, 0), (3, 4), (4, 5), (5, 6)])
    assert np.array_equal(oracle.kcore_member(7, cyc.offsets, cyc.indices, 2), [1, 1, 1, 1, 0, 0, 0])
    assert np.array_equal(oracle.kcore_member(7, cyc.offsets, cyc.indices, 3), np.zeros(7))
    assert np.array_equal(oracle.kcore_member(7, cyc.offsets, cyc.indices, 1), np.ones(7))
    # components: edgeless -> identity; two disjoint paths; a path is one label
    assert np.array_equal(oracle.wcc(4, np.zeros(5, np.int32), np.zeros(0, np.int32)), [0, 1, 2, 3])
    two = _g(7, [(6, 4), (4, 2), (5, 3), (3, 1), (1, 0)])
    assert np.array_equal(oracle.wcc(7, two.offsets, two.indices), [0, 0, 2, 0, 2, 0, 2])
    path = _g(50, [(i, i + 1) for i in range(49)])
    assert np.array_equal(oracle.wcc(50, path.offsets, path.indices), np.zeros(50))


def test_member_equals_decomposition_rmat16():
    """On R-MAT s16 the fixed-k peel and the bucket decomposition (an
    algorithm that never deletes below a fixed k) agree for every k."""
    g = gen.rmat(16, seed=1)
    c = oracle.kcore_g(g)
    for k in (1, 2, 8, 16, 32, 64, int(c.max()), int(c.max()) + 1):
        assert np.array_equal(oracle.kcore_member_g(g, k), (c >= k).astype(np.int32)), k


def test_wcc_scipy_cross_check():
    """Component partition against scipy.sparse.csgraph.connected_components
    (a library routine: same partition, labels = smallest id)."""
    sp = pytest.importorskip("scipy.sparse")
    csg = pytest.importorskip("scipy.sparse.csgraph")
    for g in (gen.rmat(14, seed=3), gen.grid(96, 0.45, seed=5), gen.random_graph(2000, 0.0008, seed=9)):
        A = sp.csr_matrix((np.ones(g.m), g.indices, g.offsets), shape=(g.n, g.n))
        nc, lab = csg.connected_components(A, directed=False)
        mine = oracle.wcc_g(g)
        first = np.full(nc, g.n)
        np.minimum.at(first, lab, np.arange(g.n))
        assert np.array_equal(mine, first[lab])
        assert np.unique(mine).size == nc


def test_pagerank_fixpoint_solves_the_linear_system():
    """The fixed point equals the solution of (I - d P - d/n 1 dangling^T) x =
    (1 - d)/n 1 by numpy.linalg.solve (a library routine on the dense
    system), and the Google matrix's principal eigenvector."""
    for seed, dangle in ((3, True), (4, False), (5, True)):
        g0 = gen.random_graph(14, 0.25, seed=seed, directed=True)
        if dangle:
            src = np.repeat(np.arange(g0.n), np.diff(g0.offsets))
            keep = src % 5 != 0
            g = gen.from_edges(g0.n, np.stack([src[keep], g0.indices[keep]], 1), directed=True)
        else:
            g = g0
        x, steps = oracle.pagerank_fixpoint_g(g, tol=1e-15)
        n = g.n
        outdeg = np.diff(g.offsets)
        P = np.zeros((n, n))
        for v in range(n):
            for e in range(g.in_offsets[v], g.in_offsets[v + 1]):
                P[v, g.in_indices[e]] += 1.0 / outdeg[g.in_indices[e]]
        D = np.outer(np.ones(n), (outdeg == 0).astype(float)) / n
        A = np.eye(n) - 0.85 * (P + D)
        np.testing.assert_allclose(x, np.linalg.solve(A, np.full(n, 0.15 / n)), rtol=1e-12)
        _, G = pins.pagerank_dense(n, g.offsets, g.in_offsets, g.in_indices, 0.85, 0)
        np.testing.assert_allclose(x, pins.pagerank_stationary(G), rtol=1e-10)
        assert 0 < steps < 10000


def test_pagerank_fixpoint_stopping_rule():
    """Steps and distance: a loose tolerance stops earlier, and the result is
    within tol * d / (1 - d) of the tight fixed point (contraction in L1); the
    20-step vector is within 2 d^20 of it."""
    g = gen.rmat(12, seed=4, directed=True)
    xs, ns = oracle.pagerank_fixpoint_g(g, tol=1e-15)
    for tol in (1e-4, 1e-7, 1e-10):
        x, k = oracle.pagerank_fixpoint_g(g, tol=tol)
        assert k < ns
        assert np.abs(x - xs).sum() <= tol * 0.85 / 0.15 * 1.0001
    assert np.abs(oracle.pagerank_g(g) - xs).sum() <= 2 * 0.85 ** 20


# ------------------------------------------------- belief propagation ----

def _bp_graphs():
    return [gen.random_graph(9, 0.4, seed=1, weights=(1, 64)),
            gen.random_graph(12, 0.25, seed=2, weights=(1, 64)),
            gen.random_graph(10, 0.5, seed=3),                       # unweighted: theta = 1
            gen.from_edges(6, [(0, i) for i in range(1, 6)], [1, 17, 32, 33, 64]),
            gen.from_edges(5, [(0, 1), (2, 3)], [5, 60])]             # vertex 4 isolated


def test_bp_no_coupling_keeps_priors():
    """kappa = 0 makes every potential uniform (s = 1/2): every message is
    constant, so the beliefs stay the priors; zero iterations return them."""
    for i, g in enumerate(_bp_graphs()):
        pr = gen.bp_priors(g.n, seed=i).astype(np.float64)
        for it in (0, 1, 5):
            np.testing.assert_allclose(oracle.bp_g(g, pr, kappa=0.0, iters=it), pr, rtol=0, atol=1e-15)
        np.testing.assert_array_equal(oracle.bp_g(g, pr, kappa=0.5, iters=0), pr)


def test_bp_first_iteration_is_exact_on_stars():
    """One iteration from the priors equals, at every vertex, the exact
    marginal of the MRF restricted to its star, by enumeration of all joint
    states (Section 6: sum-product message passing)."""
    for i, g in enumerate(_bp_graphs()):
        pr = gen.bp_priors(g.n, seed=10 + i).astype(np.float64)
        for kappa in (0.3, 0.9):
            got = oracle.bp_g(g, pr, kappa=kappa, iters=1)
            ref = pins.bp_star_marginals(g.n, g.offsets, g.indices, g.weights, pr, kappa)
            np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-14)


def test_bp_uniform_cycle_closed_form():
    """A cycle with one prior and one edge weight keeps all beliefs equal and
    follows the scalar tanh recurrence (an identity of the message ratio, not
    the oracle's product of messages)."""
    n = 7
    for w, kappa, p0 in ((64, 0.9, 0.8), (1, 0.5, 0.3), (40, 0.7, 0.55)):
        g = gen.from_edges(n, [(i, (i + 1) % n) for i in range(n)], [w] * n)
        pr = np.full(n, p0)
        theta = ((w - 1) % 64 - 31.5) / 31.5
        c = kappa * theta / 2.0
        for it in (1, 2, 6, 20):
            got = oracle.bp_g(g, pr, kappa=kappa, iters=it)
            np.testing.assert_allclose(got, np.full(n, pins.bp_uniform_cycle(it, p0, c)), rtol=1e-12)


def test_bp_relabelling_and_components():
    """Renumbering the vertices renumbers the beliefs; a disjoint union gives
    each part the beliefs it has alone (no mixing of indices or operands)."""
    g = gen.random_graph(11, 0.35, seed=5, weights=(1, 64))
    pr = gen.bp_priors(g.n, seed=5).astype(np.float64)
    ref = oracle.bp_g(g, pr, kappa=0.8, iters=7)
    perm = np.random.default_rng(3).permutation(g.n)        # old -> new
    src = np.repeat(np.arange(g.n), np.diff(g.offsets))
    keep = src < g.indices
    gp = gen.from_edges(g.n, np.stack([perm[src[keep]], perm[g.indices[keep]]], 1), g.weights[keep])
    prp = np.empty(g.n)
    prp[perm] = pr
    np.testing.assert_allclose(oracle.bp_g(gp, prp, kappa=0.8, iters=7)[perm], ref, rtol=1e-13)
    h = gen.random_graph(6, 0.5, seed=8, weights=(1, 64))
    ph = gen.bp_priors(h.n, seed=8).astype(np.float64)
    srch = np.repeat(np.arange(h.n), np.diff(h.offsets))
    kh = srch < h.indices
    u = gen.from_edges(g.n + h.n, np.concatenate([np.stack([src[keep], g.indices[keep]], 1),
                                                  np.stack([srch[kh] + g.n, h.indices[kh] + g.n], 1)]),
                       np.concatenate([g.weights[keep], h.weights[kh]]))
    bu = oracle.bp_g(u, np.concatenate([pr, ph]), kappa=0.8, iters=7)
    np.testing.assert_allclose(bu[:g.n], ref, rtol=1e-13)
    np.testing.assert_allclose(bu[g.n:], oracle.bp_g(h, ph, kappa=0.8, iters=7), rtol=1e-13)


# ------------------------------------------------- planted mistakes fail ----

def test_pins_catch_planted_mistakes():
    """Mutated copies of the oracle's arithmetic, planted here on the CPU, each
    fail at least one pin used above."""
    # PageRank without the dangling term loses mass
    g0 = gen.random_graph(9, 0.3, seed=11, directed=True)
    src = np.repeat(np.arange(g0.n), np.diff(g0.offsets))
    keep = src != 0                        # vertex 0 gets no out-arcs: it dangles
    g = gen.from_edges(g0.n, np.stack([src[keep], g0.indices[keep]], 1), directed=True)
    outdeg = np.diff(g.offsets)
    assert (outdeg == 0).any()
    x = np.full(g.n, 1 / g.n)
    for _ in range(20):
        y = np.zeros(g.n)
        for v in range(g.n):
            for e in range(g.in_offsets[v], g.in_offsets[v + 1]):
                u = g.in_indices[e]
                y[v] += x[u] / outdeg[u]
        x = (1 - 0.85) / g.n + 0.85 * y
    xd, _ = pins.pagerank_dense(g.n, g.offsets, g.in_offsets, g.in_indices, 0.85, 20)
    assert not np.allclose(x, xd, rtol=1e-9)
    # transposed operand (out-arcs used as in-arcs) fails the dense check
    xt, _ = pins.pagerank_dense(g.n, g.offsets, g.offsets, g.indices, 0.85, 20)
    assert not np.allclose(xt, xd, rtol=1e-9)
    # a core number off by one fails the certificate
    gu = gen.random_graph(12, 0.4, seed=2)
    c = oracle.kcore_g(gu).copy()
    c[np.argmax(c)] += 1
    with pytest.raises(AssertionError):
        pins.kcore_certificate(gu.n, gu.offsets, gu.indices, c)
    # k-core membership with "degree <= k" as the deletion rule fails the
    # subset enumeration; component labels taken as the largest id fail the
    # closure
    g5 = _g(5, [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4)])
    deg = np.diff(g5.offsets)
    member = np.ones(5, dtype=np.int64)
    changed = True
    while changed:
        changed = False
        for v in range(5):
            if member[v] and sum(member[u] for u in g5.indices[g5.offsets[v]:g5.offsets[v + 1]]) <= 2:
                member[v] = 0
                changed = True
    assert not np.array_equal(member, pins.brute_kcore_member(5, g5.offsets, g5.indices, 2))
    lab = pins.closure_min_label(5, g5.offsets, g5.indices)
    assert not np.array_equal(np.full(5, 4), lab)
    # a BFS depth off by one fails the certificate
    d = oracle.bfs_g(gu, 0).copy()
    d[np.argmax(d)] += 1
    with pytest.raises(AssertionError):
        pins.bfs_certificate(gu.n, gu.offsets, gu.indices, 0, d)
    # belief propagation: dropping the prior, flipping the coupling's sign or
    # scaling by the receiving vertex's degree only each fail the star check
    gb = gen.from_edges(6, [(0, 1), (0, 2), (0, 3), (3, 4), (4, 5), (1, 2)], [3, 50, 64, 20, 9, 41])
    pb = gen.bp_priors(gb.n, seed=21).astype(np.float64)
    star = pins.bp_star_marginals(gb.n, gb.offsets, gb.indices, gb.weights, pb, 0.9)
    deg = np.diff(gb.offsets)

    def one_iteration(no_prior=False, flip=False, own_degree=False):
        out = np.empty(gb.n)
        for v in range(gb.n):
            l1 = 0.0 if no_prior else np.log(pb[v])
            l0 = 0.0 if no_prior else np.log(1 - pb[v])
            for e in range(gb.offsets[v], gb.offsets[v + 1]):
                u = gb.indices[e]
                th = ((int(gb.weights[e]) - 1) % 64 - 31.5) / 31.5 * (-1 if flip else 1)
                s = 0.5 * (1 + 0.9 * th / (deg[v] if own_degree else max(deg[u], deg[v])))
                l1 += np.log(s * pb[u] + (1 - s) * (1 - pb[u]))
                l0 += np.log((1 - s) * pb[u] + s * (1 - pb[u]))
            out[v] = 1 / (1 + np.exp(l0 - l1))
        return out

    np.testing.assert_allclose(one_iteration(), star, rtol=1e-12)
    for mutant in (dict(no_prior=True), dict(flip=True), dict(own_degree=True)):
        assert not np.allclose(one_iteration(**mutant), star, rtol=1e-9), mutant
