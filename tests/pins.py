"""Independent checks used to pin the oracle (and, on the GPU, the engine).

Nothing here calls the oracle: brute force, closed forms and certificates
written straight from the definitions.
"""
from __future__ import annotations

import itertools

import numpy as np

INF = 0xFFFFFFFF


def dense_adj(n, offsets, indices, weights=None):
    """Dense weight matrix (inf where no arc); unit weights when None."""
    W = np.full((n, n), np.inf)
    for v in range(n):
        for e in range(offsets[v], offsets[v + 1]):
            w = 1.0 if weights is None else float(weights[e])
            W[v, indices[e]] = min(W[v, indices[e]], w)
    np.fill_diagonal(W, 0.0)
    return W


def floyd_warshall(W):
    D = W.copy()
    n = D.shape[0]
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    return D


def fw_depth(n, offsets, indices, src):
    D = floyd_warshall(dense_adj(n, offsets, indices))[src]
    return np.where(np.isinf(D), -1, D).astype(np.int64)


def fw_dist(n, offsets, indices, weights, src):
    D = floyd_warshall(dense_adj(n, offsets, indices, weights))[src]
    return np.where(np.isinf(D), INF, D).astype(np.uint64)


def brute_core(n, offsets, indices, in_offsets=None, in_indices=None):
    """core(v) = max k such that some vertex set S containing v induces a
    subgraph whose every vertex has degree >= k (degree = arcs incident within
    S, in- plus out-arcs for a digraph).  Enumerates all 2^n subsets."""
    A = np.zeros((n, n), dtype=np.int64)
    for v in range(n):
        for e in range(offsets[v], offsets[v + 1]):
            A[v, indices[e]] += 1
    if in_offsets is not None:
        # every arc u->v counts once at each end: total degree = row + column
        Ad = A + A.T
    else:
        Ad = A
    core = np.zeros(n, dtype=np.int64)
    for mask in range(1, 1 << n):
        S = np.array([(mask >> i) & 1 for i in range(n)], dtype=bool)
        sub = Ad[np.ix_(S, S)]
        mindeg = sub.sum(axis=1).min()
        core[S] = np.maximum(core[S], mindeg)
    return core


def bfs_certificate(n, offsets, indices, src, depth):
    """Complete characterisation of BFS depths on an undirected graph."""
    depth = np.asarray(depth, dtype=np.int64)
    assert depth[src] == 0
    src_of = np.repeat(np.arange(n), np.diff(offsets))
    du, dv = depth[src_of], depth[indices]
    reached_u, reached_v = du >= 0, dv >= 0
    # no arc joins a reached and an unreached vertex
    assert not np.any(reached_u != reached_v), "edge between reached and unreached vertex"
    both = reached_u & reached_v
    assert np.all(np.abs(du[both] - dv[both]) <= 1), "adjacent depths differ by more than 1"
    # every reached vertex other than the source has a parent one level up
    has_parent = np.zeros(n, dtype=bool)
    par = both & (du == dv - 1)
    has_parent[indices[par]] = True
    need = (depth > 0)
    assert np.all(has_parent[need]), "reached vertex without a parent"
    return True


def sssp_certificate(n, offsets, indices, weights, src, dist):
    dist = np.asarray(dist, dtype=np.uint64)
    assert dist[src] == 0
    src_of = np.repeat(np.arange(n), np.diff(offsets))
    du, dv = dist[src_of], dist[indices]
    w = np.asarray(weights, dtype=np.uint64)
    fin_u = du != INF
    # triangle inequality on every arc out of a reached vertex
    assert np.all(dv[fin_u] <= du[fin_u] + w[fin_u]), "arc violates dist[v] <= dist[u] + w"
    # the unreached set is closed
    assert np.all(dv[fin_u] != INF)
    # every reached vertex but the source has a tight in-arc
    tight = fin_u & (dv == du + w)
    has = np.zeros(n, dtype=bool)
    has[indices[tight]] = True
    need = (dist != INF) & (np.arange(n) != src)
    assert np.all(has[need]), "reached vertex without a tight arc"
    return True


def kcore_certificate(n, offsets, indices, core, in_offsets=None, in_indices=None):
    """Necessary conditions: (i) every v has >= core(v) incident arcs to
    vertices with core >= core(v); (ii) core(v) <= degree(v); (iii) the
    h-index fixpoint core(v) = H({core(u)}) over incident arcs."""
    core = np.asarray(core, dtype=np.int64)
    nbr_lists = []
    for v in range(n):
        nb = list(indices[offsets[v]:offsets[v + 1]])
        if in_offsets is not None:
            nb += list(in_indices[in_offsets[v]:in_offsets[v + 1]])
        nbr_lists.append(np.asarray(nb, dtype=np.int64))
    for v in range(n):
        cu = core[nbr_lists[v]] if len(nbr_lists[v]) else np.zeros(0, dtype=np.int64)
        assert core[v] <= len(cu)
        assert (cu >= core[v]).sum() >= core[v]
        s = np.sort(cu)[::-1]
        h = 0
        for i, c in enumerate(s):
            if c >= i + 1:
                h = i + 1
        assert h == core[v], (v, h, core[v])
    return True


def kcore_certificate_fast(n, offsets, indices, core, in_offsets=None, in_indices=None):
    """Vectorised (i) and (ii) for large graphs."""
    core = np.asarray(core, dtype=np.int64)
    def count(off, idx):
        src_of = np.repeat(np.arange(n), np.diff(off))
        ok = core[idx] >= core[src_of]
        return np.bincount(src_of[ok], minlength=n), np.diff(off)
    c1, d1 = count(offsets, indices)
    if in_offsets is not None:
        c2, d2 = count(in_offsets, in_indices)
        c1, d1 = c1 + c2, d1 + d2
    assert np.all(core <= d1)
    assert np.all(c1 >= core)
    return True


def pagerank_dense(n, offsets, in_offsets, in_indices, d, iters):
    """PageRank as repeated multiplication by the dense Google matrix
    G = d * (P + dangling / n) + (1 - d) / n, P[v, u] = 1/outdeg(u) per arc u->v."""
    P = np.zeros((n, n))
    outdeg = np.diff(offsets)
    for v in range(n):
        for e in range(in_offsets[v], in_offsets[v + 1]):
            u = in_indices[e]
            P[v, u] += 1.0 / outdeg[u]
    dang = (outdeg == 0).astype(float)
    G = d * (P + np.outer(np.ones(n), dang) / n) + (1 - d) / n
    x = np.full(n, 1.0 / n)
    for _ in range(iters):
        x = G @ x
    return x, G


def pagerank_stationary(G):
    """Principal eigenvector of the column-stochastic Google matrix, via numpy.linalg.eig."""
    vals, vecs = np.linalg.eig(G)
    k = int(np.argmin(np.abs(vals - 1.0)))
    v = np.real(vecs[:, k])
    return v / v.sum()


def all_graphs(n):
    """Every labelled simple undirected graph on n vertices, as edge lists."""
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        yield [pairs[i] for i in range(len(pairs)) if (mask >> i) & 1]


def brute_kcore_member(n, offsets, indices, k, in_offsets=None, in_indices=None):
    """Membership in the k-core straight from its definition: the union of
    every vertex set S whose induced subgraph gives each vertex of S at least
    k incident arcs inside S (in- plus out-arcs for a digraph).  Enumerates
    all 2^n subsets."""
    A = np.zeros((n, n), dtype=np.int64)
    for v in range(n):
        for e in range(offsets[v], offsets[v + 1]):
            A[v, indices[e]] += 1
    Ad = A + A.T if in_offsets is not None else A
    member = np.zeros(n, dtype=np.int64)
    for mask in range(1, 1 << n):
        S = np.array([(mask >> i) & 1 for i in range(n)], dtype=bool)
        if Ad[np.ix_(S, S)].sum(axis=1).min() >= k:
            member[S] = 1
    return member


def closure_min_label(n, offsets, indices):
    """Smallest vertex reachable from each vertex when arcs are taken in
    both directions: Floyd-Warshall transitive closure of the symmetrised
    adjacency, then the first reachable id per row."""
    R = np.eye(n, dtype=bool)
    for v in range(n):
        for e in range(offsets[v], offsets[v + 1]):
            R[v, indices[e]] = R[indices[e], v] = True
    for k in range(n):
        R = R | (R[:, k:k + 1] & R[k:k + 1, :])
    return np.array([int(np.nonzero(R[v])[0][0]) for v in range(n)], dtype=np.int64)


# ------------------------------------------------- belief propagation ----

def bp_potential(w_e, du, dv, kappa):
    """Agreement probability s of the pairwise potential of edge {u, v}
    (psi(x, y) = s if x == y else 1 - s): the binary MRF the belief
    propagation workloads define, coupling sign and strength from the arc
    weight (weights 1..64 span -1..1), scaled by the larger endpoint degree."""
    theta = 1.0 if w_e is None else ((int(w_e) - 1) % 64 - 31.5) / 31.5
    return 0.5 * (1.0 + kappa * theta / max(du, dv))


def bp_star_marginals(n, offsets, indices, weights, prior, kappa):
    """For every vertex v, the exact marginal P(x_v = 1) of the MRF restricted
    to v's star (v, its neighbours, the edges {v, u}), with every vertex's
    prior as its unary potential, by enumerating all 2^(deg + 1) joint
    states.  One synchronous sum-product iteration from the priors must give
    exactly these values: a neighbour's message is then built from its prior
    alone, as in the star."""
    deg = np.diff(np.asarray(offsets, dtype=np.int64))
    out = np.empty(n)
    for v in range(n):
        nb = [(int(indices[e]), None if weights is None else int(weights[e]))
              for e in range(offsets[v], offsets[v + 1])]
        z = np.zeros(2)
        for xs in itertools.product((0, 1), repeat=len(nb) + 1):
            xv = xs[0]
            p = prior[v] if xv == 1 else 1.0 - prior[v]
            for (u, we), xu in zip(nb, xs[1:]):
                p *= prior[u] if xu == 1 else 1.0 - prior[u]
                s = bp_potential(we, deg[u], deg[v], kappa)
                p *= s if xu == xv else 1.0 - s
            z[xv] += p
        out[v] = z[1] / z.sum()
    return out


def bp_uniform_cycle(n_iter, p0, c):
    """Belief of every vertex of a cycle whose vertices share the prior p0 and
    whose edges share the potential (1 + c) / 2 (by symmetry all beliefs stay
    equal): in the q = 2b - 1 coordinates one sum-product iteration is
    q' = tanh(atanh(q0) + 2 atanh(c q)) (the message ratio of an edge is
    (1 + c q) / (1 - c q) = exp(2 atanh(c q))), q0 = 2 p0 - 1."""
    q0 = 2.0 * p0 - 1.0
    q = q0
    for _ in range(n_iter):
        q = np.tanh(np.arctanh(q0) + 2.0 * np.arctanh(c * q))
    return 0.5 * (1.0 + q)
