/*
 * CPU oracle for the ACC graph engine.  TEST INFRASTRUCTURE ONLY: nothing in
 * the product path may call, link or load this file; it exists so that the
 * tests, the smoke check and the CPU-baseline leg of the benchmark can compare
 * the GPU results with a plain, serial, obviously correct computation.
 *
 * It shares no code with the HIP engine.  Every function is the textbook
 * definition of what the paper's iterative method converges to:
 *
 *   BFS      Section 6 ("traverses a graph level by level"): the depth of every
 *            vertex = hop distance from the source, by a FIFO queue.
 *   SSSP     Section 2.1 / 3.3 (positive weights, distance array, iterate
 *            until no vertex is updated): shortest path lengths, by
 *            Dijkstra's algorithm with a binary heap (lazy deletion) in 64-bit
 *            arithmetic; cross-checked by a worklist Bellman-Ford and by the
 *            synchronous round form that the paper's worked example follows.
 *   k-core   Section 6 (delete vertices of degree < k until every remaining
 *            vertex has degree >= k), extended to the full decomposition:
 *            core(v) = largest k with v in the k-core.  Batagelj-Zaversnik
 *            bucket algorithm ("An O(m) algorithm for cores decomposition of
 *            networks", 2003) and naive level-by-level peeling.
 *            Fixed-k membership, the paper's own k-core (Section 6, k = 16;
 *            k = 32 in its run-time comparison): repeatedly delete every
 *            vertex whose degree is below k; the survivors form the k-core.
 *   WCC      Section 3.2 (connected components with a voting / minimum
 *            combine): the label of a vertex is the smallest vertex id in
 *            its weakly connected component (arcs taken without direction),
 *            by union-find.
 *   PageRank Section 6 (pull, sum of in-neighbour contributions): 20
 *            synchronous iterations in fp64, x0 = 1/n,
 *            x'(v) = (1-d)/n + d * (sum_{u->v} x(u)/outdeg(u) + D/n),
 *            D = sum of x over vertices without out-arcs.
 *            The same recurrence iterated to its fixed point (Section 6:
 *            "till all vertices have stable rank values"): until one step
 *            changes the vector by at most tol in L1.
 *   BP       Section 6 ("Belief propagation": sum-product message passing on
 *            a Markov random field, the vertex's probability as its state)
 *            and Section 3.2 (every vertex active, updates summed): a binary
 *            pairwise MRF, synchronous iterations in fp64 of
 *              b'(v, x) ~ phi_v(x) * prod_{u in N(v)} m_{u->v}(x),
 *              m_{u->v}(x) = sum_y psi_uv(y, x) * b(u, y),
 *            starting from b = phi; products taken as sums of logarithms.
 *
 * Graph layout: CSR int32 offsets[n+1] / indices[m] (out-arcs); directed
 * graphs also pass the CSC (in-arcs).  Undirected graphs store both arcs.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SXO_INF 0xFFFFFFFFu

/* ---------------------------------------------------------------- BFS --- */
int sxo_bfs(int32_t n, const int32_t *off, const int32_t *idx, int32_t src, int32_t *depth) {
    if (n < 0 || (n > 0 && (src < 0 || src >= n))) return -1;
    for (int32_t v = 0; v < n; ++v) depth[v] = -1;
    if (n == 0) return 0;
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!queue) return -2;
    int64_t head = 0, tail = 0;
    depth[src] = 0;
    queue[tail++] = src;
    while (head < tail) {
        int32_t v = queue[head++];
        for (int64_t e = off[v]; e < off[v + 1]; ++e) {
            int32_t u = idx[e];
            if (depth[u] < 0) { depth[u] = depth[v] + 1; queue[tail++] = u; }
        }
    }
    free(queue);
    return 0;
}

/* --------------------------------------------------------------- SSSP --- */
typedef struct { uint64_t d; int32_t v; } heap_item;

static void heap_push(heap_item *h, int64_t *len, heap_item it) {
    int64_t i = (*len)++;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p].d <= it.d) break;
        h[i] = h[p]; i = p;
    }
    h[i] = it;
}
static heap_item heap_pop(heap_item *h, int64_t *len) {
    heap_item top = h[0];
    heap_item last = h[--(*len)];
    int64_t i = 0, n = *len;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        uint64_t sd = last.d;
        if (l < n && h[l].d < sd) { s = l; sd = h[l].d; }
        if (r < n && h[r].d < sd) { s = r; }
        if (s == i) break;
        h[i] = h[s]; i = s;
    }
    if (n > 0) h[i] = last;
    return top;
}

/* Dijkstra.  dist[v] = 0xFFFFFFFF when unreachable.  Returns -3 if a finite
 * distance does not fit below 0xFFFFFFFF. */
int sxo_dijkstra(int32_t n, const int32_t *off, const int32_t *idx, const uint32_t *w,
                 int32_t src, uint32_t *dist) {
    if (n < 0 || (n > 0 && (src < 0 || src >= n))) return -1;
    for (int32_t v = 0; v < n; ++v) dist[v] = SXO_INF;
    if (n == 0) return 0;
    int64_t m = off[n];
    uint64_t *d = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    char *done = (char *)calloc((size_t)n, 1);
    heap_item *h = (heap_item *)malloc(sizeof(heap_item) * (size_t)(m + 1));
    if (!d || !done || !h) { free(d); free(done); free(h); return -2; }
    for (int32_t v = 0; v < n; ++v) d[v] = UINT64_MAX;
    int64_t len = 0;
    d[src] = 0;
    heap_item s0 = {0, src};
    heap_push(h, &len, s0);
    int rc = 0;
    while (len > 0) {
        heap_item it = heap_pop(h, &len);
        int32_t v = it.v;
        if (done[v]) continue;
        done[v] = 1;
        for (int64_t e = off[v]; e < off[v + 1]; ++e) {
            int32_t u = idx[e];
            uint64_t nd = d[v] + (uint64_t)w[e];
            if (nd < d[u]) { d[u] = nd; heap_item ni = {nd, u}; heap_push(h, &len, ni); }
        }
    }
    for (int32_t v = 0; v < n; ++v) {
        if (d[v] == UINT64_MAX) continue;
        if (d[v] >= SXO_INF) { rc = -3; continue; }
        dist[v] = (uint32_t)d[v];
    }
    free(d); free(done); free(h);
    return rc;
}

/* Bellman-Ford, worklist form: only vertices whose distance changed are
 * relaxed again (FIFO worklist, each vertex queued at most once at a time). */
int sxo_bellman_ford(int32_t n, const int32_t *off, const int32_t *idx, const uint32_t *w,
                     int32_t src, uint32_t *dist) {
    if (n < 0 || (n > 0 && (src < 0 || src >= n))) return -1;
    for (int32_t v = 0; v < n; ++v) dist[v] = SXO_INF;
    if (n == 0) return 0;
    uint64_t *d = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    char *inq = (char *)calloc((size_t)n, 1);
    if (!d || !q || !inq) { free(d); free(q); free(inq); return -2; }
    for (int32_t v = 0; v < n; ++v) d[v] = UINT64_MAX;
    int64_t head = 0, cnt = 0;  /* circular queue */
    d[src] = 0; q[0] = src; cnt = 1; inq[src] = 1;
    while (cnt > 0) {
        int32_t v = q[head]; head = (head + 1) % n; --cnt; inq[v] = 0;
        for (int64_t e = off[v]; e < off[v + 1]; ++e) {
            int32_t u = idx[e];
            uint64_t nd = d[v] + (uint64_t)w[e];
            if (nd < d[u]) {
                d[u] = nd;
                if (!inq[u]) { q[(head + cnt) % n] = u; ++cnt; inq[u] = 1; }
            }
        }
    }
    int rc = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (d[v] == UINT64_MAX) continue;
        if (d[v] >= SXO_INF) { rc = -3; continue; }
        dist[v] = (uint32_t)d[v];
    }
    free(d); free(q); free(inq);
    return rc;
}

/* Synchronous frontier rounds, the form of the worked example of Section 2.1:
 * round r relaxes every arc out of the vertices whose distance changed in
 * round r-1 (round 1: the source), using the distances as they stood at the
 * start of the round.  update_round[v] = last round that lowered dist[v]
 * (0 for the source, -1 never).  Returns the number of rounds that changed
 * something, or a negative error. */
int sxo_sssp_rounds(int32_t n, const int32_t *off, const int32_t *idx, const uint32_t *w,
                    int32_t src, uint32_t *dist, int32_t *update_round, int32_t max_rounds) {
    if (n < 0 || (n > 0 && (src < 0 || src >= n))) return -1;
    for (int32_t v = 0; v < n; ++v) { dist[v] = SXO_INF; update_round[v] = -1; }
    if (n == 0) return 0;
    uint64_t *d = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    uint64_t *nd = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    char *act = (char *)calloc((size_t)n, 1);
    if (!d || !nd || !act) { free(d); free(nd); free(act); return -2; }
    for (int32_t v = 0; v < n; ++v) d[v] = UINT64_MAX;
    d[src] = 0; act[src] = 1; update_round[src] = 0;
    int32_t r = 0;
    for (;;) {
        if (max_rounds >= 0 && r >= max_rounds) break;
        memcpy(nd, d, sizeof(uint64_t) * (size_t)n);
        for (int32_t v = 0; v < n; ++v) {
            if (!act[v]) continue;
            for (int64_t e = off[v]; e < off[v + 1]; ++e) {
                uint64_t c = d[v] + (uint64_t)w[e];
                if (c < nd[idx[e]]) nd[idx[e]] = c;
            }
        }
        int changed = 0;
        for (int32_t v = 0; v < n; ++v) {
            act[v] = nd[v] < d[v];
            if (act[v]) { changed = 1; update_round[v] = r + 1; }
        }
        memcpy(d, nd, sizeof(uint64_t) * (size_t)n);
        if (!changed) break;
        ++r;
    }
    int rc = r;
    for (int32_t v = 0; v < n; ++v) {
        if (d[v] == UINT64_MAX) continue;
        if (d[v] >= SXO_INF) { rc = -3; continue; }
        dist[v] = (uint32_t)d[v];
    }
    free(d); free(nd); free(act);
    return rc;
}

/* ------------------------------------------------------------- k-core --- */
/* The degree of v counts every arc incident to v: out-arcs from the CSR and,
 * for a directed graph (in_off != NULL), in-arcs from the CSC.  Removing v
 * lowers the degree of the other endpoint of each of its arcs by one. */

static int32_t total_degree(const int32_t *off, const int32_t *in_off, int32_t v) {
    int32_t d = off[v + 1] - off[v];
    if (in_off) d += in_off[v + 1] - in_off[v];
    return d;
}

/* Batagelj-Zaversnik: vertices kept in an array sorted by current degree with
 * bucket starts; repeatedly take the vertex of least degree, fix its core,
 * and move each neighbour of larger degree one bucket down. */
int sxo_kcore_bz(int32_t n, const int32_t *off, const int32_t *idx,
                 const int32_t *in_off, const int32_t *in_idx, int32_t *core) {
    if (n < 0) return -1;
    if (n == 0) return 0;
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *vert = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t md = 0;
    if (!deg || !vert || !pos) { free(deg); free(vert); free(pos); return -2; }
    for (int32_t v = 0; v < n; ++v) { deg[v] = total_degree(off, in_off, v); if (deg[v] > md) md = deg[v]; }
    int32_t *bin = (int32_t *)calloc((size_t)md + 1, sizeof(int32_t));
    if (!bin) { free(deg); free(vert); free(pos); return -2; }
    for (int32_t v = 0; v < n; ++v) bin[deg[v]]++;
    int32_t start = 0;
    for (int32_t d = 0; d <= md; ++d) { int32_t c = bin[d]; bin[d] = start; start += c; }
    for (int32_t v = 0; v < n; ++v) { pos[v] = bin[deg[v]]; vert[pos[v]] = v; bin[deg[v]]++; }
    for (int32_t d = md; d >= 1; --d) bin[d] = bin[d - 1];
    bin[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t v = vert[i];
        for (int pass = 0; pass < 2; ++pass) {
            const int32_t *o = pass ? in_off : off, *x = pass ? in_idx : idx;
            if (!o) continue;
            for (int64_t e = o[v]; e < o[v + 1]; ++e) {
                int32_t u = x[e];
                if (deg[u] > deg[v]) {
                    int32_t du = deg[u], pu = pos[u], pw = bin[du], w = vert[pw];
                    if (u != w) { pos[u] = pw; vert[pu] = w; pos[w] = pu; vert[pw] = u; }
                    bin[du]++;
                    deg[u]--;
                }
            }
        }
    }
    for (int32_t v = 0; v < n; ++v) core[v] = deg[v];
    free(deg); free(vert); free(pos); free(bin);
    return 0;
}

/* Naive peeling, level by level: at level k remove, until none is left, every
 * remaining vertex whose current degree is <= k; those get core number k. */
int sxo_kcore_peel(int32_t n, const int32_t *off, const int32_t *idx,
                   const int32_t *in_off, const int32_t *in_idx, int32_t *core) {
    if (n < 0) return -1;
    if (n == 0) return 0;
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    char *alive = (char *)malloc((size_t)n);
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!deg || !alive || !cur) { free(deg); free(alive); free(cur); return -2; }
    for (int32_t v = 0; v < n; ++v) { deg[v] = total_degree(off, in_off, v); alive[v] = 1; core[v] = -1; }
    int64_t remaining = n;
    for (int32_t k = 0; remaining > 0; ++k) {
        for (;;) {
            int64_t nc = 0;
            for (int32_t v = 0; v < n; ++v)
                if (alive[v] && deg[v] <= k) cur[nc++] = v;
            if (nc == 0) break;
            for (int64_t i = 0; i < nc; ++i) { alive[cur[i]] = 0; core[cur[i]] = k; }
            remaining -= nc;
            for (int64_t i = 0; i < nc; ++i) {
                int32_t v = cur[i];
                for (int pass = 0; pass < 2; ++pass) {
                    const int32_t *o = pass ? in_off : off, *x = pass ? in_idx : idx;
                    if (!o) continue;
                    for (int64_t e = o[v]; e < o[v + 1]; ++e)
                        if (alive[x[e]]) deg[x[e]]--;
                }
            }
        }
    }
    free(deg); free(alive); free(cur);
    return 0;
}

/* Membership in the k-core for one k (Section 6): a FIFO queue of vertices
 * whose degree fell below k; each is deleted once and lowers the degree of
 * every neighbour still present.  member[v] = 1 for the survivors, else 0. */
int sxo_kcore_member(int32_t n, const int32_t *off, const int32_t *idx,
                     const int32_t *in_off, const int32_t *in_idx, int32_t k, int32_t *member) {
    if (n < 0 || k < 0) return -1;
    if (n == 0) return 0;
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!deg || !queue) { free(deg); free(queue); return -2; }
    int64_t head = 0, tail = 0;
    for (int32_t v = 0; v < n; ++v) {
        deg[v] = total_degree(off, in_off, v);
        member[v] = 1;
        if (deg[v] < k) { member[v] = 0; queue[tail++] = v; }
    }
    while (head < tail) {
        int32_t v = queue[head++];
        for (int pass = 0; pass < 2; ++pass) {
            const int32_t *o = pass ? in_off : off, *x = pass ? in_idx : idx;
            if (!o) continue;
            for (int64_t e = o[v]; e < o[v + 1]; ++e) {
                int32_t u = x[e];
                if (!member[u]) continue;
                if (--deg[u] < k) { member[u] = 0; queue[tail++] = u; }
            }
        }
    }
    free(deg); free(queue);
    return 0;
}

/* ---------------------------------------------------------------- WCC --- */
/* Union-find with path halving over every arc (CSR, and the CSC of a
 * directed graph, which holds the same arcs reversed); the label of a
 * component is its smallest vertex id (the root is always the smaller id). */
static int32_t uf_find(int32_t *parent, int32_t v) {
    while (parent[v] != v) { parent[v] = parent[parent[v]]; v = parent[v]; }
    return v;
}

int sxo_wcc(int32_t n, const int32_t *off, const int32_t *idx, int32_t *label) {
    if (n < 0) return -1;
    for (int32_t v = 0; v < n; ++v) label[v] = v;
    for (int32_t v = 0; v < n; ++v)
        for (int64_t e = off[v]; e < off[v + 1]; ++e) {
            int32_t a = uf_find(label, v), b = uf_find(label, idx[e]);
            if (a < b) label[b] = a;
            else if (b < a) label[a] = b;
        }
    for (int32_t v = 0; v < n; ++v) label[v] = uf_find(label, v);
    return 0;
}

/* ----------------------------------------------------------- PageRank --- */
/* out_deg from the CSR; in-arcs from the CSC (for an undirected graph pass the
 * CSR twice). */
int sxo_pagerank(int32_t n, const int32_t *off, const int32_t *in_off, const int32_t *in_idx,
                 double d, int32_t iters, double *x_out) {
    if (n < 0 || iters < 0) return -1;
    if (n == 0) return 0;
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    if (!x || !y) { free(x); free(y); return -2; }
    for (int32_t v = 0; v < n; ++v) x[v] = 1.0 / (double)n;
    for (int32_t t = 0; t < iters; ++t) {
        double dangling = 0.0;
        for (int32_t u = 0; u < n; ++u)
            if (off[u + 1] == off[u]) dangling += x[u];
        for (int32_t v = 0; v < n; ++v) {
            double s = 0.0;
            for (int64_t e = in_off[v]; e < in_off[v + 1]; ++e) {
                int32_t u = in_idx[e];
                s += x[u] / (double)(off[u + 1] - off[u]);
            }
            y[v] = (1.0 - d) / (double)n + d * (s + dangling / (double)n);
        }
        double *t2 = x; x = y; y = t2;
    }
    memcpy(x_out, x, sizeof(double) * (size_t)n);
    free(x); free(y);
    return 0;
}

/* PageRank to its fixed point: the recurrence above, iterated until the L1
 * norm of one step's change is at most tol (or max_iters steps).  The map is a
 * contraction with factor d in L1, so the result lies within tol * d / (1 - d)
 * of the fixed point.  Returns the number of steps taken (negative on bad
 * input). */
int sxo_pagerank_fixpoint(int32_t n, const int32_t *off, const int32_t *in_off, const int32_t *in_idx,
                          double d, double tol, int32_t max_iters, double *x_out) {
    if (n < 0 || max_iters < 0 || !(tol >= 0.0)) return -1;
    if (n == 0) return 0;
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    if (!x || !y) { free(x); free(y); return -2; }
    for (int32_t v = 0; v < n; ++v) x[v] = 1.0 / (double)n;
    int32_t t = 0;
    for (; t < max_iters; ++t) {
        double dangling = 0.0;
        for (int32_t u = 0; u < n; ++u)
            if (off[u + 1] == off[u]) dangling += x[u];
        double change = 0.0;
        for (int32_t v = 0; v < n; ++v) {
            double s = 0.0;
            for (int64_t e = in_off[v]; e < in_off[v + 1]; ++e) {
                int32_t u = in_idx[e];
                s += x[u] / (double)(off[u + 1] - off[u]);
            }
            y[v] = (1.0 - d) / (double)n + d * (s + dangling / (double)n);
            change += fabs(y[v] - x[v]);
        }
        double *t2 = x; x = y; y = t2;
        if (change <= tol) { ++t; break; }
    }
    memcpy(x_out, x, sizeof(double) * (size_t)n);
    free(x); free(y);
    return t;
}

/* ---------------------------------------------------- belief propagation --- */
/* Binary pairwise MRF over an undirected graph (both arcs stored).  Vertex v
 * has the prior phi_v(1) = prior[v], phi_v(0) = 1 - prior[v].  The edge
 * {u, v} carries the potential psi_uv(x, y) = s_uv when x == y and 1 - s_uv
 * otherwise, with
 *   s_uv     = (1 + kappa * theta_uv / max(deg u, deg v)) / 2,
 *   theta_uv = (((w_uv - 1) mod 64) - 31.5) / 31.5   (1 when w is NULL),
 * the coupling sign and strength taken from the arc weight (weights in
 * [1, 64] span [-1, 1]).  One iteration: every vertex's belief is its prior
 * times the product over its neighbours u of the message
 *   m_{u->v}(x) = sum_y psi_uv(y, x) b(u, y),
 * normalised to sum to 1 (Section 6: sum-product message passing with the
 * vertex probability as the metadata; Section 3.2: all vertices active, the
 * per-neighbour terms summed -- here the logarithms of the messages).
 * belief[v] = b(v, 1) after `iters` iterations (b = phi before the first). */
int sxo_bp(int32_t n, const int32_t *off, const int32_t *idx, const uint32_t *w, const double *prior,
           double kappa, int32_t iters, double *belief) {
    if (n < 0 || iters < 0) return -1;
    if (n == 0) return 0;
    double *b = (double *)malloc(sizeof(double) * (size_t)n);
    double *nb = (double *)malloc(sizeof(double) * (size_t)n);
    if (!b || !nb) { free(b); free(nb); return -2; }
    for (int32_t v = 0; v < n; ++v) {
        if (!(prior[v] > 0.0 && prior[v] < 1.0)) { free(b); free(nb); return -3; }
        b[v] = prior[v];
    }
    for (int32_t t = 0; t < iters; ++t) {
        for (int32_t v = 0; v < n; ++v) {
            double l1 = log(prior[v]), l0 = log(1.0 - prior[v]);
            const int64_t dv = off[v + 1] - off[v];
            for (int64_t e = off[v]; e < off[v + 1]; ++e) {
                const int32_t u = idx[e];
                const int64_t du = off[u + 1] - off[u];
                const double theta = w ? ((double)((w[e] - 1u) % 64u) - 31.5) / 31.5 : 1.0;
                const double s = 0.5 * (1.0 + kappa * theta / (double)(du > dv ? du : dv));
                const double m1 = s * b[u] + (1.0 - s) * (1.0 - b[u]);
                const double m0 = (1.0 - s) * b[u] + s * (1.0 - b[u]);
                l1 += log(m1);
                l0 += log(m0);
            }
            /* normalise: b(v, 1) = e^l1 / (e^l0 + e^l1) */
            nb[v] = 1.0 / (1.0 + exp(l0 - l1));
        }
        double *t2 = b; b = nb; nb = t2;
    }
    memcpy(belief, b, sizeof(double) * (size_t)n);
    free(b); free(nb);
    return 0;
}
