/*
 * Seeded synthetic graph inputs: R-MAT (Chakrabarti et al., the generator
 * family the paper evaluates on, Section 6 "Graph Benchmarks"), 2D grids with
 * random edge deletion (stand-ins for the high-diameter road graphs of the
 * paper's dataset table) and per-edge random weights ("a random generator ...
 * one weight for each edge", Section 6).
 *
 * This module builds inputs only.  It contains none of the graph algorithms:
 * both the CPU oracle and the HIP engine consume what it produces.
 *
 * Randomness is counter based: the i-th draw of stream `seed` is the i-th
 * output of SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014), i.e. mix(seed + (i + 1) * golden), so any
 * draw can be computed independently of all others, in any order and in
 * parallel, and the output is identical for every thread count.
 *
 * Output layout (CSR): int32 offsets[n+1], int32 indices[m] with every row
 * sorted ascending, duplicates and self loops removed.  Undirected graphs store
 * both arcs of every edge, so the CSR is symmetric.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
/* i-th output of the SplitMix64 sequence seeded with `seed` */
static inline uint64_t sm64_at(uint64_t seed, uint64_t i) {
    return sm64_mix(seed + (i + 1) * GOLDEN);
}

uint64_t sxg_splitmix64_at(uint64_t seed, uint64_t i) { return sm64_at(seed, i); }

typedef struct {
    int32_t n;
    int64_t m;
    int32_t *offsets;   /* [n+1] */
    int32_t *indices;   /* [m]   */
} sxg_csr;

void sxg_free(sxg_csr *g) {
    if (!g) return;
    free(g->offsets); free(g->indices);
    g->offsets = NULL; g->indices = NULL; g->n = 0; g->m = 0;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}
static void sort_row(int32_t *p, int64_t len) {
    if (len < 24) {
        for (int64_t i = 1; i < len; ++i) {
            int32_t v = p[i]; int64_t j = i - 1;
            while (j >= 0 && p[j] > v) { p[j + 1] = p[j]; --j; }
            p[j + 1] = v;
        }
    } else {
        qsort(p, (size_t)len, sizeof(int32_t), cmp_i32);
    }
}

/* Sort every row of a bucketed arc array, drop duplicates, compact into CSR.
 * `cnt` holds the raw row lengths; `buf` the raw arcs at rows starting at
 * raw offsets `roff`. */
static int finish_csr(int32_t n, const int64_t *roff, int32_t *buf, sxg_csr *out) {
    int64_t *newdeg = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!newdeg) return -2;
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t v = 0; v < n; ++v) {
        int32_t *p = buf + roff[v];
        int64_t len = roff[v + 1] - roff[v];
        sort_row(p, len);
        int64_t k = 0;
        for (int64_t i = 0; i < len; ++i)
            if (k == 0 || p[i] != p[k - 1]) p[k++] = p[i];
        newdeg[v] = k;
    }
    int32_t *off = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    if (!off) { free(newdeg); return -2; }
    int64_t acc = 0;
    for (int64_t v = 0; v < n; ++v) { off[v] = (int32_t)acc; acc += newdeg[v]; if (acc > INT32_MAX) { free(newdeg); free(off); return -3; } }
    off[n] = (int32_t)acc;
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(acc > 0 ? acc : 1));
    if (!idx) { free(newdeg); free(off); return -2; }
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t v = 0; v < n; ++v)
        memcpy(idx + off[v], buf + roff[v], sizeof(int32_t) * (size_t)newdeg[v]);
    free(newdeg);
    out->n = n; out->m = acc; out->offsets = off; out->indices = idx;
    return 0;
}

/* R-MAT edge `e`: for each of `scale` levels pick one quadrant of the
 * adjacency matrix with probabilities a, b, c, d=1-a-b-c, using a 32-bit
 * uniform draw per level (two draws per 64-bit SplitMix64 output). */
static inline void rmat_edge(uint64_t seed, int scale, uint64_t e,
                             uint32_t ta, uint32_t tab, uint32_t tabc,
                             int32_t *pu, int32_t *pv) {
    uint32_t u = 0, v = 0;
    int words = (scale + 1) / 2;
    for (int w = 0; w < words; ++w) {
        uint64_t h = sm64_at(seed, e * (uint64_t)words + (uint64_t)w);
        for (int half = 0; half < 2; ++half) {
            int lvl = 2 * w + half;
            if (lvl >= scale) break;
            uint32_t r = half ? (uint32_t)(h & 0xffffffffu) : (uint32_t)(h >> 32);
            uint32_t rb, cb;
            if (r < ta) { rb = 0; cb = 0; }
            else if (r < tab) { rb = 0; cb = 1; }
            else if (r < tabc) { rb = 1; cb = 0; }
            else { rb = 1; cb = 1; }
            u = (u << 1) | rb; v = (v << 1) | cb;
        }
    }
    *pu = (int32_t)u; *pv = (int32_t)v;
}

static uint32_t prob32(double p) {
    if (p <= 0.0) return 0u;
    if (p >= 1.0) return 0xffffffffu;
    return (uint32_t)(p * 4294967296.0);
}

/* R-MAT graph with 2^scale vertices and edge_factor * 2^scale generated edges.
 * directed = 0: symmetrised.  Self loops and duplicates are removed.
 * Returns 0 on success, -1 bad args, -2 out of memory, -3 too many arcs. */
int sxg_rmat(int scale, int edge_factor, double a, double b, double c,
             uint64_t seed, int directed, sxg_csr *out) {
    if (!out || scale < 1 || scale > 30 || edge_factor < 0) return -1;
    if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return -1;
    int32_t n = (int32_t)1 << scale;
    uint64_t ne = (uint64_t)edge_factor << scale;
    uint32_t ta = prob32(a), tab = prob32(a + b), tabc = prob32(a + b + c);
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cnt) return -2;
    /* pass 1: row lengths */
    #pragma omp parallel for schedule(static)
    for (uint64_t e = 0; e < ne; ++e) {
        int32_t u, v;
        rmat_edge(seed, scale, e, ta, tab, tabc, &u, &v);
        if (u == v) continue;
        #pragma omp atomic
        cnt[u + 1]++;
        if (!directed) {
            #pragma omp atomic
            cnt[v + 1]++;
        }
    }
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    int64_t total = cnt[n];
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!buf || !pos) { free(cnt); free(buf); free(pos); return -2; }
    memcpy(pos, cnt, sizeof(int64_t) * (size_t)(n + 1));
    /* pass 2: regenerate the same edges and scatter them into their rows */
    #pragma omp parallel for schedule(static)
    for (uint64_t e = 0; e < ne; ++e) {
        int32_t u, v;
        rmat_edge(seed, scale, e, ta, tab, tabc, &u, &v);
        if (u == v) continue;
        int64_t p;
        #pragma omp atomic capture
        p = pos[u]++;
        buf[p] = v;
        if (!directed) {
            #pragma omp atomic capture
            p = pos[v]++;
            buf[p] = u;
        }
    }
    free(pos);
    int rc = finish_csr(n, cnt, buf, out);
    free(cnt); free(buf);
    return rc;
}

/* side x side 4-neighbour grid, vertex id = row * side + col.  Edge ids:
 * horizontal (r,c)-(r,c+1) -> r*(side-1)+c; vertical (r,c)-(r+1,c) ->
 * side*(side-1) + r*side + c.  Each edge is deleted independently with
 * probability p_del (draw = SplitMix64 output number edge_id). */
int sxg_grid(int32_t side, double p_del, uint64_t seed, sxg_csr *out) {
    if (!out || side < 1 || side > 46340 || p_del < 0 || p_del > 1) return -1;
    int64_t n64 = (int64_t)side * side;
    int32_t n = (int32_t)n64;
    uint32_t tdel = prob32(p_del);
    int64_t hbase = 0, vbase = (int64_t)side * (side - 1);
    #define KEEP(id) ((uint32_t)(sm64_at(seed, (uint64_t)(id)) >> 32) >= tdel)
    int32_t *off = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    if (!off) return -2;
    off[0] = 0;
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!deg) { free(off); return -2; }
    #pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n64; ++v) {
        int64_t r = v / side, c = v % side;
        int d = 0;
        if (r > 0 && KEEP(vbase + (r - 1) * side + c)) d++;
        if (c > 0 && KEEP(hbase + r * (side - 1) + c - 1)) d++;
        if (c < side - 1 && KEEP(hbase + r * (side - 1) + c)) d++;
        if (r < side - 1 && KEEP(vbase + r * side + c)) d++;
        deg[v] = d;
    }
    int64_t acc = 0;
    for (int64_t v = 0; v < n64; ++v) { off[v] = (int32_t)acc; acc += deg[v]; }
    off[n] = (int32_t)acc;
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(acc > 0 ? acc : 1));
    if (!idx) { free(off); free(deg); return -2; }
    #pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n64; ++v) {
        int64_t r = v / side, c = v % side;
        int64_t p = off[v];
        if (r > 0 && KEEP(vbase + (r - 1) * side + c)) idx[p++] = (int32_t)(v - side);
        if (c > 0 && KEEP(hbase + r * (side - 1) + c - 1)) idx[p++] = (int32_t)(v - 1);
        if (c < side - 1 && KEEP(hbase + r * (side - 1) + c)) idx[p++] = (int32_t)(v + 1);
        if (r < side - 1 && KEEP(vbase + r * side + c)) idx[p++] = (int32_t)(v + side);
    }
    #undef KEEP
    free(deg);
    out->n = n; out->m = acc; out->offsets = off; out->indices = idx;
    return 0;
}

/* Weight of the arc u->v, uniform in [lo, hi].  symmetric != 0 gives both
 * arcs of an undirected edge the same weight (keyed on {min, max}). */
static inline uint32_t edge_weight(uint64_t seed, int32_t u, int32_t v,
                                   uint32_t lo, uint32_t hi, int symmetric) {
    uint32_t a = (uint32_t)u, b = (uint32_t)v;
    if (symmetric && a > b) { uint32_t t = a; a = b; b = t; }
    uint64_t key = ((uint64_t)a << 32) | b;
    uint64_t h = sm64_at(seed, key);
    uint64_t range = (uint64_t)hi - lo + 1;
    return lo + (uint32_t)(((h >> 32) * range) >> 32);
}

int sxg_weights(int32_t n, const int32_t *offsets, const int32_t *indices,
                uint32_t lo, uint32_t hi, uint64_t seed, int symmetric,
                uint32_t *w_out) {
    if (n < 0 || !offsets || lo > hi || !w_out) return -1;
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t v = 0; v < n; ++v)
        for (int64_t e = offsets[v]; e < offsets[v + 1]; ++e)
            w_out[e] = edge_weight(seed, (int32_t)v, indices[e], lo, hi, symmetric);
    return 0;
}

/* Transpose a CSR (out-arcs) into a CSC (in-arcs): in_indices rows sorted
 * ascending.  Optional weights follow their arcs. */
int sxg_transpose(int32_t n, int64_t m, const int32_t *offsets, const int32_t *indices,
                  const uint32_t *w, int32_t *in_offsets, int32_t *in_indices, uint32_t *in_w) {
    if (n < 0 || !offsets || !in_offsets || (m > 0 && (!indices || !in_indices))) return -1;
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cnt) return -2;
    for (int64_t e = 0; e < m; ++e) cnt[indices[e] + 1]++;
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    for (int64_t i = 0; i <= n; ++i) in_offsets[i] = (int32_t)cnt[i];
    /* rows of the source are visited in ascending order, so every in-row is
     * filled in ascending source order: sorted without a sort */
    for (int64_t v = 0; v < n; ++v)
        for (int64_t e = offsets[v]; e < offsets[v + 1]; ++e) {
            int64_t p = cnt[indices[e]]++;
            in_indices[p] = (int32_t)v;
            if (w && in_w) in_w[p] = w[e];
        }
    free(cnt);
    return 0;
}

int sxg_num_threads(void) { return omp_get_max_threads(); }
