// Host driver and C ABI of libsimdx.so (declarations and contracts in
// include/simdx.h).
//
// The driver owns device residency of the graph, the per-graph engine
// workspace, the persistent-grid sizing (Section 5, Eq. 1: the number of
// co-resident workgroups follows from the kernel's register and LDS use, here
// taken from the HIP occupancy API for our own code objects) and the run loop:
// a handful of persistent launches in fused mode, one launch per phase and
// iteration with the host deciding in between otherwise.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "simdx.h"
#include "sx_kernels.hpp"

using namespace sx;

static thread_local std::string g_last_error;

static sx_status fail(sx_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(SX_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                                \
  } while (0)

struct sx_ctx {
  int device;
  int cus;
  int cooperative;
  std::vector<float> mlp;  // learned-policy parameters (host copy)
  float *d_mlp = nullptr;
};

struct sx_graph {
  sx_ctx *ctx;
  DevGraph g;
  Work w;
  int weighted;
  int directed;
  std::vector<void *> owned;  // device allocations to free
  Ctrl *h_ctrl = nullptr;     // pinned host mirror of the first lines of Ctrl
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

struct sx_program {
  sx_ctx *ctx;
  sx_algo_params ap;
  sx_policy pol;
};

extern "C" {

const char *sx_status_str(sx_status s) {
  switch (s) {
    case SX_OK: return "ok";
    case SX_EINVAL: return "invalid argument";
    case SX_ENOMEM: return "out of memory";
    case SX_EHIP: return "HIP runtime error";
    case SX_EUNSUPPORTED: return "unsupported";
    case SX_EDEADLOCK: return "global barrier watchdog fired (workgroups not co-resident)";
    case SX_EOVERFLOW: return "distance overflow";
    case SX_ESTATE: return "bad state";
  }
  return "unknown status";
}

const char *sx_last_error(void) { return g_last_error.c_str(); }

int32_t sx_eq1_ctas(int32_t regs_per_sm, int32_t regs_per_thread, int32_t threads_per_wg,
                    int32_t sms) {
  if (regs_per_sm <= 0 || regs_per_thread <= 0 || threads_per_wg <= 0 || sms <= 0) return -1;
  const long long per = (long long)regs_per_sm / ((long long)regs_per_thread * threads_per_wg);
  return (int32_t)(per * sms);
}

sx_status sx_ctx_create(int hip_device, sx_ctx **out) {
  if (!out) return fail(SX_EINVAL, "out is NULL");
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (hip_device < 0 || hip_device >= ndev)
    return fail(SX_EINVAL, "device %d out of range (%d devices)", hip_device, ndev);
  HIP_TRY(hipSetDevice(hip_device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, hip_device));
  sx_ctx *c = new sx_ctx();
  c->device = hip_device;
  c->cus = prop.multiProcessorCount;
  c->cooperative = prop.cooperativeLaunch;
  *out = c;
  return SX_OK;
}

void sx_ctx_destroy(sx_ctx *c) {
  if (!c) return;
  if (c->d_mlp) (void)hipFree(c->d_mlp);
  delete c;
}

}  // extern "C"

// ------------------------------------------------------------- graphs ---
static sx_status dalloc(sx_graph *G, void **p, size_t bytes) {
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) return fail(SX_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  G->owned.push_back(*p);
  return SX_OK;
}

template <class T>
static sx_status dalloc_t(sx_graph *G, T **p, size_t count) {
  return dalloc(G, (void **)p, count * sizeof(T));
}

static void free_graph(sx_graph *G) {
  if (!G) return;
  for (void *p : G->owned) (void)hipFree(p);
  if (G->h_ctrl) (void)hipHostFree(G->h_ctrl);
  if (G->ev0) (void)hipEventDestroy(G->ev0);
  if (G->ev1) (void)hipEventDestroy(G->ev1);
  delete G;
}

static const int kChunk = 4 * kBlock;  // arcs per large-bin item

static sx_status validate_host(const sx_graph_desc *d) {
  const int32_t *off = d->offsets;
  if (off[0] != 0) return fail(SX_EINVAL, "offsets[0] != 0");
  for (int32_t v = 0; v < d->n; ++v)
    if (off[v + 1] < off[v]) return fail(SX_EINVAL, "offsets not monotone at %d", v);
  if ((int64_t)off[d->n] != d->m) return fail(SX_EINVAL, "offsets[n] != m");
  for (int64_t e = 0; e < d->m; ++e)
    if (d->indices[e] < 0 || d->indices[e] >= d->n)
      return fail(SX_EINVAL, "indices[%lld] = %d out of range", (long long)e, d->indices[e]);
  if (d->weights)
    for (int64_t e = 0; e < d->m; ++e)
      if (d->weights[e] == 0) return fail(SX_EINVAL, "weights[%lld] is zero", (long long)e);
  return SX_OK;
}

extern "C" sx_status sx_graph_load(sx_ctx *ctx, const sx_graph_desc *d, void *hip_stream,
                                   sx_graph **out) {
  if (!ctx || !d || !out) return fail(SX_EINVAL, "NULL argument");
  if (d->n < 0) return fail(SX_EINVAL, "n < 0");
  if (d->m < 0 || d->m >= (int64_t)INT32_MAX) return fail(SX_EINVAL, "m = %lld out of range", (long long)d->m);
  if (!d->offsets || (d->m > 0 && !d->indices)) return fail(SX_EINVAL, "missing CSR arrays");
  const bool undirected = (d->flags & SX_UNDIRECTED) != 0;
  if (undirected && (d->in_offsets || d->in_indices))
    return fail(SX_EINVAL, "undirected graph with in-neighbour arrays");
  if (!undirected && (!d->in_offsets || (d->m > 0 && !d->in_indices)))
    return fail(SX_EINVAL, "directed graph needs in_offsets / in_indices (CSC)");
  if (!undirected && d->weights && !d->in_weights)
    return fail(SX_EINVAL, "directed weighted graph needs in_weights");
  const bool dev = (d->flags & SX_DEVICE_PTRS) != 0;
  if ((d->flags & SX_VALIDATE) && !dev) {
    sx_status s = validate_host(d);
    if (s != SX_OK) return s;
  }
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)hip_stream;
  sx_graph *G = new sx_graph();
  G->ctx = ctx;
  G->weighted = d->weights != nullptr || d->m == 0;  // no arcs: trivially weighted
  G->directed = !undirected;
  const int n = d->n;
  const long long m = d->m;
  sx_status s;
#define TRY(x)                 \
  do {                         \
    s = (x);                   \
    if (s != SX_OK) {          \
      free_graph(G);           \
      return s;                \
    }                          \
  } while (0)
#define HTRY(x)                                                                   \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      free_graph(G);                                                              \
      return fail(SX_EHIP, "%s failed: %s", #x, hipGetErrorString(e_));           \
    }                                                                             \
  } while (0)
  DevGraph &g = G->g;
  g.n = n;
  g.m = m;
  g.directed = !undirected;
  auto upload = [&](const void *src, size_t bytes, const void **dst) -> sx_status {
    if (!src) { *dst = nullptr; return SX_OK; }
    if (dev) { *dst = src; return SX_OK; }
    void *p = nullptr;
    sx_status r = dalloc(G, &p, bytes);
    if (r != SX_OK) return r;
    if (bytes) {
      hipError_t e = hipMemcpyAsync(p, src, bytes, hipMemcpyHostToDevice, st);
      if (e != hipSuccess) return fail(SX_EHIP, "hipMemcpyAsync: %s", hipGetErrorString(e));
    }
    *dst = p;
    return SX_OK;
  };
  TRY(upload(d->offsets, sizeof(int) * (size_t)(n + 1), (const void **)&g.off));
  TRY(upload(d->indices, sizeof(int) * (size_t)m, (const void **)&g.idx));
  TRY(upload(d->weights, sizeof(unsigned) * (size_t)m, (const void **)&g.w));
  if (undirected) {
    g.in_off = g.off;
    g.in_idx = g.idx;
    g.in_w = g.w;
  } else {
    TRY(upload(d->in_offsets, sizeof(int) * (size_t)(n + 1), (const void **)&g.in_off));
    TRY(upload(d->in_indices, sizeof(int) * (size_t)m, (const void **)&g.in_idx));
    TRY(upload(d->in_weights, sizeof(unsigned) * (size_t)m, (const void **)&g.in_w));
  }
  // workspace
  Work &w = G->w;
  const size_t nn = (size_t)std::max(n, 1);
  const size_t words = (nn + 63) / 64 + 1;
  const size_t large_cap = nn + (size_t)(m / kChunk) + 2 + (size_t)(m / kChunk);
  w.qcap_small = (unsigned)nn;
  w.qcap_med = (unsigned)nn;
  w.qcap_large = (unsigned)std::min<size_t>(large_cap, 0xFFFFFFF0u);
  for (int p = 0; p < 2; ++p) {
    TRY(dalloc_t(G, &w.q[p][0], nn));
    TRY(dalloc_t(G, &w.q[p][1], nn));
    TRY(dalloc_t(G, &w.ql[p], large_cap));
    TRY(dalloc_t(G, &w.contrib[p], nn));
    TRY(dalloc_t(G, &w.alive[p], nn));
  }
  for (int b = 0; b < NBINS; ++b) TRY(dalloc_t(G, &w.bits[b], words));
  TRY(dalloc_t(G, &w.fbits, words));
  TRY(dalloc_t(G, &w.wavecnt, (size_t)kMaxGrid * kWaves * NBINS));
  TRY(dalloc_t(G, &w.wgc, (size_t)kMaxGrid));
  TRY(dalloc_t(G, &w.stamp, nn));
  TRY(dalloc_t(G, &w.deg, nn));
  TRY(dalloc_t(G, &w.dang, (size_t)4 * kMaxGrid));
  TRY(dalloc_t(G, &w.ctrl, 1));
  HTRY(hipMemsetAsync(w.ctrl, 0, sizeof(Ctrl), st));
  HTRY(hipHostMalloc((void **)&G->h_ctrl, sizeof(Ctrl), hipHostMallocDefault));
  HTRY(hipEventCreate(&G->ev0));
  HTRY(hipEventCreate(&G->ev1));
  HTRY(hipStreamSynchronize(st));
#undef TRY
#undef HTRY
  *out = G;
  return SX_OK;
}

extern "C" void sx_graph_destroy(sx_graph *g) { free_graph(g); }

extern "C" sx_status sx_graph_info(const sx_graph *g, int32_t *n, int64_t *m, int32_t *directed,
                                   int32_t *weighted) {
  if (!g) return fail(SX_EINVAL, "NULL graph");
  if (n) *n = g->g.n;
  if (m) *m = g->g.m;
  if (directed) *directed = g->directed;
  if (weighted) *weighted = g->weighted;
  return SX_OK;
}

// ----------------------------------------------------------- programs ---
extern "C" sx_status sx_program_register(sx_ctx *ctx, const sx_algo_params *p, sx_program **out) {
  if (!ctx || !p || !out) return fail(SX_EINVAL, "NULL argument");
  if (p->algo < SX_BFS || p->algo > SX_PAGERANK) return fail(SX_EINVAL, "unknown algorithm %d", (int)p->algo);
  if (p->algo == SX_PAGERANK && (p->pr_iters < 0 || !(p->pr_damping >= 0.f && p->pr_damping <= 1.f)))
    return fail(SX_EINVAL, "bad PageRank parameters");
  sx_program *P = new sx_program();
  P->ctx = ctx;
  P->ap = *p;
  memset(&P->pol, 0, sizeof P->pol);
  *out = P;
  return SX_OK;
}

extern "C" void sx_program_destroy(sx_program *p) { delete p; }

extern "C" sx_status sx_program_set_policy(sx_program *p, const sx_policy *pol) {
  if (!p || !pol) return fail(SX_EINVAL, "NULL argument");
  if (pol->direction < 0 || pol->direction > 2) return fail(SX_EINVAL, "bad direction");
  if (pol->filter < 0 || pol->filter > 2) return fail(SX_EINVAL, "bad filter");
  if (pol->fused < 0 || pol->fused > 2) return fail(SX_EINVAL, "bad fused");
  if (pol->policy < 0 || pol->policy > 1) return fail(SX_EINVAL, "bad policy");
  if (pol->bin_small < 0 || pol->bin_large < 0 || pol->online_cap < 0 || pol->grid_wgs < 0)
    return fail(SX_EINVAL, "negative policy field");
  if (pol->bin_small && pol->bin_large && pol->bin_large < pol->bin_small)
    return fail(SX_EINVAL, "bin_large < bin_small");
  if (pol->grid_wgs > kMaxGrid) return fail(SX_EINVAL, "grid_wgs > %d", kMaxGrid);
  if (pol->policy == SX_POLICY_LEARNED && p->ctx->mlp.empty())
    return fail(SX_ESTATE, "learned policy requested but no MLP loaded");
  p->pol = *pol;
  return SX_OK;
}

// ---------------------------------------------------------- occupancy ---
// Persistent grid (Section 5, Eq. 1): resident workgroups per CU for this
// kernel x number of CUs.
static int persistent_grid(sx_ctx *ctx, const void *kernel, int requested) {
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock, 0) != hipSuccess || per < 1)
    per = 1;
  int grid = per * ctx->cus;
  grid = std::min(grid, kMaxGrid);
  if (requested > 0) grid = std::min(grid, requested);
  return grid;
}

static int plain_grid(sx_ctx *ctx, const void *kernel) {
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock, 0) != hipSuccess || per < 1)
    per = 1;
  return std::min(per * ctx->cus, kMaxGrid);
}

static Params make_params(const sx_program *p, const sx_graph *G, int grid) {
  Params P;
  memset(&P, 0, sizeof P);
  const sx_policy &pol = p->pol;
  P.t1 = pol.bin_small > 0 ? pol.bin_small : 64;
  P.t2 = pol.bin_large > 0 ? pol.bin_large : 256;
  if (P.t2 < P.t1) P.t2 = P.t1;
  P.chunk = kChunk;
  const long long per_wave = pol.online_cap > 0 ? pol.online_cap : 64;
  long long cap = per_wave * (long long)grid * kWaves;
  if (pol.filter == SX_FILTER_ONLINE) cap = LLONG_MAX;
  P.online_cap = (unsigned)std::min<long long>(cap, 0xFFFFFFF0ll);
  P.filter = pol.filter;
  P.direction = pol.direction;
  P.alpha = 14.0f;
  P.beta = 24.0f;
  // a BFS level or a Bellman-Ford round adds at least one vertex to the set
  // of settled ones, so n + 2 iterations bound every correct run
  P.max_iters = G->g.n + 2;
  P.pr_d = p->ap.pr_damping;
  P.pr_iters = p->ap.pr_iters;
  (void)G;
  return P;
}

static sx_status read_ctrl(sx_graph *G, hipStream_t st) {
  HIP_TRY(hipMemcpyAsync(G->h_ctrl, G->w.ctrl, offsetof(Ctrl, flags), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return SX_OK;
}

static sx_status ctrl_error(const Ctrl *c) {
  if (c->state.v[0] == EXIT_LIMIT) return fail(SX_EHIP, "iteration limit reached (engine bug)");
  if (c->error.v[0] == SX_ERR_DEADLOCK)
    return fail(SX_EDEADLOCK, "global barrier watchdog fired");
  if (c->error.v[0] == SX_ERR_OVERFLOW) return fail(SX_EOVERFLOW, "distance reached 0xFFFFFFFF");
  if (c->error.v[0]) return fail(SX_EHIP, "device error %u", c->error.v[0]);
  return SX_OK;
}

static void fill_stats(const Ctrl *c, int launches, float ms, sx_run_stats *stats) {
  if (!stats) return;
  stats->edges_inspected = (int64_t)(*(const unsigned long long *)&c->stats.v[0]);
  stats->vertex_expansions = (int64_t)(*(const unsigned long long *)&c->stats.v[2]);
  stats->ballot_iters = (int32_t)c->stats.v[4];
  stats->pull_iters = (int32_t)c->stats.v[5];
  stats->iterations = (int32_t)c->stats.v[6];
  stats->launches = launches;
  stats->device_ms = ms;
}

// ---------------------------------------------------- BFS / SSSP runs ---
static sx_status run_traversal(sx_program *p, sx_graph *G, int src, void *d_out, hipStream_t st,
                               sx_run_stats *stats) {
  const int sssp = p->ap.algo == SX_SSSP;
  sx_ctx *ctx = p->ctx;
  const bool fused = p->pol.fused != SX_UNFUSED;
  int grid;
  if (fused) {
    grid = std::min(persistent_grid(ctx, trav_kernel(TK_PUSH_FUSED, sssp), p->pol.grid_wgs),
                    persistent_grid(ctx, trav_kernel(TK_PULL_FUSED, sssp), p->pol.grid_wgs));
  } else {
    grid = plain_grid(ctx, trav_kernel(TK_PUSH_STEP, sssp));
    if (p->pol.grid_wgs > 0) grid = std::min(grid, p->pol.grid_wgs);
  }
  TravArgs a;
  memset(&a, 0, sizeof a);
  a.g = G->g;
  a.w = G->w;
  a.P = make_params(p, G, grid);
  a.state_i = (int *)d_out;
  a.src = src;
  // unexplored arcs (BFS direction rule)
  int h_off[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(h_off, G->g.off + src, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  unsigned long long mu = (unsigned long long)(G->g.m - (h_off[1] - h_off[0]));
  int launches = 0;
  HIP_TRY(hipEventRecord(G->ev0, st));
  HIP_TRY(trav_init(a, sssp, mu, st));
  ++launches;
  if (fused) {
    bool pull_next = p->pol.direction == SX_DIR_PULL;
    for (int batch = 0;; ++batch) {
      for (int k = 0; k < 4; ++k) {
        HIP_TRY(trav_launch(pull_next ? TK_PULL_FUSED : TK_PUSH_FUSED, sssp, a, 0, grid, st));
        ++launches;
        pull_next = !pull_next;
      }
      HIP_TRY(hipEventRecord(G->ev1, st));
      sx_status s = read_ctrl(G, st);
      if (s != SX_OK) return s;
      s = ctrl_error(G->h_ctrl);
      if (s != SX_OK) return s;
      if (G->h_ctrl->state.v[0] == EXIT_DONE) break;
      if (batch > 1000000) return fail(SX_EHIP, "run did not converge");
    }
  } else {
    bool pulling = p->pol.direction == SX_DIR_PULL;
    for (int it = 0;; ++it) {
      if (!pulling) {
        HIP_TRY(reset_slot(G->w.ctrl, (it + 2) % 3, st));
        HIP_TRY(trav_launch(TK_PUSH_STEP, sssp, a, it, grid, st));
        launches += 2;
      } else {
        HIP_TRY(trav_launch(TK_PULL_SCAN, sssp, a, it, grid, st));
        HIP_TRY(reset_slot(G->w.ctrl, (it + 1) % 3, st));
        HIP_TRY(trav_launch(TK_PULL_LISTS, sssp, a, it, grid, st));
        HIP_TRY(trav_launch(TK_PULL_STEP, sssp, a, it, grid, st));
        launches += 4;
      }
      sx_status s = read_ctrl(G, st);
      if (s != SX_OK) return s;
      s = ctrl_error(G->h_ctrl);
      if (s != SX_OK) return s;
      const Counters &q = G->h_ctrl->q[(it + 1) % 3];
      DecideIn in;
      in.nf = q.nf;
      in.mf = q.mf;
      in.ovf = q.overflow;
      in.it = it;
      in.pulling = pulling;
      in.vote = !sssp;
      in.n = G->g.n;
      in.m = G->g.m;
      Decision d = decide_core(in, a.P, mu);
      if (d.done) break;
      bool rebuild = d.ballot;
      if (pulling && d.to_push) { pulling = false; rebuild = q.overflow != 0; }
      else if (!pulling && d.to_pull) pulling = true;
      if (rebuild && !pulling) {
        HIP_TRY(trav_launch(TK_BALLOT1, sssp, a, it, grid, st));
        HIP_TRY(trav_launch(TK_BALLOT2, sssp, a, it, grid, st));
        launches += 2;
      }
    }
    HIP_TRY(hipEventRecord(G->ev1, st));
    sx_status s = read_ctrl(G, st);
    if (s != SX_OK) return s;
  }
  HIP_TRY(hipEventSynchronize(G->ev1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, G->ev0, G->ev1));
  fill_stats(G->h_ctrl, launches, ms, stats);
  return SX_OK;
}

// ------------------------------------------------------------- k-core ---
static sx_status run_kcore(sx_program *p, sx_graph *G, void *d_out, hipStream_t st,
                           sx_run_stats *stats) {
  if (G->g.n == 0) {
    if (stats) memset(stats, 0, sizeof *stats);
    return SX_OK;
  }
  const int grid = persistent_grid(p->ctx, kcore_kernel(), p->pol.grid_wgs);
  KArgs a;
  memset(&a, 0, sizeof a);
  a.g = G->g;
  a.w = G->w;
  a.P = make_params(p, G, grid);
  a.core = (int *)d_out;
  int launches = 0;
  HIP_TRY(hipEventRecord(G->ev0, st));
  HIP_TRY(kcore_launch(a, grid, st, true));
  ++launches;
  for (;;) {
    HIP_TRY(kcore_launch(a, grid, st, false));
    ++launches;
    HIP_TRY(hipEventRecord(G->ev1, st));
    sx_status s = read_ctrl(G, st);
    if (s != SX_OK) return s;
    s = ctrl_error(G->h_ctrl);
    if (s != SX_OK) return s;
    if (G->h_ctrl->state.v[0] == EXIT_DONE) break;
    if (launches > 64) return fail(SX_EHIP, "k-core did not finish");
  }
  HIP_TRY(hipEventSynchronize(G->ev1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, G->ev0, G->ev1));
  fill_stats(G->h_ctrl, launches, ms, stats);
  return SX_OK;
}

// ----------------------------------------------------------- PageRank ---
static sx_status run_pagerank(sx_program *p, sx_graph *G, void *d_out, hipStream_t st,
                              sx_run_stats *stats) {
  const int n = G->g.n;
  if (n == 0) {
    if (stats) memset(stats, 0, sizeof *stats);
    return SX_OK;
  }
  const int grid = persistent_grid(p->ctx, pagerank_kernel(), p->pol.grid_wgs);
  PrArgs a;
  memset(&a, 0, sizeof a);
  a.g = G->g;
  a.w = G->w;
  a.P = make_params(p, G, grid);
  a.rank = (float *)d_out;
  const float d = p->ap.pr_damping;
  a.base_teleport = (float)((1.0 - (double)d) / (double)n);
  a.inv_n = (float)(1.0 / (double)n);
  a.iters = p->ap.pr_iters;
  HIP_TRY(hipEventRecord(G->ev0, st));
  if (a.iters == 0) {
    std::vector<float> h((size_t)n, a.inv_n);
    HIP_TRY(hipMemcpyAsync(d_out, h.data(), sizeof(float) * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
  } else {
    HIP_TRY(pagerank_launch(a, grid, st));
  }
  HIP_TRY(hipEventRecord(G->ev1, st));
  sx_status s = read_ctrl(G, st);
  if (s != SX_OK) return s;
  s = ctrl_error(G->h_ctrl);
  if (s != SX_OK) return s;
  HIP_TRY(hipEventSynchronize(G->ev1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, G->ev0, G->ev1));
  fill_stats(G->h_ctrl, 2, ms, stats);
  return SX_OK;
}

extern "C" sx_status sx_run(sx_program *p, const sx_graph *gc, int32_t source, void *d_out,
                            void *hip_stream, sx_run_stats *stats) {
  if (!p || !gc || !d_out) return fail(SX_EINVAL, "NULL argument");
  sx_graph *G = const_cast<sx_graph *>(gc);
  if (G->ctx != p->ctx) return fail(SX_EINVAL, "graph and program belong to different contexts");
  HIP_TRY(hipSetDevice(p->ctx->device));
  hipStream_t st = (hipStream_t)hip_stream;
  const int n = G->g.n;
  switch (p->ap.algo) {
    case SX_BFS:
    case SX_SSSP:
      if (n == 0) return fail(SX_EINVAL, "empty graph has no source");
      if (source < 0 || source >= n) return fail(SX_EINVAL, "source %d out of range [0, %d)", source, n);
      if (p->ap.algo == SX_SSSP && !G->weighted) return fail(SX_EINVAL, "SSSP needs edge weights");
      return run_traversal(p, G, source, d_out, st, stats);
    case SX_KCORE:
      return run_kcore(p, G, d_out, st, stats);
    case SX_PAGERANK:
      return run_pagerank(p, G, d_out, st, stats);
  }
  return fail(SX_EINVAL, "unknown algorithm");
}

extern "C" sx_status sx_read_vertices(const sx_graph *g, sx_algo algo, const void *d_out,
                                      void *host_out, void *hip_stream) {
  if (!g || !d_out || !host_out) return fail(SX_EINVAL, "NULL argument");
  (void)algo;  // every output type is 4 bytes wide
  hipStream_t st = (hipStream_t)hip_stream;
  HIP_TRY(hipMemcpyAsync(host_out, d_out, (size_t)g->g.n * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return SX_OK;
}

extern "C" sx_status sx_kernel_info_get(sx_ctx *ctx, const char *name, sx_kernel_info *out) {
  if (!ctx || !name || !out) return fail(SX_EINVAL, "NULL argument");
  struct Named { const char *name; const void *k; bool persistent; };
  const Named table[] = {
      {"bfs_push_fused", trav_kernel(TK_PUSH_FUSED, 0), true},
      {"bfs_pull_fused", trav_kernel(TK_PULL_FUSED, 0), true},
      {"sssp_push_fused", trav_kernel(TK_PUSH_FUSED, 1), true},
      {"sssp_pull_fused", trav_kernel(TK_PULL_FUSED, 1), true},
      {"bfs_push_step", trav_kernel(TK_PUSH_STEP, 0), false},
      {"bfs_pull_step", trav_kernel(TK_PULL_STEP, 0), false},
      {"sssp_push_step", trav_kernel(TK_PUSH_STEP, 1), false},
      {"sssp_pull_step", trav_kernel(TK_PULL_STEP, 1), false},
      {"ballot_count", trav_kernel(TK_BALLOT1, 0), false},
      {"ballot_write", trav_kernel(TK_BALLOT2, 0), false},
      {"kcore_fused", kcore_kernel(), true},
      {"pagerank_fused", pagerank_kernel(), true},
  };
  for (const Named &t : table) {
    if (strcmp(t.name, name) != 0) continue;
    hipFuncAttributes fa;
    HIP_TRY(hipFuncGetAttributes(&fa, t.k));
    out->vgprs = fa.numRegs;
    out->sgprs = 0;
    out->lds_bytes = (int32_t)fa.sharedSizeBytes;
    out->block = kBlock;
    int per = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, t.k, kBlock, 0));
    out->wgs_per_cu = per;
    out->cus = ctx->cus;
    out->grid_wgs = std::min(per * ctx->cus, kMaxGrid);
    return SX_OK;
  }
  return fail(SX_EINVAL, "unknown kernel name '%s'", name);
}
