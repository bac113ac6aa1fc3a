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
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "simdx.h"
#include "sx_kernels.hpp"
#include "sx_policy.hpp"

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

// Launches enqueued beyond the last run's count in the first batch of a
// sequenced traversal (the count can differ by one or two between runs:
// the order of atomic updates changes SSSP's intermediate lists)
static constexpr int kSeqHintMargin = 2;
// Sequenced k-core grid for graphs up to 2^23 vertices and 2^28 arcs
static constexpr int kKcoreSmallGrid = 256;
static constexpr long long kKcoreSmallN = 1ll << 23;
static constexpr long long kKcoreSmallArcs = 1ll << 28;

// Workspace of sx_run_static, for callers that cannot allocate device
// memory: one array per device, held until the process ends.  Host code
// never passes the array's name to a kernel (it is a host-side stand-in):
// the device address comes from hipGetSymbolAddress, per device, in
// sx_ctx_create.
static constexpr size_t kStaticScratchBytes = 256ull << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// Zero `words` 32-bit words (the control block of a static-workspace run;
// a kernel rather than hipMemsetAsync, so that the call can be captured).
__global__ void k_static_clear(unsigned *p, unsigned long long words) {
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (unsigned long long)gridDim.x * blockDim.x)
    p[i] = 0u;
}

struct sx_ctx {
  int device;
  int cus;
  int cooperative;
  double wall_khz = 100000.0;  // rate of the device's constant wall clock
  std::vector<float> mlp;  // learned-policy parameters (host copy)
  float *d_mlp = nullptr;  // and on the device
  // training scratch, grown on demand: per sample y[4], h[64], delta[68], loss
  float *d_scratch = nullptr;
  size_t scratch_samples = 0;
  // batched mode: team workspaces sized for (team_n, team_m), kept for reuse
  std::vector<void *> team_allocs;
  std::vector<Work> team_work;
  int team_n = 0;
  long long team_m = 0;
  sx_batch_config tuned{0, 0, 0};
  // batched mode: device query table, order, team workspace table, queue
  // counter and statistics, grown on demand and kept; timing events
  void *bq = nullptr, *bo = nullptr, *bw = nullptr, *bh = nullptr, *bs = nullptr;
  int batch_cap_q = 0, batch_cap_t = 0;
  hipEvent_t be0 = nullptr, be1 = nullptr;
  // sx_run_static: this device's static workspace (from
  // hipGetSymbolAddress), pinned control-block mirrors and events, all set
  // up here so that the call itself allocates nothing
  unsigned char *d_static = nullptr;
  Ctrl *hs_ctrl[2] = {nullptr, nullptr};
  hipEvent_t sev[4] = {nullptr, nullptr, nullptr, nullptr};
};

struct sx_graph {
  sx_ctx *ctx;
  DevGraph g;
  Work w;
  int weighted;
  int directed;
  std::vector<void *> owned;  // device allocations to free
  Ctrl *h_ctrl = nullptr;     // pinned host mirrors of the first lines of Ctrl
  Ctrl *h_ctrl2 = nullptr;    // (two: one per batch in flight)
  hipEvent_t ev0 = nullptr, ev1 = nullptr, evb[2] = {nullptr, nullptr};
  // degree-ordered renumbering (SX_REORDER): old id -> new id on the device
  // and the host, and the run's state array in the new numbering
  bool reordered = false;
  int *d_inv = nullptr;
  std::vector<int> h_inv;
  unsigned *d_xdist = nullptr;  // SSSP / WCC expansion record (TravArgs::xdist)
  void *state = nullptr;
  long long weight_sum = -1;  // sum of the arc weights, once SX_DELTA_AUTO needed it
  // where the lists of the next iteration sit after sx_run_iterations:
  // record slot, region parity, run grid (-1: no such run yet)
  int next_slot = -1, next_parity = 0, next_grid = 0;
  // launches the last sequenced BFS / SSSP / WCC run on this graph needed
  // (0: none yet): the next run enqueues that many plus kSeqHintMargin in its
  // first batch instead of 16, so few launches run after the end
  int seq_hint[3] = {0, 0, 0};
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
  int khz = 0;
  HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, hip_device));
  // the static workspace's address on this device (each device holds its
  // own copy of the array), with the device current
  void *sp = nullptr;
  HIP_TRY(hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)));
  if (!sp) return fail(SX_EHIP, "hipGetSymbolAddress returned no address for the static workspace");
  sx_ctx *c = new sx_ctx();
  c->device = hip_device;
  c->cus = prop.multiProcessorCount;
  c->cooperative = prop.cooperativeLaunch;
  if (khz > 0) c->wall_khz = (double)khz;
  c->d_static = (unsigned char *)sp;
  hipError_t e = hipSuccess;
  for (int i = 0; i < 2 && e == hipSuccess; ++i)
    e = hipHostMalloc((void **)&c->hs_ctrl[i], sizeof(Ctrl), hipHostMallocDefault);
  for (int i = 0; i < 4 && e == hipSuccess; ++i)
    e = i < 2 ? hipEventCreate(&c->sev[i]) : hipEventCreateWithFlags(&c->sev[i], hipEventDisableTiming);
  if (e != hipSuccess) {
    sx_ctx_destroy(c);
    return fail(SX_EHIP, "context set-up: %s", hipGetErrorString(e));
  }
  *out = c;
  return SX_OK;
}

void sx_ctx_destroy(sx_ctx *c) {
  if (!c) return;
  if (c->d_mlp) (void)hipFree(c->d_mlp);
  if (c->d_scratch) (void)hipFree(c->d_scratch);
  for (void *p : c->team_allocs) (void)hipFree(p);
  for (void *p : {c->bq, c->bo, c->bw, c->bh, c->bs})
    if (p) (void)hipFree(p);
  if (c->be0) (void)hipEventDestroy(c->be0);
  if (c->be1) (void)hipEventDestroy(c->be1);
  for (Ctrl *h : c->hs_ctrl)
    if (h) (void)hipHostFree(h);
  for (hipEvent_t e : c->sev)
    if (e) (void)hipEventDestroy(e);
  delete c;
}

sx_status sx_policy_load_mlp(sx_ctx *ctx, const float *params, int64_t nparams) {
  if (!ctx || !params) return fail(SX_EINVAL, "NULL argument");
  if (nparams != SX_MLP_NPARAMS) return fail(SX_EINVAL, "nparams %lld != %d", (long long)nparams, SX_MLP_NPARAMS);
  HIP_TRY(hipSetDevice(ctx->device));
  if (!ctx->d_mlp) HIP_TRY(hipMalloc(&ctx->d_mlp, sizeof(float) * SX_MLP_NPARAMS));
  HIP_TRY(hipMemcpy(ctx->d_mlp, params, sizeof(float) * SX_MLP_NPARAMS, hipMemcpyHostToDevice));
  ctx->mlp.assign(params, params + SX_MLP_NPARAMS);
  return SX_OK;
}

static sx_status mlp_scratch(sx_ctx *ctx, int n, float **Y, float **H, float **D, float **L) {
  const size_t per = 4 + 64 + 68 + 1;
  if ((size_t)n > ctx->scratch_samples) {
    if (ctx->d_scratch) (void)hipFree(ctx->d_scratch);
    ctx->d_scratch = nullptr;
    ctx->scratch_samples = 0;
    hipError_t e = hipMalloc(&ctx->d_scratch, sizeof(float) * per * (size_t)n);
    if (e != hipSuccess) return fail(SX_ENOMEM, "MLP scratch: %s", hipGetErrorString(e));
    ctx->scratch_samples = (size_t)n;
  }
  float *b = ctx->d_scratch;
  *Y = b;
  *H = b + 4 * (size_t)n;
  *D = b + 68 * (size_t)n;
  *L = b + 136 * (size_t)n;
  return SX_OK;
}

sx_status sx_mlp_forward(sx_ctx *ctx, const float *P, const float *X, int32_t n, float *Y,
                         void *hip_stream) {
  if (!ctx || !P || (n > 0 && (!X || !Y))) return fail(SX_EINVAL, "NULL argument");
  if (n < 0) return fail(SX_EINVAL, "n < 0");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(mlp_forward_wave(P, X, n, Y, (hipStream_t)hip_stream));
  return SX_OK;
}

sx_status sx_mlp_forward_host(const float *P, const float *X, int32_t n, float *Y) {
  if (!P || n < 0 || (n > 0 && (!X || !Y))) return fail(SX_EINVAL, "bad argument");
  for (int32_t i = 0; i < n; ++i) mlp_eval_host(P, X + (size_t)i * kMlpIn, Y + (size_t)i * kMlpOut);
  return SX_OK;
}

sx_status sx_mlp_loss_grad(sx_ctx *ctx, const float *P, const float *X, const float *T,
                           const float *M, int32_t n, float *loss, float *G, void *hip_stream) {
  if (!ctx || !P || !X || !T || !M || !loss || !G) return fail(SX_EINVAL, "NULL argument");
  if (n <= 0) return fail(SX_EINVAL, "n must be positive");
  HIP_TRY(hipSetDevice(ctx->device));
  float *Y, *H, *D, *L;
  sx_status s = mlp_scratch(ctx, n, &Y, &H, &D, &L);
  if (s != SX_OK) return s;
  HIP_TRY(mlp_loss_grad(P, X, T, M, n, Y, H, D, L, loss, G, (hipStream_t)hip_stream));
  return SX_OK;
}

sx_status sx_mlp_adam(sx_ctx *ctx, float *P, const float *G, float *Mo, float *Vo, int32_t step,
                      float lr, float b1, float b2, float eps, void *hip_stream) {
  if (!ctx || !P || !G || !Mo || !Vo) return fail(SX_EINVAL, "NULL argument");
  if (step < 1) return fail(SX_EINVAL, "step counts from 1");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(mlp_adam(P, G, Mo, Vo, step, lr, b1, b2, eps, (hipStream_t)hip_stream));
  return SX_OK;
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
  if (G->h_ctrl2) (void)hipHostFree(G->h_ctrl2);
  if (G->ev0) (void)hipEventDestroy(G->ev0);
  if (G->ev1) (void)hipEventDestroy(G->ev1);
  for (hipEvent_t e : G->evb)
    if (e) (void)hipEventDestroy(e);
  delete G;
}


// Worklist storage for grids of up to `gmax` workgroups (regions: workgroup b
// of G owns 1/G of every bin array).  The sizes make every list a ballot scan
// builds fit its regions for any G <= gmax:
//   a scan over `count` positions gives each workgroup at most
//   count / G + 512 of them (ranges are multiples of 512), so the small and
//   medium arrays hold 2n + 1024 gmax entries (the first n + 512 gmax for
//   scans, the rest headroom for the online filter);
//   a large vertex adds ceil(deg / chunk) <= deg / chunk + 1 items, so a
//   range of r vertices adds at most r + arcs / chunk: the large array holds
//   n + 1024 gmax + gmax (ceil(arcs / chunk) + 1) entries, with arcs the
//   degree sum (2m for the k-core of a directed graph: in- plus out-arcs);
//   the k-core alive lists are binned like the worklists, with the same
//   capacities (a scan re-emits at most the entries it reads).
struct Sizing {
  size_t tot_s, tot_l, words, fwords;
};
static Sizing work_sizing(long long n, long long m, bool directed, int gmax) {
  Sizing z;
  const size_t nn = (size_t)std::max<long long>(n, 1);
  const size_t arcs = (size_t)(directed ? 2 * m : m);
  z.tot_s = 2 * nn + 1024 * (size_t)gmax;
  z.tot_l = nn + 1024 * (size_t)gmax + (size_t)(gmax + 1) * ((arcs + kChunk - 1) / kChunk + 1);
  z.words = (nn + 63) / 64 + 1;
  z.fwords = (nn + 63) / 64 + 1;
  return z;
}

// Allocate a workspace through `al(void **, bytes)`; `full` adds the k-core
// and PageRank arrays.
// Entries of the expansion record (TravArgs::xdist): per vertex, then per
// large-bin chunk.
static size_t xrec_entries(long long n, long long m) {
  return 2 * (size_t)std::max<long long>(n, 0) + (size_t)(std::max<long long>(m, 0) / kChunk) + 2;
}

template <class Alloc>
static sx_status work_alloc(Alloc al, long long n, long long m, bool directed, int gmax, bool full,
                            Work &w) {
  memset(&w, 0, sizeof w);
  const Sizing z = work_sizing(n, m, directed, gmax);
  if (z.tot_l > 0xFFFFFFF0ull || z.tot_s > 0xFFFFFFF0ull)
    return fail(SX_EUNSUPPORTED, "graph too large for 32-bit worklist indices");
  const size_t nn = (size_t)std::max<long long>(n, 1);
  sx_status r;
#define ALLOC(ptr, bytes)                                  \
  do {                                                     \
    if ((r = al((void **)&(ptr), (bytes))) != SX_OK) return r; \
  } while (0)
  for (int p = 0; p < 2; ++p) {
    ALLOC(w.reg_s[p], 4 * z.tot_s);
    ALLOC(w.reg_m[p], 4 * z.tot_s);
    ALLOC(w.reg_l[p], 8 * z.tot_l);
  }
  w.tot_s = (unsigned)z.tot_s;
  w.tot_m = (unsigned)z.tot_s;
  w.tot_l = (unsigned)z.tot_l;
  ALLOC(w.rec, sizeof(RecSlot) * NSLOTS);
  for (int b = 0; b < NBINS; ++b) ALLOC(w.bits[b], 8 * z.words);
  ALLOC(w.fbits, 8 * z.fwords);
  ALLOC(w.stamp, 4 * nn);
  ALLOC(w.ctrl, sizeof(Ctrl));
  if (full) {
    for (int p = 0; p < 2; ++p) {
      ALLOC(w.al_s[p], 4 * z.tot_s);
      ALLOC(w.al_m[p], 4 * z.tot_s);
      ALLOC(w.al_l[p], 8 * z.tot_l);
      ALLOC(w.contrib[p], 4 * nn);
    }
    ALLOC(w.alive_min, 4 * 2 * kMaxGrid);
    ALLOC(w.deg, 4 * nn);
    ALLOC(w.dang, 4 * 4 * kMaxGrid);
    ALLOC(w.prd, 4 * nn);
    ALLOC(w.prp, 4 * 2 * 8 * kMaxGrid);
    ALLOC(w.bph, 4 * nn);
    for (int p = 0; p < 2; ++p) ALLOC(w.bpq[p], 8 * nn);
  }
#undef ALLOC
  return SX_OK;
}

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
  if (d->flags & SX_REORDER) {
    // renumber by decreasing degree into arrays the graph owns; temporaries
    // are freed once the build has finished on the stream
    std::vector<void *> temps;
    auto own = [&](void **p, size_t bytes) -> hipError_t {
      return dalloc(G, p, bytes) == SX_OK ? hipSuccess : hipErrorOutOfMemory;
    };
    auto tmp = [&](void **p, size_t bytes) -> hipError_t {
      hipError_t e = hipMalloc(p, bytes ? bytes : 1);
      if (e == hipSuccess) temps.push_back(*p);
      return e;
    };
    G->h_inv.resize((size_t)n);
    DevGraph g2;
    const hipError_t e = reorder_build(g, own, tmp, st, g2, &G->d_inv, G->h_inv.data());
    for (void *p : temps) (void)hipFree(p);
    if (e != hipSuccess) {
      free_graph(G);
      return fail(e == hipErrorOutOfMemory ? SX_ENOMEM : SX_EHIP, "renumbering: %s", hipGetErrorString(e));
    }
    g = g2;
    G->reordered = true;
    TRY(dalloc(G, &G->state, sizeof(int) * (size_t)(n > 0 ? n : 1)));
  }
  // workspace
  Work &w = G->w;
  TRY(work_alloc([&](void **p, size_t bytes) { return dalloc(G, p, bytes); }, n, m, !undirected,
                 kMaxGrid, true, w));
  TRY(dalloc(G, (void **)&G->d_xdist, sizeof(unsigned) * xrec_entries(n, m)));
  HTRY(hipMemsetAsync(w.ctrl, 0, sizeof(Ctrl), st));
  HTRY(hipHostMalloc((void **)&G->h_ctrl, sizeof(Ctrl), hipHostMallocDefault));
  HTRY(hipHostMalloc((void **)&G->h_ctrl2, sizeof(Ctrl), hipHostMallocDefault));
  HTRY(hipEventCreate(&G->ev0));
  HTRY(hipEventCreate(&G->ev1));
  HTRY(hipEventCreateWithFlags(&G->evb[0], hipEventDisableTiming));
  HTRY(hipEventCreateWithFlags(&G->evb[1], hipEventDisableTiming));
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
  if (p->algo < SX_BFS || p->algo > SX_BP) return fail(SX_EINVAL, "unknown algorithm %d", (int)p->algo);
  if (p->algo == SX_BP && (p->bp_iters < 0 || !(p->bp_kappa >= 0.f && p->bp_kappa < 1.f)))
    return fail(SX_EINVAL, "bad belief-propagation parameters (bp_iters >= 0, 0 <= bp_kappa < 1)");
  if (p->algo == SX_KCORE && p->kcore_k < 0) return fail(SX_EINVAL, "kcore_k < 0");
  if (p->algo == SX_PAGERANK && (p->pr_iters < 0 || !(p->pr_damping >= 0.f && p->pr_damping <= 1.f) ||
                                 !(p->pr_tol >= 0.f && p->pr_tol < 1.f) ||
                                 (p->pr_tol > 0.f && !(p->pr_damping < 1.f))))
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
  if (pol->fused < 0 || pol->fused > 4) return fail(SX_EINVAL, "bad fused");
  if (pol->watchdog_us < 0) return fail(SX_EINVAL, "watchdog_us < 0");
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
// Graphs from this many arcs up, with at least 8 arcs per vertex, run the
// wide sequenced traversal kernel; sparse graphs keep the unconstrained one
// however large, since their thousands of small levels pay for its spills
// on every level (4096^2 grid BFS: 160 ms wide, 47 ms on the 2048^2 grid).
static const long long kBigGraphArcs = 1ll << 25;

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

// the heuristic's bin thresholds (lane / wavefront / workgroup)
static const int kDefaultT1 = 64, kDefaultT2 = 512;

static Params make_params(const sx_program *p, const sx_graph *G, int grid) {
  Params P;
  memset(&P, 0, sizeof P);
  const sx_policy &pol = p->pol;
  P.t1 = pol.bin_small > 0 ? pol.bin_small : kDefaultT1;
  // 512: below it a vertex's arcs are one or two steps of a wavefront (four
  // arcs per lane); as a workgroup item they would leave most of its 2,048
  // lanes-times-arcs idle (R-MAT s22: BFS 0.56 -> 0.42 ms, SSSP 3.1 -> 2.8 ms
  // against 256; k-core is flat from 384 to 768 and slower from 1,024 up)
  P.t2 = pol.bin_large > 0 ? pol.bin_large : kDefaultT2;
  if (P.t2 < P.t1) P.t2 = P.t1;
  P.chunk = kChunk;
  // online filter limit per workgroup and bin: the caller's entries per
  // wavefront (JIT filter only); otherwise the whole region
  const long long lim = pol.filter == SX_FILTER_JIT && pol.online_cap > 0
                            ? (long long)pol.online_cap * kWaves : 0;
  P.online_cap = (unsigned)std::min<long long>(lim, 0xFFFFFFF0ll);
  (void)grid;
  P.filter = pol.filter;
  P.direction = pol.direction;
  P.alpha = 14.0f;
  P.beta = 24.0f;
  P.alpha_w = 0.5f;
  P.beta_w = 4.0f;
  // a BFS level or a Bellman-Ford round adds at least one vertex to the set
  // of settled ones, so n + 2 iterations bound every correct run.  With
  // buckets, each bucket takes at most (its vertices + 1) rounds: 2n + 4.
  const bool seq_arr = p->pol.fused == SX_SEQUENCED || p->pol.fused == SX_FUSE_AUTO;
  P.delta = p->ap.algo == SX_SSSP && seq_arr ? p->ap.sssp_delta : 0u;
  P.delta_after = 0;
  P.max_iters = G ? (P.delta ? (int)std::min<long long>(2ll * G->g.n + 4, INT_MAX / 2) : G->g.n + 2)
                  : INT_MAX / 2;
  P.pr_d = p->ap.pr_damping;
  P.pr_iters = p->ap.pr_iters;
  P.learned = pol.policy == SX_POLICY_LEARNED ? 1 : 0;
  P.bins_fixed = (pol.bin_small > 0 || pol.bin_large > 0) ? 1 : 0;
  P.kfix = p->ap.algo == SX_KCORE ? p->ap.kcore_k : 0;
  // the one-workgroup tail pays only once little work is left: one CU's LDS
  // atomics take the decrements the grid spreads over all CUs (R-MAT s22
  // from 35,827 vertices / 36 M arcs on: 6.8 ms against 5.7 on the grid;
  // s15-s18 from 8-16 K vertices: 25-44 % faster)
  P.ktail = 0;
  P.ktail_arcs = ~0ull;
  if (p->ap.algo == SX_KCORE && P.kfix == 0 && p->pol.kcore_tail >= 0) {
    P.ktail = p->pol.kcore_tail ? std::min(p->pol.kcore_tail, kTailMax) : kTailDefault;
    if (p->pol.kcore_tail == 0) P.ktail_arcs = kTailDefaultArcs;
  }
  P.watchdog = pol.watchdog_us > 0
                   ? (unsigned long long)((double)pol.watchdog_us * p->ctx->wall_khz / 1000.0)
                   : (unsigned long long)(2.0 * p->ctx->wall_khz * 1000.0);
  if (p->ap.algo == SX_WCC) {
    // every vertex starts active, so the first iteration pulls; a pull step
    // reads every in-arc once without atomics, a push step the frontier's
    // arcs with an atomic minimum per improvement: pull while the
    // frontier's arcs exceed m / 2, push again below m / 8
    P.alpha_w = 2.0f;
    P.beta_w = 8.0f;
  }
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
  if (c->error.v[0] == SX_ERR_CAPACITY)
    return fail(SX_EHIP, "a scanned worklist exceeded its regions (engine bug)");
  if (c->error.v[0] == SX_ERR_TAIL)
    return fail(SX_EHIP, "the k-core tail's compacted rows disagree with the degrees (engine bug)");
  if (c->error.v[0] == SX_ERR_INPUT)
    return fail(SX_EINVAL, "an input value is outside its domain (belief-propagation prior not in (0, 1))");
  if (c->error.v[0]) return fail(SX_EHIP, "device error %u", c->error.v[0]);
  return SX_OK;
}

// Drive a sequenced run: enqueue launches (`launch(L)` enqueues launch L) in
// batches until the run-state line reports an end phase.  The first batch
// (`first` launches) is checked before anything else is enqueued, so a short
// run costs no idle launches; from then on two batches are in flight (the
// host reads the state copied after batch i while batch i + 1 runs), so the
// GPU does not wait for the host.  A launch after the end returns at once
// (about 2 us).  On return `*fin` points at the pinned copy of the control
// block taken after the batch that ended the run.
template <class Launch>
static sx_status seq_drive(sx_graph *G, hipStream_t st, int first, int maxb, unsigned limit,
                           Launch launch, int &launches, const Ctrl **fin, unsigned *fin_phase = nullptr) {
  struct Pend {
    Ctrl *h;
    hipEvent_t ev;
    unsigned L;
  } pend[2] = {{G->h_ctrl, G->evb[0], 0u}, {G->h_ctrl2, G->evb[1], 0u}};
  unsigned L = 0;
  int batch = first;
  auto enqueue = [&](Pend &p) -> sx_status {
    for (int k = 0; k < batch; ++k) HIP_TRY(launch(L++));
    launches += batch;
    HIP_TRY(hipMemcpyAsync(p.h, G->w.ctrl, offsetof(Ctrl, flags), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(p.ev, st));
    p.L = L;
    batch = std::min(batch * 2, maxb);
    return SX_OK;
  };
  sx_status s = enqueue(pend[0]);
  if (s != SX_OK) return s;
  int cur = 0;
  bool piped = false;
  for (;;) {
    Pend &p = pend[cur];
    HIP_TRY(hipEventSynchronize(p.ev));
    s = ctrl_error(p.h);
    if (s != SX_OK) return s;
    const unsigned ph = p.h->seq[p.L & 1].v[0];
    if (ph == SEQ_LIMIT) return fail(SX_EHIP, "iteration limit reached (engine bug)");
    if (ph >= SEQ_DONE) {
      *fin = p.h;
      if (fin_phase) *fin_phase = ph;
      return SX_OK;
    }
    if (L > limit) return fail(SX_EHIP, "run did not converge");
    if (!piped) {
      // second and third batch: from here on one batch stays in flight
      s = enqueue(pend[cur ^ 1]);
      if (s != SX_OK) return s;
      piped = true;
    }
    s = enqueue(p);
    if (s != SX_OK) return s;
    cur ^= 1;
  }
}

// grid: workgroups of the run's phase kernels (the barrier stall is averaged
// over them); khz: the device wall clock's rate.
static void fill_stats(const Ctrl *c, int launches, float ms, int grid, double khz,
                       sx_run_stats *stats) {
  if (!stats) return;
  memset(stats, 0, sizeof *stats);
  unsigned long long e = 0, x = 0, wt = 0;
  for (int i = 0; i < kStatLines; ++i) {
    e += *(const unsigned long long *)&c->statw[i].v[0];
    x += *(const unsigned long long *)&c->statw[i].v[2];
    wt += *(const unsigned long long *)&c->statw[i].v[4];
  }
  stats->barrier_wait_ms = grid > 0 ? (double)wt / (double)grid / khz : 0.0;
  stats->policy_evals = (int32_t)c->pol.v[0];
  for (int k = 0; k < 8; ++k) memcpy(&stats->policy_x[k], &c->pol.v[1 + k], 4);
  for (int k = 0; k < 4; ++k) memcpy(&stats->policy_y[k], &c->pol.v[9 + k], 4);
  stats->edges_inspected = (int64_t)e;
  stats->vertex_expansions = (int64_t)x;
  stats->ballot_iters = (int32_t)c->stats.v[4];
  stats->pull_iters = (int32_t)c->stats.v[5];
  stats->iterations = (int32_t)c->stats.v[6];
  stats->launches = launches;
  stats->device_ms = ms;
  stats->scan_entries = (int64_t)(*(const unsigned long long *)&c->stats.v[8]);
}

// ---------------------------------------------------- BFS / SSSP runs ---
// Totals of one record slot (the host side of view_build).
struct HostTotals {
  unsigned long long cnt[NBINS], mf;
  unsigned nf, ovf;
};
static sx_status read_totals(const Work &w, int slot, int grid, hipStream_t st,
                             std::vector<RecSlot> &buf, HostTotals &T) {
  buf.resize(1);
  HIP_TRY(hipMemcpyAsync(buf.data(), w.rec + slot, sizeof(RecSlot), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  memset(&T, 0, sizeof T);
  const RecSlot &r = buf[0];
  for (int b = 0; b < grid; ++b) {
    for (int i = 0; i < NBINS; ++i) T.cnt[i] += r.cnt[i][b];
    T.nf += r.nf[b] & ~kRecOvf;
    T.ovf |= (r.nf[b] & kRecOvf) ? 1u : 0u;
    T.mf += r.mf[b];
  }
  return SX_OK;
}

// The host decision of the one-phase loop: decide_core plus the learned
// policy, evaluated exactly as the device does it.
// Host-side record of the network's decisions (one-phase arrangement).
struct HostPolicyLog {
  int evals = 0;
  float x[8] = {0}, y[4] = {0};
};

static Decision host_decide(const sx_ctx *ctx, const sx_policy &pol, Params &P, bool sssp,
                            const sx_graph *G, int it, bool pulling, const HostTotals &T,
                            unsigned long long &mu, PolicyState &ps, HostPolicyLog *log = nullptr) {
  DecideIn in;
  in.nf = T.nf;
  in.mf = T.mf;
  in.ovf = T.ovf;
  in.it = it;
  in.pulling = pulling;
  in.vote = !sssp;
  in.n = G->g.n;
  in.m = G->g.m;
  Decision d = decide_core(in, P, mu);
  if (!d.done && P.learned && in.mf >= kPolicyMinArcs) {
    float x[kMlpIn], y[kMlpOut];
    policy_features(in.nf, in.mf, sssp ? (unsigned long long)G->g.m : mu, G->g.n, G->g.m, ps,
                    pulling, x);
    mlp_eval_host(ctx->mlp.data(), x, y);
    if (log) {
      ++log->evals;
      memcpy(log->x, x, sizeof log->x);
      memcpy(log->y, y, sizeof log->y);
    }
    apply_network(y, pulling, in.ovf != 0, pol.direction, P.filter, P.bins_fixed != 0, kDefaultT1,
                  std::max(kDefaultT1, kDefaultT2), d, P.t1, P.t2);
  }
  ps.nf_prev = in.nf;
  ps.reached += in.nf;
  return d;
}

// SX_DELTA_AUTO: buckets of about 40 mean arc weights, from iteration 64 on,
// on graphs of at least 2^21 vertices with fewer than 8 arcs per vertex
// (meshes and road-like graphs, thousands of iterations: on the 4096^2 grid with weights in
// [1, 1000] the best widths measured were 20,000-50,000, and on the 2048^2
// grid buckets save 30 %), none on denser graphs, whose few iterations
// buckets only multiply (R-MAT s22: every width tried was slower), nor on
// smaller ones, where the extra iterations cost more than the re-expansions
// they save (1024^2 grid: 5 % slower).
static sx_status auto_delta(sx_graph *G, hipStream_t st, unsigned *delta) {
  *delta = 0;
  const long long n = G->g.n, m = G->g.m;
  if (!G->g.w || n < (1ll << 21) || m <= 0 || m >= 8 * n) return SX_OK;
  if (G->weight_sum < 0) {
    unsigned long long *d = (unsigned long long *)&G->w.ctrl->aux.v[4];
    HIP_TRY(weight_sum(G->g.w, m, d, st));
    unsigned long long h = 0;
    HIP_TRY(hipMemcpyAsync(&h, d, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    G->weight_sum = (long long)h;
  }
  const double w = std::floor(40.0 * (double)G->weight_sum / (double)m + 0.5);
  *delta = (unsigned)std::min(std::max(w, 1.0), 2147483647.0);
  return SX_OK;
}

static int trav_algo(const sx_program *p) {
  return p->ap.algo == SX_SSSP ? ALG_SSSP : (p->ap.algo == SX_WCC ? ALG_WCC : ALG_BFS);
}

// large dense graphs take the wide sequenced kernel (three workgroups per CU)
static int trav_seq_kind(const sx_graph *G) {
  return G->g.m >= kBigGraphArcs && G->g.m >= 8ll * G->g.n ? TK_SEQ_WIDE : TK_SEQ;
}

// Workgroups of a traversal run's phase kernels under the program's policy.
static int traversal_grid(sx_program *p, const sx_graph *G, int max_it) {
  const int algo = trav_algo(p);
  sx_ctx *ctx = p->ctx;
  const bool fused = max_it == 0 && (p->pol.fused == SX_FUSED || p->pol.fused == SX_FUSED_ALL);
  const int fk = p->pol.fused == SX_FUSED_ALL ? TK_FUSED_ALL : TK_FUSED;
  const bool sequenced = max_it == 0 && (p->pol.fused == SX_SEQUENCED || p->pol.fused == SX_FUSE_AUTO);
  int grid;
  if (sequenced) {
    grid = plain_grid(ctx, trav_kernel(trav_seq_kind(G), algo));
    if (p->pol.grid_wgs > 0) grid = std::min(grid, p->pol.grid_wgs);
  } else if (fused) {
    // the push and pull kernels of selective fusion share the run's lists,
    // whose regions are laid out for one grid: both must fit it
    grid = persistent_grid(ctx, trav_kernel(fk, algo), p->pol.grid_wgs);
    if (fk == TK_FUSED)
      grid = std::min(grid, persistent_grid(ctx, trav_kernel(TK_FUSED_PULL, algo), p->pol.grid_wgs));
  } else {
    grid = plain_grid(ctx, trav_kernel(TK_PUSH_STEP, algo));
    if (p->pol.grid_wgs > 0) grid = std::min(grid, p->pol.grid_wgs);
  }
  return grid;
}

// max_it > 0: stop the one-phase arrangement after that many iterations and
// note where the next iteration's lists are (sx_run_iterations).
static sx_status run_traversal(sx_program *p, sx_graph *G, int src, void *d_out, hipStream_t st,
                               sx_run_stats *stats, int max_it = 0) {
  const int algo = trav_algo(p);
  const bool wcc = algo == ALG_WCC;
  // aggregation (minimum) programs decide with the SSSP rule
  const bool aggr = algo != ALG_BFS;
  sx_ctx *ctx = p->ctx;
  const bool fused = max_it == 0 && (p->pol.fused == SX_FUSED || p->pol.fused == SX_FUSED_ALL);
  const int fk = p->pol.fused == SX_FUSED_ALL ? TK_FUSED_ALL : TK_FUSED;
  const bool sequenced = max_it == 0 && (p->pol.fused == SX_SEQUENCED || p->pol.fused == SX_FUSE_AUTO);
  const int seq_kind = trav_seq_kind(G);
  const int grid = traversal_grid(p, G, max_it);
  TravArgs a;
  memset(&a, 0, sizeof a);
  a.g = G->g;
  a.w = G->w;
  a.P = make_params(p, G, grid);
  a.state_i = (int *)d_out;
  a.src = src;
  a.mlp = ctx->d_mlp;
  a.wcc_inv = wcc && G->reordered ? G->d_inv : nullptr;
  // the expansion record pays where a listed vertex is often improved
  // again within its own step before its expansion (R-MAT s22: a third of
  // the expansions skipped); on sparse graphs (4096^2 grid, unbucketed
  // SSSP: no expansion skipped, 15 % slower) it only adds a dependent load,
  // so graphs of fewer than 8 arcs per vertex run without it
  a.xdist = G->g.m >= 8ll * G->g.n ? G->d_xdist : nullptr;
  if (a.P.learned && !ctx->d_mlp) return fail(SX_ESTATE, "learned policy without loaded MLP");
  if (algo == ALG_SSSP && a.P.delta == SX_DELTA_AUTO) {
    sx_status s = auto_delta(G, st, &a.P.delta);
    if (s != SX_OK) return s;
    // a run that ends within this many iterations is not high-diameter:
    // it keeps the plain relaxation (sparse random and R-MAT graphs with
    // 4-6 arcs per vertex lost 5-13 % to buckets from the first iteration)
    a.P.delta_after = 64;
  }
  // every WCC vertex starts active: unless the caller forces push, the first
  // iteration pulls; a push start builds its lists with a ballot scan
  const bool pull_first = p->pol.direction == SX_DIR_PULL || (wcc && p->pol.direction == SX_DIR_AUTO);
  int launches = 0;
  HIP_TRY(hipEventRecord(G->ev0, st));
  // unexplored arcs (BFS direction rule) are computed on the device
  // (with the first state of a sequenced run: one launch less, and the host
  // enqueues the first phases while the set-up runs)
  HIP_TRY(trav_init(a, algo, 0ull, grid, st, pull_first, sequenced));
  ++launches;
  const Ctrl *fin = G->h_ctrl;
  HostPolicyLog plog;
  if (sequenced) {
    // a launch after the run's end returns at once but still costs ~5 us (768
    // workgroups of the wide kernel): size the first batch by the last run of
    // this algorithm on this graph (another source: a different count; too
    // few launches only cost one host round trip before the next batch)
    int &hint = G->seq_hint[algo];
    const int first = hint > 0 ? std::min(hint + kSeqHintMargin, 64) : 16;
    sx_status s = seq_drive(
        G, st, first, 64, (unsigned)(8 * (long long)G->g.n + 1024),
        [&](unsigned L) { return trav_launch(seq_kind, algo, a, (int)L, 0, grid, st); }, launches, &fin);
    if (s != SX_OK) return s;
    // Ctrl::stats word 12: the index + 1 of the launch that ended the run
    hint = (int)fin->stats.v[12];
    HIP_TRY(hipEventRecord(G->ev1, st));
  } else if (fused) {
    if (wcc && !pull_first) {
      // iteration 0's lists (every vertex) by a ballot scan; state word 2
      // tells the persistent kernel they are there
      HIP_TRY(trav_launch(TK_BALLOT, algo, a, -1, 0, grid, st));
      ++launches;
    }
    int pull_next = pull_first ? 1 : 0;
    for (int batch = 0;; ++batch) {
      // all fusion switches direction inside its one kernel: launches after
      // the run's end return at once
      for (int k = 0; k < 4; ++k) {
        const int kind = fk == TK_FUSED_ALL ? fk : (pull_next ? TK_FUSED_PULL : TK_FUSED);
        HIP_TRY(trav_launch(kind, algo, a, 0, 0, grid, st));
        ++launches;
        pull_next ^= 1;
        if (fk == TK_FUSED_ALL) break;
      }
      HIP_TRY(hipEventRecord(G->ev1, st));
      sx_status s = read_ctrl(G, st);
      if (s != SX_OK) return s;
      s = ctrl_error(G->h_ctrl);
      if (s != SX_OK) return s;
      if (G->h_ctrl->state.v[0] == EXIT_DONE) break;
      if (fk == TK_FUSED_ALL && G->h_ctrl->state.v[0] != EXIT_NONE)
        return fail(SX_EHIP, "all-fused run ended with state %u", G->h_ctrl->state.v[0]);
      if (batch > 1000000) return fail(SX_EHIP, "run did not converge");
    }
  } else {
    bool pulling = pull_first;
    bool rebuilt = false;
    PolicyState ps{0u, 0ull};
    if (wcc && !pull_first) {
      HIP_TRY(trav_launch(TK_BALLOT, algo, a, -1, 0, grid, st));
      launches += 1;
      rebuilt = true;
    }
    sx_status s0 = read_ctrl(G, st);
    if (s0 != SX_OK) return s0;
    unsigned long long mu = *(const unsigned long long *)&G->h_ctrl->state.v[6];
    std::vector<RecSlot> buf;
    G->next_slot = -1;
    for (int it = 0;; ++it) {
      if (max_it > 0 && it >= max_it) {
        // stop before iteration `it`: its lists are the online lists of the
        // last step (slot it % 3) or a ballot rebuild (slot SLOT_SCAN); a
        // pull iteration next has no push list
        if (!pulling) {
          G->next_slot = rebuilt ? SLOT_SCAN : it % 3;
          G->next_parity = it & 1;
          G->next_grid = grid;
        }
        break;
      }
      if (!pulling) {
        HIP_TRY(trav_launch(TK_PUSH_STEP, algo, a, it, rebuilt ? 1 : 0, grid, st));
        launches += 1;
      } else {
        HIP_TRY(trav_launch(TK_PULL_SCAN, algo, a, it, 0, grid, st));
        HIP_TRY(trav_launch(TK_PULL_STEP, algo, a, it, 0, grid, st));
        launches += 2;
      }
      sx_status s = read_ctrl(G, st);
      if (s != SX_OK) return s;
      s = ctrl_error(G->h_ctrl);
      if (s != SX_OK) return s;
      HostTotals T;
      s = read_totals(G->w, (it + 1) % 3, grid, st, buf, T);
      if (s != SX_OK) return s;
      Decision d = host_decide(ctx, p->pol, a.P, aggr, G, it, pulling, T, mu, ps, &plog);
      if (d.done) break;
      bool rebuild = false;
      if (!pulling) {
        if (d.to_pull) pulling = true;
        else rebuild = d.ballot;
      } else if (d.to_push) {
        pulling = false;
        rebuild = T.ovf != 0;
      }
      rebuilt = false;
      if (rebuild) {
        HIP_TRY(trav_launch(TK_BALLOT, algo, a, it, 0, grid, st));
        launches += 1;
        rebuilt = true;
      }
    }
    HIP_TRY(hipEventRecord(G->ev1, st));
    sx_status s = read_ctrl(G, st);
    if (s != SX_OK) return s;
  }
  HIP_TRY(hipEventSynchronize(G->ev1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, G->ev0, G->ev1));
  fill_stats(fin, launches, ms, grid, ctx->wall_khz, stats);
  if (stats && !sequenced && !fused) {
    // the one-phase arrangement decides on the host
    stats->policy_evals = plog.evals;
    memcpy(stats->policy_x, plog.x, sizeof plog.x);
    memcpy(stats->policy_y, plog.y, sizeof plog.y);
  }
  return SX_OK;
}

// ------------------------------------------------------------- k-core ---
static sx_status run_kcore(sx_program *p, sx_graph *G, void *d_out, hipStream_t st,
                           sx_run_stats *stats) {
  if (G->g.n == 0) {
    if (stats) memset(stats, 0, sizeof *stats);
    return SX_OK;
  }
  const bool sequenced = p->pol.fused != SX_FUSED;
  // a phase's fixed cost (the launch, the record prefix over the
  // workgroups' records) grows with the grid: undirected R-MAT s18 / s20 /
  // s22 decompose 5.8 / 5.0 / 1.3 % faster on 256 workgroups than on 512,
  // while directed s24 (16.8 M vertices, 537 M in- plus out-arcs) is 7.4 %
  // slower; graphs up to kKcoreSmallN vertices and kKcoreSmallArcs arcs take
  // 256 unless the caller sets the grid
  const long long karcs = (long long)G->g.m * (G->g.directed ? 2 : 1);
  const int seq_cap = p->pol.grid_wgs > 0 ? p->pol.grid_wgs
                      : (G->g.n <= kKcoreSmallN && karcs <= kKcoreSmallArcs) ? kKcoreSmallGrid
                                                                               : kMaxGrid;
  const int grid = sequenced ? std::min(plain_grid(p->ctx, kcore_seq_kernel()), seq_cap)
                             : persistent_grid(p->ctx, kcore_kernel(), p->pol.grid_wgs);
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
  if (sequenced) {
    HIP_TRY(kcore_seq_launch(a, 0, grid, st, true));
    const Ctrl *fin = G->h_ctrl;
    unsigned ph = 0;
    sx_status s = seq_drive(
        G, st, 16, 16, (unsigned)(16 * (long long)G->g.n + 1024),
        [&](unsigned L) { return kcore_seq_launch(a, L, grid, st, false); }, launches, &fin, &ph);
    if (s != SX_OK) return s;
    if (ph == KP_TAIL) {
      // the last levels in one workgroup (compaction, then the peel)
      HIP_TRY(kcore_tail_launch(a, grid, st));
      launches += 4;
      s = read_ctrl(G, st);
      if (s != SX_OK) return s;
      s = ctrl_error(G->h_ctrl);
      if (s != SX_OK) return s;
      fin = G->h_ctrl;
    }
    if (a.P.kfix) HIP_TRY(kcore_membership(a.core, G->g.n, st));
    HIP_TRY(hipEventRecord(G->ev1, st));
    HIP_TRY(hipEventSynchronize(G->ev1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, G->ev0, G->ev1));
    fill_stats(fin, launches, ms, grid, p->ctx->wall_khz, stats);
    return SX_OK;
  }
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
  if (a.P.kfix) {
    HIP_TRY(kcore_membership(a.core, G->g.n, st));
    HIP_TRY(hipEventRecord(G->ev1, st));
  }
  HIP_TRY(hipEventSynchronize(G->ev1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, G->ev0, G->ev1));
  fill_stats(G->h_ctrl, launches, ms, grid, p->ctx->wall_khz, stats);
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
  const bool conv = p->ap.pr_tol > 0.f;
  const int grid = persistent_grid(p->ctx, pagerank_kernel(conv), p->pol.grid_wgs);
  PrArgs a;
  memset(&a, 0, sizeof a);
  a.g = G->g;
  a.w = G->w;
  a.P = make_params(p, G, grid);
  // a PageRank workgroup takes a whole vertex (no chunks), so the large bin
  // starts higher than for the traversals (directed R-MAT s24: 38.2 ms at
  // 512, 36.2 ms at 2,048)
  if (p->pol.bin_large <= 0) a.P.t2 = std::max(a.P.t1, 2048);
  a.rank = (float *)d_out;
  const float d = p->ap.pr_damping;
  a.base_teleport = (float)((1.0 - (double)d) / (double)n);
  a.inv_n = (float)(1.0 / (double)n);
  a.iters = p->ap.pr_iters;
  if (conv) {
    // run to convergence: a pending change of at most thr per vertex leaves
    // an L1 error of at most n thr / (1 - d) = tol / 2; a pull step that
    // changes the vector by at most tol (1 - d) / d is within tol of the
    // fixed point (contraction with factor d in L1)
    a.conv = 1;
    a.max_pull = a.iters > 0 ? a.iters : 1000;
    a.thr = (float)((double)p->ap.pr_tol * (1.0 - (double)d) / (2.0 * (double)n));
    a.stop_change = (float)((double)p->ap.pr_tol * (1.0 - (double)d) / std::max((double)d, 1e-30));
  }
  HIP_TRY(hipEventRecord(G->ev0, st));
  if (a.iters == 0 && !conv) {
    std::vector<float> h((size_t)n, a.inv_n);
    HIP_TRY(hipMemcpyAsync(d_out, h.data(), sizeof(float) * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
  } else {
    HIP_TRY(pagerank_launch(a, grid, st));
  }
  int launches = 2;
  if (conv) {
    // the pull kernel ends the run or hands it to the push kernel
    sx_status s0 = read_ctrl(G, st);
    if (s0 != SX_OK) return s0;
    s0 = ctrl_error(G->h_ctrl);
    if (s0 != SX_OK) return s0;
    if (G->h_ctrl->state.v[0] == EXIT_SWITCH) {
      const int pgrid = persistent_grid(p->ctx, pagerank_push_kernel(), p->pol.grid_wgs);
      HIP_TRY(pagerank_push_launch(a, pgrid, st));
      ++launches;
    }
  }
  HIP_TRY(hipEventRecord(G->ev1, st));
  sx_status s = read_ctrl(G, st);
  if (s != SX_OK) return s;
  s = ctrl_error(G->h_ctrl);
  if (s != SX_OK) return s;
  if (conv && G->h_ctrl->state.v[0] != EXIT_DONE)
    return fail(SX_EHIP, "PageRank run ended in state %u", G->h_ctrl->state.v[0]);
  HIP_TRY(hipEventSynchronize(G->ev1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, G->ev0, G->ev1));
  fill_stats(G->h_ctrl, launches, ms, grid, p->ctx->wall_khz, stats);
  return SX_OK;
}

// ------------------------------------------------- belief propagation ---
static sx_status run_bp(sx_program *p, sx_graph *G, void *d_belief, hipStream_t st, sx_run_stats *stats) {
  const int n = G->g.n;
  if (n == 0 || p->ap.bp_iters == 0) {
    if (stats) memset(stats, 0, sizeof *stats);
    return SX_OK;
  }
  const int grid = persistent_grid(p->ctx, bp_kernel(), p->pol.grid_wgs);
  BpArgs a;
  memset(&a, 0, sizeof a);
  a.g = G->g;
  a.w = G->w;
  a.P = make_params(p, G, grid);
  // a workgroup takes a whole vertex (no chunks), as in PageRank
  if (p->pol.bin_large <= 0) a.P.t2 = std::max(a.P.t1, 2048);
  a.belief = (float *)d_belief;
  a.kappa = p->ap.bp_kappa;
  a.iters = p->ap.bp_iters;
  HIP_TRY(hipEventRecord(G->ev0, st));
  HIP_TRY(bp_launch(a, grid, st));
  HIP_TRY(hipEventRecord(G->ev1, st));
  sx_status s = read_ctrl(G, st);
  if (s != SX_OK) return s;
  s = ctrl_error(G->h_ctrl);
  if (s != SX_OK) return s;
  HIP_TRY(hipEventSynchronize(G->ev1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, G->ev0, G->ev1));
  fill_stats(G->h_ctrl, 4, ms, grid, p->ctx->wall_khz, stats);
  return SX_OK;
}

// ------------------------------------------------ policy data collection ---
namespace {
struct Snapshot {
  std::vector<std::pair<void *, size_t>> items;  // (device source, bytes)
  std::vector<void *> copies;
  sx_status save(hipStream_t st) {
    for (size_t i = 0; i < items.size(); ++i)
      HIP_TRY(hipMemcpyAsync(copies[i], items[i].first, items[i].second, hipMemcpyDeviceToDevice, st));
    return SX_OK;
  }
  sx_status restore(hipStream_t st) {
    for (size_t i = 0; i < items.size(); ++i)
      HIP_TRY(hipMemcpyAsync(items[i].first, copies[i], items[i].second, hipMemcpyDeviceToDevice, st));
    return SX_OK;
  }
  ~Snapshot() {
    for (void *c : copies) (void)hipFree(c);
  }
};
}  // namespace

extern "C" sx_status sx_policy_collect(sx_program *p, const sx_graph *gc, int32_t src, void *d_out,
                                       void *hip_stream, int32_t stride, float *features,
                                       float *arm_ms, int32_t max_records, int32_t *nrecords) {
  if (!p || !gc || !d_out || !features || !arm_ms || !nrecords) return fail(SX_EINVAL, "NULL argument");
  if (p->ap.algo != SX_BFS && p->ap.algo != SX_SSSP) return fail(SX_EINVAL, "BFS or SSSP only");
  sx_graph *G = const_cast<sx_graph *>(gc);
  if (src < 0 || src >= G->g.n) return fail(SX_EINVAL, "source out of range");
  if (G->reordered) return fail(SX_EUNSUPPORTED, "policy collection on a renumbered graph (SX_REORDER)");
  if (p->ap.algo == SX_SSSP && !G->weighted) return fail(SX_EINVAL, "SSSP needs edge weights");
  if (stride < 1) stride = 1;
  HIP_TRY(hipSetDevice(p->ctx->device));
  hipStream_t st = (hipStream_t)hip_stream;
  const int sssp = p->ap.algo == SX_SSSP;
  const int n = G->g.n;
  const int grid = plain_grid(p->ctx, trav_kernel(TK_PUSH_STEP, sssp));
  TravArgs a;
  memset(&a, 0, sizeof a);
  a.g = G->g;
  a.w = G->w;
  sx_program hp = *p;
  hp.pol.policy = SX_POLICY_HEURISTIC;
  hp.pol.fused = SX_UNFUSED;
  a.P = make_params(&hp, G, grid);
  a.state_i = (int *)d_out;
  a.src = src;
  const Work &w = G->w;
  Snapshot snap;
  for (int par = 0; par < 2; ++par) {
    snap.items.push_back({w.reg_s[par], sizeof(int) * (size_t)w.tot_s});
    snap.items.push_back({w.reg_m[par], sizeof(int) * (size_t)w.tot_m});
    snap.items.push_back({w.reg_l[par], sizeof(unsigned long long) * (size_t)w.tot_l});
  }
  snap.items.push_back({w.rec, sizeof(RecSlot) * NSLOTS});
  snap.items.push_back({d_out, sizeof(int) * (size_t)n});
  snap.items.push_back({w.stamp, sizeof(int) * (size_t)n});
  // the expansion record: an arm's expansions must not make the replay skip
  snap.items.push_back({G->d_xdist, sizeof(unsigned) * xrec_entries(n, G->g.m)});
  snap.items.push_back({w.ctrl, sizeof(Ctrl)});
  for (auto &it : snap.items) {
    void *c = nullptr;
    hipError_t e = hipMalloc(&c, it.second);
    if (e != hipSuccess) return fail(SX_ENOMEM, "snapshot: %s", hipGetErrorString(e));
    snap.copies.push_back(c);
  }
  int h_off[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(h_off, G->g.off + src, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  unsigned long long mu = (unsigned long long)(G->g.m - (h_off[1] - h_off[0]));
  HIP_TRY(trav_init(a, sssp, mu, grid, st));
  const int arm_t[4][2] = {{16, 256}, {64, 256}, {64, 1024}, {256, 2048}};
  // features of the decision before iteration `it`, computed exactly as the
  // device does after the previous iteration (before iteration 0: the source
  // alone)
  PolicyState ps{0u, 0ull};
  float xnext[8];
  policy_features(1u, (unsigned long long)(h_off[1] - h_off[0]),
                  sssp ? (unsigned long long)G->g.m : mu, n, G->g.m, ps, false, xnext);
  bool last_ovf = false, pulling = false, rebuilt = false;
  int rec = 0;
  hipEvent_t e0 = G->ev0, e1 = G->ev1;
  std::vector<RecSlot> buf;
  for (int it = 0;; ++it) {
    if (rec < max_records && it % stride == 0) {
      float *x = features + (size_t)rec * 8;
      for (int i = 0; i < 8; ++i) x[i] = xnext[i];
      float *t = arm_ms + (size_t)rec * SX_POLICY_ARMS;
      sx_status s = snap.save(st);
      if (s != SX_OK) return s;
      for (int arm = 0; arm < SX_POLICY_ARMS; ++arm) {
        TravArgs b = a;
        // arm 0 pushes the online lists: not available after a pull
        // iteration or an overflow
        if (arm == 0 && (pulling || last_ovf)) { t[arm] = NAN; continue; }
        HIP_TRY(hipEventRecord(e0, st));
        if (arm >= 1 && arm <= 4) {
          b.P.t1 = arm_t[arm - 1][0];
          b.P.t2 = arm_t[arm - 1][1];
          HIP_TRY(trav_launch(TK_BALLOT, sssp, b, it - 1, 0, grid, st));
          HIP_TRY(trav_launch(TK_PUSH_STEP, sssp, b, it, 1, grid, st));
        } else if (arm == 0) {
          HIP_TRY(trav_launch(TK_PUSH_STEP, sssp, b, it, rebuilt ? 1 : 0, grid, st));
        } else {
          HIP_TRY(trav_launch(TK_PULL_SCAN, sssp, b, it, 0, grid, st));
          HIP_TRY(trav_launch(TK_PULL_STEP, sssp, b, it, 0, grid, st));
        }
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        t[arm] = ms;
        s = snap.restore(st);
        if (s != SX_OK) return s;
      }
      HIP_TRY(hipStreamSynchronize(st));
      ++rec;
    }
    // the heuristic's own iteration, exactly as in the one-phase run loop
    if (!pulling) {
      HIP_TRY(trav_launch(TK_PUSH_STEP, sssp, a, it, rebuilt ? 1 : 0, grid, st));
    } else {
      HIP_TRY(trav_launch(TK_PULL_SCAN, sssp, a, it, 0, grid, st));
      HIP_TRY(trav_launch(TK_PULL_STEP, sssp, a, it, 0, grid, st));
    }
    sx_status s = read_ctrl(G, st);
    if (s != SX_OK) return s;
    s = ctrl_error(G->h_ctrl);
    if (s != SX_OK) return s;
    HostTotals T;
    s = read_totals(w, (it + 1) % 3, grid, st, buf, T);
    if (s != SX_OK) return s;
    Params P0 = a.P;
    const PolicyState ps_before = ps;
    Decision d = host_decide(p->ctx, hp.pol, P0, sssp, G, it, pulling, T, mu, ps);
    policy_features(T.nf, T.mf, sssp ? (unsigned long long)G->g.m : mu, n, G->g.m, ps_before,
                    pulling, xnext);
    last_ovf = T.ovf != 0;
    if (d.done) break;
    bool rebuild = false;
    if (!pulling) {
      if (d.to_pull) pulling = true;
      else rebuild = d.ballot;
    } else if (d.to_push) {
      pulling = false;
      rebuild = T.ovf != 0;
    }
    rebuilt = false;
    if (rebuild) {
      HIP_TRY(trav_launch(TK_BALLOT, sssp, a, it, 0, grid, st));
      rebuilt = true;
      last_ovf = false;
    }
  }
  HIP_TRY(hipStreamSynchronize(st));
  *nrecords = rec;
  return SX_OK;
}

// -------------------------------------------------------------- batches ---
static const int kMaxTeam = 64;  // workgroups per team (sx_batch_config)

static sx_status team_workspaces(sx_ctx *ctx, int nteams, int n, long long m) {
  if ((int)ctx->team_work.size() >= nteams && ctx->team_n >= n && ctx->team_m >= m) return SX_OK;
  for (void *p : ctx->team_allocs) (void)hipFree(p);
  ctx->team_allocs.clear();
  ctx->team_work.clear();
  n = std::max(n, ctx->team_n);
  m = std::max(m, ctx->team_m);
  auto al = [&](void **p, size_t bytes) -> sx_status {
    hipError_t e = hipMalloc(p, bytes ? bytes : 256);
    if (e != hipSuccess) return fail(SX_ENOMEM, "team workspace: %s", hipGetErrorString(e));
    ctx->team_allocs.push_back(*p);
    return SX_OK;
  };
  for (int t = 0; t < nteams; ++t) {
    Work w;
    // teams have at most kMaxTeam workgroups; directed graphs of the batch
    // only push / pull (no k-core), so `arcs` is m
    sx_status r = work_alloc(al, n, m, false, kMaxTeam, false, w);
    if (r != SX_OK) return r;
    HIP_TRY(hipMemset(w.ctrl, 0, sizeof(Ctrl)));
    ctx->team_work.push_back(w);
  }
  ctx->team_n = n;
  ctx->team_m = m;
  return SX_OK;
}

static sx_status validate_queries(sx_ctx *ctx, const sx_query *q, int32_t nq, int *nmax,
                                  long long *mmax) {
  if (!ctx || (nq > 0 && !q) || nq < 0) return fail(SX_EINVAL, "bad batch arguments");
  *nmax = 0;
  *mmax = 0;
  for (int i = 0; i < nq; ++i) {
    const sx_graph *g = q[i].g;
    if (!g || !q[i].d_out) return fail(SX_EINVAL, "query %d: NULL graph or output", i);
    if (g->ctx != ctx) return fail(SX_EINVAL, "query %d: graph of another context", i);
    if (q[i].algo != SX_BFS && q[i].algo != SX_SSSP) return fail(SX_EINVAL, "query %d: BFS or SSSP only", i);
    if (q[i].source < 0 || q[i].source >= g->g.n) return fail(SX_EINVAL, "query %d: source out of range", i);
    if (q[i].algo == SX_SSSP && !g->weighted) return fail(SX_EINVAL, "query %d: SSSP needs weights", i);
    if (g->reordered) return fail(SX_EUNSUPPORTED, "query %d: renumbered graph (SX_REORDER) in a batch", i);
    *nmax = std::max(*nmax, g->g.n);
    *mmax = std::max(*mmax, g->g.m);
  }
  return SX_OK;
}

extern "C" sx_status sx_run_batch(sx_ctx *ctx, const sx_query *q, int32_t nq, const sx_policy *pol,
                                  const sx_batch_config *cfg, void *hip_stream,
                                  sx_run_stats *per_query, double *batch_ms) {
  int nmax;
  long long mmax;
  sx_status s = validate_queries(ctx, q, nq, &nmax, &mmax);
  if (s != SX_OK) return s;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)hip_stream;
  if (nq == 0) {
    if (batch_ms) *batch_ms = 0.0;
    return SX_OK;
  }
  sx_batch_config c{4, 0, 0};
  if (cfg) c = *cfg;
  else if (ctx->tuned.team_wgs > 0) c = ctx->tuned;
  int per = 0;
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_kernel(), kBlock, 0));
  const int grid = std::max(1, std::min(per * ctx->cus, kMaxGrid));
  if (c.team_wgs < 1 || c.team_wgs > kMaxTeam) return fail(SX_EINVAL, "team_wgs must be in 1..%d", kMaxTeam);
  const int team = std::min(c.team_wgs, grid);
  const int nteams = grid / team;
  s = team_workspaces(ctx, nteams, nmax, mmax);
  if (s != SX_OK) return s;
  // programme-level parameters as for a single run
  sx_program prog;
  memset(&prog, 0, sizeof prog);
  prog.ctx = ctx;
  prog.ap.algo = SX_BFS;
  if (pol) prog.pol = *pol;
  if (c.bin_small > 0) prog.pol.bin_small = c.bin_small;
  if (c.bin_large > 0) prog.pol.bin_large = c.bin_large;
  if (prog.pol.policy == SX_POLICY_LEARNED && !ctx->d_mlp)
    return fail(SX_ESTATE, "learned policy requested but no MLP loaded");
  BatchArgs b;
  memset(&b, 0, sizeof b);
  b.P = make_params(&prog, nullptr, team);
  b.mlp = ctx->d_mlp;
  b.nq = nq;
  b.nteams = nteams;
  b.team = team;
  // device-side query table, order (largest expected time first), stats
  std::vector<BatchQuery> hq((size_t)nq);
  std::vector<std::pair<double, int>> key((size_t)nq);
  for (int i = 0; i < nq; ++i) {
    const DevGraph &g = q[i].g->g;
    hq[i].g = g;
    hq[i].state = (int *)q[i].d_out;
    hq[i].algo = q[i].algo == SX_SSSP ? 1 : 0;
    hq[i].src = q[i].source;
    hq[i].mu0 = 0;
    const double avg = g.n ? (double)g.m / g.n : 0.0;
    // low average degree: a mesh-like, high-diameter graph whose run time
    // grows with sqrt(n) levels; otherwise with the arcs
    const double est = avg < 6.0 ? 2e3 * std::sqrt((double)g.n) : (double)g.m;
    key[i] = {-(est * (hq[i].algo ? 2.0 : 1.0)), i};
  }
  std::sort(key.begin(), key.end());
  std::vector<int> order((size_t)nq);
  for (int i = 0; i < nq; ++i) order[i] = key[i].second;
  // device tables kept in the context and grown on demand, so a repeated
  // batch allocates nothing
  if (nq > ctx->batch_cap_q || nteams > ctx->batch_cap_t || !ctx->bh) {
    for (void **pp : {&ctx->bq, &ctx->bo, &ctx->bw, &ctx->bh, &ctx->bs}) {
      if (*pp) (void)hipFree(*pp);
      *pp = nullptr;
    }
    ctx->batch_cap_q = ctx->batch_cap_t = 0;
    const int cq = std::max(nq, 256), ct = std::max(nteams, kMaxGrid);
    HIP_TRY(hipMalloc(&ctx->bq, sizeof(BatchQuery) * cq));
    HIP_TRY(hipMalloc(&ctx->bo, sizeof(int) * cq));
    HIP_TRY(hipMalloc(&ctx->bw, sizeof(Work) * ct));
    HIP_TRY(hipMalloc(&ctx->bh, 256));
    HIP_TRY(hipMalloc(&ctx->bs, sizeof(BatchStat) * cq));
    ctx->batch_cap_q = cq;
    ctx->batch_cap_t = ct;
  }
  if (!ctx->be0) HIP_TRY(hipEventCreate(&ctx->be0));
  if (!ctx->be1) HIP_TRY(hipEventCreate(&ctx->be1));
  HIP_TRY(hipMemcpyAsync(ctx->bq, hq.data(), sizeof(BatchQuery) * nq, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(ctx->bo, order.data(), sizeof(int) * nq, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(ctx->bw, ctx->team_work.data(), sizeof(Work) * nteams, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemsetAsync(ctx->bs, 0, sizeof(BatchStat) * nq, st));
  b.q = (const BatchQuery *)ctx->bq;
  b.order = (const int *)ctx->bo;
  b.work = (const Work *)ctx->bw;
  b.queue_head = (unsigned *)ctx->bh;
  b.stats = (BatchStat *)ctx->bs;
  hipEvent_t e0 = ctx->be0, e1 = ctx->be1;
  HIP_TRY(hipEventRecord(e0, st));
  HIP_TRY(batch_launch(b, grid, st));
  HIP_TRY(hipEventRecord(e1, st));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  std::vector<BatchStat> hs((size_t)nq);
  HIP_TRY(hipMemcpy(hs.data(), ctx->bs, sizeof(BatchStat) * nq, hipMemcpyDeviceToHost));
  // team errors (watchdog) and per-query completion
  for (int t = 0; t < nteams; ++t) {
    unsigned err = 0;
    HIP_TRY(hipMemcpy(&err, &ctx->team_work[t].ctrl->error.v[0], 4, hipMemcpyDeviceToHost));
    if (err == SX_ERR_DEADLOCK) return fail(SX_EDEADLOCK, "team %d barrier watchdog fired", t);
    if (err == SX_ERR_OVERFLOW) return fail(SX_EOVERFLOW, "distance overflow in team %d", t);
    if (err == SX_ERR_CAPACITY) return fail(SX_EHIP, "team %d: scanned worklist exceeded its regions", t);
    if (err) return fail(SX_EHIP, "team %d device error %u", t, err);
  }
  for (int i = 0; i < nq; ++i)
    if (hs[i].status != EXIT_DONE) return fail(SX_EHIP, "query %d did not finish (status %d)", i, hs[i].status);
  if (per_query)
    for (int i = 0; i < nq; ++i) {
      memset(&per_query[i], 0, sizeof per_query[i]);
      per_query[i].iterations = hs[i].iterations;
      per_query[i].launches = 1;
      per_query[i].pull_iters = hs[i].pull_iters;
      per_query[i].ballot_iters = hs[i].ballot_iters;
      per_query[i].edges_inspected = (int64_t)hs[i].edges;
      per_query[i].vertex_expansions = (int64_t)hs[i].expansions;
      per_query[i].device_ms = ms;
    }
  if (batch_ms) *batch_ms = ms;
  return SX_OK;
}

extern "C" sx_status sx_batch_autotune(sx_ctx *ctx, const sx_query *q, int32_t nq, const sx_policy *pol,
                                       void *hip_stream, sx_batch_config *best, double *best_ms) {
  if (!best) return fail(SX_EINVAL, "NULL argument");
  const int teams[] = {1, 2, 4, 8, 16, 32};
  const int bins[][2] = {{64, 256}, {32, 1024}};
  double bms = 1e300;
  sx_batch_config bc{4, 0, 0};
  for (int t : teams)
    for (auto &bb : bins) {
      sx_batch_config c{t, bb[0], bb[1]};
      double ms = 0.0;
      sx_status s = sx_run_batch(ctx, q, nq, pol, &c, hip_stream, nullptr, &ms);
      if (s != SX_OK) return s;
      if (ms < bms) { bms = ms; bc = c; }
    }
  ctx->tuned = bc;
  *best = bc;
  if (best_ms) *best_ms = bms;
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
  // a renumbered graph runs on its own state array and maps the result back
  void *state = G->reordered ? G->state : d_out;
  sx_status s;
  switch (p->ap.algo) {
    case SX_BFS:
    case SX_SSSP:
      if (n == 0) return fail(SX_EINVAL, "empty graph has no source");
      if (source < 0 || source >= n) return fail(SX_EINVAL, "source %d out of range [0, %d)", source, n);
      if (p->ap.algo == SX_SSSP && !G->weighted) return fail(SX_EINVAL, "SSSP needs edge weights");
      s = run_traversal(p, G, G->reordered ? G->h_inv[(size_t)source] : source, state, st, stats);
      break;
    case SX_KCORE:
      s = run_kcore(p, G, state, st, stats);
      break;
    case SX_WCC:
      if (G->directed) return fail(SX_EUNSUPPORTED, "WCC on a directed graph");
      if (n == 0) {
        if (stats) memset(stats, 0, sizeof *stats);
        return SX_OK;
      }
      s = run_traversal(p, G, 0, state, st, stats);
      break;
    case SX_PAGERANK:
      s = run_pagerank(p, G, state, st, stats);
      break;
    case SX_BP:
      if (G->directed) return fail(SX_EUNSUPPORTED, "belief propagation on a directed graph");
      // the priors arrive in d_out, in the caller's numbering
      if (G->reordered && n > 0) HIP_TRY(reorder_permute(d_out, G->d_inv, G->state, n, st));
      s = run_bp(p, G, state, st, stats);
      break;
    default:
      return fail(SX_EINVAL, "unknown algorithm");
  }
  if (s != SX_OK || !G->reordered) return s;
  HIP_TRY(hipEventRecord(G->ev0, st));
  HIP_TRY(reorder_unpermute(G->state, G->d_inv, d_out, n, st));
  HIP_TRY(hipEventRecord(G->ev1, st));
  HIP_TRY(hipEventSynchronize(G->ev1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, G->ev0, G->ev1));
  if (stats) stats->device_ms += ms;
  return SX_OK;
}

// BFS / SSSP / WCC on a graph the caller holds in device memory, with the
// engine's workspace carved from the static array instead of allocated: the
// same kernels and host loop as sx_run on a graph loaded with
// SX_DEVICE_PTRS.  Nothing here allocates; the context's pinned mirrors and
// events were made by sx_ctx_create.
extern "C" sx_status sx_run_static(sx_program *p, const sx_graph_desc *d, int32_t source,
                                   void *d_out, void *hip_stream, sx_run_stats *stats) {
  if (!p || !d || !d_out) return fail(SX_EINVAL, "NULL argument");
  sx_ctx *ctx = p->ctx;
  if (!ctx->d_static) return fail(SX_ESTATE, "static workspace not set up");
  const int algo = p->ap.algo;
  if (algo != SX_BFS && algo != SX_SSSP && algo != SX_WCC)
    return fail(SX_EUNSUPPORTED, "sx_run_static runs BFS, SSSP or WCC only");
  if (p->pol.fused == SX_UNFUSED)
    return fail(SX_EUNSUPPORTED, "sx_run_static: the one-phase arrangement keeps host buffers");
  if (!(d->flags & SX_DEVICE_PTRS)) return fail(SX_EINVAL, "sx_run_static needs SX_DEVICE_PTRS");
  if (d->flags & SX_REORDER) return fail(SX_EUNSUPPORTED, "sx_run_static: no renumbering (SX_REORDER)");
  const bool undirected = (d->flags & SX_UNDIRECTED) != 0;
  if (d->n < 0) return fail(SX_EINVAL, "n < 0");
  if (d->m < 0 || d->m >= (int64_t)INT32_MAX) return fail(SX_EINVAL, "m = %lld out of range", (long long)d->m);
  if (!d->offsets || (d->m > 0 && !d->indices)) return fail(SX_EINVAL, "missing CSR arrays");
  if (undirected && (d->in_offsets || d->in_indices))
    return fail(SX_EINVAL, "undirected graph with in-neighbour arrays");
  if (!undirected && (!d->in_offsets || (d->m > 0 && !d->in_indices)))
    return fail(SX_EINVAL, "directed graph needs in_offsets / in_indices (CSC)");
  if (!undirected && d->weights && !d->in_weights)
    return fail(SX_EINVAL, "directed weighted graph needs in_weights");
  if (algo == SX_WCC && !undirected) return fail(SX_EUNSUPPORTED, "WCC on a directed graph");
  if (algo == SX_WCC && d->n == 0) {
    if (stats) memset(stats, 0, sizeof *stats);
    return SX_OK;
  }
  if (algo != SX_WCC) {
    if (d->n == 0) return fail(SX_EINVAL, "empty graph has no source");
    if (source < 0 || source >= d->n) return fail(SX_EINVAL, "source %d out of range [0, %d)", source, d->n);
    if (algo == SX_SSSP && !d->weights && d->m > 0) return fail(SX_EINVAL, "SSSP needs edge weights");
  }
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)hip_stream;
  // a graph object on the stack that borrows everything
  sx_graph G;
  G.ctx = ctx;
  DevGraph &g = G.g;
  g.n = d->n;
  g.m = d->m;
  g.directed = !undirected;
  g.off = d->offsets;
  g.idx = d->indices;
  g.w = d->weights;
  g.in_off = undirected ? d->offsets : d->in_offsets;
  g.in_idx = undirected ? d->indices : d->in_indices;
  g.in_w = undirected ? d->weights : d->in_weights;
  G.weighted = d->weights != nullptr || d->m == 0;
  G.directed = !undirected;
  G.h_ctrl = ctx->hs_ctrl[0];
  G.h_ctrl2 = ctx->hs_ctrl[1];
  G.ev0 = ctx->sev[0];
  G.ev1 = ctx->sev[1];
  G.evb[0] = ctx->sev[2];
  G.evb[1] = ctx->sev[3];
  // workspace laid out for the run's grid (not for the largest grid, as a
  // loaded graph's is), bump-allocated in 256-byte steps
  const int grid = traversal_grid(p, &G, 0);
  size_t used = 0;
  auto carve = [&](void **ptr, size_t bytes) -> sx_status {
    const size_t b = (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
    if (used + b > kStaticScratchBytes) {
      *ptr = nullptr;
      used += b;
      return SX_OK;  // keep counting: the total is reported below
    }
    *ptr = ctx->d_static + used;
    used += b;
    return SX_OK;
  };
  sx_status s = work_alloc(carve, d->n, d->m, !undirected, grid, false, G.w);
  if (s != SX_OK) return s;
  s = carve((void **)&G.d_xdist, sizeof(unsigned) * xrec_entries(d->n, d->m));
  if (s != SX_OK) return s;
  if (used > kStaticScratchBytes)
    return fail(SX_EINVAL,
                "sx_run_static: the graph needs %zu bytes of workspace at a grid of %d workgroups; the "
                "static workspace holds %zu",
                used, grid, kStaticScratchBytes);
  const unsigned long long words = sizeof(Ctrl) / 4;
  hipLaunchKernelGGL(k_static_clear, dim3(64), dim3(256), 0, st, (unsigned *)G.w.ctrl, words);
  HIP_TRY(hipGetLastError());
  return run_traversal(p, &G, source, d_out, st, stats);
}

extern "C" sx_status sx_run_iterations(sx_program *p, const sx_graph *gc, int32_t source,
                                       void *d_out, void *hip_stream, int32_t iterations,
                                       sx_run_stats *stats) {
  if (!p || !gc || !d_out) return fail(SX_EINVAL, "NULL argument");
  if (iterations < 1) return fail(SX_EINVAL, "iterations must be positive");
  sx_graph *G = const_cast<sx_graph *>(gc);
  if (G->ctx != p->ctx) return fail(SX_EINVAL, "graph and program belong to different contexts");
  if (p->ap.algo != SX_BFS && p->ap.algo != SX_SSSP && p->ap.algo != SX_WCC)
    return fail(SX_EINVAL, "BFS, SSSP or WCC only");
  if (G->reordered) return fail(SX_EUNSUPPORTED, "renumbered graph (SX_REORDER)");
  const int n = G->g.n;
  if (p->ap.algo == SX_WCC) {
    if (G->directed) return fail(SX_EUNSUPPORTED, "WCC on a directed graph");
    source = 0;
  }
  if (n == 0 || source < 0 || source >= n) return fail(SX_EINVAL, "source out of range");
  if (p->ap.algo == SX_SSSP && !G->weighted) return fail(SX_EINVAL, "SSSP needs edge weights");
  HIP_TRY(hipSetDevice(p->ctx->device));
  return run_traversal(p, G, source, d_out, (hipStream_t)hip_stream, stats, iterations);
}

extern "C" sx_status sx_frontier_get(const sx_graph *g, int32_t *vertices, int32_t *bins, int32_t cap,
                                     int32_t *count, int32_t *from_ballot, uint64_t *words,
                                     int64_t nwords, void *hip_stream) {
  if (!g || !count || (cap > 0 && (!vertices || !bins)) || cap < 0 || nwords < 0 ||
      (nwords > 0 && !words))
    return fail(SX_EINVAL, "bad argument");
  if (g->next_slot < 0) return fail(SX_ESTATE, "no push list: call sx_run_iterations first");
  hipStream_t st = (hipStream_t)hip_stream;
  HIP_TRY(hipSetDevice(g->ctx->device));
  const Work &w = g->w;
  const int G = g->next_grid, par = g->next_parity;
  std::vector<RecSlot> rec(1);
  HIP_TRY(hipMemcpyAsync(rec.data(), w.rec + g->next_slot, sizeof(RecSlot), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const unsigned caps[NBINS] = {w.tot_s / (unsigned)G, w.tot_m / (unsigned)G, w.tot_l / (unsigned)G};
  int32_t k = 0;
  for (int b = 0; b < NBINS; ++b) {
    for (int r = 0; r < G; ++r) {
      const unsigned c = std::min(rec[0].cnt[b][r], caps[b]);
      if (!c) continue;
      if (b < BIN_LARGE) {
        std::vector<int> h(c);
        const int *src = (b == BIN_SMALL ? w.reg_s[par] : w.reg_m[par]) + (size_t)r * caps[b];
        HIP_TRY(hipMemcpy(h.data(), src, sizeof(int) * c, hipMemcpyDeviceToHost));
        for (unsigned i = 0; i < c; ++i) {
          if (k < cap) { vertices[k] = h[i]; bins[k] = b; }
          ++k;
        }
      } else {
        std::vector<unsigned long long> h(c);
        HIP_TRY(hipMemcpy(h.data(), w.reg_l[par] + (size_t)r * caps[b], sizeof(unsigned long long) * c,
                          hipMemcpyDeviceToHost));
        for (unsigned i = 0; i < c; ++i) {
          if ((h[i] >> 32) != 0) continue;   // one entry per vertex: its first chunk
          if (k < cap) { vertices[k] = (int32_t)(h[i] & 0xffffffffu); bins[k] = b; }
          ++k;
        }
      }
    }
  }
  *count = k;
  if (from_ballot) *from_ballot = g->next_slot == SLOT_SCAN ? 1 : 0;
  if (nwords > 0) {
    const int64_t have = ((int64_t)g->g.n + 63) / 64;
    const int64_t nw = std::min(nwords, have);
    std::vector<unsigned long long> acc((size_t)nw, 0ull), h((size_t)nw);
    for (int b = 0; b < NBINS; ++b) {
      HIP_TRY(hipMemcpy(h.data(), w.bits[b], sizeof(unsigned long long) * nw, hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < nw; ++i) acc[i] |= h[i];
    }
    for (int64_t i = 0; i < nwords; ++i) words[i] = i < nw ? acc[i] : 0ull;
  }
  return SX_OK;
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
  struct Named { const char *name; const void *k; bool persistent; int block = kBlock; };
  const Named table[] = {
      {"bfs_fused", trav_kernel(TK_FUSED, ALG_BFS), true},
      {"sssp_fused", trav_kernel(TK_FUSED, ALG_SSSP), true},
      {"wcc_fused", trav_kernel(TK_FUSED, ALG_WCC), true},
      {"bfs_fused_pull", trav_kernel(TK_FUSED_PULL, ALG_BFS), true},
      {"sssp_fused_pull", trav_kernel(TK_FUSED_PULL, ALG_SSSP), true},
      {"wcc_fused_pull", trav_kernel(TK_FUSED_PULL, ALG_WCC), true},
      {"bfs_fused_all", trav_kernel(TK_FUSED_ALL, ALG_BFS), true},
      {"sssp_fused_all", trav_kernel(TK_FUSED_ALL, ALG_SSSP), true},
      {"wcc_fused_all", trav_kernel(TK_FUSED_ALL, ALG_WCC), true},
      {"wcc_seq", trav_kernel(TK_SEQ, ALG_WCC), false},
      {"wcc_seq_wide", trav_kernel(TK_SEQ_WIDE, ALG_WCC), false},
      {"bfs_seq", trav_kernel(TK_SEQ, 0), false},
      {"sssp_seq", trav_kernel(TK_SEQ, 1), false},
      {"bfs_seq_wide", trav_kernel(TK_SEQ_WIDE, 0), false},
      {"sssp_seq_wide", trav_kernel(TK_SEQ_WIDE, 1), false},
      {"bfs_push_step", trav_kernel(TK_PUSH_STEP, 0), false},
      {"bfs_pull_step", trav_kernel(TK_PULL_STEP, 0), false},
      {"sssp_push_step", trav_kernel(TK_PUSH_STEP, 1), false},
      {"sssp_pull_step", trav_kernel(TK_PULL_STEP, 1), false},
      {"ballot_scan", trav_kernel(TK_BALLOT, 0), false},
      {"pull_scan", trav_kernel(TK_PULL_SCAN, 0), false},
      {"kcore_fused", kcore_kernel(), true},
      {"kcore_tail", kcore_tail_kernel(), false, kTailThreads},
      {"kcore_seq", kcore_seq_kernel(), false},
      {"pagerank_fused", pagerank_kernel(), true},
      {"pagerank_until_stable", pagerank_kernel(true), true},
      {"pagerank_push_tail", pagerank_push_kernel(), true},
      {"bp_fused", bp_kernel(), true},
      {"batch", batch_kernel(), true},
  };
  for (const Named &t : table) {
    if (strcmp(t.name, name) != 0) continue;
    hipFuncAttributes fa;
    HIP_TRY(hipFuncGetAttributes(&fa, t.k));
    out->vgprs = fa.numRegs;
    out->sgprs = 0;
    out->lds_bytes = (int32_t)fa.sharedSizeBytes;
    out->block = t.block;
    int per = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, t.k, t.block, 0));
    out->wgs_per_cu = per;
    out->cus = ctx->cus;
    // the k-core tail runs one workgroup
    out->grid_wgs = t.block == kBlock ? std::min(per * ctx->cus, kMaxGrid) : 1;
    return SX_OK;
  }
  return fail(SX_EINVAL, "unknown kernel name '%s'", name);
}
