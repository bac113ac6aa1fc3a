// PageRank as an ACC program (Section 6, "PageRank": pull from the in-
// neighbours with a sum as the merge operation), in FP32 for a fixed number
// of synchronous iterations:
//   x_0(v)     = 1/n
//   x_{t+1}(v) = (1-d)/n + d * ( sum_{u->v} x_t(u)/outdeg(u) + D_t/n ),
//   D_t        = sum of x_t over vertices without out-arcs.
//
//   Active   every vertex, every iteration.
//   Compute  contribution x_t(u) / outdeg(u), stored per vertex once per
//            iteration so that each arc costs one gather.
//   Combine  sum over the in-arcs (aggregation), single writer per vertex.
//
// Task management: all vertices are active, so the binned lists are built by
// one ballot-filter pass before the first iteration (the paper observes
// PageRank needs the ballot filter exactly once) and reused.  Every sum --
// per vertex over its in-arcs, and the dangling mass over vertices -- is a
// compensated (TwoSum) FP32 summation in a fixed order, so the result is
// reproducible bit for bit and its error stays near the rounding of the
// stored FP32 values.  One persistent launch runs all iterations with one
// global barrier each.
#include "sx_frontier.hpp"
#include "sx_kernels.hpp"

namespace sx {


struct LdsPr {
  LdsView view;
  LdsBallot ball;
  long long red[kWaves];
  float f[2 * kWaves];
};

// Dangling mass D_t from the per-workgroup partials of iteration t.
SX_DEV float dangling_total(const float *part, int nparts, float *lds) {
  CSum a{0.f, 0.f};
  for (int i = threadIdx.x; i < nparts; i += kBlock) a = cmerge(a, CSum{part[2 * i], part[2 * i + 1]});
  a = wg_merge(a, lds);
  return a.s + a.c;
}

// Binned vertex lists (by in-degree, one item per vertex), built once by the
// ballot filter into slot SLOT_SCAN, parity 0.
SX_DEV void pr_lists(const PrArgs &a, LdsPr &lds) {
  const int *io = a.g.in_off;
  auto pred = [](int v) { (void)v; return true; };
  auto deg = [&](int v) { return io[v + 1] - io[v]; };
  auto ident = [](int i) { return i; };
  const VGrid vg = hw_grid();
  ballot_fill(vg, a.g.n, pred, deg, ident, a.P, 0x7fffffff, a.w.bits, regions(a.w, 0, vg.nb),
              a.w.rec + SLOT_SCAN, lds.ball);
}

// One vertex's new value from its in-arc sum; returns the dangling share.
SX_DEV void pr_finish_vertex(const PrArgs &a, int v, CSum s, float D, bool last, float *dst,
                             CSum &dang) {
  const float d = a.P.pr_d;
  const float r = a.base_teleport + d * ((s.s + s.c) + D * a.inv_n);
  const int od = a.g.off[v + 1] - a.g.off[v];
  if (last) a.rank[v] = r;
  else if (od > 0) dst[v] = r / (float)od;
  if (od == 0) cadd(dang, r);
}

// s += src[ii[e]] for e = e0, e0 + stride, ... < end, in that order.  The
// indices and contributions of kIlp consecutive terms are loaded before any
// of them is added, so a lane has kIlp gathers in flight instead of one; the
// additions keep their order, so the sum is the same bits.
SX_DEV void gather(CSum &s, const float *src, const int *ii, int e0, int end, int stride,
                   long long &edges) {
  int e = e0;
  for (; e + (kIlp - 1) * stride < end; e += kIlp * stride) {
    int u[kIlp];
    float x[kIlp];
#pragma unroll
    for (int r = 0; r < kIlp; ++r) u[r] = ii[e + r * stride];
#pragma unroll
    for (int r = 0; r < kIlp; ++r) x[r] = src[u[r]];
#pragma unroll
    for (int r = 0; r < kIlp; ++r) cadd(s, x[r]);
    edges += kIlp;
  }
  for (; e < end; e += stride) {
    cadd(s, src[ii[e]]);
    ++edges;
  }
}

SX_DEV void pr_iteration(const PrArgs &a, int t, const ViewRef &L, const Totals &T, LdsPr &lds) {
  const Work &w = a.w;
  const float *src = w.contrib[t & 1];
  float *dst = w.contrib[(t + 1) & 1];
  const float D = dangling_total(w.dang + (size_t)(t & 1) * 2 * kMaxGrid, gridDim.x, lds.f);
  const bool last = t == a.iters - 1;
  const int *io = a.g.in_off, *ii = a.g.in_idx;
  const int lane = lane_id();
  CSum dang{0.f, 0.f};
  long long edges = 0;
  // one workgroup per large vertex
  for (unsigned i = blockIdx.x; i < T.cnt[BIN_LARGE]; i += gridDim.x) {
    const int v = (int)(L.large(i) & 0xffffffffu);
    if ((unsigned)v >= (unsigned)a.g.n) continue;
    const int beg = io[v], end = io[v + 1];
    CSum s{0.f, 0.f};
    gather(s, src, ii, beg + (int)threadIdx.x, end, kBlock, edges);
    s = wg_merge(s, lds.f);
    if (threadIdx.x == 0) pr_finish_vertex(a, v, s, D, last, dst, dang);
  }
  const unsigned gw = blockIdx.x * kWaves + wave_in_wg();
  const unsigned nw = gridDim.x * kWaves;
  // one wavefront per medium vertex
  for (unsigned i = gw; i < T.cnt[BIN_MED]; i += nw) {
    const int v = L.med(i);
    if ((unsigned)v >= (unsigned)a.g.n) continue;
    const int beg = io[v], end = io[v + 1];
    CSum s{0.f, 0.f};
    gather(s, src, ii, beg + lane, end, 64, edges);
    s = wave_merge(s);
    if (lane == 0) pr_finish_vertex(a, v, s, D, last, dst, dang);
  }
  // one lane per small vertex
  for (unsigned i = gw * 64u + lane; i < T.cnt[BIN_SMALL]; i += nw * 64u) {
    const int v = L.small(i);
    if ((unsigned)v >= (unsigned)a.g.n) continue;
    const int beg = io[v], end = io[v + 1];
    CSum s{0.f, 0.f};
    gather(s, src, ii, beg, end, 1, edges);
    pr_finish_vertex(a, v, s, D, last, dst, dang);
  }
  dang = wg_merge(dang, lds.f);
  if (threadIdx.x == 0) {
    float *part = w.dang + (size_t)((t + 1) & 1) * 2 * kMaxGrid;
    part[2 * blockIdx.x] = dang.s;
    part[2 * blockIdx.x + 1] = dang.c;
  }
  add_stats(w.ctrl, blockIdx.x, edges, 0ull, lds.red);
}

__global__ void __launch_bounds__(kBlock) k_pr_fused(PrArgs a) {
  __shared__ LdsPr lds;
  Ctrl *C = a.w.ctrl;
  const VGrid vg = hw_grid();
  GridBarrier bar(C, load_relaxed(&C->bar_gen.v[0]), a.P.watchdog);
  pr_lists(a, lds);
  if (!bar.sync()) return;
  ViewRef L;
  L.V = &lds.view;
  L.R = regions(a.w, 0, vg.nb);
  L.G = vg.nb;
  const Totals T = view_build(a.w.rec + SLOT_SCAN, vg.nb, L.R, lds.view, lds.red);
  if (T.ovf) {
    if (threadIdx.x == 0) store_relaxed(&C->error.v[0], (unsigned)SX_ERR_CAPACITY);
    return;
  }
  for (int t = 0; t < a.iters; ++t) {
    pr_iteration(a, t, L, T, lds);
    if (!bar.sync()) return;
  }
  if (vg.bid == 0 && threadIdx.x == 0) {
    store_relaxed(&C->state.v[0], (unsigned)EXIT_DONE);
    store_relaxed(&C->stats.v[6], (unsigned)a.iters);
    store_relaxed(&C->stats.v[4], 1u);
    atomic_add_u64((unsigned long long *)&C->statw[0].v[2],
                   (unsigned long long)a.iters * ((unsigned long long)T.cnt[0] + T.cnt[1] + T.cnt[2]));
  }
}

// x_0 = 1/n: contributions and the dangling partials of iteration 0 (same
// grid as the persistent kernel, so partial i belongs to workgroup i).
__global__ void __launch_bounds__(kBlock) k_pr_init(PrArgs a) {
  __shared__ float lf[2 * kWaves];
  const int n = a.g.n;
  CSum dang{0.f, 0.f};
  for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < n;
       v += (long long)gridDim.x * kBlock) {
    const int od = a.g.off[v + 1] - a.g.off[v];
    if (od > 0) a.w.contrib[0][v] = a.inv_n / (float)od;
    else cadd(dang, a.inv_n);
  }
  dang = wg_merge(dang, lf);
  if (threadIdx.x == 0) {
    a.w.dang[2 * blockIdx.x] = dang.s;
    a.w.dang[2 * blockIdx.x + 1] = dang.c;
  }
  if (blockIdx.x == 0) reset_barrier(a.w.ctrl);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Ctrl *C = a.w.ctrl;
    for (int i = 0; i < 32; ++i) { C->state.v[i] = 0; C->stats.v[i] = 0; }
    C->error.v[0] = 0;
  }
  if (blockIdx.x == 1 || gridDim.x == 1)
    reset_stat_lines(a.w.ctrl);
}

hipError_t pagerank_launch(const PrArgs &a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_pr_init, dim3(grid), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_pr_fused, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

const void *pagerank_kernel() { return (const void *)k_pr_fused; }

}  // namespace sx
