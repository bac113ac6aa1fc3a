// Belief propagation as an ACC program (Section 6, "Belief propagation":
// sum-product message passing on a Markov random field, with the vertex's
// probability as its metadata; Section 3.2: every vertex active in every
// iteration, the updates of its neighbours summed), in FP32 for a fixed
// number of synchronous iterations over a binary pairwise MRF.
//
// The model: vertex v has the prior phi_v(1) = p_v; the edge {u, v} has the
// potential psi(x, y) = s_uv if x == y else 1 - s_uv with
//   s_uv = (1 + c_uv) / 2,   c_uv = kappa * theta_uv / max(deg u, deg v),
//   theta_uv = (((w_uv - 1) mod 64) - 31.5) / 31.5  (1 on an unweighted graph).
// With q = 2 b - 1, the message of u to v has the ratio
//   m_{u->v}(1) / m_{u->v}(0) = (1 + c_uv q_u) / (1 - c_uv q_u) = exp(2 atanh(c_uv q_u)),
// so one sum-product iteration is, in the logit / 2 of the belief,
//   x_v = atanh(2 p_v - 1) + sum_{u in N(v)} atanh(c_uv q_u),   q_v' = tanh(x_v),
// and the belief is b_v = 1 / (1 + exp(-2 x_v)).
//
//   Active   every vertex, every iteration.
//   Compute  atanh(c_uv q_u) from the neighbour's (q_u, deg u), stored per
//            vertex once per iteration (one 8-byte gather per arc) and the
//            arc's weight (read with the neighbour id, coalesced).
//   Combine  sum over the neighbours (aggregation), single writer per
//            vertex, compensated FP32 in a fixed order.
//
// Task management as for PageRank: the binned vertex lists come from one
// ballot-filter pass before the first iteration (Section 4: BP needs the
// ballot filter exactly once) and are reused; one persistent launch runs all
// iterations, with one global barrier each (Section 5).
#include "sx_frontier.hpp"
#include "sx_kernels.hpp"

namespace sx {

struct LdsBp {
  LdsView view;
  LdsBallot ball;
  long long red[kWaves];
  float f[2 * kWaves];
};

// Coupling sign and strength of an arc from its weight (weights 1..64 span
// -1..1; an unweighted graph couples every edge with theta = 1).
SX_DEV float bp_theta(const unsigned *w, long long e) {
  return w ? ((float)((w[e] - 1u) & 63u) - 31.5f) / 31.5f : 1.f;
}

// (q, deg) of the first kHotBp vertices, copied into LDS by every workgroup
// at the start of each iteration: after the degree-ordered renumbering they
// are the highest-degree neighbours, and a gather served by LDS is one
// request fewer at the L2 (the pull's bound, as for PageRank).
constexpr int kHotBp = 4096;

// s += atanh(c_uv q_u) over the arcs e = e0, e0 + stride, ... < end of
// vertex v (degree dv), kIlp arcs in flight per lane, added in order (an
// index below nhot reads the LDS copy hot).
SX_DEV void bp_gather(CSum &s, const BpArgs &a, const float2 *src, float dv, long long e0, long long end,
                      int stride, long long &edges, const float2 *hot, int nhot) {
  const int *ii = a.g.idx;
  const unsigned *ww = a.g.w;
  long long e = e0;
  for (; e + (long long)(kIlp - 1) * stride < end; e += (long long)kIlp * stride) {
    int u[kIlp];
    float th[kIlp];
    float2 su[kIlp];
#pragma unroll
    for (int r = 0; r < kIlp; ++r) {
      u[r] = ii[e + r * stride];
      th[r] = bp_theta(ww, e + r * stride);
    }
#pragma unroll
    for (int r = 0; r < kIlp; ++r) su[r] = u[r] < nhot ? hot[u[r]] : src[u[r]];
#pragma unroll
    for (int r = 0; r < kIlp; ++r) cadd(s, atanhf(a.kappa * th[r] / fmaxf(su[r].y, dv) * su[r].x));
    edges += kIlp;
  }
  for (; e < end; e += stride) {
    const int uu = ii[e];
    const float2 su = uu < nhot ? hot[uu] : src[uu];
    cadd(s, atanhf(a.kappa * bp_theta(ww, e) / fmaxf(su.y, dv) * su.x));
    ++edges;
  }
}

// One vertex's new state from its neighbour sum: (q, deg) for the next
// iteration, or the belief after the last one.
SX_DEV void bp_finish_vertex(const BpArgs &a, int v, CSum s, float dv, bool last, float2 *dst) {
  const float x = a.w.bph[v] + (s.s + s.c);
  if (last) a.belief[v] = 1.f / (1.f + expf(-2.f * x));
  else dst[v] = make_float2(tanhf(x), dv);
}

SX_DEV void bp_iteration(const BpArgs &a, int t, const ViewRef &L, const Totals &T, LdsBp &lds,
                         float2 *hot) {
  const float2 *src = a.w.bpq[t & 1];
  const int nhot = a.g.n < kHotBp ? a.g.n : kHotBp;
  for (int i = threadIdx.x; i < nhot; i += kBlock) hot[i] = src[i];
  __syncthreads();
  float2 *dst = a.w.bpq[(t + 1) & 1];
  const bool last = t == a.iters - 1;
  const int *off = a.g.off;
  const int lane = lane_id();
  long long edges = 0;
  // one workgroup per large vertex
  for (unsigned i = blockIdx.x; i < T.cnt[BIN_LARGE]; i += gridDim.x) {
    const int v = (int)(L.large(i) & 0xffffffffu);
    if ((unsigned)v >= (unsigned)a.g.n) continue;
    const long long beg = off[v], end = off[v + 1];
    const float dv = (float)(end - beg);
    CSum s{0.f, 0.f};
    bp_gather(s, a, src, dv, beg + threadIdx.x, end, kBlock, edges, hot, nhot);
    s = wg_merge(s, lds.f);
    if (threadIdx.x == 0) bp_finish_vertex(a, v, s, dv, last, dst);
  }
  const unsigned gw = blockIdx.x * kWaves + wave_in_wg();
  const unsigned nw = gridDim.x * kWaves;
  // one wavefront per medium vertex
  for (unsigned i = gw; i < T.cnt[BIN_MED]; i += nw) {
    const int v = L.med(i);
    if ((unsigned)v >= (unsigned)a.g.n) continue;
    const long long beg = off[v], end = off[v + 1];
    const float dv = (float)(end - beg);
    CSum s{0.f, 0.f};
    bp_gather(s, a, src, dv, beg + lane, end, 64, edges, hot, nhot);
    s = wave_merge(s);
    if (lane == 0) bp_finish_vertex(a, v, s, dv, last, dst);
  }
  // one lane per small vertex
  for (unsigned i = gw * 64u + lane; i < T.cnt[BIN_SMALL]; i += nw * 64u) {
    const int v = L.small(i);
    if ((unsigned)v >= (unsigned)a.g.n) continue;
    const long long beg = off[v], end = off[v + 1];
    const float dv = (float)(end - beg);
    CSum s{0.f, 0.f};
    bp_gather(s, a, src, dv, beg, end, 1, edges, hot, nhot);
    bp_finish_vertex(a, v, s, dv, last, dst);
  }
  add_stats(a.w.ctrl, blockIdx.x, edges, 0ull, lds.red);
}

__global__ void __launch_bounds__(kBlock) k_bp_fused(BpArgs a) {
  __shared__ LdsBp lds;
  __shared__ float2 hot[kHotBp];
  Ctrl *C = a.w.ctrl;
  const VGrid vg = hw_grid();
  GridBarrier bar(C, load_relaxed(&C->bar_gen.v[0]), a.P.watchdog);
  // every vertex, binned by degree: one ballot-filter pass
  const int *off = a.g.off;
  auto pred = [](int v) { (void)v; return true; };
  auto deg = [&](int v) { return off[v + 1] - off[v]; };
  auto ident = [](int i) { return i; };
  ballot_fill(vg, a.g.n, pred, deg, ident, a.P, 0x7fffffff, a.w.bits, regions(a.w, 0, vg.nb),
              a.w.rec + SLOT_SCAN, lds.ball);
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
    bp_iteration(a, t, L, T, lds, hot);
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

// Set-up: the prior field atanh(2 p - 1) and iteration 0's (q, degree) from
// the priors; a prior outside (0, 1) (or NaN) raises SX_ERR_INPUT.
__global__ void __launch_bounds__(kBlock) k_bp_init(BpArgs a) {
  Ctrl *C = a.w.ctrl;
  if (blockIdx.x == 0) reset_barrier(C);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int i = 0; i < 32; ++i) { C->state.v[i] = 0; C->stats.v[i] = 0; }
    C->error.v[0] = 0;
  }
  if (blockIdx.x == 1 || gridDim.x == 1) reset_stat_lines(C);
  bool bad = false;
  for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < a.g.n;
       v += (long long)gridDim.x * kBlock) {
    const float p = a.belief[v];
    if (!(p > 0.f && p < 1.f)) bad = true;
    const float q = 2.f * p - 1.f;
    a.w.bph[v] = atanhf(q);
    a.w.bpq[0][v] = make_float2(q, (float)(a.g.off[v + 1] - a.g.off[v]));
  }
  // a flag of its own (cleared by the launch before), turned into the error
  // word by the launch after, so that it cannot race with the reset above
  if (ballot(bad) && lane_id() == 0) atomic_or_u64((unsigned long long *)&C->aux.v[0], 1ull);
}

// Turns the input flag into the error word once the set-up is complete.
__global__ void k_bp_check(Ctrl *C) {
  if (threadIdx.x == 0 && C->aux.v[0]) C->error.v[0] = SX_ERR_INPUT;
}

__global__ void k_bp_clear_flag(Ctrl *C) {
  if (threadIdx.x == 0) {
    C->aux.v[0] = 0u;
    C->aux.v[1] = 0u;
  }
}

hipError_t bp_launch(const BpArgs &a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_bp_clear_flag, dim3(1), dim3(64), 0, s, a.w.ctrl);
  hipLaunchKernelGGL(k_bp_init, dim3(grid), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_bp_check, dim3(1), dim3(64), 0, s, a.w.ctrl);
  hipLaunchKernelGGL(k_bp_fused, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

const void *bp_kernel() { return (const void *)k_bp_fused; }

}  // namespace sx
