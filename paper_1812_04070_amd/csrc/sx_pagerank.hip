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
//
// Run to convergence (pr_tol > 0; Section 6: PageRank iterates until the
// ranks are stable, starts with pull and switches to push near the end,
// because most vertices are then stable, the switch chosen by a decision
// tree).  Pull iterations as above also record each vertex's change; the
// tree after every iteration: (1) the step changed the vector by at most
// stop_change in L1 -> done; (2) at most n/2 vertices (the majority is
// stable) have a non-uniform change above thr and their out-arcs are at
// most m / kPushArcCost (a push sends an atomic add per arc where a pull
// gathers one value: MI355X runs the pull about ten times as many arcs per
// second), or max_pull iterations ran -> push tail; (3) otherwise pull
// again.  The tail is the delta-accumulative form: every vertex keeps
// its pending change; a listed vertex takes its change (atomic exchange),
// adds it to its rank and sends d * change / outdeg to each out-neighbour
// (atomic add); a neighbour whose pending change crosses thr joins the next
// list (online filter, one entry per vertex through a stamp; an overflowing
// list is rebuilt by a ballot pass over the pending changes).  The tail
// drops the uniform redistribution of vertices without out-arcs, and the
// uniform part of the last pull step's change: with B = I - d A (A the arcs
// only), the fixed point is proportional to x + B^-1 r for any pending r
// whose uniform part is removed, because B^-1 1 is itself proportional to
// the fixed point (Sherman-Morrison on the rank-one dangling term).  So the
// tail ends with one normalisation to sum 1.  A pending change at most thr
// per vertex leaves an L1 error of at most n thr / (1 - d).
#include "sx_frontier.hpp"
#include "sx_kernels.hpp"

namespace sx {


// a push step's cost per arc in units of a pull step's (decision tree)
constexpr float kPushArcCost = 16.f;

struct LdsPr {
  LdsView view;
  LdsBallot ball;
  LdsBins bins;
  long long red[kWaves];
  float f[2 * kWaves];
  float share;
};

SX_DEV float atomic_add_f32(float *p, float v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, SX_AG);
}
SX_DEV float atomic_exch_f32(float *p, float v) {
  return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, SX_AG);
}

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

// The contributions of the first kHotPr vertices, copied into LDS by every
// workgroup at the start of each pull iteration.  After the degree-ordered
// renumbering they are the highest-degree sources (the first 8,192 of
// directed R-MAT s24 send 21 % of its arcs), and a gather served by LDS is
// one request fewer at the L2, whose request rate bounds the pull more than
// its misses do (s24: 36.3 -> 34.4 ms for 20 iterations, the same bits;
// 16,384 entries cost a workgroup per CU and gained nothing).
constexpr int kHotPr = 8192;

// Stage src[0, nhot) into hot (every thread of the workgroup).
SX_DEV void stage_hot(float *hot, const float *src, int nhot) {
  for (int i = threadIdx.x; i < nhot; i += kBlock) hot[i] = src[i];
  __syncthreads();
}

// s += src[ii[e]] for e = e0, e0 + stride, ... < end, in that order (an
// index below nhot reads the LDS copy hot instead).  The indices and
// contributions of kIlp consecutive terms are loaded before any of them is
// added, so a lane has kIlp gathers in flight instead of one; the additions
// keep their order, so the sum is the same bits.
SX_DEV void gather(CSum &s, const float *src, const int *ii, int e0, int end, int stride,
                   long long &edges, const float *hot, int nhot) {
  int e = e0;
  for (; e + (kIlp - 1) * stride < end; e += kIlp * stride) {
    int u[kIlp];
    float x[kIlp];
#pragma unroll
    for (int r = 0; r < kIlp; ++r) u[r] = ii[e + r * stride];
#pragma unroll
    for (int r = 0; r < kIlp; ++r) x[r] = u[r] < nhot ? hot[u[r]] : src[u[r]];
#pragma unroll
    for (int r = 0; r < kIlp; ++r) cadd(s, x[r]);
    edges += kIlp;
  }
  for (; e < end; e += stride) {
    const int u = ii[e];
    cadd(s, u < nhot ? hot[u] : src[u]);
    ++edges;
  }
}

// Tracked form for the run to convergence: the rank array holds x_t and
// becomes x_{t+1}; the pending change without its uniform part cu goes to
// prd; the workgroup counts changes above thr and sums the L1 change.
struct Track {
  float cu;                     // uniform part of this step's change: d (D_t - D_{t-1}) / n
  float active;                 // vertices with a non-uniform change above thr
  CSum change;                  // L1 norm of x_{t+1} - x_t
  CSum arcs;                    // their out-arcs (what a push step would send)
};
SX_DEV void pr_finish_tracked(const PrArgs &a, int v, CSum s, float D, float *dst, CSum &dang,
                              Track &tr) {
  const float d = a.P.pr_d;
  const float r = a.base_teleport + d * ((s.s + s.c) + D * a.inv_n);
  const float r0 = a.rank[v];
  a.rank[v] = r;
  const float pend = (r - r0) - tr.cu;
  a.w.prd[v] = pend;
  cadd(tr.change, fabsf(r - r0));
  const int od = a.g.off[v + 1] - a.g.off[v];
  if (fabsf(pend) > a.thr) {
    tr.active += 1.f;
    cadd(tr.arcs, (float)od);
  }
  if (od > 0) dst[v] = r / (float)od;
  else cadd(dang, r);
}

template <bool kTrack>
SX_DEV void pr_iteration(const PrArgs &a, int t, const ViewRef &L, const Totals &T, LdsPr &lds,
                         float D, Track &tr, float *hot) {
  const Work &w = a.w;
  const float *src = w.contrib[t & 1];
  const int nhot = a.g.n < kHotPr ? a.g.n : kHotPr;
  stage_hot(hot, src, nhot);
  float *dst = w.contrib[(t + 1) & 1];
  const bool last = !kTrack && t == a.iters - 1;
  auto finish = [&](int v, CSum s, CSum &dang) {
    if constexpr (kTrack) pr_finish_tracked(a, v, s, D, dst, dang, tr);
    else pr_finish_vertex(a, v, s, D, last, dst, dang);
  };
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
    gather(s, src, ii, beg + (int)threadIdx.x, end, kBlock, edges, hot, nhot);
    s = wg_merge(s, lds.f);
    if (threadIdx.x == 0) finish(v, s, dang);
  }
  const unsigned gw = blockIdx.x * kWaves + wave_in_wg();
  const unsigned nw = gridDim.x * kWaves;
  // one wavefront per medium vertex
  for (unsigned i = gw; i < T.cnt[BIN_MED]; i += nw) {
    const int v = L.med(i);
    if ((unsigned)v >= (unsigned)a.g.n) continue;
    const int beg = io[v], end = io[v + 1];
    CSum s{0.f, 0.f};
    gather(s, src, ii, beg + lane, end, 64, edges, hot, nhot);
    s = wave_merge(s);
    if (lane == 0) finish(v, s, dang);
  }
  // one lane per small vertex
  for (unsigned i = gw * 64u + lane; i < T.cnt[BIN_SMALL]; i += nw * 64u) {
    const int v = L.small(i);
    if ((unsigned)v >= (unsigned)a.g.n) continue;
    const int beg = io[v], end = io[v + 1];
    CSum s{0.f, 0.f};
    gather(s, src, ii, beg, end, 1, edges, hot, nhot);
    finish(v, s, dang);
  }
  dang = wg_merge(dang, lds.f);
  if (threadIdx.x == 0) {
    float *part = w.dang + (size_t)((t + 1) & 1) * 2 * kMaxGrid;
    part[2 * blockIdx.x] = dang.s;
    part[2 * blockIdx.x + 1] = dang.c;
  }
  if constexpr (kTrack) {
    const CSum ch = wg_merge(tr.change, lds.f);
    const CSum ac = wg_merge(CSum{tr.active, 0.f}, lds.f);
    const CSum ar = wg_merge(tr.arcs, lds.f);
    if (threadIdx.x == 0) {
      float *q = w.prp + ((size_t)(t & 1) * kMaxGrid + blockIdx.x) * 8;
      q[0] = ac.s + ac.c;
      q[1] = ch.s;
      q[2] = ch.c;
      q[3] = ar.s;
      q[4] = ar.c;
    }
  }
  add_stats(w.ctrl, blockIdx.x, edges, 0ull, lds.red);
}

__global__ void __launch_bounds__(kBlock) k_pr_fused(PrArgs a) {
  __shared__ LdsPr lds;
  __shared__ float hot[kHotPr];
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
    const float D = dangling_total(a.w.dang + (size_t)(t & 1) * 2 * kMaxGrid, gridDim.x, lds.f);
    Track none{0.f, 0.f, CSum{0.f, 0.f}};
    pr_iteration<false>(a, t, L, T, lds, D, none, hot);
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

// ------------------------------------------------------ the push tail ---
// Push step j over the list `V` (whole vertices, binned by out-degree): each
// listed vertex takes its pending change, adds it to its rank and sends
// d * change / outdeg to its out-neighbours; a neighbour whose pending change
// crosses thr (first time in this step: stamp j + 1) joins the list of step
// j + 1 (slot (j + 1) % 3, parity (j + 1) & 1).  Every append call is made by
// whole wavefronts (wave- or workgroup-uniform trip counts).
SX_DEV void pr_push_step(const PrArgs &a, int j, const ViewRef &V, const Totals &T, LdsPr &lds) {
  const Work &w = a.w;
  const int *off = a.g.off, *idx = a.g.idx;
  float *pend = w.prd;
  const float d = a.P.pr_d, thr = a.thr;
  const Regions NR = regions(w, (j + 1) & 1, gridDim.x);
  bins_begin(lds.bins, NR, a.P.online_cap);
  WaveStats st;
  long long edges = 0;
  const int lane = lane_id();
  // one arc v -> u carrying `share` (ok: a real arc); convergent
  auto send = [&](bool ok, int u, float share) {
    bool act = false;
    int du = 0;
    if (ok && share != 0.f) {
      const float old = atomic_add_f32(&pend[u], share);
      act = fabsf(old) <= thr && fabsf(old + share) > thr &&
            atomic_exch_i32(&w.stamp[u], j + 1) != j + 1;
      if (act) du = off[u + 1] - off[u];
      ++edges;
    }
    bins_append(act, u, du, NR, blockIdx.x, a.P, 0x7fffffff, lds.bins, st);
  };
  // a vertex's own change: added to its rank, its share per out-arc returned
  auto take = [&](int v, int od) {
    const float c = atomic_exch_f32(&pend[v], 0.f);
    a.rank[v] += c;
    return od > 0 ? d * c / (float)od : 0.f;
  };
  // one workgroup per large vertex
  for (unsigned i = blockIdx.x; i < T.cnt[BIN_LARGE]; i += gridDim.x) {
    const int v = (int)(V.large(i) & 0xffffffffu);
    if ((unsigned)v >= (unsigned)a.g.n) continue;
    const int beg = off[v], end = off[v + 1];
    if (threadIdx.x == 0) lds.share = take(v, end - beg);
    __syncthreads();
    const float share = lds.share;
    for (int e0 = beg; e0 < end; e0 += kBlock) {
      const int e = e0 + (int)threadIdx.x;
      const bool ok = e < end;
      send(ok, ok ? idx[e] : 0, share);
    }
    __syncthreads();
  }
  const unsigned gw = blockIdx.x * kWaves + wave_in_wg();
  const unsigned nw = gridDim.x * kWaves;
  // one wavefront per medium vertex
  for (unsigned i = gw; i < T.cnt[BIN_MED]; i += nw) {
    const int v = V.med(i);
    if ((unsigned)v >= (unsigned)a.g.n) continue;
    const int beg = off[v], end = off[v + 1];
    float share = 0.f;
    if (lane == 0) share = take(v, end - beg);
    share = __shfl(share, 0);
    for (int e0 = beg; e0 < end; e0 += 64) {
      const int e = e0 + lane;
      const bool ok = e < end;
      send(ok, ok ? idx[e] : 0, share);
    }
  }
  // one lane per small vertex, the wavefront stepping through the longest row
  for (unsigned base = gw * 64u; base < T.cnt[BIN_SMALL]; base += nw * 64u) {
    const unsigned i = base + lane;
    int v = -1, beg = 0, od = 0;
    float share = 0.f;
    if (i < T.cnt[BIN_SMALL]) {
      const int x = V.small(i);
      if ((unsigned)x < (unsigned)a.g.n) {
        v = x;
        beg = off[v];
        od = off[v + 1] - beg;
        share = take(v, od);
      }
    }
    int longest = od;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) longest = max(longest, __shfl_xor(longest, o));
    for (int r = 0; r < longest; ++r) {
      const bool ok = r < od;
      send(ok, ok ? idx[beg + r] : 0, share);
    }
  }
  bins_end(lds.bins, st, w.rec + ((j + 1) % 3), blockIdx.x);
  add_stats(w.ctrl, blockIdx.x, edges, blockIdx.x == 0 ? (unsigned long long)T.cnt[0] + T.cnt[1] + T.cnt[2] : 0ull,
            lds.red);
}

// Every vertex with a pending change above thr, binned by out-degree (whole
// vertices), into regions parity p, slot SLOT_SCAN.
SX_DEV void pr_push_ballot(const PrArgs &a, int p, LdsPr &lds) {
  const int *off = a.g.off;
  const float *pend = a.w.prd;
  const float thr = a.thr;
  auto pred = [&](int v) { return fabsf(pend[v]) > thr; };
  auto deg = [&](int v) { return off[v + 1] - off[v]; };
  auto ident = [](int i) { return i; };
  ballot_fill(hw_grid(), a.g.n, pred, deg, ident, a.P, 0x7fffffff, a.w.bits, regions(a.w, p, gridDim.x),
              a.w.rec + SLOT_SCAN, lds.ball);
  if (blockIdx.x == 0 && threadIdx.x == 0) atomic_add_u32(&a.w.ctrl->stats.v[4], 1u);
}

// Sum of a per-workgroup value at q[(par * kMaxGrid + b) * 8 + k] over the
// grid, fixed order (identical in every workgroup).
SX_DEV CSum partial_sum(const float *prp, int par, int k, int kc, float *lf) {
  CSum acc{0.f, 0.f};
  for (unsigned b = threadIdx.x; b < gridDim.x; b += kBlock) {
    const float *q = prp + ((size_t)par * kMaxGrid + b) * 8;
    acc = cmerge(acc, CSum{q[k], kc >= 0 ? q[kc] : 0.f});
  }
  return wg_merge(acc, lf);
}

// Normalisation to sum 1 (every workgroup of the grid; a global barrier
// between the partial sums and the division); false if the barrier failed.
SX_DEV bool pr_normalize(const PrArgs &a, const VGrid &vg, GridBarrier &bar, LdsPr &lds) {
  const int n = a.g.n;
  CSum sum{0.f, 0.f};
  for (long long v = (long long)vg.bid * kBlock + threadIdx.x; v < n; v += (long long)vg.nb * kBlock)
    cadd(sum, a.rank[v]);
  sum = wg_merge(sum, lds.f);
  if (threadIdx.x == 0) {
    float *q = a.w.prp + ((size_t)0 * kMaxGrid + vg.bid) * 8;
    q[6] = sum.s;
    q[7] = sum.c;
  }
  if (!bar.sync()) return false;
  const CSum tot = partial_sum(a.w.prp, 0, 6, 7, lds.f);
  const float S1 = tot.s + tot.c;
  for (long long v = (long long)vg.bid * kBlock + threadIdx.x; v < n; v += (long long)vg.nb * kBlock)
    a.rank[v] = a.rank[v] / S1;
  return true;
}

// The run's end: statistics and the exit reason (one thread).
SX_DEV void pr_conv_done(Ctrl *C, int pulls, int steps, unsigned long long entries) {
  store_relaxed(&C->state.v[0], (unsigned)EXIT_DONE);
  store_relaxed(&C->stats.v[6], (unsigned)(pulls + steps));
  store_relaxed(&C->stats.v[5], (unsigned)pulls);
  atomic_add_u32(&C->stats.v[4], 1u);
  atomic_add_u64((unsigned long long *)&C->statw[0].v[2], entries);
}

// Ctrl::aux words the pull kernel hands to the push kernel: [0] uniform part
// of the last step's change (float bits), [1] pull iterations, [2,3] list
// entries processed.
enum { PRX_CU = 0, PRX_PULLS = 1, PRX_ENTRIES = 2 };

// Selective fusion for the run to convergence (Section 5: one persistent
// kernel per direction, a direction change ends the launch): the pull
// kernel runs the pull iterations and the decision tree; converged, it
// normalises and ends the run; otherwise it exits with EXIT_SWITCH and the
// host launches the push kernel.  Each kernel runs at the occupancy of its
// own registers (one kernel holding both ran the pull at one workgroup per
// CU: 2.5 against 1.8 ms per iteration at s24).
__global__ void __launch_bounds__(kBlock) k_pr_conv_pull(PrArgs a) {
  __shared__ LdsPr lds;
  __shared__ float hot[kHotPr];
  Ctrl *C = a.w.ctrl;
  const VGrid vg = hw_grid();
  GridBarrier bar(C, load_relaxed(&C->bar_gen.v[0]), a.P.watchdog);
  const int n = a.g.n;
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
  float Dprev = 0.f, cu = 0.f;
  int t = 0;
  bool tail = false;
  for (;; ++t) {
    const float D = dangling_total(a.w.dang + (size_t)(t & 1) * 2 * kMaxGrid, gridDim.x, lds.f);
    cu = t == 0 ? 0.f : a.P.pr_d * (D - Dprev) * a.inv_n;
    Dprev = D;
    Track tr{cu, 0.f, CSum{0.f, 0.f}, CSum{0.f, 0.f}};
    pr_iteration<true>(a, t, L, T, lds, D, tr, hot);
    if (!bar.sync()) return;
    // the decision tree, evaluated identically by every workgroup
    const CSum ch = partial_sum(a.w.prp, t & 1, 1, 2, lds.f);
    const CSum ac = partial_sum(a.w.prp, t & 1, 0, -1, lds.f);
    const CSum ar = partial_sum(a.w.prp, t & 1, 3, 4, lds.f);
    if (ch.s + ch.c <= a.stop_change) break;
    if ((t >= 1 && ac.s + ac.c <= 0.5f * (float)n && (ar.s + ar.c) * kPushArcCost <= (float)a.g.m) ||
        t + 1 >= a.max_pull) {
      tail = true;
      break;
    }
  }
  const int pulls = t + 1;
  const unsigned long long entries = (unsigned long long)pulls * ((unsigned long long)T.cnt[0] + T.cnt[1] + T.cnt[2]);
  if (tail) {
    if (vg.bid == 0 && threadIdx.x == 0) {
      store_relaxed(&C->aux.v[PRX_CU], __float_as_uint(cu));
      store_relaxed(&C->aux.v[PRX_PULLS], (unsigned)pulls);
      store_relaxed((unsigned long long *)&C->aux.v[PRX_ENTRIES], entries);
      store_relaxed(&C->state.v[0], (unsigned)EXIT_SWITCH);
    }
    return;
  }
  if (!pr_normalize(a, vg, bar, lds)) return;
  if (vg.bid == 0 && threadIdx.x == 0) pr_conv_done(C, pulls, 0, entries);
}

// The push tail (after k_pr_conv_pull exited with EXIT_SWITCH), then the
// normalisation.
__global__ void __launch_bounds__(kBlock) k_pr_conv_push(PrArgs a) {
  __shared__ LdsPr lds;
  Ctrl *C = a.w.ctrl;
  const VGrid vg = hw_grid();
  GridBarrier bar(C, load_relaxed(&C->bar_gen.v[0]), a.P.watchdog);
  const int n = a.g.n;
  if (load_relaxed(&C->state.v[0]) != (unsigned)EXIT_SWITCH) return;
  const float cu = __uint_as_float(load_relaxed(&C->aux.v[PRX_CU]));
  const int pulls = (int)load_relaxed(&C->aux.v[PRX_PULLS]);
  const unsigned long long entries = load_relaxed((const unsigned long long *)&C->aux.v[PRX_ENTRIES]);
  // the rank without the last step's pending change (its uniform part cu
  // dropped, see above); no vertex listed yet
  for (long long v = (long long)vg.bid * kBlock + threadIdx.x; v < n; v += (long long)vg.nb * kBlock) {
    a.rank[v] = a.rank[v] - a.w.prd[v] - cu;
    a.w.stamp[v] = -1;
  }
  pr_push_ballot(a, 0, lds);
  if (!bar.sync()) return;
  int slot = SLOT_SCAN, steps = 0;
  for (int j = 0;; ++j) {
    if (j > 100000) {
      if (vg.bid == 0 && threadIdx.x == 0) store_relaxed(&C->state.v[0], (unsigned)EXIT_LIMIT);
      return;
    }
    ViewRef V;
    V.V = &lds.view;
    V.R = regions(a.w, j & 1, vg.nb);
    V.G = vg.nb;
    Totals S = view_build(a.w.rec + slot, vg.nb, V.R, lds.view, lds.red);
    if (S.nf == 0) break;
    if (S.ovf) {
      // the online list overflowed its regions: rebuilt by a ballot pass
      pr_push_ballot(a, j & 1, lds);
      if (!bar.sync()) return;
      S = view_build(a.w.rec + SLOT_SCAN, vg.nb, V.R, lds.view, lds.red);
      if (S.ovf) {
        if (threadIdx.x == 0) store_relaxed(&C->error.v[0], (unsigned)SX_ERR_CAPACITY);
        return;
      }
      if (S.nf == 0) break;
    }
    pr_push_step(a, j, V, S, lds);
    ++steps;
    if (!bar.sync()) return;
    slot = (j + 1) % 3;
  }
  if (!pr_normalize(a, vg, bar, lds)) return;
  if (vg.bid == 0 && threadIdx.x == 0) pr_conv_done(C, pulls, steps, entries);
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
    if (a.conv) a.rank[v] = a.inv_n;
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
  if (a.conv) hipLaunchKernelGGL(k_pr_conv_pull, dim3(grid), dim3(kBlock), 0, s, a);
  else hipLaunchKernelGGL(k_pr_fused, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t pagerank_push_launch(const PrArgs &a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_pr_conv_push, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

const void *pagerank_kernel(bool conv) { return conv ? (const void *)k_pr_conv_pull : (const void *)k_pr_fused; }
const void *pagerank_push_kernel() { return (const void *)k_pr_conv_push; }

}  // namespace sx
