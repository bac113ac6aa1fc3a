// Frontier traversal engine for BFS and SSSP: the ACC processing loop of
// Section 3.3 (compute on the small / medium / large lists, combine, record
// active vertices, global barrier, overflow check, next lists) with the
// just-in-time task management of Section 4 and the push/pull kernel fusion
// of Section 5.
//
// Each algorithm is an ACC triple (Section 3.2):
//   BFS   Active: depth == level + 1 (newly visited).  Compute: level + 1.
//         Combine: vote -- any single update is correct, so push claims an
//         unvisited vertex with one compare-and-swap and pull stops at the
//         first in-neighbour found in the frontier (collaborative early
//         termination, Section 3.3 "Comparison").
//   SSSP  Active: distance lowered in the previous iteration (Figure
//         tech-compute(a)).  Compute: dist(v) + w(v,u).  Combine: minimum
//         (aggregation): push lowers dist(u) with an atomic minimum, pull
//         reduces over the in-arcs and the single owner writes, no atomics.
//
// Kernels, per algorithm:
//   push_fused / pull_fused  persistent: iterate in one direction, separated
//                            by the software global barrier, until the
//                            frontier is empty or the direction changes.
//   push_step / ballot_count_k / ballot_write_k / pull_scan / pull_step
//                            the same phases as one launch each (no fusion).
#include "sx_frontier.hpp"
#include "sx_kernels.hpp"
#include "sx_policy.hpp"

namespace sx {

// Phases are kept out of line so that a fused kernel needs the registers of
// its largest phase, not of all of them at once (Section 5: fusion raises
// register use and so lowers the number of resident threads).
#define SX_PHASE __device__ __forceinline__

// ------------------------------------------------------------- ACC ops ---
struct BfsOps {
  static constexpr bool kVote = true;
  int *depth;
  int it;
  // push Compute + Combine for arc v->u; true when u becomes active
  SX_DEV bool push(int v, int u, int arc, const DevGraph &g, unsigned &err) const {
    (void)v; (void)arc; (void)g; (void)err;
    return load_relaxed(&depth[u]) == -1 && atomic_cas_i32(&depth[u], -1, it + 1);
  }
  SX_DEV bool next_active(int v) const { return load_relaxed(&depth[v]) == it + 1; }
  SX_DEV bool in_frontier(int v) const { return load_relaxed(&depth[v]) == it; }
  SX_DEV bool pull_candidate(int v) const { return load_relaxed(&depth[v]) == -1; }
};

struct SsspOps {
  static constexpr bool kVote = false;
  unsigned *dist;
  int *stamp;
  int it;
  SX_DEV bool push(int v, int u, int arc, const DevGraph &g, unsigned &err) const {
    const unsigned dv = load_relaxed(&dist[v]);
    const unsigned nd = dv + g.w[arc];
    if (nd < dv || nd == 0xFFFFFFFFu) { err = SX_ERR_OVERFLOW; return false; }
    if (nd >= load_relaxed(&dist[u])) return false;
    const unsigned old = atomic_min_u32(&dist[u], nd);
    if (nd >= old) return false;
    return atomic_exch_i32(&stamp[u], it + 1) != it + 1;
  }
  SX_DEV bool next_active(int v) const { return load_relaxed(&stamp[v]) == it + 1; }
  SX_DEV bool in_frontier(int v) const { return load_relaxed(&stamp[v]) == it; }
  SX_DEV bool pull_candidate(int v) const { (void)v; return true; }
};

SX_DEV void reset_counters(Counters *q) {
  for (int b = 0; b < NBINS; ++b) store_relaxed(&q->cnt[b], 0u);
  store_relaxed(&q->nf, 0u);
  store_relaxed(&q->mf, 0ull);
  store_relaxed(&q->overflow, 0u);
}

SX_DEV int degree_of(const int *off, int v) { return off[v + 1] - off[v]; }

SX_DEV Lists lists_for(const Work &w, int parity, Counters *c) {
  Lists L;
  L.s = w.q[parity][0];
  L.m = w.q[parity][1];
  L.l = w.ql[parity];
  L.c = c;
  L.cap_s = w.qcap_small;
  L.cap_m = w.qcap_med;
  L.cap_l = w.qcap_large;
  return L;
}

SX_DEV unsigned online_cap(const Work &w, const Params &P, int bin) {
  const unsigned q = bin == 0 ? w.qcap_small : bin == 1 ? w.qcap_med : w.qcap_large;
  return P.online_cap < q ? P.online_cap : q;
}

struct LdsTrav {
  int small[kWaves][192];
  unsigned cnt[kWaves * 8];
  long long red[kWaves];
  int flag;
};

// --------------------------------------------------------- push phase ---
// Compute + combine over the current lists (parity it & 1, counters slot it),
// online filter into the next lists (parity it+1, slot it+1).
template <class Ops>
SX_PHASE void push_phase(const VGrid &vg, const TravArgs &a, const Params &P, const Ops &ops, int it, LdsTrav &lds) {
  Ctrl *C = a.w.ctrl;
  Counters *cur = &C->q[it % 3], *nxt = &C->q[(it + 1) % 3];
  // counts are clamped to the list capacities: reads never leave the lists
  const unsigned cs = min(load_relaxed(&cur->cnt[0]), a.w.qcap_small),
                 cm = min(load_relaxed(&cur->cnt[1]), a.w.qcap_med),
                 cl = min(load_relaxed(&cur->cnt[2]), a.w.qcap_large);
  const int p = it & 1;
  Lists NL = lists_for(a.w, p ^ 1, nxt);
  NL.cap_s = online_cap(a.w, P, 0);
  NL.cap_m = online_cap(a.w, P, 1);
  NL.cap_l = online_cap(a.w, P, 2);
  const DevGraph &g = a.g;
  WaveStats st;
  unsigned err = 0;
  long long edges = 0;
  auto op = [&](int v, int u, int arc, bool ok) {
    bool act = false;
    int du = 0;
    if (ok) {
      ++edges;
      if (ops.push(v, u, arc, g, err)) { act = true; du = degree_of(g.off, u); }
    }
    online_append(act, u, du, NL, P, P.chunk, st);
  };
  const unsigned gw = vg.bid * kWaves + wave_in_wg();
  const unsigned nw = vg.nb * kWaves;
  visit_large(vg, g.n, a.w.ql[p], cl, g.off, g.idx, P.chunk, op);
  visit_med(g.n, a.w.q[p][1], cm, g.off, g.idx, op, gw, nw);
  visit_small(g.n, a.w.q[p][0], cs, g.off, g.idx, op, gw, nw, lds.small[wave_in_wg()]);
  flush_stats(st, nxt);
  const long long e = wave_sum_ll(edges);
  if (lane_id() == 0) {
    if (e) atomic_add_u64((unsigned long long *)&C->stats.v[0], (unsigned long long)e);
    if (err) store_relaxed(&C->error.v[0], err);
  }
  // worklist entries processed this iteration (vertex expansions)
  if (vg.bid == 0 && threadIdx.x == 0)
    atomic_add_u64((unsigned long long *)&C->stats.v[2], (unsigned long long)(cs + cm) + cl);
}

// --------------------------------------------------------- ballot filter ---
// Rebuild the next lists (parity it+1) from vertex metadata: pass 1 counts.
template <class Ops>
SX_PHASE void ballot_pass1(const VGrid &vg, const TravArgs &a, const Params &P, const Ops &ops, LdsTrav &lds) {
  const Work &w = a.w;
  Tiling T(a.g.n, vg.nb * kWaves);
  const int *off = a.g.off;
  auto pred = [&](int v) { return ops.next_active(v); };
  auto deg = [&](int v) { return degree_of(off, v); };
  ballot_count(vg, a.g.n, T, pred, deg, P, P.chunk, w.bits, w.wavecnt, w.wgc, lds.cnt);
}

// pass 2 writes the sorted lists and (workgroup 0) their counts.
SX_PHASE void ballot_pass2(const VGrid &vg, const TravArgs &a, const Params &P, int it, LdsTrav &lds) {
  const Work &w = a.w;
  Tiling T(a.g.n, vg.nb * kWaves);
  const int *off = a.g.off;
  auto deg = [&](int v) { return degree_of(off, v); };
  const int p = (it + 1) & 1;
  WgCount tot;
  auto ident = [](int i) { return i; };
  ballot_write(vg, a.g.n, T, deg, ident, P.chunk, w.bits, w.wavecnt, w.wgc,
               w.q[p][0], w.q[p][1], w.ql[p], tot, lds.cnt, lds.red);
  if (vg.bid == 0 && threadIdx.x == 0) {
    Counters *nxt = &w.ctrl->q[(it + 1) % 3];
    store_relaxed(&nxt->cnt[0], tot.cnt[0]);
    store_relaxed(&nxt->cnt[1], tot.cnt[1]);
    store_relaxed(&nxt->cnt[2], tot.cnt[2]);
    store_relaxed(&nxt->overflow, 0u);
    atomic_add_u32(&w.ctrl->stats.v[4], 1u);
  }
}

// ----------------------------------------------------------- pull phases ---
// Scan: frontier bitmap of iteration it, and the sorted candidate lists
// (pass 1 of a ballot filter whose predicate is "may still change").
template <class Ops>
SX_PHASE void pull_scan(const VGrid &vg, const TravArgs &a, const Params &P0, const Ops &ops, LdsTrav &lds) {
  const Work &w = a.w;
  Tiling T(a.g.n, vg.nb * kWaves);
  const int *off = a.g.in_off;
  const int n = a.g.n;
  // frontier words
  {
    const unsigned gw = vg.bid * kWaves + wave_in_wg();
    const long long start = (long long)gw * T.tile;
    for (int s = 0; s < T.tile && start + s < n; s += 64) {
      const long long v = start + s + lane_id();
      const bool f = v < n && ops.in_frontier((int)v);
      const uint64_t mk = ballot(f);
      if (lane_id() == 0) w.fbits[(start + s) >> 6] = mk;
    }
  }
  auto pred = [&](int v) { return degree_of(off, v) > 0 && ops.pull_candidate(v); };
  auto deg = [&](int v) { return degree_of(off, v); };
  ballot_count(vg, n, T, pred, deg, P0, 0x7fffffff, w.bits, w.wavecnt, w.wgc, lds.cnt);
}

// Write the candidate lists into the parity-`it` buffers (not read by anyone
// else in a pull iteration); counts go to slot it.
SX_PHASE void pull_lists(const VGrid &vg, const TravArgs &a, int it, LdsTrav &lds) {
  const Work &w = a.w;
  Tiling T(a.g.n, vg.nb * kWaves);
  const int *off = a.g.in_off;
  auto deg = [&](int v) { return degree_of(off, v); };
  const int p = it & 1;
  WgCount tot;
  auto ident = [](int i) { return i; };
  ballot_write(vg, a.g.n, T, deg, ident, 0x7fffffff, w.bits, w.wavecnt, w.wgc,
               w.q[p][0], w.q[p][1], w.ql[p], tot, lds.cnt, lds.red);
  if (vg.bid == 0 && threadIdx.x == 0) {
    Counters *cur = &w.ctrl->q[it % 3];
    store_relaxed(&cur->cnt[0], tot.cnt[0]);
    store_relaxed(&cur->cnt[1], tot.cnt[1]);
    store_relaxed(&cur->cnt[2], tot.cnt[2]);
  }
}

SX_DEV bool fbit(const unsigned long long *fb, int u) { return (fb[u >> 6] >> (u & 63)) & 1ull; }

// Pull compute over the candidate lists (parity it, slot it).  Found /
// improved vertices are recorded by the online filter into the next lists
// (parity it+1, slot it+1) so that a switch back to push needs no scan.
template <class Ops>
SX_PHASE void pull_phase(const VGrid &vg, const TravArgs &a, const Params &P, const Ops &ops, int it, LdsTrav &lds) {
  Ctrl *C = a.w.ctrl;
  Counters *cur = &C->q[it % 3], *nxt = &C->q[(it + 1) % 3];
  // counts are clamped to the list capacities: reads never leave the lists
  const unsigned cs = min(load_relaxed(&cur->cnt[0]), a.w.qcap_small),
                 cm = min(load_relaxed(&cur->cnt[1]), a.w.qcap_med),
                 cl = min(load_relaxed(&cur->cnt[2]), a.w.qcap_large);
  const int p = it & 1;
  Lists NL = lists_for(a.w, p ^ 1, nxt);
  NL.cap_s = online_cap(a.w, P, 0);
  NL.cap_m = online_cap(a.w, P, 1);
  NL.cap_l = online_cap(a.w, P, 2);
  const DevGraph &g = a.g;
  const unsigned long long *fb = a.w.fbits;
  WaveStats st;
  long long edges = 0;
  const int lane = lane_id();
  const unsigned gw = vg.bid * kWaves + wave_in_wg();
  const unsigned nw = vg.nb * kWaves;
  // One workgroup per large candidate
  for (unsigned i = vg.bid; i < cl; i += vg.nb) {
    const int v = (int)(a.w.ql[p][i] & 0xffffffffu);
    if ((unsigned)v >= (unsigned)g.n) continue;
    const int beg = g.in_off[v], end = g.in_off[v + 1];
    unsigned best = 0xFFFFFFFFu;
    if (!Ops::kVote) best = load_relaxed(&((unsigned *)a.state_i)[v]);
    bool found = false;
    for (int b = beg; b < end; b += kBlock) {
      const int arc = b + (int)threadIdx.x;
      bool hit = false;
      if (arc < end) {
        ++edges;
        const int u = g.in_idx[arc];
        if (fbit(fb, u)) {
          hit = true;
          if (!Ops::kVote) {
            const unsigned c = load_relaxed(&((unsigned *)a.state_i)[u]) + g.in_w[arc];
            best = c < best ? c : best;
          }
        }
      }
      if (Ops::kVote) {
        found = __syncthreads_or(hit);
        if (found) break;
      }
    }
    bool act = false;
    if (Ops::kVote) {
      if (found && threadIdx.x == 0) { store_relaxed(&a.state_i[v], it + 1); act = true; }
    } else {
      best = wave_min_u(best);
      if (lane == 0) lds.cnt[wave_in_wg()] = best;
      __syncthreads();
      if (threadIdx.x == 0) {
        for (int w2 = 0; w2 < kWaves; ++w2) best = lds.cnt[w2] < best ? lds.cnt[w2] : best;
        if (best < load_relaxed(&((unsigned *)a.state_i)[v])) {
          store_relaxed(&((unsigned *)a.state_i)[v], best);
          store_relaxed(&a.w.stamp[v], it + 1);
          act = true;
        }
      }
      __syncthreads();
    }
    if (wave_in_wg() == 0) online_append(act, v, end - beg, NL, P, P.chunk, st);
  }
  // One wavefront per medium candidate
  for (unsigned i = gw; i < cm; i += nw) {
    const int v = a.w.q[p][1][i];
    if ((unsigned)v >= (unsigned)g.n) continue;
    const int beg = g.in_off[v], end = g.in_off[v + 1];
    unsigned best = 0xFFFFFFFFu;
    bool found = false;
    for (int b = beg; b < end; b += 64) {
      const int arc = b + lane;
      bool hit = false;
      if (arc < end) {
        ++edges;
        const int u = g.in_idx[arc];
        if (fbit(fb, u)) {
          hit = true;
          if (!Ops::kVote) {
            const unsigned c = load_relaxed(&((unsigned *)a.state_i)[u]) + g.in_w[arc];
            best = c < best ? c : best;
          }
        }
      }
      if (Ops::kVote && ballot(hit)) { found = true; break; }
    }
    bool act = false;
    if (Ops::kVote) {
      if (found && lane == 0) { store_relaxed(&a.state_i[v], it + 1); act = true; }
    } else {
      best = wave_min_u(best);
      if (lane == 0 && best < load_relaxed(&((unsigned *)a.state_i)[v])) {
        store_relaxed(&((unsigned *)a.state_i)[v], best);
        store_relaxed(&a.w.stamp[v], it + 1);
        act = true;
      }
    }
    online_append(act, v, end - beg, NL, P, P.chunk, st);
  }
  // One lane per small candidate
  for (unsigned c0 = gw * 64u; c0 < cs; c0 += nw * 64u) {
    const unsigned i = c0 + lane;
    bool act = false;
    int v = 0, d = 0;
    if (i < cs && (unsigned)a.w.q[p][0][i] < (unsigned)g.n) {
      v = a.w.q[p][0][i];
      const int beg = g.in_off[v], end = g.in_off[v + 1];
      d = end - beg;
      // four in-arcs per round: their ids and bitmap words are loaded
      // independently, so a lane waits for two memory round trips per four
      // arcs instead of per arc
      if (Ops::kVote) {
        int arc = beg;
        for (; arc + 4 <= end; arc += 4) {
          const int u0 = g.in_idx[arc], u1 = g.in_idx[arc + 1], u2 = g.in_idx[arc + 2],
                    u3 = g.in_idx[arc + 3];
          edges += 4;
          if (fbit(fb, u0) | fbit(fb, u1) | fbit(fb, u2) | fbit(fb, u3)) { act = true; break; }
        }
        for (; !act && arc < end; ++arc) {
          ++edges;
          if (fbit(fb, g.in_idx[arc])) act = true;
        }
        if (act) store_relaxed(&a.state_i[v], it + 1);
      } else {
        unsigned best = load_relaxed(&((unsigned *)a.state_i)[v]);
        const unsigned old = best;
        const unsigned *dist = (const unsigned *)a.state_i;
        int arc = beg;
        for (; arc + 4 <= end; arc += 4) {
          int u[4];
          bool h[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) u[j] = g.in_idx[arc + j];
#pragma unroll
          for (int j = 0; j < 4; ++j) h[j] = fbit(fb, u[j]);
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (h[j]) {
              const unsigned c = load_relaxed(&dist[u[j]]) + g.in_w[arc + j];
              best = c < best ? c : best;
            }
          edges += 4;
        }
        for (; arc < end; ++arc) {
          ++edges;
          const int u1 = g.in_idx[arc];
          if (fbit(fb, u1)) {
            const unsigned c = load_relaxed(&dist[u1]) + g.in_w[arc];
            best = c < best ? c : best;
          }
        }
        if (best < old) {
          store_relaxed(&((unsigned *)a.state_i)[v], best);
          store_relaxed(&a.w.stamp[v], it + 1);
          act = true;
        }
      }
    }
    online_append(act, v, d, NL, P, P.chunk, st);
  }
  flush_stats(st, nxt);
  const long long e = wave_sum_ll(edges);
  if (lane == 0 && e) atomic_add_u64((unsigned long long *)&C->stats.v[0], (unsigned long long)e);
  if (vg.bid == 0 && threadIdx.x == 0) {
    atomic_add_u64((unsigned long long *)&C->stats.v[2], (unsigned long long)(cs + cm) + cl);
    atomic_add_u32(&C->stats.v[5], 1u);
  }
}

// --------------------------------------------------------- decisions ---
// Uniform per-workgroup run state, saved in Ctrl::state across launches:
// [0] exit reason [1] iteration [6,7] unexplored arcs [8] previous frontier
// size [10,11] vertices activated so far [12] t1 [13] t2.
struct RunState {
  int it;
  unsigned long long mu;
  PolicyState ps;
  Params P;
};

SX_DEV void load_state(const TravArgs &a, RunState &s) {
  Ctrl *C = a.w.ctrl;
  s.it = (int)load_relaxed(&C->state.v[1]);
  s.mu = load_relaxed((unsigned long long *)&C->state.v[6]);
  s.ps.nf_prev = load_relaxed(&C->state.v[8]);
  s.ps.reached = load_relaxed((unsigned long long *)&C->state.v[10]);
  s.P = a.P;
  const unsigned t1 = load_relaxed(&C->state.v[12]), t2 = load_relaxed(&C->state.v[13]);
  if (t1) { s.P.t1 = (int)t1; s.P.t2 = (int)t2; }
}

SX_DEV void finish(const VGrid &vg, Ctrl *C, int reason, const RunState &s) {
  if (vg.bid == 0 && threadIdx.x == 0) {
    store_relaxed(&C->state.v[0], (unsigned)reason);
    store_relaxed(&C->state.v[1], (unsigned)s.it);
    store_relaxed((unsigned long long *)&C->state.v[6], s.mu);
    store_relaxed(&C->state.v[8], s.ps.nf_prev);
    store_relaxed((unsigned long long *)&C->state.v[10], s.ps.reached);
    store_relaxed(&C->state.v[12], (unsigned)s.P.t1);
    store_relaxed(&C->state.v[13], (unsigned)s.P.t2);
  }
}

struct LdsPolicy {
  float p[kMlpParams];
  float h[2 * kMlpHid];
  float y[kMlpOut];
};

// The decision after iteration s.it: the rule of decide_core, then -- with
// the learned policy -- the MLP's choices where the caller left them open.
// Overflow always forces the ballot rebuild: the online lists are incomplete.
template <class Ops>
SX_DEV Decision decide(const TravArgs &a, RunState &s, bool pulling, LdsPolicy *pol) {
  Counters *nxt = &a.w.ctrl->q[(s.it + 1) % 3];
  DecideIn in;
  in.nf = load_relaxed(&nxt->nf);
  in.mf = load_relaxed(&nxt->mf);
  in.ovf = load_relaxed(&nxt->overflow);
  in.it = s.it;
  in.pulling = pulling;
  in.vote = Ops::kVote;
  in.n = a.g.n;
  in.m = a.g.m;
  Decision d = decide_core(in, s.P, s.mu);
  if (!d.done && a.P.learned) {
    float x[kMlpIn];
    policy_features(in.nf, in.mf, Ops::kVote ? s.mu : (unsigned long long)a.g.m, a.g.n, a.g.m, s.ps,
                    pulling, x);
    __syncthreads();
    if (wave_in_wg() == 0) {
      float y[kMlpOut];
      mlp_eval_wave(pol->p, x, pol->h, y);
      if (lane_id() == 0)
        for (int k = 0; k < kMlpOut; ++k) pol->y[k] = y[k];
    }
    __syncthreads();
    const float y0 = pol->y[0], y1 = pol->y[1], y2 = pol->y[2], y3 = pol->y[3];
    if (a.P.direction == 0) {
      if (!pulling) d.to_pull = y0 > 0.f;
      else d.to_push = !(y0 > 0.f);
    }
    if (!pulling && !d.to_pull) d.ballot = in.ovf || (a.P.filter == 0 ? y1 > 0.f : a.P.filter == 2);
    if (!a.P.bins_fixed) {
      s.P.t1 = 1 << clamp_log2(y2, 2, 8);
      const int t2 = 1 << clamp_log2(y3, 6, 12);
      s.P.t2 = t2 > s.P.t1 ? t2 : s.P.t1;
    }
  }
  s.ps.nf_prev = in.nf;
  s.ps.reached += in.nf;
  return d;
}

template <class Ops>
SX_DEV Ops make_ops(const TravArgs &a, int it);
template <>
SX_DEV BfsOps make_ops<BfsOps>(const TravArgs &a, int it) { return BfsOps{a.state_i, it}; }
template <>
SX_DEV SsspOps make_ops<SsspOps>(const TravArgs &a, int it) {
  return SsspOps{(unsigned *)a.state_i, a.w.stamp, it};
}

SX_DEV void load_policy(const TravArgs &a, LdsPolicy &pol) {
  if (!a.P.learned) return;
  for (int i = threadIdx.x; i < kMlpParams; i += kBlock) pol.p[i] = a.mlp[i];
  __syncthreads();
}

SX_DEV bool entry_done(Ctrl *C) {
  const unsigned e = load_relaxed(&C->state.v[0]);
  return e == EXIT_DONE || e == EXIT_LIMIT || e == EXIT_ERROR;
}

// -------------------------------------------------- persistent kernels ---
template <class Ops>
__global__ void __launch_bounds__(kBlock) k_push_fused(TravArgs a) {
  __shared__ LdsTrav lds;
  __shared__ LdsPolicy pol;
  Ctrl *C = a.w.ctrl;
  const VGrid vg = hw_grid();
  GridBarrier bar(C, load_relaxed(&C->bar_gen.v[0]));
  if (entry_done(C) || bar.failed()) return;
  RunState s;
  load_state(a, s);
  load_policy(a, pol);
  // a list that overflowed while pulling is rebuilt before the first push
  if (load_relaxed(&C->q[s.it % 3].overflow)) {
    Ops ops = make_ops<Ops>(a, s.it - 1);
    ballot_pass1(vg, a, s.P, ops, lds);
    if (!bar.sync()) { finish(vg, C, EXIT_ERROR, s); return; }
    ballot_pass2(vg, a, s.P, s.it - 1, lds);
    if (!bar.sync()) { finish(vg, C, EXIT_ERROR, s); return; }
  }
  for (;;) {
    if (vg.bid == 0 && threadIdx.x == 0) {
      Counters *old = &C->q[(s.it + 2) % 3];
      for (int b = 0; b < NBINS; ++b) store_relaxed(&old->cnt[b], 0u);
      store_relaxed(&old->nf, 0u);
      store_relaxed(&old->mf, 0ull);
      store_relaxed(&old->overflow, 0u);
      atomic_add_u32(&C->stats.v[6], 1u);
    }
    Ops ops = make_ops<Ops>(a, s.it);
    push_phase(vg, a, s.P, ops, s.it, lds);
    if (!bar.sync()) { finish(vg, C, EXIT_ERROR, s); return; }
    if (load_relaxed(&C->error.v[0])) { finish(vg, C, EXIT_ERROR, s); return; }
    Decision d = decide<Ops>(a, s, false, &pol);
    if (d.done) { ++s.it; finish(vg, C, s.it >= a.P.max_iters ? EXIT_LIMIT : EXIT_DONE, s); return; }
    if (d.to_pull) { ++s.it; finish(vg, C, EXIT_SWITCH, s); return; }
    if (d.ballot) {
      ballot_pass1(vg, a, s.P, ops, lds);
      if (!bar.sync()) { finish(vg, C, EXIT_ERROR, s); return; }
      ballot_pass2(vg, a, s.P, s.it, lds);
      if (!bar.sync()) { finish(vg, C, EXIT_ERROR, s); return; }
    }
    ++s.it;
  }
}

template <class Ops>
__global__ void __launch_bounds__(kBlock) k_pull_fused(TravArgs a) {
  __shared__ LdsTrav lds;
  __shared__ LdsPolicy pol;
  Ctrl *C = a.w.ctrl;
  const VGrid vg = hw_grid();
  GridBarrier bar(C, load_relaxed(&C->bar_gen.v[0]));
  if (entry_done(C) || bar.failed()) return;
  RunState s;
  load_state(a, s);
  load_policy(a, pol);
  for (;;) {
    Ops ops = make_ops<Ops>(a, s.it);
    pull_scan(vg, a, s.P, ops, lds);
    if (!bar.sync()) { finish(vg, C, EXIT_ERROR, s); return; }
    if (vg.bid == 0 && threadIdx.x == 0) {
      // this iteration appends to slot it+1; a push iteration that may follow
      // appends to slot it+2: both start empty (nobody reads either now)
      reset_counters(&C->q[(s.it + 1) % 3]);
      reset_counters(&C->q[(s.it + 2) % 3]);
      atomic_add_u32(&C->stats.v[6], 1u);
    }
    pull_lists(vg, a, s.it, lds);
    if (!bar.sync()) { finish(vg, C, EXIT_ERROR, s); return; }
    pull_phase(vg, a, s.P, ops, s.it, lds);
    if (!bar.sync()) { finish(vg, C, EXIT_ERROR, s); return; }
    if (load_relaxed(&C->error.v[0])) { finish(vg, C, EXIT_ERROR, s); return; }
    Decision d = decide<Ops>(a, s, true, &pol);
    if (d.done) { ++s.it; finish(vg, C, s.it >= a.P.max_iters ? EXIT_LIMIT : EXIT_DONE, s); return; }
    if (d.to_push) { ++s.it; finish(vg, C, EXIT_SWITCH, s); return; }
    ++s.it;
  }
}

// ------------------------------------------------ one-phase kernels ---
// The same phases, one launch each; the host reads the counters between
// launches and takes the decisions (no fusion).  `P` carries the thresholds
// the host chose for this iteration.
template <class Ops>
__global__ void __launch_bounds__(kBlock) k_push_step(TravArgs a, int it) {
  __shared__ LdsTrav lds;
  const VGrid vg = hw_grid();
  Ops ops = make_ops<Ops>(a, it);
  push_phase(vg, a, a.P, ops, it, lds);
}
template <class Ops>
__global__ void __launch_bounds__(kBlock) k_ballot1(TravArgs a, int it) {
  __shared__ LdsTrav lds;
  const VGrid vg = hw_grid();
  Ops ops = make_ops<Ops>(a, it);
  ballot_pass1(vg, a, a.P, ops, lds);
}
__global__ void __launch_bounds__(kBlock) k_ballot2(TravArgs a, int it) {
  __shared__ LdsTrav lds;
  const VGrid vg = hw_grid();
  ballot_pass2(vg, a, a.P, it, lds);
}
template <class Ops>
__global__ void __launch_bounds__(kBlock) k_pull_scan(TravArgs a, int it) {
  __shared__ LdsTrav lds;
  const VGrid vg = hw_grid();
  Ops ops = make_ops<Ops>(a, it);
  pull_scan(vg, a, a.P, ops, lds);
}
__global__ void __launch_bounds__(kBlock) k_pull_lists(TravArgs a, int it) {
  __shared__ LdsTrav lds;
  const VGrid vg = hw_grid();
  pull_lists(vg, a, it, lds);
}
template <class Ops>
__global__ void __launch_bounds__(kBlock) k_pull_step(TravArgs a, int it) {
  __shared__ LdsTrav lds;
  const VGrid vg = hw_grid();
  Ops ops = make_ops<Ops>(a, it);
  pull_phase(vg, a, a.P, ops, it, lds);
}

// ------------------------------------------------------ sequenced mode ---
// The fused loop of Section 5 with the kernel boundary as its global
// barrier: every launch runs exactly one phase and hands the run state to
// the next launch through Ctrl::seq (launch L reads seq[L & 1] and writes
// seq[(L + 1) & 1]).  After a compute phase the next launch first takes the
// decision -- every workgroup reads the same counters and decides the same
// way, as after a barrier -- and then runs the phase it chose.  The host
// enqueues launches ahead in batches and reads the state only between
// batches, so there is no host round trip per iteration, the per-phase
// synchronisation costs one kernel boundary (~2.5 us on MI355X, against
// ~6-10 us for a software barrier over a full persistent grid) and each
// phase runs at the occupancy of its own small register budget.
enum : unsigned {
  PH_PUSH = 0, PH_BALLOT1 = 1, PH_BALLOT2 = 2, PH_PULL_SCAN = 3, PH_PULL_LISTS = 4,
  PH_PULL = 5, PH_DONE = 6, PH_ERROR = 7, PH_LIMIT = 8
};
// seq line layout: [0] phase [1] iteration [2,3] unexplored arcs [4] previous
// frontier size [6,7] activated so far [8] t1 [9] t2 [10] pulling [11] a
// decision is due before the phase
struct SeqState {
  unsigned phase, it, pulling, decide;
  unsigned long long mu, reached;
  unsigned nf_prev, t1, t2;
};
SX_DEV SeqState seq_load(const Line &l) {
  SeqState s;
  s.phase = load_relaxed(&l.v[0]);
  s.it = load_relaxed(&l.v[1]);
  s.mu = load_relaxed((const unsigned long long *)&l.v[2]);
  s.nf_prev = load_relaxed(&l.v[4]);
  s.reached = load_relaxed((const unsigned long long *)&l.v[6]);
  s.t1 = load_relaxed(&l.v[8]);
  s.t2 = load_relaxed(&l.v[9]);
  s.pulling = load_relaxed(&l.v[10]);
  s.decide = load_relaxed(&l.v[11]);
  return s;
}
SX_DEV void seq_store(Line &l, const SeqState &s) {
  store_relaxed(&l.v[0], s.phase);
  store_relaxed(&l.v[1], s.it);
  store_relaxed((unsigned long long *)&l.v[2], s.mu);
  store_relaxed(&l.v[4], s.nf_prev);
  store_relaxed((unsigned long long *)&l.v[6], s.reached);
  store_relaxed(&l.v[8], s.t1);
  store_relaxed(&l.v[9], s.t2);
  store_relaxed(&l.v[10], s.pulling);
  store_relaxed(&l.v[11], s.decide);
}

template <class Ops>
__global__ void __launch_bounds__(kBlock) k_seq(TravArgs a, unsigned L) {
  __shared__ LdsTrav lds;
  __shared__ LdsPolicy pol;
  Ctrl *C = a.w.ctrl;
  const VGrid vg = hw_grid();
  SeqState q = seq_load(C->seq[L & 1]);
  Line &out = C->seq[(L + 1) & 1];
  const bool lead = vg.bid == 0 && threadIdx.x == 0;
  if (q.phase >= PH_DONE) {
    if (lead) seq_store(out, q);
    return;
  }
  if (load_relaxed(&C->error.v[0])) {
    q.phase = PH_ERROR;
    if (lead) seq_store(out, q);
    return;
  }
  RunState s;
  s.it = (int)q.it;
  s.mu = q.mu;
  s.ps.nf_prev = q.nf_prev;
  s.ps.reached = q.reached;
  s.P = a.P;
  if (q.t1) { s.P.t1 = (int)q.t1; s.P.t2 = (int)q.t2; }
  if (q.decide) {
    load_policy(a, pol);
    const bool pulling = q.pulling != 0;
    Decision d = decide<Ops>(a, s, pulling, &pol);
    q.decide = 0;
    if (d.done) {
      q.phase = (s.it + 1 >= a.P.max_iters) ? PH_LIMIT : PH_DONE;
    } else if (!pulling) {
      if (d.to_pull) { q.pulling = 1; q.phase = PH_PULL_SCAN; ++s.it; }
      else if (d.ballot) q.phase = PH_BALLOT1;           // rebuild the lists of it+1
      else { q.phase = PH_PUSH; ++s.it; }
    } else {
      if (d.to_push) {
        q.pulling = 0;
        if (load_relaxed(&C->q[(s.it + 1) % 3].overflow)) q.phase = PH_BALLOT1;
        else { q.phase = PH_PUSH; ++s.it; }
      } else { q.phase = PH_PULL_SCAN; ++s.it; }
    }
    if (q.phase >= PH_DONE) {
      q.it = (unsigned)s.it;
      if (lead) seq_store(out, q);
      return;
    }
  }
  const int it = s.it;
  Ops ops = make_ops<Ops>(a, it);
  unsigned next = q.phase;
  switch (q.phase) {
    case PH_PUSH:
      if (lead) {
        reset_counters(&C->q[(it + 2) % 3]);
        atomic_add_u32(&C->stats.v[6], 1u);
      }
      push_phase(vg, a, s.P, ops, it, lds);
      q.decide = 1;
      break;
    case PH_BALLOT1:
      ballot_pass1(vg, a, s.P, ops, lds);
      next = PH_BALLOT2;
      break;
    case PH_BALLOT2:
      ballot_pass2(vg, a, s.P, it, lds);
      next = PH_PUSH;
      ++s.it;
      break;
    case PH_PULL_SCAN:
      if (lead) {
        reset_counters(&C->q[(it + 1) % 3]);
        reset_counters(&C->q[(it + 2) % 3]);
        atomic_add_u32(&C->stats.v[6], 1u);
      }
      pull_scan(vg, a, s.P, ops, lds);
      next = PH_PULL_LISTS;
      break;
    case PH_PULL_LISTS:
      pull_lists(vg, a, it, lds);
      next = PH_PULL;
      break;
    case PH_PULL:
      pull_phase(vg, a, s.P, ops, it, lds);
      q.decide = 1;
      break;
  }
  if (lead) {
    q.phase = next;
    q.it = (unsigned)s.it;
    q.mu = s.mu;
    q.nf_prev = s.ps.nf_prev;
    q.reached = s.ps.reached;
    q.t1 = (unsigned)s.P.t1;
    q.t2 = (unsigned)s.P.t2;
    seq_store(out, q);
  }
}

// first state of a sequenced run (after k_trav_init)
__global__ void k_seq_start(Ctrl *C, unsigned pull_first) {
  if (threadIdx.x == 0) {
    SeqState q{};
    q.phase = pull_first ? PH_PULL_SCAN : PH_PUSH;
    q.pulling = pull_first;
    q.mu = *(unsigned long long *)&C->state.v[6];
    seq_store(C->seq[0], q);
  }
}

// ------------------------------------------------- batched queries ---
// Many BFS / SSSP queries over graphs of uneven size in one persistent
// launch.  The hardware grid is split into teams of `team` workgroups; each
// team owns a workspace (lists, stamps, bitmaps, control block with its own
// barrier lines) and repeatedly takes the next query from a shared counter
// (queries are ordered largest first), runs it to completion with the same
// push / pull phases, JIT filters and decisions as the single-query kernels
// -- both directions inside one kernel, switching in place -- synchronised by
// a barrier over the team only, then takes the next.  Teams never wait for
// each other, so a 6-level R-MAT query and a 4,000-level grid query overlap.

// Initialise one query on the team: vertex state, stamps, counters, the
// source as the first list.  Ends with a team barrier.
SX_DEV bool batch_init(const VGrid &vg, const TravArgs &a, bool sssp, unsigned long long mu0,
                       GridBarrier &bar) {
  const int n = a.g.n;
  const long long tid = (long long)vg.bid * kBlock + threadIdx.x, nt = (long long)vg.nb * kBlock;
  for (long long v = tid; v < n; v += nt) {
    if (sssp) {
      ((unsigned *)a.state_i)[v] = v == a.src ? 0u : 0xFFFFFFFFu;
      a.w.stamp[v] = v == a.src ? 0 : -1;
    } else {
      a.state_i[v] = v == a.src ? 0 : -1;
    }
  }
  Ctrl *C = a.w.ctrl;
  if (vg.bid == 0 && threadIdx.x == 0) {
    for (int s = 0; s < 3; ++s) reset_counters(&C->q[s]);
    for (int i = 0; i < 32; ++i) {
      store_relaxed(&C->state.v[i], 0u);
      store_relaxed(&C->stats.v[i], 0u);
    }
    store_relaxed((unsigned long long *)&C->state.v[6], mu0);
  }
  if (!bar.sync()) return false;
  if (vg.bid == 0 && threadIdx.x < 64) {
    Lists L = lists_for(a.w, 0, &C->q[0]);
    WaveStats st;
    const bool me = threadIdx.x == 0;
    const int d = me ? degree_of(a.g.off, a.src) : 0;
    online_append(me, a.src, d, L, a.P, a.P.chunk, st);
    flush_stats(st, &C->q[0]);
  }
  return bar.sync();
}

template <class Ops>
SX_DEV bool batch_query(const VGrid &vg, const TravArgs &a, GridBarrier &bar, LdsTrav &lds,
                        LdsPolicy &pol) {
  Ctrl *C = a.w.ctrl;
  RunState s;
  load_state(a, s);
  bool pulling = a.P.direction == 2;
  for (;;) {
    if (!pulling) {
      if (vg.bid == 0 && threadIdx.x == 0) {
        reset_counters(&C->q[(s.it + 2) % 3]);
        atomic_add_u32(&C->stats.v[6], 1u);
      }
      Ops ops = make_ops<Ops>(a, s.it);
      push_phase(vg, a, s.P, ops, s.it, lds);
      if (!bar.sync()) return false;
      if (load_relaxed(&C->error.v[0])) return false;
      Decision d = decide<Ops>(a, s, false, &pol);
      if (d.done) { ++s.it; finish(vg, C, s.it >= a.P.max_iters ? EXIT_LIMIT : EXIT_DONE, s); break; }
      if (d.to_pull) { pulling = true; ++s.it; continue; }
      if (d.ballot) {
        ballot_pass1(vg, a, s.P, ops, lds);
        if (!bar.sync()) return false;
        ballot_pass2(vg, a, s.P, s.it, lds);
        if (!bar.sync()) return false;
      }
      ++s.it;
    } else {
      Ops ops = make_ops<Ops>(a, s.it);
      pull_scan(vg, a, s.P, ops, lds);
      if (!bar.sync()) return false;
      if (vg.bid == 0 && threadIdx.x == 0) {
        reset_counters(&C->q[(s.it + 1) % 3]);
        reset_counters(&C->q[(s.it + 2) % 3]);
        atomic_add_u32(&C->stats.v[6], 1u);
      }
      pull_lists(vg, a, s.it, lds);
      if (!bar.sync()) return false;
      pull_phase(vg, a, s.P, ops, s.it, lds);
      if (!bar.sync()) return false;
      if (load_relaxed(&C->error.v[0])) return false;
      Decision d = decide<Ops>(a, s, true, &pol);
      if (d.done) { ++s.it; finish(vg, C, s.it >= a.P.max_iters ? EXIT_LIMIT : EXIT_DONE, s); break; }
      if (d.to_push) {
        pulling = false;
        if (load_relaxed(&C->q[(s.it + 1) % 3].overflow)) {
          ballot_pass1(vg, a, s.P, ops, lds);
          if (!bar.sync()) return false;
          ballot_pass2(vg, a, s.P, s.it, lds);
          if (!bar.sync()) return false;
        }
      }
      ++s.it;
    }
  }
  return bar.sync();
}

__global__ void __launch_bounds__(kBlock) k_batch(BatchArgs b) {
  __shared__ LdsTrav lds;
  __shared__ LdsPolicy pol;
  const unsigned team = blockIdx.x / (unsigned)b.team;
  const VGrid vg{blockIdx.x % (unsigned)b.team, (unsigned)b.team};
  if (team >= (unsigned)b.nteams) return;
  const Work w = b.work[team];
  Ctrl *C = w.ctrl;
  GridBarrier bar(C, load_relaxed(&C->bar_gen.v[0]), vg);
  TravArgs a;
  a.w = w;
  a.P = b.P;
  a.mlp = b.mlp;
  load_policy(a, pol);
  for (;;) {
    if (vg.bid == 0 && threadIdx.x == 0)
      store_relaxed(&C->aux.v[20], atomic_add_u32(b.queue_head, 1u));
    if (!bar.sync()) break;
    const unsigned qi = load_relaxed(&C->aux.v[20]);
    if (qi >= (unsigned)b.nq) break;
    const BatchQuery Q = b.q[b.order[qi]];
    a.g = Q.g;
    a.state_i = Q.state;
    a.src = Q.src;
    a.P.max_iters = Q.g.n + 2;
    const bool sssp = Q.algo == 1;
    const unsigned long long mu0 = (unsigned long long)(Q.g.m - degree_of(Q.g.off, Q.src));
    if (!batch_init(vg, a, sssp, mu0, bar)) break;
    const bool ok = sssp ? batch_query<SsspOps>(vg, a, bar, lds, pol)
                         : batch_query<BfsOps>(vg, a, bar, lds, pol);
    if (vg.bid == 0 && threadIdx.x == 0) {
      BatchStat &r = b.stats[b.order[qi]];
      r.iterations = (int)load_relaxed(&C->stats.v[6]);
      r.pull_iters = (int)load_relaxed(&C->stats.v[5]);
      r.ballot_iters = (int)load_relaxed(&C->stats.v[4]);
      r.edges = load_relaxed((unsigned long long *)&C->stats.v[0]);
      r.expansions = load_relaxed((unsigned long long *)&C->stats.v[2]);
      r.status = ok ? (int)load_relaxed(&C->state.v[0]) : -1;
      r.team = (int)team;
    }
    if (!ok) break;
  }
}

__global__ void k_batch_reset(BatchArgs b) {
  // barrier generations restart at 0 for every team; the query counter at 0
  const unsigned team = blockIdx.x;
  if (team >= (unsigned)b.nteams) return;
  Ctrl *C = b.work[team].ctrl;
  reset_barrier(C);
  if (threadIdx.x == 0) C->error.v[0] = 0u;
  if (team == 0 && threadIdx.x == 0) *b.queue_head = 0u;
}

// Reset the counters of slot `slot` (one-phase mode; the fused kernels do it
// in place).
__global__ void k_reset_slot(Ctrl *C, int slot) {
  if (threadIdx.x == 0) {
    Counters *q = &C->q[slot];
    for (int b = 0; b < NBINS; ++b) q->cnt[b] = 0;
    q->nf = 0;
    q->mf = 0;
    q->overflow = 0;
  }
}

// ------------------------------------------------------------ set-up ---
// Vertex state initialisation and the source as the first frontier (slot 0,
// parity 0).  BFS: depth = -1, depth[src] = 0.  SSSP: dist = inf,
// dist[src] = 0, stamp = -1, stamp[src] = 0.
__global__ void k_trav_init(TravArgs a, int is_sssp, unsigned long long mu0) {
  const int n = a.g.n;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (long long)gridDim.x * blockDim.x) {
    if (is_sssp) {
      ((unsigned *)a.state_i)[v] = v == a.src ? 0u : 0xFFFFFFFFu;
      a.w.stamp[v] = v == a.src ? 0 : -1;
    } else {
      a.state_i[v] = v == a.src ? 0 : -1;
    }
  }
  if (blockIdx.x == 0) reset_barrier(a.w.ctrl);
  if (blockIdx.x == 0 && threadIdx.x < 64) {
    Ctrl *C = a.w.ctrl;
    if (threadIdx.x == 0) {
      for (int s = 0; s < 3; ++s) {
        for (int b = 0; b < NBINS; ++b) C->q[s].cnt[b] = 0;
        C->q[s].nf = 0;
        C->q[s].mf = 0;
        C->q[s].overflow = 0;
      }
      for (int i = 0; i < 32; ++i) { C->state.v[i] = 0; C->stats.v[i] = 0; }
      C->error.v[0] = 0;
      // arcs not yet explored: all but the source's
      *(unsigned long long *)&C->state.v[6] =
          mu0 ? mu0 : (unsigned long long)(a.g.m - degree_of(a.g.off, a.src));
    }
    __builtin_amdgcn_wave_barrier();
    __threadfence_block();
    Lists L = lists_for(a.w, 0, &a.w.ctrl->q[0]);
    WaveStats st;
    const bool me = threadIdx.x == 0;
    const int d = me ? degree_of(a.g.off, a.src) : 0;
    online_append(me, a.src, d, L, a.P, a.P.chunk, st);
    flush_stats(st, &a.w.ctrl->q[0]);
  }
}

// explicit instantiations used by the host driver
template __global__ void k_push_fused<BfsOps>(TravArgs);
template __global__ void k_pull_fused<BfsOps>(TravArgs);
template __global__ void k_push_fused<SsspOps>(TravArgs);
template __global__ void k_pull_fused<SsspOps>(TravArgs);
template __global__ void k_push_step<BfsOps>(TravArgs, int);
template __global__ void k_push_step<SsspOps>(TravArgs, int);
template __global__ void k_ballot1<BfsOps>(TravArgs, int);
template __global__ void k_ballot1<SsspOps>(TravArgs, int);
template __global__ void k_pull_scan<BfsOps>(TravArgs, int);
template __global__ void k_pull_scan<SsspOps>(TravArgs, int);
template __global__ void k_pull_step<BfsOps>(TravArgs, int);
template __global__ void k_pull_step<SsspOps>(TravArgs, int);

}  // namespace sx

// ------------------------------------------------------ host launchers ---
namespace sx {

const void *trav_kernel(int kind, int sssp) {
  switch (kind) {
    case TK_PUSH_FUSED: return sssp ? (const void *)k_push_fused<SsspOps> : (const void *)k_push_fused<BfsOps>;
    case TK_PULL_FUSED: return sssp ? (const void *)k_pull_fused<SsspOps> : (const void *)k_pull_fused<BfsOps>;
    case TK_PUSH_STEP: return sssp ? (const void *)k_push_step<SsspOps> : (const void *)k_push_step<BfsOps>;
    case TK_BALLOT1: return sssp ? (const void *)k_ballot1<SsspOps> : (const void *)k_ballot1<BfsOps>;
    case TK_BALLOT2: return (const void *)k_ballot2;
    case TK_PULL_SCAN: return sssp ? (const void *)k_pull_scan<SsspOps> : (const void *)k_pull_scan<BfsOps>;
    case TK_PULL_LISTS: return (const void *)k_pull_lists;
    case TK_PULL_STEP: return sssp ? (const void *)k_pull_step<SsspOps> : (const void *)k_pull_step<BfsOps>;
    default: return nullptr;
  }
}

hipError_t trav_launch(int kind, int sssp, const TravArgs &a, int it, int grid, hipStream_t s) {
  const dim3 g(grid), b(kBlock);
  switch (kind) {
    case TK_PUSH_FUSED:
      if (sssp) hipLaunchKernelGGL(k_push_fused<SsspOps>, g, b, 0, s, a);
      else hipLaunchKernelGGL(k_push_fused<BfsOps>, g, b, 0, s, a);
      break;
    case TK_PULL_FUSED:
      if (sssp) hipLaunchKernelGGL(k_pull_fused<SsspOps>, g, b, 0, s, a);
      else hipLaunchKernelGGL(k_pull_fused<BfsOps>, g, b, 0, s, a);
      break;
    case TK_PUSH_STEP:
      if (sssp) hipLaunchKernelGGL(k_push_step<SsspOps>, g, b, 0, s, a, it);
      else hipLaunchKernelGGL(k_push_step<BfsOps>, g, b, 0, s, a, it);
      break;
    case TK_BALLOT1:
      if (sssp) hipLaunchKernelGGL(k_ballot1<SsspOps>, g, b, 0, s, a, it);
      else hipLaunchKernelGGL(k_ballot1<BfsOps>, g, b, 0, s, a, it);
      break;
    case TK_BALLOT2: hipLaunchKernelGGL(k_ballot2, g, b, 0, s, a, it); break;
    case TK_PULL_SCAN:
      if (sssp) hipLaunchKernelGGL(k_pull_scan<SsspOps>, g, b, 0, s, a, it);
      else hipLaunchKernelGGL(k_pull_scan<BfsOps>, g, b, 0, s, a, it);
      break;
    case TK_PULL_LISTS: hipLaunchKernelGGL(k_pull_lists, g, b, 0, s, a, it); break;
    case TK_PULL_STEP:
      if (sssp) hipLaunchKernelGGL(k_pull_step<SsspOps>, g, b, 0, s, a, it);
      else hipLaunchKernelGGL(k_pull_step<BfsOps>, g, b, 0, s, a, it);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t trav_init(const TravArgs &a, int sssp, unsigned long long mu0, hipStream_t s) {
  int grid = (a.g.n + kBlock - 1) / kBlock;
  if (grid < 1) grid = 1;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_trav_init, dim3(grid), dim3(kBlock), 0, s, a, sssp, mu0);
  return hipGetLastError();
}

hipError_t seq_start(Ctrl *c, bool pull_first, hipStream_t s) {
  hipLaunchKernelGGL(k_seq_start, dim3(1), dim3(64), 0, s, c, pull_first ? 1u : 0u);
  return hipGetLastError();
}

hipError_t seq_launch(int sssp, const TravArgs &a, unsigned L, int grid, hipStream_t s) {
  if (sssp) hipLaunchKernelGGL(k_seq<SsspOps>, dim3(grid), dim3(kBlock), 0, s, a, L);
  else hipLaunchKernelGGL(k_seq<BfsOps>, dim3(grid), dim3(kBlock), 0, s, a, L);
  return hipGetLastError();
}

const void *seq_kernel(int sssp) {
  return sssp ? (const void *)k_seq<SsspOps> : (const void *)k_seq<BfsOps>;
}

hipError_t batch_launch(const BatchArgs &b, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reset, dim3(b.nteams), dim3(256), 0, s, b);
  hipLaunchKernelGGL(k_batch, dim3(grid), dim3(kBlock), 0, s, b);
  return hipGetLastError();
}

const void *batch_kernel() { return (const void *)k_batch; }

hipError_t reset_slot(Ctrl *c, int slot, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_slot, dim3(1), dim3(64), 0, s, c, slot);
  return hipGetLastError();
}

}  // namespace sx
