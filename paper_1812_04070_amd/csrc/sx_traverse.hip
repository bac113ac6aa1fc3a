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
SX_PHASE void push_phase(const TravArgs &a, const Ops &ops, int it, LdsTrav &lds) {
  Ctrl *C = a.w.ctrl;
  Counters *cur = &C->q[it % 3], *nxt = &C->q[(it + 1) % 3];
  // counts are clamped to the list capacities: reads never leave the lists
  const unsigned cs = min(load_relaxed(&cur->cnt[0]), a.w.qcap_small),
                 cm = min(load_relaxed(&cur->cnt[1]), a.w.qcap_med),
                 cl = min(load_relaxed(&cur->cnt[2]), a.w.qcap_large);
  const int p = it & 1;
  Lists NL = lists_for(a.w, p ^ 1, nxt);
  NL.cap_s = online_cap(a.w, a.P, 0);
  NL.cap_m = online_cap(a.w, a.P, 1);
  NL.cap_l = online_cap(a.w, a.P, 2);
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
    online_append(act, u, du, NL, a.P, a.P.chunk, st);
  };
  const unsigned gw = blockIdx.x * kWaves + wave_in_wg();
  const unsigned nw = gridDim.x * kWaves;
  visit_large(a.w.ql[p], cl, g.off, g.idx, a.P.chunk, op);
  visit_med(a.w.q[p][1], cm, g.off, g.idx, op, gw, nw);
  visit_small(a.w.q[p][0], cs, g.off, g.idx, op, gw, nw, lds.small[wave_in_wg()]);
  flush_stats(st, nxt);
  const long long e = wave_sum_ll(edges);
  if (lane_id() == 0) {
    if (e) atomic_add_u64((unsigned long long *)&C->stats.v[0], (unsigned long long)e);
    if (err) store_relaxed(&C->error.v[0], err);
  }
  // worklist entries processed this iteration (vertex expansions)
  if (blockIdx.x == 0 && threadIdx.x == 0)
    atomic_add_u64((unsigned long long *)&C->stats.v[2], (unsigned long long)(cs + cm) + cl);
}

// --------------------------------------------------------- ballot filter ---
// Rebuild the next lists (parity it+1) from vertex metadata: pass 1 counts.
template <class Ops>
SX_PHASE void ballot_pass1(const TravArgs &a, const Ops &ops, LdsTrav &lds) {
  const Work &w = a.w;
  Tiling T(a.g.n, gridDim.x * kWaves);
  const int *off = a.g.off;
  auto pred = [&](int v) { return ops.next_active(v); };
  auto deg = [&](int v) { return degree_of(off, v); };
  ballot_count(a.g.n, T, pred, deg, a.P, a.P.chunk, w.bits, w.wavecnt, w.wgc, lds.cnt);
}

// pass 2 writes the sorted lists and (workgroup 0) their counts.
SX_PHASE void ballot_pass2(const TravArgs &a, int it, LdsTrav &lds) {
  const Work &w = a.w;
  Tiling T(a.g.n, gridDim.x * kWaves);
  const int *off = a.g.off;
  auto deg = [&](int v) { return degree_of(off, v); };
  const int p = (it + 1) & 1;
  WgCount tot;
  auto ident = [](int i) { return i; };
  ballot_write(a.g.n, T, deg, ident, a.P.chunk, w.bits, w.wavecnt, w.wgc,
               w.q[p][0], w.q[p][1], w.ql[p], tot, lds.cnt, lds.red);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
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
SX_PHASE void pull_scan(const TravArgs &a, const Ops &ops, LdsTrav &lds) {
  const Work &w = a.w;
  Tiling T(a.g.n, gridDim.x * kWaves);
  const int *off = a.g.in_off;
  const int n = a.g.n;
  // frontier words
  {
    const unsigned gw = blockIdx.x * kWaves + wave_in_wg();
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
  Params P = a.P;
  ballot_count(n, T, pred, deg, P, 0x7fffffff, w.bits, w.wavecnt, w.wgc, lds.cnt);
}

// Write the candidate lists into the parity-`it` buffers (not read by anyone
// else in a pull iteration); counts go to slot it.
SX_PHASE void pull_lists(const TravArgs &a, int it, LdsTrav &lds) {
  const Work &w = a.w;
  Tiling T(a.g.n, gridDim.x * kWaves);
  const int *off = a.g.in_off;
  auto deg = [&](int v) { return degree_of(off, v); };
  const int p = it & 1;
  WgCount tot;
  auto ident = [](int i) { return i; };
  ballot_write(a.g.n, T, deg, ident, 0x7fffffff, w.bits, w.wavecnt, w.wgc,
               w.q[p][0], w.q[p][1], w.ql[p], tot, lds.cnt, lds.red);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
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
SX_PHASE void pull_phase(const TravArgs &a, const Ops &ops, int it, LdsTrav &lds) {
  Ctrl *C = a.w.ctrl;
  Counters *cur = &C->q[it % 3], *nxt = &C->q[(it + 1) % 3];
  // counts are clamped to the list capacities: reads never leave the lists
  const unsigned cs = min(load_relaxed(&cur->cnt[0]), a.w.qcap_small),
                 cm = min(load_relaxed(&cur->cnt[1]), a.w.qcap_med),
                 cl = min(load_relaxed(&cur->cnt[2]), a.w.qcap_large);
  const int p = it & 1;
  Lists NL = lists_for(a.w, p ^ 1, nxt);
  NL.cap_s = online_cap(a.w, a.P, 0);
  NL.cap_m = online_cap(a.w, a.P, 1);
  NL.cap_l = online_cap(a.w, a.P, 2);
  const DevGraph &g = a.g;
  const unsigned long long *fb = a.w.fbits;
  WaveStats st;
  long long edges = 0;
  const int lane = lane_id();
  const unsigned gw = blockIdx.x * kWaves + wave_in_wg();
  const unsigned nw = gridDim.x * kWaves;
  // One workgroup per large candidate
  for (unsigned i = blockIdx.x; i < cl; i += gridDim.x) {
    const int v = (int)(a.w.ql[p][i] & 0xffffffffu);
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
    if (wave_in_wg() == 0) online_append(act, v, end - beg, NL, a.P, a.P.chunk, st);
  }
  // One wavefront per medium candidate
  for (unsigned i = gw; i < cm; i += nw) {
    const int v = a.w.q[p][1][i];
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
    online_append(act, v, end - beg, NL, a.P, a.P.chunk, st);
  }
  // One lane per small candidate
  for (unsigned c0 = gw * 64u; c0 < cs; c0 += nw * 64u) {
    const unsigned i = c0 + lane;
    bool act = false;
    int v = 0, d = 0;
    if (i < cs) {
      v = a.w.q[p][0][i];
      const int beg = g.in_off[v], end = g.in_off[v + 1];
      d = end - beg;
      if (Ops::kVote) {
        for (int arc = beg; arc < end; ++arc) {
          ++edges;
          if (fbit(fb, g.in_idx[arc])) { act = true; break; }
        }
        if (act) store_relaxed(&a.state_i[v], it + 1);
      } else {
        unsigned best = load_relaxed(&((unsigned *)a.state_i)[v]);
        const unsigned old = best;
        for (int arc = beg; arc < end; ++arc) {
          ++edges;
          const int u = g.in_idx[arc];
          if (fbit(fb, u)) {
            const unsigned c = load_relaxed(&((unsigned *)a.state_i)[u]) + g.in_w[arc];
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
    online_append(act, v, d, NL, a.P, a.P.chunk, st);
  }
  flush_stats(st, nxt);
  const long long e = wave_sum_ll(edges);
  if (lane == 0 && e) atomic_add_u64((unsigned long long *)&C->stats.v[0], (unsigned long long)e);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    atomic_add_u64((unsigned long long *)&C->stats.v[2], (unsigned long long)(cs + cm) + cl);
    atomic_add_u32(&C->stats.v[5], 1u);
  }
}

// --------------------------------------------------------- decisions ---
template <class Ops>
SX_DEV Decision decide(const TravArgs &a, int it, bool pulling, unsigned long long &mu) {
  Counters *nxt = &a.w.ctrl->q[(it + 1) % 3];
  DecideIn in;
  in.nf = load_relaxed(&nxt->nf);
  in.mf = load_relaxed(&nxt->mf);
  in.ovf = load_relaxed(&nxt->overflow);
  in.it = it;
  in.pulling = pulling;
  in.vote = Ops::kVote;
  in.n = a.g.n;
  in.m = a.g.m;
  return decide_core(in, a.P, mu);
}

SX_DEV void finish(Ctrl *C, int reason, int it, unsigned long long mu) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    store_relaxed(&C->state.v[0], (unsigned)reason);
    store_relaxed(&C->state.v[1], (unsigned)it);
    store_relaxed((unsigned long long *)&C->state.v[6], mu);
  }
}

template <class Ops>
SX_DEV Ops make_ops(const TravArgs &a, int it);
template <>
SX_DEV BfsOps make_ops<BfsOps>(const TravArgs &a, int it) { return BfsOps{a.state_i, it}; }
template <>
SX_DEV SsspOps make_ops<SsspOps>(const TravArgs &a, int it) {
  return SsspOps{(unsigned *)a.state_i, a.w.stamp, it};
}

// -------------------------------------------------- persistent kernels ---
template <class Ops>
__global__ void __launch_bounds__(kBlock) k_push_fused(TravArgs a) {
  __shared__ LdsTrav lds;
  Ctrl *C = a.w.ctrl;
  GridBarrier bar(C, load_relaxed(&C->bar_gen.v[0]));
  int it = (int)load_relaxed(&C->state.v[1]);
  unsigned long long mu = load_relaxed((unsigned long long *)&C->state.v[6]);
  const unsigned entry = load_relaxed(&C->state.v[0]);
  if (entry == EXIT_DONE || entry == EXIT_LIMIT || entry == EXIT_ERROR || bar.failed()) return;
  // a list that overflowed while pulling is rebuilt before the first push
  if (load_relaxed(&C->q[it % 3].overflow)) {
    Ops ops = make_ops<Ops>(a, it - 1);
    ballot_pass1(a, ops, lds);
    if (!bar.sync()) { finish(C, EXIT_ERROR, it, mu); return; }
    ballot_pass2(a, it - 1, lds);
    if (!bar.sync()) { finish(C, EXIT_ERROR, it, mu); return; }
  }
  for (;;) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      Counters *old = &C->q[(it + 2) % 3];
      for (int b = 0; b < NBINS; ++b) store_relaxed(&old->cnt[b], 0u);
      store_relaxed(&old->nf, 0u);
      store_relaxed(&old->mf, 0ull);
      store_relaxed(&old->overflow, 0u);
      atomic_add_u32(&C->stats.v[6], 1u);
    }
    Ops ops = make_ops<Ops>(a, it);
    push_phase(a, ops, it, lds);
    if (!bar.sync()) { finish(C, EXIT_ERROR, it, mu); return; }
    if (load_relaxed(&C->error.v[0])) { finish(C, EXIT_ERROR, it, mu); return; }
    Decision d = decide<Ops>(a, it, false, mu);
    if (d.done && it + 1 >= a.P.max_iters) { finish(C, EXIT_LIMIT, it + 1, mu); return; }
    if (d.done) { finish(C, EXIT_DONE, it + 1, mu); return; }
    if (d.to_pull) { finish(C, EXIT_SWITCH, it + 1, mu); return; }
    if (d.ballot) {
      ballot_pass1(a, ops, lds);
      if (!bar.sync()) { finish(C, EXIT_ERROR, it, mu); return; }
      ballot_pass2(a, it, lds);
      if (!bar.sync()) { finish(C, EXIT_ERROR, it, mu); return; }
    }
    ++it;
  }
}

template <class Ops>
__global__ void __launch_bounds__(kBlock) k_pull_fused(TravArgs a) {
  __shared__ LdsTrav lds;
  Ctrl *C = a.w.ctrl;
  GridBarrier bar(C, load_relaxed(&C->bar_gen.v[0]));
  int it = (int)load_relaxed(&C->state.v[1]);
  unsigned long long mu = load_relaxed((unsigned long long *)&C->state.v[6]);
  const unsigned entry = load_relaxed(&C->state.v[0]);
  if (entry == EXIT_DONE || entry == EXIT_LIMIT || entry == EXIT_ERROR || bar.failed()) return;
  for (;;) {
    Ops ops = make_ops<Ops>(a, it);
    pull_scan(a, ops, lds);
    if (!bar.sync()) { finish(C, EXIT_ERROR, it, mu); return; }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      Counters *nx = &C->q[(it + 1) % 3];
      for (int b = 0; b < NBINS; ++b) store_relaxed(&nx->cnt[b], 0u);
      store_relaxed(&nx->nf, 0u);
      store_relaxed(&nx->mf, 0ull);
      store_relaxed(&nx->overflow, 0u);
      atomic_add_u32(&C->stats.v[6], 1u);
    }
    pull_lists(a, it, lds);
    if (!bar.sync()) { finish(C, EXIT_ERROR, it, mu); return; }
    pull_phase(a, ops, it, lds);
    if (!bar.sync()) { finish(C, EXIT_ERROR, it, mu); return; }
    if (load_relaxed(&C->error.v[0])) { finish(C, EXIT_ERROR, it, mu); return; }
    Decision d = decide<Ops>(a, it, true, mu);
    if (d.done && it + 1 >= a.P.max_iters) { finish(C, EXIT_LIMIT, it + 1, mu); return; }
    if (d.done) { finish(C, EXIT_DONE, it + 1, mu); return; }
    if (d.to_push) { finish(C, EXIT_SWITCH, it + 1, mu); return; }
    ++it;
  }
}

// ------------------------------------------------ one-phase kernels ---
// The same phases, one launch each; the host reads the counters between
// launches and takes the decisions (no fusion).
template <class Ops>
__global__ void __launch_bounds__(kBlock) k_push_step(TravArgs a, int it) {
  __shared__ LdsTrav lds;
  Ops ops = make_ops<Ops>(a, it);
  push_phase(a, ops, it, lds);
}
template <class Ops>
__global__ void __launch_bounds__(kBlock) k_ballot1(TravArgs a, int it) {
  __shared__ LdsTrav lds;
  Ops ops = make_ops<Ops>(a, it);
  ballot_pass1(a, ops, lds);
}
__global__ void __launch_bounds__(kBlock) k_ballot2(TravArgs a, int it) {
  __shared__ LdsTrav lds;
  ballot_pass2(a, it, lds);
}
template <class Ops>
__global__ void __launch_bounds__(kBlock) k_pull_scan(TravArgs a, int it) {
  __shared__ LdsTrav lds;
  Ops ops = make_ops<Ops>(a, it);
  pull_scan(a, ops, lds);
}
__global__ void __launch_bounds__(kBlock) k_pull_lists(TravArgs a, int it) {
  __shared__ LdsTrav lds;
  pull_lists(a, it, lds);
}
template <class Ops>
__global__ void __launch_bounds__(kBlock) k_pull_step(TravArgs a, int it) {
  __shared__ LdsTrav lds;
  Ops ops = make_ops<Ops>(a, it);
  pull_phase(a, ops, it, lds);
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
      *(unsigned long long *)&C->state.v[6] = mu0;
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

hipError_t reset_slot(Ctrl *c, int slot, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_slot, dim3(1), dim3(64), 0, s, c, slot);
  return hipGetLastError();
}

}  // namespace sx
