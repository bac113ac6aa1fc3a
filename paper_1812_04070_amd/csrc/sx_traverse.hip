// Frontier traversal engine for BFS and SSSP: the ACC processing loop of
// Section 3.3 (compute on the small / medium / large lists, combine, record
// active vertices, synchronise, overflow check, next lists) with the
// just-in-time task management of Section 4 and the push/pull kernel fusion
// of Section 5.
//
// Each algorithm is an ACC triple (Section 3.2):
//   BFS   Active: depth == level + 1 (newly visited).  Compute: level + 1.
//         Combine: vote -- any single update is correct, so push claims an
//         unvisited vertex with one compare-and-swap and pull stops at the
//         first in-neighbour found in the frontier (collaborative early
//         termination, Section 3.3).
//   SSSP  Active: distance lowered in the previous iteration (Figure
//         tech-compute(a)).  Compute: dist(v) + w(v,u).  Combine: minimum
//         (aggregation): push lowers dist(u) with an atomic minimum, pull
//         reduces over the in-arcs and the single owner writes, no atomics.
//   WCC   (connected components, Section 3.2) Active: label lowered in the
//         previous iteration; every vertex at the start, with its own id as
//         label.  Compute: label(v).  Combine: minimum, as for SSSP.  At the
//         fixpoint every vertex holds the smallest id of its component.
//
// The same phases run in four arrangements:
//   fused      persistent kernels, one per direction, iterating until the
//              frontier empties or the direction changes, phases separated by
//              the software global barrier (the paper's design, Section 5);
//   one-phase  one launch per phase, the host reading the records and
//              deciding between launches (the paper's no-fusion baseline);
//   sequenced  one launch per phase, the decision taken on the device at the
//              start of the next launch, launches enqueued ahead by the host;
//   batched    many queries, each run by a team of workgroups (k_batch).
//
// Worklist bookkeeping (sx_frontier.hpp): record slot it % 3 holds the lists
// the online filter built for iteration it (parity it & 1 of the region
// arrays); slot SLOT_SCAN the lists of the last ballot scan (a rebuild of the
// push lists, or the pull candidates).
#include "sx_frontier.hpp"
#include "sx_kernels.hpp"
#include "sx_policy.hpp"

namespace sx {

#define SX_PHASE __device__ __forceinline__

// ------------------------------------------------------------- ACC ops ---
struct BfsOps {
  static constexpr bool kVote = true;
  static constexpr bool kWeighted = false;
  int *depth;
  int it;
  // push Compute + Combine for kIlp arcs v->u per lane; act[r]: u becomes
  // active.  All depth loads, then all claims, are in flight together.
  SX_DEV void push(const int *v, const int *u, const int *arc, const bool *ok, const DevGraph &g,
                   unsigned &err, bool *act, unsigned &lowest) const {
    (void)v; (void)arc; (void)g; (void)err; (void)lowest;
    int d[kIlp], got[kIlp];
#pragma unroll
    for (int r = 0; r < kIlp; ++r) d[r] = ok[r] ? depth[u[r]] : 0;
#pragma unroll
    for (int r = 0; r < kIlp; ++r)
      got[r] = ok[r] && d[r] == -1 ? atomic_cas_old_i32(&depth[u[r]], -1, it + 1) : 0;
#pragma unroll
    for (int r = 0; r < kIlp; ++r) act[r] = ok[r] && d[r] == -1 && got[r] == -1;
  }
  SX_DEV bool next_active(int v) const { return depth[v] == it + 1; }
  SX_DEV bool in_frontier(int v) const { return depth[v] == it; }
  SX_DEV bool pull_candidate(int v) const { return depth[v] == -1; }
};

struct SsspOps {
  static constexpr bool kVote = false;
  static constexpr bool kWeighted = true;
  unsigned *dist;
  int *stamp;
  int it;
  // relax kIlp arcs per lane: loads, then the atomic minimums, then the
  // stamps of the improved targets, each stage with all arcs in flight;
  // `lowest` keeps the smallest distance this lane set
  SX_DEV void push(const int *v, const int *u, const int *arc, const bool *ok, const DevGraph &g,
                   unsigned &err, bool *act, unsigned &lowest) const {
    unsigned dv[kIlp], w[kIlp], du[kIlp], nd[kIlp], old[kIlp];
    bool tr[kIlp];
#pragma unroll
    for (int r = 0; r < kIlp; ++r) {
      dv[r] = ok[r] ? dist[v[r]] : 0u;
      w[r] = ok[r] ? g.w[arc[r]] : 0u;
      du[r] = ok[r] ? dist[u[r]] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kIlp; ++r) {
      nd[r] = dv[r] + w[r];
      const bool bad = nd[r] < dv[r] || nd[r] == 0xFFFFFFFFu;
      if (ok[r] && bad) err = SX_ERR_OVERFLOW;
      tr[r] = ok[r] && !bad && nd[r] < du[r];
      old[r] = tr[r] ? atomic_min_u32(&dist[u[r]], nd[r]) : 0u;
    }
    int st[kIlp];
#pragma unroll
    for (int r = 0; r < kIlp; ++r) {
      tr[r] = tr[r] && nd[r] < old[r];
      st[r] = tr[r] ? atomic_exch_i32(&stamp[u[r]], it + 1) : 0;
      if (tr[r] && nd[r] < lowest) lowest = nd[r];
    }
#pragma unroll
    for (int r = 0; r < kIlp; ++r) act[r] = tr[r] && st[r] != it + 1;
  }
  SX_DEV bool next_active(int v) const { return stamp[v] == it + 1; }
  SX_DEV bool in_frontier(int v) const { return stamp[v] == it; }
  SX_DEV bool pull_candidate(int v) const { (void)v; return true; }
};

// Minimum-label propagation: the SSSP relaxation with a zero arc weight (the
// label a vertex offers is its own), so labels never overflow.
struct WccOps {
  static constexpr bool kVote = false;
  static constexpr bool kWeighted = false;
  unsigned *dist;               // labels
  int *stamp;
  int it;
  SX_DEV void push(const int *v, const int *u, const int *arc, const bool *ok, const DevGraph &g,
                   unsigned &err, bool *act, unsigned &lowest) const {
    (void)arc; (void)g; (void)err; (void)lowest;
    unsigned lv[kIlp], lu[kIlp], old[kIlp];
    bool tr[kIlp];
#pragma unroll
    for (int r = 0; r < kIlp; ++r) {
      lv[r] = ok[r] ? dist[v[r]] : 0u;
      lu[r] = ok[r] ? dist[u[r]] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kIlp; ++r) {
      tr[r] = ok[r] && lv[r] < lu[r];
      old[r] = tr[r] ? atomic_min_u32(&dist[u[r]], lv[r]) : 0u;
    }
    int st[kIlp];
#pragma unroll
    for (int r = 0; r < kIlp; ++r) {
      tr[r] = tr[r] && lv[r] < old[r];
      st[r] = tr[r] ? atomic_exch_i32(&stamp[u[r]], it + 1) : 0;
    }
#pragma unroll
    for (int r = 0; r < kIlp; ++r) act[r] = tr[r] && st[r] != it + 1;
  }
  SX_DEV bool next_active(int v) const { return stamp[v] == it + 1; }
  SX_DEV bool in_frontier(int v) const { return stamp[v] == it; }
  SX_DEV bool pull_candidate(int v) const { (void)v; return true; }
};

SX_DEV int degree_of(const int *off, int v) { return off[v + 1] - off[v]; }

// What a frontier neighbour u offers v over arc `arc` in a pull step: its
// distance plus the arc weight (SSSP; err on a sum that reaches infinity) or
// its label (WCC).
template <class Ops>
SX_DEV unsigned pull_offer(const unsigned *dist, const DevGraph &g, int u, int arc, unsigned &err) {
  const unsigned du = dist[u];
  if constexpr (!Ops::kWeighted) {
    (void)g; (void)arc; (void)err;
    return du;
  } else {
    const unsigned c = du + g.in_w[arc];
    if (c < du || c == 0xFFFFFFFFu) {
      err = SX_ERR_OVERFLOW;
      return 0xFFFFFFFFu;
    }
    return c;
  }
}

struct LdsTrav {
  int small[kWaves][192];
  LdsBins bins;
  LdsView view;
  LdsBallot ball;
  long long red[kWaves];
  unsigned cnt[kWaves];
  unsigned sq[33];                 // the run-state line and the error word
  unsigned skip;                   // push step: the current large item is skipped
};

SX_DEV void raise_error(Ctrl *C, unsigned e) { store_relaxed(&C->error.v[0], e); }

// --------------------------------------------------------- push phase ---
// Compute + combine over the current lists (view `cur`, totals T); the
// online filter records the activated vertices into slot it+1 (parity it+1).
//
// Delta-stepping (SSSP, bound B below 0xFFFFFFFF; Section 3.3 of the paper
// adopts it to widen the set of vertices relaxed together): only list
// vertices with distance < B are expanded; the others are carried into the
// next lists unexpanded (stamped as active for iteration it+1, so a ballot
// rebuild finds them too).  Distances only fall, so a vertex read as far by
// the carrying pass and as near by its visitor is both carried and expanded
// (redundant, never lost).  The smallest distance set or carried in the
// step goes to Ctrl::aux[(it+1) % 3], from which the next decision moves B.
constexpr unsigned kDedupMinList = 1u << 16;

template <class Ops, bool kDedup = true>
SX_PHASE void push_phase(const VGrid &vg, const TravArgs &a, const Params &P, const Ops &ops, int it,
                         const ViewRef &cur, const Totals &T, LdsTrav &lds,
                         unsigned B = 0xFFFFFFFFu) {
  const DevGraph &g = a.g;
  const Regions NR = regions(a.w, (it + 1) & 1, vg.nb);
  bins_begin(lds.bins, NR, P.online_cap);
  WaveStats st;
  unsigned err = 0;
  long long edges = 0;
  unsigned lowest = 0xFFFFFFFFu;
  const bool buckets = !Ops::kVote && B != 0xFFFFFFFFu;
  // the smallest distance is also kept before the buckets engage
  const bool record = !Ops::kVote && P.delta != 0u;
  // a far vertex (distance >= B) reads as -1, which every visitor skips
  auto near = [&](int v) -> int {
    if constexpr (Ops::kVote) {
      return v;
    } else {
      return buckets && (unsigned)v < (unsigned)g.n && ops.dist[v] >= B ? -1 : v;
    }
  };
  // A listed vertex whose value equals the one its last expansion started
  // from is skipped (reads as -1): that expansion recorded the value before
  // relaxing any arc and read the source value of each arc afterwards, and
  // values only fall, so every arc was relaxed with exactly this value.  A
  // vertex improved while listed, before its own expansion, is expanded
  // with the new value and listed again for the next step, where it is
  // skipped (R-MAT s22 SSSP: a third of the expansions).  Only the small and
  // medium visitors (one expander per vertex) record and skip; `writer` is
  // the lane whose result the visitor uses.  Only steps with long lists do
  // (kDedupMinList), on graphs of 8+ arcs per vertex (the host passes no
  // record otherwise): the
  // test puts a dependent load before each row's, which the thousands of
  // short steps of a high-diameter graph would each pay, and sparse graphs
  // re-improve their vertices with new values, not the same one (a record
  // left stale by a step without it only holds a value above the vertex's
  // current one, so it never matches).  The batched kernel
  // compiles it out (kDedup false): its spilling register budget would pay
  // for it in every step.
  const bool dedup = kDedup && !Ops::kVote && a.xdist && T.nf >= kDedupMinList;
  auto fresh = [&](int v, bool writer) -> int {
    if constexpr (Ops::kVote) {
      return v;
    } else {
      if (!dedup || !writer || (unsigned)v >= (unsigned)g.n) return v;
      const unsigned d = ops.dist[v];
      if (a.xdist[v] == d) return -1;
      a.xdist[v] = d;
      return v;
    }
  };
  if constexpr (!Ops::kVote) {
    if (buckets) {
      const unsigned cs = T.cnt[BIN_SMALL], cm = T.cnt[BIN_MED], cl = T.cnt[BIN_LARGE];
      const unsigned total = cs + cm + cl;
      const unsigned tid = vg.bid * kBlock + threadIdx.x, nt = vg.nb * kBlock;
      // wave-uniform trip count: all lanes take part in the appends
      for (unsigned base = tid - lane_id(); base < total; base += nt) {
        const unsigned i = base + lane_id();
        bool carry = false;
        int v = -1;
        if (i < total) {
          unsigned long long item;
          if (i < cs) item = (unsigned)cur.small(i);
          else if (i < cs + cm) item = (unsigned)cur.med(i - cs);
          else item = cur.large(i - cs - cm);
          v = (int)(item & 0xffffffffu);
          const bool first = i < cs + cm || (item >> 32) == 0;   // one chunk per vertex
          if (first && (unsigned)v < (unsigned)g.n) {
            const unsigned d = ops.dist[v];
            if (d >= B) {
              if (d < lowest) lowest = d;
              carry = atomic_exch_i32(&ops.stamp[v], it + 1) != it + 1;
            }
          }
        }
        const int dv = carry ? degree_of(g.off, v) : 0;
        bins_append(carry, v, dv, NR, vg.bid, P, P.chunk, lds.bins, st);
      }
    }
  }
  auto op = [&](const int *v, const int *u, const int *arc, const bool *ok) {
    bool act[kIlp];
    ops.push(v, u, arc, ok, g, err, act, lowest);
    int du[kIlp];
#pragma unroll
    for (int r = 0; r < kIlp; ++r) {
      edges += ok[r] ? 1 : 0;
      du[r] = act[r] ? degree_of(g.off, u[r]) : 0;
    }
#pragma unroll
    for (int r = 0; r < kIlp; ++r) bins_append(act[r], u[r], du[r], NR, vg.bid, P, P.chunk, lds.bins, st);
  };
  const unsigned gw = vg.bid * kWaves + wave_in_wg();
  const unsigned nw = vg.nb * kWaves;
  // (the medium and large visitors call their accessor with every lane of a
  // wavefront on one entry: lane 0's reading decides for the wavefront)
  // The large bin records per chunk (each chunk has one expanding workgroup
  // per step): thread 0 takes the decision for the whole workgroup between
  // two barriers, so that the record is written before any wavefront reads
  // the source value and every wavefront follows it.  Not with buckets
  // (whose near / far test each wavefront takes for itself).
  const bool cdedup = dedup && !buckets && P.chunk == kChunk;
  visit_large(vg, g.n,
              [&](unsigned i) {
                unsigned long long x = cur.large(i);
                if (buckets) {
                  const int far = __shfl(near((int)(x & 0xffffffffu)) < 0 ? 1 : 0, 0);
                  if (far) x |= 0xffffffffull;
                }
                if constexpr (!Ops::kVote) {
                  if (cdedup) {
                    __syncthreads();   // every wavefront has read the last item's decision
                    if (threadIdx.x == 0) {
                      unsigned sk = 0;
                      const int v = (int)(x & 0xffffffffu);
                      if ((unsigned)v < (unsigned)g.n) {
                        const unsigned d = ops.dist[v];
                        unsigned *rec = a.xdist + g.n + (size_t)(g.off[v] / kChunk) + (size_t)(x >> 32) + (size_t)v;
                        if (*rec == d) sk = 1;
                        else *rec = d;
                      }
                      lds.skip = sk;
                    }
                    __syncthreads();
                    if (lds.skip) x |= 0xffffffffull;
                  }
                }
                return x;
              },
              T.cnt[BIN_LARGE], g.off, g.idx, P.chunk, op);
  visit_med(g.n,
            [&](unsigned i) {
              const int v = cur.med(i);
              if constexpr (Ops::kVote) return v;
              if (!buckets && !dedup) return v;
              return __shfl(fresh(near(v), lane_id() == 0), 0);
            },
            T.cnt[BIN_MED], g.off, g.idx, op, gw, nw);
  visit_small(g.n, [&](unsigned i) { return fresh(near(cur.small(i)), true); }, T.cnt[BIN_SMALL], g.off,
              g.idx, op, gw, nw, lds.small[wave_in_wg()]);
  bins_end(lds.bins, st, a.w.rec + ((it + 1) % 3), vg.bid);   // ends with a barrier
  if (record) {
    const unsigned m = wave_min_u(lowest);
    if (lane_id() == 0) lds.cnt[wave_in_wg()] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned x = 0xFFFFFFFFu;
      for (int w2 = 0; w2 < kWaves; ++w2) x = lds.cnt[w2] < x ? lds.cnt[w2] : x;
      if (x != 0xFFFFFFFFu) atomic_min_u32(&a.w.ctrl->aux.v[(it + 1) % 3], x);
      // the word step it+1 lowers; its last reader was the decision before
      // this step
      if (vg.bid == 0) store_relaxed(&a.w.ctrl->aux.v[(it + 2) % 3], 0xFFFFFFFFu);
    }
  }
  if (err) raise_error(a.w.ctrl, err);
  add_stats(a.w.ctrl, vg.bid, edges,
            vg.bid == 0 ? (unsigned long long)T.cnt[0] + T.cnt[1] + T.cnt[2] : 0ull, lds.red);
}

// --------------------------------------------------------- ballot filter ---
// Rebuild the lists of iteration it+1 (parity it+1) from vertex metadata,
// sorted and unique, into slot SLOT_SCAN.
template <class Ops>
SX_PHASE void ballot_next(const VGrid &vg, const TravArgs &a, const Params &P, const Ops &ops, int it,
                          LdsTrav &lds) {
  const Work &w = a.w;
  const int *off = a.g.off;
  auto pred = [&](int v) { return ops.next_active(v); };
  auto deg = [&](int v) { return degree_of(off, v); };
  auto ident = [](int i) { return i; };
  const Regions R = regions(w, (it + 1) & 1, vg.nb);
  ballot_fill(vg, a.g.n, pred, deg, ident, P, P.chunk, w.bits, R,
              w.rec + SLOT_SCAN, lds.ball);
  if (vg.bid == 0 && threadIdx.x == 0) atomic_add_u32(&w.ctrl->stats.v[4], 1u);
}

// ----------------------------------------------------------- pull phases ---
// Scan: the frontier bitmap of iteration it, and the sorted candidate lists
// (vertices that may still change, binned by in-degree, one item each) into
// parity it, slot SLOT_SCAN.
template <class Ops>
SX_PHASE void pull_scan(const VGrid &vg, const TravArgs &a, const Params &P, const Ops &ops, int it,
                        LdsTrav &lds) {
  const Work &w = a.w;
  const int *off = a.g.in_off;
  const int n = a.g.n;
  {
    const long long tiles = ((long long)n + 63) / 64;
    for (long long t = (long long)vg.bid * kWaves + wave_in_wg(); t < tiles;
         t += (long long)vg.nb * kWaves) {
      const long long v = t * 64 + lane_id();
      const bool f = v < n && ops.in_frontier((int)v);
      const uint64_t mk = ballot(f);
      if (lane_id() == 0) w.fbits[t] = mk;
    }
  }
  auto pred = [&](int v) { return degree_of(off, v) > 0 && ops.pull_candidate(v); };
  auto deg = [&](int v) { return degree_of(off, v); };
  auto ident = [](int i) { return i; };
  const Regions R = regions(w, it & 1, vg.nb);
  ballot_fill(vg, n, pred, deg, ident, P, 0x7fffffff, w.bits, R,
              w.rec + SLOT_SCAN, lds.ball);
}

SX_DEV bool fbit(const unsigned long long *fb, int u) { return (fb[u >> 6] >> (u & 63)) & 1ull; }

// Pull compute over the candidates (view `cand`, totals T).  Found / improved
// vertices are recorded by the online filter into slot it+1 (parity it+1),
// binned by out-degree, so that a switch back to push needs no scan.
template <class Ops>
SX_PHASE void pull_phase(const VGrid &vg, const TravArgs &a, const Params &P, int it,
                         const ViewRef &cand, const Totals &T, LdsTrav &lds) {
  const DevGraph &g = a.g;
  const Regions NR = regions(a.w, (it + 1) & 1, vg.nb);
  bins_begin(lds.bins, NR, P.online_cap);
  const unsigned long long *fb = a.w.fbits;
  unsigned *dist = (unsigned *)a.state_i;
  WaveStats st;
  long long edges = 0;
  unsigned err = 0;
  const int lane = lane_id();
  const unsigned gw = vg.bid * kWaves + wave_in_wg();
  const unsigned nw = vg.nb * kWaves;
  const unsigned cs = T.cnt[BIN_SMALL], cm = T.cnt[BIN_MED], cl = T.cnt[BIN_LARGE];
  auto out_deg = [&](int v, int in_deg) { return g.directed ? degree_of(g.off, v) : in_deg; };
  // One workgroup per large candidate
  for (unsigned i = vg.bid; i < cl; i += vg.nb) {
    const int v = (int)(cand.large(i) & 0xffffffffu);
    if ((unsigned)v >= (unsigned)g.n) continue;
    const int beg = g.in_off[v], end = g.in_off[v + 1];
    unsigned best = 0xFFFFFFFFu;
    if (!Ops::kVote) best = dist[v];
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
            const unsigned c = pull_offer<Ops>(dist, g, u, arc, err);
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
        if (best < dist[v]) {
          store_relaxed(&dist[v], best);
          store_relaxed(&a.w.stamp[v], it + 1);
          act = true;
        }
      }
      __syncthreads();
    }
    if (wave_in_wg() == 0)
      bins_append(act, v, act ? out_deg(v, end - beg) : 0, NR, vg.bid, P, P.chunk, lds.bins, st);
  }
  // One wavefront per medium candidate
  for (unsigned i = gw; i < cm; i += nw) {
    const int v = cand.med(i);
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
            const unsigned c = pull_offer<Ops>(dist, g, u, arc, err);
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
      if (lane == 0 && best < dist[v]) {
        store_relaxed(&dist[v], best);
        store_relaxed(&a.w.stamp[v], it + 1);
        act = true;
      }
    }
    bins_append(act, v, act ? out_deg(v, end - beg) : 0, NR, vg.bid, P, P.chunk, lds.bins, st);
  }
  // One lane per small candidate; four in-arcs per round (their ids and
  // bitmap words load independently: two memory round trips per four arcs)
  for (unsigned c0 = gw * 64u; c0 < cs; c0 += nw * 64u) {
    const unsigned i = c0 + lane;
    bool act = false;
    int v = 0, d = 0;
    if (i < cs) {
      const int x = cand.small(i);
      if ((unsigned)x < (unsigned)g.n) {
        v = x;
        const int beg = g.in_off[v], end = g.in_off[v + 1];
        d = end - beg;
        int arc = beg;
        if (Ops::kVote) {
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
          unsigned best = dist[v];
          const unsigned old = best;
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
                const unsigned cc = pull_offer<Ops>(dist, g, u[j], arc + j, err);
                best = cc < best ? cc : best;
              }
            edges += 4;
          }
          for (; arc < end; ++arc) {
            ++edges;
            const int u1 = g.in_idx[arc];
            if (fbit(fb, u1)) {
              const unsigned cc = pull_offer<Ops>(dist, g, u1, arc, err);
              best = cc < best ? cc : best;
            }
          }
          if (best < old) {
            store_relaxed(&dist[v], best);
            store_relaxed(&a.w.stamp[v], it + 1);
            act = true;
          }
        }
      }
    }
    bins_append(act, v, act ? out_deg(v, d) : 0, NR, vg.bid, P, P.chunk, lds.bins, st);
  }
  bins_end(lds.bins, st, a.w.rec + ((it + 1) % 3), vg.bid);
  if (err) raise_error(a.w.ctrl, err);
  add_stats(a.w.ctrl, vg.bid, edges, vg.bid == 0 ? (unsigned long long)cs + cm + cl : 0ull, lds.red);
  if (vg.bid == 0 && threadIdx.x == 0) atomic_add_u32(&a.w.ctrl->stats.v[5], 1u);
}

// The view of one record slot / parity (all threads); returns the totals.
SX_DEV Totals make_view(const VGrid &vg, const TravArgs &a, int slot, int parity, LdsTrav &lds,
                        ViewRef &ref) {
  ref.V = &lds.view;
  ref.R = regions(a.w, parity, vg.nb);
  ref.G = vg.nb;
  return view_build(a.w.rec + slot, vg.nb, ref.R, lds.view, lds.red);
}

// A list built by a ballot scan never exceeds its regions (the host sizes
// them for any scan); if one did, stop with an error instead of computing on
// an incomplete list.
SX_DEV bool scan_fits(const TravArgs &a, const Totals &T) {
  if (!T.ovf) return true;
  if (threadIdx.x == 0) raise_error(a.w.ctrl, SX_ERR_CAPACITY);
  return false;
}

// --------------------------------------------------------- decisions ---
struct RunState {
  int it;
  unsigned long long mu;
  PolicyState ps;
  Params P;
  unsigned B = 0xFFFFFFFFu;     // delta-stepping bound (sequenced SSSP)
  unsigned dropped = 0;         // 1: buckets dropped for the rest of the run
};

struct LdsPolicy {
  alignas(16) float p[kMlpParams + 4];
  float y[kMlpOut];
};

// The decision after iteration s.it from the totals of its output lists:
// the rule of decide_core, then -- with the learned policy -- the MLP's
// choices where the caller left them open.  Overflow always forces the
// ballot rebuild: the online lists are incomplete.
template <class Ops>
SX_DEV Decision decide(const TravArgs &a, RunState &s, bool pulling, const Totals &T,
                       LdsPolicy *pol, bool lead, bool stage = false) {
  DecideIn in;
  in.nf = T.nf;
  in.mf = T.mf;
  in.ovf = T.ovf;
  in.it = s.it;
  in.pulling = pulling;
  in.vote = Ops::kVote;
  in.n = a.g.n;
  in.m = a.g.m;
  Decision d = decide_core(in, s.P, s.mu);
  if (!d.done && a.P.learned && in.mf >= kPolicyMinArcs) {
    float x[kMlpIn];
    policy_features(in.nf, in.mf, Ops::kVote ? s.mu : (unsigned long long)a.g.m, a.g.n, a.g.m, s.ps,
                    pulling, x);
    // stage the weights only for a decision the network takes (the barrier
    // below orders the copy before the evaluation)
    if (stage)
      for (int i = threadIdx.x; i < kMlpParams; i += kBlock) pol->p[i] = a.mlp[i];
    __syncthreads();
    if (wave_in_wg() == 0) {
      float y[kMlpOut];
      mlp_eval_wave(pol->p, x, y);
      if (lane_id() == 0)
        for (int k = 0; k < kMlpOut; ++k) pol->y[k] = y[k];
      // the last evaluation of the run goes to the statistics (workgroup 0)
      if (lane_id() == 0 && lead) {
        Line &pl = a.w.ctrl->pol;
        for (int k = 0; k < kMlpIn; ++k) store_relaxed(&pl.v[1 + k], __float_as_uint(x[k]));
        for (int k = 0; k < kMlpOut; ++k) store_relaxed(&pl.v[1 + kMlpIn + k], __float_as_uint(y[k]));
        store_relaxed(&pl.v[0], load_relaxed(&pl.v[0]) + 1u);
      }
    }
    __syncthreads();
    const float y[kMlpOut] = {pol->y[0], pol->y[1], pol->y[2], pol->y[3]};
    apply_network(y, pulling, in.ovf != 0, a.P.direction, a.P.filter, a.P.bins_fixed != 0, a.P.t1, a.P.t2, d,
                  s.P.t1, s.P.t2);
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
template <>
SX_DEV WccOps make_ops<WccOps>(const TravArgs &a, int it) {
  return WccOps{(unsigned *)a.state_i, a.w.stamp, it};
}

// Stage the network's weights in LDS (all threads; a barrier must follow
// before the first decision: every caller passes one).
SX_DEV void load_policy(const TravArgs &a, LdsPolicy &pol) {
  if (!a.P.learned) return;
  for (int i = threadIdx.x; i < kMlpParams; i += kBlock) pol.p[i] = a.mlp[i];
}

// Ctrl::state for the fused kernels: [0] exit reason [1] iteration [2] the
// lists of the iteration come from a ballot scan [6,7] unexplored arcs [8]
// previous frontier size [10,11] activated so far [12] t1 [13] t2
SX_DEV void load_state(const TravArgs &a, RunState &s, bool &rebuilt) {
  Ctrl *C = a.w.ctrl;
  s.it = (int)load_relaxed(&C->state.v[1]);
  rebuilt = load_relaxed(&C->state.v[2]) != 0;
  s.mu = load_relaxed((unsigned long long *)&C->state.v[6]);
  s.ps.nf_prev = load_relaxed(&C->state.v[8]);
  s.ps.reached = load_relaxed((unsigned long long *)&C->state.v[10]);
  s.P = a.P;
  const unsigned t1 = load_relaxed(&C->state.v[12]), t2 = load_relaxed(&C->state.v[13]);
  if (t1) { s.P.t1 = (int)t1; s.P.t2 = (int)t2; }
}

SX_DEV void finish(const VGrid &vg, Ctrl *C, int reason, const RunState &s, bool rebuilt) {
  if (vg.bid == 0 && threadIdx.x == 0) {
    store_relaxed(&C->state.v[0], (unsigned)reason);
    store_relaxed(&C->state.v[1], (unsigned)s.it);
    store_relaxed(&C->state.v[2], rebuilt ? 1u : 0u);
    store_relaxed((unsigned long long *)&C->state.v[6], s.mu);
    store_relaxed(&C->state.v[8], s.ps.nf_prev);
    store_relaxed((unsigned long long *)&C->state.v[10], s.ps.reached);
    store_relaxed(&C->state.v[12], (unsigned)s.P.t1);
    store_relaxed(&C->state.v[13], (unsigned)s.P.t2);
  }
}

SX_DEV bool entry_done(Ctrl *C) {
  const unsigned e = load_relaxed(&C->state.v[0]);
  return e == EXIT_DONE || e == EXIT_LIMIT || e == EXIT_ERROR;
}

// ------------------------------------------------ one query, in a loop ---
// The iteration loop of one query over a (virtual) grid synchronised by
// `bar`.  kDir 0 / 1: the push / pull kernel of selective fusion -- only that
// direction's phases are compiled in, and a direction change leaves the loop
// (EXIT_SWITCH) so that the host launches the other kernel; kDir 2: both
// directions, switching in place (all fusion and the batched kernel).
// Returns the exit reason.
template <class Ops, int kDir, bool kDedup = true>
SX_DEV int run_loop(const VGrid &vg, const TravArgs &a, GridBarrier &bar, LdsTrav &lds,
                    LdsPolicy &pol, RunState &s, bool &pulling, bool &rebuilt) {
  constexpr bool both = kDir == 2;
  Ctrl *C = a.w.ctrl;
  ViewRef ref;
  Totals T;
  if constexpr (kDir != 1) {
    if (!pulling) {
      // the lists of s.it: online (slot it % 3) unless a scan rebuilt them;
      // an online list that overflowed (appended by a pull iteration) is
      // rebuilt
      if (!rebuilt) {
        T = make_view(vg, a, s.it % 3, s.it & 1, lds, ref);
        if (T.ovf) {
          Ops ops = make_ops<Ops>(a, s.it - 1);
          ballot_next(vg, a, s.P, ops, s.it - 1, lds);
          if (!bar.sync()) return EXIT_ERROR;
          rebuilt = true;
        }
      }
      if (rebuilt) {
        T = make_view(vg, a, SLOT_SCAN, s.it & 1, lds, ref);
        if (!scan_fits(a, T)) return EXIT_ERROR;
      }
    }
  }
  for (;;) {
    if (!pulling) {
      if constexpr (kDir == 1) {
        return EXIT_SWITCH;
      } else {
        if (vg.bid == 0 && threadIdx.x == 0) atomic_add_u32(&C->stats.v[6], 1u);
        Ops ops = make_ops<Ops>(a, s.it);
        push_phase<Ops, kDedup>(vg, a, s.P, ops, s.it, ref, T, lds);
        if (!bar.sync()) return EXIT_ERROR;
        T = make_view(vg, a, (s.it + 1) % 3, (s.it + 1) & 1, lds, ref);
        Decision d = decide<Ops>(a, s, false, T, &pol, vg.bid == 0);
        rebuilt = false;
        if (d.done) { ++s.it; return s.it >= a.P.max_iters ? EXIT_LIMIT : EXIT_DONE; }
        if (d.to_pull) {
          ++s.it;
          pulling = true;
          if (!both) return EXIT_SWITCH;
          continue;
        }
        if (d.ballot) {
          ballot_next(vg, a, s.P, ops, s.it, lds);
          if (!bar.sync()) return EXIT_ERROR;
          T = make_view(vg, a, SLOT_SCAN, (s.it + 1) & 1, lds, ref);
          if (!scan_fits(a, T)) return EXIT_ERROR;
          rebuilt = true;
        }
        ++s.it;
      }
    } else {
      if constexpr (kDir == 0) {
        return EXIT_SWITCH;
      } else {
        if (vg.bid == 0 && threadIdx.x == 0) atomic_add_u32(&C->stats.v[6], 1u);
        Ops ops = make_ops<Ops>(a, s.it);
        pull_scan(vg, a, s.P, ops, s.it, lds);
        if (!bar.sync()) return EXIT_ERROR;
        T = make_view(vg, a, SLOT_SCAN, s.it & 1, lds, ref);
        if (!scan_fits(a, T)) return EXIT_ERROR;
        pull_phase<Ops>(vg, a, s.P, s.it, ref, T, lds);
        if (!bar.sync()) return EXIT_ERROR;
        T = make_view(vg, a, (s.it + 1) % 3, (s.it + 1) & 1, lds, ref);
        Decision d = decide<Ops>(a, s, true, T, &pol, vg.bid == 0);
        if (d.done) { ++s.it; return s.it >= a.P.max_iters ? EXIT_LIMIT : EXIT_DONE; }
        ++s.it;
        if (d.to_push) {
          pulling = false;
          rebuilt = false;
          if (T.ovf) {
            Ops o2 = make_ops<Ops>(a, s.it - 1);
            ballot_next(vg, a, s.P, o2, s.it - 1, lds);
            if (!bar.sync()) return EXIT_ERROR;
            T = make_view(vg, a, SLOT_SCAN, s.it & 1, lds, ref);
            if (!scan_fits(a, T)) return EXIT_ERROR;
            rebuilt = true;
          }
          if (!both) return EXIT_SWITCH;
        }
      }
    }
  }
}

// -------------------------------------------------- persistent kernels ---
// kMode 0 / 1: selective fusion, the paper's design (Section 5, Table
// table-compile): one persistent kernel per direction, each holding only
// its own direction's phases; a direction change exits the kernel and the
// host launches the other one.  kMode 2: all fusion, both directions in one
// persistent kernel that switches in place (the loop the batched kernel
// runs), at the register cost of both directions' code in one kernel.
template <class Ops, int kMode>
__global__ void __launch_bounds__(kBlock) k_fused(TravArgs a) {
  __shared__ LdsTrav lds;
  __shared__ LdsPolicy pol;
  Ctrl *C = a.w.ctrl;
  const VGrid vg = hw_grid();
  GridBarrier bar(C, load_relaxed(&C->bar_gen.v[0]), a.P.watchdog);
  if (entry_done(C) || bar.failed()) return;
  RunState s;
  bool rebuilt;
  load_state(a, s, rebuilt);
  load_policy(a, pol);
  // the direction the run is in: state word 3 (1 = pulling), kept across
  // the launches of a run
  bool pulling = load_relaxed(&C->state.v[3]) != 0;
  const int r = run_loop<Ops, kMode>(vg, a, bar, lds, pol, s, pulling, rebuilt);
  finish(vg, C, r, s, rebuilt);
  if (vg.bid == 0 && threadIdx.x == 0) store_relaxed(&C->state.v[3], pulling ? 1u : 0u);
}

// ------------------------------------------------ one-phase kernels ---
// The same phases, one launch each; the host reads the records between
// launches and takes the decisions (no fusion).  `P` carries the thresholds
// the host chose.
template <class Ops>
__global__ void __launch_bounds__(kBlock) k_push_step(TravArgs a, int it, int rebuilt) {
  __shared__ LdsTrav lds;
  const VGrid vg = hw_grid();
  ViewRef ref;
  const Totals T = make_view(vg, a, rebuilt ? SLOT_SCAN : it % 3, it & 1, lds, ref);
  if (rebuilt && !scan_fits(a, T)) return;
  if (vg.bid == 0 && threadIdx.x == 0) atomic_add_u32(&a.w.ctrl->stats.v[6], 1u);
  Ops ops = make_ops<Ops>(a, it);
  push_phase(vg, a, a.P, ops, it, ref, T, lds);
}
template <class Ops>
__global__ void __launch_bounds__(kBlock) k_ballot(TravArgs a, int it) {
  __shared__ LdsTrav lds;
  const VGrid vg = hw_grid();
  Ops ops = make_ops<Ops>(a, it);
  ballot_next(vg, a, a.P, ops, it, lds);
}
template <class Ops>
__global__ void __launch_bounds__(kBlock) k_pull_scan(TravArgs a, int it) {
  __shared__ LdsTrav lds;
  const VGrid vg = hw_grid();
  if (vg.bid == 0 && threadIdx.x == 0) atomic_add_u32(&a.w.ctrl->stats.v[6], 1u);
  Ops ops = make_ops<Ops>(a, it);
  pull_scan(vg, a, a.P, ops, it, lds);
}
template <class Ops>
__global__ void __launch_bounds__(kBlock) k_pull_step(TravArgs a, int it) {
  __shared__ LdsTrav lds;
  const VGrid vg = hw_grid();
  ViewRef ref;
  const Totals T = make_view(vg, a, SLOT_SCAN, it & 1, lds, ref);
  if (!scan_fits(a, T)) return;
  pull_phase<Ops>(vg, a, a.P, it, ref, T, lds);
}

// ------------------------------------------------------ sequenced mode ---
// The fused loop of Section 5 with the kernel boundary as its global
// barrier: every launch runs one phase and hands the run state to the next
// launch through Ctrl::seq (launch L reads seq[L & 1] and writes
// seq[(L + 1) & 1]).  After a compute phase the next launch first takes the
// decision -- every workgroup reads the same records and decides the same
// way, as after a barrier -- and then runs the phase it chose.  The host
// enqueues launches ahead in batches and reads the state only between
// batches: no host round trip per iteration, one kernel boundary (~2.5 us on
// MI355X, against ~6-10 us for a software barrier over a full persistent
// grid) per phase, and each phase at the occupancy of its own registers.
enum : unsigned { PH_PUSH = 0, PH_BALLOT = 1, PH_PULL_SCAN = 2, PH_PULL = 3 };
// seq line: [0] phase [1] iteration [2,3] unexplored arcs [4] previous
// frontier size [6,7] activated so far [8] t1 [9] t2 [10] pulling [11] a
// decision is due [12] the push lists come from a ballot scan [13] the
// delta-stepping bound (0: not set yet) [14] buckets dropped (pull steps)
SX_DEV void seq_store(Line &l, unsigned phase, const RunState &s, unsigned pulling, unsigned due,
                      unsigned rebuilt) {
  store_relaxed(&l.v[0], phase);
  store_relaxed(&l.v[1], (unsigned)s.it);
  store_relaxed((unsigned long long *)&l.v[2], s.mu);
  store_relaxed(&l.v[4], s.ps.nf_prev);
  store_relaxed((unsigned long long *)&l.v[6], s.ps.reached);
  store_relaxed(&l.v[8], (unsigned)s.P.t1);
  store_relaxed(&l.v[9], (unsigned)s.P.t2);
  store_relaxed(&l.v[10], pulling);
  store_relaxed(&l.v[11], due);
  store_relaxed(&l.v[12], rebuilt);
  store_relaxed(&l.v[13], s.B);
  store_relaxed(&l.v[14], s.dropped);
}

// kMinWaves = 6 (the wide form, for large graphs): at least six wavefronts
// per SIMD (80 VGPRs, a few spilled to scratch), three workgroups per CU
// instead of two, which the latency-bound push steps of large graphs turn
// into throughput (R-MAT s22 SSSP 3.39 -> 3.09 ms).  The spills lengthen
// each phase's critical path, so graphs with small frontiers and thousands
// of iterations use kMinWaves = 1 (the compiler's own choice, no spills).
// Returns whether the launch ran a phase of an active run.
template <class Ops>
SX_DEV bool seq_body(const TravArgs &a, unsigned L, LdsTrav &lds, LdsPolicy &pol) {
  Ctrl *C = a.w.ctrl;
  const VGrid vg = hw_grid();
  Line &out = C->seq[(L + 1) & 1];
  const bool lead = vg.bid == 0 && threadIdx.x == 0;
  fetch_line(C->seq[L & 1], C, lds.sq);
  const unsigned *in = lds.sq;
  unsigned phase = in[0];
  RunState s;
  s.it = (int)in[1];
  s.mu = (unsigned long long)in[2] | ((unsigned long long)in[3] << 32);
  s.ps.nf_prev = in[4];
  s.ps.reached = (unsigned long long)in[6] | ((unsigned long long)in[7] << 32);
  s.P = a.P;
  if (in[8]) { s.P.t1 = (int)in[8]; s.P.t2 = (int)in[9]; }
  unsigned pulling = in[10];
  const unsigned due = in[11];
  unsigned rebuilt = in[12];
  s.B = in[13] ? in[13] : (a.P.delta && a.P.delta_after == 0 ? a.P.delta : 0xFFFFFFFFu);
  s.dropped = in[14];
  if (phase >= SEQ_DONE) {
    if (lead) seq_store(out, phase, s, pulling, 0, rebuilt);
    return false;
  }
  if (in[32]) {
    if (lead) seq_store(out, SEQ_ERROR, s, pulling, 0, rebuilt);
    return false;
  }
  seq_stall_enter(C, vg.bid);
  ViewRef ref;
  Totals T;
  bool have_view = false;
  if (due) {
    T = make_view(vg, a, (s.it + 1) % 3, (s.it + 1) & 1, lds, ref);
    // one launch per phase: the weights are staged only by a launch whose
    // decision evaluates the network
    Decision d = decide<Ops>(a, s, pulling != 0, T, &pol, vg.bid == 0, true);
    if (d.done) {
      ++s.it;
      if (lead) {
        seq_store(out, s.it >= a.P.max_iters ? SEQ_LIMIT : SEQ_DONE, s, pulling, 0, 0);
        // the run needed launches 0..L: the host sizes the next run's first
        // batch of launches on this graph by it (Ctrl::stats word 12, unused
        // by the other programs; k_trav_init clears it)
        store_relaxed(&C->stats.v[12], L + 1u);
      }
      return true;
    }
    // delta-stepping: once no listed vertex lies below the bound, move it to
    // the end of the bucket holding the smallest listed distance (empty
    // buckets are skipped); pull steps relax without buckets
    // (buckets that engage late start at the bucket of the smallest
    // listed distance)
    if (a.P.delta && !s.dropped) {
      if (pulling || d.to_pull) {
        s.B = 0xFFFFFFFFu;
        s.dropped = 1;
      } else {
        const unsigned lo = load_relaxed(&C->aux.v[(s.it + 1) % 3]);
        const bool engage = s.B == 0xFFFFFFFFu && s.it + 1 >= a.P.delta_after;
        if (lo != 0xFFFFFFFFu && (engage || (s.B != 0xFFFFFFFFu && lo >= s.B))) {
          const unsigned long long nb = ((unsigned long long)lo / a.P.delta + 1ull) * a.P.delta;
          s.B = nb >= 0xFFFFFFFFull ? 0xFFFFFFFFu : (unsigned)nb;
        }
      }
    }
    if (!pulling) {
      if (d.to_pull) { pulling = 1; phase = PH_PULL_SCAN; ++s.it; }
      else if (d.ballot) phase = PH_BALLOT;
      else { phase = PH_PUSH; ++s.it; rebuilt = 0; have_view = true; }
    } else if (d.to_push) {
      pulling = 0;
      rebuilt = 0;
      if (T.ovf) phase = PH_BALLOT;
      else { phase = PH_PUSH; ++s.it; have_view = true; }
    } else {
      phase = PH_PULL_SCAN;
      ++s.it;
    }
  }
  const int it = s.it;
  Ops ops = make_ops<Ops>(a, it);
  switch (phase) {
    case PH_PUSH:
      if (!have_view) {
        T = make_view(vg, a, rebuilt ? SLOT_SCAN : it % 3, it & 1, lds, ref);
        if (rebuilt && !scan_fits(a, T)) break;
      }
      if (lead) atomic_add_u32(&C->stats.v[6], 1u);
      push_phase(vg, a, s.P, ops, it, ref, T, lds, s.B);
      if (lead) seq_store(out, PH_PUSH, s, 0, 1, 0);
      break;
    case PH_BALLOT:
      // rebuild the lists of it+1, then push them
      ballot_next(vg, a, s.P, ops, it, lds);
      ++s.it;
      if (lead) seq_store(out, PH_PUSH, s, 0, 0, 1);
      break;
    case PH_PULL_SCAN:
      if (lead) atomic_add_u32(&C->stats.v[6], 1u);
      pull_scan(vg, a, s.P, ops, it, lds);
      if (lead) seq_store(out, PH_PULL, s, 1, 0, 0);
      break;
    case PH_PULL:
      T = make_view(vg, a, SLOT_SCAN, it & 1, lds, ref);
      if (!scan_fits(a, T)) break;
      pull_phase<Ops>(vg, a, s.P, it, ref, T, lds);
      if (lead) seq_store(out, PH_PULL, s, 1, 1, 0);
      break;
  }
  // a capacity error leaves `out` unwritten: the next launch sees the error
  if (lead && load_relaxed(&C->error.v[0]) == SX_ERR_CAPACITY)
    seq_store(out, SEQ_ERROR, s, pulling, 0, rebuilt);
  return true;
}

template <class Ops, int kMinWaves>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kMinWaves))) k_seq(TravArgs a, unsigned L) {
  __shared__ LdsTrav lds;
  __shared__ LdsPolicy pol;
  if (seq_body<Ops>(a, L, lds, pol)) seq_stall_leave(a.w.ctrl, blockIdx.x);
}

// First state of a sequenced run, written by k_trav_init's first thread
// after the run state (one thread; nothing reads it before the first k_seq).
// all_active: every vertex is active in iteration 0 (WCC), so a push start
// first builds the lists of iteration 0 by a ballot scan (iteration -1's next
// lists).
SX_DEV void seq_first_state(Ctrl *C, unsigned pull_first, unsigned all_active) {
  Line &l = C->seq[0];
  for (int i = 0; i < 32; ++i) l.v[i] = 0u;
  l.v[0] = pull_first ? PH_PULL_SCAN : (all_active ? PH_BALLOT : PH_PUSH);
  if (!pull_first && all_active) l.v[1] = 0xFFFFFFFFu;
  l.v[10] = pull_first;
  *(unsigned long long *)&l.v[2] = *(unsigned long long *)&C->state.v[6];
  // delta-stepping: smallest distance set by each step (three rotating words)
  for (int i = 0; i < 3; ++i) C->aux.v[i] = 0xFFFFFFFFu;
}

// ------------------------------------------------------------ set-up ---
// Vertex state: BFS depth -1 (source 0); SSSP distance infinity (source 0)
// and stamp -1 (source 0); WCC label = own id (the caller's id on a
// renumbered graph) and stamp 0 (all active).
SX_DEV void init_state(const VGrid &vg, const TravArgs &a, bool sssp, bool wcc = false) {
  const int n = a.g.n;
  const long long tid = (long long)vg.bid * kBlock + threadIdx.x, nt = (long long)vg.nb * kBlock;
  if (a.xdist && (sssp || wcc)) {
    const long long nx = 2ll * n + a.g.m / kChunk + 2;
    for (long long i = tid; i < nx; i += nt) a.xdist[i] = 0xFFFFFFFFu;
  }
  for (long long v = tid; v < n; v += nt) {
    if (wcc) {
      const int at = a.wcc_inv ? a.wcc_inv[v] : (int)v;
      a.state_i[at] = (int)v;
      a.w.stamp[at] = 0;
    } else if (sssp) {
      ((unsigned *)a.state_i)[v] = v == a.src ? 0u : 0xFFFFFFFFu;
      a.w.stamp[v] = v == a.src ? 0 : -1;
    } else {
      a.state_i[v] = v == a.src ? 0 : -1;
    }
  }
}

// The source as the lists of iteration 0 (slot 0, parity 0) of a grid of G
// workgroups: workgroup 0 holds it, every other record is empty.  Called by
// one whole wavefront.
SX_DEV void init_source(const TravArgs &a, unsigned G) {
  const Regions R = regions(a.w, 0, G);
  const int d = degree_of(a.g.off, a.src);
  const int b = bin_of(d, a.P);
  const int lane = lane_id();
  if (lane == 0) {
    if (b == BIN_SMALL) R.s[0] = a.src;
    else if (b == BIN_MED) R.m[0] = a.src;
  }
  const long long k = b == BIN_LARGE ? chunks_of(d, a.P.chunk) : 0;
  const long long kk = k < (long long)R.cap_l ? k : (long long)R.cap_l;
  for (long long c = lane; c < kk; c += 64)
    R.l[c] = ((unsigned long long)c << 32) | (unsigned)a.src;
  for (unsigned w = lane; w < G; w += 64) {
    const bool me = w == 0;
    unsigned c[NBINS];
    for (int i = 0; i < NBINS; ++i) c[i] = me && i == b ? (b == BIN_LARGE ? (unsigned)kk : 1u) : 0u;
    rec_write(a.w.rec, w, c, me ? 1u : 0u, me ? (unsigned long long)d : 0ull, me && kk < k);
  }
}

// Run set-up: vertex state, a fresh control block, the source list (WCC:
// none; its first lists come from a ballot scan or a pull step, and the
// persistent and one-phase arrangements are told so by state word 2).
// Launched with any grid of at least 2 workgroups; G = the run's grid.
__global__ void k_trav_init(TravArgs a, int algo, unsigned long long mu0, unsigned G,
                            unsigned pull_first, unsigned sequenced) {
  const bool wcc = algo == ALG_WCC;
  init_state(hw_grid(), a, algo == ALG_SSSP, wcc);
  Ctrl *C = a.w.ctrl;
  if (blockIdx.x == 0) reset_barrier(C);
  if (blockIdx.x == 0 && threadIdx.x < 64) {
    if (threadIdx.x == 0) {
      for (int i = 0; i < 32; ++i) { C->state.v[i] = 0; C->stats.v[i] = 0; }
      C->error.v[0] = 0;
      // arcs not yet explored: all but the source's
      *(unsigned long long *)&C->state.v[6] =
          wcc ? 0ull : (mu0 ? mu0 : (unsigned long long)(a.g.m - degree_of(a.g.off, a.src)));
      if (wcc) C->state.v[2] = 1u;
      C->state.v[3] = pull_first;
      if (sequenced) seq_first_state(C, pull_first, wcc ? 1u : 0u);
    }
    if (!wcc) init_source(a, G);
  }
  if (blockIdx.x == 1) reset_stat_lines(C);
}

// ------------------------------------------------- batched queries ---
// Many BFS / SSSP queries over graphs of uneven size in one persistent
// launch.  The hardware grid is split into teams of `team` workgroups; each
// team owns a workspace (bins, records, stamps, bitmaps, a control block
// with its own barrier lines) and repeatedly takes the next query from a
// shared counter (queries are ordered largest first), runs it to completion
// with the same phases and decisions as the single-query kernels -- both
// directions in one loop, switching in place -- synchronised by a barrier
// over the team only, then takes the next.  Teams never wait for each other,
// so a 6-level R-MAT query and a 4,000-level grid query overlap.
template <class Ops>
SX_DEV bool batch_query(const VGrid &vg, const TravArgs &a, GridBarrier &bar, LdsTrav &lds,
                        LdsPolicy &pol, unsigned long long mu0) {
  RunState s;
  s.it = 0;
  s.mu = mu0;
  s.ps.nf_prev = 0;
  s.ps.reached = 0;
  s.P = a.P;
  bool pulling = a.P.direction == 2, rebuilt = false;
  const int r = run_loop<Ops, 2, false>(vg, a, bar, lds, pol, s, pulling, rebuilt);
  finish(vg, a.w.ctrl, r, s, false);
  if (r == EXIT_ERROR) return false;
  return bar.sync();
}

// Four wavefronts per SIMD (128 VGPRs, spilling): two workgroups per CU, so
// twice the teams run at once (256 queries over 64 graphs: 609 -> 561 ms).
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) k_batch(BatchArgs b) {
  __shared__ LdsTrav lds;
  __shared__ LdsPolicy pol;
  const unsigned team = blockIdx.x / (unsigned)b.team;
  const VGrid vg{blockIdx.x % (unsigned)b.team, (unsigned)b.team};
  if (team >= (unsigned)b.nteams) return;
  const Work w = b.work[team];
  Ctrl *C = w.ctrl;
  GridBarrier bar(C, load_relaxed(&C->bar_gen.v[0]), b.P.watchdog, vg);
  TravArgs a;
  a.w = w;
  a.P = b.P;
  a.mlp = b.mlp;
  a.wcc_inv = nullptr;
  a.xdist = nullptr;   // no expansion record in batches
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
    init_state(vg, a, sssp);
    // the previous query's statistics were read before the barrier above
    if (vg.bid < (unsigned)kStatLines && threadIdx.x == 0) {
      Line &l = C->statw[vg.bid];
      store_relaxed((unsigned long long *)&l.v[0], 0ull);
      store_relaxed((unsigned long long *)&l.v[2], 0ull);
    }
    if (vg.bid == 0 && threadIdx.x == 0) {
      for (int i = 0; i < 32; ++i) {
        store_relaxed(&C->state.v[i], 0u);
        store_relaxed(&C->stats.v[i], 0u);
      }
    }
    if (vg.bid == 0 && threadIdx.x < 64) init_source(a, vg.nb);
    if (!bar.sync()) break;
    const unsigned long long mu0 = (unsigned long long)(Q.g.m - degree_of(Q.g.off, Q.src));
    const bool ok = sssp ? batch_query<SsspOps>(vg, a, bar, lds, pol, mu0)
                         : batch_query<BfsOps>(vg, a, bar, lds, pol, mu0);
    if (vg.bid == 0 && threadIdx.x == 0) {
      BatchStat &r = b.stats[b.order[qi]];
      r.iterations = (int)load_relaxed(&C->stats.v[6]);
      r.pull_iters = (int)load_relaxed(&C->stats.v[5]);
      r.ballot_iters = (int)load_relaxed(&C->stats.v[4]);
      unsigned long long e = 0, x = 0;
      for (int i = 0; i < kStatLines && i < b.team; ++i) {
        e += load_relaxed((unsigned long long *)&C->statw[i].v[0]);
        x += load_relaxed((unsigned long long *)&C->statw[i].v[2]);
      }
      r.edges = e;
      r.expansions = x;
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
  reset_stat_lines(C);
  if (threadIdx.x == 0) C->error.v[0] = 0u;
  if (team == 0 && threadIdx.x == 0) *b.queue_head = 0u;
}

}  // namespace sx

// ------------------------------------------------------ host launchers ---
namespace sx {

// Kernel of kind `kind` for algorithm `algo` (ALG_BFS / ALG_SSSP / ALG_WCC).
template <class Ops>
static const void *trav_kernel_t(int kind) {
  switch (kind) {
    case TK_FUSED: return (const void *)k_fused<Ops, 0>;
    case TK_FUSED_PULL: return (const void *)k_fused<Ops, 1>;
    case TK_FUSED_ALL: return (const void *)k_fused<Ops, 2>;
    case TK_PUSH_STEP: return (const void *)k_push_step<Ops>;
    case TK_BALLOT: return (const void *)k_ballot<Ops>;
    case TK_PULL_SCAN: return (const void *)k_pull_scan<Ops>;
    case TK_PULL_STEP: return (const void *)k_pull_step<Ops>;
    case TK_SEQ: return (const void *)k_seq<Ops, 1>;
    case TK_SEQ_WIDE: return (const void *)k_seq<Ops, 6>;
    default: return nullptr;
  }
}

const void *trav_kernel(int kind, int algo) {
  switch (algo) {
    case ALG_BFS: return trav_kernel_t<BfsOps>(kind);
    case ALG_SSSP: return trav_kernel_t<SsspOps>(kind);
    case ALG_WCC: return trav_kernel_t<WccOps>(kind);
    default: return nullptr;
  }
}

template <class Ops>
static hipError_t trav_launch_t(int kind, const TravArgs &a, int it, int arg, int grid,
                                hipStream_t s) {
  const dim3 g(grid), b(kBlock);
  switch (kind) {
    case TK_FUSED: hipLaunchKernelGGL((k_fused<Ops, 0>), g, b, 0, s, a); break;
    case TK_FUSED_PULL: hipLaunchKernelGGL((k_fused<Ops, 1>), g, b, 0, s, a); break;
    case TK_FUSED_ALL: hipLaunchKernelGGL((k_fused<Ops, 2>), g, b, 0, s, a); break;
    case TK_PUSH_STEP: hipLaunchKernelGGL(k_push_step<Ops>, g, b, 0, s, a, it, arg); break;
    case TK_BALLOT: hipLaunchKernelGGL(k_ballot<Ops>, g, b, 0, s, a, it); break;
    case TK_PULL_SCAN: hipLaunchKernelGGL(k_pull_scan<Ops>, g, b, 0, s, a, it); break;
    case TK_PULL_STEP: hipLaunchKernelGGL(k_pull_step<Ops>, g, b, 0, s, a, it); break;
    case TK_SEQ: hipLaunchKernelGGL((k_seq<Ops, 1>), g, b, 0, s, a, (unsigned)it); break;
    case TK_SEQ_WIDE: hipLaunchKernelGGL((k_seq<Ops, 6>), g, b, 0, s, a, (unsigned)it); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t trav_launch(int kind, int algo, const TravArgs &a, int it, int arg, int grid,
                       hipStream_t s) {
  switch (algo) {
    case ALG_BFS: return trav_launch_t<BfsOps>(kind, a, it, arg, grid, s);
    case ALG_SSSP: return trav_launch_t<SsspOps>(kind, a, it, arg, grid, s);
    case ALG_WCC: return trav_launch_t<WccOps>(kind, a, it, arg, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t trav_init(const TravArgs &a, int algo, unsigned long long mu0, int run_grid,
                     hipStream_t s, bool pull_first, bool sequenced) {
  int grid = (a.g.n + kBlock - 1) / kBlock;
  if (grid < 2) grid = 2;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_trav_init, dim3(grid), dim3(kBlock), 0, s, a, algo, mu0, (unsigned)run_grid,
                     pull_first ? 1u : 0u, sequenced ? 1u : 0u);
  return hipGetLastError();
}

// Sum of the m arc weights into *out (zeroed first): one 64-bit atomic per
// wavefront.  Used once per graph to choose a delta-stepping width.
__global__ void __launch_bounds__(256) k_weight_sum(const unsigned *w, long long m,
                                                    unsigned long long *out) {
  long long s = 0;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < m;
       e += (long long)gridDim.x * blockDim.x)
    s += (long long)w[e];
  s = wave_sum_ll(s);
  if (lane_id() == 0 && s) atomic_add_u64(out, (unsigned long long)s);
}

hipError_t weight_sum(const unsigned *w, long long m, unsigned long long *out, hipStream_t s) {
  hipError_t e = hipMemsetAsync(out, 0, sizeof(unsigned long long), s);
  if (e != hipSuccess) return e;
  if (m <= 0) return hipSuccess;
  long long grid = (m + 255) / 256;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_weight_sum, dim3((unsigned)grid), dim3(256), 0, s, w, m, out);
  return hipGetLastError();
}

hipError_t batch_launch(const BatchArgs &b, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reset, dim3(b.nteams), dim3(256), 0, s, b);
  hipLaunchKernelGGL(k_batch, dim3(grid), dim3(kBlock), 0, s, b);
  return hipGetLastError();
}

const void *batch_kernel() { return (const void *)k_batch; }

}  // namespace sx
