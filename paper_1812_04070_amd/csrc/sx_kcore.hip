// k-core decomposition as an ACC program (Section 6, "k-Core": delete the
// vertices of degree below k until every remaining vertex has at least k
// neighbours), extended from one k to all of them: level by level, for
// k = 0, 1, 2, ... every vertex still present whose current degree is <= k is
// deleted and gets core number k, until no vertex is left.
//
//   Active   alive and degree <= k.
//   Compute  deleting v lowers the degree of each neighbour by one.
//   Combine  sum (aggregation).  Push: an atomic decrement per arc; following
//            the paper's k-core note, a neighbour whose degree is already
//            <= k is not decremented any more (it is deleted at this level
//            anyway).  Pull: every alive vertex counts its neighbours deleted
//            in this step and lowers its own degree once, without atomics.
//            A vertex is activated by the update that takes its degree from
//            above k to k or below, so it enters a frontier exactly once.
//
// A vertex deleted in step j carries stamp j (set when it enters the list of
// step j, together with its core number), so a pull step only needs
// stamp[u] == j to recognise the vertices being deleted.
//
// Task management: a level starts with a scan of the alive list (binned like
// the worklists, per-workgroup regions, one record slot per parity): entries
// still alive with degree <= k form the level's frontier, the others are
// re-emitted into the other alive list, with their minimum degree per
// workgroup so that empty levels are skipped.  The deletions within a level
// are chained by the online filter, with the JIT switch of Section 4 (an
// overflowing online list is replaced by a fresh scan at the same level).
// Direction (Section 5, switching to pull for large frontiers): a step pulls
// when the frontier's arcs exceed the alive arcs / kPullAlpha.  In R-MAT
// graphs the dense last levels delete thousands of high-degree vertices per
// step; pushing them costs one device-scope atomic per arc (MI355X sustains
// ~13 G/s of them over scattered addresses) while a pull step reads the
// alive arcs at memory speed.  A directed graph counts in- plus out-arcs and
// walks both its CSR and CSC rows.
#include "sx_frontier.hpp"
#include "sx_kernels.hpp"

namespace sx {

// Decrements of high-degree neighbours in push steps are summed per
// workgroup in a small LDS table and applied with one atomic per
// (workgroup, vertex) at the end of the step: most arcs of the low-degree
// vertices that a level deletes lead to a few hubs, and device-scope atomics
// on one address are serialised (~11 ns each).  Summing is exact: the
// activation test needs only the value before and after each atomic.
constexpr int kHot = 4096;         // table entries (power of two, 32 KB of LDS)
constexpr int kHotProbes = 8;
constexpr int kHotDeg = 64;        // current degree from which a target is summed
constexpr unsigned long long kHotMinArcs = 65536;  // steps below this push directly
// Local cascades: a vertex that a push step activates is deleted by the same
// workgroup within the same step when its degree is below kLocalDeg and the
// workgroup's budget (kLocalQ queued vertices, kLocalArcs arcs) has room;
// the others wait for the next step, where the whole grid shares them (one
// workgroup walking a dense level's cascade alone would take longer than the
// grid-wide steps it saves).  The deletions of one level form chains (a deletion takes a
// neighbour to k, which is deleted next, ...); on R-MAT s22 a level needs ~3
// grid-wide steps without this, most of them with a handful of vertices and
// each paying a launch and a record prefix.  Every vertex is still deleted
// exactly once (by the update that activated it), so the result is the same.
constexpr int kLocalDeg = 256;
constexpr int kLocalQ = 2048;
constexpr unsigned kLocalArcs = 8192;   // arcs a workgroup takes on locally per step
constexpr float kPullAlpha = 8.f;  // pull when frontier arcs > alive arcs / alpha

struct LdsK {
  int hkey[kHot];
  int hcnt[kHot];
  unsigned short hlist[kHot];      // slots in use, in order of first use
  unsigned hn;
  int lq[kLocalQ];                 // local cascade queue
  unsigned lq_head, lq_tail, lq_arcs;
  int small[kWaves][192];
  LdsBins bins, bins2;
  LdsView view;
  long long red[kWaves];
  unsigned wmin[kWaves];
  unsigned sq[33];                 // the run-state line and the error word
};

SX_DEV int total_degree(const DevGraph &g, int v) {
  int d = g.off[v + 1] - g.off[v];
  if (g.directed) d += g.in_off[v + 1] - g.in_off[v];
  return d;
}

// The alive list of parity p as regions of a grid of G workgroups.
SX_DEV Regions alive_regions(const Work &w, int p, unsigned G) {
  Regions r;
  r.s = w.al_s[p];
  r.m = w.al_m[p];
  r.l = w.al_l[p];
  r.cap_s = w.tot_s / G;
  r.cap_m = w.tot_m / G;
  r.cap_l = w.tot_l / G;
  return r;
}

// The view of a list: record slot `slot`, regions R.
SX_DEV Totals kview(const VGrid &vg, const Work &w, int slot, const Regions &R, LdsK &lds,
                    ViewRef &ref) {
  ref.V = &lds.view;
  ref.R = R;
  ref.G = vg.nb;
  return view_build(w.rec + slot, vg.nb, R, lds.view, lds.red);
}

// A vertex enters the list of step `step` at level k: its core number and
// deletion stamp are set now (single writer: the update that activated it).
SX_DEV void mark_deleted(const KArgs &a, int v, int k, int step) {
  a.core[v] = k;
  a.w.stamp[v] = step;
}

// Level scan number s at level k, building the list of peel step j.  Every
// entry of the alive list (view `A`, parity s & 1) is tested once per lane:
// alive with degree > k -> re-emitted into alive parity (s + 1) & 1; alive
// with degree <= k, or activated for step j by an online list that
// overflowed -> the frontier (parity j & 1, slot SLOT_SCAN).
SX_DEV void kscan(const VGrid &vg, const KArgs &a, int k, int s, int j, const ViewRef &A,
                  const Totals &TA, LdsK &lds) {
  const Work &w = a.w;
  const DevGraph &g = a.g;
  const Regions SR = alive_regions(w, (s + 1) & 1, vg.nb);
  const Regions FR = regions(w, j & 1, vg.nb);
  bins_begin(lds.bins, SR, 0);
  bins_begin(lds.bins2, FR, 0);
  WaveStats ss, fs;
  unsigned mind = 0xFFFFFFFFu;
  const unsigned tid = vg.bid * kBlock + threadIdx.x, nt = vg.nb * kBlock;
  const unsigned cs = TA.cnt[BIN_SMALL], cm = TA.cnt[BIN_MED], cl = TA.cnt[BIN_LARGE];
  const unsigned total = cs + cm + cl;
  // wave-uniform trip count: all lanes take part in the appends
  for (unsigned base = tid - lane_id(); base < total; base += nt) {
    const unsigned i = base + lane_id();
    bool ok = i < total;
    int bin = BIN_SMALL;
    unsigned long long item = 0;
    if (ok) {
      if (i < cs) item = (unsigned)A.small(i);
      else if (i < cs + cm) { bin = BIN_MED; item = (unsigned)A.med(i - cs); }
      else { bin = BIN_LARGE; item = A.large(i - cs - cm); }
    }
    const int v = (int)(item & 0xffffffffu);
    const bool first = bin != BIN_LARGE || (item >> 32) == 0;
    ok = ok && (unsigned)v < (unsigned)g.n;
    bool keep = false, front = false;
    int d = 0, td = 0;
    if (ok) {
      const int c = a.core[v];
      d = w.deg[v];
      keep = c == -1 && d > k;
      front = first && ((c == -1 && d <= k) || (c == k && w.stamp[v] == j));
      if (keep || front) td = total_degree(g, v);
      if (keep) mind = (unsigned)d < mind ? (unsigned)d : mind;
    }
    bins_put(keep, bin, item, first, td, SR, vg.bid, lds.bins, ss);
    if (front) mark_deleted(a, v, k, j);
    bins_append(front, v, td, FR, vg.bid, a.P, a.P.chunk, lds.bins2, fs);
  }
  bins_end(lds.bins, ss, w.rec + SLOT_ALIVE + ((s + 1) & 1), vg.bid);
  bins_end(lds.bins2, fs, w.rec + SLOT_SCAN, vg.bid);
  mind = wave_min_u(mind);
  if (lane_id() == 0) lds.wmin[wave_in_wg()] = mind;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < kWaves; ++i) mind = lds.wmin[i] < mind ? lds.wmin[i] : mind;
    w.alive_min[(size_t)((s + 1) & 1) * kMaxGrid + vg.bid] = mind;
    if (vg.bid == 0) {
      atomic_add_u32(&w.ctrl->stats.v[4], 1u);
      atomic_add_u64((unsigned long long *)&w.ctrl->stats.v[8], (unsigned long long)total);
    }
  }
  __syncthreads();
}

// Minimum survivor degree of the last scan (alive parity p), all threads.
SX_DEV unsigned alive_min_degree(const VGrid &vg, const Work &w, int p, LdsK &lds) {
  unsigned m = 0xFFFFFFFFu;
  for (unsigned b = threadIdx.x; b < vg.nb; b += kBlock) {
    const unsigned x = w.alive_min[(size_t)p * kMaxGrid + b];
    m = x < m ? x : m;
  }
  m = wave_min_u(m);
  if (lane_id() == 0) lds.wmin[wave_in_wg()] = m;
  __syncthreads();
  unsigned mind = 0xFFFFFFFFu;
  for (int i = 0; i < kWaves; ++i) mind = lds.wmin[i] < mind ? lds.wmin[i] : mind;
  __syncthreads();
  return mind;
}

// Push step j: the vertices of the list (view `cur`) lower the degrees of
// their neighbours; activated neighbours form the list of step j + 1 (online
// filter into slot (j + 1) % 3, parity (j + 1) & 1).
SX_DEV void kpeel_push(const VGrid &vg, const KArgs &a, int k, int j, const ViewRef &cur,
                       const Totals &T, LdsK &lds) {
  const Work &w = a.w;
  const DevGraph &g = a.g;
  const unsigned cs = T.cnt[BIN_SMALL], cm = T.cnt[BIN_MED], cl = T.cnt[BIN_LARGE];
  // the table pays for its set-up and flush only in large steps
  const bool hot = T.mf >= kHotMinArcs;
  if (hot) {
    for (int i = threadIdx.x; i < kHot; i += kBlock) {
      lds.hkey[i] = -1;
      lds.hcnt[i] = 0;
    }
    if (threadIdx.x == 0) lds.hn = 0;
  }
  if (threadIdx.x == 0) {
    lds.lq_head = 0;
    lds.lq_tail = 0;
    lds.lq_arcs = 0;
  }
  const Regions NR = regions(w, (j + 1) & 1, vg.nb);
  bins_begin(lds.bins, NR, a.P.online_cap);   // its barrier also covers the table
  WaveStats st;
  long long edges = 0;
  int *deg = w.deg;
  // one decrement of u into the table; false when its probe sequence is full
  auto hot_add = [&](int u) {
    const unsigned h = ((unsigned)u * 2654435761u) >> 20;
    for (int p = 0; p < kHotProbes; ++p) {
      const unsigned s = (h + (unsigned)p) & (kHot - 1);
      const int prev = atomicCAS(&lds.hkey[s], -1, u);
      if (prev == -1 || prev == u) {
        atomicAdd(&lds.hcnt[s], 1);
        if (prev == -1) lds.hlist[atomicAdd(&lds.hn, 1u)] = (unsigned short)s;
        return true;
      }
    }
    return false;
  };
  // An activated vertex u (degree du): into the local queue (deleted in this
  // step, stamp j) or the next step's list (stamp j + 1).  Called
  // convergently by whole wavefronts.
  auto activate = [&](bool act, int u, int du) {
    const bool want = act && du < kLocalDeg;
    const uint64_t mk = ballot(want);
    bool local = false;
    if (mk) {
      const int incl = wave_incl_scan(want ? du : 0);
      unsigned base = 0, abase = 0;
      if (lane_id() == 63) {
        base = atomicAdd(&lds.lq_tail, (unsigned)__popcll(mk));
        abase = atomicAdd(&lds.lq_arcs, (unsigned)incl);
      }
      base = __shfl(base, 63);
      abase = __shfl(abase, 63);
      if (want) {
        const unsigned pos = base + lane_prefix(mk);
        if (pos < (unsigned)kLocalQ) {
          // a reserved slot is always written: -1 (skipped) when over budget
          local = abase + (unsigned)incl <= kLocalArcs;
          lds.lq[pos] = local ? u : -1;
        }
      }
    }
    if (act) mark_deleted(a, u, k, local ? j : j + 1);
    bins_append(act && !local, u, du, NR, vg.bid, a.P, a.P.chunk, lds.bins, st);
  };
  bool use_hot = hot;
  // kIlp arcs per lane: all degree loads, then all decrements, then the
  // degrees of the activated targets, each stage with every arc in flight
  auto op = [&](const int *v, const int *u, const int *arc, const bool *ok) {
    (void)v; (void)arc;
    int d[kIlp], old[kIlp], du[kIlp];
    bool dec[kIlp], act[kIlp];
#pragma unroll
    for (int r = 0; r < kIlp; ++r) d[r] = ok[r] ? deg[u[r]] : 0;  // stale (higher) costs an atomic
#pragma unroll
    for (int r = 0; r < kIlp; ++r) {
      edges += ok[r] ? 1 : 0;
      dec[r] = ok[r] && d[r] > k && !(use_hot && d[r] >= kHotDeg && hot_add(u[r]));
    }
#pragma unroll
    for (int r = 0; r < kIlp; ++r) old[r] = dec[r] ? atomic_sub_i32(&deg[u[r]], 1) : 0;
#pragma unroll
    for (int r = 0; r < kIlp; ++r) {
      act[r] = dec[r] && old[r] == k + 1;
      du[r] = act[r] ? total_degree(g, u[r]) : 0;
    }
#pragma unroll
    for (int r = 0; r < kIlp; ++r) activate(act[r], u[r], du[r]);
  };
  const unsigned gw = vg.bid * kWaves + wave_in_wg();
  const unsigned nw = vg.nb * kWaves;
  for (int pass = 0; pass < (g.directed ? 2 : 1); ++pass) {
    const int *off = pass ? g.in_off : g.off;
    const int *idx = pass ? g.in_idx : g.idx;
    visit_large(vg, g.n, [&](unsigned i) { return cur.large(i); }, cl, off, idx, a.P.chunk, op);
    visit_med(g.n, [&](unsigned i) { return cur.med(i); }, cm, off, idx, op, gw, nw);
    visit_small(g.n, [&](unsigned i) { return cur.small(i); }, cs, off, idx, op, gw, nw,
                lds.small[wave_in_wg()]);
  }
  // apply the summed decrements: u is activated by the atomic whose range
  // (old - c, old] holds k, i.e. old > k >= old - c
  __syncthreads();
  const unsigned used = hot ? lds.hn : 0u;
  for (unsigned t0 = 0; t0 < used; t0 += kBlock * kIlp) {
    int u[kIlp], c[kIlp], old[kIlp], du[kIlp];
    bool act[kIlp];
#pragma unroll
    for (int r = 0; r < kIlp; ++r) {
      const unsigned t = t0 + r * kBlock + threadIdx.x;
      const int slot = t < used ? (int)lds.hlist[t] : 0;
      u[r] = t < used ? lds.hkey[slot] : -1;
      c[r] = t < used ? lds.hcnt[slot] : 0;
      if (!(u[r] >= 0 && c[r] > 0 && (unsigned)u[r] < (unsigned)g.n)) c[r] = 0;
    }
#pragma unroll
    for (int r = 0; r < kIlp; ++r) old[r] = c[r] ? atomic_sub_i32(&deg[u[r]], c[r]) : 0;
#pragma unroll
    for (int r = 0; r < kIlp; ++r) {
      act[r] = c[r] && old[r] > k && old[r] - c[r] <= k;
      du[r] = act[r] ? total_degree(g, u[r]) : 0;
    }
#pragma unroll
    for (int r = 0; r < kIlp; ++r) activate(act[r], u[r], du[r]);
  }
  // drain the local queue: batches [head, tail) until no deletion adds more
  // (the summing table is not used here: it was flushed above)
  use_hot = false;
  unsigned long long local_done = 0;
  for (;;) {
    __syncthreads();
    const unsigned h = lds.lq_head;
    const unsigned t = lds.lq_tail < (unsigned)kLocalQ ? lds.lq_tail : (unsigned)kLocalQ;
    __syncthreads();
    if (h >= t) break;
    for (int pass = 0; pass < (g.directed ? 2 : 1); ++pass) {
      const int *off = pass ? g.in_off : g.off;
      const int *idx = pass ? g.in_idx : g.idx;
      visit_small(g.n, [&](unsigned i) { return lds.lq[h + i]; }, t - h, off, idx, op,
                  (unsigned)wave_in_wg(), (unsigned)kWaves, lds.small[wave_in_wg()]);
    }
    local_done += t - h;
    if (threadIdx.x == 0) lds.lq_head = t;
  }
  bins_end(lds.bins, st, w.rec + ((j + 1) % 3), vg.bid);
  add_stats(w.ctrl, vg.bid, edges,
            (vg.bid == 0 ? (unsigned long long)cs + cm + cl : 0ull) + (threadIdx.x == 0 ? local_done : 0ull),
            lds.red);
}

// Pull step j: every alive vertex of the alive list (view `A`) counts its
// neighbours with stamp j and lowers its own degree by that count (a large
// vertex per chunk of arcs, one atomic per chunk); activated vertices form
// the list of step j + 1.
SX_DEV void kpeel_pull(const VGrid &vg, const KArgs &a, int k, int j, const ViewRef &A,
                       const Totals &TA, LdsK &lds) {
  const Work &w = a.w;
  const DevGraph &g = a.g;
  const int *stamp = w.stamp;
  int *deg = w.deg;
  const Regions NR = regions(w, (j + 1) & 1, vg.nb);
  bins_begin(lds.bins, NR, a.P.online_cap);
  WaveStats st;
  long long edges = 0;
  const int lane = lane_id();
  const int passes = g.directed ? 2 : 1;
  // small vertices: one lane each, four arcs per round
  auto count_row = [&](const int *idx, int beg, int end) {
    int c = 0;
    int e = beg;
    for (; e + 4 <= end; e += 4) {
      const int u0 = idx[e], u1 = idx[e + 1], u2 = idx[e + 2], u3 = idx[e + 3];
      c += (stamp[u0] == j) + (stamp[u1] == j) + (stamp[u2] == j) + (stamp[u3] == j);
    }
    for (; e < end; ++e) c += stamp[idx[e]] == j;
    edges += end - beg;
    return c;
  };
  auto settle = [&](int v, int c, bool &act, int &du) {
    // single writer of deg[v]: no other update of v in a pull step
    const int d = deg[v];
    deg[v] = d - c;
    if (d > k && d - c <= k) {
      act = true;
      du = total_degree(g, v);
      mark_deleted(a, v, k, j + 1);
    }
  };
  const unsigned gw = vg.bid * kWaves + wave_in_wg();
  const unsigned nw = vg.nb * kWaves;
  const unsigned cs = TA.cnt[BIN_SMALL], cm = TA.cnt[BIN_MED], cl = TA.cnt[BIN_LARGE];
  for (unsigned c0 = gw * 64u; c0 < cs; c0 += nw * 64u) {
    const unsigned i = c0 + lane;
    bool act = false;
    int v = 0, du = 0;
    if (i < cs) {
      const int x = A.small(i);
      if ((unsigned)x < (unsigned)g.n && a.core[x] == -1) {
        v = x;
        int c = count_row(g.idx, g.off[v], g.off[v + 1]);
        if (passes == 2) c += count_row(g.in_idx, g.in_off[v], g.in_off[v + 1]);
        if (c) settle(v, c, act, du);
      }
    }
    bins_append(act, v, du, NR, vg.bid, a.P, a.P.chunk, lds.bins, st);
  }
  // medium vertices: one wavefront each
  for (unsigned i = gw; i < cm; i += nw) {
    const int v = A.med(i);
    if ((unsigned)v >= (unsigned)g.n || __shfl(a.core[v], 0) != -1) continue;
    int c = 0;
    for (int pass = 0; pass < passes; ++pass) {
      const int *off = pass ? g.in_off : g.off;
      const int *idx = pass ? g.in_idx : g.idx;
      const int beg = off[v], end = off[v + 1];
      for (int e = beg + lane; e < end; e += 64) {
        c += stamp[idx[e]] == j;
        ++edges;
      }
    }
    c = wave_sum_i(c);
    bool act = false;
    int du = 0;
    if (lane == 0 && c) settle(v, c, act, du);
    bins_append(act, v, du, NR, vg.bid, a.P, a.P.chunk, lds.bins, st);
  }
  // large vertices: one workgroup per chunk of arcs, one atomic per chunk.
  // The workgroup that settles another chunk of v may set core[v] while this
  // one reads it, so the test is agreed on by a barrier: every wavefront must
  // take the same branch around the reduction's barriers below.
  for (unsigned i = vg.bid; i < cl; i += vg.nb) {
    const unsigned long long it = A.large(i);
    const int v = (int)(it & 0xffffffffu);
    if ((unsigned)v >= (unsigned)g.n) continue;
    if (!__syncthreads_and(a.core[v] == -1)) continue;
    const long long ch = (long long)(it >> 32) * a.P.chunk;
    int c = 0;
    for (int pass = 0; pass < passes; ++pass) {
      const int *off = pass ? g.in_off : g.off;
      const int *idx = pass ? g.in_idx : g.idx;
      const long long vb = off[v], ve = off[v + 1];
      const long long b0 = vb + ch < ve ? vb + ch : ve;
      const long long e0 = b0 + a.P.chunk < ve ? b0 + a.P.chunk : ve;
      for (long long e = b0 + threadIdx.x; e < e0; e += kBlock) {
        c += stamp[idx[e]] == j;
        ++edges;
      }
    }
    c = (int)wg_sum_ll<kBlock>(c, lds.red);
    bool act = false;
    int du = 0;
    if (threadIdx.x == 0 && c) {
      const int old = atomic_sub_i32(&deg[v], c);
      if (old > k && old - c <= k) {
        act = true;
        du = total_degree(g, v);
        mark_deleted(a, v, k, j + 1);
      }
    }
    if (wave_in_wg() == 0) bins_append(act, v, du, NR, vg.bid, a.P, a.P.chunk, lds.bins, st);
  }
  bins_end(lds.bins, st, w.rec + ((j + 1) % 3), vg.bid);
  add_stats(w.ctrl, vg.bid, edges, vg.bid == 0 ? (unsigned long long)cs + cm + cl : 0ull, lds.red);
  if (vg.bid == 0 && threadIdx.x == 0) atomic_add_u32(&w.ctrl->stats.v[5], 1u);
}

// Run state: level k, scans done s, peel steps done j, the list of step j
// comes from a scan, the arcs of the alive list of the last scan.
struct KState {
  int k, s, j;
  bool from_scan;
  unsigned long long alive_arcs;
  unsigned alive_n = 0;           // vertices of the alive list of the last scan
};

// What follows a scan: 1 peel, 0 scan again at a higher level (k updated),
// -1 done.  T: the frontier, TA: the survivors.
SX_DEV int after_scan(const VGrid &vg, const KArgs &a, KState &q, const Totals &T,
                      const Totals &TA, LdsK &lds) {
  q.alive_arcs = TA.mf;
  q.alive_n = TA.nf;
  // no survivors: the frontier's core numbers are set (by the scan), and
  // nobody is left to receive its decrements
  if (TA.nf == 0) return -1;
  if (T.nf > 0) return 1;
  // fixed k: a scan that finds nothing to delete ends the run
  if (a.P.kfix) return -1;
  // empty level: jump to the smallest surviving degree
  const unsigned mind = alive_min_degree(vg, a.w, q.s & 1, lds);
  q.k = (int)mind > q.k + 1 ? (int)mind : q.k + 1;
  return 0;
}

// Direction of the next peel step: the policy's fixed direction, else pull
// when the step's arcs exceed the alive arcs / kPullAlpha.
SX_DEV bool pull_step(const KState &q, const Totals &T, const Params &P) {
  if (P.direction == 1) return false;
  if (P.direction == 2) return true;
  return (double)T.mf * kPullAlpha > (double)q.alive_arcs;
}

// One peel step: pull over the alive list or push from the step's list.
// `have` / `T` / `ref`: the view of the step's list, when already built.
SX_DEV void kpeel(const VGrid &vg, const KArgs &a, const KState &q, bool pull, bool have,
                  Totals &T, ViewRef &ref, LdsK &lds) {
  if (pull) {
    const Totals TA = kview(vg, a.w, SLOT_ALIVE + (q.s & 1), alive_regions(a.w, q.s & 1, vg.nb),
                            lds, ref);
    kpeel_pull(vg, a, q.k, q.j, ref, TA, lds);
  } else {
    if (!have)
      T = kview(vg, a.w, q.from_scan ? SLOT_SCAN : q.j % 3, regions(a.w, q.j & 1, vg.nb), lds, ref);
    kpeel_push(vg, a, q.k, q.j, ref, T, lds);
  }
}

// A scan: the view of the alive list, then kscan.
SX_DEV void kscan_phase(const VGrid &vg, const KArgs &a, const KState &q, LdsK &lds) {
  ViewRef A;
  const Totals TA = kview(vg, a.w, SLOT_ALIVE + (q.s & 1), alive_regions(a.w, q.s & 1, vg.nb), lds, A);
  kscan(vg, a, q.k, q.s, q.j, A, TA, lds);
}

// Persistent kernel: the whole decomposition in one launch.
// Ctrl::aux: [10] k [11] scans [12] peel steps [13] lists of the next peel
// come from a scan [14] next step kind (0 scan, 1 peel) [16,17] alive arcs
enum { AUX_K = 10, AUX_SCAN = 11, AUX_STEP = 12, AUX_FROM = 13, AUX_KIND = 14, AUX_ARCS = 16 };

__global__ void __launch_bounds__(kBlock) k_kcore_fused(KArgs a) {
  __shared__ LdsK lds;
  Ctrl *C = a.w.ctrl;
  const VGrid vg = hw_grid();
  GridBarrier bar(C, load_relaxed(&C->bar_gen.v[0]), a.P.watchdog);
  fetch_line(C->aux, C, lds.sq);
  KState q;
  q.k = (int)lds.sq[AUX_K];
  q.s = (int)lds.sq[AUX_SCAN];
  q.j = (int)lds.sq[AUX_STEP];
  q.from_scan = lds.sq[AUX_FROM] != 0;
  q.alive_arcs = (unsigned long long)lds.sq[AUX_ARCS] | ((unsigned long long)lds.sq[AUX_ARCS + 1] << 32);
  int kind = (int)lds.sq[AUX_KIND];
  auto save = [&](int reason) {
    if (vg.bid == 0 && threadIdx.x == 0) {
      store_relaxed(&C->state.v[0], (unsigned)reason);
      store_relaxed(&C->aux.v[AUX_K], (unsigned)q.k);
      store_relaxed(&C->aux.v[AUX_SCAN], (unsigned)q.s);
      store_relaxed(&C->aux.v[AUX_STEP], (unsigned)q.j);
      store_relaxed(&C->aux.v[AUX_FROM], q.from_scan ? 1u : 0u);
      store_relaxed(&C->aux.v[AUX_KIND], (unsigned)kind);
      store_relaxed((unsigned long long *)&C->aux.v[AUX_ARCS], q.alive_arcs);
    }
  };
  if (load_relaxed(&C->state.v[0]) != EXIT_NONE || lds.sq[32]) return;
  // every step deletes at least one vertex or raises k: bound the loop
  const long long limit = 4ll * a.g.n + 64;
  ViewRef ref;
  Totals V;
  bool have = false, pull = false;
  for (long long guard = 0;; ++guard) {
    if (guard > limit) { save(EXIT_LIMIT); return; }
    if (kind == 0) {
      kscan_phase(vg, a, q, lds);
      if (!bar.sync()) { save(EXIT_ERROR); return; }
      ++q.s;
      V = kview(vg, a.w, SLOT_SCAN, regions(a.w, q.j & 1, vg.nb), lds, ref);
      const Totals TA = rec_totals(a.w.rec + SLOT_ALIVE + (q.s & 1), vg.nb, lds.red);
      if (V.ovf || TA.ovf) {
        if (threadIdx.x == 0) store_relaxed(&C->error.v[0], (unsigned)SX_ERR_CAPACITY);
        save(EXIT_ERROR);
        return;
      }
      const int r = after_scan(vg, a, q, V, TA, lds);
      if (r < 0) { save(EXIT_DONE); return; }
      if (r == 0) continue;
      kind = 1;
      q.from_scan = true;
      have = true;
      pull = pull_step(q, V, a.P);
    } else {
      kpeel(vg, a, q, pull, have, V, ref, lds);
      if (!bar.sync()) { save(EXIT_ERROR); return; }
      if (vg.bid == 0 && threadIdx.x == 0) atomic_add_u32(&C->stats.v[6], 1u);
      ++q.j;
      V = kview(vg, a.w, q.j % 3, regions(a.w, q.j & 1, vg.nb), lds, ref);
      have = true;
      q.from_scan = false;
      if (V.nf == 0 && a.P.kfix) { save(EXIT_DONE); return; }
      if (V.nf == 0) { ++q.k; kind = 0; continue; }
      if (V.ovf || a.P.filter == 2) { kind = 0; continue; }   // rebuild by a scan at the same k
      pull = pull_step(q, V, a.P);
    }
  }
}

// Sequenced form of the same loop: one launch per phase (scan, peel), the
// decision taken at the start of the launch after it; launch L reads
// Ctrl::seq[L & 1] and writes seq[(L+1) & 1]: [0] phase [1] k [2] scans [3]
// peel steps [4] decision due (1 after a scan, 2 after a peel) [5] the list
// of the next peel comes from a scan [6,7] alive arcs [8] alive vertices
// (both of the last scan) [30] L + 1 when launch L (a peel) appended to the
// next list.
enum : unsigned { KP_SCAN = 0, KP_PEEL = 1, KP_DONE = 6, KP_ERROR = 7, KP_LIMIT = 8 };

// Returns whether the launch ran a phase of an active run.
SX_DEV bool kcore_seq_body(const KArgs &a, unsigned L, LdsK &lds) {
  Ctrl *C = a.w.ctrl;
  const VGrid vg = hw_grid();
  Line &out = C->seq[(L + 1) & 1];
  fetch_line(C->seq[L & 1], C, lds.sq);
  unsigned phase = lds.sq[0];
  KState q;
  q.k = (int)lds.sq[1];
  q.s = (int)lds.sq[2];
  q.j = (int)lds.sq[3];
  unsigned due = lds.sq[4];
  q.from_scan = lds.sq[5] != 0;
  q.alive_arcs = (unsigned long long)lds.sq[6] | ((unsigned long long)lds.sq[7] << 32);
  q.alive_n = lds.sq[8];
  const bool lead = vg.bid == 0 && threadIdx.x == 0;
  auto save = [&](unsigned ph) {
    if (lead) {
      store_relaxed(&out.v[0], ph);
      store_relaxed(&out.v[1], (unsigned)q.k);
      store_relaxed(&out.v[2], (unsigned)q.s);
      store_relaxed(&out.v[3], (unsigned)q.j);
      store_relaxed(&out.v[4], due);
      store_relaxed(&out.v[5], q.from_scan ? 1u : 0u);
      store_relaxed((unsigned long long *)&out.v[6], q.alive_arcs);
      store_relaxed(&out.v[8], q.alive_n);
    }
  };
  if (phase >= KP_DONE) { save(phase); return false; }
  if (lds.sq[32]) { due = 0; save(KP_ERROR); return false; }
  if ((long long)q.s + q.j > 4ll * a.g.n + 64) { due = 0; save(KP_LIMIT); return false; }
  seq_stall_enter(C, vg.bid);
  ViewRef ref;
  Totals V;
  bool have = false, pull = false;
  // the scan this launch may run starts a level with nothing pending (the
  // run's first scan, or the previous level exhausted): the tail may take over
  bool boundary = due == 0 && phase == KP_SCAN;
  if (due == 1) {
    V = kview(vg, a.w, SLOT_SCAN, regions(a.w, q.j & 1, vg.nb), lds, ref);
    have = true;
    const Totals TA = rec_totals(a.w.rec + SLOT_ALIVE + (q.s & 1), vg.nb, lds.red);
    if (V.ovf || TA.ovf) {
      if (lead) store_relaxed(&C->error.v[0], (unsigned)SX_ERR_CAPACITY);
      due = 0;
      save(KP_ERROR);
      return true;
    }
    const int r = after_scan(vg, a, q, V, TA, lds);
    due = 0;
    if (r < 0) { save(KP_DONE); return true; }
    if (r == 0) { phase = KP_SCAN; boundary = true; }
    else { phase = KP_PEEL; q.from_scan = true; pull = pull_step(q, V, a.P); }
  } else if (due == 2 && lds.sq[30] != L) {
    // the peel appended nothing (no workgroup stamped the line): next level
    // (fixed k: the level is exhausted, the run is done)
    q.from_scan = false;
    due = 0;
    if (a.P.kfix) { save(KP_DONE); return true; }
    ++q.k;
    phase = KP_SCAN;
    boundary = true;
  } else if (due == 2) {
    V = kview(vg, a.w, q.j % 3, regions(a.w, q.j & 1, vg.nb), lds, ref);
    have = true;
    q.from_scan = false;
    due = 0;
    if (V.nf == 0 && a.P.kfix) { save(KP_DONE); return true; }
    if (V.nf == 0) { ++q.k; phase = KP_SCAN; boundary = true; }
    else if (V.ovf || a.P.filter == 2) phase = KP_SCAN;
    else { phase = KP_PEEL; pull = pull_step(q, V, a.P); }
  }
  if (phase == KP_SCAN && boundary && a.P.ktail > 0) {
    // few vertices and arcs left (the last scan's survivors bound them; the
    // whole graph before the first scan) and their arcs fit the tail's
    // rows: hand the rest to the one-workgroup tail
    const bool first = q.s == 0;
    const unsigned long long an = first ? (unsigned long long)a.g.n : q.alive_n;
    const unsigned long long aa = first ? (unsigned long long)a.g.m * (a.g.directed ? 2 : 1) : q.alive_arcs;
    if (an <= (unsigned long long)a.P.ktail && aa <= a.P.ktail_arcs && aa + 8ull * an <= 4ull * a.w.tot_l) {
      if (lead) {
        store_relaxed(&C->aux.v[KT_K], (unsigned)q.k);
        store_relaxed(&C->aux.v[KT_N], 0u);
      }
      save(KP_TAIL);
      return true;
    }
  }
  if (phase == KP_SCAN) {
    kscan_phase(vg, a, q, lds);
    ++q.s;
    due = 1;
    save(KP_SCAN);
  } else {
    kpeel(vg, a, q, pull, have, V, ref, lds);
    if (lead) atomic_add_u32(&C->stats.v[6], 1u);
    // a workgroup that appended to the next list stamps the line the next
    // launch reads with L + 1 (unique per launch, so nothing is cleared; a
    // stale match only costs the record prefix the decision builds anyway)
    if (threadIdx.x == 0 && (lds.bins.cnt[0] | lds.bins.cnt[1] | lds.bins.cnt[2] | lds.bins.ovf))
      store_relaxed(&out.v[30], L + 1);
    ++q.j;
    due = 2;
    save(KP_PEEL);
  }
  return true;
}

__global__ void __launch_bounds__(kBlock) k_kcore_seq(KArgs a, unsigned L) {
  __shared__ LdsK lds;
  if (kcore_seq_body(a, L, lds)) seq_stall_leave(a.w.ctrl, blockIdx.x);
}

// first scan at level k0 (0: the decomposition; k - 1 for membership in the
// k-core)
__global__ void k_kcore_seq_start(Ctrl *C, unsigned k0) {
  if (threadIdx.x < 32) C->seq[0].v[threadIdx.x] = threadIdx.x == 1 ? k0 : 0u;
}

hipError_t kcore_seq_launch(const KArgs &a, unsigned L, int grid, hipStream_t s, bool start) {
  if (start)
    hipLaunchKernelGGL(k_kcore_seq_start, dim3(1), dim3(64), 0, s, a.w.ctrl,
                       a.P.kfix > 0 ? (unsigned)(a.P.kfix - 1) : 0u);
  else hipLaunchKernelGGL(k_kcore_seq, dim3(grid), dim3(kBlock), 0, s, a, L);
  return hipGetLastError();
}

__global__ void k_kcore_member(int *core, int n) {
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (long long)gridDim.x * blockDim.x)
    core[v] = core[v] == -1 ? 1 : 0;
}

hipError_t kcore_membership(int *core, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  long long grid = ((long long)n + 255) / 256;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_kcore_member, dim3((unsigned)grid), dim3(256), 0, s, core, n);
  return hipGetLastError();
}

const void *kcore_seq_kernel() { return (const void *)k_kcore_seq; }

// Set-up, launched with the run's grid: core -1, stamp -1, current degrees,
// and alive list 0 = every vertex (workgroup b appends a contiguous range of
// about n / G vertices through the online filter into its regions).
__global__ void __launch_bounds__(kBlock) k_kcore_init(KArgs a) {
  __shared__ LdsBins bins;
  const VGrid vg = hw_grid();
  const int n = a.g.n;
  const Regions R = alive_regions(a.w, 0, vg.nb);
  bins_begin(bins, R, 0);
  WaveStats st;
  const long long per = ((long long)n + vg.nb - 1) / vg.nb;
  const long long lo = (long long)vg.bid * per;
  const long long hi = lo + per < n ? lo + per : n;
  for (long long base = lo; base < hi; base += kBlock) {
    const long long v = base + threadIdx.x;
    const bool ok = v < hi;
    int td = 0;
    if (ok) {
      td = total_degree(a.g, (int)v);
      a.core[v] = -1;
      a.w.stamp[v] = -1;
      a.w.deg[v] = td;
    }
    bins_append(ok, (int)v, td, R, vg.bid, a.P, a.P.chunk, bins, st);
  }
  bins_end(bins, st, a.w.rec + SLOT_ALIVE, vg.bid);
  Ctrl *C = a.w.ctrl;
  if (vg.bid == 0) reset_barrier(C);
  if (vg.bid == 0 && threadIdx.x == 0) {
    for (int i = 0; i < 32; ++i) { C->state.v[i] = 0; C->stats.v[i] = 0; C->aux.v[i] = 0; }
    // fixed k: the first scan is at level k - 1
    if (a.P.kfix > 0) C->aux.v[AUX_K] = (unsigned)(a.P.kfix - 1);
    C->error.v[0] = 0;
  }
  if (vg.bid == 1 || vg.nb == 1) reset_stat_lines(C);
}

hipError_t kcore_launch(const KArgs &a, int grid, hipStream_t s, bool init) {
  if (init) hipLaunchKernelGGL(k_kcore_init, dim3(grid), dim3(kBlock), 0, s, a);
  else hipLaunchKernelGGL(k_kcore_fused, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

const void *kcore_kernel() { return (const void *)k_kcore_fused; }

}  // namespace sx
