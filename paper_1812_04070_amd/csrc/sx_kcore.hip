// k-core decomposition as an ACC program (Section 6, "k-Core": delete the
// vertices of degree below k until every remaining vertex has at least k
// neighbours), extended from one k to all of them: level by level, for
// k = 0, 1, 2, ... every vertex still present whose current degree is <= k is
// deleted and gets core number k, until no vertex is left.
//
//   Active   alive and degree <= k.
//   Compute  deleting v lowers the degree of each neighbour by one.
//   Combine  sum (aggregation), here as an atomic decrement.  Following the
//            paper's k-core note, a neighbour whose degree is already <= k is
//            not decremented any more: it is being deleted at this level
//            anyway.  The decrement that takes a degree from k+1 to k is the
//            only one that activates the neighbour, so every vertex enters a
//            frontier exactly once.
//
// Task management: a level starts with a ballot-filter scan of the vertices
// still alive.  Every workgroup keeps its own alive list (a region of the
// alive arrays) and scans only that: the frontier (degree <= k) goes
// sorted and binned into its bin regions, the survivors (degree > k) are
// compacted into its region of the other alive array, with their count and
// minimum degree in per-workgroup words, so that empty levels are skipped
// without a grid-wide atomic.  The deletions within a level are chained by
// the online filter.  The JIT switch of Section 4 applies: an overflowing
// online filter is replaced by a fresh scan.  A directed graph counts in- plus
// out-arcs; deleting v decrements through both its CSR and CSC rows.
#include "sx_frontier.hpp"
#include "sx_kernels.hpp"

namespace sx {

// Decrements of high-degree neighbours are summed per workgroup in a small
// LDS table and applied with one atomic per (workgroup, vertex) at the end of
// the peel step.  In R-MAT graphs most arcs of the low-degree vertices that a
// level deletes lead to a few hubs; one device-scope atomic per arc on the
// same address is serialised (about 11 ns each on MI355X), which made the
// large peel steps ~20x slower than their memory traffic.  Summing is exact:
// the activation test needs only the value before and after each atomic.
constexpr int kHot = 256;          // table entries (power of two)
constexpr int kHotDeg = 64;        // current degree from which a target is summed

struct LdsK {
  int hkey[kHot];
  int hcnt[kHot];
  int small[kWaves][192];
  LdsBins bins;
  LdsView view;
  LdsBallot ball;
  long long red[kWaves];
  unsigned wmin[kWaves];
  unsigned surv;
  unsigned sq[33];                 // the run-state line and the error word
};

SX_DEV int total_degree(const DevGraph &g, int v) {
  int d = g.off[v + 1] - g.off[v];
  if (g.directed) d += g.in_off[v + 1] - g.in_off[v];
  return d;
}

// Alive regions: workgroup b of G owns entries [b * cap, b * cap + cnt) of
// each alive array, cap a multiple of 64 (scan positions align with the
// ballot words).
SX_DEV unsigned alive_cap(const Work &w, unsigned G) { return (w.tot_a / G) & ~63u; }

// Level scan number s at level k: reads this workgroup's alive list in
// alive[s & 1], writes the frontier into parity `fp`, slot SLOT_SCAN, and the
// survivors into alive[(s + 1) & 1] with their count / minimum degree.
SX_DEV void kscan(const VGrid &vg, const KArgs &a, int k, int s, int fp, LdsK &lds) {
  const Work &w = a.w;
  const DevGraph &g = a.g;
  const unsigned G = vg.nb, bid = vg.bid;
  const unsigned cap = alive_cap(w, G);
  const long long lo = (long long)bid * cap;
  const unsigned cnt = w.alive_cnt[(size_t)(s & 1) * kMaxGrid + bid];
  const long long hi = lo + (cnt < cap ? cnt : cap);
  const int *A = w.alive[s & 1];
  int *B = w.alive[(s + 1) & 1] + lo;
  if (threadIdx.x == 0) lds.surv = 0;
  __syncthreads();
  unsigned mind = 0xFFFFFFFFu;
  auto probe = [&](long long i, bool ok) {
    int v = 0, d = 0;
    bool alive = false;
    if (ok) {
      v = A[i];
      alive = (unsigned)v < (unsigned)g.n && a.core[v] == -1;
      if (alive) d = w.deg[v];
    }
    const bool keep = alive && d > k;
    const uint64_t mk = ballot(keep);
    if (mk) {
      const int leader = __ffsll((long long)mk) - 1;
      unsigned base = 0;
      if (lane_id() == leader) base = atomicAdd(&lds.surv, (unsigned)__popcll(mk));
      base = __shfl(base, leader);
      if (keep) {
        B[base + lane_prefix(mk)] = v;
        mind = (unsigned)d < mind ? (unsigned)d : mind;
      }
    }
    return alive && d <= k;
  };
  auto degree = [&](int v) { return total_degree(g, v); };
  auto vof = [&](long long i) { return A[i]; };
  ballot_fill_range(lo, hi, bid, probe, degree, vof, a.P, a.P.chunk, w.bits, regions(w, fp, G),
                    w.rec + SLOT_SCAN, lds.ball);
  mind = wave_min_u(mind);
  if (lane_id() == 0) lds.wmin[wave_in_wg()] = mind;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < kWaves; ++i) mind = lds.wmin[i] < mind ? lds.wmin[i] : mind;
    w.alive_cnt[(size_t)((s + 1) & 1) * kMaxGrid + bid] = lds.surv;
    w.alive_min[(size_t)((s + 1) & 1) * kMaxGrid + bid] = mind;
    if (bid == 0) atomic_add_u32(&w.ctrl->stats.v[4], 1u);
  }
}

// Survivors of the last scan (alive parity p): total count and minimum
// degree over all workgroups (all threads get both).
SX_DEV void alive_totals(const VGrid &vg, const Work &w, int p, LdsK &lds, unsigned long long &cnt,
                         unsigned &mind) {
  long long c = 0;
  unsigned m = 0xFFFFFFFFu;
  for (unsigned b = threadIdx.x; b < vg.nb; b += kBlock) {
    c += w.alive_cnt[(size_t)p * kMaxGrid + b];
    const unsigned x = w.alive_min[(size_t)p * kMaxGrid + b];
    m = x < m ? x : m;
  }
  cnt = (unsigned long long)wg_sum_ll<kBlock>(c, lds.red);
  m = wave_min_u(m);
  if (lane_id() == 0) lds.wmin[wave_in_wg()] = m;
  __syncthreads();
  mind = 0xFFFFFFFFu;
  for (int i = 0; i < kWaves; ++i) mind = lds.wmin[i] < mind ? lds.wmin[i] : mind;
  __syncthreads();
}

SX_DEV Totals kview(const VGrid &vg, const KArgs &a, int slot, int parity, LdsK &lds, ViewRef &ref) {
  ref.V = &lds.view;
  ref.R = regions(a.w, parity, vg.nb);
  ref.G = vg.nb;
  return view_build(a.w.rec + slot, vg.nb, ref.R, lds.view, lds.red);
}

// Peel step j: delete the frontier (view `cur`), decrement the neighbours,
// online filter into slot (j + 1) % 3, parity (j + 1) & 1.
SX_DEV void kpeel(const VGrid &vg, const KArgs &a, int k, int j, const ViewRef &cur, const Totals &T,
                  LdsK &lds) {
  const Work &w = a.w;
  const DevGraph &g = a.g;
  const unsigned cs = T.cnt[BIN_SMALL], cm = T.cnt[BIN_MED], cl = T.cnt[BIN_LARGE];
  // mark the frontier deleted with core number k
  {
    const unsigned tid = vg.bid * kBlock + threadIdx.x, nt = vg.nb * kBlock;
    const unsigned un = (unsigned)g.n;
    for (unsigned i = tid; i < cs; i += nt) {
      const int v = cur.small(i);
      if ((unsigned)v < un) a.core[v] = k;
    }
    for (unsigned i = tid; i < cm; i += nt) {
      const int v = cur.med(i);
      if ((unsigned)v < un) a.core[v] = k;
    }
    for (unsigned i = tid; i < cl; i += nt) {
      const unsigned long long it = cur.large(i);
      const unsigned v = (unsigned)(it & 0xffffffffu);
      if ((it >> 32) == 0 && v < un) a.core[v] = k;
    }
  }
  for (int i = threadIdx.x; i < kHot; i += kBlock) {
    lds.hkey[i] = -1;
    lds.hcnt[i] = 0;
  }
  const Regions NR = regions(w, (j + 1) & 1, vg.nb);
  bins_begin(lds.bins, NR, a.P.online_cap);   // its barrier also covers the table
  WaveStats st;
  long long edges = 0;
  int *deg = w.deg;
  // one decrement of u into the table; false when its probe sequence is full
  auto hot_add = [&](int u) {
    const unsigned h = ((unsigned)u * 2654435761u) >> 24;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const unsigned s = (h + (unsigned)p) & (kHot - 1);
      const int prev = atomicCAS(&lds.hkey[s], -1, u);
      if (prev == -1 || prev == u) {
        atomicAdd(&lds.hcnt[s], 1);
        return true;
      }
    }
    return false;
  };
  auto op = [&](int v, int u, int arc, bool ok) {
    (void)v; (void)arc;
    bool act = false;
    int du = 0;
    if (ok) {
      ++edges;
      const int d = deg[u];   // a stale (higher) value only costs an atomic
      if (d > k && !(d >= kHotDeg && hot_add(u))) {
        const int old = atomic_sub_i32(&deg[u], 1);
        if (old == k + 1) { act = true; du = total_degree(g, u); }
      }
    }
    bins_append(act, u, du, NR, vg.bid, a.P, a.P.chunk, lds.bins, st);
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
  // (old - c, old] holds k + 1 ... i.e. old > k >= old - c
  __syncthreads();
  if (wave_in_wg() < kHot / 64) {
    const int u = lds.hkey[threadIdx.x];
    const int c = lds.hcnt[threadIdx.x];
    bool act = false;
    int du = 0;
    if (u >= 0 && c > 0 && (unsigned)u < (unsigned)g.n) {
      const int old = atomic_sub_i32(&deg[u], c);
      if (old > k && old - c <= k) { act = true; du = total_degree(g, u); }
    }
    bins_append(act, u, du, NR, vg.bid, a.P, a.P.chunk, lds.bins, st);
  }
  bins_end(lds.bins, st, w.rec + ((j + 1) % 3), vg.bid);
  add_stats(w.ctrl, vg.bid, edges, vg.bid == 0 ? (unsigned long long)cs + cm + cl : 0ull, lds.red);
}

// The run state of a decomposition: level k, scans done s, peel steps done
// j, and whether the lists of peel j come from a scan.
struct KState {
  int k, s, j;
  bool from_scan;
};

// What to do after a scan: 1 peel, 0 scan again at a higher level (k
// updated), -1 done.
SX_DEV int after_scan(const VGrid &vg, const KArgs &a, KState &q, const Totals &T, LdsK &lds) {
  if (T.nf > 0) return 1;
  unsigned long long surv;
  unsigned mind;
  alive_totals(vg, a.w, q.s & 1, lds, surv, mind);
  if (surv == 0) return -1;
  // empty level: jump to the smallest surviving degree
  q.k = (int)mind > q.k + 1 ? (int)mind : q.k + 1;
  return 0;
}

// Persistent kernel: the whole decomposition in one launch.
// Ctrl::aux: [10] k [11] scans [12] peel steps [13] lists of the next peel
// come from a scan [14] next step kind (0 scan, 1 peel)
enum { AUX_K = 10, AUX_SCAN = 11, AUX_STEP = 12, AUX_FROM = 13, AUX_KIND = 14 };

__global__ void __launch_bounds__(kBlock) k_kcore_fused(KArgs a) {
  __shared__ LdsK lds;
  Ctrl *C = a.w.ctrl;
  const VGrid vg = hw_grid();
  GridBarrier bar(C, load_relaxed(&C->bar_gen.v[0]));
  KState q;
  q.k = (int)load_relaxed(&C->aux.v[AUX_K]);
  q.s = (int)load_relaxed(&C->aux.v[AUX_SCAN]);
  q.j = (int)load_relaxed(&C->aux.v[AUX_STEP]);
  q.from_scan = load_relaxed(&C->aux.v[AUX_FROM]) != 0;
  int kind = (int)load_relaxed(&C->aux.v[AUX_KIND]);
  auto save = [&](int reason) {
    if (vg.bid == 0 && threadIdx.x == 0) {
      store_relaxed(&C->state.v[0], (unsigned)reason);
      store_relaxed(&C->aux.v[AUX_K], (unsigned)q.k);
      store_relaxed(&C->aux.v[AUX_SCAN], (unsigned)q.s);
      store_relaxed(&C->aux.v[AUX_STEP], (unsigned)q.j);
      store_relaxed(&C->aux.v[AUX_FROM], q.from_scan ? 1u : 0u);
      store_relaxed(&C->aux.v[AUX_KIND], (unsigned)kind);
    }
  };
  if (load_relaxed(&C->state.v[0]) != EXIT_NONE || bar.failed()) return;
  // every step deletes at least one vertex or raises k: bound the loop
  const long long limit = 4ll * a.g.n + 64;
  ViewRef ref;
  Totals V;
  bool have = false;
  for (long long guard = 0;; ++guard) {
    if (guard > limit) { save(EXIT_LIMIT); return; }
    if (kind == 0) {
      kscan(vg, a, q.k, q.s, q.j & 1, lds);
      if (!bar.sync()) { save(EXIT_ERROR); return; }
      ++q.s;
      const Totals T = kview(vg, a, SLOT_SCAN, q.j & 1, lds, ref);
      if (T.ovf) {
        if (threadIdx.x == 0) store_relaxed(&C->error.v[0], (unsigned)SX_ERR_CAPACITY);
        save(EXIT_ERROR);
        return;
      }
      const int r = after_scan(vg, a, q, T, lds);
      if (r < 0) { save(EXIT_DONE); return; }
      if (r == 0) continue;
      kind = 1;
      q.from_scan = true;
      V = T;
      have = true;
    } else {
      // the view of the peel's lists was built by the decision before it,
      // except when the kernel starts here
      if (!have) V = kview(vg, a, q.from_scan ? SLOT_SCAN : q.j % 3, q.j & 1, lds, ref);
      kpeel(vg, a, q.k, q.j, ref, V, lds);
      if (!bar.sync()) { save(EXIT_ERROR); return; }
      if (vg.bid == 0 && threadIdx.x == 0) atomic_add_u32(&C->stats.v[6], 1u);
      ++q.j;
      V = kview(vg, a, q.j % 3, q.j & 1, lds, ref);
      have = true;
      q.from_scan = false;
      if (V.nf == 0) { ++q.k; kind = 0; continue; }
      if (V.ovf || a.P.filter == 2) { kind = 0; continue; }   // rebuild by a scan at the same k
    }
  }
}

// Sequenced form of the same loop: one launch per phase (scan, peel), the
// decision taken at the start of the launch after it; launch L reads
// Ctrl::seq[L & 1] and writes seq[(L+1) & 1]: [0] phase [1] k [2] scans [3]
// peel steps [4] decision due (1 after a scan, 2 after a peel) [5] the lists
// of the next peel come from a scan.
enum : unsigned { KP_SCAN = 0, KP_PEEL = 1, KP_DONE = 6, KP_ERROR = 7, KP_LIMIT = 8 };

__global__ void __launch_bounds__(kBlock) k_kcore_seq(KArgs a, unsigned L) {
  __shared__ LdsK lds;
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
  const bool lead = vg.bid == 0 && threadIdx.x == 0;
  auto save = [&](unsigned ph) {
    if (lead) {
      store_relaxed(&out.v[0], ph);
      store_relaxed(&out.v[1], (unsigned)q.k);
      store_relaxed(&out.v[2], (unsigned)q.s);
      store_relaxed(&out.v[3], (unsigned)q.j);
      store_relaxed(&out.v[4], due);
      store_relaxed(&out.v[5], q.from_scan ? 1u : 0u);
    }
  };
  if (phase >= KP_DONE) { save(phase); return; }
  if (lds.sq[32]) { due = 0; save(KP_ERROR); return; }
  if ((long long)q.s + q.j > 4ll * a.g.n + 64) { due = 0; save(KP_LIMIT); return; }
  ViewRef ref;
  Totals V;
  bool have = false;
  if (due == 1) {
    const Totals T = kview(vg, a, SLOT_SCAN, q.j & 1, lds, ref);
    V = T;
    have = true;
    if (T.ovf) {
      if (lead) store_relaxed(&C->error.v[0], (unsigned)SX_ERR_CAPACITY);
      due = 0;
      save(KP_ERROR);
      return;
    }
    const int r = after_scan(vg, a, q, T, lds);
    due = 0;
    if (r < 0) { save(KP_DONE); return; }
    if (r == 0) phase = KP_SCAN;
    else { phase = KP_PEEL; q.from_scan = true; }
  } else if (due == 2) {
    V = kview(vg, a, q.j % 3, q.j & 1, lds, ref);
    have = true;
    q.from_scan = false;
    due = 0;
    if (V.nf == 0) { ++q.k; phase = KP_SCAN; }
    else if (V.ovf || a.P.filter == 2) phase = KP_SCAN;
    else phase = KP_PEEL;
  }
  if (phase == KP_SCAN) {
    kscan(vg, a, q.k, q.s, q.j & 1, lds);
    ++q.s;
    due = 1;
    save(KP_SCAN);
  } else {
    // the decision above built the view of exactly these lists
    if (!have) V = kview(vg, a, q.from_scan ? SLOT_SCAN : q.j % 3, q.j & 1, lds, ref);
    kpeel(vg, a, q.k, q.j, ref, V, lds);
    if (lead) atomic_add_u32(&C->stats.v[6], 1u);
    ++q.j;
    due = 2;
    save(KP_PEEL);
  }
}

__global__ void k_kcore_seq_start(Ctrl *C) {
  if (threadIdx.x < 32) C->seq[0].v[threadIdx.x] = 0u;   // first scan of level 0
}

hipError_t kcore_seq_launch(const KArgs &a, unsigned L, int grid, hipStream_t s, bool start) {
  if (start) hipLaunchKernelGGL(k_kcore_seq_start, dim3(1), dim3(64), 0, s, a.w.ctrl);
  else hipLaunchKernelGGL(k_kcore_seq, dim3(grid), dim3(kBlock), 0, s, a, L);
  return hipGetLastError();
}

const void *kcore_seq_kernel() { return (const void *)k_kcore_seq; }

// Set-up for a run on G workgroups: core -1, current degrees, alive list 0 =
// every vertex, workgroup b holding a contiguous range of per = (n / G
// rounded up to 64) vertices.
__global__ void k_kcore_init(KArgs a, unsigned G) {
  const int n = a.g.n;
  const unsigned cap = alive_cap(a.w, G);
  const long long per = (((long long)n + G - 1) / G + 63) / 64 * 64;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (long long)gridDim.x * blockDim.x) {
    a.core[v] = -1;
    a.w.deg[v] = total_degree(a.g, (int)v);
    const long long b = v / per;
    a.w.alive[0][b * cap + (v - b * per)] = (int)v;
  }
  for (long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x; b < G;
       b += (long long)gridDim.x * blockDim.x) {
    const long long lo = b * per;
    const long long c = lo >= n ? 0 : (n - lo < per ? n - lo : per);
    a.w.alive_cnt[b] = (unsigned)c;
  }
  Ctrl *C = a.w.ctrl;
  if (blockIdx.x == 0) reset_barrier(C);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int i = 0; i < 32; ++i) { C->state.v[i] = 0; C->stats.v[i] = 0; C->aux.v[i] = 0; }
    C->error.v[0] = 0;
  }
  if (blockIdx.x == 1)
    for (int i = threadIdx.x; i < kStatLines * 4; i += blockDim.x) C->statw[i / 4].v[i % 4] = 0u;
}

hipError_t kcore_launch(const KArgs &a, int grid, hipStream_t s, bool init) {
  if (init) {
    int g = (a.g.n + kBlock - 1) / kBlock;
    g = g < 2 ? 2 : (g > 4096 ? 4096 : g);
    hipLaunchKernelGGL(k_kcore_init, dim3(g), dim3(kBlock), 0, s, a, (unsigned)grid);
  } else {
    hipLaunchKernelGGL(k_kcore_fused, dim3(grid), dim3(kBlock), 0, s, a);
  }
  return hipGetLastError();
}

const void *kcore_kernel() { return (const void *)k_kcore_fused; }

}  // namespace sx
