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
// Task management: a level starts with a ballot-filter scan over the list of
// vertices still alive (sorted, binned frontier of degree <= k, plus the
// compacted list of survivors and their minimum degree so that empty levels
// are skipped); the deletions within a level are chained by the online
// filter.  The JIT switch of Section 4 applies: an overflowing online filter
// is replaced by a fresh scan of the alive list.  A directed graph counts in-
// plus out-arcs; deleting v decrements through both its CSR and CSC rows.
#include "sx_frontier.hpp"
#include "sx_kernels.hpp"

namespace sx {


struct LdsK {
  int small[kWaves][192];
  unsigned cnt[kWaves * 8];
  long long red[kWaves];
};

SX_DEV int total_degree(const DevGraph &g, int v) {
  int d = g.off[v + 1] - g.off[v];
  if (g.directed) d += g.in_off[v + 1] - g.in_off[v];
  return d;
}

// aux line layout: scan number s reads alive list (s & 1) whose length is
// aux[s % 3], appends the survivors to list (s+1) & 1, length aux[(s+1) % 3],
// and their minimum degree to aux[3 + s % 3]; it resets the slots of scan
// s+2 (length) and s+1 (minimum), which nobody reads any more.  [10] level
// k, [11] scan number, [12] next step kind (0 scan, 1 peel), [13] step index.
enum { AUX_K = 10, AUX_SCAN = 11, AUX_KIND = 12, AUX_STEP = 13 };

// Level scan, pass 1: positions [0, cA) of the alive list.
SX_DEV void kscan_pass1(const KArgs &a, int k, int scan_no, LdsK &lds) {
  const Work &w = a.w;
  Ctrl *C = w.ctrl;
  const int pa = scan_no & 1;
  const int cA = (int)load_relaxed(&C->aux.v[scan_no % 3]);
  const int *A = w.alive[pa];
  int *B = w.alive[pa ^ 1];
  unsigned *surv = &C->aux.v[(scan_no + 1) % 3];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    store_relaxed(&C->aux.v[(scan_no + 2) % 3], 0u);
    store_relaxed(&C->aux.v[3 + (scan_no + 1) % 3], 0xFFFFFFFFu);
  }
  const DevGraph &g = a.g;
  Tiling T(cA, gridDim.x * kWaves);
  // survivors: alive with degree > k, appended (one atomic per wavefront)
  {
    const unsigned gw = blockIdx.x * kWaves + wave_in_wg();
    const long long start = (long long)gw * T.tile;
    unsigned mind = 0xFFFFFFFFu;
    for (int s = 0; s < T.tile && start + s < cA; s += 64) {
      const long long i = start + s + lane_id();
      bool keep = false;
      int v = 0;
      if (i < cA) {
        v = A[i];
        if (a.core[v] == -1) {
          const int d = w.deg[v];
          if (d > k) { keep = true; mind = (unsigned)d < mind ? (unsigned)d : mind; }
        }
      }
      const uint64_t mk = ballot(keep);
      if (mk) {
        unsigned base = 0;
        if (lane_id() == 0) base = atomic_add_u32(surv, (unsigned)__popcll(mk));
        base = __shfl(base, 0);
        if (keep) B[base + lane_prefix(mk)] = v;
      }
    }
    mind = wave_min_u(mind);
    if (lane_id() == 0 && mind != 0xFFFFFFFFu)
      __hip_atomic_fetch_min(&C->aux.v[3 + scan_no % 3], mind, __ATOMIC_RELAXED, SX_AG);
  }
  // frontier: alive with degree <= k, ballot words per degree bin
  auto pred = [&](int i) {
    const int v = A[i];
    return a.core[v] == -1 && w.deg[v] <= k;
  };
  auto degree = [&](int i) { return total_degree(g, A[i]); };
  ballot_count(hw_grid(), cA, T, pred, degree, a.P, a.P.chunk, w.bits, w.wavecnt, w.wgc, lds.cnt);
}

// Level scan, pass 2: sorted binned frontier into parity `qp`, counts into
// slot `slot`; returns the frontier size (vertices + large items, identical
// in all workgroups).
SX_DEV unsigned kscan_pass2(const KArgs &a, int qp, int slot, int scan_no, LdsK &lds) {
  const Work &w = a.w;
  Ctrl *C = w.ctrl;
  const int cA = (int)load_relaxed(&C->aux.v[scan_no % 3]);
  const int *A = w.alive[scan_no & 1];
  const DevGraph &g = a.g;
  Tiling T(cA, gridDim.x * kWaves);
  auto degree = [&](int v) { return total_degree(g, v); };
  auto vof = [&](int i) { return A[i]; };
  WgCount tot;
  ballot_write(hw_grid(), cA, T, degree, vof, a.P.chunk, w.bits, w.wavecnt, w.wgc, w.q[qp][0], w.q[qp][1],
               w.ql[qp], tot, lds.cnt, lds.red);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Counters *q = &C->q[slot];
    store_relaxed(&q->cnt[0], tot.cnt[0]);
    store_relaxed(&q->cnt[1], tot.cnt[1]);
    store_relaxed(&q->cnt[2], tot.cnt[2]);
    store_relaxed(&q->nf, tot.cnt[0] + tot.cnt[1] + tot.cnt[2]);
    store_relaxed(&q->overflow, 0u);
    atomic_add_u32(&C->stats.v[4], 1u);
  }
  return tot.cnt[0] + tot.cnt[1] + tot.cnt[2];
}

// Peel step: delete the frontier (slot `slot`, parity `qp`), decrement the
// neighbours, online filter into slot (slot+1)%3, parity qp^1.
SX_DEV void kpeel(const KArgs &a, int k, int qp, int slot, LdsK &lds) {
  const Work &w = a.w;
  Ctrl *C = w.ctrl;
  Counters *cur = &C->q[slot], *nxt = &C->q[(slot + 1) % 3];
  // counts are clamped to the list capacities: reads never leave the lists
  const unsigned cs = min(load_relaxed(&cur->cnt[0]), w.qcap_small),
                 cm = min(load_relaxed(&cur->cnt[1]), w.qcap_med),
                 cl = min(load_relaxed(&cur->cnt[2]), w.qcap_large);
  const DevGraph &g = a.g;
  // mark the frontier deleted with core number k
  {
    const unsigned tid = blockIdx.x * kBlock + threadIdx.x, nt = gridDim.x * kBlock;
    const unsigned un = (unsigned)g.n;
    for (unsigned i = tid; i < cs; i += nt) {
      const int v = w.q[qp][0][i];
      if ((unsigned)v < un) a.core[v] = k;
    }
    for (unsigned i = tid; i < cm; i += nt) {
      const int v = w.q[qp][1][i];
      if ((unsigned)v < un) a.core[v] = k;
    }
    for (unsigned i = tid; i < cl; i += nt) {
      const unsigned long long it = w.ql[qp][i];
      const unsigned v = (unsigned)(it & 0xffffffffu);
      if ((it >> 32) == 0 && v < un) a.core[v] = k;
    }
  }
  Lists NL;
  NL.s = w.q[qp ^ 1][0];
  NL.m = w.q[qp ^ 1][1];
  NL.l = w.ql[qp ^ 1];
  NL.c = nxt;
  NL.cap_s = a.P.online_cap < w.qcap_small ? a.P.online_cap : w.qcap_small;
  NL.cap_m = a.P.online_cap < w.qcap_med ? a.P.online_cap : w.qcap_med;
  NL.cap_l = a.P.online_cap < w.qcap_large ? a.P.online_cap : w.qcap_large;
  WaveStats st;
  long long edges = 0;
  int *deg = w.deg;
  auto op = [&](int v, int u, int arc, bool ok) {
    (void)v; (void)arc;
    bool act = false;
    int du = 0;
    if (ok) {
      ++edges;
      if (load_relaxed(&deg[u]) > k) {
        const int old = atomic_sub_i32(&deg[u], 1);
        if (old == k + 1) { act = true; du = total_degree(g, u); }
      }
    }
    online_append(act, u, du, NL, a.P, a.P.chunk, st);
  };
  const unsigned gw = blockIdx.x * kWaves + wave_in_wg();
  const unsigned nw = gridDim.x * kWaves;
  for (int pass = 0; pass < (g.directed ? 2 : 1); ++pass) {
    const int *off = pass ? g.in_off : g.off;
    const int *idx = pass ? g.in_idx : g.idx;
    visit_large(hw_grid(), g.n, w.ql[qp], cl, off, idx, a.P.chunk, op);
    visit_med(g.n, w.q[qp][1], cm, off, idx, op, gw, nw);
    visit_small(g.n, w.q[qp][0], cs, off, idx, op, gw, nw, lds.small[wave_in_wg()]);
  }
  flush_stats(st, nxt);
  const long long e = wave_sum_ll(edges);
  if (lane_id() == 0 && e) atomic_add_u64((unsigned long long *)&C->stats.v[0], (unsigned long long)e);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    atomic_add_u64((unsigned long long *)&C->stats.v[2], (unsigned long long)(cs + cm) + cl);
    Counters *old = &C->q[(slot + 2) % 3];
    for (int b = 0; b < NBINS; ++b) store_relaxed(&old->cnt[b], 0u);
    store_relaxed(&old->nf, 0u);
    store_relaxed(&old->mf, 0ull);
    store_relaxed(&old->overflow, 0u);
  }
}

// Persistent kernel: the whole decomposition in one launch.
__global__ void __launch_bounds__(kBlock) k_kcore_fused(KArgs a) {
  __shared__ LdsK lds;
  Ctrl *C = a.w.ctrl;
  GridBarrier bar(C, load_relaxed(&C->bar_gen.v[0]));
  int k = (int)load_relaxed(&C->aux.v[AUX_K]);
  int scan_no = (int)load_relaxed(&C->aux.v[AUX_SCAN]);
  int kind = (int)load_relaxed(&C->aux.v[AUX_KIND]);
  int step = (int)load_relaxed(&C->aux.v[AUX_STEP]);
  auto save = [&](int reason) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      store_relaxed(&C->state.v[0], (unsigned)reason);
      store_relaxed(&C->aux.v[AUX_K], (unsigned)k);
      store_relaxed(&C->aux.v[AUX_SCAN], (unsigned)scan_no);
      store_relaxed(&C->aux.v[AUX_KIND], (unsigned)kind);
      store_relaxed(&C->aux.v[AUX_STEP], (unsigned)step);
    }
  };
  if (load_relaxed(&C->state.v[0]) != EXIT_NONE || bar.failed()) return;
  // every step removes at least one vertex or advances k; bound the loop
  const long long limit = 4ll * a.g.n + 64;
  for (long long guard = 0;; ++guard) {
    if (guard > limit) { save(EXIT_LIMIT); return; }
    const int slot = (step + 1) % 3, qp = (step + 1) & 1;
    if (kind == 0) {
      // scan: frontier of the level into (slot, qp), survivors into the
      // other alive list
      kscan_pass1(a, k, scan_no, lds);
      if (!bar.sync()) { save(EXIT_ERROR); return; }
      const unsigned nfr = kscan_pass2(a, qp, slot, scan_no, lds);
      if (!bar.sync()) { save(EXIT_ERROR); return; }
      const unsigned survivors = load_relaxed(&C->aux.v[(scan_no + 1) % 3]);
      const unsigned mind = load_relaxed(&C->aux.v[3 + scan_no % 3]);
      ++scan_no;
      if (nfr == 0) {
        if (survivors == 0) { save(EXIT_DONE); return; }
        // empty level: jump to the smallest surviving degree
        k = (int)mind > k + 1 ? (int)mind : k + 1;
        continue;
      }
      kind = 1;
      ++step;
    } else {
      // peel the frontier of step-1's output
      const int cslot = step % 3, cqp = step & 1;
      kpeel(a, k, cqp, cslot, lds);
      if (!bar.sync()) { save(EXIT_ERROR); return; }
      if (blockIdx.x == 0 && threadIdx.x == 0) atomic_add_u32(&C->stats.v[6], 1u);
      Counters *nx = &C->q[(cslot + 1) % 3];
      const unsigned nf = load_relaxed(&nx->nf);
      const unsigned ovf = load_relaxed(&nx->overflow);
      if (nf == 0) { ++k; kind = 0; continue; }
      if (ovf || a.P.filter == 2) { kind = 0; continue; }   // rebuild by a scan at the same k
      ++step;
    }
    (void)slot;
  }
}

// Sequenced form of the same loop: one launch per phase (scan pass 1, scan
// pass 2, peel), the decision taken at the start of the launch after a
// scan or a peel; launch L reads Ctrl::seq[L & 1] and writes seq[(L+1) & 1]:
// [0] phase [1] k [2] scan number [3] step [4] decision due (1 after a scan,
// 2 after a peel).
enum : unsigned { KP_SCAN1 = 0, KP_SCAN2 = 1, KP_PEEL = 2, KP_DONE = 6, KP_ERROR = 7, KP_LIMIT = 8 };

__global__ void __launch_bounds__(kBlock) k_kcore_seq(KArgs a, unsigned L) {
  __shared__ LdsK lds;
  Ctrl *C = a.w.ctrl;
  const Line &in = C->seq[L & 1];
  Line &out = C->seq[(L + 1) & 1];
  unsigned phase = load_relaxed(&in.v[0]);
  int k = (int)load_relaxed(&in.v[1]);
  int scan_no = (int)load_relaxed(&in.v[2]);
  int step = (int)load_relaxed(&in.v[3]);
  unsigned due = load_relaxed(&in.v[4]);
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  auto save = [&](unsigned ph) {
    if (lead) {
      store_relaxed(&out.v[0], ph);
      store_relaxed(&out.v[1], (unsigned)k);
      store_relaxed(&out.v[2], (unsigned)scan_no);
      store_relaxed(&out.v[3], (unsigned)step);
      store_relaxed(&out.v[4], due);
    }
  };
  if (phase >= KP_DONE) { save(phase); return; }
  if (load_relaxed(&C->error.v[0])) { due = 0; save(KP_ERROR); return; }
  if (step > 4 * a.g.n + 64) { due = 0; save(KP_LIMIT); return; }
  if (due == 1) {
    // after a scan (scan_no already advanced): frontier of the level or a jump
    const int s_prev = scan_no - 1;
    Counters *q = &C->q[(step + 1) % 3];
    const unsigned nfr = load_relaxed(&q->nf);
    const unsigned survivors = load_relaxed(&C->aux.v[(s_prev + 1) % 3]);
    const unsigned mind = load_relaxed(&C->aux.v[3 + s_prev % 3]);
    if (nfr == 0) {
      if (survivors == 0) { due = 0; save(KP_DONE); return; }
      k = (int)mind > k + 1 ? (int)mind : k + 1;
      phase = KP_SCAN1;
    } else {
      phase = KP_PEEL;
      ++step;
    }
    due = 0;
  } else if (due == 2) {
    Counters *nx = &C->q[(step % 3 + 1) % 3];
    const unsigned nf = load_relaxed(&nx->nf);
    const unsigned ovf = load_relaxed(&nx->overflow);
    if (nf == 0) { ++k; phase = KP_SCAN1; }
    else if (ovf || a.P.filter == 2) phase = KP_SCAN1;
    else { phase = KP_PEEL; ++step; }
    due = 0;
  }
  switch (phase) {
    case KP_SCAN1:
      kscan_pass1(a, k, scan_no, lds);
      save(KP_SCAN2);
      return;
    case KP_SCAN2:
      kscan_pass2(a, (step + 1) & 1, (step + 1) % 3, scan_no, lds);
      ++scan_no;
      due = 1;
      save(KP_SCAN2);
      return;
    case KP_PEEL:
      kpeel(a, k, step & 1, step % 3, lds);
      if (lead) atomic_add_u32(&C->stats.v[6], 1u);
      due = 2;
      save(KP_PEEL);
      return;
  }
}

__global__ void k_kcore_seq_start(Ctrl *C) {
  if (threadIdx.x < 32) C->seq[0].v[threadIdx.x] = 0u;   // scan 1 of level 0
}

hipError_t kcore_seq_launch(const KArgs &a, unsigned L, int grid, hipStream_t s, bool start) {
  if (start) hipLaunchKernelGGL(k_kcore_seq_start, dim3(1), dim3(64), 0, s, a.w.ctrl);
  else hipLaunchKernelGGL(k_kcore_seq, dim3(grid), dim3(kBlock), 0, s, a, L);
  return hipGetLastError();
}

const void *kcore_seq_kernel() { return (const void *)k_kcore_seq; }

__global__ void k_kcore_init(KArgs a) {
  const int n = a.g.n;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (long long)gridDim.x * blockDim.x) {
    a.core[v] = -1;
    a.w.deg[v] = total_degree(a.g, (int)v);
    a.w.alive[0][v] = (int)v;
  }
  if (blockIdx.x == 0) reset_barrier(a.w.ctrl);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Ctrl *C = a.w.ctrl;
    for (int s = 0; s < 3; ++s) {
      for (int b = 0; b < NBINS; ++b) C->q[s].cnt[b] = 0;
      C->q[s].nf = 0;
      C->q[s].mf = 0;
      C->q[s].overflow = 0;
    }
    for (int i = 0; i < 32; ++i) { C->state.v[i] = 0; C->stats.v[i] = 0; C->aux.v[i] = 0; }
    C->error.v[0] = 0;
    C->aux.v[0] = (unsigned)n;       // alive list 0 = all vertices
    C->aux.v[3] = 0xFFFFFFFFu;
    C->aux.v[4] = 0xFFFFFFFFu;
    C->aux.v[5] = 0xFFFFFFFFu;
  }
}

hipError_t kcore_launch(const KArgs &a, int grid, hipStream_t s, bool init) {
  if (init) {
    int g = (a.g.n + kBlock - 1) / kBlock;
    g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
    hipLaunchKernelGGL(k_kcore_init, dim3(g), dim3(kBlock), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_kcore_fused, dim3(grid), dim3(kBlock), 0, s, a);
  }
  return hipGetLastError();
}

const void *kcore_kernel() { return (const void *)k_kcore_fused; }

}  // namespace sx
