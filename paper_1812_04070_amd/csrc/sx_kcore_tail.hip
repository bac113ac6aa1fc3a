// The tail of the k-core decomposition (Section 6, "k-Core", carried on
// level by level as in sx_kcore.hip) in one workgroup.
//
// In R-MAT graphs the last levels keep a dense core of a few ten thousand
// vertices (s22: 35,827 vertices with 36 M arcs between them from level
// 213 on) that the grid peels a handful of vertices at a time: several
// hundred launches whose cost is their chain of dependent device-scope
// atomics and loads, not their work.  Once a level ends with at most
// Params::ktail vertices alive, the sequenced loop stops (KP_TAIL) and:
//
//   k_ktail_ids     numbers the alive vertices (core -1) 0..N-1;
//   k_ktail_offsets (one workgroup) lays out their rows of the alive
//                   subgraph, each padded to a multiple of 8 arcs, and the
//                   work items of the fill;
//   k_ktail_fill    writes each row: the local ids (16 bits) of the
//                   alive neighbours, over out- and in-arcs of a directed
//                   graph as the decrements of the peel count them;
//   k_ktail_peel    (one workgroup of 1024 threads) keeps the N current
//                   degrees in LDS and peels the remaining levels in
//                   rounds: every alive vertex of degree <= k is deleted
//                   (core k), then each listed vertex lowers the degree of
//                   its alive neighbours with LDS atomics; a round that
//                   deletes nothing moves k to the smallest degree left.
//
// The degree a vertex has when the level ends is exactly its number of
// alive neighbour arcs (every deleted neighbour lowered it once, the peel
// steps' skipped decrements only concern vertices deleted in that level),
// so the rows hold deg[v] entries; the fill checks this and raises
// SX_ERR_TAIL rather than write past a row.  The buffers are the
// frontier regions and the PageRank contributions, idle in a k-core run
// from the hand-over on.
#include "sx_frontier.hpp"
#include "sx_kernels.hpp"

namespace sx {

constexpr int kTailWaves = kTailThreads / 64;
constexpr int kTailList = 1024;         // deletions listed per round (one per thread)
constexpr int kTailIlp = 4;             // 16-byte loads in flight per lane
constexpr int kFillArcs = 512;          // arcs per fill work item (8 per lane)
constexpr unsigned kDel = 0x80000000u;  // degree word: deleted
constexpr unsigned short kPad = 0xFFFFu;

// Buffers of the tail (see above).
struct TailBufs {
  int *lid;                 // [n] vertex -> local id (alive vertices only)
  int *gid;                 // [N] local id -> vertex
  unsigned *fill;           // [N] arcs written into each row
  unsigned *roff;           // [N + 1] row offsets (multiples of 8)
  unsigned *witem;          // [N + 1] first fill work item of each vertex
  unsigned short *arcs;     // rows
  unsigned long long cap;   // entries of `arcs`
};

SX_DEV TailBufs tail_bufs(const Work &w) {
  TailBufs b;
  b.lid = (int *)w.contrib[0];
  b.gid = w.reg_s[0];
  b.fill = (unsigned *)w.reg_m[0];
  b.roff = (unsigned *)w.reg_s[1];
  b.witem = (unsigned *)w.reg_m[1];
  b.arcs = (unsigned short *)w.reg_l[0];
  b.cap = 4ull * w.tot_l;
  return b;
}

SX_DEV int total_deg(const DevGraph &g, int v) {
  int d = g.off[v + 1] - g.off[v];
  if (g.directed) d += g.in_off[v + 1] - g.in_off[v];
  return d;
}

__global__ void __launch_bounds__(kBlock) k_ktail_ids(KArgs a) {
  const TailBufs b = tail_bufs(a.w);
  Ctrl *C = a.w.ctrl;
  const int n = a.g.n;
  const long long stride = (long long)gridDim.x * kBlock;
  // wave-uniform trip count: the ballot and the leader's atomic need every lane
  for (long long w0 = (long long)blockIdx.x * kBlock + (threadIdx.x & ~63u); w0 < n; w0 += stride) {
    const long long v = w0 + lane_id();
    const bool alive = v < n && a.core[v] == -1;
    const uint64_t mk = ballot(alive);
    unsigned base = 0;
    if (lane_id() == 0 && mk) base = atomic_add_u32(&C->aux.v[KT_N], (unsigned)__popcll(mk));
    base = __shfl(base, 0);
    if (alive) {
      const unsigned id = base + lane_prefix(mk);
      if (id < (unsigned)kTailMax) {
        b.lid[v] = (int)id;
        b.gid[id] = (int)v;
        b.fill[id] = 0u;
      }
    }
  }
}

// Exclusive prefix of one value per thread over the workgroup (kTailThreads).
SX_DEV unsigned long long tail_scan(unsigned long long x, unsigned long long *sh, unsigned long long &total) {
  const int lane = lane_id(), w = threadIdx.x >> 6;
  unsigned long long incl = x;
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  if (lane == 63) sh[w] = incl;
  __syncthreads();
  unsigned long long before = 0, all = 0;
  for (int i = 0; i < kTailWaves; ++i) {
    if (i < w) before += sh[i];
    all += sh[i];
  }
  __syncthreads();
  total = all;
  return before + incl - x;
}

__global__ void __launch_bounds__(kTailThreads) k_ktail_offsets(KArgs a) {
  __shared__ unsigned long long sh[kTailWaves];
  const TailBufs b = tail_bufs(a.w);
  Ctrl *C = a.w.ctrl;
  const unsigned N = load_relaxed(&C->aux.v[KT_N]);
  if (N > (unsigned)kTailMax) {
    if (threadIdx.x == 0) store_relaxed(&C->error.v[0], (unsigned)SX_ERR_TAIL);
    return;
  }
  // thread t takes the contiguous ids [t * per, (t + 1) * per)
  const unsigned per = (N + kTailThreads - 1) / kTailThreads;
  const unsigned i0 = threadIdx.x * per < N ? threadIdx.x * per : N;
  const unsigned i1 = i0 + per < N ? i0 + per : N;
  unsigned long long sa = 0, sw = 0;
  for (unsigned i = i0; i < i1; ++i) {
    const int v = b.gid[i];
    sa += ((unsigned)a.w.deg[v] + 7u) & ~7u;
    sw += ((unsigned)total_deg(a.g, v) + kFillArcs - 1) / kFillArcs;
  }
  unsigned long long ta = 0, tw = 0;
  unsigned long long ra = tail_scan(sa, sh, ta);
  unsigned long long rw = tail_scan(sw, sh, tw);
  if (ta > b.cap || ta >= 0xFFFFFFF0ull || tw >= 0xFFFFFFF0ull) {
    if (threadIdx.x == 0) store_relaxed(&C->error.v[0], (unsigned)SX_ERR_TAIL);
    return;
  }
  for (unsigned i = i0; i < i1; ++i) {
    const int v = b.gid[i];
    const unsigned d = (unsigned)a.w.deg[v];
    b.roff[i] = (unsigned)ra;
    b.witem[i] = (unsigned)rw;
    // the padding of the row
    for (unsigned p = d; p < ((d + 7u) & ~7u); ++p) b.arcs[ra + p] = kPad;
    ra += (d + 7u) & ~7u;
    rw += ((unsigned)total_deg(a.g, v) + kFillArcs - 1) / kFillArcs;
  }
  if (threadIdx.x == 0) {
    b.roff[N] = (unsigned)ta;
    b.witem[N] = (unsigned)tw;
  }
}

// One wavefront per work item: kFillArcs arcs of one vertex's concatenated
// rows (out-arcs, then in-arcs of a directed graph), eight per lane.
__global__ void __launch_bounds__(kBlock) k_ktail_fill(KArgs a) {
  const TailBufs b = tail_bufs(a.w);
  Ctrl *C = a.w.ctrl;
  const DevGraph &g = a.g;
  const unsigned N = load_relaxed(&C->aux.v[KT_N]);
  if (N > (unsigned)kTailMax || load_relaxed(&C->error.v[0])) return;
  const unsigned items = b.witem[N];
  const int lane = lane_id();
  const unsigned nw = gridDim.x * (kBlock / 64);
  for (unsigned it = blockIdx.x * (kBlock / 64) + wave_in_wg(); it < items; it += nw) {
    // the vertex whose items hold `it`: witem[i] <= it < witem[i + 1]
    unsigned lo = 0, hi = N - 1;
    while (lo < hi) {
      const unsigned mid = (lo + hi + 1) >> 1;
      if (b.witem[mid] <= it) lo = mid;
      else hi = mid - 1;
    }
    const unsigned i = lo;
    const int v = b.gid[i];
    const int dout = g.off[v + 1] - g.off[v];
    const int td = total_deg(g, v);
    const int e0 = (int)(it - b.witem[i]) * kFillArcs;
    int u[8];
    bool ok[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = e0 + r * 64 + lane;
      ok[r] = e < td;
      u[r] = ok[r] ? (e < dout ? g.idx[g.off[v] + e] : g.in_idx[g.in_off[v] + (e - dout)]) : 0;
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) ok[r] = ok[r] && a.core[u[r]] == -1;
    unsigned cnt = 0;
#pragma unroll
    for (int r = 0; r < 8; ++r) cnt += (unsigned)__popcll(ballot(ok[r]));
    unsigned base = 0;
    if (lane == 0 && cnt) base = atomic_add_u32(&b.fill[i], cnt);
    base = __shfl(base, 0);
    const unsigned d = (unsigned)a.w.deg[v];
    if (base + cnt > d) {
      // more alive neighbours than the degree says: the rows would overlap
      if (lane == 0) store_relaxed(&C->error.v[0], (unsigned)SX_ERR_TAIL);
      continue;
    }
    unsigned pos = base;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint64_t mk = ballot(ok[r]);
      if (ok[r]) b.arcs[b.roff[i] + pos + lane_prefix(mk)] = (unsigned short)b.lid[u[r]];
      pos += (unsigned)__popcll(mk);
    }
  }
}

__global__ void __launch_bounds__(kTailThreads) k_ktail_peel(KArgs a) {
  __shared__ unsigned dg[kTailMax];
  __shared__ unsigned lroff[kTailList];      // row start of each listed vertex
  __shared__ unsigned lpre[kTailList + 1];   // prefix of their rows, in 8-arc chunks
  __shared__ unsigned long long sh[kTailWaves];
  __shared__ unsigned s_cnt, s_min[kTailWaves];
  const TailBufs b = tail_bufs(a.w);
  Ctrl *C = a.w.ctrl;
  const unsigned N = load_relaxed(&C->aux.v[KT_N]);
  if (N > (unsigned)kTailMax || load_relaxed(&C->error.v[0])) return;
  // every vertex the fill did not complete would peel with a wrong degree
  for (unsigned i = threadIdx.x; i < N; i += kTailThreads) {
    const unsigned d = (unsigned)a.w.deg[b.gid[i]];
    dg[i] = d;
    if (b.fill[i] != d) store_relaxed(&C->error.v[0], (unsigned)SX_ERR_TAIL);
  }
  __syncthreads();
  if (load_relaxed(&C->error.v[0])) return;
  unsigned k = load_relaxed(&C->aux.v[KT_K]);
  unsigned left = N, rounds = 0;
  const int lane = lane_id(), wv = threadIdx.x >> 6;
  const uint4 *arcs4 = (const uint4 *)b.arcs;
  while (left > 0) {
    if (rounds > 4u * N + 64u) {   // every round deletes a vertex or raises k past a degree
      if (threadIdx.x == 0) store_relaxed(&C->error.v[0], (unsigned)SX_ERR_TAIL);
      return;
    }
    ++rounds;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    // deletions of this round: every alive vertex of degree <= k that fits
    // the list (the others stay candidates for the next round)
    unsigned mn = 0xFFFFFFFFu;
    for (unsigned i = threadIdx.x; i < N; i += kTailThreads) {
      const unsigned d = dg[i];
      if (d & kDel) continue;
      if (d <= k) {
        const unsigned slot = atomicAdd(&s_cnt, 1u);
        if (slot < (unsigned)kTailList) {
          const unsigned r0 = b.roff[i], r1 = b.roff[i + 1];
          lroff[slot] = r0 >> 3;
          lpre[slot] = (r1 - r0) >> 3;
          dg[i] = d | kDel;
          a.core[b.gid[i]] = (int)k;
        }
      } else if (d < mn) {
        mn = d;
      }
    }
    mn = wave_min_u(mn);
    if (lane == 0) s_min[wv] = mn;
    __syncthreads();
    const unsigned listed = s_cnt < (unsigned)kTailList ? s_cnt : (unsigned)kTailList;
    if (listed == 0) {
      unsigned m = 0xFFFFFFFFu;
      for (int i = 0; i < kTailWaves; ++i) m = s_min[i] < m ? s_min[i] : m;
      k = m > k + 1 ? m : k + 1;
      __syncthreads();
      continue;
    }
    left -= listed;
    // prefix of the listed rows' chunk counts (one entry per thread)
    const unsigned len = threadIdx.x < listed ? lpre[threadIdx.x] : 0u;
    unsigned long long tot = 0;
    const unsigned ex = (unsigned)tail_scan(len, sh, tot);
    if (threadIdx.x < listed) lpre[threadIdx.x] = ex;
    if (threadIdx.x == 0) lpre[listed] = (unsigned)tot;
    __syncthreads();
    // the listed rows as one stream of 8-arc chunks: wavefront w walks a
    // contiguous share, its lanes on consecutive chunks (coalesced), kTailIlp
    // loads in flight per lane; each lane follows the row it is in forward
    const unsigned total = (unsigned)tot;
    const unsigned share = ((total + kTailWaves - 1) / kTailWaves + 63u) & ~63u;
    const unsigned c_lo = wv * share, c_hi = c_lo + share < total ? c_lo + share : total;
    unsigned own = 0;
    if (c_lo + lane < c_hi) {
      // the row holding chunk c_lo + lane: lpre[own] <= c < lpre[own + 1]
      unsigned lo = 0, hi = listed - 1;
      const unsigned c = c_lo + lane;
      while (lo < hi) {
        const unsigned mid = (lo + hi + 1) >> 1;
        if (lpre[mid] <= c) lo = mid;
        else hi = mid - 1;
      }
      own = lo;
    }
    for (unsigned c0 = c_lo; c0 < c_hi; c0 += 64u * kTailIlp) {
      uint4 x[kTailIlp];
      bool ok[kTailIlp];
#pragma unroll
      for (int r = 0; r < kTailIlp; ++r) {
        const unsigned c = c0 + 64u * r + lane;
        ok[r] = c < c_hi;
        if (ok[r]) {
          while (lpre[own + 1] <= c) ++own;
          x[r] = arcs4[lroff[own] + (c - lpre[own])];
        }
      }
#pragma unroll
      for (int r = 0; r < kTailIlp; ++r) {
        if (!ok[r]) continue;
        const unsigned wd[4] = {x[r].x, x[r].y, x[r].z, x[r].w};
#pragma unroll
        for (int h = 0; h < 8; ++h) {
          const unsigned t = (wd[h >> 1] >> ((h & 1) * 16)) & 0xFFFFu;
          if (t != kPad && t < N && !(dg[t] & kDel)) atomicSub(&dg[t], 1u);
        }
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) atomic_add_u32(&C->stats.v[6], rounds);
}

hipError_t kcore_tail_launch(const KArgs &a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_ktail_ids, dim3(grid), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_ktail_offsets, dim3(1), dim3(kTailThreads), 0, s, a);
  hipLaunchKernelGGL(k_ktail_fill, dim3(grid), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_ktail_peel, dim3(1), dim3(kTailThreads), 0, s, a);
  return hipGetLastError();
}

const void *kcore_tail_kernel() { return (const void *)k_ktail_peel; }

}  // namespace sx
