// Just-in-time task management (Section 4) on CDNA4.
//
// Worklists are split by degree into three bins (Section 4, step I):
//   small  (deg < t1)        one lane per vertex          (the Thread kernel)
//   medium (t1 <= deg < t2)  one 64-lane wavefront        (the Warp kernel)
//   large  (deg >= t2)       one workgroup per chunk of   (the CTA kernel; hub
//                            `chunk` arcs                  rows are split so a
//                                                          single vertex can
//                                                          occupy many CUs)
// Two filters build the next worklists (Section 4):
//   online filter  active vertices are appended while compute runs, one
//                  atomic per wavefront and bin (ballot -> popcount -> lane
//                  prefix); unsorted; overflows when a bin passes its capacity;
//   ballot filter  after a barrier, wavefronts scan contiguous tiles of the
//                  vertex metadata, turn the active test into 64-bit ballot
//                  words, and a grid-wide exclusive scan of the per-tile counts
//                  places every tile: the lists come out sorted and unique.
#pragma once

#include "sx_device.hpp"

namespace sx {

// Next-iteration worklists and their counters.
struct Lists {
  int *s;                       // small bin vertices
  int *m;                       // medium bin vertices
  unsigned long long *l;        // large bin items: chunk << 32 | vertex
  Counters *c;
  unsigned cap_s, cap_m, cap_l; // capacities (online filter overflow limits)
};

SX_DEV int bin_of(int deg, const Params &P) {
  return deg < P.t1 ? BIN_SMALL : (deg < P.t2 ? BIN_MED : BIN_LARGE);
}
SX_DEV int chunks_of(int deg, int chunk) {
  return (int)(((long long)deg + chunk - 1) / chunk);
}

// Per-wavefront statistics accumulated in registers and flushed once.
struct WaveStats {
  unsigned nf = 0;
  unsigned long long mf = 0;
};

// Online filter: every lane of the wavefront calls this (convergent).  Lanes
// with `valid` append vertex v (degree deg) to its bin.  Large vertices add
// one item per chunk of arcs.  Sets c->overflow when a bin passes capacity.
SX_DEV void online_append(bool valid, int v, int deg, const Lists &L, const Params &P, int chunk,
                          WaveStats &st) {
  const uint64_t any = ballot(valid);
  if (any == 0) return;
  const int lane = lane_id();
  const int b = valid ? bin_of(deg, P) : -1;
  if (valid) { st.nf += 1; st.mf += (unsigned long long)deg; }
#pragma unroll
  for (int bin = 0; bin < 2; ++bin) {
    const uint64_t mk = ballot(b == bin);
    if (mk == 0) continue;
    const int leader = __ffsll((long long)mk) - 1;
    unsigned base = 0;
    if (lane == leader) base = atomic_add_u32(&L.c->cnt[bin], (unsigned)__popcll(mk));
    base = __shfl(base, leader);
    const unsigned cap = bin == 0 ? L.cap_s : L.cap_m;
    if (b == bin) {
      const unsigned pos = base + lane_prefix(mk);
      if (pos < cap) (bin == 0 ? L.s : L.m)[pos] = v;
    }
    if (lane == leader && base + (unsigned)__popcll(mk) > cap) store_relaxed(&L.c->overflow, 1u);
  }
  const uint64_t ml = ballot(b == BIN_LARGE);
  if (ml) {
    const int k = (b == BIN_LARGE) ? chunks_of(deg, chunk) : 0;
    const int incl = wave_incl_scan(k);
    const int total = __shfl(incl, 63);
    unsigned base = 0;
    if (lane == 63) base = atomic_add_u32(&L.c->cnt[BIN_LARGE], (unsigned)total);
    base = __shfl(base, 63);
    const unsigned pos = base + (unsigned)(incl - k);
    for (int c = 0; c < k; ++c)
      if (pos + c < L.cap_l) L.l[pos + c] = ((unsigned long long)c << 32) | (unsigned)v;
    if (lane == 63 && base + (unsigned)total > L.cap_l) store_relaxed(&L.c->overflow, 1u);
  }
}

// Flush per-wavefront frontier statistics into the counters (one atomic per
// wavefront per phase).
SX_DEV void flush_stats(WaveStats &st, Counters *c) {
  const int nf = wave_sum_i((int)st.nf);
  const long long mf = wave_sum_ll((long long)st.mf);
  if (lane_id() == 0 && nf) {
    atomic_add_u32(&c->nf, (unsigned)nf);
    atomic_add_u64(&c->mf, (unsigned long long)mf);
  }
  st.nf = 0; st.mf = 0;
}

// ------------------------------------------------------- ballot filter ---
// Tiles: global wavefront gw owns vertices [gw*tile, (gw+1)*tile), tile a
// multiple of 64, so consecutive wavefronts own consecutive ranges and the
// concatenation in wavefront order is sorted.
struct Tiling {
  int tile;
  unsigned nwaves;
  SX_DEV Tiling(int n, unsigned nw) : nwaves(nw) {
    long long t = ((long long)n + nw - 1) / nw;
    tile = (int)((t + 63) / 64 * 64);
    if (tile < 64) tile = 64;
  }
};

// Pass 1: evaluate `pred(v) -> bool` and the degree for every vertex of this
// wavefront's tile; store ballot words per bin; accumulate per-wave and
// per-workgroup counts.  `wavecnt` (global) receives [gw][NBINS] counts;
// `wgc` (global) the workgroup totals.  Every thread of the workgroup calls.
template <class Pred, class Deg>
SX_DEV void ballot_count(const VGrid &vg, int n, const Tiling &T, Pred pred, Deg degree, const Params &P, int chunk,
                         unsigned long long *const bits[NBINS], unsigned *wavecnt, WgCount *wgc,
                         unsigned *lds /* kWaves * 6 */) {
  const unsigned gw = vg.bid * kWaves + wave_in_wg();
  const int lane = lane_id();
  const long long start = (long long)gw * T.tile;
  unsigned c[NBINS] = {0, 0, 0};
  unsigned long long mf = 0;
  for (int s = 0; s < T.tile; s += 64) {
    const long long v = start + s + lane;
    bool p = false;
    int d = 0;
    if (v < n) {
      p = pred((int)v);
      if (p) d = degree((int)v);
    }
    const int b = p ? bin_of(d, P) : -1;
    if (start + s < n) {
      const long long word = (start + s) >> 6;
#pragma unroll
      for (int bin = 0; bin < NBINS; ++bin) {
        const uint64_t mk = ballot(b == bin);
        if (lane == 0) bits[bin][word] = mk;
        if (bin < BIN_LARGE) c[bin] += (unsigned)__popcll(mk);
      }
      const int k = (b == BIN_LARGE) ? chunks_of(d, chunk) : 0;
      c[BIN_LARGE] += (unsigned)wave_sum_i(k);
      mf += (unsigned long long)wave_sum_ll(p ? d : 0);
    }
  }
  if (lane == 0) {
    for (int bin = 0; bin < NBINS; ++bin) {
      wavecnt[gw * NBINS + bin] = c[bin];
      lds[wave_in_wg() * 6 + bin] = c[bin];
    }
    lds[wave_in_wg() * 6 + 3] = (unsigned)(mf & 0xffffffffu);
    lds[wave_in_wg() * 6 + 4] = (unsigned)(mf >> 32);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    WgCount t{};
    for (int w = 0; w < kWaves; ++w) {
      for (int bin = 0; bin < NBINS; ++bin) t.cnt[bin] += lds[w * 6 + bin];
      t.mf += (unsigned long long)lds[w * 6 + 3] | ((unsigned long long)lds[w * 6 + 4] << 32);
    }
    // vertices = small + medium + (large vertices, counted from the words in pass 2)
    wgc[vg.bid] = t;
  }
  __syncthreads();
}

// Pass 2: place this wavefront's actives (position i of the scanned range
// holds vertex vertex_of(i)).  Grid totals are returned in `tot`, identical
// in every workgroup.
template <class Deg, class VertexOf>
SX_DEV void ballot_write(const VGrid &vg, int n, const Tiling &T, Deg degree, VertexOf vertex_of, int chunk,
                         unsigned long long *const bits[NBINS], const unsigned *wavecnt,
                         const WgCount *wgc, int *out_s, int *out_m, unsigned long long *out_l,
                         WgCount &tot, unsigned *lds /* kWaves * 8 */, long long *red /* kWaves */) {
  // workgroup base = sum over lower workgroups, grid totals = sum over all;
  // 32-bit counts (n < 2^31 and large items <= n + m / chunk).
  unsigned acc[2 * NBINS];
#pragma unroll
  for (int i = 0; i < 2 * NBINS; ++i) acc[i] = 0;
  unsigned long long mf = 0;
#pragma unroll 1
  for (unsigned b = threadIdx.x; b < vg.nb; b += kBlock) {
    const WgCount w = wgc[b];
    const bool lower = b < vg.bid;
#pragma unroll
    for (int bin = 0; bin < NBINS; ++bin) {
      acc[NBINS + bin] += w.cnt[bin];
      acc[bin] += lower ? w.cnt[bin] : 0u;
    }
    mf += w.mf;
  }
  // workgroup reduction of the 6 counts and mf through LDS
#pragma unroll
  for (int i = 0; i < 2 * NBINS; ++i) acc[i] = (unsigned)wave_sum_i((int)acc[i]);
  mf = (unsigned long long)wave_sum_ll((long long)mf);
  __syncthreads();
  if (lane_id() == 0) {
#pragma unroll
    for (int i = 0; i < 2 * NBINS; ++i) lds[wave_in_wg() * 8 + i] = acc[i];
    red[wave_in_wg()] = (long long)mf;
  }
  __syncthreads();
  unsigned r[2 * NBINS];
#pragma unroll
  for (int i = 0; i < 2 * NBINS; ++i) {
    unsigned t = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) t += lds[w * 8 + i];
    r[i] = t;
  }
  unsigned long long mft = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) mft += (unsigned long long)red[w];
  __syncthreads();
  const unsigned wv = wave_in_wg();
  const unsigned gw = vg.bid * kWaves + wv;
  unsigned pos[NBINS];
#pragma unroll
  for (int bin = 0; bin < NBINS; ++bin) {
    unsigned p = r[bin];
#pragma unroll 1
    for (unsigned w = vg.bid * kWaves; w < gw; ++w) p += wavecnt[w * NBINS + bin];
    pos[bin] = p;
  }
  const int lane = lane_id();
  const long long start = (long long)gw * T.tile;
  unsigned large_vertices = 0;
  for (int s = 0; s < T.tile && start + s < n; s += 64) {
    const long long word = (start + s) >> 6;
    const uint64_t ms = bits[BIN_SMALL][word];
    const uint64_t mm = bits[BIN_MED][word];
    const uint64_t ml = bits[BIN_LARGE][word];
    const bool in_any = ((ms | mm | ml) >> lane) & 1ull;
    const int v = in_any ? vertex_of((int)(start + s + lane)) : 0;
    if ((ms >> lane) & 1ull) out_s[pos[BIN_SMALL] + lane_prefix(ms)] = v;
    if ((mm >> lane) & 1ull) out_m[pos[BIN_MED] + lane_prefix(mm)] = v;
    pos[BIN_SMALL] += (unsigned)__popcll(ms);
    pos[BIN_MED] += (unsigned)__popcll(mm);
    if (ml) {
      const int k = ((ml >> lane) & 1ull) ? chunks_of(degree(v), chunk) : 0;
      const int incl = wave_incl_scan(k);
      const unsigned p = pos[BIN_LARGE] + (unsigned)(incl - k);
      for (int c = 0; c < k; ++c) out_l[p + c] = ((unsigned long long)c << 32) | (unsigned)v;
      pos[BIN_LARGE] += (unsigned)__shfl(incl, 63);
      large_vertices += (unsigned)__popcll(ml);
    }
  }
  tot.cnt[0] = r[NBINS + 0];
  tot.cnt[1] = r[NBINS + 1];
  tot.cnt[2] = r[NBINS + 2];
  tot.mf = mft;
  tot.nf = 0;  // filled by the caller when needed
  (void)large_vertices;
}

// ------------------------------------------------- worklist traversal ---
// Visit every arc of every worklist entry.  `op(v, u, arc, lane_valid)` is
// called convergently by whole wavefronts; it returns nothing and performs
// Compute + Combine for arc v->u and the online append itself.

// Small bin: a wavefront takes 64 vertices, stages their row starts and a
// prefix sum of their degrees in LDS, then walks the concatenated arcs 64 at
// a time (one arc per lane), so lanes stay busy however degrees vary.
// Worklist entries outside [0, n) are skipped (a defence: lists only ever
// hold vertex ids, but a read never leaves the CSR).
template <class Op>
SX_DEV void visit_small(int n, const int *list, unsigned cnt, const int *off, const int *idx, Op &op,
                        unsigned gw, unsigned nwaves, int *lds /* 3*64 per wave */) {
  const int lane = lane_id();
  int *l_v = lds, *l_beg = lds + 64, *l_ex = lds + 128;
  for (unsigned c = gw; c * 64u < cnt; c += nwaves) {
    const unsigned i = c * 64u + lane;
    int v = -1, beg = 0, deg = 0;
    if (i < cnt) {
      const int x = list[i];
      if ((unsigned)x < (unsigned)n) {
        v = x;
        beg = off[v];
        deg = off[v + 1] - beg;
      }
    }
    const int incl = wave_incl_scan(deg);
    const int total = __shfl(incl, 63);
    l_v[lane] = v;
    l_beg[lane] = beg;
    l_ex[lane] = incl - deg;
    __builtin_amdgcn_wave_barrier();
    for (int j = 0; j < total; j += 64) {
      const int e = j + lane;
      const bool ok = e < total;
      int owner = 0;
      if (ok) {
        // largest owner with l_ex[owner] <= e
        int lo = 0, hi = 63;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (l_ex[mid] <= e) lo = mid; else hi = mid - 1;
        }
        owner = lo;
      }
      const int arc = ok ? l_beg[owner] + (e - l_ex[owner]) : 0;
      const int vv = ok ? l_v[owner] : 0;
      const int u = ok ? idx[arc] : 0;
      op(vv, u, arc, ok);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Medium bin: one wavefront per vertex.
template <class Op>
SX_DEV void visit_med(int n, const int *list, unsigned cnt, const int *off, const int *idx, Op &op,
                      unsigned gw, unsigned nwaves) {
  const int lane = lane_id();
  for (unsigned i = gw; i < cnt; i += nwaves) {
    const int v = list[i];
    if ((unsigned)v >= (unsigned)n) continue;
    const int beg = off[v], end = off[v + 1];
    for (int a = beg; a < end; a += 64) {
      const int arc = a + lane;
      const bool ok = arc < end;
      const int u = ok ? idx[arc] : 0;
      op(v, u, arc, ok);
    }
  }
}

// Large bin: one workgroup per item (a chunk of `chunk` arcs of one vertex).
template <class Op>
SX_DEV void visit_large(const VGrid &vg, int n, const unsigned long long *list, unsigned cnt,
                        const int *off, const int *idx, int chunk, Op &op) {
  for (unsigned i = vg.bid; i < cnt; i += vg.nb) {
    const unsigned long long it = list[i];
    const int v = (int)(it & 0xffffffffu);
    if ((unsigned)v >= (unsigned)n) continue;
    const int c = (int)(it >> 32);
    const int vb = off[v], ve = off[v + 1];
    const long long b0 = (long long)vb + (long long)c * chunk;
    const int beg = (int)b0;
    const int end = (int)((b0 + chunk) < ve ? (b0 + chunk) : ve);
    for (int a = beg; a < end; a += kBlock) {
      const int arc = a + (int)threadIdx.x;
      const bool ok = arc < end;
      const int u = ok ? idx[arc] : 0;
      op(v, u, arc, ok);
    }
  }
}

}  // namespace sx
