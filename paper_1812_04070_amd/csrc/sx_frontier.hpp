// Just-in-time task management (Section 4) on CDNA4.
//
// Worklists are split by degree into three bins (Section 4, step I):
//   small  (deg < t1)        processed a lane per vertex   (the Thread kernel)
//   medium (t1 <= deg < t2)  a 64-lane wavefront per vertex (the Warp kernel)
//   large  (deg >= t2)       a workgroup per chunk of       (the CTA kernel; hub
//                            `chunk` arcs                    rows are split so a
//                                                           single vertex can
//                                                           occupy many CUs)
//
// Storage follows the paper's thread bins (Section 3.3): every workgroup
// appends into its own region of each bin array -- positions come from an
// LDS counter, so building a worklist needs no global atomic at all -- and
// at the end of the phase publishes one record per workgroup (items per
// bin, vertices, their arcs, overflow).  On MI355X this matters: every
// device-scope atomic on one address is serialised (~11 ns each, measured),
// so one atomic per wavefront on a shared queue counter costs ~70 us per
// phase with 6,000 wavefronts.  The next phase builds, in LDS, the prefix of
// the records and reads item i of a bin from the region that holds it: the
// concatenation of the regions in workgroup order is the worklist.
//
// Two filters fill the bins (Section 4):
//   online filter  active vertices are appended while compute runs (ballot ->
//                  popcount -> one LDS atomic per wavefront and bin -> lane
//                  offsets by mbcnt); a region that is full sets the
//                  overflow flag: the JIT control then rebuilds the lists with
//   ballot filter  each workgroup scans a contiguous range of vertex metadata
//                  in wavefront-contiguous tiles, turns the active test into
//                  64-bit ballot words, counts them, and writes the actives in
//                  tile order: the lists come out sorted and unique.
#pragma once

#include "sx_device.hpp"

namespace sx {

SX_DEV int bin_of(int deg, const Params &P) {
  return deg < P.t1 ? BIN_SMALL : (deg < P.t2 ? BIN_MED : BIN_LARGE);
}
SX_DEV int chunks_of(int deg, int chunk) {
  return (int)(((long long)deg + chunk - 1) / chunk);
}

// One parity of the bin arrays, seen by a grid of G workgroups.
struct Regions {
  int *s, *m;
  unsigned long long *l;
  unsigned cap_s, cap_m, cap_l;
};
SX_DEV Regions regions(const Work &w, int parity, unsigned G) {
  Regions r;
  r.s = w.reg_s[parity];
  r.m = w.reg_m[parity];
  r.l = w.reg_l[parity];
  r.cap_s = w.tot_s / G;
  r.cap_m = w.tot_m / G;
  r.cap_l = w.tot_l / G;
  return r;
}

// ---------------------------------------------------------- producing ---
struct LdsBins {
  unsigned cnt[NBINS];
  unsigned ovf;
  unsigned lim[NBINS];
  unsigned nf[kWaves];
  unsigned long long mf[kWaves];
};

// Per-lane frontier statistics, reduced once at the end of the phase.
struct WaveStats {
  unsigned nf = 0;
  unsigned long long mf = 0;
};

// Start of a producing phase (all threads).  `limit` caps each bin's region
// use (the online-filter overflow threshold); 0 = the whole region.
SX_DEV void bins_begin(LdsBins &b, const Regions &R, unsigned limit) {
  if (threadIdx.x == 0) {
    for (int i = 0; i < NBINS; ++i) b.cnt[i] = 0;
    b.ovf = 0;
    b.lim[0] = limit && limit < R.cap_s ? limit : R.cap_s;
    b.lim[1] = limit && limit < R.cap_m ? limit : R.cap_m;
    b.lim[2] = limit && limit < R.cap_l ? limit : R.cap_l;
  }
  __syncthreads();
}

// Online filter: every lane of the wavefront calls (convergent).  Lanes with
// `valid` append vertex v (degree deg) to its bin in this workgroup's region;
// a large vertex adds one item per chunk of arcs.
SX_DEV void bins_append(bool valid, int v, int deg, const Regions &R, unsigned bid, const Params &P,
                        int chunk, LdsBins &b, WaveStats &st) {
  const uint64_t any = ballot(valid);
  if (any == 0) return;
  const int lane = lane_id();
  const int bn = valid ? bin_of(deg, P) : -1;
  if (valid) { st.nf += 1; st.mf += (unsigned long long)deg; }
#pragma unroll
  for (int bin = 0; bin < 2; ++bin) {
    const uint64_t mk = ballot(bn == bin);
    if (mk == 0) continue;
    const int leader = __ffsll((long long)mk) - 1;
    unsigned base = 0;
    if (lane == leader) base = atomicAdd(&b.cnt[bin], (unsigned)__popcll(mk));
    base = __shfl(base, leader);
    if (bn == bin) {
      const unsigned pos = base + lane_prefix(mk);
      if (pos < b.lim[bin]) {
        if (bin == 0) R.s[(size_t)bid * R.cap_s + pos] = v;
        else R.m[(size_t)bid * R.cap_m + pos] = v;
      } else {
        b.ovf = 1;
      }
    }
  }
  const uint64_t ml = ballot(bn == BIN_LARGE);
  if (ml) {
    const int k = (bn == BIN_LARGE) ? chunks_of(deg, chunk) : 0;
    const int incl = wave_incl_scan(k);
    const int total = __shfl(incl, 63);
    unsigned base = 0;
    if (lane == 63) base = atomicAdd(&b.cnt[BIN_LARGE], (unsigned)total);
    base = __shfl(base, 63);
    const unsigned pos = base + (unsigned)(incl - k);
    for (int c = 0; c < k; ++c) {
      if (pos + c < b.lim[BIN_LARGE])
        R.l[(size_t)bid * R.cap_l + pos + c] = ((unsigned long long)c << 32) | (unsigned)v;
      else
        b.ovf = 1;
    }
  }
}

// Publish workgroup `bid`'s record in slot `rs` (one thread).
SX_DEV void rec_write(RecSlot *rs, unsigned bid, const unsigned cnt[NBINS], unsigned nf,
                      unsigned long long mf, bool ovf) {
  for (int i = 0; i < NBINS; ++i) rs->cnt[i][bid] = cnt[i];
  rs->nf[bid] = (nf & ~kRecOvf) | (ovf ? kRecOvf : 0u);
  rs->mf[bid] = mf;
}

// Online filter for entries that are already binned (re-emitting a list):
// lanes with `valid` append `item` (a vertex id, or a large item chunk << 32
// | vertex) to bin `bin`; entries with `vertex` count as one vertex of `deg`
// arcs in the statistics (small and medium entries, first chunks).
SX_DEV void bins_put(bool valid, int bin, unsigned long long item, bool vertex, int deg,
                     const Regions &R, unsigned bid, LdsBins &b, WaveStats &st) {
  if (ballot(valid) == 0) return;
  const int lane = lane_id();
  if (valid && vertex) { st.nf += 1; st.mf += (unsigned long long)deg; }
#pragma unroll
  for (int bn = 0; bn < NBINS; ++bn) {
    const uint64_t mk = ballot(valid && bin == bn);
    if (mk == 0) continue;
    const int leader = __ffsll((long long)mk) - 1;
    unsigned base = 0;
    if (lane == leader) base = atomicAdd(&b.cnt[bn], (unsigned)__popcll(mk));
    base = __shfl(base, leader);
    if (valid && bin == bn) {
      const unsigned pos = base + lane_prefix(mk);
      if (pos < b.lim[bn]) {
        if (bn == BIN_SMALL) R.s[(size_t)bid * R.cap_s + pos] = (int)item;
        else if (bn == BIN_MED) R.m[(size_t)bid * R.cap_m + pos] = (int)item;
        else R.l[(size_t)bid * R.cap_l + pos] = item;
      } else {
        b.ovf = 1;
      }
    }
  }
}

// End of a producing phase (all threads): publish this workgroup's record.
// Counts past the limit mark overflow; entries beyond it were not written.
SX_DEV void bins_end(LdsBins &b, WaveStats &st, RecSlot *rs, unsigned bid) {
  const int nf = wave_sum_i((int)st.nf);
  const long long mf = wave_sum_ll((long long)st.mf);
  if (lane_id() == 0) {
    b.nf[wave_in_wg()] = (unsigned)nf;
    b.mf[wave_in_wg()] = (unsigned long long)mf;
  }
  st.nf = 0;
  st.mf = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned tnf = 0;
    unsigned long long tmf = 0;
    for (int w = 0; w < kWaves; ++w) { tnf += b.nf[w]; tmf += b.mf[w]; }
    bool ovf = b.ovf != 0;
    unsigned c[NBINS];
    for (int i = 0; i < NBINS; ++i) {
      c[i] = b.cnt[i] < b.lim[i] ? b.cnt[i] : b.lim[i];
      if (b.cnt[i] > b.lim[i]) ovf = true;
    }
    rec_write(rs, bid, c, tnf, tmf, ovf);
  }
  __syncthreads();
}

// ---------------------------------------------------------- consuming ---
struct LdsView {
  unsigned pre[NBINS][kMaxGrid + 1];
  unsigned tmp[kWaves * 4];
  long long wnf[kWaves], wmf[kWaves];
};

struct Totals {
  unsigned cnt[NBINS];          // items per bin (within the regions)
  unsigned nf;                  // vertices appended (all, also past capacity)
  unsigned long long mf;
  unsigned ovf;                 // some region overflowed
};

// Prefix of the records of one slot (all threads); the totals are identical
// in every workgroup.  Thread t owns records 2t and 2t+1 and reads them with
// one 8-byte load per field.
SX_DEV uint2 rec_pair(const unsigned *a, unsigned w0, unsigned G) {
  if (w0 + 1 < G) return *(const uint2 *)(a + w0);
  return make_uint2(w0 < G ? a[w0] : 0u, 0u);
}

SX_DEV Totals view_build(const RecSlot *rs, unsigned G, const Regions &R, LdsView &V,
                         long long *red /* kWaves */) {
  (void)red;
  const unsigned t = threadIdx.x;
  const unsigned w0 = 2 * t;
  const unsigned caps[NBINS] = {R.cap_s, R.cap_m, R.cap_l};
  unsigned ovf = 0;
  unsigned c0[NBINS], c1[NBINS];
  int incl[NBINS];
#pragma unroll
  for (int b = 0; b < NBINS; ++b) {
    const uint2 p = rec_pair(rs->cnt[b], w0, G);
    c0[b] = p.x < caps[b] ? p.x : caps[b];
    c1[b] = p.y < caps[b] ? p.y : caps[b];
    ovf |= (p.x > caps[b] || p.y > caps[b]) ? 1u : 0u;
  }
  const uint2 nfp = rec_pair(rs->nf, w0, G);
  unsigned long long mf = 0;
  if (w0 < G) mf += rs->mf[w0];
  if (w0 + 1 < G) mf += rs->mf[w0 + 1];
  ovf |= ((nfp.x | nfp.y) & kRecOvf) ? 1u : 0u;
  // one exchange through LDS for the three bin scans and the totals
#pragma unroll
  for (int b = 0; b < NBINS; ++b) incl[b] = wave_incl_scan((int)(c0[b] + c1[b]));
  const long long nf = wave_sum_ll((long long)(nfp.x & ~kRecOvf) + (long long)(nfp.y & ~kRecOvf));
  const long long mfw = wave_sum_ll((long long)mf);
  const unsigned ovw = ballot(ovf != 0) ? 1u : 0u;
  const int wv = wave_in_wg();
  if (lane_id() == 63) {
#pragma unroll
    for (int b = 0; b < NBINS; ++b) V.tmp[wv * 4 + b] = (unsigned)incl[b];
    V.tmp[wv * 4 + 3] = ovw;
    V.wnf[wv] = nf;
    V.wmf[wv] = mfw;
  }
  __syncthreads();
  Totals T;
  T.nf = 0;
  T.mf = 0;
  T.ovf = 0;
#pragma unroll
  for (int b = 0; b < NBINS; ++b) T.cnt[b] = 0;
  unsigned base[NBINS] = {0, 0, 0};
  for (int w = 0; w < kWaves; ++w) {
#pragma unroll
    for (int b = 0; b < NBINS; ++b) {
      const unsigned x = V.tmp[w * 4 + b];
      if (w < wv) base[b] += x;
      T.cnt[b] += x;
    }
    T.ovf |= V.tmp[w * 4 + 3];
    T.nf += (unsigned)V.wnf[w];
    T.mf += (unsigned long long)V.wmf[w];
  }
#pragma unroll
  for (int b = 0; b < NBINS; ++b) {
    const unsigned ex = base[b] + (unsigned)(incl[b] - (int)(c0[b] + c1[b]));
    if (w0 < G) V.pre[b][w0] = ex;
    if (w0 + 1 < G) V.pre[b][w0 + 1] = ex + c0[b];
    if (t == 0) V.pre[b][G] = T.cnt[b];
  }
  __syncthreads();
  return T;
}

// Totals of one record slot without the prefix (all threads).
SX_DEV Totals rec_totals(const RecSlot *rs, unsigned G, long long *red /* kWaves */) {
  long long c[NBINS] = {0, 0, 0}, nf = 0, mf = 0, ovf = 0;
  for (unsigned w = threadIdx.x; w < G; w += kBlock) {
    for (int b = 0; b < NBINS; ++b) c[b] += rs->cnt[b][w];
    const unsigned x = rs->nf[w];
    nf += x & ~kRecOvf;
    ovf |= (x & kRecOvf) ? 1 : 0;
    mf += (long long)rs->mf[w];
  }
  Totals T;
  for (int b = 0; b < NBINS; ++b) T.cnt[b] = (unsigned)wg_sum_ll<kBlock>(c[b], red);
  T.nf = (unsigned)wg_sum_ll<kBlock>(nf, red);
  T.mf = (unsigned long long)wg_sum_ll<kBlock>(mf, red);
  T.ovf = wg_sum_ll<kBlock>(ovf, red) ? 1u : 0u;
  return T;
}

// largest r < G with pre[r] <= i (for i < pre[G])
SX_DEV unsigned view_find(const unsigned *pre, unsigned G, unsigned i) {
  unsigned lo = 0, hi = G - 1;
  while (lo < hi) {
    const unsigned mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Item i of each bin through a view (lambdas for the visitors)
struct ViewRef {
  const LdsView *V;
  Regions R;
  unsigned G;
  SX_DEV int small(unsigned i) const {
    const unsigned r = view_find(V->pre[BIN_SMALL], G, i);
    return R.s[(size_t)r * R.cap_s + (i - V->pre[BIN_SMALL][r])];
  }
  SX_DEV int med(unsigned i) const {
    const unsigned r = view_find(V->pre[BIN_MED], G, i);
    return R.m[(size_t)r * R.cap_m + (i - V->pre[BIN_MED][r])];
  }
  SX_DEV unsigned long long large(unsigned i) const {
    const unsigned r = view_find(V->pre[BIN_LARGE], G, i);
    return R.l[(size_t)r * R.cap_l + (i - V->pre[BIN_LARGE][r])];
  }
};

// ------------------------------------------------------- ballot filter ---
// Workgroup `bid` scans positions [lo, hi) (lo a multiple of 64); wavefront w
// takes a contiguous sub-range, so the output order is the position order.
// probe(pos, valid) is called convergently by whole wavefronts and returns
// whether the entry at `pos` is active (false where !valid); vertex_of(pos)
// and degree(v) give its vertex and degree.  The ballot words go to `bits`
// (one 64-bit word per 64 positions per bin), are counted, and after a
// workgroup barrier re-read and written into this workgroup's regions.  One
// pass over the metadata and no grid-wide step: the range is contiguous, so
// the concatenation of the regions in workgroup order is sorted.
struct LdsBallot {
  unsigned wcnt[kWaves][NBINS];
  unsigned wnf[kWaves];
  unsigned wovf[kWaves];
  unsigned long long wmf[kWaves];
};

template <class Probe, class Deg, class VertexOf>
SX_DEV void ballot_fill_range(long long lo, long long hi, unsigned bid, Probe probe, Deg degree,
                              VertexOf vertex_of, const Params &P, int chunk,
                              unsigned long long *const bits[NBINS], const Regions &R,
                              RecSlot *rec_slot, LdsBallot &lb) {
  const long long len = hi > lo ? hi - lo : 0;
  const long long per_wave = ((len + kWaves - 1) / kWaves + 63) / 64 * 64;
  const int lane = lane_id(), wv = wave_in_wg();
  const long long start = lo + (long long)wv * per_wave;
  const long long end = start + per_wave < hi ? start + per_wave : hi;
  unsigned c[NBINS] = {0, 0, 0};
  unsigned long long mf = 0;
  unsigned nfv = 0;
  for (long long s = start; s < end; s += 64) {
    const long long i = s + lane;
    const bool p = probe(i, i < end);
    const int d = p ? degree(vertex_of(i)) : 0;
    const int b = p ? bin_of(d, P) : -1;
    const long long word = s >> 6;
#pragma unroll
    for (int bin = 0; bin < NBINS; ++bin) {
      const uint64_t mk = ballot(b == bin);
      if (lane == 0) bits[bin][word] = mk;
      if (bin < BIN_LARGE) c[bin] += (unsigned)__popcll(mk);
    }
    const int k = (b == BIN_LARGE) ? chunks_of(d, chunk) : 0;
    c[BIN_LARGE] += (unsigned)wave_sum_i(k);
    nfv += (unsigned)__popcll(ballot(p));
    mf += (unsigned long long)wave_sum_ll(p ? d : 0);
  }
  if (lane == 0) {
    for (int bin = 0; bin < NBINS; ++bin) lb.wcnt[wv][bin] = c[bin];
    lb.wnf[wv] = nfv;
    lb.wmf[wv] = mf;
  }
  __syncthreads();
  unsigned pos[NBINS] = {0, 0, 0}, tot[NBINS] = {0, 0, 0};
  for (int w = 0; w < kWaves; ++w)
    for (int bin = 0; bin < NBINS; ++bin) {
      if (w < wv) pos[bin] += lb.wcnt[w][bin];
      tot[bin] += lb.wcnt[w][bin];
    }
  const unsigned caps[NBINS] = {R.cap_s, R.cap_m, R.cap_l};
  bool ovf = false;
  for (long long s = start; s < end; s += 64) {
    const long long word = s >> 6;
    const uint64_t ms = bits[BIN_SMALL][word];
    const uint64_t mm = bits[BIN_MED][word];
    const uint64_t ml = bits[BIN_LARGE][word];
    const bool in_any = ((ms | mm | ml) >> lane) & 1ull;
    const int v = in_any ? vertex_of(s + lane) : 0;
    if ((ms >> lane) & 1ull) {
      const unsigned q = pos[BIN_SMALL] + lane_prefix(ms);
      if (q < caps[BIN_SMALL]) R.s[(size_t)bid * R.cap_s + q] = v;
      else ovf = true;
    }
    if ((mm >> lane) & 1ull) {
      const unsigned q = pos[BIN_MED] + lane_prefix(mm);
      if (q < caps[BIN_MED]) R.m[(size_t)bid * R.cap_m + q] = v;
      else ovf = true;
    }
    pos[BIN_SMALL] += (unsigned)__popcll(ms);
    pos[BIN_MED] += (unsigned)__popcll(mm);
    if (ml) {
      const int k = ((ml >> lane) & 1ull) ? chunks_of(degree(v), chunk) : 0;
      const int incl = wave_incl_scan(k);
      const unsigned q = pos[BIN_LARGE] + (unsigned)(incl - k);
      for (int cc = 0; cc < k; ++cc) {
        if (q + cc < caps[BIN_LARGE])
          R.l[(size_t)bid * R.cap_l + q + cc] = ((unsigned long long)cc << 32) | (unsigned)v;
        else
          ovf = true;
      }
      pos[BIN_LARGE] += (unsigned)__shfl(incl, 63);
    }
  }
  const bool any_ovf = ballot(ovf) != 0;
  if (lane == 0) lb.wovf[wv] = any_ovf ? 1u : 0u;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tmf = 0;
    unsigned tnf = 0, o = 0, c[NBINS];
    for (int w = 0; w < kWaves; ++w) { tmf += lb.wmf[w]; tnf += lb.wnf[w]; o |= lb.wovf[w]; }
    for (int bin = 0; bin < NBINS; ++bin) {
      c[bin] = tot[bin] < caps[bin] ? tot[bin] : caps[bin];
      if (tot[bin] > caps[bin]) o = 1;
    }
    rec_write(rec_slot, bid, c, tnf, tmf, o != 0);
  }
  __syncthreads();
}

// Positions [0, count) split over the grid in contiguous ranges (multiples
// of 64 * kWaves); pred(i) is the active test of position i, vertex_of(i)
// its vertex.
template <class Pred, class Deg, class VertexOf>
SX_DEV void ballot_fill(const VGrid &vg, int count, Pred pred, Deg degree, VertexOf vertex_of,
                        const Params &P, int chunk, unsigned long long *const bits[NBINS],
                        const Regions &R, RecSlot *rec_slot, LdsBallot &lb) {
  const long long unit = 64 * kWaves;
  const long long per_wg = (((long long)count + vg.nb - 1) / vg.nb + unit - 1) / unit * unit;
  const long long lo = (long long)vg.bid * per_wg;
  const long long hi = lo + per_wg < count ? lo + per_wg : count;
  auto probe = [&](long long i, bool ok) { return ok && pred((int)i); };
  auto vof = [&](long long i) { return vertex_of((int)i); };
  ballot_fill_range(lo, hi, vg.bid, probe, degree, vof, P, chunk, bits, R, rec_slot, lb);
}

// ------------------------------------------------- worklist traversal ---
// Visit every arc of every worklist entry.  `op(v, u, arc, ok)` receives
// kIlp arcs per lane (arrays of kIlp: source, target, arc index, lane
// valid), is called convergently by whole wavefronts, and performs Compute +
// Combine for those arcs and the online appends itself.  Handing a lane
// several independent arcs at once lets an op issue all their loads, then
// all their atomics, before waiting for any: the chain target id -> target
// state -> atomic costs its latency once per kIlp arcs instead of once per
// arc.  Entries outside [0, n) are skipped (a defence: lists only ever hold
// vertex ids).
constexpr int kIlp = 4;

// Small bin: a wavefront takes up to 64 vertices, stages their row starts
// and a prefix sum of their degrees in LDS, then walks the concatenated arcs
// 64 * kIlp at a time, so lanes stay busy however degrees vary.
template <class Acc, class Op>
SX_DEV void visit_small(int n, Acc item, unsigned cnt, const int *off, const int *idx, Op &op,
                        unsigned gw, unsigned nwaves, int *lds /* 3*64 per wave */) {
  // Group size: enough vertices per wavefront task that every wavefront of
  // the grid gets about one task, at most 64.  A fixed 64 would leave most
  // wavefronts idle on lists of tens of thousands of vertices while a few
  // walk 64 rows each, round after round.
  const unsigned per = (cnt + nwaves - 1) / (nwaves ? nwaves : 1);
  const int gs = per < 1 ? 1 : (per > 64 ? 64 : (int)per);
  const int lane = lane_id();
  int *l_v = lds, *l_beg = lds + 64, *l_ex = lds + 128;
  for (unsigned c = gw; c * (unsigned)gs < cnt; c += nwaves) {
    const unsigned i = c * (unsigned)gs + lane;
    int v = -1, beg = 0, deg = 0;
    if (lane < gs && i < cnt) {
      const int x = item(i);
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
    for (int j = 0; j < total; j += 64 * kIlp) {
      int vv[kIlp], u[kIlp], arc[kIlp];
      bool ok[kIlp];
#pragma unroll
      for (int r = 0; r < kIlp; ++r) {
        const int e = j + r * 64 + lane;
        ok[r] = e < total;
        int owner = 0;
        if (ok[r]) {
          int lo = 0, hi = gs - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (l_ex[mid] <= e) lo = mid;
            else hi = mid - 1;
          }
          owner = lo;
        }
        arc[r] = ok[r] ? l_beg[owner] + (e - l_ex[owner]) : 0;
        vv[r] = ok[r] ? l_v[owner] : 0;
      }
#pragma unroll
      for (int r = 0; r < kIlp; ++r) u[r] = ok[r] ? idx[arc[r]] : 0;
      op(vv, u, arc, ok);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Medium bin: one wavefront per vertex, 64 * kIlp arcs per step.
template <class Acc, class Op>
SX_DEV void visit_med(int n, Acc item, unsigned cnt, const int *off, const int *idx, Op &op,
                      unsigned gw, unsigned nwaves) {
  const int lane = lane_id();
  for (unsigned i = gw; i < cnt; i += nwaves) {
    const int v = item(i);
    if ((unsigned)v >= (unsigned)n) continue;
    const int beg = off[v], end = off[v + 1];
    for (int a = beg; a < end; a += 64 * kIlp) {
      int vv[kIlp], u[kIlp], arc[kIlp];
      bool ok[kIlp];
#pragma unroll
      for (int r = 0; r < kIlp; ++r) {
        arc[r] = a + r * 64 + lane;
        ok[r] = arc[r] < end;
        vv[r] = v;
        u[r] = ok[r] ? idx[arc[r]] : 0;
      }
      op(vv, u, arc, ok);
    }
  }
}

// Large bin: one workgroup per item (a chunk of `chunk` arcs of one vertex),
// kBlock * kIlp arcs per step.
template <class Acc, class Op>
SX_DEV void visit_large(const VGrid &vg, int n, Acc item, unsigned cnt, const int *off,
                        const int *idx, int chunk, Op &op) {
  for (unsigned i = vg.bid; i < cnt; i += vg.nb) {
    const unsigned long long it = item(i);
    const int v = (int)(it & 0xffffffffu);
    if ((unsigned)v >= (unsigned)n) continue;
    const int c = (int)(it >> 32);
    const int vb = off[v], ve = off[v + 1];
    const long long b0 = (long long)vb + (long long)c * chunk;
    const int beg = (int)(b0 < ve ? b0 : ve);
    const int end = (int)((b0 + chunk) < ve ? (b0 + chunk) : ve);
    for (int a = beg; a < end; a += kBlock * kIlp) {
      int vv[kIlp], u[kIlp], arc[kIlp];
      bool ok[kIlp];
#pragma unroll
      for (int r = 0; r < kIlp; ++r) {
        arc[r] = a + r * kBlock + (int)threadIdx.x;
        ok[r] = arc[r] < end;
        vv[r] = v;
        u[r] = ok[r] ? idx[arc[r]] : 0;
      }
      op(vv, u, arc, ok);
    }
  }
}

// Statistics: arcs inspected and worklist entries processed, added by each
// workgroup into one of 64 lines (spread so that the atomics do not
// serialise on one address).
SX_DEV void add_stats(Ctrl *C, unsigned bid, long long edges_lane, unsigned long long entries,
                      long long *red) {
  const long long e = wg_sum_ll<kBlock>(edges_lane, red);
  if (threadIdx.x == 0) {
    Line &l = C->statw[bid % kStatLines];
    if (e) atomic_add_u64((unsigned long long *)&l.v[0], (unsigned long long)e);
    if (entries) atomic_add_u64((unsigned long long *)&l.v[2], entries);
  }
}

}  // namespace sx
