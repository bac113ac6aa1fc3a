// Types shared by the host driver and the HIP kernels of the ACC engine.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace sx {

constexpr int kBlock = 512;              // threads per workgroup (8 wavefronts)
constexpr int kChunk = 4 * kBlock;       // arcs per large-bin item (traversals)
constexpr int kTailMax = 36864;          // k-core tail: vertices whose degrees
                                         // one workgroup's LDS holds
constexpr int kTailThreads = 1024;       // and the workgroup's threads
constexpr int kTailDefault = 16384;      // the tail's default hand-over: this
constexpr unsigned long long kTailDefaultArcs = 1ull << 22;  // many vertices
                                         // and arcs at most
constexpr int kWaves = kBlock / 64;
constexpr int kMaxGrid = 1024;           // upper bound on workgroups per grid
// watchdog of the software global barrier: how long one wait may last, in
// ticks of the constant-rate wall clock (s_memrealtime, 100 MHz on gfx950)
constexpr unsigned long long kWatchdogTicks = 200000000ull;   // 2 s
constexpr int kStatLines = 64;           // statistics spread over 64 lines

// SX_ERR_CAPACITY: a list built by a ballot scan did not fit its regions
// (the host sizes them so that this cannot happen)
// SX_ERR_INPUT: an input value outside its domain (a belief-propagation
// prior not in (0, 1))
// SX_ERR_TAIL: the k-core tail's compacted rows disagree with the degrees
enum : unsigned { SX_ERR_NONE = 0, SX_ERR_DEADLOCK = 1, SX_ERR_OVERFLOW = 2, SX_ERR_CAPACITY = 3,
                  SX_ERR_INPUT = 4, SX_ERR_TAIL = 5 };

// kernel exit reasons written to Ctrl::state
enum : int { EXIT_NONE = 0, EXIT_DONE = 1, EXIT_SWITCH = 2, EXIT_ERROR = 3, EXIT_LIMIT = 4 };

// worklist bins (Section 4 step I: small / medium / large lists)
enum : int { BIN_SMALL = 0, BIN_MED = 1, BIN_LARGE = 2, NBINS = 3 };

// record slots: 0..2 rotate with the iteration (the lists a compute phase
// appends for the next iteration); 3 holds lists built by a ballot scan;
// 4 and 5 the k-core alive lists (by scan parity)
enum : int { NSLOTS = 6, SLOT_SCAN = 3, SLOT_ALIVE = 4 };

struct alignas(128) Line {
  unsigned v[32];
};

// What the workgroups appended to their bins in one phase (their "thread
// bins" in the paper's terms, Section 3.3), one slot per list, stored field
// by field so that a consumer reads only the counts it needs: items per bin,
// vertices (bit 31: a bin overflowed its capacity) and their arcs.
constexpr unsigned kRecOvf = 0x80000000u;
struct RecSlot {
  unsigned cnt[NBINS][kMaxGrid];
  unsigned nf[kMaxGrid];
  unsigned long long mf[kMaxGrid];
};

// Control block: one per graph workspace, in device memory.
struct Ctrl {
  Line bar_gen;                 // barrier generation
  Line error;                   // SX_ERR_*
  Line state;                   // run state of the fused kernels
  Line stats;                   // u32 [4] ballot scans, [5] pull iterations,
                                // [6] iterations; u64 [8] k-core scan entries
  Line aux;                     // algorithm scratch
  Line pol;                     // learned policy: [0] network evaluations,
                                // [1..8] features and [9..12] outputs of the
                                // last evaluation (float bits)
  Line seq[2];                  // sequenced mode: run state handed from launch
                                // L (reads seq[L&1]) to launch L+1
  Line statw[kStatLines];       // u64 [0] arcs inspected, [2] worklist entries
                                // processed, [4] wall-clock ticks workgroups
                                // spent waiting at global barriers; workgroup
                                // b adds into line b % 64
  Line flags[kMaxGrid];         // per workgroup: [0] barrier arrival word,
                                // [4,5] wall clock at the end of its last
                                // launch (sequenced arrangement)
};

// Device-resident graph (CSR, optional CSC) and engine workspace pointers.
struct DevGraph {
  int n;
  long long m;
  const int *off;
  const int *idx;
  const unsigned *w;
  const int *in_off;            // == off for undirected graphs
  const int *in_idx;
  const unsigned *in_w;
  int directed;
};

// Worklists are kept in per-workgroup regions: workgroup b owns entries
// [b * cap, (b+1) * cap) of each bin array, with cap = total / (workgroups).
struct Work {
  int *reg_s[2], *reg_m[2];        // [parity] small / medium bin regions
  unsigned long long *reg_l[2];    // [parity] large items: chunk << 32 | vertex
  unsigned tot_s, tot_m, tot_l;    // entries per bin array (all regions)
  RecSlot *rec;                    // [NSLOTS]
  unsigned long long *bits[NBINS]; // ballot words, one per 64 scan positions
  unsigned long long *fbits;       // frontier bitmap (pull)
  int *stamp;                      // per-vertex int: SSSP iteration stamps
  int *deg;                        // k-core current degree
  int *al_s[2], *al_m[2];          // k-core alive lists, binned like the
  unsigned long long *al_l[2];     // worklists (same capacities), by parity
  unsigned *alive_min;             // [2][kMaxGrid] minimum survivor degree
  float *contrib[2];               // PageRank contributions (double buffered)
  float *dang;                     // PageRank dangling partials [2][kMaxGrid][2]
  float *prd;                      // PageRank to convergence: pending change per vertex
  float *prp;                      // and per-workgroup partials [2][kMaxGrid][8]
  float *bph;                      // belief propagation: prior field atanh(2p - 1)
  float2 *bpq[2];                  // and (2 b - 1, degree) per vertex, double buffered
  Ctrl *ctrl;
};

// Uniform per-run parameters.
struct Params {
  int t1;                       // degree < t1 -> small bin (lane)
  int t2;                       // degree >= t2 -> large bin (workgroup chunks)
  int chunk;                    // arcs per large-bin item
  unsigned online_cap;          // online filter: entries per workgroup and bin
                                // before overflow (0: the whole region)
  int filter;                   // 0 JIT, 1 online, 2 ballot
  int direction;                // 0 auto, 1 push, 2 pull
  float alpha, beta;            // direction heuristic (vote)
  float alpha_w, beta_w;        // direction heuristic (aggregation)
  int max_iters;
  float pr_d;
  int pr_iters;
  int learned;                  // 1: the policy MLP decides (sx_policy.hpp)
  int bins_fixed;               // 1: the caller fixed t1 / t2
  unsigned delta;               // SSSP bucket width (0: no buckets)
  int delta_after;              // iterations run before the buckets engage
  int kfix;                     // k-core: 0 full decomposition, k > 0
                                // membership in the k-core only
  int ktail;                    // k-core: hand the rest of the decomposition
                                // to the one-workgroup tail once a level ends
                                // with at most this many vertices (0: never)
  unsigned long long ktail_arcs;  // and with their rows (arcs to deleted
                                  // vertices included) at most this long
  unsigned long long watchdog;  // barrier wait budget (wall-clock ticks)
};

struct TravArgs {
  DevGraph g;
  Work w;
  Params P;
  int *state_i;                 // BFS depth (int32) or SSSP dist (uint32) array
  int src;
  const float *mlp;             // policy parameters (device) when P.learned
  // WCC on a renumbered graph: old id -> new id; vertex inv[v] starts with
  // label v (its id in the caller's numbering), so that the minimum label of
  // a component is its smallest original id.  NULL: label = own id.
  const int *wcc_inv;
  // SSSP / WCC expansion record (see push_phase): [0, n) the value each
  // vertex's last small- or medium-bin expansion started from, then per
  // large-bin chunk the same, chunk c of vertex v at n + off[v] / kChunk +
  // c + v (unique; n + m / kChunk + 2 entries); ~0u: none.  NULL: no
  // record, every listed vertex expands.
  unsigned *xdist;
};

// Batched queries (see k_batch).
struct BatchQuery {
  DevGraph g;
  int *state;                   // the query's output array
  int algo;                     // 0 BFS, 1 SSSP
  int src;
  unsigned long long mu0;       // arcs not yet explored after the source
};
struct BatchStat {
  int iterations, pull_iters, ballot_iters, status, team, pad;
  unsigned long long edges, expansions;
};
struct BatchArgs {
  const BatchQuery *q;
  const int *order;             // processing order (largest first)
  int nq;
  const Work *work;             // [nteams] team workspaces (device)
  int nteams, team;             // team count and workgroups per team
  unsigned *queue_head;
  Params P;
  const float *mlp;
  BatchStat *stats;             // [nq]
};

struct KArgs {
  DevGraph g;
  Work w;
  Params P;
  int *core;                    // output core numbers, -1 while alive
};

struct PrArgs {
  DevGraph g;
  Work w;
  Params P;
  float *rank;                  // output
  float base_teleport;          // (1-d)/n
  float inv_n;                  // 1/n
  int iters;
  // run to convergence (pull, then the delta-accumulative push tail):
  int conv;                     // 1: iterate until stable instead of `iters`
  int max_pull;                 // pull iterations after which the tail starts anyway
  float thr;                    // a pending change above this is pushed
  float stop_change;            // pull converged: one step changed at most this (L1)
};

struct BpArgs {
  DevGraph g;
  Work w;
  Params P;
  float *belief;                // in: prior P(x_v = 1); out: belief after iters
  float kappa;                  // coupling scale of the pairwise potentials
  int iters;
};

// Direction and filter choice for the next iteration (Sections 4 and 5).
// Evaluated identically by every workgroup after a barrier in the fused
// kernels, and by the host between launches in one-phase mode.
struct Decision {
  bool done, to_pull, to_push, ballot;
};
struct DecideIn {
  unsigned nf;                  // next frontier vertices
  unsigned long long mf;        // and their arcs
  unsigned ovf;                 // online filter overflowed
  int it;
  bool pulling, vote;
  int n;
  long long m;
};

// BFS (vote): push -> pull when the frontier's arcs exceed the unexplored
// arcs / alpha, pull -> push when the frontier falls below n / beta (the
// direction-optimising rule of Beamer et al., which the paper's push/pull
// switching follows for BFS: push first and last, pull in between).  SSSP
// (aggregation): pull while the frontier's arcs exceed m / alpha_w, back to
// push below m / beta_w.  A pull iteration of SSSP reads every in-arc (no
// early exit under a minimum), so it would pay only when the frontier's arcs
// exceed m by the ratio of the two arc rates.  With four arcs per lane in
// flight, pushing is faster at every iteration measured on MI355X (R-MAT
// s22: 3.09 ms pushing throughout against 3.60 ms with the one pull
// iteration that alpha_w = 1.25 chose), so alpha_w = 0.5: a frontier's arcs
// never exceed 2m, and pull stays available to the policy and the caller.  JIT filter choice: the online filter's lists
// are used unless a region overflowed.
__host__ __device__ inline Decision decide_core(const DecideIn &in, const Params &P,
                                                unsigned long long &mu) {
  Decision d{false, false, false, false};
  if (in.nf == 0 || in.it + 1 >= P.max_iters) { d.done = true; return d; }
  if (in.vote) mu = mu > in.mf ? mu - in.mf : 0ull;
  const int dir = P.direction;
  if (!in.pulling) {
    bool pull;
    if (dir == 1) pull = false;
    else if (dir == 2) pull = true;
    else if (in.vote) pull = (double)in.mf > (double)mu / P.alpha;
    else pull = (double)in.mf > (double)in.m / P.alpha_w;
    d.to_pull = pull;
    d.ballot = !pull && (P.filter == 2 || (P.filter == 0 && in.ovf));
  } else {
    bool push;
    if (dir == 2) push = false;
    else if (dir == 1) push = true;
    else if (in.vote) push = (double)in.nf < (double)in.n / P.beta;
    else push = (double)in.mf < (double)in.m / P.beta_w;
    d.to_push = push;
  }
  return d;
}

}  // namespace sx
