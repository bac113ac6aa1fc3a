// Types shared by the host driver and the HIP kernels of the ACC engine.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace sx {

constexpr int kBlock = 512;              // threads per workgroup (8 wavefronts)
constexpr int kWaves = kBlock / 64;
constexpr int kMaxGrid = 2048;           // upper bound on persistent workgroups
constexpr unsigned kSpinLimit = 1u << 22; // watchdog: polls of ~128 cycles each

enum : unsigned { SX_ERR_NONE = 0, SX_ERR_DEADLOCK = 1, SX_ERR_OVERFLOW = 2 };

// kernel exit reasons written to Ctrl::state
enum : int { EXIT_NONE = 0, EXIT_DONE = 1, EXIT_SWITCH = 2, EXIT_ERROR = 3, EXIT_LIMIT = 4 };

// worklist bins (Section 4 step I: small / medium / large lists)
enum : int { BIN_SMALL = 0, BIN_MED = 1, BIN_LARGE = 2, NBINS = 3 };

struct alignas(128) Line {
  unsigned v[32];
};

// Per-iteration counters, triple buffered by iteration (it % 3): slot it is
// read during iteration it, slot it+1 is appended to, slot it+2 is reset.
struct alignas(128) Counters {
  unsigned cnt[NBINS];          // entries per bin (large: chunk items)
  unsigned nf;                  // vertices in the frontier
  unsigned long long mf;        // sum of their degrees
  unsigned overflow;            // online filter overflowed
  unsigned pad[25];
};

// Control block: one per graph workspace, in device memory.
struct Ctrl {
  Line bar_gen;                 // barrier generation
  Line error;                   // SX_ERR_*
  Line state;                   // [0] exit reason [1] iteration [2] level/k
                                // [3] direction [4] launches-in-kernel
  Line stats;                   // u64 [0] edges, [1] expansions; u32 [4]
                                // ballot iters, [5] pull iters, [6] iterations
  Counters q[3];
  Line aux;                     // algorithm scratch (k-core: min alive degree)
  Line seq[2];                  // sequenced mode: run state handed from launch
                                // L (reads seq[L&1]) to launch L+1
  Line flags[kMaxGrid];         // barrier arrival words, one line per workgroup
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

// Per-workgroup ballot-filter totals, written in pass 1, read in pass 2.
struct WgCount {
  unsigned cnt[NBINS];
  unsigned nf;
  unsigned long long mf;
};

struct Work {
  int *q[2][2];                 // [parity][small, med] vertex queues
  unsigned long long *ql[2];    // [parity] large items: chunk << 32 | vertex
  unsigned long long *bits[NBINS]; // ballot words per bin, n/64 each
  unsigned long long *fbits;    // frontier bitmap (pull)
  unsigned *wavecnt;            // per-wavefront ballot counts [kMaxGrid*kWaves][NBINS]
  WgCount *wgc;                 // per-workgroup ballot totals [kMaxGrid]
  int *stamp;                   // per-vertex int: SSSP/k-core iteration stamps
  int *deg;                     // k-core current degree
  float *contrib[2];            // PageRank contributions (double buffered)
  float *dang;                  // PageRank dangling partials [2][kMaxGrid][2]
  int *alive[2];                // k-core alive lists
  Ctrl *ctrl;
  unsigned qcap_small, qcap_med, qcap_large;
};

// Uniform per-run parameters.
struct Params {
  int t1;                       // degree < t1 -> small bin (lane)
  int t2;                       // degree >= t2 -> large bin (workgroup chunks)
  int chunk;                    // arcs per large-bin item
  unsigned online_cap;          // online filter capacity (entries, all bins)
  int filter;                   // 0 JIT, 1 online, 2 ballot
  int direction;                // 0 auto, 1 push, 2 pull
  float alpha, beta;            // direction heuristic
  int max_iters;
  float pr_d;
  int pr_iters;
  int learned;                  // 1: the policy MLP decides (sx_policy.hpp)
  int bins_fixed;               // 1: the caller fixed t1 / t2
};

struct TravArgs {
  DevGraph g;
  Work w;
  Params P;
  int *state_i;                 // BFS depth (int32) or SSSP dist (uint32) array
  int src;
  const float *mlp;             // policy parameters (device) when P.learned
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
// switching follows for BFS: push first and last, pull in between).  SSSP:
// pull while the frontier's arcs exceed m / alpha.  JIT filter choice: the
// online filter's lists are used unless a bin overflowed.
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
    else pull = (double)in.mf > (double)in.m / P.alpha;
    d.to_pull = pull;
    d.ballot = !pull && (P.filter == 2 || (P.filter == 0 && in.ovf));
  } else {
    bool push;
    if (dir == 2) push = false;
    else if (dir == 1) push = true;
    else if (in.vote) push = (double)in.nf < (double)in.n / P.beta;
    else push = (double)in.mf < (double)in.m / P.beta;
    d.to_push = push;
  }
  return d;
}

}  // namespace sx
