// Host-side entry points of the HIP kernels (launch helpers).
#pragma once

#include <functional>

#include "sx_types.hpp"

namespace sx {

// traversal kernels; trav_launch's `it` is the iteration (TK_SEQ: the launch
// number) and `arg` whether the push lists come from a ballot scan
// (TK_PUSH_STEP).  TK_FUSED / TK_FUSED_PULL: the push / pull persistent
// kernels of selective fusion; TK_FUSED_ALL: both directions in one.
enum TravKernel { TK_FUSED, TK_PUSH_STEP, TK_BALLOT, TK_PULL_SCAN, TK_PULL_STEP, TK_SEQ, TK_SEQ_WIDE,
                  TK_FUSED_ALL, TK_FUSED_PULL, TK_COUNT };
// traversal programs
enum TravAlgo { ALG_BFS = 0, ALG_SSSP = 1, ALG_WCC = 2 };

const void *trav_kernel(int kind, int algo);
hipError_t trav_launch(int kind, int algo, const TravArgs &a, int it, int arg, int grid,
                       hipStream_t s);
// pull_first: the run's first iteration pulls (read by the persistent
// kernels); sequenced: also write the first state of a sequenced run
hipError_t trav_init(const TravArgs &a, int algo, unsigned long long mu0, int run_grid,
                     hipStream_t s, bool pull_first = false, bool sequenced = false);
hipError_t batch_launch(const BatchArgs &b, int grid, hipStream_t s);
hipError_t weight_sum(const unsigned *w, long long m, unsigned long long *out, hipStream_t s);
// phases of the sequenced mode (Ctrl::seq[..].v[0])
enum : unsigned { SEQ_DONE = 6, SEQ_ERROR = 7, SEQ_LIMIT = 8 };
const void *batch_kernel();

hipError_t kcore_launch(const KArgs &a, int grid, hipStream_t s, bool init);
const void *kcore_kernel();
hipError_t kcore_seq_launch(const KArgs &a, unsigned L, int grid, hipStream_t s, bool start);
// core[v] = 1 where v survived (core[v] == -1, fixed-k membership), else 0
hipError_t kcore_membership(int *core, int n, hipStream_t s);
const void *kcore_seq_kernel();
// the one-workgroup tail of a decomposition the sequenced loop handed over
// (state KP_TAIL; Ctrl::aux[KT_K] the level to go on with, aux[KT_N] zero)
enum : unsigned { KP_TAIL = 9 };
enum { KT_K = 24, KT_N = 25 };
hipError_t kcore_tail_launch(const KArgs &a, int grid, hipStream_t s);
const void *kcore_tail_kernel();

hipError_t pagerank_launch(const PrArgs &a, int grid, hipStream_t s);
// conv: the pull kernel of the run to convergence (launched after k_pr_init
// by pagerank_launch); its push tail is a kernel of its own
const void *pagerank_kernel(bool conv = false);
hipError_t pagerank_push_launch(const PrArgs &a, int grid, hipStream_t s);
const void *pagerank_push_kernel();

hipError_t bp_launch(const BpArgs &a, int grid, hipStream_t s);
const void *bp_kernel();

// Degree-ordered renumbering (graph loading option).  `own` allocates
// device memory that the graph keeps, `tmp` memory freed after the build.
// out: the renumbered graph; *d_inv / h_inv[n]: old id -> new id.
using RkAlloc = std::function<hipError_t(void **, size_t)>;
hipError_t reorder_build(const DevGraph &g, const RkAlloc &own, const RkAlloc &tmp, hipStream_t s,
                         DevGraph &out, int **d_inv, int *h_inv);
// out[v] = in[inv[v]] for 4-byte elements
hipError_t reorder_unpermute(const void *in, const int *inv, void *out, int n, hipStream_t s);
// out[inv[v]] = in[v] for 4-byte elements
hipError_t reorder_permute(const void *in, const int *inv, void *out, int n, hipStream_t s);

hipError_t mlp_forward(const float *P, const float *X, int n, float *Y, float *H, hipStream_t s);
// the in-kernel inference (mlp_eval_wave, one wavefront per sample)
hipError_t mlp_forward_wave(const float *P, const float *X, int n, float *Y, hipStream_t s);
hipError_t mlp_loss_grad(const float *P, const float *X, const float *T, const float *M, int n,
                         float *Y, float *H, float *D, float *L, float *loss, float *G,
                         hipStream_t s);
hipError_t mlp_adam(float *P, const float *G, float *Mo, float *Vo, int step, float lr, float b1,
                    float b2, float eps, hipStream_t s);

}  // namespace sx
