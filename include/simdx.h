/*
 * simdx.h — C ABI of libsimdx.so, an MI355X (gfx950) implementation of the
 * Active-Compute-Combine (ACC) graph-processing method of
 * "SIMD-X: Programming and Processing of Graph Algorithms on GPUs"
 * (Liu and Huang, arXiv 1812.04070).
 *
 * The problem statement the calls follow (Section 2.1): a graph G = (V, E, w)
 * with vertex metadata ("the distance array") is computed on iteratively,
 * from a source until no vertex is updated.  An algorithm is the triple
 * Active / Compute / Combine of Section 3.2; this library ships five of them
 * (BFS, SSSP, k-core, PageRank of Section 6, and connected components, which
 * Section 3.2 names among the algorithms of its Combine step) and a program
 * selects one.
 *
 * Conventions shared by every call
 *  - Every call returns sx_status; SX_OK is 0, errors are negative.  Output
 *    parameters are written only on SX_OK.  Nothing aborts and no C++
 *    exception crosses the ABI.  sx_last_error() returns a thread-local text
 *    describing the last failure on the calling thread.
 *  - Opaque objects (sx_ctx, sx_graph, sx_program) are created and freed by
 *    the library.  Destroy graphs and programs before their context.
 *  - A hip_stream argument is a hipStream_t passed as void* (NULL = the null
 *    stream).  Calls that read results back synchronise that stream.
 *  - Integer layouts: vertex ids int32, CSR offsets int32 (so m < 2^31),
 *    edge weights uint32.  Vertex arrays have n elements.
 *  - One context serves one HIP device; calls on one context from several
 *    host threads at once are not supported.
 */
#ifndef SIMDX_H
#define SIMDX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SX_OK = 0,
  SX_EINVAL = -1,        /* bad argument: see sx_last_error()                  */
  SX_ENOMEM = -2,        /* device or host allocation failed                   */
  SX_EHIP = -3,          /* a HIP runtime call failed (text in sx_last_error) */
  SX_EUNSUPPORTED = -4,  /* combination not supported (e.g. device lacks it)   */
  SX_EDEADLOCK = -5,     /* grid-barrier watchdog fired: workgroups were not
                            all resident (Section 5, deadlock of the software
                            global barrier); engine state undefined, the graph
                            stays valid                                        */
  SX_EOVERFLOW = -6,     /* an SSSP distance reached 0xFFFFFFFF              */
  SX_ESTATE = -7         /* call made in the wrong state                       */
} sx_status;

typedef struct sx_ctx sx_ctx;
typedef struct sx_graph sx_graph;
typedef struct sx_program sx_program;

/* Create a context on HIP device `hip_device` (its ordinal).  Queries the
 * device (compute units, cooperative-launch support) once. */
sx_status sx_ctx_create(int hip_device, sx_ctx **out);
void sx_ctx_destroy(sx_ctx *ctx);
const char *sx_status_str(sx_status s);
const char *sx_last_error(void);

/* ------------------------------------------------------------- graphs --- */
/* Storage format (Section 6, "Storage Format"): CSR of out-neighbours; an
 * undirected graph stores both arcs of every edge (symmetric CSR) and needs
 * no in-neighbour structure; a directed graph adds the CSR of in-neighbours
 * (CSC) for pull processing. */
enum {
  SX_UNDIRECTED = 1u,    /* CSR is symmetric; in_* must be NULL               */
  SX_DEVICE_PTRS = 2u,   /* pointers are device memory: borrowed, not copied;
                            the caller keeps them alive until destroy          */
  SX_VALIDATE = 4u,      /* check offsets monotone and ids in range (host)    */
  SX_REORDER = 8u        /* renumber vertices by decreasing degree on load
                            (device arrays the graph owns, ~2x the CSR while
                            building); runs take and return original ids, the
                            mapping costs one gather per run; not for batches
                            or policy collection (SX_EUNSUPPORTED)            */
};

typedef struct {
  int32_t n;                 /* vertices                                       */
  int64_t m;                 /* arcs (entries of indices); must be < 2^31      */
  const int32_t *offsets;    /* [n+1], offsets[0] = 0, offsets[n] = m          */
  const int32_t *indices;    /* [m] out-neighbours, rows sorted ascending      */
  const uint32_t *weights;   /* [m] arc weights, > 0; NULL if unweighted       */
  const int32_t *in_offsets; /* [n+1] CSC; NULL for undirected graphs          */
  const int32_t *in_indices; /* [m] in-neighbours                              */
  const uint32_t *in_weights;/* [m] or NULL                                    */
  uint32_t flags;            /* SX_UNDIRECTED | SX_DEVICE_PTRS | SX_VALIDATE |
                                SX_REORDER                                     */
} sx_graph_desc;

/* Make the graph resident on the device (host arrays are copied; the caller
 * may free them on return) and allocate the per-graph engine workspace
 * (frontier queues, bitmaps, control block: about 40 bytes per vertex).
 * Errors: SX_EINVAL (n < 0, m out of range, missing arrays, a directed graph
 * without CSC, validation failure), SX_ENOMEM, SX_EHIP. */
sx_status sx_graph_load(sx_ctx *ctx, const sx_graph_desc *desc, void *hip_stream, sx_graph **out);
void sx_graph_destroy(sx_graph *g);
sx_status sx_graph_info(const sx_graph *g, int32_t *n, int64_t *m, int32_t *directed, int32_t *weighted);

/* ----------------------------------------------------------- programs --- */
/* The six ACC programs (Section 3.2 for the Active/Compute/Combine triple,
 * Section 6 for the algorithms):
 *  SX_BFS      active = newly visited; compute = level + 1; combine = vote
 *              (any one update suffices).  Output int32 depth, -1 unreached.
 *  SX_SSSP     active = distance lowered in the last iteration; compute =
 *              dist(v) + w(v,u); combine = minimum (aggregation).  Output
 *              uint32 distance, 0xFFFFFFFF unreached.
 *  SX_KCORE    active = alive with degree <= level; compute = remove v and
 *              lower the neighbour's degree; combine = sum.  Extended from
 *              the paper's fixed-k membership to the full decomposition:
 *              output int32 core number (v is in the k-core iff core >= k).
 *              Degree counts in- plus out-arcs for a directed graph.
 *              With kcore_k = k > 0 the program computes the paper's own
 *              k-core instead (Section 6): vertices of degree below k are
 *              deleted until none is left, a neighbour already below k is not
 *              decremented further, and the output is int32 membership, 1 for
 *              the vertices of the k-core and 0 for the others.
 *  SX_PAGERANK all vertices active; compute = rank(u)/outdeg(u); combine =
 *              sum; pr_iters synchronous iterations with damping pr_damping,
 *              uniform start 1/n, rank of vertices without out-arcs spread
 *              uniformly.  Output float rank (FP32 arithmetic).
 *  SX_WCC      connected components by minimum-label propagation: every
 *              vertex starts active with its own id as label; compute =
 *              label(v); combine = minimum.  Output int32 label = the
 *              smallest vertex id of the vertex's component (unique, so
 *              comparable bit for bit).  Undirected graphs only
 *              (SX_EUNSUPPORTED otherwise); the source is ignored (pass -1).
 *  SX_BP       belief propagation (Section 6: sum-product message passing,
 *              the vertex probability as metadata; Section 3.2: every vertex
 *              active, updates summed) on a binary pairwise Markov random
 *              field over an undirected graph: vertex v has the prior
 *              phi_v(1) = p_v, edge {u, v} the potential psi(x, y) = s_uv
 *              when x == y and 1 - s_uv otherwise, s_uv = (1 + bp_kappa *
 *              theta_uv / max(deg u, deg v)) / 2, theta_uv = (((w_uv - 1)
 *              mod 64) - 31.5) / 31.5 (arc weights 1..64 span -1..1; 1 on an
 *              unweighted graph).  bp_iters synchronous iterations
 *              b'(v, x) ~ phi_v(x) prod_{u in N(v)} sum_y psi(y, x) b(u, y)
 *              from b = phi.  d_out holds the priors p_v (float, each in
 *              (0, 1), else SX_EINVAL) on entry and the beliefs b(v, 1) on
 *              return (FP32 arithmetic, compensated sums).  Undirected
 *              graphs only (SX_EUNSUPPORTED otherwise); pass source -1. */
typedef enum { SX_BFS = 0, SX_SSSP = 1, SX_KCORE = 2, SX_PAGERANK = 3, SX_WCC = 4, SX_BP = 5 } sx_algo;

/* sssp_delta: bucket width of delta-stepping for SX_SSSP (Section 3.3: the
 * vertices whose distances lie in the lowest non-empty bucket [B - delta, B)
 * are relaxed together; the others stay listed, unexpanded, until the bound
 * B reaches them).  0 = no buckets: every listed vertex is expanded in every
 * iteration (plain frontier relaxation).  SX_DELTA_AUTO = the engine
 * chooses: 40 times the mean arc weight on graphs of at least 2^21 vertices
 * with fewer than 8 arcs per vertex, engaging after 64 iterations (runs that
 * end sooner stay unbucketed), no buckets on denser or smaller graphs (the
 * weights are summed on the device once per graph, before the run's timed
 * region).  Results are identical for any
 * value; it changes the work and the iteration count only.  Used by the
 * sequenced arrangement (SX_FUSE_AUTO / SX_SEQUENCED); the persistent and
 * unfused arrangements and batches relax without buckets, and a run that
 * switches to pull steps drops the buckets from then on. */
typedef struct {
  sx_algo algo;
  float pr_damping;      /* PageRank damping d (0.85)                          */
  int32_t pr_iters;      /* PageRank iterations (20)                           */
  uint32_t sssp_delta;   /* SSSP bucket width (0 = none)                       */
  int32_t kcore_k;       /* SX_KCORE: 0 = full decomposition (core numbers);
                            k > 0 = membership in the k-core (1 / 0)          */
  float pr_tol;          /* SX_PAGERANK: 0 = exactly pr_iters synchronous
                            pull iterations; > 0 = run until stable (Section
                            6): pull iterations while most vertices still
                            change, then the delta-accumulative push tail,
                            switched by a fixed decision tree (converged: stop;
                            at most n/2 vertices (the majority is stable)
                            changing by more than pr_tol (1 - d) / (2n) and
                            their out-arcs at most m / 16, or pr_iters pull
                            iterations done (0: 1,000): push; else pull); the
                            result lies within about pr_tol (L1) of the fixed
                            point, up to FP32 rounding; 0 <= pr_tol < 1      */
  float bp_kappa;        /* SX_BP: coupling scale, 0 <= bp_kappa < 1 (0 leaves
                            every potential uniform; the synchronous update is
                            a contraction with factor about bp_kappa)        */
  int32_t bp_iters;      /* SX_BP: iterations (0 returns the priors)          */
} sx_algo_params;
#define SX_DELTA_AUTO 0xFFFFFFFFu

sx_status sx_program_register(sx_ctx *ctx, const sx_algo_params *params, sx_program **out);
void sx_program_destroy(sx_program *p);

/* Per-iteration choices (Sections 4 and 5).  Each field 0 = automatic.
 *  direction  SX_DIR_AUTO | SX_DIR_PUSH | SX_DIR_PULL
 *  filter     SX_FILTER_JIT (online filter, ballot filter on overflow) |
 *             SX_FILTER_ONLINE (online filter without a capacity limit of
 *             its own: a workgroup may fill its whole region, about 2n / G
 *             entries per bin; a full region still falls back to the ballot
 *             filter, which keeps results exact) |
 *             SX_FILTER_BALLOT (always rebuild the worklist by ballot scan)
 *  bin_small  degree below which one lane takes a vertex (default 64)
 *  bin_large  degree from which a workgroup takes chunks of a vertex (512)
 *  online_cap SX_FILTER_JIT only: online-filter capacity in entries per
 *             wavefront and bin (a workgroup of 8 wavefronts overflows past
 *             8 x online_cap entries in a bin); 0 = the workgroup's region
 *  fused      SX_FUSED (selective fusion, Section 5: one persistent kernel
 *             per direction + software global barrier; a direction change
 *             launches the other kernel) | SX_FUSED_ALL (all fusion, Table
 *             table-compile: both directions in one persistent kernel that
 *             switches in place; BFS, SSSP and WCC, other programs take
 *             SX_FUSED) | SX_UNFUSED (one launch per phase and iteration,
 *             the host deciding between launches) | SX_SEQUENCED (one launch
 *             per phase, decisions taken on the device at the start of the
 *             next launch, launches enqueued ahead: the kernel boundary is
 *             the global barrier; a BFS / SSSP / WCC run enqueues first as
 *             many launches as the previous run of that algorithm on the
 *             same sx_graph needed, plus two, else 16) | 0 = auto
 *             (sequenced for BFS, SSSP and k-core, fused for PageRank)
 *  policy     SX_POLICY_HEURISTIC | SX_POLICY_LEARNED (MLP; needs
 *             sx_policy_load_mlp first)                                       */
enum { SX_DIR_AUTO = 0, SX_DIR_PUSH = 1, SX_DIR_PULL = 2 };
enum { SX_FILTER_JIT = 0, SX_FILTER_ONLINE = 1, SX_FILTER_BALLOT = 2 };
enum { SX_FUSE_AUTO = 0, SX_FUSED = 1, SX_UNFUSED = 2, SX_SEQUENCED = 3, SX_FUSED_ALL = 4 };
enum { SX_POLICY_HEURISTIC = 0, SX_POLICY_LEARNED = 1 };

typedef struct {
  int32_t direction;
  int32_t filter;
  int32_t bin_small;
  int32_t bin_large;
  int32_t online_cap;
  int32_t fused;
  int32_t policy;
  int32_t grid_wgs;      /* persistent grid size; 0 = occupancy x CUs (Eq. 1) */
  int32_t watchdog_us;   /* how long one wait at the software global barrier
                            may last before the run fails with SX_EDEADLOCK,
                            in microseconds of wall-clock time; 0 = 2 s      */
  int32_t kcore_tail;    /* k-core decomposition (sequenced arrangement): once
                            a level ends with at most this many vertices
                            left, the rest of the decomposition runs in one
                            workgroup whose LDS holds their degrees (the
                            alive subgraph compacted first); at most 36,864
                            (the most that fits).  0 = 16,384 vertices whose
                            rows, arcs to deleted vertices included, hold
                            at most 2^22 arcs (one CU's LDS atomics are
                            slower than the grid on more work); negative =
                            never.  Results are identical either way.        */
} sx_policy;

sx_status sx_program_set_policy(sx_program *p, const sx_policy *pol);

/* ---------------------------------------------------------------- run --- */
typedef struct {
  int32_t iterations;        /* BSP iterations (levels / rounds / sweeps)     */
  int32_t launches;          /* kernel launches issued for the run (sequenced:
                                also those enqueued ahead that found the run
                                over and returned at once)                    */
  int32_t pull_iters;        /* iterations processed in pull direction        */
  int32_t ballot_iters;      /* iterations whose worklist came from the ballot
                                filter                                         */
  int64_t edges_inspected;   /* arcs read by compute                          */
  int64_t vertex_expansions; /* worklist entries processed                    */
  double device_ms;          /* stream time of the run (HIP events)           */
  int64_t scan_entries;      /* list entries read by k-core level scans       */
  double barrier_wait_ms;    /* global-barrier stall: the time a workgroup
                                waits for the others, averaged over the run's
                                workgroups.  Persistent kernels: arrival to
                                release at each software barrier.  Sequenced
                                arrangement (the kernel boundary is the
                                barrier): end of a workgroup's phase to the
                                start of the same workgroup slot's next phase.
                                Wall-clock stamps on the device; 0 for the
                                one-phase arrangement                         */
  int32_t policy_evals;      /* decisions the learned network took           */
  float policy_x[8];         /* features and outputs of the last of them     */
  float policy_y[4];
} sx_run_stats;

/* Run program p on graph g.  source: start vertex (BFS, SSSP), ignored (pass
 * -1) for k-core and PageRank.  d_out: caller-owned device array of n
 * elements (int32 depth | uint32 dist | int32 core | float rank).  Blocks the
 * host until the run is complete.  stats may be NULL.
 * Errors: SX_EINVAL (source out of range, SSSP on an unweighted graph, wrong
 * d_out), SX_EDEADLOCK, SX_EOVERFLOW, SX_EHIP. */
sx_status sx_run(sx_program *p, const sx_graph *g, int32_t source, void *d_out,
                 void *hip_stream, sx_run_stats *stats);

/* -------------------------------------------- no-allocation variant --- */
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): sx_run for
 * BFS, SSSP or WCC on a graph the caller already holds in device memory,
 * described by d (SX_DEVICE_PTRS required; SX_UNDIRECTED as for
 * sx_graph_load; SX_REORDER and SX_VALIDATE not accepted), with the engine's
 * worklists, ballot words, stamps and control block carved from one static
 * device array of 256 MiB per device (a file-scope __device__ array, held
 * from the first sx_ctx_create on the device until the process ends)
 * instead of a graph workspace.  Same kernels, policies (except SX_UNFUSED,
 * rejected with SX_EUNSUPPORTED), results and statistics as sx_run on the
 * same graph loaded with SX_DEVICE_PTRS.  The call allocates nothing: the
 * context's pinned control-block mirrors and events come from
 * sx_ctx_create.
 * Size limit: the workspace takes about 61 n + 32 KiB G + 16 (G + 1)
 * (m / 2048 + 1) + 300 KiB bytes for a grid of G workgroups (the
 * program's grid, at most policy grid_wgs when that is set; 512 by default
 * on MI355X); a graph that needs more than 256 MiB fails with SX_EINVAL and
 * a message giving the bytes it needs (R-MAT scale 20, 16 M arcs: about
 * 140 MiB at 512 workgroups).
 * Concurrency: every call on a device shares that device's array and every
 * call through one context shares its mirrors: calls that overlap on one
 * GPU race (serialise them, e.g. on one stream from one thread).  The array
 * keeps the last call's contents; the call clears what must start at zero
 * (the control block) with a kernel on the stream.
 * Errors: as sx_run; SX_EINVAL also for a missing SX_DEVICE_PTRS or an
 * oversize graph; SX_EUNSUPPORTED for other algorithms, SX_UNFUSED,
 * SX_REORDER and directed WCC. */
sx_status sx_run_static(sx_program *p, const sx_graph_desc *d, int32_t source, void *d_out,
                        void *hip_stream, sx_run_stats *stats);

/* ------------------------------------------------ frontier inspection --- */
/* Run BFS, SSSP or WCC for at most `iterations` iterations in the one-phase
 * arrangement (SX_UNFUSED, whatever the program's policy says about fusion;
 * direction, filter and bins as the policy says) and stop before iteration
 * `iterations`, leaving the worklist that iteration would process in the
 * graph's workspace for sx_frontier_get.  d_out holds the vertex state at
 * that point.  Iteration 0 processes the source (WCC: every vertex).
 * Errors: as sx_run; SX_EUNSUPPORTED for renumbered graphs. */
sx_status sx_run_iterations(sx_program *p, const sx_graph *g, int32_t source, void *d_out,
                            void *hip_stream, int32_t iterations, sx_run_stats *stats);

/* The worklist left by the last sx_run_iterations on g, as the next push
 * iteration reads it (Section 4): for each bin in turn (0 small, 1 medium, 2
 * large), the workgroups' regions in workgroup order; a large vertex appears
 * once.  vertices / bins: host arrays of cap entries (bins[i] = the bin of
 * vertices[i]); *count = the list's length (may exceed cap: only cap entries
 * are written).  *from_ballot (nullable) = 1 when the list was built by the
 * ballot filter (then each bin is sorted and unique), 0 for the online
 * filter (order of arrival).  words (nullable, nwords entries): the ballot
 * filter's words of its last scan, OR-ed over the bins: bit j of word i
 * stands for vertex 64 i + j.  SX_ESTATE when the run stopped before a pull
 * iteration (no push list) or no such run was made.  Synchronises the
 * stream. */
sx_status sx_frontier_get(const sx_graph *g, int32_t *vertices, int32_t *bins, int32_t cap,
                          int32_t *count, int32_t *from_ballot, uint64_t *words, int64_t nwords,
                          void *hip_stream);

/* Copy a vertex array (n elements of the algorithm's output type) from the
 * device to host memory; synchronises the stream. */
sx_status sx_read_vertices(const sx_graph *g, sx_algo algo, const void *d_out, void *host_out,
                           void *hip_stream);

/* ------------------------------------------------------------ batches --- */
/* Many BFS / SSSP queries over several graphs in one persistent launch (a
 * project extension).  The grid is split into teams of team_wgs workgroups;
 * each team takes queries from a shared queue (largest first) and runs each
 * to completion with the same push/pull phases, filters and policy as sx_run,
 * synchronised by a barrier over the team alone.  Results are identical to
 * one sx_run per query.  Queries may share a graph; each needs its own d_out
 * (device, n elements of the algorithm's output type). */
typedef struct {
  const sx_graph *g;
  sx_algo algo;          /* SX_BFS or SX_SSSP                                */
  int32_t source;
  void *d_out;
} sx_query;

typedef struct {
  int32_t team_wgs;      /* workgroups per team (1..64)                      */
  int32_t bin_small;     /* bin thresholds (0 = policy / defaults)           */
  int32_t bin_large;
} sx_batch_config;

/* Run the batch.  pol: direction/filter/policy as for sx_run (NULL =
 * defaults); cfg NULL = the configuration last chosen by sx_batch_autotune
 * for this context, else team_wgs 4.  per_query (nullable, nq entries)
 * receives each query's counters; *batch_ms (nullable) the stream time.
 * The team workspaces (about 30 bytes per vertex of the largest graph, per
 * team) are kept in the context for reuse.
 * Errors: SX_EINVAL (bad query, graph of another context), SX_ENOMEM,
 * SX_EDEADLOCK, SX_EHIP. */
sx_status sx_run_batch(sx_ctx *ctx, const sx_query *queries, int32_t nq, const sx_policy *pol,
                       const sx_batch_config *cfg, void *hip_stream, sx_run_stats *per_query,
                       double *batch_ms);

/* Autotuner: times the batch under each candidate configuration (team sizes
 * 1, 2, 4, 8, 16, 32 x bin thresholds (64,256), (32,1024)), keeps the fastest
 * in the context for later sx_run_batch calls and returns it (and its time).
 * The queries' outputs hold the result of the last candidate run. */
sx_status sx_batch_autotune(sx_ctx *ctx, const sx_query *queries, int32_t nq, const sx_policy *pol,
                            void *hip_stream, sx_batch_config *best, double *best_ms);

/* Library/build facts for the measurement harness: kernel register use and
 * persistent-grid sizing (the Eq. 1 analogue).  name: one of "bfs_fused",
 * "sssp_fused", "wcc_fused" (the push kernels of selective fusion),
 * "bfs_fused_pull", "sssp_fused_pull", "wcc_fused_pull" (its pull kernels),
 * "bfs_fused_all", "sssp_fused_all", "wcc_fused_all" (all fusion), "bfs_seq", "sssp_seq", "wcc_seq",
 * "bfs_seq_wide", "sssp_seq_wide", "wcc_seq_wide" (the sequenced kernels for
 * graphs of 2^25 arcs or more, built for three workgroups per CU),
 * "bfs_push_step", "bfs_pull_step", "sssp_push_step",
 * "sssp_pull_step", "ballot_scan", "pull_scan", "kcore_fused", "kcore_seq",
 * "kcore_tail" (the peel of the one-workgroup tail: block 1024, grid 1),
 * "pagerank_fused", "pagerank_until_stable" (pr_tol > 0: its pull kernel),
 * "pagerank_push_tail" (its push kernel), "bp_fused", "batch".
 * Errors: SX_EINVAL (unknown name), SX_EHIP. */
typedef struct {
  int32_t vgprs, sgprs, lds_bytes, block, wgs_per_cu, grid_wgs, cus;
} sx_kernel_info;
sx_status sx_kernel_info_get(sx_ctx *ctx, const char *name, sx_kernel_info *out);

/* ------------------------------------------------------ learned policy --- */
/* A project extension, not in the paper: a small FP32 MLP, 8 frontier
 * features -> 32 -> 32 -> 4 (ReLU), chooses each iteration's direction
 * (output 0 > 0: pull), worklist filter (output 1 > 0: ballot) and bin
 * thresholds (outputs 2, 3: log2 of the small/medium and medium/large degree
 * thresholds).  Parameters are SX_MLP_NPARAMS floats: W1[32][8] row-major,
 * b1[32], W2[32][32], b2[32], W3[4][32], b3[4].  The outputs never change a
 * result, only the schedule.  The network is consulted for frontiers of at
 * least 32,768 arcs; below that (where no choice gains more than the inference
 * costs) the heuristic decides.
 * Features (float[8]) of the decision after an iteration: log2(1+nf)/24,
 * log2(1+mf)/32, log2(1+mu)/32, nf/n, min(reached/n, 4)/4,
 * (log2(1+nf) - log2(1+nf_prev))/8, log2(1+mf/nf)/16, pulling?1:0, where nf
 * and mf are the next frontier's vertices and arcs, mu the unexplored arcs
 * (BFS) or m (SSSP) and reached the vertices activated so far. */
#define SX_MLP_NPARAMS 1476
#define SX_MLP_FEATURES 8
#define SX_MLP_OUTPUTS 4

/* Copy host parameters into the context; programs with policy
 * SX_POLICY_LEARNED use them from then on.  SX_EINVAL unless nparams ==
 * SX_MLP_NPARAMS. */
sx_status sx_policy_load_mlp(sx_ctx *ctx, const float *params, int64_t nparams);

/* Batch inference: d_x device [n][8] -> d_y device [n][4], one wavefront
 * per sample through the same device function the engine's in-kernel
 * decisions evaluate. */
sx_status sx_mlp_forward(sx_ctx *ctx, const float *d_params, const float *d_x, int32_t n, float *d_y,
                         void *hip_stream);

/* The same inference on the host, as the one-phase arrangement's host-side
 * decisions evaluate it: host arrays params [SX_MLP_NPARAMS], x [n][8],
 * y [n][4].  Pure host arithmetic (no device call).  SX_EINVAL on NULL or
 * n < 0. */
sx_status sx_mlp_forward_host(const float *params, const float *x, int32_t n, float *y);

/* Mean loss over n samples and its gradient (device pointers).  d_target and
 * d_mask are [n][4]: outputs 0 and 1 take a binary cross-entropy on logits
 * against 0/1 targets, outputs 2 and 3 half the squared error; mask entries
 * are non-negative weights of the terms (0 drops a term, 1 keeps it).  d_loss: device float[1]; d_grad: device
 * float[SX_MLP_NPARAMS].  Sums run in sample order (deterministic). */
sx_status sx_mlp_loss_grad(sx_ctx *ctx, const float *d_params, const float *d_x, const float *d_target,
                           const float *d_mask, int32_t n, float *d_loss, float *d_grad,
                           void *hip_stream);

/* One Adam step (bias-corrected; step counts from 1) on device arrays of
 * SX_MLP_NPARAMS floats. */
sx_status sx_mlp_adam(sx_ctx *ctx, float *d_params, const float *d_grad, float *d_m, float *d_v,
                      int32_t step, float lr, float beta1, float beta2, float eps, void *hip_stream);

/* Timing records for training the policy.  Runs program p (BFS or SSSP) from
 * `source` in one-phase mode under the heuristic policy and, before every
 * `stride`-th iteration, times each of SX_POLICY_ARMS ways of running that
 * iteration from the same saved state (the state is restored after each arm,
 * so the run's result is unchanged).  Arms: 0 push on the online-filter lists
 * (NaN when they overflowed), 1-4 push after a ballot-filter rebuild with bin
 * thresholds (16,256) (64,256) (64,1024) (256,2048), 5 pull.  Writes up to
 * max_records rows: features [8] (as for the learned policy, at the decision
 * before the iteration) and arm_ms [6] (stream time of the arm).  *nrecords
 * receives the row count.  Host arrays; the run's output lands in d_out. */
#define SX_POLICY_ARMS 6
sx_status sx_policy_collect(sx_program *p, const sx_graph *g, int32_t source, void *d_out,
                            void *hip_stream, int32_t stride, float *features, float *arm_ms,
                            int32_t max_records, int32_t *nrecords);

/* Eq. 1 of Section 5: number of co-resident workgroups from a per-SM register
 * budget, registers per thread and threads per workgroup:
 *   floor(regs_per_sm / (regs_per_thread * threads_per_wg)) * sms.
 * Pure host arithmetic; returns -1 on non-positive input. */
int32_t sx_eq1_ctas(int32_t regs_per_sm, int32_t regs_per_thread, int32_t threads_per_wg, int32_t sms);

#ifdef __cplusplus
}
#endif
#endif /* SIMDX_H */
