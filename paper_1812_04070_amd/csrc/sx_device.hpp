// Device primitives of the ACC engine for CDNA4 (gfx950, wave64).
//
//  - wavefront ballot / popcount / lane-prefix (mbcnt) helpers, used by both
//    task-management filters of Section 4: the online filter appends active
//    vertices with one atomic per wavefront, the ballot filter turns a
//    coalesced scan of vertex metadata into 64-bit ballot words;
//  - workgroup reductions through LDS;
//  - the software global barrier that holds the persistent fused kernels of
//    Section 5 together, with a watchdog so that a grid that is not fully
//    resident reports an error instead of hanging.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sx_types.hpp"

#define SX_AG __HIP_MEMORY_SCOPE_AGENT
#define SX_DEV __device__ __forceinline__

namespace sx {

// ------------------------------------------------------------ wavefront ---
SX_DEV int lane_id() { return __lane_id(); }
SX_DEV int wave_in_wg() { return threadIdx.x >> 6; }

SX_DEV uint64_t ballot(bool p) { return __ballot(p); }

// number of set bits of `mask` in lanes below this lane
SX_DEV unsigned lane_prefix(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

SX_DEV int wave_sum_i(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
SX_DEV long long wave_sum_ll(long long v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
SX_DEV unsigned wave_min_u(unsigned v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) { unsigned t = __shfl_xor(v, o); v = t < v ? t : v; }
  return v;
}
// inclusive prefix sum over the wavefront
SX_DEV int wave_incl_scan(int v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o);
    if (l >= o) v += t;
  }
  return v;
}

// ---------------------------------------------------------- atomics -------
SX_DEV unsigned atomic_add_u32(unsigned *p, unsigned v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, SX_AG);
}
SX_DEV unsigned long long atomic_add_u64(unsigned long long *p, unsigned long long v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, SX_AG);
}
SX_DEV unsigned atomic_min_u32(unsigned *p, unsigned v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, SX_AG);
}
SX_DEV int atomic_sub_i32(int *p, int v) {
  return __hip_atomic_fetch_sub(p, v, __ATOMIC_RELAXED, SX_AG);
}
SX_DEV bool atomic_cas_i32(int *p, int expected, int desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, SX_AG);
}
// compare-and-swap returning the value found (== expected when it swapped),
// so that several can be in flight before the first result is looked at
SX_DEV int atomic_cas_old_i32(int *p, int expected, int desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       SX_AG);
  return expected;
}
SX_DEV int atomic_exch_i32(int *p, int v) {
  return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, SX_AG);
}
SX_DEV unsigned long long atomic_or_u64(unsigned long long *p, unsigned long long v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, SX_AG);
}
template <class T>
SX_DEV T load_relaxed(const T *p) {
  return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, SX_AG);
}
template <class T>
SX_DEV void store_relaxed(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, SX_AG);
}

// ------------------------------------------------------- workgroup -------
// Sum of one int per thread over the workgroup; every thread gets the total.
// `red` must hold kBlock/64 ints of LDS.
template <int kBlock>
SX_DEV long long wg_sum_ll(long long v, long long *red) {
  v = wave_sum_ll(v);
  if (lane_id() == 0) red[wave_in_wg()] = v;
  __syncthreads();
  long long t = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

// ------------------------------------------------ compensated sums -----
// FP32 sums with an error term (Knuth's TwoSum), merged in a fixed order, so
// that a sum over thousands of terms keeps its error near the rounding of
// the terms and is the same bits on every run.
struct CSum {
  float s, c;
};
// Knuth's TwoSum: s + x = t + e exactly
SX_DEV void cadd(CSum &a, float x) {
  const float t = a.s + x;
  const float z = t - a.s;
  const float e = (a.s - (t - z)) + (x - z);
  a.s = t;
  a.c += e;
}
SX_DEV CSum cmerge(CSum a, CSum b) {
  CSum r{a.s, a.c + b.c};
  cadd(r, b.s);
  return r;
}
SX_DEV CSum wave_merge(CSum a) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    CSum b{__shfl_xor(a.s, o), __shfl_xor(a.c, o)};
    a = cmerge(a, b);
  }
  return a;
}
// fixed-order workgroup merge; result valid in every thread
SX_DEV CSum wg_merge(CSum a, float *lds /* 2*kWaves */) {
  a = wave_merge(a);
  __syncthreads();
  if (lane_id() == 0) {
    lds[2 * wave_in_wg()] = a.s;
    lds[2 * wave_in_wg() + 1] = a.c;
  }
  __syncthreads();
  CSum r{lds[0], lds[1]};
  for (int w = 1; w < kWaves; ++w) r = cmerge(r, CSum{lds[2 * w], lds[2 * w + 1]});
  __syncthreads();
  return r;
}

// A (virtual) grid: workgroup `bid` of `nb` cooperating workgroups.  The
// single-query kernels use the hardware grid; the batched kernel splits the
// hardware grid into teams and gives each team its own virtual grid.
struct VGrid {
  unsigned bid, nb;
};
SX_DEV VGrid hw_grid() { return VGrid{blockIdx.x, gridDim.x}; }

// ---------------------------------------------------- global barrier ------
// Lock-array barrier (Section 5: every workgroup writes its own status word;
// one monitor workgroup waits for all of them and then releases everybody).
// Deadlock freedom comes from launching no more workgroups than can be
// resident at once (the Eq. 1 analogue, computed from the occupancy API on
// the host).  Each wait loop has a watchdog: when a wait has lasted `budget`
// ticks of the wall clock it raises ctrl->error = SX_ERR_DEADLOCK and every
// workgroup leaves the kernel at its next check.
//
// Arrival is a plain release store to a private 128-byte line, so arrivals
// never serialise on one address; the monitor's threads poll the flags in
// parallel.  gen is the barrier generation, kept per workgroup in a register
// and identical in all workgroups.  The time each workgroup spends between
// its arrival and its release is added to the statistics (barrier stall).
SX_DEV unsigned long long wall_ticks() { return wall_clock64(); }

struct GridBarrier {
  Ctrl *c;
  unsigned nblk, rank;
  unsigned gen;
  unsigned long long budget;

  SX_DEV GridBarrier(Ctrl *ctrl, unsigned start_gen, unsigned long long wd)
      : c(ctrl), nblk(gridDim.x), rank(blockIdx.x), gen(start_gen), budget(wd) {}
  SX_DEV GridBarrier(Ctrl *ctrl, unsigned start_gen, unsigned long long wd, const VGrid &vg)
      : c(ctrl), nblk(vg.nb), rank(vg.bid), gen(start_gen), budget(wd) {}

  SX_DEV bool failed() const { return load_relaxed(&c->error.v[0]) != 0u; }

  // Returns false when the watchdog fired or an error was raised (by any
  // workgroup).  The error word is read by one thread and shared through
  // LDS: hundreds of workgroups x 8 wavefronts loading one address would
  // queue on a single L2 channel.
  SX_DEV bool sync() {
    __shared__ unsigned s_err;
    const unsigned target = gen + 1;
    if (nblk == 1) {
      // a single workgroup: the workgroup barrier orders its global memory
      __syncthreads();
      if (threadIdx.x == 0) s_err = load_relaxed(&c->error.v[0]);
      __syncthreads();
      gen = target;
      return s_err == 0u;
    }
    __syncthreads();
    const unsigned long long t0 = wall_ticks();
    bool ok = true;
    if (rank == 0) {
      for (unsigned b = 1 + threadIdx.x; b < nblk; b += blockDim.x) {
        while (load_relaxed(&c->flags[b].v[0]) != target) {
          __builtin_amdgcn_s_sleep(2);
          if (failed()) { ok = false; break; }
          if (wall_ticks() - t0 > budget) {
            store_relaxed(&c->error.v[0], (unsigned)SX_ERR_DEADLOCK);
            ok = false;
            break;
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __syncthreads();
      if (threadIdx.x == 0)
        __hip_atomic_store(&c->bar_gen.v[0], target, __ATOMIC_RELEASE, SX_AG);
    } else if (threadIdx.x == 0) {
      __hip_atomic_store(&c->flags[rank].v[0], target, __ATOMIC_RELEASE, SX_AG);
      while (load_relaxed(&c->bar_gen.v[0]) != target) {
        __builtin_amdgcn_s_sleep(2);
        if (failed()) break;
        if (wall_ticks() - t0 > budget) {
          store_relaxed(&c->error.v[0], (unsigned)SX_ERR_DEADLOCK);
          break;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    if (threadIdx.x == 0) {
      s_err = load_relaxed(&c->error.v[0]) | (ok ? 0u : 1u);
      __hip_atomic_fetch_add((unsigned long long *)&c->statw[rank % kStatLines].v[4],
                             wall_ticks() - t0, __ATOMIC_RELAXED, SX_AG);
    }
    gen = target;
    __syncthreads();
    return ok && s_err == 0u;
  }
};

// Barrier stall of the sequenced arrangement, whose global barrier is the
// kernel boundary: workgroup b of launch L+1 adds the time since workgroup b
// of launch L ended (the wait for the slowest workgroup of launch L plus the
// launch gap).  Called by thread 0 of every workgroup of a launch that runs a
// phase; the first launch of a run finds no end time and adds nothing.
SX_DEV void seq_stall_enter(Ctrl *c, unsigned bid) {
  if (threadIdx.x != 0) return;
  const unsigned long long now = wall_ticks();
  const unsigned long long last = load_relaxed((const unsigned long long *)&c->flags[bid].v[4]);
  if (last && now > last)
    __hip_atomic_fetch_add((unsigned long long *)&c->statw[bid % kStatLines].v[4], now - last,
                           __ATOMIC_RELAXED, SX_AG);
}
// End of a launch that ran a phase (all threads of the workgroup call it).
SX_DEV void seq_stall_leave(Ctrl *c, unsigned bid) {
  __syncthreads();
  if (threadIdx.x == 0) store_relaxed((unsigned long long *)&c->flags[bid].v[4], wall_ticks());
}

// Words of the control block that every workgroup reads at the start of a
// launch: one wavefront loads the 128-byte line (and the error word) and
// shares them through LDS, for the same reason as in GridBarrier::sync.
SX_DEV void fetch_line(const Line &l, const Ctrl *c, unsigned *dst /* 33 words of LDS */) {
  if (threadIdx.x < 32) dst[threadIdx.x] = load_relaxed(&l.v[threadIdx.x]);
  else if (threadIdx.x == 32) dst[32] = load_relaxed(&c->error.v[0]);
  __syncthreads();
}

// Start every run from barrier generation 0 (called by one workgroup of the
// run's initialisation kernel, which completes before the persistent kernel
// starts on the same stream).
SX_DEV void reset_barrier(Ctrl *c) {
  for (int b = threadIdx.x; b < kMaxGrid; b += blockDim.x) {
    c->flags[b].v[0] = 0u;
    c->flags[b].v[4] = 0u;
    c->flags[b].v[5] = 0u;
  }
  if (threadIdx.x == 0) c->bar_gen.v[0] = 0u;
}

// Zero the statistics lines (words 0-5 of each) and the policy line; called
// by one workgroup of a run's initialisation kernel.
SX_DEV void reset_stat_lines(Ctrl *c) {
  for (int i = threadIdx.x; i < kStatLines * 6; i += blockDim.x) c->statw[i / 6].v[i % 6] = 0u;
  if (threadIdx.x < 32) c->pol.v[threadIdx.x] = 0u;
}

}  // namespace sx
