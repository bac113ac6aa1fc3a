// The learned per-iteration policy (a project extension; the paper's own
// choices are the online/ballot JIT rule of Section 4 and the push/pull
// switching of Section 5).  A small FP32 MLP, 8 frontier features -> 32 -> 32
// -> 4, ReLU hidden layers, chooses for the next iteration:
//   y0 > 0  pull (else push)
//   y1 > 0  rebuild the push worklist with the ballot filter (else online)
//   y2      log2 of the small/medium bin threshold   (rounded, clamped 2..8)
//   y3      log2 of the medium/large bin threshold   (rounded, clamped 6..12)
// Parameters (1,476 floats): W1[32][8], b1[32], W2[32][32], b2[32], W3[4][32],
// b3[4].  Every workgroup evaluates the network on the same features in the
// same order, so every workgroup takes the same decision without an extra
// barrier.
#pragma once

#include "sx_device.hpp"

namespace sx {

constexpr int kMlpIn = 8, kMlpHid = 32, kMlpOut = 4;
constexpr int kMlpW1 = 0, kMlpB1 = kMlpW1 + kMlpHid * kMlpIn, kMlpW2 = kMlpB1 + kMlpHid,
              kMlpB2 = kMlpW2 + kMlpHid * kMlpHid, kMlpW3 = kMlpB2 + kMlpHid,
              kMlpB3 = kMlpW3 + kMlpOut * kMlpHid, kMlpParams = kMlpB3 + kMlpOut;
static_assert(kMlpParams == 1476, "parameter count");

// The network is consulted for frontiers of at least this many arcs: an
// in-kernel decision by the network adds about 1.5 us to its launch (weights
// staged into LDS by every workgroup, one wavefront evaluating), which the
// thousands of light iterations of a grid pay without any gain (1024^2 grid
// SSSP, 2,600 iterations of 10^4 to 10^5 arcs: 35.6 -> 38.0 ms with the
// network consulted from 32,768 arcs); from 2^18 arcs an iteration takes
// 50 us or more.
constexpr unsigned long long kPolicyMinArcs = 1ull << 18;

// Frontier features of the decision after iteration it.
struct PolicyState {
  unsigned nf_prev;             // frontier size of the previous decision
  unsigned long long reached;   // vertices activated so far (cumulative)
};

// FP32 throughout: the same function computes the features on the host
// (timing collection) and on the device (every decision, on its critical
// path), where double-precision transcendentals would cost microseconds.
__host__ __device__ inline float log2p1(float x) { return log2f(1.f + (x > 0.f ? x : 0.f)); }

__host__ __device__ inline void policy_features(unsigned nf, unsigned long long mf,
                                                unsigned long long mu, int n, long long m,
                                                const PolicyState &ps, bool pulling, float x[8]) {
  const float dn = n > 0 ? (float)n : 1.f;
  const float lnf = log2p1((float)nf);
  x[0] = lnf / 24.f;
  x[1] = log2p1((float)mf) / 32.f;
  x[2] = log2p1((float)mu) / 32.f;
  x[3] = (float)nf / dn;
  const float vis = (float)ps.reached / dn;
  x[4] = vis < 4.f ? vis / 4.f : 1.f;
  x[5] = (lnf - log2p1((float)ps.nf_prev)) / 8.f;
  x[6] = log2p1((float)mf / (nf > 0 ? (float)nf : 1.f)) / 16.f;
  x[7] = pulling ? 1.f : 0.f;
  (void)m;
}

// Forward pass by one wavefront; weights `P` (LDS, staged at kernel start,
// 16-byte aligned), features `x` identical in every lane; the outputs are
// returned in every lane.  Lanes l and l + 32 own hidden unit l; the hidden
// vectors move between lanes by shuffles: about 60 dependent ALU / shuffle
// steps, a fraction of a microsecond.  Every workgroup runs the same
// instruction sequence on the same inputs, so every workgroup gets the same
// bits.
SX_DEV void mlp_eval_wave(const float *P, const float x[8], float y[4]) {
  const int lane = lane_id();
  const int l = lane & 31;
  const float4 w1a = *(const float4 *)(P + kMlpW1 + l * kMlpIn);
  const float4 w1b = *(const float4 *)(P + kMlpW1 + l * kMlpIn + 4);
  float h1 = P[kMlpB1 + l];
  h1 += w1a.x * x[0];
  h1 += w1a.y * x[1];
  h1 += w1a.z * x[2];
  h1 += w1a.w * x[3];
  h1 += w1b.x * x[4];
  h1 += w1b.y * x[5];
  h1 += w1b.z * x[6];
  h1 += w1b.w * x[7];
  h1 = h1 > 0.f ? h1 : 0.f;
  const float4 *w2 = (const float4 *)(P + kMlpW2 + l * kMlpHid);
  float h2 = P[kMlpB2 + l];
#pragma unroll
  for (int q = 0; q < kMlpHid / 4; ++q) {
    const float4 w = w2[q];
    h2 += w.x * __shfl(h1, 4 * q);
    h2 += w.y * __shfl(h1, 4 * q + 1);
    h2 += w.z * __shfl(h1, 4 * q + 2);
    h2 += w.w * __shfl(h1, 4 * q + 3);
  }
  h2 = h2 > 0.f ? h2 : 0.f;
  // lanes 0-31 form outputs 0 and 1, lanes 32-63 outputs 2 and 3
  const int k0 = lane < 32 ? 0 : 2;
  float p0 = P[kMlpW3 + k0 * kMlpHid + l] * h2;
  float p1 = P[kMlpW3 + (k0 + 1) * kMlpHid + l] * h2;
#pragma unroll
  for (int o = 16; o >= 1; o >>= 1) {
    p0 += __shfl_xor(p0, o);
    p1 += __shfl_xor(p1, o);
  }
  y[0] = __shfl(p0, 0) + P[kMlpB3 + 0];
  y[1] = __shfl(p1, 0) + P[kMlpB3 + 1];
  y[2] = __shfl(p0, 32) + P[kMlpB3 + 2];
  y[3] = __shfl(p1, 32) + P[kMlpB3 + 3];
}

// Host evaluation of the same network (one-phase mode decides on the host).
inline void mlp_eval_host(const float *P, const float x[8], float y[4]) {
  float h1[kMlpHid], h2[kMlpHid];
  for (int l = 0; l < kMlpHid; ++l) {
    float s = P[kMlpB1 + l];
    for (int i = 0; i < kMlpIn; ++i) s += P[kMlpW1 + l * kMlpIn + i] * x[i];
    h1[l] = s > 0.f ? s : 0.f;
  }
  for (int l = 0; l < kMlpHid; ++l) {
    float s = P[kMlpB2 + l];
    for (int i = 0; i < kMlpHid; ++i) s += P[kMlpW2 + l * kMlpHid + i] * h1[i];
    h2[l] = s > 0.f ? s : 0.f;
  }
  for (int k = 0; k < kMlpOut; ++k) {
    float s = P[kMlpB3 + k];
    for (int i = 0; i < kMlpHid; ++i) s += P[kMlpW3 + k * kMlpHid + i] * h2[i];
    y[k] = s;
  }
}

__host__ __device__ inline int clamp_log2(float v, int lo, int hi) {
  int r = (int)floorf(v + 0.5f);
  return r < lo ? lo : (r > hi ? hi : r);
}

// How far a logit must lean away from the heuristic's choice before the
// network's choice replaces it.  On the 361 training records the heuristic
// runs within 0.6 % of the best of the six arms per iteration (22.06 ms
// against 21.92 ms summed); the trained network's picks cost 23.14 ms when
// followed at margin 0, 23.08 at 1, 22.43 at 2 and 22.06 (the heuristic's)
// at 4: the margin is the smallest at which the network costs nothing on
// its own training data.
constexpr float kPolicyMargin = 4.0f;

// The heuristic's decision d for the next iteration, amended by the network's
// outputs y where the caller left the choice open (direction SX_DIR_AUTO,
// filter SX_FILTER_JIT, bins not fixed): each logit is shifted toward the
// heuristic's own choice by kPolicyMargin, and the bin thresholds follow the
// network only for a ballot rebuild the network chose; otherwise they are
// the run's (dflt_t1, dflt_t2).  Shared by the device decision and the
// one-phase host loop.
__host__ __device__ inline void apply_network(const float y[kMlpOut], bool pulling, bool ovf, int direction,
                                              int filter, bool bins_fixed, int dflt_t1, int dflt_t2,
                                              Decision &d, int &t1, int &t2) {
  if (direction == 0) {
    const bool h_pull = pulling ? !d.to_push : d.to_pull;
    const bool n_pull = y[0] + (h_pull ? kPolicyMargin : -kPolicyMargin) > 0.f;
    if (!pulling) d.to_pull = n_pull;
    else d.to_push = !n_pull;
  }
  bool net_ballot = false;
  if (!pulling && !d.to_pull) {
    if (filter == 0) {
      const bool h_ballot = d.ballot;
      const bool b = y[1] + (h_ballot ? kPolicyMargin : -kPolicyMargin) > 0.f;
      net_ballot = b && !h_ballot;
      d.ballot = ovf || b;
    } else {
      d.ballot = ovf || filter == 2;
    }
  }
  if (!bins_fixed) {
    if (net_ballot) {
      t1 = 1 << clamp_log2(y[2], 2, 8);
      const int u = 1 << clamp_log2(y[3], 6, 12);
      t2 = u > t1 ? u : t1;
    } else {
      t1 = dflt_t1;
      t2 = dflt_t2;
    }
  }
}

}  // namespace sx
