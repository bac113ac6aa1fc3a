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

// Frontier features of the decision after iteration it.
struct PolicyState {
  unsigned nf_prev;             // frontier size of the previous decision
  unsigned long long reached;   // vertices activated so far (cumulative)
};

__host__ __device__ inline float log2p1(double x) {
  return (float)(log2(1.0 + (x > 0 ? x : 0.0)));
}

__host__ __device__ inline void policy_features(unsigned nf, unsigned long long mf,
                                                unsigned long long mu, int n, long long m,
                                                const PolicyState &ps, bool pulling, float x[8]) {
  const double dn = n > 0 ? (double)n : 1.0;
  x[0] = log2p1(nf) / 24.f;
  x[1] = log2p1((double)mf) / 32.f;
  x[2] = log2p1((double)mu) / 32.f;
  x[3] = (float)((double)nf / dn);
  const double vis = (double)ps.reached / dn;
  x[4] = (float)(vis < 4.0 ? vis / 4.0 : 1.0);
  x[5] = (log2p1(nf) - log2p1(ps.nf_prev)) / 8.f;
  x[6] = log2p1((double)mf / (nf > 0 ? (double)nf : 1.0)) / 16.f;
  x[7] = pulling ? 1.f : 0.f;
  (void)m;
}

// Forward pass by one wavefront (lanes 0..31 own a hidden unit).  `P` are the
// parameters (LDS), `x` the features, `h` 64 floats of LDS scratch; the
// outputs are returned in every lane.
SX_DEV void mlp_eval_wave(const float *P, const float x[8], float *h, float y[4]) {
  const int l = lane_id();
  if (l < kMlpHid) {
    float s = P[kMlpB1 + l];
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i) s += P[kMlpW1 + l * kMlpIn + i] * x[i];
    h[l] = s > 0.f ? s : 0.f;
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  if (l < kMlpHid) {
    float s = P[kMlpB2 + l];
    for (int i = 0; i < kMlpHid; ++i) s += P[kMlpW2 + l * kMlpHid + i] * h[i];
    h[kMlpHid + l] = s > 0.f ? s : 0.f;
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
#pragma unroll
  for (int k = 0; k < kMlpOut; ++k) {
    float s = P[kMlpB3 + k];
    for (int i = 0; i < kMlpHid; ++i) s += P[kMlpW3 + k * kMlpHid + i] * h[kMlpHid + i];
    y[k] = s;
  }
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

}  // namespace sx
