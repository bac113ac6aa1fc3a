// Training and batch inference of the policy MLP (see sx_policy.hpp).
//
//   forward   one thread per sample: h1, h2, y stored for the backward pass
//   delta     one thread per sample: dL/dy (BCE on logits for outputs 0-1,
//             squared error for 2-3, each masked), back through W3 and W2
//             with the ReLU masks; per-sample loss
//   reduce    one thread per parameter: the gradient summed over samples in
//             sample order with compensated FP32 summation (deterministic)
//   adam      one thread per parameter (Kingma & Ba, bias-corrected)
//
// The network is tiny (1,476 parameters), so the contractions are
// latency-bound vector code, not MFMA work.
#include "sx_kernels.hpp"
#include "sx_policy.hpp"

namespace sx {

struct CSumF {
  float s, c;
};
SX_DEV void csum_add(CSumF &a, float x) {
  const float t = a.s + x;
  const float z = t - a.s;
  a.c += (a.s - (t - z)) + (x - z);
  a.s = t;
}

__global__ void __launch_bounds__(256) k_mlp_forward(const float *__restrict__ P,
                                                     const float *__restrict__ X, int n,
                                                     float *__restrict__ Y, float *__restrict__ H) {
  __shared__ float p[kMlpParams];
  for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) p[i] = P[i];
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  float x[kMlpIn];
#pragma unroll
  for (int i = 0; i < kMlpIn; ++i) x[i] = X[(size_t)s * kMlpIn + i];
  float h1[kMlpHid];
#pragma unroll
  for (int j = 0; j < kMlpHid; ++j) {
    float a = p[kMlpB1 + j];
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i) a += p[kMlpW1 + j * kMlpIn + i] * x[i];
    h1[j] = a > 0.f ? a : 0.f;
  }
  float y[kMlpOut];
#pragma unroll
  for (int k = 0; k < kMlpOut; ++k) y[k] = p[kMlpB3 + k];
  for (int j = 0; j < kMlpHid; ++j) {
    float a = p[kMlpB2 + j];
#pragma unroll
    for (int i = 0; i < kMlpHid; ++i) a += p[kMlpW2 + j * kMlpHid + i] * h1[i];
    const float h2 = a > 0.f ? a : 0.f;
    if (H) H[(size_t)s * 2 * kMlpHid + kMlpHid + j] = h2;
#pragma unroll
    for (int k = 0; k < kMlpOut; ++k) y[k] += p[kMlpW3 + k * kMlpHid + j] * h2;
  }
  if (H)
    for (int j = 0; j < kMlpHid; ++j) H[(size_t)s * 2 * kMlpHid + j] = h1[j];
#pragma unroll
  for (int k = 0; k < kMlpOut; ++k) Y[(size_t)s * kMlpOut + k] = y[k];
}

SX_DEV float sigmoidf_(float z) { return 1.f / (1.f + expf(-z)); }
SX_DEV float bce_logits(float z, float t) {
  return fmaxf(z, 0.f) - z * t + log1pf(expf(-fabsf(z)));
}

// D layout per sample: d1[32], d2[32], d3[4] (already divided by n).
__global__ void __launch_bounds__(256) k_mlp_delta(const float *__restrict__ P,
                                                   const float *__restrict__ Y,
                                                   const float *__restrict__ T,
                                                   const float *__restrict__ M,
                                                   const float *__restrict__ H, int n,
                                                   float *__restrict__ D, float *__restrict__ L) {
  __shared__ float p[kMlpParams];
  for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) p[i] = P[i];
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const float *y = Y + (size_t)s * kMlpOut;
  const float *t = T + (size_t)s * kMlpOut;
  const float *m = M + (size_t)s * kMlpOut;
  const float inv = 1.f / (float)n;
  float d3[kMlpOut];
  d3[0] = m[0] * (sigmoidf_(y[0]) - t[0]) * inv;
  d3[1] = m[1] * (sigmoidf_(y[1]) - t[1]) * inv;
  d3[2] = m[2] * (y[2] - t[2]) * inv;
  d3[3] = m[3] * (y[3] - t[3]) * inv;
  L[s] = m[0] * bce_logits(y[0], t[0]) + m[1] * bce_logits(y[1], t[1]) +
         0.5f * m[2] * (y[2] - t[2]) * (y[2] - t[2]) + 0.5f * m[3] * (y[3] - t[3]) * (y[3] - t[3]);
  const float *h1 = H + (size_t)s * 2 * kMlpHid;
  const float *h2 = h1 + kMlpHid;
  float *o = D + (size_t)s * (2 * kMlpHid + kMlpOut);
  float d2[kMlpHid];
  for (int j = 0; j < kMlpHid; ++j) {
    float a = 0.f;
#pragma unroll
    for (int k = 0; k < kMlpOut; ++k) a += p[kMlpW3 + k * kMlpHid + j] * d3[k];
    d2[j] = h2[j] > 0.f ? a : 0.f;
    o[kMlpHid + j] = d2[j];
  }
  for (int i = 0; i < kMlpHid; ++i) {
    float a = 0.f;
    for (int j = 0; j < kMlpHid; ++j) a += p[kMlpW2 + j * kMlpHid + i] * d2[j];
    o[i] = h1[i] > 0.f ? a : 0.f;
  }
#pragma unroll
  for (int k = 0; k < kMlpOut; ++k) o[2 * kMlpHid + k] = d3[k];
}

// One thread per parameter (plus one for the loss): gradient summed over
// samples in order.
__global__ void __launch_bounds__(256) k_mlp_reduce(const float *__restrict__ X,
                                                    const float *__restrict__ H,
                                                    const float *__restrict__ D,
                                                    const float *__restrict__ L, int n,
                                                    float *__restrict__ G, float *__restrict__ loss) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q > kMlpParams) return;
  const int dstride = 2 * kMlpHid + kMlpOut;
  CSumF acc{0.f, 0.f};
  if (q == kMlpParams) {
    for (int s = 0; s < n; ++s) csum_add(acc, L[s]);
    loss[0] = (acc.s + acc.c) / (float)n;
    return;
  }
  // which parameter: delta row (dsel, j) times input column (isel, i)
  int doff, j, src, i;  // src: 0 = x, 1 = h1, 2 = h2, 3 = bias (1)
  if (q < kMlpB1) { j = q / kMlpIn; i = q % kMlpIn; doff = 0; src = 0; }
  else if (q < kMlpW2) { j = q - kMlpB1; i = 0; doff = 0; src = 3; }
  else if (q < kMlpB2) { const int r = q - kMlpW2; j = r / kMlpHid; i = r % kMlpHid; doff = kMlpHid; src = 1; }
  else if (q < kMlpW3) { j = q - kMlpB2; i = 0; doff = kMlpHid; src = 3; }
  else if (q < kMlpB3) { const int r = q - kMlpW3; j = r / kMlpHid; i = r % kMlpHid; doff = 2 * kMlpHid; src = 2; }
  else { j = q - kMlpB3; i = 0; doff = 2 * kMlpHid; src = 3; }
  for (int s = 0; s < n; ++s) {
    const float d = D[(size_t)s * dstride + doff + j];
    float a;
    if (src == 0) a = X[(size_t)s * kMlpIn + i];
    else if (src == 1) a = H[(size_t)s * 2 * kMlpHid + i];
    else if (src == 2) a = H[(size_t)s * 2 * kMlpHid + kMlpHid + i];
    else a = 1.f;
    csum_add(acc, d * a);
  }
  G[q] = acc.s + acc.c;
}

__global__ void __launch_bounds__(256) k_mlp_adam(float *__restrict__ P, const float *__restrict__ G,
                                                  float *__restrict__ Mo, float *__restrict__ Vo,
                                                  int step, float lr, float b1, float b2, float eps) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kMlpParams) return;
  const float g = G[q];
  const float m = b1 * Mo[q] + (1.f - b1) * g;
  const float v = b2 * Vo[q] + (1.f - b2) * g * g;
  Mo[q] = m;
  Vo[q] = v;
  const float mh = m / (1.f - powf(b1, (float)step));
  const float vh = v / (1.f - powf(b2, (float)step));
  P[q] -= lr * mh / (sqrtf(vh) + eps);
}

// Batch inference through the function the engine's decisions call
// (mlp_eval_wave): weights staged in LDS, one wavefront per sample.
__global__ void __launch_bounds__(256) k_mlp_forward_wave(const float *__restrict__ P,
                                                          const float *__restrict__ X, int n,
                                                          float *__restrict__ Y) {
  __shared__ __attribute__((aligned(16))) float p[kMlpParams + 4];
  for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) p[i] = P[i];
  __syncthreads();
  const int waves = (int)(gridDim.x * blockDim.x / 64);
  for (int s = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6); s < n; s += waves) {
    float x[kMlpIn], y[kMlpOut];
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i) x[i] = X[(size_t)s * kMlpIn + i];
    mlp_eval_wave(p, x, y);
    if (lane_id() < kMlpOut) {
      float v = y[0];
      if (lane_id() == 1) v = y[1];
      else if (lane_id() == 2) v = y[2];
      else if (lane_id() == 3) v = y[3];
      Y[(size_t)s * kMlpOut + lane_id()] = v;
    }
  }
}

hipError_t mlp_forward_wave(const float *P, const float *X, int n, float *Y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int grid = (n + 3) / 4;
  if (grid > 2048) grid = 2048;
  hipLaunchKernelGGL(k_mlp_forward_wave, dim3(grid), dim3(256), 0, s, P, X, n, Y);
  return hipGetLastError();
}

hipError_t mlp_forward(const float *P, const float *X, int n, float *Y, float *H, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3((n + 255) / 256), dim3(256), 0, s, P, X, n, Y, H);
  return hipGetLastError();
}

hipError_t mlp_loss_grad(const float *P, const float *X, const float *T, const float *M, int n,
                         float *Y, float *H, float *D, float *L, float *loss, float *G,
                         hipStream_t s) {
  if (n <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mlp_forward, dim3((n + 255) / 256), dim3(256), 0, s, P, X, n, Y, H);
  hipLaunchKernelGGL(k_mlp_delta, dim3((n + 255) / 256), dim3(256), 0, s, P, Y, T, M, H, n, D, L);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 1 + 255) / 256), dim3(256), 0, s, X, H, D, L, n,
                     G, loss);
  return hipGetLastError();
}

hipError_t mlp_adam(float *P, const float *G, float *Mo, float *Vo, int step, float lr, float b1,
                    float b2, float eps, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, P, G, Mo, Vo, step,
                     lr, b1, b2, eps);
  return hipGetLastError();
}

}  // namespace sx
