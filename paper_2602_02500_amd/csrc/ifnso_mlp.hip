// Learned coefficients: a small MLP mapping spectral moments of the Gram powers to the
// per-matrix coefficients of the Gram-basis polynomial with exponents {0,1,2,4,8,16}.
//
//   m_j = tr(G^(2^j)) / h (j = 0..7),  phi_j = log2(m_j) / (8 * 2^j)
//   h1 = gelu(W1 phi + b1), h2 = gelu(W2 h1 + b2), z = W3 h2 + b3,  c = z + (1 - sum z) / 6
//
// gelu is the exact-erf form. Training minimises the spectral form of ||Y - U V^T||_F^2 / h,
// (1/h) sum_i (f(s_i) - 1)^2 with f(x) = x * sum_k c_k x^(2 e_k), over normalised singular
// values s_i; the polynomial acts on each singular value independently, so the loss needs the
// singular values only. The paper names such dynamic coefficients as future work (Sec. 4).
//
// Kernels: training step (one wave per sample: forward, loss, backward into a per-sample
// gradient row), a fixed-order gradient reduction fused with Adam, feature extraction from a
// spectrum, batch inference, and the in-pipeline kernel that forms the features from the level
// partials of a plan and writes each problem's coefficients.
#include <hip/hip_runtime.h>
#include <math.h>

#include "ifnso_common.hpp"
#include "ifnso_launch.hpp"
#include "ifnso_tile.hpp"

namespace ifnso {
namespace mlp {

constexpr int IN = 8, HID = 64, OUT = 6;
constexpr int OW1 = 0, OB1 = OW1 + HID * IN, OW2 = OB1 + HID, OB2 = OW2 + HID * HID, OW3 = OB2 + HID,
              OB3 = OW3 + OUT * HID, NP = OB3 + OUT;
static_assert(NP == 5126, "parameter count");
constexpr int EXP[OUT] = {0, 1, 2, 4, 8, 16};

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float x) {
  return 0.5f * (1.f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Forward pass of one sample by one wave; fills the shared activations and c (lane o < 6).
struct Act {
  float phi[IN], a1[HID], h1[HID], a2[HID], h2[HID], z[OUT], c[OUT];
};

__device__ __forceinline__ void forward(const float *__restrict__ th, Act &s) {
  const int l = threadIdx.x & 63;
  float a = th[OB1 + l];
#pragma unroll
  for (int k = 0; k < IN; k++) a = fmaf(th[OW1 + l * IN + k], s.phi[k], a);
  s.a1[l] = a;
  s.h1[l] = gelu(a);
  __syncthreads();
  a = th[OB2 + l];
  for (int k = 0; k < HID; k++) a = fmaf(th[OW2 + l * HID + k], s.h1[k], a);
  s.a2[l] = a;
  s.h2[l] = gelu(a);
  __syncthreads();
  if (l < OUT) {
    a = th[OB3 + l];
    for (int k = 0; k < HID; k++) a = fmaf(th[OW3 + l * HID + k], s.h2[k], a);
    s.z[l] = a;
  }
  __syncthreads();
  if (l < OUT) {
    float zs = 0.f;
#pragma unroll
    for (int o = 0; o < OUT; o++) zs += s.z[o];
    s.c[l] = s.z[l] + (1.f - zs) / (float)OUT;
  }
  __syncthreads();
}

// log2 m_j (j = 0..7) of a spectrum, in float64 log space (no power underflows).
__device__ void spectrum_log2_moments(const float *sig, int n, double *out /*[8], lane 0 writes*/) {
  const int l = threadIdx.x & 63;
  double ss = 0.0;
  for (int i = l; i < n; i += 64) ss += (double)sig[i] * sig[i];
  ss = wave_sum_d(ss);
  const double l2ss = log2(ss);
  for (int j = 0; j < IN; j++) {
    const double p = exp2((double)j);
    double mx = -INFINITY;
    for (int i = l; i < n; i += 64)
      if (sig[i] > 0.f) mx = fmax(mx, p * (2.0 * log2((double)sig[i]) - l2ss));
    mx = wave_max_d(mx);
    double acc = 0.0;
    for (int i = l; i < n; i += 64)
      if (sig[i] > 0.f) acc += exp2(p * (2.0 * log2((double)sig[i]) - l2ss) - mx);
    acc = wave_sum_d(acc);
    if (l == 0) out[j] = mx + log2(acc) - log2((double)n);
  }
}

__global__ __launch_bounds__(64) void k_features(const float *sig, const int32_t *nsig, int smax, float *feats) {
  __shared__ double lm[IN];
  const int s = blockIdx.x;
  spectrum_log2_moments(sig + (int64_t)s * smax, nsig[s], lm);
  __syncthreads();
  if (threadIdx.x < IN) feats[s * IN + threadIdx.x] = (float)(lm[threadIdx.x] / (8.0 * exp2((double)threadIdx.x)));
}

__global__ __launch_bounds__(64) void k_forward(const float *feats, const float *th, double *coeffs) {
  __shared__ Act s;
  const int b = blockIdx.x, l = threadIdx.x;
  if (l < IN) s.phi[l] = feats[b * IN + l];
  __syncthreads();
  forward(th, s);
  if (l < OUT) coeffs[b * OUT + l] = (double)s.c[l];
}

// One sample per wave: forward, spectral loss, backward; gradient row grads[s][NP], loss[s].
__global__ __launch_bounds__(64) void k_train(const float *feats, const float *sig, const int32_t *nsig, int smax,
                                              const float *th, float *grads, float *losses) {
  __shared__ Act s;
  __shared__ float dz[OUT], da2[HID], da1[HID];
  const int b = blockIdx.x, l = threadIdx.x;
  if (l < IN) s.phi[l] = feats[b * IN + l];
  __syncthreads();
  forward(th, s);
  // spectral loss and dL/dc
  const float *sg = sig + (int64_t)b * smax;
  const int n = nsig[b];
  float ss = 0.f;
  for (int i = l; i < n; i += 64) ss = fmaf(sg[i], sg[i], ss);
  ss = wave_sum_f(ss);
  const float inv = 1.f / sqrtf(ss);
  float c[OUT];
#pragma unroll
  for (int o = 0; o < OUT; o++) c[o] = s.c[o];
  float lsum = 0.f, dc[OUT] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int i = l; i < n; i += 64) {
    const float x = sg[i] * inv;
    float pw[OUT];
    const float x2 = x * x, x4 = x2 * x2, x8 = x4 * x4, x16 = x8 * x8, x32 = x16 * x16;
    pw[0] = x;
    pw[1] = x * x2;
    pw[2] = x * x4;
    pw[3] = x * x8;
    pw[4] = x * x16;
    pw[5] = x * x32;
    float f = 0.f;
#pragma unroll
    for (int o = 0; o < OUT; o++) f = fmaf(c[o], pw[o], f);
    const float r = f - 1.f;
    lsum = fmaf(r, r, lsum);
#pragma unroll
    for (int o = 0; o < OUT; o++) dc[o] = fmaf(r, pw[o], dc[o]);
  }
  lsum = wave_sum_f(lsum);
  float dcs[OUT];
#pragma unroll
  for (int o = 0; o < OUT; o++) dcs[o] = wave_sum_f(dc[o]) * (2.f / (float)n);
  float mean = 0.f;
#pragma unroll
  for (int o = 0; o < OUT; o++) mean += dcs[o];
  mean /= (float)OUT;
  if (l < OUT) dz[l] = dcs[l] - mean;
  __syncthreads();
  float *g = grads + (int64_t)b * NP;
  // layer 3
#pragma unroll
  for (int o = 0; o < OUT; o++) g[OW3 + o * HID + l] = dz[o] * s.h2[l];
  if (l < OUT) g[OB3 + l] = dz[l];
  float dh2 = 0.f;
#pragma unroll
  for (int o = 0; o < OUT; o++) dh2 = fmaf(th[OW3 + o * HID + l], dz[o], dh2);
  da2[l] = dh2 * gelu_d(s.a2[l]);
  __syncthreads();
  // layer 2
  for (int j = 0; j < HID; j++) g[OW2 + j * HID + l] = da2[j] * s.h1[l];
  g[OB2 + l] = da2[l];
  float dh1 = 0.f;
  for (int j = 0; j < HID; j++) dh1 = fmaf(th[OW2 + j * HID + l], da2[j], dh1);
  da1[l] = dh1 * gelu_d(s.a1[l]);
  __syncthreads();
  // layer 1
#pragma unroll
  for (int k = 0; k < IN; k++) g[OW1 + l * IN + k] = da1[l] * s.phi[k];
  g[OB1 + l] = da1[l];
  if (l == 0) losses[b] = lsum / (float)n;
}

// Mean gradient over the batch in sample order, then one Adam step (PyTorch's update rule).
__global__ __launch_bounds__(256) void k_adam(int n, const float *grads, const float *losses, float *th, float *m,
                                              float *v, int t, float lr, float b1, float b2, float eps, float *gout,
                                              float *lout) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0 && lout) {
    float ls = 0.f;
    for (int s = 0; s < n; s++) ls += losses[s];
    *lout = ls / (float)n;
  }
  if (p >= NP) return;
  float gs = 0.f;
  for (int s = 0; s < n; s++) gs += grads[(int64_t)s * NP + p];
  const float g = gs / (float)n;
  if (gout) gout[p] = g;
  const float mm = b1 * m[p] + (1.f - b1) * g;
  const float vv = b2 * v[p] + (1.f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  const float mh = mm / (1.f - powf(b1, (float)t));
  const float vh = vv / (1.f - powf(b2, (float)t));
  th[p] -= lr * mh / (sqrtf(vh) + eps);
}

// In-pipeline inference for a learned plan: features from the level partials, the network,
// and the per-problem coefficient slots (falling back to the fixed ones when a prediction is
// not finite). Level l holds S_l * B_l = G^(2^(l-1)); log2 S_1 = -log2 ||A||^2 and
// log2 S_(l+1) = 2 log2 S_l + round(log2 ||B_l||_F^2).
__global__ __launch_bounds__(64) void k_learned(const StageArgs a, const float *th, const double *fixed_slots) {
  __shared__ Act s;
  __shared__ double lm[IN];
  __shared__ int ok;
  const int l = threadIdx.x;
  const ProbDev &P = a.tasks ? a.probs[blockIdx.x] : a.one;
  const int nt = P.nt;
  const int64_t nt2 = (int64_t)nt * nt;
  const double nA2 = wave_sum(P.norm_part, nt);
  double l2S = -log2(nA2);
  for (int lev = 1; lev <= IN - 1; lev++) {
    const double tr = wave_sum(P.diag_part + lev * nt, nt);
    const double nb = wave_sum_upper(P.lvl_part + lev * nt2, nt);
    if (l == 0) lm[lev - 1] = l2S + log2(tr) - log2((double)P.h);
    if (lev == IN - 1 && l == 0) lm[IN - 1] = 2.0 * l2S + log2(nb) - log2((double)P.h);
    const double r = (nb > 0.0 && isfinite(nb)) ? rint(log2(nb)) : 0.0;
    l2S = 2.0 * l2S + r;
  }
  __syncthreads();
  if (l < IN) s.phi[l] = (float)(lm[l] / (8.0 * exp2((double)l)));
  if (l == 0) ok = 1;
  __syncthreads();
  forward(th, s);
  if (l < OUT && !isfinite(s.c[l])) atomicAnd(&ok, 0);
  __syncthreads();
  if (l < kSlots) {
    double cv = fixed_slots[l];
    if (ok && l < OUT) cv = (double)s.c[l];
    else if (ok) cv = 0.0;
    P.coef[l] = cv;
  }
  if (P.stats) {
    if (l == 0) P.stats[0] = nA2;
    if (l < IN) P.stats[1 + l] = lm[l];
    if (l < kMaxTerms) P.stats[9 + l] = l < kSlots ? (ok && l < OUT ? (double)s.c[l] : (ok ? 0.0 : fixed_slots[l])) : 0.0;
    if (l == 0) P.stats[25] = ok ? 1.0 : 0.0;
  }
}

}  // namespace mlp

hipError_t launch_mlp_features(int n, const float *sig, const int32_t *nsig, int smax, float *feats, hipStream_t s) {
  hipLaunchKernelGGL(mlp::k_features, dim3(n), dim3(64), 0, s, sig, nsig, smax, feats);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(int n, const float *feats, const float *params, double *coeffs, hipStream_t s) {
  hipLaunchKernelGGL(mlp::k_forward, dim3(n), dim3(64), 0, s, feats, params, coeffs);
  return hipGetLastError();
}

hipError_t launch_mlp_train(int n, const float *feats, const float *sig, const int32_t *nsig, int smax, float *params,
                            float *m, float *v, int t, float lr, float b1, float b2, float eps, float *gout,
                            float *lout, float *grads, float *losses, hipStream_t s) {
  hipLaunchKernelGGL(mlp::k_train, dim3(n), dim3(64), 0, s, feats, sig, nsig, smax, params, grads, losses);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp::k_adam, dim3((mlp::NP + 255) / 256), dim3(256), 0, s, n, grads, losses, params, m, v, t, lr,
                     b1, b2, eps, gout, lout);
  return hipGetLastError();
}

hipError_t launch_learned(const StageArgs &a, int nprob, const float *params, const double *fixed_slots,
                          hipStream_t s) {
  hipLaunchKernelGGL(mlp::k_learned, dim3(nprob), dim3(64), 0, s, a, params, fixed_slots);
  return hipGetLastError();
}

}  // namespace ifnso
