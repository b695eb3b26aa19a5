// Muon optimizer step around a plan's batched orthogonalisation: the momentum update and the
// orthogonalisation input before it, the weight update after it. Memory-bound elementwise
// passes: one grid row per problem, four consecutive columns per thread when every row is
// 16-byte aligned, one element otherwise.
#include <hip/hip_runtime.h>

#include "ifnso_common.hpp"
#include "ifnso_launch.hpp"
#include "ifnso_tile.hpp"

namespace ifnso {
namespace muon {

__device__ __forceinline__ float ld_in(const void *p, int64_t i, bool bf16) {
  return bf16 ? bf16_to_f32(((const uint16_t *)p)[i]) : ((const float *)p)[i];
}

__device__ __forceinline__ void st_in(void *p, int64_t i, float v, bool bf16) {
  if (bf16) ((uint16_t *)p)[i] = f32_to_bf16(v);
  else ((float *)p)[i] = v;
}

__device__ __forceinline__ float4 ld4_in(const void *p, int64_t i, bool bf16) {
  if (bf16) {
    const uint2 q = *(const uint2 *)((const uint16_t *)p + i);
    return make_float4(__uint_as_float(q.x << 16), __uint_as_float(q.x & 0xffff0000u), __uint_as_float(q.y << 16),
                       __uint_as_float(q.y & 0xffff0000u));
  }
  return *(const float4 *)((const float *)p + i);
}

__device__ __forceinline__ void st4_in(void *p, int64_t i, float4 v, bool bf16) {
  if (bf16) {
    *(uint2 *)((uint16_t *)p + i) = make_uint2((uint32_t)f32_to_bf16(v.x) | ((uint32_t)f32_to_bf16(v.y) << 16),
                                               (uint32_t)f32_to_bf16(v.z) | ((uint32_t)f32_to_bf16(v.w) << 16));
  } else {
    *(float4 *)((float *)p + i) = v;
  }
}

// per element: b' = mu b + g (float32); u = nesterov ? g + mu b' : b'
__device__ __forceinline__ float momentum1(float g, float &b, float mu, bool nesterov) {
  b = mu * b + g;
  return nesterov ? g + mu * b : b;
}

__global__ __launch_bounds__(kThreads) void k_muon_pre(const MuonArgs a) {
  const MuonProb &P = a.probs[blockIdx.y];
  const bool ib = a.in_bf16 != 0, nv = a.nesterov != 0;
  const float mu = a.momentum;
  if (P.vec) {
    const int64_t cq = P.cols / 4, n = P.rows * cq;
    for (int64_t q = blockIdx.x * (int64_t)kThreads + threadIdx.x; q < n; q += (int64_t)gridDim.x * kThreads) {
      const int64_t r = q / cq, c = (q - r * cq) * 4;
      const float4 g = ld4_in(P.G, r * P.ldg + c, ib);
      float4 b = *(const float4 *)(P.B + r * P.ldb + c);
      float4 u;
      u.x = momentum1(g.x, b.x, mu, nv);
      u.y = momentum1(g.y, b.y, mu, nv);
      u.z = momentum1(g.z, b.z, mu, nv);
      u.w = momentum1(g.w, b.w, mu, nv);
      *(float4 *)(P.B + r * P.ldb + c) = b;
      st4_in(P.U, r * P.ldu + c, u, ib);
    }
  } else {
    const int64_t n = P.rows * P.cols;
    for (int64_t q = blockIdx.x * (int64_t)kThreads + threadIdx.x; q < n; q += (int64_t)gridDim.x * kThreads) {
      const int64_t r = q / P.cols, c = q - r * P.cols;
      float b = P.B[r * P.ldb + c];
      const float u = momentum1(ld_in(P.G, r * P.ldg + c, ib), b, mu, nv);
      P.B[r * P.ldb + c] = b;
      st_in(P.U, r * P.ldu + c, u, ib);
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_muon_post(const MuonArgs a) {
  const MuonProb &P = a.probs[blockIdx.y];
  const bool ob = a.out_bf16 != 0;
  const float dec = a.decay, st = P.step;
  if (P.vec) {
    const int64_t cq = P.cols / 4, n = P.rows * cq;
    for (int64_t q = blockIdx.x * (int64_t)kThreads + threadIdx.x; q < n; q += (int64_t)gridDim.x * kThreads) {
      const int64_t r = q / cq, c = (q - r * cq) * 4;
      const float4 y = ld4_in(P.Y, r * P.ldy + c, ob);
      float4 w = *(const float4 *)(P.W + r * P.ldw + c);
      w = make_float4(dec * w.x - st * y.x, dec * w.y - st * y.y, dec * w.z - st * y.z, dec * w.w - st * y.w);
      *(float4 *)(P.W + r * P.ldw + c) = w;
    }
  } else {
    const int64_t n = P.rows * P.cols;
    for (int64_t q = blockIdx.x * (int64_t)kThreads + threadIdx.x; q < n; q += (int64_t)gridDim.x * kThreads) {
      const int64_t r = q / P.cols, c = q - r * P.cols;
      float &w = P.W[r * P.ldw + c];
      w = dec * w - st * ld_in(P.Y, r * P.ldy + c, ob);
    }
  }
}

}  // namespace muon

hipError_t launch_muon_pre(const MuonArgs &a, int nprob, int per_problem, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  hipLaunchKernelGGL(muon::k_muon_pre, dim3(per_problem, nprob), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_muon_post(const MuonArgs &a, int nprob, int per_problem, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  hipLaunchKernelGGL(muon::k_muon_post, dim3(per_problem, nprob), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace ifnso
