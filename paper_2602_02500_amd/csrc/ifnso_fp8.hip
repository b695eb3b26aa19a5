// Memory-bound passes of the e4m3 compute mode: per-tensor amax and sum of squares of the
// input, quantisation of A (transposed for tall inputs) to OCP e4m3 with a power-of-two scale,
// and the largest row sum of squares of a quantised operand, from which the scale of the next
// power follows. The e4m3 Gram and squaring GEMMs live with the other 256 x 256 kernels; their
// epilogues quantise each power as they store it.
//
// Scale rule: s = 2^e with e = floor(log2(448 / amax)) (448 is e4m3's largest finite value),
// so the scaled maximum lies in (224, 448] and the scaling itself is exact; e is clamped to
// [-63, 63] so that 1 / s^2 stays a normal float. Conversion: v_cvt_pk_fp8_f32, round to
// nearest even.
//
// These kernels take problems from blockIdx.y (one problem per grid row) and stride over the
// problem's work with blockIdx.x, so they need no task list.
#include <hip/hip_runtime.h>
#include <math.h>

#include "ifnso_common.hpp"
#include "ifnso_launch.hpp"
#include "ifnso_tile.hpp"

namespace ifnso {
namespace e4m3 {

__device__ __forceinline__ const ProbDev &problem(const StageArgs &a) { return a.probs ? a.probs[blockIdx.y] : a.one; }

__device__ __forceinline__ float scale_from_amax(float amax) { return ldexpf(1.f, e4m3_scale_exp(amax)); }

// four floats -> four e4m3 bytes, first value in the lowest byte
__device__ __forceinline__ uint32_t pack4(float a, float b, float c, float d) {
  int v = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  v = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, v, true);
  return (uint32_t)v;
}

__device__ __forceinline__ uint4 pack16(const float (&x)[16], float s) {
  return make_uint4(pack4(s * x[0], s * x[1], s * x[2], s * x[3]), pack4(s * x[4], s * x[5], s * x[6], s * x[7]),
                    pack4(s * x[8], s * x[9], s * x[10], s * x[11]),
                    pack4(s * x[12], s * x[13], s * x[14], s * x[15]));
}

// sum of squares of the four e4m3 values in a word (exact: each square has 8 significant bits)
__device__ __forceinline__ double sumsq_e4m3(uint32_t w) {
  const double x0 = __builtin_amdgcn_cvt_f32_fp8((int)w, 0), x1 = __builtin_amdgcn_cvt_f32_fp8((int)w, 1);
  const double x2 = __builtin_amdgcn_cvt_f32_fp8((int)w, 2), x3 = __builtin_amdgcn_cvt_f32_fp8((int)w, 3);
  return fma(x3, x3, fma(x2, x2, fma(x1, x1, x0 * x0)));
}

__device__ __forceinline__ void unpack8(const uint4 &v, float *x) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int i = 0; i < 4; i++) {
    x[2 * i] = __uint_as_float(w[i] << 16);
    x[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
  }
}

__device__ __forceinline__ float block_max(float v, float *scratch) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
  __syncthreads();
  v = fmaxf(fmaxf(scratch[0], scratch[1]), fmaxf(scratch[2], scratch[3]));
  __syncthreads();
  return v;
}

// ---------------------------------------------------------------------------------------------
// pre-pass: per chunk of rq storage rows of M, the float64 sum of squares and max |value|
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_prepass(const StageArgs a) {
  __shared__ double dscr[12];
  __shared__ float fscr[4];
  const ProbDev &P = problem(a);
  const int rows = P.trans ? P.w : P.h, cols = P.trans ? P.h : P.w;
  const uint16_t *M = (const uint16_t *)P.M;
  const bool vec = P.vecM && (cols % 8) == 0;
  for (int c = blockIdx.x; c < P.nq; c += gridDim.x) {
    const int r0 = c * P.rq, r1 = min(rows, r0 + P.rq);
    double ss = 0.0;
    float mx = 0.f;
    if (vec) {
      // 8-element groups, kThreads apart in row-major order; each thread keeps the (row, group)
      // of its kU slots and advances them without a division, and issues the kU 16-byte loads
      // of an iteration before using them
      constexpr int kU = 4;
      const int gpr = cols / 8;  // 8-element groups per row
      const int ng = (r1 - r0) * gpr;  // below kQElems / 8 + cols / 8
      const int dr = kU * kThreads / gpr, dk = kU * kThreads % gpr;
      int rr[kU], kk[kU];
      rr[0] = r0 + (int)threadIdx.x / gpr;
      kk[0] = (int)threadIdx.x % gpr;
#pragma unroll
      for (int u = 1; u < kU; u++) {
        rr[u] = rr[u - 1] + kThreads / gpr;
        kk[u] = kk[u - 1] + kThreads % gpr;
        if (kk[u] >= gpr) {
          kk[u] -= gpr;
          rr[u]++;
        }
      }
      for (int g = threadIdx.x; g < ng; g += kU * kThreads) {
        uint4 v[kU];
#pragma unroll
        for (int u = 0; u < kU; u++)
          v[u] = g + u * kThreads < ng ? *(const uint4 *)(M + (int64_t)rr[u] * P.ldm + kk[u] * 8) : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int u = 0; u < kU; u++) {
          float x[8];
          unpack8(v[u], x);
          float s8 = 0.f;  // squares of bfloat16 values are exact in float32
#pragma unroll
          for (int i = 0; i < 8; i++) {
            s8 = fmaf(x[i], x[i], s8);
            mx = fmaxf(mx, fabsf(x[i]));
          }
          ss += (double)s8;
          rr[u] += dr;
          kk[u] += dk;
          if (kk[u] >= gpr) {
            kk[u] -= gpr;
            rr[u]++;
          }
        }
      }
    } else {
      const int64_t n = (int64_t)(r1 - r0) * cols;
      for (int64_t e = threadIdx.x; e < n; e += kThreads) {
        const int r = r0 + (int)(e / cols), k = (int)(e % cols);
        const float x = bf16_to_f32(M[(int64_t)r * P.ldm + k]);
        ss = fma((double)x, (double)x, ss);
        mx = fmaxf(mx, fabsf(x));
      }
    }
    double u0 = 0.0, u1 = 0.0;
    block_sum3(ss, u0, u1, dscr);
    mx = block_max(mx, fscr);
    if (threadIdx.x == 0) {
      P.q_part[c] = ss;
      P.q_amax[c] = mx;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// quantise A: q8[i][k] = e4m3(s A[i][k]) for k < w, 0 for w <= k < ldq (A = M, or M^T when tall).
// Block 0 of each problem also stores ||A||_F^2 (fixed-order sum of the chunk partials) in
// norm_part[0] (zeros in the other slots), the scale and the maximum.
// ---------------------------------------------------------------------------------------------
constexpr int kTile = 64;

__global__ __launch_bounds__(kThreads) void k_quant_input(const StageArgs a) {
  __shared__ float fscr[4];
  __shared__ double dscr[12];
  __shared__ uint16_t tile[kTile][kTile + 2];
  const ProbDev &P = problem(a);
  float mx = 0.f;
  for (int i = threadIdx.x; i < P.nq; i += kThreads) mx = fmaxf(mx, P.q_amax[i]);
  mx = block_max(mx, fscr);
  const float s = scale_from_amax(mx);
  if (blockIdx.x == 0) {
    if (threadIdx.x < 64) {
      const double t = wave_sum(P.q_part, P.nq);
      if (threadIdx.x == 0) {
        P.norm_part[0] = t;
        P.q_scale[0] = s;
        P.q_scale[1] = mx;
      }
    }
    for (int i = 1 + threadIdx.x; i < P.nt; i += kThreads) P.norm_part[i] = 0.0;
    if (P.qrmax)  // the row maxima of this call start from zero
      for (int i = threadIdx.x; i <= kMaxLevels; i += kThreads) P.qrmax[i] = 0ull;
  }
  const uint16_t *M = (const uint16_t *)P.M;
  const int h = P.h, w = P.w;
  const int64_t ldq = P.ldq;
  const int gpr = (int)(ldq / 16);  // 16-element groups per row of q8
  if (!P.trans) {
    // one wave per chunk of 64 16-element groups (1024 columns of q8) of a row; the chunk's sum
    // of squares of the codes (exact in float64, summed over the wave in a fixed order) goes to
    // qrow_in when the plan keeps it. No barrier: each wave moves on by itself.
    const bool vec = P.vecM && (w % 8) == 0;
    const int nch = (gpr + 63) / 64;
    const int lane = threadIdx.x & 63;
    const int64_t units = (int64_t)h * nch, wstep = (int64_t)gridDim.x * (kThreads / 64);
    for (int64_t u = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); u < units; u += wstep) {
      const int i = (int)(u / nch), c = (int)(u - (int64_t)i * nch);
      const int g = c * 64 + lane, k = g * 16;
      double ss = 0.0;
      if (g < gpr) {
        const uint16_t *src = M + (int64_t)i * P.ldm + k;
        float x[16];
        if (vec) {
          const uint4 v0 = k < w ? *(const uint4 *)src : make_uint4(0, 0, 0, 0);
          const uint4 v1 = k + 8 < w ? *(const uint4 *)(src + 8) : make_uint4(0, 0, 0, 0);
          unpack8(v0, x);
          unpack8(v1, x + 8);
        } else {
#pragma unroll
          for (int j = 0; j < 16; j++) x[j] = k + j < w ? bf16_to_f32(src[j]) : 0.f;
        }
        const uint4 q = pack16(x, s);
        *(uint4 *)(P.q8 + (int64_t)i * ldq + k) = q;
        ss = sumsq_e4m3(q.x) + sumsq_e4m3(q.y) + sumsq_e4m3(q.z) + sumsq_e4m3(q.w);
      }
      if (P.qrow_in) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) ss += __shfl_xor(ss, off, 64);
        if (lane == 0) P.qrow_in[(int64_t)i * P.qnch + c] = ss;
      }
    }
    return;
  }
  // tall M (w x h storage): 64 x 64 tiles through LDS
  const bool vec = P.vecM && (h % 8) == 0;
  const int ti = (h + kTile - 1) / kTile, tk = (int)((ldq + kTile - 1) / kTile);
  for (int t = blockIdx.x; t < ti * tk; t += gridDim.x) {
    const int i0 = (t % ti) * kTile, k0 = (t / ti) * kTile;
    {
      const int kk = threadIdx.x >> 2, ii = (threadIdx.x & 3) * 16;
      const int k = k0 + kk;
      const uint16_t *src = M + (int64_t)k * P.ldm + i0 + ii;
      if (vec && k < w && i0 + ii + 16 <= h) {
        const uint4 v0 = *(const uint4 *)src, v1 = *(const uint4 *)(src + 8);
        const uint16_t *e0 = (const uint16_t *)&v0, *e1 = (const uint16_t *)&v1;
#pragma unroll
        for (int j = 0; j < 8; j++) {
          tile[kk][ii + j] = e0[j];
          tile[kk][ii + 8 + j] = e1[j];
        }
      } else {
#pragma unroll
        for (int j = 0; j < 16; j++) tile[kk][ii + j] = (k < w && i0 + ii + j < h) ? src[j] : (uint16_t)0;
      }
    }
    __syncthreads();
    {
      // row i0 + ii, 16 of the tile's 64 columns per thread; the four threads of a row (a lane
      // quad) add their sums of squares of the codes for qrow_in
      const int ii = threadIdx.x >> 2, kq = (threadIdx.x & 3) * 16;
      double ss = 0.0;
      if (i0 + ii < h && k0 + kq < ldq) {
        float x[16];
#pragma unroll
        for (int j = 0; j < 16; j++) x[j] = bf16_to_f32(tile[kq + j][ii]);
        const uint4 q = pack16(x, s);
        *(uint4 *)(P.q8 + (int64_t)(i0 + ii) * ldq + k0 + kq) = q;
        ss = sumsq_e4m3(q.x) + sumsq_e4m3(q.y) + sumsq_e4m3(q.z) + sumsq_e4m3(q.w);
      }
      ss += __shfl_xor(ss, 1, 64);
      ss += __shfl_xor(ss, 2, 64);
      if (P.qrow_in && (threadIdx.x & 3) == 0 && i0 + ii < h) P.qrow_in[(int64_t)(i0 + ii) * P.qnch + k0 / kTile] = ss;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// largest row sum of squares of an e4m3 operand (its codes): of level a.level's copy (hp x hp;
// a wave takes four rows at a time, 16 bytes per lane, with float64 partials summed over the wave
// in a fixed order) or, for level 0, of A (from the chunk sums the quantisation wrote); the
// workgroup's maximum goes into qrmax[a.level] as an atomic maximum of the float64 bit pattern
// (every value is >= 0, so the patterns order as the values and the result does not depend on
// the order of the updates).
// ---------------------------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_row_max(const StageArgs a) {
  __shared__ double wmax[kThreads / 64];
  const ProbDev &P = problem(a);
  const int l = a.level;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double mx = 0.0;
  if (l == 0) {  // A: the rows' chunk sums from the input quantisation, added in chunk order
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < P.h; i += gridDim.x * kThreads) {
      double s = 0.0;
      for (int c = 0; c < P.qnch; c++) s += P.qrow_in[(int64_t)i * P.qnch + c];
      mx = fmax(mx, s);
    }
  }
  const uint8_t *q = P.ql[l & 1];
  const int rows = l == 0 ? 0 : P.hp;
  const int64_t ld = P.hp;  // a multiple of 16 bytes
  for (int r0 = blockIdx.x * kQRowsPerBlock; r0 < rows; r0 += gridDim.x * kQRowsPerBlock) {
    const int r1 = min(rows, r0 + kQRowsPerBlock);
    // kR rows per wave pass: their loads are issued together and their wave sums interleave
    constexpr int kR = 4;
    for (int r = r0 + wave * kR; r < r1; r += (kThreads / 64) * kR) {
      double s[kR];
#pragma unroll
      for (int j = 0; j < kR; j++) s[j] = 0.0;
      for (int64_t k = (int64_t)lane * 16; k < ld; k += 64 * 16) {
        uint4 v[kR];
#pragma unroll
        for (int j = 0; j < kR; j++)
          v[j] = r + j < r1 ? *(const uint4 *)(q + (int64_t)(r + j) * ld + k) : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < kR; j++)
          s[j] += sumsq_e4m3(v[j].x) + sumsq_e4m3(v[j].y) + sumsq_e4m3(v[j].z) + sumsq_e4m3(v[j].w);
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
        for (int j = 0; j < kR; j++) s[j] += __shfl_xor(s[j], off, 64);
#pragma unroll
      for (int j = 0; j < kR; j++) mx = fmax(mx, s[j]);  // rows past r1 add zero sums
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));  // level 0: per-thread rows
  if (lane == 0) wmax[wave] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kThreads / 64; w++) mx = fmax(mx, wmax[w]);
    atomicMax((unsigned long long *)(P.qrmax + l), (unsigned long long)__double_as_longlong(mx));
  }
}

__global__ void k_export(const ProbDev P, double *out) {
  if (threadIdx.x == 0) {
    out[0] = P.norm_part[0];
    out[1] = (double)P.q_scale[1];
    out[2] = (double)P.q_scale[0];
  }
}

}  // namespace e4m3

// Grid of a memory-bound e4m3 pass: `per_problem` workgroups for each of `nprob` problems.
hipError_t launch_e4m3_pass(int which, const StageArgs &a, int nprob, int per_problem, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  const dim3 grid(per_problem, nprob);
  if (which == kE4m3Prepass) hipLaunchKernelGGL(e4m3::k_prepass, grid, dim3(kThreads), 0, s, a);
  else if (which == kE4m3QuantInput) hipLaunchKernelGGL(e4m3::k_quant_input, grid, dim3(kThreads), 0, s, a);
  else hipLaunchKernelGGL(e4m3::k_row_max, grid, dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_e4m3_export(const ProbDev &P, double *out, hipStream_t s) {
  hipLaunchKernelGGL(e4m3::k_export, dim3(1), dim3(64), 0, s, P, out);
  return hipGetLastError();
}

}  // namespace ifnso
