// Stage kernels of libifnso for gfx950.
//
// A plan runs, for every problem, the stages of the polynomial (Algorithm 1 of the
// paper, in the Gram or the complement basis):
//   Gram      G_raw = A A^T on upper tiles; fused float64 partials of ||A||_F^2 (diagonal
//             tiles, from the staged operand registers), of ||G_raw||_F^2 and of tr(G_raw).
//   square j  level j+1 = (level j)^2 on upper tiles, written back as a full symmetric
//             operand; the running sum P accumulates c * level in float32.
//   product   Y = s (c0 A + P A), written in M's orientation and dtype.
// Each stage is one persistent launch over a task list that holds the tiles of every
// problem; scalars (norms, level scales, coefficients) are recomputed by each workgroup
// from the float64 partials of earlier stages, in a fixed order, so results do not depend
// on scheduling.
//
// Level scaling (Gram basis): the stored operand of level l is B_l with true value
// S_l * B_l. Level 1 stores G_raw, S_1 = s_g (1/||A||_F^2, 1/||G_raw||_F or 1 by norm).
// Squaring stores B_{l+1} = F_{l+1} * B_l^2 with F_{l+1} = 2^-round(log2 ||B_l||_F^2), so
// every stored level keeps unit-order entries even when the true power underflows float32;
// S_{l+1} = S_l^2 / F_{l+1}. Complement basis: levels hold D_l = T_1^(2^(l-1)) - I with
// D_1 = -s_g G_raw and D_{l+1} = 2 D_l + D_l^2 (the shifted form keeps small 1 - T
// entries exact), and the identity parts are folded into the coefficient of X.
#include <hip/hip_runtime.h>
#include <math.h>

#include "ifnso_common.hpp"
#include "ifnso_launch.hpp"
#include "ifnso_tile.hpp"

namespace ifnso {

// ---------------------------------------------------------------------------------------------
// per-problem scalars from the float64 partials
// ---------------------------------------------------------------------------------------------
struct Scalars {
  double nA2;   // ||A||_F^2
  double g2;    // ||G_raw||_F^2
  double sg;    // scale of the level-1 operand (G = sg * G_raw)
  double sout;  // output scale s
  bool zero;
};

__device__ __forceinline__ Scalars problem_scalars(const ProbDev &P, int norm) {
  Scalars s;
  s.nA2 = wave_sum(P.norm_part, P.nt);
  s.g2 = wave_sum_upper(P.lvl_part + (int64_t)1 * P.nt * P.nt, P.nt);
  s.zero = !(s.nA2 > 0.0);
  if (norm == kFrob) {
    s.sg = s.zero ? 0.0 : 1.0 / s.nA2;
    s.sout = s.zero ? 0.0 : 1.0 / sqrt(s.nA2);
  } else if (norm == kGramFrob) {
    const double o = sqrt(s.g2);
    s.sg = s.zero ? 0.0 : 1.0 / o;
    s.sout = s.zero ? 0.0 : 1.0 / sqrt(o);
  } else if (norm == kGelfand2) {
    // s^2 = ||G_raw^2||_F^(1/2); slot 2 holds the partials of ||G_raw^2||_F^2
    const double o = sqrt(sqrt(wave_sum_upper(P.lvl_part + (int64_t)2 * P.nt * P.nt, P.nt)));
    s.sg = s.zero ? 0.0 : 1.0 / o;
    s.sout = s.zero ? 0.0 : 1.0 / sqrt(o);
  } else {
    s.sg = 1.0;
    s.sout = 1.0;
  }
  return s;
}

__device__ __forceinline__ double pow2_inv_round(double nb) {
  if (!(nb > 0.0) || !isfinite(nb)) return 1.0;
  return exp2(-rint(log2(nb)));
}

// Gram basis: scale S_level of the stored operand of `level` (level >= 1).
__device__ __forceinline__ double level_scale(const ProbDev &P, double sg, int level) {
  double S = sg;
  const int64_t nt2 = (int64_t)P.nt * P.nt;
  for (int l = 1; l < level; l++) {
    const double F = pow2_inv_round(wave_sum_upper(P.lvl_part + l * nt2, P.nt));
    S = S * S / F;
  }
  return S;
}

// ---------------------------------------------------------------------------------------------
// task fetch: a device task list (grouped launches) or tiles decoded from the index
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ Task decode_upper(int t, int nt) {
  int tm = 0;
  while (t >= nt - tm) {
    t -= nt - tm;
    tm++;
  }
  return Task{0, tm, tm + t, 0};
}

template <int TS>
__device__ __forceinline__ Task fetch_task(const StageArgs &a, int t, int stage) {
  if (a.tasks) return a.tasks[t];
  const ProbDev &P = a.one;
  if (stage != kStageProduct) return decode_upper(t, P.nt);
  const bool tall_map = (a.ns_step <= 0) && P.trans;
  const int ncols = ((tall_map ? P.h : P.w) + TS - 1) / TS;
  return Task{0, t / ncols, t % ncols, 0};
}

__device__ __forceinline__ const ProbDev &prob_of(const StageArgs &a, const Task &task) {
  return a.tasks ? a.probs[task.p] : a.one;
}

// ---------------------------------------------------------------------------------------------
// epilogue helpers: the accumulator tile staged in LDS, four consecutive elements stored at once
// ---------------------------------------------------------------------------------------------
template <typename TL, int TS>
__device__ __forceinline__ void stage_tile(const TL &tile, float *ep) {  // ep: TS x TS, row-major
#pragma unroll
  for (int fm = 0; fm < TL::FM; fm++)
#pragma unroll
    for (int fn = 0; fn < TL::FN; fn++)
#pragma unroll
      for (int r = 0; r < 16; r++) ep[TL::row_of(fm, r) * TS + TL::col_of(fn)] = tile.acc[fm][fn][r];
}

template <typename T>
__device__ __forceinline__ void store4(T *p, float4 v);
template <>
__device__ __forceinline__ void store4<float>(float *p, float4 v) {
  *(float4 *)p = v;
}
template <>
__device__ __forceinline__ void store4<uint16_t>(uint16_t *p, float4 v) {
  *(uint2 *)p = make_uint2((uint32_t)f32_to_bf16(v.x) | ((uint32_t)f32_to_bf16(v.y) << 16),
                           (uint32_t)f32_to_bf16(v.z) | ((uint32_t)f32_to_bf16(v.w) << 16));
}

// ---------------------------------------------------------------------------------------------
// Gram
// ---------------------------------------------------------------------------------------------
// float32 (the Gram, squaring and product kernels): two workgroups per CU. The float32 matrix
// instruction is slow enough that one workgroup's loads and epilogue hide behind the other's
// MFMAs; the register cap makes the compiler spill (the Gram also inside its K loops), which
// costs less than the overlap gains.
template <typename T, int TS>
__global__ __launch_bounds__(kThreads, sizeof(T) == 4 ? 2 : 1) void k_gram(const StageArgs a) {
  using TL = Tile<T, TS, TS>;
  __shared__ __attribute__((aligned(16))) char smem[TL::LDS_BYTES];
  __shared__ int s_last;
  // Split K (single-problem launches with few tiles): task t is chunk t % S of tile t / S. Each
  // chunk stores its partial tile; the last chunk of a tile to finish sums the S partials in
  // chunk order (so the result does not depend on which one finishes last) and runs the epilogue.
  const int S = a.ksplit > 1 ? a.ksplit : 1;
  for (int t = blockIdx.x; t < a.ntasks * S; t += gridDim.x) {
    const int tt = t / S, chunk = t % S;
    const Task task = fetch_task<TS>(a, tt, kStageGram);
    const ProbDev &P = prob_of(a, task);
    const int m0 = task.tm * TS, n0 = task.tn * TS;
    const bool diag = task.tm == task.tn;
    const bool first_step = a.ns_step <= 0;
    // a tile of the padding beyond h is zero: its first chunk writes it without partials
    const bool pad = m0 >= P.h || n0 >= P.h;
    if (pad && chunk != 0) continue;  // uniform over the workgroup
    const int k0 = S > 1 ? chunk * a.kchunk : 0;
    const int klen = S > 1 ? min(a.kchunk, P.w - k0) : P.w;
    TL tile;
    double nrm = 0.0;
    if (pad) {
      tile.zero();
    } else if (!first_step) {  // classical NS, later steps: X_k (wide, K-major) from the workspace
      const T *X = (const T *)P.xbuf[(a.ns_step - 1) & 1] + k0;
      nrm = tile.template run<false, false>(smem, X, P.ldx, m0, P.h, true, X, P.ldx, n0, P.h, true, klen, false);
    } else if (P.trans) {
      const T *M = (const T *)P.M + (int64_t)k0 * P.ldm;
      nrm = tile.template run<true, true>(smem, M, P.ldm, m0, P.h, P.vecM, M, P.ldm, n0, P.h, P.vecM, klen, diag);
    } else {
      const T *M = (const T *)P.M + k0;
      nrm = tile.template run<false, false>(smem, M, P.ldm, m0, P.h, P.vecM, M, P.ldm, n0, P.h, P.vecM, klen, diag);
    }
    T *op = (T *)P.opnd[0];
    const int64_t hp = P.hp;
    const bool keep_f32 = (a.J >= 1 && !a.agg) || a.ns_step >= 0 || a.learned;
    double lv = 0.0, dg = 0.0;
    // epilogue through LDS, as in the squaring: row chunks, then the mirrored block
    float *ep = (float *)smem;
    __syncthreads();
    if (S > 1 && !pad) {
      float *part = P.gpart + ((int64_t)tt * S + chunk) * (TS * TS);
#pragma unroll
      for (int fm = 0; fm < TL::FM; fm++)
#pragma unroll
        for (int fn = 0; fn < TL::FN; fn++)
#pragma unroll
          for (int r = 0; r < 16; r++) part[TL::row_of(fm, r) * TS + TL::col_of(fn)] = tile.acc[fm][fn][r];
      P.gnrm[((int64_t)tt * S + chunk) * kThreads + threadIdx.x] = nrm;
      __threadfence();
      __syncthreads();
      if (threadIdx.x == 0) s_last = atomicAdd(P.gcnt + tt, 1u) == (uint32_t)(S - 1);
      __syncthreads();
      if (!s_last) continue;  // the same for the whole workgroup
      __threadfence();
      const float *base = P.gpart + (int64_t)tt * S * (TS * TS);
      for (int q = threadIdx.x; q < TS * TS / 4; q += kThreads) {
        float4 v = *(const float4 *)(base + q * 4);
        for (int c = 1; c < S; c++) {
          const float4 w4 = *(const float4 *)(base + (int64_t)c * (TS * TS) + q * 4);
          v = make_float4(v.x + w4.x, v.y + w4.y, v.z + w4.z, v.w + w4.w);
        }
        *(float4 *)(ep + q * 4) = v;
      }
      nrm = 0.0;
      for (int c = 0; c < S; c++) nrm += P.gnrm[((int64_t)tt * S + c) * kThreads + threadIdx.x];
      if (threadIdx.x == 0) P.gcnt[tt] = 0u;  // ready for the next launch
    } else {
      stage_tile<TL, TS>(tile, ep);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < TS * TS / 4; q += kThreads) {
      const int row = q / (TS / 4), c4 = (q % (TS / 4)) * 4;
      const int i = m0 + row, j = n0 + c4;
      const int64_t ij = (int64_t)i * hp + j;
      const float4 v = *(const float4 *)(ep + row * TS + c4);
      store4<T>(op + ij, v);
      // both triangles: the 256-tile squaring kernels read whole diagonal 256 blocks
      if (keep_f32) *(float4 *)(P.accf + ij) = v;
      const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const double dv = (double)vv[e];
        lv = fma(dv, diag ? dv : 2.0 * dv, lv);
        if (i == j + e) dg += dv;
      }
    }
    if (!diag) {
      for (int q = threadIdx.x; q < TS * TS / 4; q += kThreads) {
        const int row = q / (TS / 4), c4 = (q % (TS / 4)) * 4;
        const int64_t ji = (int64_t)(n0 + row) * hp + m0 + c4;
        const float4 v = make_float4(ep[(c4 + 0) * TS + row], ep[(c4 + 1) * TS + row], ep[(c4 + 2) * TS + row],
                                     ep[(c4 + 3) * TS + row]);
        store4<T>(op + ji, v);
        if (keep_f32) *(float4 *)(P.accf + ji) = v;
      }
    }
    if (!diag || !first_step) nrm = 0.0;
    block_sum3(lv, dg, nrm, (double *)smem);
    if (threadIdx.x == 0) {
      const int nt = P.nt;
      P.lvl_part[(int64_t)1 * nt * nt + task.tm * nt + task.tn] = lv;
      if (diag) {
        P.diag_part[1 * nt + task.tm] = dg;
        if (first_step) P.norm_part[task.tm] = nrm;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// squaring: level -> level + 1
// ---------------------------------------------------------------------------------------------
template <typename T, int TS>
__global__ __launch_bounds__(kThreads, sizeof(T) == 4 ? 2 : 1) void k_square(const StageArgs a) {
  using TL = Tile<T, TS, TS>;
  __shared__ __attribute__((aligned(16))) char smem[TL::LDS_BYTES];
  const int level = a.level;
  int cur_p = -1;
  // per-problem factors (recomputed when the problem changes)
  float f_out = 1.f;    // stored next level = f_out * acc
  float c_acc = 0.f;    // P += c_acc * acc                 (Gram basis)
  float c_first = 0.f;  // level 1: P = c_first * G_raw + ...
  float alpha = 1.f;    // complement: D_next = 2 D + alpha * acc
  float c_next = 0.f;   // complement: P += c_next * D_next
  float dscale = 1.f;   // complement, level 1: D_1 = dscale * G_raw
  float ns_b = 0.f, ns_c = 0.f;
  for (int t = blockIdx.x; t < a.ntasks; t += gridDim.x) {
    const Task task = fetch_task<TS>(a, t, kStageSquare);
    const ProbDev &P = prob_of(a, task);
    if (task.p != cur_p) {
      cur_p = task.p;
      const Scalars sc = problem_scalars(P, a.norm);
      const int64_t nt2 = (int64_t)P.nt * P.nt;
      if (a.ns_step >= 0) {
        const double s = (a.ns_step == 0) ? sc.sg : 1.0;
        ns_b = (float)(a.ns_abc[1] * s);
        ns_c = (float)(a.ns_abc[2] * s * s);
      } else if (a.basis == kGram) {
        const double S = level_scale(P, sc.sg, level);
        f_out = (float)pow2_inv_round(wave_sum_upper(P.lvl_part + level * nt2, P.nt));
        c_acc = (float)(P.coef[level + 1] * S * S);
        c_first = (float)(P.coef[1] * sc.sg);
      } else {
        alpha = (float)(level == 1 ? sc.sg * sc.sg : 1.0);
        dscale = (float)(-sc.sg);
        c_next = (float)P.coef[level + 1];
        c_first = (float)P.coef[1];
      }
    }
    const int m0 = task.tm * TS, n0 = task.tn * TS;
    const bool diag = task.tm == task.tn;
    const int64_t hp = P.hp;
    const T *src = (const T *)P.opnd[(level - 1) & 1];
    TL tile;
    if (m0 >= P.h || n0 >= P.h) tile.zero();  // a tile of the padding beyond h: zero
    else tile.template run<false, false>(smem, src, hp, m0, P.hp, true, src, hp, n0, P.hp, true, P.h, false);
    T *dst = (T *)P.opnd[level & 1];
    const bool last = a.last;
    double lv = 0.0, dg = 0.0, unused = 0.0;
    // The accumulator goes through LDS so that one short loop over float4 row chunks does the
    // epilogue (a per-register epilogue unrolled over the tile is long code that a one-tile
    // launch pays for in instruction fetch).
    float *ep = (float *)smem;
    __syncthreads();  // the mainloop's last LDS reads
    stage_tile<TL, TS>(tile, ep);
    __syncthreads();
    // float4 row chunks, four per thread at a time so that their global reads overlap
    constexpr int CHUNKS = TS * TS / 4 / kThreads, BATCH = 4;
    static_assert(CHUNKS % BATCH == 0, "epilogue batches");
    for (int b0 = 0; b0 < CHUNKS; b0 += BATCH) {
      float4 fin[BATCH], d4[BATCH];
      if (!a.ns_norm_pass) {
#pragma unroll
        for (int u = 0; u < BATCH; u++) {
          const int q = threadIdx.x + kThreads * (b0 + u);
          const int64_t ij = (int64_t)(m0 + q / (TS / 4)) * hp + n0 + (q % (TS / 4)) * 4;
          fin[u] = *(const float4 *)(P.accf + ij);
          if (a.ns_step < 0 && a.basis != kGram && level > 1) d4[u] = *(const float4 *)(P.df[level & 1] + ij);
        }
      }
#pragma unroll
      for (int u = 0; u < BATCH; u++) {
        const int q = threadIdx.x + kThreads * (b0 + u);
        const int row = q / (TS / 4), c4 = (q % (TS / 4)) * 4;
        const int i = m0 + row, j = n0 + c4;
        const int64_t ij = (int64_t)i * hp + j;
        const float4 accv = *(const float4 *)(ep + row * TS + c4);
        const float av[4] = {accv.x, accv.y, accv.z, accv.w};
        if (a.ns_norm_pass) {
          // Gelfand q = 2: the sum of squares of G_raw^2 only; nothing is stored
#pragma unroll
          for (int e = 0; e < 4; e++) {
            const double dv = (double)av[e];
            lv = fma(dv, diag ? dv : 2.0 * dv, lv);
          }
          continue;
        }
        const float fv[4] = {fin[u].x, fin[u].y, fin[u].z, fin[u].w};
        const bool cdf = a.ns_step < 0 && a.basis != kGram && level > 1;
        const float dp[4] = {cdf ? d4[u].x : 0.f, cdf ? d4[u].y : 0.f, cdf ? d4[u].z : 0.f, cdf ? d4[u].w : 0.f};
        float ov[4], pvv[4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
          float out, pv;
          if (a.ns_step >= 0) {
            // classical NS: B = b G + c G^2 (G = s G_raw at the first step)
            out = ns_b * fv[e] + ns_c * av[e];
            pv = out;
          } else if (a.basis == kGram) {
            out = f_out * av[e];
            pv = (level == 1 ? c_first * fv[e] : fv[e]) + c_acc * av[e];
          } else {
            const float dprev = (level == 1) ? dscale * fv[e] : dp[e];
            out = 2.f * dprev + alpha * av[e];
            pv = (level == 1 ? c_first * dprev : fv[e]) + c_next * out;
          }
          ov[e] = out;
          pvv[e] = pv;
          const double dv = (double)out;
          lv = fma(dv, diag ? dv : 2.0 * dv, lv);
          if (i == j + e) dg += dv;
        }
        if (a.ns_step < 0 && a.basis != kGram && !last)
          *(float4 *)(P.df[(level + 1) & 1] + ij) = make_float4(ov[0], ov[1], ov[2], ov[3]);
        if (!last) *(float4 *)(P.accf + ij) = make_float4(pvv[0], pvv[1], pvv[2], pvv[3]);
        const float4 sv = last ? make_float4(pvv[0], pvv[1], pvv[2], pvv[3]) : make_float4(ov[0], ov[1], ov[2], ov[3]);
        store4<T>(dst + ij, sv);
        *(float4 *)(ep + row * TS + c4) = sv;  // the stored value, for the mirror
      }
    }
    if (!a.ns_norm_pass && !diag) {
      __syncthreads();
      // mirror: block (n0.., m0..) = transpose of the stored tile, written row-wise
      for (int q = threadIdx.x; q < TS * TS / 4; q += kThreads) {
        const int row = q / (TS / 4), c4 = (q % (TS / 4)) * 4;
        store4<T>(dst + (int64_t)(n0 + row) * hp + m0 + c4,
                  make_float4(ep[(c4 + 0) * TS + row], ep[(c4 + 1) * TS + row], ep[(c4 + 2) * TS + row],
                              ep[(c4 + 3) * TS + row]));
      }
    }
    block_sum3(lv, dg, unused, (double *)smem);
    if (threadIdx.x == 0 && (a.ns_step < 0 || a.ns_norm_pass)) {
      const int nt = P.nt;
      P.lvl_part[(int64_t)(level + 1) * nt * nt + task.tm * nt + task.tn] = lv;
      if (diag && !a.ns_norm_pass) P.diag_part[(level + 1) * nt + task.tm] = dg;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// product: Y = s (c0 X + P X), in M's orientation
// ---------------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ float load_el(const void *p, int64_t idx) {
  return Elem<T>::to_f(((const T *)p)[idx]);
}

template <typename T, int TS>
__global__ __launch_bounds__(kThreads, sizeof(T) == 4 ? 2 : 1) void k_product(const StageArgs a, const int out_bf16) {
  using TL = Tile<T, TS, TS>;
  __shared__ __attribute__((aligned(16))) char smem[TL::LDS_BYTES];
  int cur_p = -1;
  float sc0 = 0.f, sps = 0.f;
  for (int t = blockIdx.x; t < a.ntasks; t += gridDim.x) {
    const Task task = fetch_task<TS>(a, t, kStageProduct);
    const ProbDev &P = prob_of(a, task);
    if (task.p != cur_p) {
      cur_p = task.p;
      const Scalars sc = problem_scalars(P, a.norm);
      double c0, ps, sout;
      if (P.h == 1) {
        // A single row or column: G = x x^T / s^2 is a scalar known exactly from the float64
        // norm, so the polynomial (or the NS recursion) is evaluated in float64 here.
        const double g = (a.norm == kNone && a.ns_step < 0) ? sc.nA2 : 1.0;
        sout = sc.zero ? 0.0 : (a.norm == kNone && a.ns_step < 0 ? 1.0 : 1.0 / sqrt(sc.nA2));
        double v = 0.0;
        if (a.ns_step >= 0) {
          double x = 1.0;
          for (int k = 0; k < a.ns_steps; k++) {
            const double *c = a.ns_sched[k < a.ns_nsched ? k : a.ns_nsched - 1];
            x = x * (c[0] + x * x * (c[1] + c[2] * x * x));
          }
          v = x;
        } else {
          const double b = (a.basis == kGram) ? g : 1.0 - g;
          for (int k = 0; k < kSlots; k++) {
            const double e = k == 0 ? 0.0 : exp2((double)(k - 1));
            if (P.coef[k] != 0.0) v += P.coef[k] * pow(b, e);
          }
        }
        c0 = v;
        ps = 0.0;
      } else if (a.ns_step >= 0) {
        c0 = a.ns_abc[0];
        ps = 1.0;
        sout = (a.ns_step == 0) ? sc.sout : 1.0;
        if (a.ns_step == 0 && sc.zero) sout = 0.0;
      } else {
        sout = sc.sout;
        if (a.basis == kGram) {
          c0 = P.coef[0];
          ps = (a.J == 0 && !a.agg) ? P.coef[1] * sc.sg : 1.0;  // the aggregate stage folds c_1 S_1 into P
        } else {
          c0 = 0.0;
          for (int k = 0; k < kSlots; k++) c0 += P.coef[k];
          ps = (a.J == 0) ? -P.coef[1] * sc.sg : 1.0;
        }
        if (sc.zero && a.norm != kNone) sout = 0.0;
      }
      sc0 = (float)(sout * c0);
      sps = (float)(sout * ps);
    }
    const T *Pb = (const T *)(a.agg ? (const void *)((const char *)P.lv + (int64_t)a.p_slot * P.lv_stride)
                                    : P.opnd[a.J & 1]);
    const int64_t hp = P.hp;
    // geometry: source X_k, destination, orientation of the computed tile
    const bool ns = a.ns_step >= 0;
    const bool from_m = !ns || a.ns_step == 0;
    const T *X = from_m ? (const T *)P.M : (const T *)P.xbuf[(a.ns_step - 1) & 1];
    const int64_t ldx = from_m ? P.ldm : P.ldx;
    const bool xvec = from_m ? (P.vecM != 0) : true;
    const bool tall_map = from_m && P.trans;  // tile rows index w, cols index h
    const bool to_y = !ns || a.ns_last;
    void *dst = to_y ? P.Y : P.xbuf[a.ns_step & 1];
    const bool dst_bf16 = to_y ? (out_bf16 != 0) : (sizeof(T) == 2);
    // dst element for logical wide-orientation (i, n):
    //   to Y: trans ? Y[n][i] : Y[i][n];  to xbuf: xbuf[i][n]
    const int m0 = task.tm * TS, n0 = task.tn * TS;
    TL tile;
    if (a.p_empty || P.h == 1) {
      tile.zero();
    } else if (tall_map) {
      tile.template run<false, false>(smem, X, ldx, m0, P.w, xvec, Pb, hp, n0, P.hp, true, P.h, false);
    } else {
      tile.template run<false, true>(smem, Pb, hp, m0, P.hp, true, X, ldx, n0, P.w, xvec, P.h, false);
    }
    // Epilogue through LDS in float4 row chunks of the tile (tile row tr, column tc). X is read
    // along tc in both orientations; the destination runs along tc unless it is stored
    // transposed relative to the tile (then a second pass writes it from LDS column-wise).
    //   logical wide-orientation element (i, n): tall_map ? (tc, tr) : (tr, tc)
    //   destination: to Y, trans ? Y[n][i] : Y[i][n];  to xbuf, xbuf[i][n]
    const bool dst_t = to_y ? (P.trans && !tall_map) : tall_map;
    const int64_t ldd = to_y ? P.ldy : P.ldx;
    float *ep = (float *)smem;
    __syncthreads();
    stage_tile<TL, TS>(tile, ep);
    __syncthreads();
    for (int q = threadIdx.x; q < TS * TS / 4; q += kThreads) {
      const int row = q / (TS / 4), c4 = (q % (TS / 4)) * 4;
      const int tr = m0 + row;
      float yv[4];
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const int tc = n0 + c4 + e;
        const int i = tall_map ? tc : tr, n = tall_map ? tr : tc;
        yv[e] = 0.f;
        if (i < P.h && n < P.w) {
          const float x = load_el<T>(X, (int64_t)tr * ldx + tc);
          yv[e] = sc0 * x + sps * ep[row * TS + c4 + e];
          if (!dst_t) {
            const int64_t didx = (int64_t)tr * ldd + tc;
            if (dst_bf16) ((uint16_t *)dst)[didx] = f32_to_bf16(yv[e]);
            else ((float *)dst)[didx] = yv[e];
          }
        }
      }
      if (dst_t) *(float4 *)(ep + row * TS + c4) = make_float4(yv[0], yv[1], yv[2], yv[3]);
    }
    if (dst_t) {
      __syncthreads();
      // destination row = tile column tc, running along tile rows tr
      for (int q = threadIdx.x; q < TS * TS / 4; q += kThreads) {
        const int col = q / (TS / 4), r4 = (q % (TS / 4)) * 4;
        const int tc = n0 + col;
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int tr = m0 + r4 + e;
          const int i = tall_map ? tc : tr, n = tall_map ? tr : tc;
          if (i < P.h && n < P.w) {
            const float y = ep[(r4 + e) * TS + col];
            const int64_t didx = (int64_t)tc * ldd + tr;
            if (dst_bf16) ((uint16_t *)dst)[didx] = f32_to_bf16(y);
            else ((float *)dst)[didx] = y;
          }
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// float64 orthogonality error ||Z Z^T - I||_F (evaluation only)
// ---------------------------------------------------------------------------------------------
// Matrix-core form: a workgroup of 4 waves owns a 64 x 64 tile of Z Z^T (upper tiles only, the
// off-diagonal ones counted twice); each wave a 32 x 32 quarter as 2 x 2 tiles of
// v_mfma_f64_16x16x4_f64. Z is staged through LDS as float64, 32 K per stage. Lane layout of the
// f64 16x16x4 instruction (measured with an in-bounds probe): A[i][k] = lane (i + 16 k), B[k][j] =
// lane (j + 16 k), and D[i][j] in lane j + 16 (i % 4), element i / 4.
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename TY>
__global__ __launch_bounds__(256) void k_orth_error(const OrthArgs a) {
  constexpr int T64 = 64, KS = 32, LDZ = KS + 1;
  __shared__ double Zi[T64][LDZ];
  __shared__ double Zj[T64][LDZ];
  __shared__ double red[4];
  const int p = blockIdx.x / a.nsplit, split = blockIdx.x % a.nsplit;
  const OrthEntry E = a.e[p];
  const TY *Y = (const TY *)E.ptr;
  const bool trans = E.rows > E.cols;
  const int64_t h = trans ? E.cols : E.rows, w = trans ? E.rows : E.cols, ld = E.ld;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int l16 = lane & 15, lk = lane >> 4;
  const int nt = (int)((h + T64 - 1) / T64);
  double total = 0.0;
  auto zel = [&](int64_t i, int64_t k) -> double {
    if (i >= h || k >= w) return 0.0;
    const int64_t idx = trans ? k * ld + i : i * ld + k;
    if constexpr (sizeof(TY) == 2) return (double)bf16_to_f32(((const uint16_t *)Y)[idx]);
    else return (double)((const float *)Y)[idx];
  };
  const int ntiles = nt * (nt + 1) / 2;
  for (int t = split; t < ntiles; t += a.nsplit) {  // upper tiles dealt round-robin
    int ti = 0, rem = t;
    while (rem >= nt - ti) {
      rem -= nt - ti;
      ti++;
    }
    const int tj = ti + rem;
    {
      f64x4 acc[2][2];
#pragma unroll
      for (int u = 0; u < 2; u++)
#pragma unroll
        for (int v = 0; v < 2; v++) acc[u][v] = f64x4{0.0, 0.0, 0.0, 0.0};
      for (int64_t k0 = 0; k0 < w; k0 += KS) {
        // stage: element (r, kk) of both row blocks; consecutive threads along the contiguous
        // index of Y (k for wide Z, the row index for tall Z)
        for (int e = threadIdx.x; e < KS * T64; e += 256) {
          const int r = trans ? (e % T64) : (e / KS), kk = trans ? (e / T64) : (e % KS);
          Zi[r][kk] = zel((int64_t)ti * T64 + r, k0 + kk);
          Zj[r][kk] = zel((int64_t)tj * T64 + r, k0 + kk);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KS; k += 4) {
          double fa[2], fb[2];
#pragma unroll
          for (int u = 0; u < 2; u++) fa[u] = Zi[wr + 16 * u + l16][k + lk];
#pragma unroll
          for (int v = 0; v < 2; v++) fb[v] = Zj[wc + 16 * v + l16][k + lk];
#pragma unroll
          for (int u = 0; u < 2; u++)
#pragma unroll
            for (int v = 0; v < 2; v++) acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[u], fb[v], acc[u][v], 0, 0, 0);
        }
        __syncthreads();
      }
      const double wgt = (ti == tj) ? 1.0 : 2.0;
#pragma unroll
      for (int u = 0; u < 2; u++)
#pragma unroll
        for (int v = 0; v < 2; v++)
#pragma unroll
          for (int r = 0; r < 4; r++) {
            const int64_t gi = (int64_t)ti * T64 + wr + 16 * u + lk + 4 * r;
            const int64_t gj = (int64_t)tj * T64 + wc + 16 * v + l16;
            if (gi < h && gj < h) {
              const double e = acc[u][v][r] - (gi == gj ? 1.0 : 0.0);
              total = fma(wgt * e, e, total);
            }
          }
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) total += __shfl_xor(total, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = total;
  __syncthreads();
  if (threadIdx.x == 0) a.part[(int64_t)p * a.nsplit + split] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ void k_orth_finish(const OrthArgs a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.count) return;
  double s = 0.0;
  for (int i = 0; i < a.nsplit; i++) s += a.part[(int64_t)p * a.nsplit + i];
  a.out[p] = sqrt(s);
}

// ---------------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------------
template <typename T, int TS>
static hipError_t launch_stage_t(int stage, const StageArgs &a, int grid, int out_bf16, hipStream_t s) {
  if (a.ntasks <= 0) return hipSuccess;
  if (stage == kStageGram) hipLaunchKernelGGL((k_gram<T, TS>), dim3(grid), dim3(kThreads), 0, s, a);
  else if (stage == kStageSquare) hipLaunchKernelGGL((k_square<T, TS>), dim3(grid), dim3(kThreads), 0, s, a);
  else hipLaunchKernelGGL((k_product<T, TS>), dim3(grid), dim3(kThreads), 0, s, a, out_bf16);
  return hipGetLastError();
}

hipError_t launch_stage(int op, int ts, int stage, const StageArgs &a, int grid, int out_bf16, hipStream_t s) {
  if (op == kOpBF16) {
    if (ts == 128) return launch_stage_t<uint16_t, 128>(stage, a, grid, out_bf16, s);
  } else if (op == kOpF32) {
    if (ts == 128) return launch_stage_t<float, 128>(stage, a, grid, out_bf16, s);
  }
  return hipErrorInvalidValue;
}

__global__ void k_zero_u32(uint32_t *p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

hipError_t launch_zero_u32(uint32_t *p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t stage_occupancy(int op, int ts, int stage, int *blocks_per_cu) {
  const void *fn = nullptr;
  if (op == kOpBF16 && ts == 128) {
    fn = stage == kStageGram ? (const void *)k_gram<uint16_t, 128>
       : stage == kStageSquare ? (const void *)k_square<uint16_t, 128> : (const void *)k_product<uint16_t, 128>;
  } else if (op == kOpF32 && ts == 128) {
    fn = stage == kStageGram ? (const void *)k_gram<float, 128>
       : stage == kStageSquare ? (const void *)k_square<float, 128> : (const void *)k_product<float, 128>;
  }
  if (!fn) return hipErrorInvalidValue;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, kThreads, 0);
}

hipError_t launch_orth_error(const OrthArgs &a, int bf16, hipStream_t s) {
  const dim3 grid(a.count * a.nsplit);
  if (bf16) hipLaunchKernelGGL(k_orth_error<uint16_t>, grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_orth_error<float>, grid, dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_orth_finish, dim3((a.count + 63) / 64), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace ifnso
