// MFMA tile machinery for gfx950 (CDNA4): LDS-staged C = Aop * Bop^T tiles.
//
// Every stage of the method is a product C[m][n] = sum_k Aop[m][k] * Bop[n][k]:
//   Gram, wide M (rows <= cols):  Aop = Bop = M            (K contiguous, "K-major")
//   Gram, tall M (rows >  cols):  Aop = Bop = M^T          (M-index contiguous, "MN-major")
//   squaring:                     Aop = Bop = B (symmetric, K-major)
//   product, wide M:              Aop = P, Bop[n][k] = M[k][n]   (MN-major)
//   product, tall M:              Aop[n][k] = M[n][k], Bop = P   (K-major both)
// The workgroup has 4 waves in a 2 x 2 arrangement; each wave owns a (BM/2) x (BN/2)
// block of 32 x 32 MFMA tiles. K is staged through LDS in steps of 128 bytes per row
// (64 bfloat16 or 32 float32), double buffered, with the next step's global loads
// issued before the current step's MFMAs. LDS rows are 128 bytes (8 chunks of 16 B);
// chunk c of row r is stored at chunk c ^ ((r ^ (r >> 3)) & 7) so that both the
// row-wise fragment reads and the column-wise transposed stores spread over banks.
// MN-major operands are transposed in registers (8 x 8 bfloat16 or 4 x 4 float32
// blocks) on their way into LDS, so the MFMA always reads K-contiguous fragments.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ifnso {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// e4m3 scale exponent of a block with maximum |value| amax: e = floor(log2(448 / amax)) (448 is
// e4m3's largest finite value), so the scaled maximum lies in (224, 448] and the scaling by 2^e
// is exact; clamped to [-63, 63] so that 2^(-2e) stays a normal float; 0 for an all-zero or
// non-finite maximum.
__device__ __forceinline__ int e4m3_scale_exp(float amax) {
  if (!(amax > 0.f) || !isfinite(amax)) return 0;
  int x;
  const float f = frexpf(amax, &x);  // amax = f 2^x, f in [0.5, 1)
  const int e = (2.f * f <= 1.75f ? 9 : 8) - x;
  return e < -63 ? -63 : (e > 63 ? 63 : e);
}

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <typename T> struct Elem;
template <> struct Elem<uint16_t> {
  static constexpr int EPC = 8;   // elements per 16-byte chunk
  static constexpr int BK = 64;   // K per LDS row
  __device__ static float to_f(uint16_t v) { return bf16_to_f32(v); }
  __device__ static uint16_t from_f(float v) { return f32_to_bf16(v); }
};
template <> struct Elem<float> {
  static constexpr int EPC = 4;
  static constexpr int BK = 32;
  __device__ static float to_f(float v) { return v; }
  __device__ static float from_f(float v) { return v; }
};

__device__ __forceinline__ int lds_off(int row, int chunk) {
  return row * 128 + ((chunk ^ ((row ^ (row >> 3)) & 7)) << 4);
}

// ---------------------------------------------------------------------------------------------
// global -> registers
// ---------------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ uint4 load_chunk_masked(const T *p, int nvalid) {
  constexpr int EPC = Elem<T>::EPC;
  union { uint4 v; T e[EPC]; } u;
#pragma unroll
  for (int e = 0; e < EPC; e++) u.e[e] = (e < nvalid) ? p[e] : (T)0;
  return u.v;
}

// K-major tile: rows m0..m0+ROWS-1 of the operand, k0..k0+BK-1. Element (m, k) at base[m*ld + k].
template <typename T, int ROWS>
__device__ __forceinline__ void gload_kmaj(uint4 (&r)[8], const T *__restrict__ base, int64_t ld, int m0,
                                           int mlim, int k0, int klim, bool vec) {
  constexpr int EPC = Elem<T>::EPC;
  constexpr int CH = ROWS * 8 / kThreads;
#pragma unroll
  for (int i = 0; i < CH; i++) {
    const int q = threadIdx.x + kThreads * i;
    const int row = q >> 3, c = q & 7;
    const int m = m0 + row, k = k0 + c * EPC;
    const T *p = base + (int64_t)m * ld + k;
    if (vec && m < mlim && k + EPC <= klim) {
      r[i] = *(const uint4 *)p;
    } else if (m < mlim && k < klim) {
      r[i] = load_chunk_masked<T>(p, klim - k);
    } else {
      r[i] = make_uint4(0, 0, 0, 0);
    }
  }
}

// MN-major tile: element (m, k) at base[k*ld + m]; each thread loads an EPC(k) x EPC(m)
// block as EPC row chunks.
template <typename T, int ROWS>
__device__ __forceinline__ void gload_mnmaj(uint4 (&r)[8], const T *__restrict__ base, int64_t ld, int m0,
                                            int mlim, int k0, int klim, bool vec) {
  constexpr int EPC = Elem<T>::EPC;
  constexpr int BK = Elem<T>::BK;
  constexpr int MB = ROWS / EPC;             // blocks along m
  constexpr int NB = MB * (BK / EPC);         // blocks per tile
  constexpr int PER = (NB + kThreads - 1) / kThreads;
  static_assert(PER * EPC <= 8, "staging registers");
#pragma unroll
  for (int b = 0; b < PER; b++) {
    const int blk = threadIdx.x + kThreads * b;
#pragma unroll
    for (int i = 0; i < EPC; i++) {
      uint4 v = make_uint4(0, 0, 0, 0);
      if (blk < NB) {
        const int mb = blk % MB, kb = blk / MB;
        const int m = m0 + mb * EPC, k = k0 + kb * EPC + i;
        const T *p = base + (int64_t)k * ld + m;
        if (k < klim) {
          if (vec && m + EPC <= mlim) v = *(const uint4 *)p;
          else if (m < mlim) v = load_chunk_masked<T>(p, mlim - m);
        }
      }
      r[b * EPC + i] = v;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// registers -> LDS
// ---------------------------------------------------------------------------------------------
template <typename T, int ROWS>
__device__ __forceinline__ void sstore_kmaj(const uint4 (&r)[8], char *lds) {
  constexpr int CH = ROWS * 8 / kThreads;
#pragma unroll
  for (int i = 0; i < CH; i++) {
    const int q = threadIdx.x + kThreads * i;
    *(uint4 *)(lds + lds_off(q >> 3, q & 7)) = r[i];
  }
}

__device__ __forceinline__ uint32_t w32(const uint4 &v, int i) {
  return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

template <typename T, int ROWS>
__device__ __forceinline__ void sstore_mnmaj(const uint4 (&r)[8], char *lds) {
  constexpr int EPC = Elem<T>::EPC;
  constexpr int BK = Elem<T>::BK;
  constexpr int MB = ROWS / EPC;
  constexpr int NB = MB * (BK / EPC);
  constexpr int PER = (NB + kThreads - 1) / kThreads;
#pragma unroll
  for (int b = 0; b < PER; b++) {
    const int blk = threadIdx.x + kThreads * b;
    if (blk >= NB) break;
    const int mb = blk % MB, kb = blk / MB;
    if constexpr (EPC == 8) {
      // 8 x 8 transpose of 16-bit elements: in row i (k) word d holds m = 2d, 2d+1.
#pragma unroll
      for (int j = 0; j < 8; j++) {
        uint32_t o[4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const uint32_t a = w32(r[b * 8 + 2 * e], j >> 1), c = w32(r[b * 8 + 2 * e + 1], j >> 1);
          o[e] = (j & 1) ? ((a >> 16) | (c & 0xffff0000u)) : ((a & 0xffffu) | (c << 16));
        }
        *(uint4 *)(lds + lds_off(mb * 8 + j, kb)) = make_uint4(o[0], o[1], o[2], o[3]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const uint4 v = make_uint4(w32(r[b * 4 + 0], j), w32(r[b * 4 + 1], j), w32(r[b * 4 + 2], j),
                                   w32(r[b * 4 + 3], j));
        *(uint4 *)(lds + lds_off(mb * 4 + j, kb)) = v;
      }
    }
  }
}

// Sum of squares (float64) of the elements a thread staged for operand A.
template <typename T>
__device__ __forceinline__ double sumsq_regs(const uint4 (&r)[8], int n) {
  constexpr int EPC = Elem<T>::EPC;
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    if (i < n) {
      union { uint4 v; T e[EPC]; } u;
      u.v = r[i];
#pragma unroll
      for (int e = 0; e < EPC; e++) {
        const double x = (double)Elem<T>::to_f(u.e[e]);
        s = fma(x, x, s);
      }
    }
  }
  return s;
}

// ---------------------------------------------------------------------------------------------
// the mainloop
// ---------------------------------------------------------------------------------------------
template <typename T, int BM, int BN>
struct Tile {
  static constexpr int BK = Elem<T>::BK;
  static constexpr int WM = BM / 2, WN = BN / 2;
  static constexpr int FM = WM / 32, FN = WN / 32;
  static constexpr int LDS_A = BM * 128, LDS_B = BN * 128;
  static constexpr int LDS_STAGE = LDS_A + LDS_B;
  static constexpr int LDS_BYTES = 2 * LDS_STAGE;
  f32x16 acc[FM][FN];

  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < FM; i++)
#pragma unroll
      for (int j = 0; j < FN; j++)
#pragma unroll
        for (int r = 0; r < 16; r++) acc[i][j][r] = 0.f;
  }

  // Coordinates (within the tile) of accumulator element r of fragment (fm, fn).
  __device__ __forceinline__ static int row_of(int fm, int r) {
    const int lane = threadIdx.x & 63, wm = (threadIdx.x >> 6) >> 1;
    return wm * WM + fm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
  }
  __device__ __forceinline__ static int col_of(int fn) {
    const int lane = threadIdx.x & 63, wn = (threadIdx.x >> 6) & 1;
    return wn * WN + fn * 32 + (lane & 31);
  }

  __device__ __forceinline__ void compute(const char *As, const char *Bs) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 31, lg = lane >> 5;
    if constexpr (sizeof(T) == 2) {
#pragma unroll
      for (int kk = 0; kk < 4; kk++) {
        bf16x8 a[FM], b[FN];
#pragma unroll
        for (int i = 0; i < FM; i++) a[i] = *(const bf16x8 *)(As + lds_off(wm * WM + i * 32 + lr, 2 * kk + lg));
#pragma unroll
        for (int j = 0; j < FN; j++) b[j] = *(const bf16x8 *)(Bs + lds_off(wn * WN + j * 32 + lr, 2 * kk + lg));
#pragma unroll
        for (int i = 0; i < FM; i++)
#pragma unroll
          for (int j = 0; j < FN; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int g = 0; g < 4; g++) {
        f32x4 a[FM], b[FN];
#pragma unroll
        for (int i = 0; i < FM; i++) a[i] = *(const f32x4 *)(As + lds_off(wm * WM + i * 32 + lr, 2 * g + lg));
#pragma unroll
        for (int j = 0; j < FN; j++) b[j] = *(const f32x4 *)(Bs + lds_off(wn * WN + j * 32 + lr, 2 * g + lg));
#pragma unroll
        for (int q = 0; q < 4; q++)
#pragma unroll
          for (int i = 0; i < FM; i++)
#pragma unroll
            for (int j = 0; j < FN; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][q], b[j][q], acc[i][j], 0, 0, 0);
      }
    }
  }

  // C = Aop[am0.., :K] * Bop[bn0.., :K]^T.  AMN / BMN select MN-major operands.
  // Rows of Aop at or beyond alim (of Bop at or beyond blim) and k at or beyond K read as 0.
  // With want_norm, returns this thread's float64 sum of squares of the Aop elements it loaded.
  template <bool AMN, bool BMN>
  __device__ __forceinline__ double run(char *smem, const T *A, int64_t lda, int am0, int alim, bool avec,
                                        const T *B, int64_t ldb, int bn0, int blim, bool bvec, int K,
                                        bool want_norm) {
    uint4 ra[8], rb[8];
    double nrm = 0.0;
    constexpr int EPC = Elem<T>::EPC;
    constexpr int NB_MN = (BM / EPC) * (BK / EPC);
    constexpr int NA = AMN ? ((NB_MN + kThreads - 1) / kThreads) * EPC : BM * 8 / kThreads;
    const int nk = (K + BK - 1) / BK;
    auto gl = [&](int k0) {
      if constexpr (AMN) gload_mnmaj<T, BM>(ra, A, lda, am0, alim, k0, K, avec);
      else gload_kmaj<T, BM>(ra, A, lda, am0, alim, k0, K, avec);
      if constexpr (BMN) gload_mnmaj<T, BN>(rb, B, ldb, bn0, blim, k0, K, bvec);
      else gload_kmaj<T, BN>(rb, B, ldb, bn0, blim, k0, K, bvec);
    };
    auto st = [&](int buf) {
      char *As = smem + buf * LDS_STAGE;
      char *Bs = As + LDS_A;
      if constexpr (AMN) sstore_mnmaj<T, BM>(ra, As);
      else sstore_kmaj<T, BM>(ra, As);
      if constexpr (BMN) sstore_mnmaj<T, BN>(rb, Bs);
      else sstore_kmaj<T, BN>(rb, Bs);
    };
    zero();
    if (nk <= 0) return 0.0;
    gl(0);
    if (want_norm) nrm += sumsq_regs<T>(ra, NA);
    st(0);
    __syncthreads();
    for (int kt = 0; kt < nk; kt++) {
      const int cur = kt & 1;
      const bool more = kt + 1 < nk;
      if (more) gl((kt + 1) * BK);
      compute(smem + cur * LDS_STAGE, smem + cur * LDS_STAGE + LDS_A);
      if (more) {
        if (want_norm) nrm += sumsq_regs<T>(ra, NA);
        st(cur ^ 1);
      }
      __syncthreads();
    }
    return nrm;
  }
};

// Fixed-order workgroup sum of three doubles (xor butterfly within waves, then the
// four wave results in wave order). Result valid in every thread. Uses 96 bytes of LDS
// at `scratch`; the caller must have finished using that LDS.
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c, double *scratch) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
    c += __shfl_xor(c, off, 64);
  }
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    scratch[wave * 3 + 0] = a;
    scratch[wave * 3 + 1] = b;
    scratch[wave * 3 + 2] = c;
  }
  __syncthreads();
  a = ((scratch[0] + scratch[3]) + scratch[6]) + scratch[9];
  b = ((scratch[1] + scratch[4]) + scratch[7]) + scratch[10];
  c = ((scratch[2] + scratch[5]) + scratch[8]) + scratch[11];
  __syncthreads();
}

// Fixed-order sum of n doubles by one wave (every lane gets the result).
__device__ __forceinline__ double wave_sum(const double *p, int n) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int i = lane; i < n; i += 64) s += p[i];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

// Fixed-order sum of the upper-triangle entries of an nt x nt array.
__device__ __forceinline__ double wave_sum_upper(const double *p, int nt) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  const int n = nt * nt;
  for (int i = lane; i < n; i += 64) {
    const int r = i / nt, c = i - r * nt;
    if (c >= r) s += p[i];
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

}  // namespace ifnso
