// Fast bfloat16 (and e4m3) stage kernels for gfx950: 256 x 256 output tiles.
//
// Operands are read through buffer resource descriptors: an out-of-range chunk gets an
// offset past the descriptor's record count and reads as zero, so edge tiles need no
// branches (the host routes a problem here only when its rows are 16-byte aligned and its
// column count is a multiple of 8, so every 16-byte chunk is wholly in or out of range).
// Operands go straight from HBM into LDS (buffer_load ... lds, 16 bytes per lane); the XOR
// swizzle of the LDS rows is applied on the global side, since a wave's LDS-DMA writes land
// contiguously. An operand is K-major (levels, wide Gram inputs, tall product inputs) or
// MN-major (tall Gram inputs, wide product inputs: M read as stored, its rows running along
// K); MN-major fragments come from transposing LDS reads, so no input is copied. Two LDS
// stages of 64 (bfloat16) or 128 (e4m3) K per row; each of the 8 waves (2 x 4, two per SIMD) owns
// a 128 x 64 block of the tile (v_mfma_f32_32x32x16_bf16 / v_mfma_f32_32x32x64_f8f6f4, 128
// float32 accumulators per lane).
// Epilogues stage the float32 tile through LDS (half a tile at a time) so that stores of
// the tile and of its mirror are 16-byte vector accesses.
#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

#include "ifnso_common.hpp"
#include "ifnso_launch.hpp"
#include "ifnso_tile.hpp"

namespace ifnso {
namespace fast {

typedef __attribute__((address_space(3))) void lds_void;

constexpr int BM = 256, BN = 256, BK = 64;
// Waves per workgroup: 8 in a 2 x 4 arrangement (two waves per SIMD, so one wave's LDS reads,
// address arithmetic and waits overlap the other's MFMAs), each owning a 128 x 64 block of the
// tile.
constexpr int NW = 8;
constexpr int NT = NW * 64;                     // threads per workgroup
constexpr int WGN = NW / 2;                     // waves along N
constexpr int WM = 128, WN = BN / WGN, FM = WM / 32, FN = WN / 32;
constexpr int RPT = BM / (8 * NW);              // rows of an operand tile one thread loads per stage
constexpr int STAGE_BYTES = (BM + BN) * 128;  // 64 KiB
constexpr int LDS_BYTES = 2 * STAGE_BYTES;    // 128 KiB
constexpr uint32_t OOB = 0x80000000u;
constexpr int EP_LD = BN + 8;                 // float stride of the epilogue staging rows
constexpr int EP_BYTES = 128 * EP_LD * 4;
constexpr int SMEM_BYTES = LDS_BYTES > EP_BYTES ? LDS_BYTES : EP_BYTES;  // 132 KiB

// Values that are the same in every lane (per-task problem fields loaded from memory) are
// moved to scalar registers, so buffer descriptors and loop bounds stay in SGPRs.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint32_t uni(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ const void *uni(const void *p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return (const void *)(((uint64_t)hi << 32) | lo);
}

typedef int i32x4 __attribute__((ext_vector_type(4)));

// Buffer resource descriptor of `bytes` bytes at p, as four scalar words (base, stride 0,
// record count, gfx9 format word): offsets at or beyond the record count read as zero.
__device__ __forceinline__ i32x4 rsrc_words(const void *p, uint32_t bytes) {
  const uint64_t a = (uint64_t)uni(p);
  i32x4 r;
  r[0] = (int)(uint32_t)a;
  r[1] = (int)((uint32_t)(a >> 32) & 0xffffu);
  r[2] = (int)uni(bytes);
  r[3] = 0x00020000;
  return r;
}

// One 16-byte-per-lane load from a buffer straight into LDS at byte offset `lds` (wave-uniform;
// lane i lands at lds + 16 i). Written as a two-instruction sequence so that the compiler's
// wait-count pass does not order every later LDS read behind it: the K loop waits for these
// loads itself (wait_vmcnt + barrier) before it reads the stage they fill. The s_nop is the
// one wait state required between an SALU write of M0 and an LDS-DMA load; the load has no
// register results.
__device__ __forceinline__ void dma16(const i32x4 &r, uint32_t voff, uint32_t lds) {
  asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tbuffer_load_dwordx4 %1, %2, 0 offen lds"
               :
               : "s"(lds), "v"(voff), "s"(r)
               : "memory", "m0");
}

__device__ __forceinline__ uint32_t lds_addr(const void *p) { return (uint32_t)(uintptr_t)(lds_void *)p; }

__device__ __forceinline__ int swz(int row) { return (row ^ (row >> 3)) & 7; }

// float64 sum of squares of the A tile held in LDS (diagonal Gram tiles with K-major A).
__device__ __forceinline__ double lds_sumsq(const char *At) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < BM * 8 / NT; i++) {
    const uint4 q = *(const uint4 *)(At + (threadIdx.x + NT * i) * 16);
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const double lo = (double)__uint_as_float(w[e] << 16), hi = (double)__uint_as_float(w[e] & 0xffff0000u);
      s = fma(lo, lo, s);
      s = fma(hi, hi, s);
    }
  }
  return s;
}

// Global-memory views of generic pointers. An access through a generic (flat) pointer counts in
// both the vector-memory and the LDS wait counters, so each wait for an LDS read would also wait
// for every global load and store still in flight; through these views the accesses are global
// ones, which only the vector-memory counter tracks.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> gbl(T *p) {
  return (gptr<T>)p;
}
// 8- and 16-byte accesses through a global view q (any gptr): HIP's vector classes have no
// members for address-space-qualified objects, so these go through clang's vector types.
typedef uint32_t gu2 __attribute__((ext_vector_type(2)));
typedef uint32_t gu4 __attribute__((ext_vector_type(4)));
typedef float gf4 __attribute__((ext_vector_type(4)));
template <typename Q>
__device__ __forceinline__ void gst(Q q, uint2 v) {
  *(gptr<gu2>)q = gu2{v.x, v.y};
}
template <typename Q>
__device__ __forceinline__ void gst(Q q, uint4 v) {
  *(gptr<gu4>)q = gu4{v.x, v.y, v.z, v.w};
}
template <typename Q>
__device__ __forceinline__ void gst(Q q, float4 v) {
  *(gptr<gf4>)q = gf4{v.x, v.y, v.z, v.w};
}
template <typename Q>
__device__ __forceinline__ uint2 gld_u2(Q q) {
  const gu2 v = *(gptr<const gu2>)q;
  return make_uint2(v.x, v.y);
}
template <typename Q>
__device__ __forceinline__ uint4 gld_u4(Q q) {
  const gu4 v = *(gptr<const gu4>)q;
  return make_uint4(v.x, v.y, v.z, v.w);
}
template <typename Q>
__device__ __forceinline__ float4 gld_f4(Q q) {
  const gf4 v = *(gptr<const gf4>)q;
  return make_float4(v.x, v.y, v.z, v.w);
}

// vmcnt-only wait (expcnt and lgkmcnt left at their maxima)
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// ---------------------------------------------------------------------------------------------
// the 256 x 256 mainloop: acc = Aop[am0.., :K] * Bop[bn0.., :K]^T
// ---------------------------------------------------------------------------------------------
struct Operand {
  i32x4 w;           // buffer descriptor words, for the LDS-DMA loads
  uint32_t ld_bytes;
  int lim;           // rows (M/N index) in range
};

__device__ __forceinline__ Operand make_operand(const void *p, uint32_t bytes, uint32_t ld_bytes, int lim) {
  Operand o;
  o.w = rsrc_words(p, bytes);
  o.ld_bytes = uni(ld_bytes);
  o.lim = uni(lim);
  return o;
}

typedef int i32x8 __attribute__((ext_vector_type(8)));

// Byte offsets of one thread's rows of a K-major operand tile (ROWS / (8 NW) rows; wave-instruction
// g covers rows 8g..8g+7, lane chunk c = (lane & 7) ^ swz(row)), computed once per tile: the
// offset of chunk c at k = 0, or OOB for rows outside the operand. A K step adds k0 * ES.
template <int ROWS>
struct KRows {
  uint32_t off[ROWS / (8 * NW)];
};

template <int ROWS>
__device__ __forceinline__ void krows(KRows<ROWS> &R, uint32_t ld_bytes, int m0, int mlim) {
  const int wave = uni((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < ROWS / (8 * NW); i++) {
    const int row = (i * NW + wave) * 8 + (lane >> 3);
    const int c = (lane & 7) ^ swz(row);
    const int m = m0 + row;
    R.off[i] = m < mlim ? (uint32_t)m * ld_bytes + (uint32_t)c * 16u : OOB;
  }
}

// MN-major operand tile (bfloat16): a stage holds 64 K rows of the tile's 256 MN-contiguous
// values, 512 bytes per LDS row. Wave-instruction g covers LDS rows 2g and 2g+1; lane l loads
// LDS chunk p = l % 32 of row 2g + l / 32 from the operand's chunk p ^ mswz(row). Chunk offsets
// of the rows differ by multiples of 4, so the transposing fragment reads (four rows of four
// chunks per 16 lanes) meet no bank conflict. The per-tile offset is that of K row `row` (k0 = 0);
// a K step adds k0 * ld_bytes.
__device__ __forceinline__ int mswz(int row) { return (row & 3) << 2; }

template <int ROWS>
__device__ __forceinline__ void krows_mn(KRows<ROWS> &R, uint32_t ld_bytes, int mn0, int mnlim) {
  const int wave = uni((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < ROWS / (8 * NW); i++) {
    const int row = 2 * (i * NW + wave) + (lane >> 5);
    const int mn = mn0 + 8 * ((lane & 31) ^ mswz(row));
    R.off[i] = mn < mnlim ? (uint32_t)row * ld_bytes + (uint32_t)mn * 2u : OOB;
  }
}

// Loads rows [I0, I1) of the thread's rows of stage k0 into the LDS tile at lt. `full`: the
// whole stage lies below K (otherwise chunks (K-major) or rows (MN-major) at or beyond K read
// as zero).
template <int ROWS, int ES, int I0, int I1, bool FULL, bool MN>
__device__ __forceinline__ void issue_krows_(const KRows<ROWS> &R, uint32_t lt, const i32x4 &r, int k0, int K,
                                             uint32_t ld_bytes, int wave) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = I0; i < I1; i++) {
    const int g = i * NW + wave;
    uint32_t off = R.off[i] + (MN ? (uint32_t)k0 * ld_bytes : (uint32_t)(k0 * ES));
    if constexpr (!FULL) {
      if constexpr (MN) {
        if (k0 + 2 * g + (lane >> 5) >= K) off = OOB;
      } else {
        const int row = g * 8 + (lane >> 3);
        const int c = (lane & 7) ^ swz(row);
        if (k0 + c * (16 / ES) >= K) off = OOB;
      }
    }
    dma16(r, off, lt + g * 1024);
  }
}

template <int ROWS, int ES, int I0, int I1, bool MN = false>
__device__ __forceinline__ void issue_krows(const KRows<ROWS> &R, uint32_t lt, const i32x4 &r, int k0, int K,
                                            bool full, uint32_t ld_bytes, int wave) {
  if (full) issue_krows_<ROWS, ES, I0, I1, true, MN>(R, lt, r, k0, K, ld_bytes, wave);
  else issue_krows_<ROWS, ES, I0, I1, false, MN>(R, lt, r, k0, K, ld_bytes, wave);
}

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) s16x4 lds_s16x4;

// MFMA fragment (32 MN x 8 K per lane: lane l holds MN index mn_off + l % 32, K 8 (l / 32) ..
// + 7 of slice kk) of an MN-major stage, by two transposing LDS reads (ds_read_b64_tr_b16). In
// each group of 16 lanes, lane 4e + q addresses four MN values (4q .. 4q+3) of K row e, and
// lane j of the group receives value j % 4 of the row addressed by lane 4e + j / 4 as element e:
// MN index j, K rows 0..3. The second read covers K rows 4..7.
__device__ __forceinline__ bf16x8 tr_frag(const char *S, int mn_off, int kk) {
  const int lane = threadIdx.x & 63, g = lane >> 4, q = lane & 15;
  const int kr = 16 * kk + 8 * (g >> 1) + (q >> 2);
  const int mn = mn_off + 16 * (g & 1) + 4 * (q & 3);
  const char *p = S + kr * 512 + (((mn >> 3) ^ mswz(kr)) << 4) + (mn & 7) * 2;
  const s16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4 *)p);
  const s16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4 *)(p + 4 * 512));  // mswz(kr + 4) == mswz(kr)
  typedef short s16x8 __attribute__((ext_vector_type(8)));
  const s16x8 v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  return __builtin_bit_cast(bf16x8, v);
}

// K maps of an operand in split-bfloat16 products (a value carried as hi + lo bf16 halves stored
// side by side: [X_hi | X_lo], seg columns each). The product runs over a logical K made of
// several segments, interleaved step by step: logical step q (64 wide) is segment q mod n of
// physical step q / n, so the segments of one 64-wide K chunk follow each other and a chunk read
// again by the next segment is still in L2. Segment t reads physical segment map(t):
//   KMAP_ID   identity (no segments)
//   KMAP_MOD  n = 2, segments (0, 0): the operand is used as is against [Y_hi | Y_lo]
//   KMAP_SEG2 n = 2, segments (0, 1): [X_hi | X_lo]
//   KMAP_HHL  n = 3, segments (0, 0, 1)
//   KMAP_HLH  n = 3, segments (0, 1, 0)
// so that HHL . HLH^T = X_hi X_hi^T + X_hi X_lo^T + X_lo X_hi^T, and MOD . SEG2^T = Y M^T form
// Y_hi M^T + Y_lo M^T.
enum KMapKind : int { KMAP_ID = 0, KMAP_MOD = 1, KMAP_HHL = 2, KMAP_HLH = 3, KMAP_SEG2 = 4 };

template <int MAP>
__device__ __forceinline__ int kphys(int k, int seg) {
  if constexpr (MAP == KMAP_ID) {
    return k;
  } else {
    constexpr int n = (MAP == KMAP_MOD || MAP == KMAP_SEG2) ? 2 : 3;
    const int q = k >> 6, t = q % n;            // logical step, its segment
    const int kk = ((q / n) << 6) + (k & 63);  // position in the segment
    if constexpr (MAP == KMAP_MOD) return kk;
    else if constexpr (MAP == KMAP_SEG2) return kk + (t == 1 ? seg : 0);
    else if constexpr (MAP == KMAP_HHL) return kk + (t == 2 ? seg : 0);
    else return kk + (t == 1 ? seg : 0);
  }
}

// Both operands K-major: one barrier per K step. The loads of step k+1 go into the other LDS
// stage while step k's MFMAs run, half of them before each of the step's first two K slices (so
// the later half still has half a step to land before the next barrier); that stage was last
// read in step k-1, which every wave finished before this step's barrier. bfloat16 fragments are
// double-buffered: slice kk+1's are read from LDS while slice kk's MFMAs run.
// PA / PB: K-segment maps (segments of `seg`, a multiple of the stage depth); K is then the
// logical depth, and kvA / kvB bound the physical K of each operand (beyond it reads as zero).
template <bool F8, bool AMN = false, bool BMN = false, int PA = KMAP_ID, int PB = KMAP_ID>
__device__ __forceinline__ double mainloop_kk(f32x16 (&acc)[FM][FN], char *smem, const Operand &A, int am0,
                                              const Operand &B, int bn0, int K, bool want_norm, int seg = 0,
                                              int kvA = 0, int kvB = 0) {
  static_assert(!F8 || (!AMN && !BMN), "e4m3 operands are K-major");
  const int KA = PA == KMAP_ID ? K : kvA, KB = PB == KMAP_ID ? K : kvB;
  constexpr int ES = F8 ? 1 : 2;
  constexpr int KST = 128 / ES;           // elements per stage
  constexpr int NS = F8 ? 2 : BK / 16;    // MFMA K slices per stage
  constexpr int PER = RPT / 2;            // rows of each operand issued in each of the first two slices
  const int lane = threadIdx.x & 63, wave = uni((int)(threadIdx.x >> 6));
  const int wm = wave / WGN, wn = wave % WGN;
  const int lr = lane & 31, lg = lane >> 5;
#pragma unroll
  for (int i = 0; i < FM; i++)
#pragma unroll
    for (int j = 0; j < FN; j++)
#pragma unroll
      for (int r = 0; r < 16; r++) acc[i][j][r] = 0.f;
  const int nk = (K + KST - 1) / KST;
  if (nk <= 0) return 0.0;
  double nrm = 0.0;
  KRows<BM> RA;
  KRows<BN> RB;
  if constexpr (AMN) krows_mn<BM>(RA, A.ld_bytes, am0, A.lim);
  else krows<BM>(RA, A.ld_bytes, am0, A.lim);
  if constexpr (BMN) krows_mn<BN>(RB, B.ld_bytes, bn0, B.lim);
  else krows<BN>(RB, B.ld_bytes, bn0, B.lim);
  const uint32_t lbase = uni(lds_addr(smem));
  {
    const int ka = kphys<PA>(0, seg), kb = kphys<PB>(0, seg);
    issue_krows<BM, ES, 0, RPT, AMN>(RA, lbase, A.w, ka, KA, ka + KST <= KA, A.ld_bytes, wave);
    issue_krows<BN, ES, 0, RPT, BMN>(RB, lbase + BM * 128, B.w, kb, KB, kb + KST <= KB, B.ld_bytes, wave);
  }
  for (int kt = 0; kt < nk; kt++) {
    const int cur = kt & 1;
    wait_vmcnt<0>();
    __syncthreads();
    const char *As = smem + cur * STAGE_BYTES, *Bs = As + BM * 128;
    if constexpr (!F8) {
      if (want_norm) nrm += lds_sumsq(As);
    }
    const bool more = kt + 1 < nk;
    const int k1 = (kt + 1) * KST;
    const int ka = kphys<PA>(k1, seg), kb = kphys<PB>(k1, seg);
    const bool fulla = ka + KST <= KA, fullb = kb + KST <= KB;
    const uint32_t An = lbase + (cur ^ 1) * STAGE_BYTES, Bn = An + BM * 128;
    auto issue_slice = [&](auto sl) {
      constexpr int s = decltype(sl)::value;
      if constexpr (s < 2) {
        if (more) {
          issue_krows<BM, ES, s * PER, (s + 1) * PER, AMN>(RA, An, A.w, ka, KA, fulla, A.ld_bytes, wave);
          issue_krows<BN, ES, s * PER, (s + 1) * PER, BMN>(RB, Bn, B.w, kb, KB, fullb, B.ld_bytes, wave);
        }
      }
    };
    if constexpr (F8) {
      auto slice = [&](auto sl) {
        constexpr int kk = decltype(sl)::value;
        issue_slice(sl);
        i32x8 fa[FM], fb[FN];
#pragma unroll
        for (int i = 0; i < FM; i++) {
          const int row = wm * WM + i * 32 + lr;
          const uint4 lo = *(const uint4 *)(As + lds_off(row, 4 * kk + 2 * lg));
          const uint4 hi = *(const uint4 *)(As + lds_off(row, 4 * kk + 2 * lg + 1));
          fa[i] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
        }
#pragma unroll
        for (int j = 0; j < FN; j++) {
          const int row = wn * WN + j * 32 + lr;
          const uint4 lo = *(const uint4 *)(Bs + lds_off(row, 4 * kk + 2 * lg));
          const uint4 hi = *(const uint4 *)(Bs + lds_off(row, 4 * kk + 2 * lg + 1));
          fb[j] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
        }
#pragma unroll
        for (int i = 0; i < FM; i++)
#pragma unroll
          for (int j = 0; j < FN; j++)
            acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(fa[i], fb[j], acc[i][j], 0, 0, 0, 0, 0, 0);
      };
      slice(std::integral_constant<int, 0>{});
      slice(std::integral_constant<int, 1>{});
    } else {
      bf16x8 fa[2][FM], fb[2][FN];
      auto rd = [&](int kk, int sl) {
#pragma unroll
        for (int i = 0; i < FM; i++)
          fa[sl][i] = AMN ? tr_frag(As, wm * WM + i * 32, kk)
                          : *(const bf16x8 *)(As + lds_off(wm * WM + i * 32 + lr, 2 * kk + lg));
#pragma unroll
        for (int j = 0; j < FN; j++)
          fb[sl][j] = BMN ? tr_frag(Bs, wn * WN + j * 32, kk)
                          : *(const bf16x8 *)(Bs + lds_off(wn * WN + j * 32 + lr, 2 * kk + lg));
      };
      auto slice = [&](auto slc) {
        constexpr int kk = decltype(slc)::value;
        constexpr int sl = kk & 1;
        issue_slice(slc);
        if constexpr (kk + 1 < NS) rd(kk + 1, sl ^ 1);
#pragma unroll
        for (int i = 0; i < FM; i++)
#pragma unroll
          for (int j = 0; j < FN; j++)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[sl][i], fb[sl][j], acc[i][j], 0, 0, 0);
        if constexpr (kk + 1 < NS) {
#pragma unroll
          for (int q = 0; q < FM + FN; q++) {
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);  // two MFMAs
          }
        }
      };
      rd(0, 0);
      slice(std::integral_constant<int, 0>{});
      slice(std::integral_constant<int, 1>{});
      slice(std::integral_constant<int, 2>{});
      slice(std::integral_constant<int, 3>{});
    }
  }
  __syncthreads();  // the epilogue reuses the LDS stages
  return nrm;
}

// acc = Aop[am0.., :K] * Bop[bn0.., :K]^T. An operand is K-major (rows am0.. of a row-major
// array whose rows run along K) or, with AMN / BMN, MN-major (the array's rows run along K and
// its columns am0.. are the tile's rows: Aop = X^T). F8: OCP e4m3 operands (1 byte, 128 per LDS
// row and stage, K-major), MFMA 32x32x64.
template <bool AMN, bool BMN, bool F8 = false, int PA = KMAP_ID, int PB = KMAP_ID>
__device__ __forceinline__ double mainloop(f32x16 (&acc)[FM][FN], char *smem, const Operand &A, int am0,
                                           const Operand &B, int bn0, int K, bool want_norm, int seg = 0,
                                           int kvA = 0, int kvB = 0) {
  return mainloop_kk<F8, AMN, BMN, PA, PB>(acc, smem, A, am0, B, bn0, K, want_norm, seg, kvA, kvB);
}

// ---------------------------------------------------------------------------------------------
// epilogue staging: half a tile (rows half*128 .. +127) of float32 in LDS
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void stage_half(const f32x16 (&acc)[FM][FN], float *ep, int half) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  if (wm != half) return;
  // one base address per 32-row block; the rest are immediate offsets of the LDS stores
  float *base = ep + 4 * (lane >> 5) * EP_LD + wn * WN + (lane & 31);
#pragma unroll
  for (int i = 0; i < FM; i++) {
    float *pi = base + uni(i * 32 * EP_LD);
#pragma unroll
    for (int j = 0; j < FN; j++)
#pragma unroll
      for (int r = 0; r < 16; r++) pi[(8 * (r >> 2) + (r & 3)) * EP_LD + j * 32] = acc[i][j][r];
  }
}

// Two float32 values rounded to bfloat16 (to nearest, ties to even) and packed, a in the low
// half: one v_cvt_pk_bf16_f32.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){a, b}, bf16x2_t));
}

// ---------------------------------------------------------------------------------------------
// per-problem scalars (same definitions as the generic kernels)
// ---------------------------------------------------------------------------------------------
struct FScalars {
  double nA2, g2, sg, sout;
  bool zero;
};

// The totals P.lvl_sum[0 .. kMaxLevels], one per lane (lane l holds entry l; lanes beyond read
// zero): one load per wave; lsum(t, l) reads entry l.
__device__ __forceinline__ double lsum_load(const ProbDev &P) {
  const int l = threadIdx.x & 63;
  return l <= kMaxLevels ? P.lvl_sum[l] : 0.0;
}
__device__ __forceinline__ double lsum(double t, int l) { return __shfl(t, l, 64); }

__device__ __forceinline__ FScalars scalars(double t, int norm) {
  FScalars s;
  s.nA2 = lsum(t, 0);
  s.g2 = lsum(t, 1);
  s.zero = !(s.nA2 > 0.0);
  if (norm == kFrob) {
    s.sg = s.zero ? 0.0 : 1.0 / s.nA2;
    s.sout = s.zero ? 0.0 : 1.0 / sqrt(s.nA2);
  } else if (norm == kGramFrob) {
    const double o = sqrt(s.g2);
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

__device__ __forceinline__ double level_scale(double t, double sg, int level) {
  double S = sg;
  for (int l = 1; l < level; l++) {
    const double F = pow2_inv_round(lsum(t, l));
    S = S * S / F;
  }
  return S;
}

__device__ __forceinline__ Task decode_upper(int t, int nt) {
  int tm = 0;
  while (t >= nt - tm) {
    t -= nt - tm;
    tm++;
  }
  return Task{0, tm, tm + t, 0};
}

__device__ __forceinline__ Task fetch(const StageArgs &a, int t, int stage) {
  if (a.tasks) return a.tasks[t];
  const ProbDev &P = a.one;
  if (stage != kStageProduct) return decode_upper(t, P.hp / BM);
  const int ncols = ((P.trans ? P.h : P.w) + BN - 1) / BN;
  return Task{0, t / ncols, t % ncols, 0};
}

// Task iteration of a workgroup: either plain striding over the whole list, or the
// workgroup's XCD queue (consecutive queue entries are tiles that share operand panels, so
// the 32 workgroups of an XCD work on neighbouring tiles at the same time).
struct TaskRange {
  int base, start, stride, end;
};

__device__ __forceinline__ TaskRange task_range(const StageArgs &a) {
  if (a.tasks && a.xcd_sched) {
    const int x = blockIdx.x & 7, w = gridDim.x >> 3;
    return TaskRange{a.xcd_off[x], (int)(blockIdx.x >> 3), w, a.xcd_cnt[x]};
  }
  return TaskRange{0, (int)blockIdx.x, (int)gridDim.x, a.ntasks};
}

// The tasks a workgroup runs: with per-XCD queues and task counters (a.qctr), the next entry of
// its own XCD's queue, taken with an atomic increment of that queue's counter, and once that
// queue is empty the entries left in the other queues (in XCD order), so that no workgroup idles
// while another queue still holds work; otherwise static striding through its queue (or through
// the whole list). Which workgroup runs a tile does not change any result: every reduction is
// summed in a fixed order.
struct TaskCursor {
  TaskRange tr;
  int t, tried;
  int *slot;  // LDS word that broadcasts a taken task to the workgroup
  __device__ TaskCursor(const StageArgs &a, int *s) : tr(task_range(a)), t(tr.start), tried(0), slot(s) {}
  // g: index into the task list (or into the single problem's tiles); false when none is left
  __device__ bool next(const StageArgs &a, int &g) {
    if (!(a.qctr && a.tasks && a.xcd_sched)) {
      if (t >= tr.end) return false;
      g = tr.base + t;
      t += tr.stride;
      return true;
    }
    if (threadIdx.x == 0) {
      int v = -1;
      const int x0 = blockIdx.x & 7;
      while (tried < 8) {
        const int x = (x0 + tried) & 7;
        const uint32_t i = atomicAdd(a.qctr + x, 1u);
        if (i < (uint32_t)a.xcd_cnt[x]) {
          v = a.xcd_off[x] + (int)i;
          break;
        }
        tried++;
      }
      *slot = v;
    }
    __syncthreads();
    g = uni(*slot);
    __syncthreads();
    return g >= 0;
  }
};

__device__ __forceinline__ const ProbDev &prob(const StageArgs &a, const Task &t) {
  return a.tasks ? a.probs[t.p] : a.one;
}

// Partials of a 256 tile land in the 128-granular arrays: slot (2tm, 2tn) gets the value,
// the other covered upper slots get 0, so consumers sum the same grid as for 128 tiles.
__device__ __forceinline__ void write_level_partials(const ProbDev &P, int level, const Task &t, double lv, double dg) {
  const int nt = P.nt;
  gptr<double> lp = gbl(P.lvl_part + (int64_t)level * nt * nt);
  const int r0 = 2 * t.tm, c0 = 2 * t.tn;
  lp[r0 * nt + c0] = lv;
  lp[r0 * nt + c0 + 1] = 0.0;
  lp[(r0 + 1) * nt + c0 + 1] = 0.0;
  if (t.tm != t.tn) lp[(r0 + 1) * nt + c0] = 0.0;
  if (t.tm == t.tn) {
    gptr<double> dp = gbl(P.diag_part + level * nt);
    dp[r0] = dg;
    dp[r0 + 1] = 0.0;
  }
}

// e4m3 bytes of four floats (v_cvt_pk_fp8_f32: nearest, ties to even), the first in the lowest byte.
__device__ __forceinline__ uint32_t pack4_e4m3(float a, float b, float c, float d) {
  int v = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  v = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, v, true);
  return (uint32_t)v;
}
// e4m3 bytes of qs times the four bfloat16 values packed in two words, saturating at +-448 (the
// scale keeps every value within 448 (1 + 2^-8), which rounds to 448 anyway; the clamp keeps a
// value beyond it finite)
__device__ __forceinline__ float sat448(float v) { return __builtin_amdgcn_fmed3f(v, -448.f, 448.f); }
__device__ __forceinline__ uint32_t e4m3_of_bf16(uint32_t w0, uint32_t w1, float qs) {
  return pack4_e4m3(sat448(qs * __uint_as_float(w0 << 16)), sat448(qs * __uint_as_float(w0 & 0xffff0000u)),
                    sat448(qs * __uint_as_float(w1 << 16)), sat448(qs * __uint_as_float(w1 & 0xffff0000u)));
}

// Writes the staged half tile (rows half*128..) as bfloat16 into dst (ld hp) at the tile and,
// off the diagonal, at its mirror. `f` maps the staged float to the stored value. With Q8, also
// the e4m3 bytes of qs times the stored bfloat16 values into dst8 (ld hp), tile and mirror.
template <bool Q8 = false, typename F>
__device__ __forceinline__ void emit_sym_bf16(const float *ep, uint16_t *dst, int64_t hp, int m0, int n0, int half,
                                              bool diag, F f, uint8_t *dst8 = nullptr, float qs = 1.f) {
  // direct: each wave instruction reads one staged row (64 lanes x 16 contiguous bytes, no bank
  // conflict) and stores it as 512 contiguous bytes of bfloat16. Per-iteration offsets are
  // uniform (scalar) additions to one per-thread base.
  {
    constexpr int RS = NT / 64;  // rows per iteration
    const int row0 = threadIdx.x >> 6, c4 = (threadIdx.x & 63) * 4;
    const float *src = ep + row0 * EP_LD + c4;
    gptr<uint16_t> d = gbl(dst + (int64_t)(m0 + half * 128 + row0) * hp + n0 + c4);
#pragma unroll 4
    for (int it = 0; it < 128 / RS; it++) {
      const float4 v = *(const float4 *)(src + it * RS * EP_LD);
      const int row = row0 + it * RS;
      const uint2 o = make_uint2(pack_bf16x2(f(v.x, row, c4), f(v.y, row, c4 + 1)),
                                 pack_bf16x2(f(v.z, row, c4 + 2), f(v.w, row, c4 + 3)));
      gst(d + (int64_t)uni(it * RS) * hp, o);
      if constexpr (Q8)
        *gbl((uint32_t *)(dst8 + (int64_t)(m0 + half * 128 + row) * hp + n0 + c4)) = e4m3_of_bf16(o.x, o.y, qs);
    }
  }
  if (diag) return;
  // mirror: element (row, col) of the tile goes to (n0 + col, m0 + row). Four consecutive lanes
  // cover 32 tile rows (four chunks of 8) of one column, so a store instruction writes 64
  // contiguous bytes into each of 16 mirror rows; with the column varying across lane groups
  // the column reads of the staged half meet at most a 4-way bank conflict.
  {
    constexpr int CPI = NT / 4, NC = 256 / CPI;  // columns per iteration, iterations per 32 rows
    const int c0 = threadIdx.x >> 2, r0 = (threadIdx.x & 3) * 8;
    const float *src = ep + r0 * EP_LD + c0;
    gptr<uint16_t> d = gbl(dst + (int64_t)(n0 + c0) * hp + m0 + half * 128 + r0);
#pragma unroll 8
    for (int it = 0; it < 4 * NC; it++) {
      const int dc = CPI * (it % NC), dr = 32 * (it / NC);
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; e++) v[e] = f(src[(dr + e) * EP_LD + dc], r0 + dr + e, c0 + dc);
      uint4 o;
      o.x = pack_bf16x2(v[0], v[1]);
      o.y = pack_bf16x2(v[2], v[3]);
      o.z = pack_bf16x2(v[4], v[5]);
      o.w = pack_bf16x2(v[6], v[7]);
      gst(d + (int64_t)uni(dc) * hp + dr, o);
      if constexpr (Q8)
        gst(gbl(dst8 + (int64_t)(n0 + c0 + dc) * hp + m0 + half * 128 + r0 + dr),
            make_uint2(e4m3_of_bf16(o.x, o.y, qs), e4m3_of_bf16(o.z, o.w, qs)));
    }
  }
}

// bfloat16 value of v (round to nearest even), as a float
__device__ __forceinline__ float bf16_value(float v) { return __uint_as_float(pack_bf16x2(v, 0.f) << 16); }
// The two bfloat16 values packed in a 32-bit word (the lower address in the low half).
__device__ __forceinline__ float bf16_pair_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_pair_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// Staged half tile as a bfloat16 operand: plain (leading dimension hp), or with SPLIT as the
// pair hi = bf16(v), lo = bf16(v - hi) stored side by side ([X_hi | X_lo], leading dimension 2 hp).
template <bool SPLIT>
__device__ __forceinline__ void emit_operand(const float *ep, uint16_t *dst, int64_t hp, int m0, int n0, int half,
                                             bool diag) {
  if constexpr (SPLIT) {
    emit_sym_bf16(ep, dst, 2 * hp, m0, n0, half, diag, [](float v, int, int) { return v; });
    emit_sym_bf16(ep, dst + hp, 2 * hp, m0, n0, half, diag, [](float v, int, int) { return v - bf16_value(v); });
  } else {
    emit_sym_bf16(ep, dst, hp, m0, n0, half, diag, [](float v, int, int) { return v; });
  }
}

// Sums of three float64 values over the workgroup in a fixed order (lanes, then waves 0..NW-1).
__device__ __forceinline__ void block_sum3w(double &a, double &b, double &c, double *scratch) {
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
  a = scratch[0];
  b = scratch[1];
  c = scratch[2];
#pragma unroll
  for (int w = 1; w < NW; w++) {
    a += scratch[w * 3 + 0];
    b += scratch[w * 3 + 1];
    c += scratch[w * 3 + 2];
  }
  __syncthreads();
}

__device__ __forceinline__ float block_max(float v, float *scratch) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
  __syncthreads();
  v = scratch[0];
#pragma unroll
  for (int w = 1; w < NW; w++) v = fmaxf(v, scratch[w]);
  __syncthreads();
  return v;
}

// Sum of squares and (AMAX) max |value| of scale * tile straight from the accumulators (each
// lane's 32 x 32 blocks summed in float32, accumulated in float64); off-diagonal tiles count
// twice (mirror). The scale is a power of two, so the sums of the raw accumulators times scale^2
// (and |scale| times their maximum) are the same numbers, one multiply per value cheaper.
template <bool AMAX>
__device__ __forceinline__ void reg_partials(const f32x16 (&acc)[FM][FN], float scale, bool diag, double &lv,
                                             float &mx) {
  double sum = 0.0;
  float amax = 0.f;
#pragma unroll
  for (int i = 0; i < FM; i++)
#pragma unroll
    for (int j = 0; j < FN; j++) {
      float s2 = 0.f;
#pragma unroll
      for (int r = 0; r < 16; r++) {
        s2 = fmaf(acc[i][j][r], acc[i][j][r], s2);
        if constexpr (AMAX) amax = fmaxf(amax, fabsf(acc[i][j][r]));
      }
      sum += (double)s2;
    }
  lv += sum * ((double)scale * (double)scale) * (diag ? 1.0 : 2.0);
  if constexpr (AMAX) mx = fmaxf(mx, fabsf(scale) * amax);
}

// Level-layout epilogue: level `out` = scale * acc is stored as bfloat16 (tile and mirror) at
// lv + (out - 1) * lv_stride with the partials of its sum of squares (reg_partials) and trace
// (diagonal tiles: from the staged tile). With AMAX (e4m3 plans) the level is also stored as
// e4m3 in ql[out & 1], with the power-of-two scale of `amax`, the largest magnitude of scale *
// acc before rounding: acc is X X^T of a quantised operand X, positive semi-definite, so that
// is scale times its largest diagonal entry, scale times the largest row sum of squares of X,
// which the pass before the stage found. Rounding to bfloat16 can lift a stored value above
// amax by 2^-8 relative at most; scaled it stays below 464 and rounds to e4m3's 448.

template <bool AMAX>
__device__ __forceinline__ void store_level(const f32x16 (&acc)[FM][FN], char *smem, const ProbDev &P, int out,
                                            const Task &task, float scale, float amax = 0.f) {
  const int m0 = task.tm * BM, n0 = task.tn * BN;
  const bool diag = task.tm == task.tn;
  const int64_t hp = P.hp;
  uint16_t *dst = (uint16_t *)((char *)P.lv + (int64_t)(out - 1) * P.lv_stride);
  double lv = 0.0, dg = 0.0, unused = 0.0;
  float mx = 0.f;
  reg_partials<AMAX>(acc, scale, diag, lv, mx);
  // AMAX: the level's e4m3 scale, from the largest magnitude of the level before its rounding
  const float qs = AMAX ? ldexpf(1.f, e4m3_scale_exp(amax)) : 1.f;
  uint8_t *dst8 = AMAX ? P.ql[out & 1] : nullptr;
  float *ep = (float *)smem;
  for (int half = 0; half < 2; half++) {
    stage_half(acc, ep, half);
    __syncthreads();
    if (diag && threadIdx.x < 128) dg += (double)(scale * ep[threadIdx.x * EP_LD + half * 128 + threadIdx.x]);
    emit_sym_bf16<AMAX>(ep, dst, hp, m0, n0, half, diag, [scale](float v, int, int) { return scale * v; }, dst8, qs);
    __syncthreads();
  }
  block_sum3w(lv, dg, unused, (double *)smem);
  if (threadIdx.x == 0) {
    write_level_partials(P, out, task, lv, dg);
    if (AMAX && task.tm == 0 && task.tn == 0) {  // every tile has the same scale; one records it
      gptr<float> qsc = gbl(P.q_scale);
      qsc[2 * out] = qs;
      qsc[2 * out + 1] = amax;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------------------------
// Gram
// ---------------------------------------------------------------------------------------------
// TALL: A = M^T, read MN-major straight from M (K = rows of M); otherwise A = M, K-major.
// SPLIT: the Gram operand is stored as a split bfloat16 pair (complement-basis split plans).
template <bool TALL, bool SPLIT>
__global__ __launch_bounds__(NT, 1) void kf_gram(const StageArgs a) {
  __shared__ __attribute__((aligned(1024))) char smem[SMEM_BYTES];
  float *ep = (float *)smem;
  __shared__ int s_task;
  TaskCursor cursor(a, &s_task);
  int tg = 0;
  while (cursor.next(a, tg)) {
    Task task = fetch(a, tg, kStageGram);
    task.p = uni(task.p);
    task.tm = uni(task.tm);
    task.tn = uni(task.tn);
    const ProbDev &P = prob(a, task);
    const int m0 = task.tm * BM, n0 = task.tn * BN;
    const bool diag = task.tm == task.tn;
    // M is rows x cols with (rows, cols) = (w, h) when tall, (h, w) when wide
    const uint32_t mbytes = (uint32_t)(((int64_t)(TALL ? P.w : P.h) - 1) * P.ldm * 2 + (int64_t)(TALL ? P.h : P.w) * 2);
    const Operand op = make_operand(P.M, mbytes, (uint32_t)(P.ldm * 2), P.h);
    const int K = uni(P.w);
    f32x16 acc[FM][FN];
    double nrm = mainloop<TALL, TALL>(acc, smem, op, m0, op, n0, K, diag);
    uint16_t *dst = (uint16_t *)P.opnd[0];
    const int64_t hp = P.hp;
    const bool keep_f32 = (a.J >= 1 && !a.agg) || a.learned;
    double lv = 0.0, dg = 0.0;
    float unused_mx = 0.f;
    if (!keep_f32) reg_partials<false>(acc, 1.f, diag, lv, unused_mx);
    for (int half = 0; half < 2; half++) {
      stage_half(acc, ep, half);
      __syncthreads();
      emit_operand<SPLIT>(ep, dst, hp, m0, n0, half, diag);
      if (!keep_f32) {
        if (diag && threadIdx.x < 128) dg += (double)ep[threadIdx.x * EP_LD + half * 128 + threadIdx.x];
        __syncthreads();
        continue;
      }
      // float32 upper tile, partial sums
      for (int q = threadIdx.x; q < 128 * 64; q += NT) {
        const int row = q >> 6, c4 = (q & 63) * 4;
        const float4 v = *(const float4 *)(ep + row * EP_LD + c4);
        if (keep_f32) gst(gbl(P.accf + (int64_t)(m0 + half * 128 + row) * hp + n0 + c4), v);
        const double w = diag ? 1.0 : 2.0;
        lv += w * ((double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w);
        if (diag) {
          const int d = half * 128 + row - c4;
          if (d >= 0 && d < 4) dg += (double)(d == 0 ? v.x : d == 1 ? v.y : d == 2 ? v.z : v.w);
        }
      }
      __syncthreads();
    }
    if (!diag) nrm = 0.0;
    block_sum3w(lv, dg, nrm, (double *)smem);
    if (threadIdx.x == 0) {
      write_level_partials(P, 1, task, lv, dg);
      if (diag) {
        gptr<double> np = gbl(P.norm_part);
        np[2 * task.tm] = nrm;
        np[2 * task.tm + 1] = 0.0;
      }
    }
    __syncthreads();
  }
}

// One staged half tile (128 rows of float32 at src, row pitch EP_LD, 8 columns per lane, RS rows
// apart per lane group) gets c_last x (itself, rounded as a stored level when ROUND) plus
// w_l x level l of the same tile for l = 1..J, read from global memory (lb: this lane's first
// element of level 1; levels lv_stride bytes apart, rows 2 hp bytes apart). UR row groups per
// pass and levels four at a time: UR x 4 16-byte loads in flight per lane.
template <int UR, bool ROUND>
__device__ __forceinline__ void fold_levels(float *src, gptr<const char> lb, const float *wl, int J, int64_t hp,
                                            int64_t lv_stride, float c_last, float f_store) {
  constexpr int RS = NT / 32, UL = 4;
  for (int it = 0; it < 128 / RS; it += UR) {
    float v[UR][8];
#pragma unroll
    for (int u = 0; u < UR; u++) {
      const float4 a = *(const float4 *)(src + (it + u) * RS * EP_LD);
      const float4 b = *(const float4 *)(src + (it + u) * RS * EP_LD + 4);
      const float x[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
      for (int e = 0; e < 8; e++) v[u][e] = ROUND ? c_last * bf16_value(f_store * x[e]) : c_last * x[e];
    }
    for (int l0 = 1; l0 <= J; l0 += UL) {
      uint4 q[UR][UL];
#pragma unroll
      for (int u = 0; u < UR; u++)
#pragma unroll
        for (int k = 0; k < UL; k++)
          q[u][k] = l0 + k <= J ? gld_u4(lb + (int64_t)uni((it + u) * RS) * hp * 2 + (int64_t)(l0 + k - 1) * lv_stride)
                                : make_uint4(0, 0, 0, 0);
#pragma unroll
      for (int k = 0; k < UL; k++) {
        const float w = l0 + k <= J ? wl[l0 + k] : 0.f;
#pragma unroll
        for (int u = 0; u < UR; u++) {
          const uint32_t qw[4] = {q[u][k].x, q[u][k].y, q[u][k].z, q[u][k].w};
#pragma unroll
          for (int e = 0; e < 4; e++) {
            v[u][2 * e] += w * __uint_as_float(qw[e] << 16);
            v[u][2 * e + 1] += w * __uint_as_float(qw[e] & 0xffff0000u);
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < UR; u++) {
      *(float4 *)(src + (it + u) * RS * EP_LD) = make_float4(v[u][0], v[u][1], v[u][2], v[u][3]);
      *(float4 *)(src + (it + u) * RS * EP_LD + 4) = make_float4(v[u][4], v[u][5], v[u][6], v[u][7]);
    }
  }
}

// Last squaring with the aggregation folded in (level layout): instead of storing level J + 1,
// the tile of P = c_{J+1} S_{J+1} L_{J+1} + sum_{l <= J} c_l S_l L_l is formed from the float32
// accumulators (c_last = c_{J+1} S_J^2 times acc is the first term; the stored level would be
// F_J acc with S_{J+1} = S_J^2 / F_J) and the same tile of each stored level (symmetric, so the
// upper tile gives the mirror too), and stored, tile and mirror, in level slot J + 1. wl[l]
// holds c_l S_l (shared memory). ROUND (e4m3 plans, whose levels are all stored in bf16): the
// last level enters as w_last bf16(f_store acc), exactly as a stored level J + 1 would.
template <bool ROUND = false>
__device__ __forceinline__ void store_p_fused(const f32x16 (&acc)[FM][FN], char *smem, const float *wl,
                                              const ProbDev &P, int J, const Task &task, float c_last,
                                              float f_store = 1.f, bool split_p = false) {
  float *ep = (float *)smem;
  const int m0 = task.tm * BM, n0 = task.tn * BN;
  const bool diag = task.tm == task.tn;
  const int64_t hp = P.hp;
  uint16_t *dst = (uint16_t *)((char *)P.lv + (int64_t)J * P.lv_stride);
  const int row0 = threadIdx.x >> 5, c8 = (threadIdx.x & 31) * 8;  // 32 lanes per staged row
  // unrolled, so that the accumulators are dead while the second half is folded
#pragma unroll
  for (int half = 0; half < 2; half++) {
    stage_half(acc, ep, half);
    __syncthreads();
    float *src = ep + row0 * EP_LD + c8;
    gptr<const char> lb = gbl((const char *)P.lv + ((int64_t)(m0 + half * 128 + row0) * hp + n0 + c8) * 2);
    // two row groups per pass; in the e4m3 squaring (more registers live) one while the second
    // half's accumulators are still held (measured faster there)
    if (ROUND && half == 0) fold_levels<1, ROUND>(src, lb, wl, J, hp, P.lv_stride, c_last, f_store);
    else fold_levels<2, ROUND>(src, lb, wl, J, hp, P.lv_stride, c_last, f_store);
    __syncthreads();
    if (split_p) emit_operand<true>(ep, dst, hp, m0, n0, half, diag);  // [P_hi | P_lo], slots J and J + 1
    else emit_sym_bf16(ep, dst, hp, m0, n0, half, diag, [](float v, int, int) { return v; });
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// squaring (Gram basis and complement basis): level -> level + 1
// ---------------------------------------------------------------------------------------------
// SPLIT (complement basis): the operand is a split pair [D_hi | D_lo]; the product runs over
// K = 3 hp as D_hi D_hi + D_hi D_lo + D_lo D_hi, and the next operand is written split. The
// epilogue's 2 D term reads the same pair (about 16 significant bits), so no float32 copy of
// the levels is kept.
// FUSE (level layout, last squaring only): the aggregation is folded into the epilogue
// (store_p_fused) instead of storing the last level.
template <bool AGG, bool SPLIT = false, bool FUSE = false>
__global__ __launch_bounds__(NT, 1) void kf_square(const StageArgs a) {
  static_assert(!(AGG && SPLIT), "split operands are a complement-basis option");
  static_assert(!FUSE || AGG, "the aggregation folds into level-layout squarings");
  __shared__ __attribute__((aligned(1024))) char smem[SMEM_BYTES];
  __shared__ float wl[kMaxLevels];  // fused aggregation: c_l S_l of the stored levels
  float *ep = (float *)smem;
  const int level = a.level;
  constexpr bool fuse = FUSE;
  int cur_p = -1;
  float f_out = 1.f, c_acc = 0.f, c_first = 0.f, alpha = 1.f, c_next = 0.f, dscale = 1.f;
  __shared__ int s_task;
  TaskCursor cursor(a, &s_task);
  int tg = 0;
  while (cursor.next(a, tg)) {
    Task task = fetch(a, tg, kStageSquare);
    task.p = uni(task.p);
    task.tm = uni(task.tm);
    task.tn = uni(task.tn);
    const ProbDev &P = prob(a, task);
    if (task.p != cur_p) {
      cur_p = task.p;
      const double ls = lsum_load(P);
      const FScalars sc = scalars(ls, a.norm);
      if (a.basis == kGram) {
        const double S = level_scale(ls, sc.sg, level);
        f_out = (float)pow2_inv_round(lsum(ls, level));
        c_acc = (float)(P.coef[level + 1] * S * S);
        c_first = (float)(P.coef[1] * sc.sg);
        if constexpr (fuse) {  // weights of the stored levels 1..J (the same recursion as level_scale)
          double Sl = sc.sg;
          for (int l = 1; l <= level; l++) {
            if (threadIdx.x == 0) wl[l] = (float)(P.coef[l] * Sl);
            Sl = Sl * Sl / pow2_inv_round(lsum(ls, l));
          }
        }
      } else {
        alpha = (float)(level == 1 ? sc.sg * sc.sg : 1.0);
        dscale = (float)(-sc.sg);
        c_next = (float)P.coef[level + 1];
        c_first = (float)P.coef[1];
      }
    }
    const int m0 = task.tm * BM, n0 = task.tn * BN;
    const bool diag = task.tm == task.tn;
    const int64_t hp = P.hp;
    const int64_t ldo = SPLIT ? 2 * hp : hp;  // operand leading dimension
    const uint32_t bytes = (uint32_t)(hp * ldo * 2);
    const void *srcp = AGG ? (const void *)((const char *)P.lv + (int64_t)(level - 1) * P.lv_stride)
                           : (const void *)P.opnd[(level - 1) & 1];
    const Operand op = make_operand(srcp, bytes, (uint32_t)(ldo * 2), P.hp);
    f32x16 acc[FM][FN];
    if constexpr (SPLIT)
      mainloop<false, false, false, KMAP_HHL, KMAP_HLH>(acc, smem, op, m0, op, n0, uni(3 * P.hp), false, uni(P.hp),
                                                       uni(2 * P.hp), uni(2 * P.hp));
    else
      mainloop<false, false>(acc, smem, op, m0, op, n0, uni(P.h), false);
    uint16_t *dst = AGG ? (uint16_t *)((char *)P.lv + (int64_t)level * P.lv_stride) : (uint16_t *)P.opnd[level & 1];
    const bool last = a.last;
    double lv = 0.0, dg = 0.0, unused = 0.0;
    if constexpr (AGG) {
      if constexpr (fuse) store_p_fused<false>(acc, smem, wl, P, level, task, c_acc, 1.f, a.split_p != 0);  // wl written before the mainloop
      else store_level<false>(acc, smem, P, level + 1, task, f_out);
      continue;
    } else {
    for (int half = 0; half < 2; half++) {
      stage_half(acc, ep, half);
      __syncthreads();
      // pass 1 (row-wise, upper tile): new level value `out`, running sum P; the staged value
      // is replaced by what is stored (out, or P on the last level) for the bf16 emit. The
      // float32 reads of a batch are issued together (they do not wait on the batch's stores).
      constexpr int PER = 128 * 64 / NT, BATCH = SPLIT ? 4 : 8;
      for (int b0 = 0; b0 < PER; b0 += BATCH) {
        float4 pin[BATCH], dpv[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; u++) {
          const int q = threadIdx.x + NT * (b0 + u);
          const int row = q >> 6, c4 = (q & 63) * 4;
          const int64_t gi = (int64_t)(m0 + half * 128 + row) * hp + n0 + c4;
          pin[u] = gld_f4(gbl(P.accf + gi));
          if constexpr (SPLIT) {
            // D_level from its split operand (hi + lo) instead of a float32 copy
            if (level > 1) {
              gptr<const uint16_t> so = gbl((const uint16_t *)P.opnd[(level - 1) & 1]) + (int64_t)(m0 + half * 128 + row) * (2 * hp) +
                                   n0 + c4;
              const uint2 h2 = gld_u2(so), l2 = gld_u2(so + hp);
              dpv[u] = make_float4(bf16_pair_lo(h2.x) + bf16_pair_lo(l2.x), bf16_pair_hi(h2.x) + bf16_pair_hi(l2.x),
                                   bf16_pair_lo(h2.y) + bf16_pair_lo(l2.y), bf16_pair_hi(h2.y) + bf16_pair_hi(l2.y));
            }
          } else if (a.basis != kGram && level > 1) {
            dpv[u] = gld_f4(gbl(P.df[level & 1] + gi));
          }
        }
#pragma unroll
        for (int u = 0; u < BATCH; u++) {
          const int q = threadIdx.x + NT * (b0 + u);
          const int row = q >> 6, c4 = (q & 63) * 4;
          float *sp = ep + row * EP_LD + c4;
          const int64_t gi = (int64_t)(m0 + half * 128 + row) * hp + n0 + c4;
          const float4 accv = *(const float4 *)sp;
          float4 outv, pv;
          if (a.basis == kGram) {
            outv = make_float4(f_out * accv.x, f_out * accv.y, f_out * accv.z, f_out * accv.w);
            const float sp0 = level == 1 ? c_first : 1.f;
            pv = make_float4(sp0 * pin[u].x + c_acc * accv.x, sp0 * pin[u].y + c_acc * accv.y,
                             sp0 * pin[u].z + c_acc * accv.z, sp0 * pin[u].w + c_acc * accv.w);
          } else {
            const float4 dprev = level == 1 ? make_float4(dscale * pin[u].x, dscale * pin[u].y, dscale * pin[u].z,
                                                          dscale * pin[u].w)
                                            : dpv[u];
            outv = make_float4(2.f * dprev.x + alpha * accv.x, 2.f * dprev.y + alpha * accv.y,
                               2.f * dprev.z + alpha * accv.z, 2.f * dprev.w + alpha * accv.w);
            const float4 p0 = level == 1 ? make_float4(c_first * dprev.x, c_first * dprev.y, c_first * dprev.z,
                                                       c_first * dprev.w)
                                         : pin[u];
            pv = make_float4(p0.x + c_next * outv.x, p0.y + c_next * outv.y, p0.z + c_next * outv.z,
                             p0.w + c_next * outv.w);
            if (!SPLIT && !last) gst(gbl(P.df[(level + 1) & 1] + gi), outv);
          }
          if (!last) gst(gbl(P.accf + gi), pv);
          const double w = diag ? 1.0 : 2.0;
          lv += w * ((double)outv.x * outv.x + (double)outv.y * outv.y + (double)outv.z * outv.z +
                     (double)outv.w * outv.w);
          if (diag) {
            const int d = half * 128 + row - c4;
            if (d >= 0 && d < 4) dg += (double)(d == 0 ? outv.x : d == 1 ? outv.y : d == 2 ? outv.z : outv.w);
          }
          // split operands: selected per component, since a select of the two float4 values went
          // through the stack (2.7 % of the split squaring); the unsplit kernel allocates its
          // registers better with the plain select (16 % faster than per component)
          if constexpr (SPLIT)
            *(float4 *)sp = make_float4(last ? pv.x : outv.x, last ? pv.y : outv.y, last ? pv.z : outv.z,
                                        last ? pv.w : outv.w);
          else
            *(float4 *)sp = last ? pv : outv;
        }
      }
      __syncthreads();
      emit_operand<SPLIT>(ep, dst, hp, m0, n0, half, diag);
      __syncthreads();
    }
    block_sum3w(lv, dg, unused, (double *)smem);
    if (threadIdx.x == 0) write_level_partials(P, level + 1, task, lv, dg);
    __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------------------------
// e4m3 Gram and squaring: both operands are one e4m3 buffer with one scale s (the Gram: A's
// copy q8, K contiguous; a squaring: its level's copy ql[level & 1], written by the epilogue
// that produced the level); the float32 accumulator holds s^2 times the product, removed by the
// exact power-of-two factor 1/s^2 in the epilogue. Every epilogue stores its level as in the
// bfloat16 level layout and, through store_level<true>, its e4m3 copy for the next squaring,
// with the scale of the largest row sum of squares of the operand codes (qrmax) times the
// epilogue's factor.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ float inv_square(float s) { return 1.f / s / s; }

__global__ __launch_bounds__(NT, 1) void kf_gram8(const StageArgs a) {
  __shared__ __attribute__((aligned(1024))) char smem[SMEM_BYTES];
  __shared__ int s_task;
  TaskCursor cursor(a, &s_task);
  int tg = 0;
  while (cursor.next(a, tg)) {
    Task task = fetch(a, tg, kStageGram);
    task.p = uni(task.p);
    task.tm = uni(task.tm);
    task.tn = uni(task.tn);
    const ProbDev &P = prob(a, task);
    const float dscale = inv_square(P.q_scale[0]);
    const float amax = (float)(dscale * __longlong_as_double((long long)P.qrmax[0]));
    const int ldq = uni((int)P.ldq);
    const Operand op = make_operand(P.q8, (uint32_t)((int64_t)P.h * ldq), (uint32_t)ldq, P.h);
    f32x16 acc[FM][FN];
    mainloop<false, false, true>(acc, smem, op, task.tm * BM, op, task.tn * BN, ldq, false);
    store_level<true>(acc, smem, P, 1, task, dscale, amax);
  }
}

// FUSE: last squaring with the aggregation folded in (store_p_fused, the last level rounded to
// bf16 as a stored level would be).
template <bool FUSE = false>
__global__ __launch_bounds__(NT, 1) void kf_square8(const StageArgs a) {
  __shared__ __attribute__((aligned(1024))) char smem[SMEM_BYTES];
  __shared__ float wl[kMaxLevels];
  const int level = a.level;
  int cur_p = -1;
  float f_out = 1.f, w_last = 0.f, amax_next = 0.f;
  __shared__ int s_task;
  TaskCursor cursor(a, &s_task);
  int tg = 0;
  while (cursor.next(a, tg)) {
    Task task = fetch(a, tg, kStageSquare);
    task.p = uni(task.p);
    task.tm = uni(task.tm);
    task.tn = uni(task.tn);
    const ProbDev &P = prob(a, task);
    if (task.p != cur_p) {
      cur_p = task.p;
      const double ls = lsum_load(P);
      f_out = (float)pow2_inv_round(lsum(ls, level)) * inv_square(P.q_scale[2 * level]);
      amax_next = (float)(f_out * __longlong_as_double((long long)P.qrmax[level]));
      if constexpr (FUSE) {  // c_l S_l of the stored levels 1..J, and c_{J+1} S_{J+1}
        double Sl = scalars(ls, a.norm).sg;
        for (int l = 1; l <= level + 1; l++) {
          const float w = (float)(P.coef[l] * Sl);
          if (l <= level) {
            if (threadIdx.x == 0) wl[l] = w;
            Sl = Sl * Sl / pow2_inv_round(lsum(ls, l));
          } else {
            w_last = w;
          }
        }
      }
    }
    const int64_t hp = P.hp;
    const Operand op = make_operand(P.ql[level & 1], (uint32_t)(hp * hp), (uint32_t)hp, P.hp);
    f32x16 acc[FM][FN];
    mainloop<false, false, true>(acc, smem, op, task.tm * BM, op, task.tn * BN, uni(P.h), false);
    if constexpr (FUSE) store_p_fused<true>(acc, smem, wl, P, level, task, w_last, f_out);
    else store_level<true>(acc, smem, P, level + 1, task, f_out, amax_next);
  }
}

// ---------------------------------------------------------------------------------------------
// product: Y = s (c0 A + P A) in M's orientation (IFNSO only)
// ---------------------------------------------------------------------------------------------
// SPLIT: P is a split pair [P_hi | P_lo] and the product runs over K = 2 hp against M taken twice.
template <bool TRANS, bool SPLIT = false>
__global__ __launch_bounds__(NT, 1) void kf_product(const StageArgs a, const int out_bf16) {
  __shared__ __attribute__((aligned(1024))) char smem[SMEM_BYTES];
  float *ep = (float *)smem;
  int cur_p = -1;
  float sc0 = 0.f, sps = 0.f;
  __shared__ int s_task;
  TaskCursor cursor(a, &s_task);
  int tg = 0;
  while (cursor.next(a, tg)) {
    Task task = fetch(a, tg, kStageProduct);
    task.p = uni(task.p);
    task.tm = uni(task.tm);
    task.tn = uni(task.tn);
    const ProbDev &P = prob(a, task);
    if (task.p != cur_p) {
      cur_p = task.p;
      const FScalars sc = scalars(lsum_load(P), a.norm);
      double c0, ps, sout = sc.sout;
      if (P.h == 1) {
        // a single row or column: the polynomial of the scalar Gram, in float64
        const double g = (a.norm == kNone) ? sc.nA2 : 1.0;
        sout = sc.zero ? 0.0 : (a.norm == kNone ? 1.0 : 1.0 / sqrt(sc.nA2));
        const double b = (a.basis == kGram) ? g : 1.0 - g;
        double v = 0.0;
        for (int k = 0; k < kSlots; k++)
          if (P.coef[k] != 0.0) v += P.coef[k] * pow(b, k == 0 ? 0.0 : exp2((double)(k - 1)));
        c0 = v;
        ps = 0.0;
      } else if (a.basis == kGram) {
        c0 = P.coef[0];
        ps = (a.J == 0 && !a.agg) ? P.coef[1] * sc.sg : 1.0;  // the aggregate stage folds c_1 S_1 into P
      } else {
        c0 = 0.0;
        for (int k = 0; k < kSlots; k++) c0 += P.coef[k];
        ps = (a.J == 0) ? -P.coef[1] * sc.sg : 1.0;
      }
      if (sc.zero && a.norm != kNone) sout = 0.0;
      sc0 = (float)(sout * c0);
      sps = (float)(sout * ps);
    }
    const int64_t hp = P.hp;
    const int m0 = task.tm * BM, n0 = task.tn * BN;
    // M is rows x cols with (rows, cols) = (w, h) when tall, (h, w) when wide; its w index is
    // the output tile's row (tall, K-major) or column (wide, MN-major) index either way
    const uint32_t mbytes = (uint32_t)(((int64_t)(TRANS ? P.w : P.h) - 1) * P.ldm * 2 + (int64_t)(TRANS ? P.h : P.w) * 2);
    const Operand Mo = make_operand(P.M, mbytes, (uint32_t)(P.ldm * 2), P.w);
    const int64_t ldp = SPLIT ? 2 * hp : hp;
    const void *pp = a.agg ? (const void *)((const char *)P.lv + (int64_t)a.p_slot * P.lv_stride) : P.opnd[a.J & 1];
    const Operand Po = make_operand(pp, (uint32_t)(hp * ldp * 2), (uint32_t)(ldp * 2), P.hp);
    const int Kp = uni(P.h);
    f32x16 acc[FM][FN];
    const int rows_out = P.trans ? P.w : P.h, cols_out = P.trans ? P.h : P.w;
    if (a.p_empty || P.h == 1) {
#pragma unroll
      for (int i = 0; i < FM; i++)
#pragma unroll
        for (int j = 0; j < FN; j++)
#pragma unroll
          for (int r = 0; r < 16; r++) acc[i][j][r] = 0.f;
    } else if constexpr (TRANS) {
      // Y_out[n][i] = sum_k M[n][k] P[i][k]
      if constexpr (SPLIT)
        mainloop<false, false, false, KMAP_MOD, KMAP_SEG2>(acc, smem, Mo, m0, Po, n0, uni(2 * P.hp), false, uni(P.hp), Kp,
                                                           uni(2 * P.hp));
      else
        mainloop<false, false>(acc, smem, Mo, m0, Po, n0, Kp, false);
    } else {
      // Y[i][n] = sum_k P[i][k] M[k][n]
      if constexpr (SPLIT)
        mainloop<false, true, false, KMAP_SEG2, KMAP_MOD>(acc, smem, Po, m0, Mo, n0, uni(2 * P.hp), false, uni(P.hp),
                                                          uni(2 * P.hp), Kp);
      else
        mainloop<false, true>(acc, smem, Po, m0, Mo, n0, Kp, false);
    }
    // each thread owns one 8-column chunk of RS rows apart; row offsets are uniform additions.
    // The half tile's M reads are issued before its staging, so they land during it.
    constexpr int RS = NT / 32, PER = 128 / RS;
    const int row0 = threadIdx.x >> 5, c8 = (threadIdx.x & 31) * 8;
    const int c = n0 + c8;
    const bool cin = c < cols_out;
#pragma unroll
    for (int half = 0; half < 2; half++) {
      const int r0 = m0 + half * 128 + row0;
      gptr<const uint16_t> mp = gbl((const uint16_t *)P.M) + (int64_t)r0 * P.ldm + c;
      uint4 xm[PER];
#pragma unroll
      for (int u = 0; u < PER; u++)
        xm[u] = (cin && r0 + u * RS < rows_out) ? gld_u4(mp + (int64_t)uni(u * RS) * P.ldm)
                                                 : make_uint4(0, 0, 0, 0);
      stage_half(acc, ep, half);
      __syncthreads();
      const float *src = ep + row0 * EP_LD + c8;
#pragma unroll
      for (int u = 0; u < PER; u++) {
        if (!cin || r0 + u * RS >= rows_out) continue;
        const float *sp = src + u * RS * EP_LD;
        const uint32_t xw[4] = {xm[u].x, xm[u].y, xm[u].z, xm[u].w};
        float y[8];
#pragma unroll
        for (int e = 0; e < 4; e++) {
          y[2 * e] = sc0 * __uint_as_float(xw[e] << 16) + sps * sp[2 * e];
          y[2 * e + 1] = sc0 * __uint_as_float(xw[e] & 0xffff0000u) + sps * sp[2 * e + 1];
        }
        const int64_t yo = (int64_t)(r0 + u * RS) * P.ldy + c;
        if (out_bf16) {
          gst(gbl((uint16_t *)P.Y + yo), make_uint4(pack_bf16x2(y[0], y[1]), pack_bf16x2(y[2], y[3]),
                                                   pack_bf16x2(y[4], y[5]), pack_bf16x2(y[6], y[7])));
        } else {
          gptr<float> yp = gbl((float *)P.Y + yo);
          gst(yp, make_float4(y[0], y[1], y[2], y[3]));
          gst(yp + 4, make_float4(y[4], y[5], y[6], y[7]));
        }
      }
      __syncthreads();
    }
  }
}


// ---------------------------------------------------------------------------------------------
// aggregate: P = sum_{l=1}^{J+1} c_l S_l B_l (level layout); P overwrites level 1 in place
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void kf_aggregate(const StageArgs a) {
  __shared__ float wsh[kMaxLevels];
  for (int t = blockIdx.x; t < a.ntasks; t += gridDim.x) {
    const Task task = a.tasks ? a.tasks[t] : Task{0, t, 0, 0};
    const ProbDev &P = a.tasks ? a.probs[task.p] : a.one;
    __syncthreads();
    if (threadIdx.x < 64) {  // one wave: level weights c_l S_l in float64, then float32
      const double ls = lsum_load(P);
      const FScalars sc = scalars(ls, a.norm);
      double S = sc.sg;
      for (int l = 1; l <= a.J + 1; l++) {
        if (threadIdx.x == 0) wsh[l] = (float)(P.coef[l] * S);
        if (l <= a.J) {
          const double F = pow2_inv_round(lsum(ls, l));
          S = S * S / F;
        }
      }
    }
    __syncthreads();
    const int64_t n = (int64_t)P.hp * P.hp;
    const int64_t e0 = (int64_t)task.tm * kAggChunk;
    const int64_t e1 = e0 + kAggChunk < n ? e0 + kAggChunk : n;
    const int L = a.J + 1;
    gptr<char> base = gbl((char *)P.lv);
    constexpr int U = 4;  // chunks of 8 elements per thread in flight
    for (int64_t e = e0 + (int64_t)threadIdx.x * 8; e < e1; e += (int64_t)kThreads * 8 * U) {
      float acc[U][8];
#pragma unroll
      for (int u = 0; u < U; u++)
#pragma unroll
        for (int i = 0; i < 8; i++) acc[u][i] = 0.f;
      for (int l = 1; l <= L; l++) {
        const float wl = wsh[l];
        gptr<const uint16_t> src = (gptr<const uint16_t>)(base + (int64_t)(l - 1) * P.lv_stride);
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
          const int64_t ee = e + (int64_t)u * kThreads * 8;
          v[u] = ee < e1 ? gld_u4(src + ee) : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
          const uint32_t w[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
          for (int q = 0; q < 4; q++) {
            acc[u][2 * q] += wl * __uint_as_float(w[q] << 16);
            acc[u][2 * q + 1] += wl * __uint_as_float(w[q] & 0xffff0000u);
          }
        }
      }
      gptr<uint16_t> dst = (gptr<uint16_t>)base;
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int64_t ee = e + (int64_t)u * kThreads * 8;
        if (ee < e1)
          gst(dst + ee, make_uint4(pack_bf16x2(acc[u][0], acc[u][1]), pack_bf16x2(acc[u][2], acc[u][3]),
                                   pack_bf16x2(acc[u][4], acc[u][5]), pack_bf16x2(acc[u][6], acc[u][7])));
      }
    }
  }
}

}  // namespace fast


// Totals of the partial sums that a stage has just written, one workgroup per problem:
// lvl_sum[level] = the upper-tile sum of lvl_part level `level`, and with the Gram (level 1) also
// lvl_sum[0] = the sum of norm_part. Each thread adds a fixed strided subset in order, then the
// lanes and the waves are combined in a fixed order, so the totals do not depend on the schedule
// of the stage before. The tile kernels read these totals (lsum_load) instead of summing the
// partials again in every workgroup that starts on a problem.
__global__ __launch_bounds__(kThreads) void kf_level_sums(const StageArgs a, int batched, int level) {
  const ProbDev &P = batched ? a.probs[blockIdx.x] : a.one;
  __shared__ double red[kThreads / 64][2];
  const int nt = P.nt;
  const int n = nt * nt;
  const double *lp = P.lvl_part + (int64_t)level * n;
  double s = 0.0, t = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    const int r = i / nt, c = i - r * nt;
    if (c >= r) s += lp[i];
  }
  if (level == 1)
    for (int i = threadIdx.x; i < nt; i += kThreads) t += P.norm_part[i];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    s += __shfl_xor(s, off, 64);
    t += __shfl_xor(t, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6][0] = s;
    red[threadIdx.x >> 6][1] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    s = red[0][0];
    t = red[0][1];
    for (int w = 1; w < kThreads / 64; w++) {
      s += red[w][0];
      t += red[w][1];
    }
    P.lvl_sum[level] = s;
    if (level == 1) P.lvl_sum[0] = t;
  }
}

hipError_t launch_level_sums(const StageArgs &a, int nprob, int level, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  hipLaunchKernelGGL(kf_level_sums, dim3(nprob), dim3(kThreads), 0, s, a, a.probs ? 1 : 0, level);
  return hipGetLastError();
}

hipError_t launch_aggregate(const StageArgs &a, int grid, hipStream_t s) {
  if (a.ntasks <= 0) return hipSuccess;
  hipLaunchKernelGGL(fast::kf_aggregate, dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fast_stage(int stage, int trans, const StageArgs &a, int grid, int out_bf16, hipStream_t s) {
  if (a.ntasks <= 0) return hipSuccess;
  const bool split = a.split != 0;
  if (stage == kStageGram) {
    if (trans && split) hipLaunchKernelGGL((fast::kf_gram<true, true>), dim3(grid), dim3(fast::NT), 0, s, a);
    else if (trans) hipLaunchKernelGGL((fast::kf_gram<true, false>), dim3(grid), dim3(fast::NT), 0, s, a);
    else if (split) hipLaunchKernelGGL((fast::kf_gram<false, true>), dim3(grid), dim3(fast::NT), 0, s, a);
    else hipLaunchKernelGGL((fast::kf_gram<false, false>), dim3(grid), dim3(fast::NT), 0, s, a);
  } else if (stage == kStageSquare) {
    if (a.agg && a.fuse_agg && a.last)
      hipLaunchKernelGGL((fast::kf_square<true, false, true>), dim3(grid), dim3(fast::NT), 0, s, a);
    else if (a.agg) hipLaunchKernelGGL((fast::kf_square<true, false>), dim3(grid), dim3(fast::NT), 0, s, a);
    else if (split) hipLaunchKernelGGL((fast::kf_square<false, true>), dim3(grid), dim3(fast::NT), 0, s, a);
    else hipLaunchKernelGGL((fast::kf_square<false, false>), dim3(grid), dim3(fast::NT), 0, s, a);
  } else {
    if (trans && split) hipLaunchKernelGGL((fast::kf_product<true, true>), dim3(grid), dim3(fast::NT), 0, s, a, out_bf16);
    else if (trans) hipLaunchKernelGGL((fast::kf_product<true, false>), dim3(grid), dim3(fast::NT), 0, s, a, out_bf16);
    else if (split) hipLaunchKernelGGL((fast::kf_product<false, true>), dim3(grid), dim3(fast::NT), 0, s, a, out_bf16);
    else hipLaunchKernelGGL((fast::kf_product<false, false>), dim3(grid), dim3(fast::NT), 0, s, a, out_bf16);
  }
  return hipGetLastError();
}

hipError_t launch_e4m3_gemm(int stage, const StageArgs &a, int grid, hipStream_t s) {
  if (a.ntasks <= 0) return hipSuccess;
  if (stage == kStageGram) hipLaunchKernelGGL(fast::kf_gram8, dim3(grid), dim3(fast::NT), 0, s, a);
  else if (a.fuse_agg && a.last) hipLaunchKernelGGL(fast::kf_square8<true>, dim3(grid), dim3(fast::NT), 0, s, a);
  else hipLaunchKernelGGL(fast::kf_square8<false>, dim3(grid), dim3(fast::NT), 0, s, a);
  return hipGetLastError();
}

hipError_t fast_occupancy(int stage, int *blocks_per_cu) {
  const void *fn = stage == kStageGram ? (const void *)fast::kf_gram<false, false>
                 : stage == kStageSquare ? (const void *)fast::kf_square<true, false> : (const void *)fast::kf_product<false, false>;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, fast::NT, 0);
}

}  // namespace ifnso
