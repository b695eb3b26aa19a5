// Internal interface between the host scheduler and the kernel translation unit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ifnso_common.hpp"

namespace ifnso {

enum Stage : int { kStageGram = 0, kStageSquare = 1, kStageProduct = 2, kStageAggregate = 3, kStagePrep = 4 };

struct OrthEntry {
  const void *ptr;
  int64_t rows, cols, ld;
};

struct OrthArgs {
  const OrthEntry *e;  // [count], device
  double *part;        // [count][nsplit], device
  double *out;         // [count], device
  int32_t nsplit;
  int32_t count;
};

hipError_t launch_stage(int op, int ts, int stage, const StageArgs &a, int grid, int out_bf16, hipStream_t s);
// n zero words at p (device), as a kernel (no memset node when captured in a graph)
hipError_t launch_zero_u32(uint32_t *p, int n, hipStream_t s);
hipError_t stage_occupancy(int op, int ts, int stage, int *blocks_per_cu);
// bfloat16 fast path, 256 x 256 tiles (see ifnso_fast.hip for the operand requirements)
hipError_t launch_fast_stage(int stage, int trans, const StageArgs &a, int grid, int out_bf16, hipStream_t s);
hipError_t fast_occupancy(int stage, int *blocks_per_cu);
// P = sum_l c_l S_l B_l over the stored levels (level layout); tasks are (problem, chunk)
hipError_t launch_aggregate(const StageArgs &a, int grid, hipStream_t s);
// 256-tile kernels: per-problem totals of the partials of level `level` (and of the norm with
// the Gram, level 1) into ProbDev::lvl_sum, one workgroup per problem.
hipError_t launch_level_sums(const StageArgs &a, int nprob, int level, hipStream_t s);
constexpr int kAggChunk = 1 << 17;  // elements per aggregate task

// e4m3 compute (ifnso_fp8.hip): memory-bound passes, one grid row per problem
enum E4m3Pass : int { kE4m3Prepass = 0, kE4m3QuantInput = 1, kE4m3RowMax = 2 };
// rows of an e4m3 operand that one workgroup of the row-maxima pass covers
constexpr int kQRowsPerBlock = 64;
hipError_t launch_e4m3_pass(int which, const StageArgs &a, int nprob, int per_problem, hipStream_t s);
// device out[3] = {||A||_F^2, max |A|, scale} of a single-problem pass
hipError_t launch_e4m3_export(const ProbDev &P, double *out, hipStream_t s);
// e4m3 Gram (level 1 from q8) and squaring (level+1 from the quantised level) on 256 tiles
hipError_t launch_e4m3_gemm(int stage, const StageArgs &a, int grid, hipStream_t s);
constexpr int kFastTS = 256;

// learned coefficients (ifnso_mlp.hip)
constexpr int kMlpParams = 5126;
hipError_t launch_mlp_features(int n, const float *sig, const int32_t *nsig, int smax, float *feats, hipStream_t s);
hipError_t launch_mlp_forward(int n, const float *feats, const float *params, double *coeffs, hipStream_t s);
hipError_t launch_mlp_train(int n, const float *feats, const float *sig, const int32_t *nsig, int smax, float *params,
                            float *m, float *v, int t, float lr, float b1, float b2, float eps, float *gout,
                            float *lout, float *grads, float *losses, hipStream_t s);
hipError_t launch_learned(const StageArgs &a, int nprob, const float *params, const double *fixed_slots,
                          hipStream_t s);

hipError_t launch_orth_error(const OrthArgs &a, int bf16, hipStream_t s);

// The fixed scratch area of ifnso_orthogonalize_static (ifnso_static.hip): its device address
// on `device`, resolved once per device (that device made current for the lookup).
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
hipError_t static_scratch(int device, void **ptr);
// bytes (a multiple of 4) from host memory to device memory `dst`, in stream order, through
// kernel arguments: `src` may be reused as soon as the call returns
hipError_t upload_table(void *dst, const void *src, size_t bytes, hipStream_t s);

// Muon step around a batched orthogonalisation (ifnso_muon.hip)
struct MuonProb {
  float *W;         // rows x cols float32, leading dimension ldw
  const void *G;    // gradient, the plan's input type, ldg
  float *B;         // momentum, float32, ldb
  void *U;          // orthogonalisation input (plan's input type), ldu
  const void *Y;    // orthogonalised update (plan's output type), ldy
  int64_t rows, cols, ldw, ldg, ldb, ldu, ldy;
  float step;       // lr * sqrt(max(1, rows / cols))
  int32_t vec;      // cols % 4 == 0, every leading dimension % 4 == 0 and 16-byte aligned bases
};

struct MuonArgs {
  const MuonProb *probs;  // device table
  float momentum;
  float decay;            // 1 - lr * weight_decay
  int32_t nesterov;
  int32_t in_bf16;        // G and U are bfloat16 (else float32)
  int32_t out_bf16;       // Y is bfloat16 (else float32)
};

// B = momentum B + G; U = Nesterov ? G + momentum B : B (one grid row per problem)
hipError_t launch_muon_pre(const MuonArgs &a, int nprob, int per_problem, hipStream_t s);
// W = decay W - step Y
hipError_t launch_muon_post(const MuonArgs &a, int nprob, int per_problem, hipStream_t s);

}  // namespace ifnso
