// Structures shared by the host scheduler and the device kernels of libifnso.
#pragma once
#include <stdint.h>

namespace ifnso {

constexpr int kMaxTerms = 16;
constexpr int kSlots = 17;       // coefficient slot 0: exponent 0; slot 1 + j: exponent 2^j
constexpr int kMaxLevels = 18;   // levels 1..17 (level l holds B^(2^(l-1)))
constexpr int kThreads = 256;    // generic 128-tile GEMMs and the memory-bound passes: 4 waves of 64
constexpr int kFeat = 8;         // learned mode: traces tr(G^(2^j)), j = 0..7
constexpr int kMaxNsSteps = 16;  // Newton-Schulz step schedules: at most this many (a, b, c)

enum Basis : int32_t { kGram = 0, kComplement = 1 };
// kGelfand2 (Newton-Schulz schedules only): s = ||(A A^T)^2||_F^(1/4), from the partials of a
// norm-only squaring of the raw Gram
enum Norm : int32_t { kFrob = 0, kGramFrob = 1, kNone = 2, kGelfand2 = 3 };
enum OpType : int32_t { kOpF32 = 0, kOpBF16 = 1, kOpFP8 = 2 };

// One problem of a call, rebuilt by the host for every call (pointers move between calls).
struct ProbDev {
  const void *M;       // input, rows x cols, row-major, leading dimension ldm
  void *Y;             // output, same shape and layout as M, leading dimension ldy
  int64_t ldm, ldy;
  int32_t h, w;        // h = min(rows, cols), w = max(rows, cols)
  int32_t trans;       // 1 when rows > cols (A = M^T)
  int32_t hp;          // h padded to the tile grid; leading dimension of every h x h buffer
  int32_t nt;          // tiles along h for the symmetric stages (hp / tile)
  int32_t vecM;        // M and Y allow 16-byte vector access
  void *opnd[2];       // h x h operand ping-pong (operand type), full symmetric
  float *accf;         // h x h float32: Gram (upper tiles), then the running sum P
  float *df[2];        // complement basis, single operands: float32 D levels (upper tiles)
  double *norm_part;   // [nt]         sum of squares of A per row block (diagonal Gram tiles)
  double *lvl_part;    // [levels][nt*nt] sum of squares of the stored level, upper tiles
  double *diag_part;   // [levels][nt]    trace partials of the stored level
  double *lvl_sum;     // [kMaxLevels + 1] totals of the partials, written by a reduction launch
                       //   after the stage that fills them (256-tile kernels): [0] the sum of
                       //   norm_part, [l] the upper-tile sum of lvl_part level l
  double *coef;        // [kSlots] coefficients of this problem (slot layout)
  double *stats;       // [IFNSO_STATS_PER_PROBLEM]
  void *xbuf[2];       // classical NS: h x w iterates (wide orientation), leading dim ldx
  int64_t ldx;
  float *gpart;        // classical NS, split Gram: [tiles][chunks][128 x 128] float32 partial tiles
  double *gnrm;        //   [tiles][chunks][threads] partial sums of squares of A
  uint32_t *gcnt;      //   [tiles] chunks finished (the last one sums the partials, then resets it)
  void *lv;            // level layout: level l (l = 1..J+1) stored at lv + (l-1) * lv_stride bytes,
  int64_t lv_stride;   //   as a full symmetric h x h operand; level 1 later holds P
  // e4m3 compute: per-tensor scaled OCP e4m3 copy of A (h rows, leading dimension ldq, K
  // contiguous, zero beyond w) for the Gram
  uint8_t *q8;
  int64_t ldq;
  // e4m3 copies of the stored levels, written by the epilogue that produces each level: level
  // l in ql[l & 1] (hp x hp, full symmetric), scaled by q_scale[2l]
  uint8_t *ql[2];
  // [kMaxLevels + 1]: the largest sum of squares over a row of the e4m3 values (codes, in
  // their scaled units) of the quantised A ([0]) and of level l ([l]); as float64 bit patterns,
  // raised by atomic maxima (every value is >= 0), zeroed when A is quantised
  uint64_t *qrmax;
  // sums of squares of the codes of A's e4m3 copy per row and chunk, [i * qnch + c], written
  // by the input quantisation (chunks: 1024 columns for wide inputs, one per wave; 64 for tall
  // ones)
  double *qrow_in;
  int32_t qnch;
  double *q_part;      // [nq] pre-pass sums of squares of M, chunks of rq storage rows
  float *q_amax;       // [nq] pre-pass max |M| per chunk
  float *q_scale;      // [2 (kMaxLevels + 1)]: [2l] scale (a power of two) of the e4m3 copy of
                       //   A (l = 0) or of level l, [2l + 1] the maximum it was chosen for
  int32_t nq, rq;
};

// One tile of work: problem index, tile row, tile column, stage-specific flags.
struct Task {
  int32_t p, tm, tn, flags;
};

struct StageArgs {
  const ProbDev *probs;  // device table (batched calls); unused when tasks == nullptr
  const Task *tasks;     // device task list; nullptr: one problem (`one`), tiles decoded on the fly
  int32_t ntasks;
  int32_t level;       // squaring: produces level+1 from level
  int32_t J;           // number of squarings of the plan
  int32_t basis;
  int32_t norm;
  int32_t last;        // squaring stage is the last one
  int32_t learned;     // learned mode: keep levels, defer aggregation
  int32_t ns_step;     // classical NS: step index (-1 for IFNSO)
  int32_t ns_last;     // classical NS: last step
  double ns_abc[3];    // classical NS: (a, b, c) of the current step
  int32_t p_empty;     // product: no terms with exponent >= 1
  int32_t ns_steps;    // classical NS: total steps (used by the h == 1 scalar path)
  int32_t ns_nsched;   // classical NS: entries of ns_sched; step k uses entry min(k, ns_nsched - 1)
  int32_t ns_norm_pass;  // squaring stage: only the float64 partials of ||G_raw^2||_F^2 (slot 2)
  int32_t ksplit;      // generic Gram: K chunks per tile (1: none)
  int32_t kchunk;      // generic Gram: K elements per chunk (a multiple of 128)
  double ns_sched[kMaxNsSteps][3];  // classical NS: the whole schedule (h == 1 scalar path)
  // XCD-aware schedule (fast kernels): workgroup b runs on XCD b % 8 and works through that
  // XCD's task queue tasks[xcd_off[x] .. + xcd_cnt[x]) with stride gridDim.x / 8
  int32_t agg;         // level layout (Gram basis, fast path): levels kept, P formed by the
                       // aggregate stage
  int32_t xcd_sched;
  int32_t xcd_off[8];
  int32_t xcd_cnt[8];
  int32_t wg_per_xcd;  // host only: workgroups per XCD of a fast launch
  int32_t split;       // complement basis, fast path: operands stored as split bf16 pairs
  int32_t fuse_agg;    // level layout: the last squaring forms P (no separate aggregate stage)
  int32_t p_slot;      // level layout: the level slot that holds P for the product
  int32_t split_p;     // level layout: the last squaring stores P as a split pair (hp x 2hp, two slots)
  // With XCD queues: 8 counters (one per queue, zero at launch) from which workgroups take
  // their next task; a workgroup whose queue is empty takes from the others. nullptr: static
  // striding through the workgroup's queue.
  uint32_t *qctr;
  ProbDev one;         // the problem of a single-problem launch
};

}  // namespace ifnso
