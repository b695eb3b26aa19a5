/*
 * ifnso.h -- C ABI of libifnso, an MI355X (gfx950) implementation of IFNSO,
 * the iteration-free Newton-Schulz orthogonalisation of Hu et al.
 * ("IFNSO: Iteration-Free Newton-Schulz Orthogonalization", arXiv 2602.02500).
 *
 * What it computes (for every problem of a plan):
 *   A = M if rows <= cols else M^T                 transposition rule, Sec. 1 and Algorithm 1
 *   X = A / s                                      s = ||A||_F (Eq. (constraint)),
 *                                                  s = ||A A^T||_F^(1/2) (Eq. (new_scale_formula)),
 *                                                  or s = 1
 *   B = X X^T            (IFNSO_BASIS_GRAM,        Eq. (new_unified_formula_0))
 *   B = I - X X^T        (IFNSO_BASIS_COMPLEMENT,  Eq. (after_matrix_formula); with the
 *                                                  Gram-Frobenius scale B is T_1 of Sec. 2.4)
 *   B^(2^j) = (B^(2^(j-1)))^2                      repeated squaring, Sec. 2.4
 *   Y = (sum_k c_k B^(e_k)) X, e_k in {0} u {2^j}  Eq. (generalized_matrix_formula), Algorithm 1
 * and returns Y in M's orientation (Y^T when M was transposed) and layout.
 *
 * Conventions shared by every entry point:
 *  - Matrices are row-major with a leading dimension (elements between the starts of
 *    consecutive rows), ld >= cols.
 *  - M, Y and the workspace are device pointers owned by the caller. The library never
 *    allocates inside a compute call and never synchronises the host; work is enqueued
 *    on the caller's HIP stream (passed as void *, a hipStream_t; NULL = default
 *    stream). Kernel-side faults surface at the caller's next synchronisation.
 *  - Errors are returned as ifnso_status; ifnso_last_error() gives a thread-local
 *    message. Argument checks happen before any HIP call, so an argument error
 *    (INVALID_ARGUMENT, UNSUPPORTED, WORKSPACE_TOO_SMALL) means that nothing was enqueued.
 *  - A zero input matrix gives Y = 0 (no epsilon is added to any normalisation).
 *  - Concurrent calls that share a workspace race; give each in-flight call its own.
 */
#ifndef IFNSO_H
#define IFNSO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IFNSO_OK = 0,
  IFNSO_ERR_INVALID_ARGUMENT = 1,   /* bad pointer, size, descriptor, or plan mismatch */
  IFNSO_ERR_UNSUPPORTED = 2,        /* a valid combination the library does not implement */
  IFNSO_ERR_WORKSPACE_TOO_SMALL = 3,
  IFNSO_ERR_HIP = 4,                /* a HIP runtime call failed; see ifnso_last_error() */
  IFNSO_ERR_INTERNAL = 5
} ifnso_status;

/* element type of M and Y in memory */
typedef enum { IFNSO_F32 = 0, IFNSO_BF16 = 1 } ifnso_dtype;

/* operand type of the matrix products (accumulation is always float32):
 *  F32   float32 operands on the FP32 matrix cores (the plain path; M must be F32)
 *  BF16  bfloat16 operands (M must be BF16)
 *  FP8_E4M3  OCP e4m3 operands (round to nearest even) for the Gram and the squarings, each
 *        with one power-of-two scale per tensor, s = 2^floor(log2(448 / amax)) (exponent
 *        clamped to [-63, 63]): for A its absolute maximum; a stored power X X^T is quantised
 *        where it is produced, with amax its largest magnitude before the bfloat16 rounding,
 *        the largest row sum of squares of the quantised X (the product is positive
 *        semi-definite), which a pass over X's e4m3 copy finds first. ||A||_F comes from a
 *        float64 pre-pass over M; the stored powers, their weighted sum and the final product
 *        use bfloat16. Gram basis only; M must be BF16; problems need h * round_up(w, 16) < 2^31
 *        and h <= 32512. */
typedef enum { IFNSO_COMPUTE_F32 = 0, IFNSO_COMPUTE_BF16 = 1, IFNSO_COMPUTE_FP8_E4M3 = 2 } ifnso_compute;

typedef enum { IFNSO_BASIS_GRAM = 0, IFNSO_BASIS_COMPLEMENT = 1 } ifnso_basis;

typedef enum {
  IFNSO_NORM_FROBENIUS = 0,       /* s = ||A||_F                 Eq. (constraint)          */
  IFNSO_NORM_GRAM_FROBENIUS = 1,  /* s = ||A A^T||_F^(1/2)        Eq. (new_scale_formula)   */
  IFNSO_NORM_NONE = 2             /* s = 1                                                  */
} ifnso_norm;

/* FIXED: the descriptor's coefficients for every problem.
 * LEARNED: per-problem coefficients predicted on the device by a small network (the paper
 *   leaves coefficients that adapt to the input to future work, Sec. 4) from the normalised
 *   traces m_j = tr(G^(2^j))/h, j = 0..7, of the Gram powers the method forms (two extra
 *   squarings supply G^32 and G^64). Requires exponents {0,1,2,4,8,16}, the Gram basis, the
 *   Frobenius norm and bf16 compute; the descriptor's coefficients are the fallback for any
 *   problem whose prediction is not finite. Network: see IFNSO_MLP_NUM_PARAMS below. */
typedef enum { IFNSO_COEFF_FIXED = 0, IFNSO_COEFF_LEARNED = 1 } ifnso_coeff_mode;

enum {
  IFNSO_FLAG_ENFORCE_SUM_ONE = 1, /* reject coefficients with |sum c - 1| > 1e-12 */
  /* Bitwise reproducibility. Always in force: every reduction (norms, traces, level scales,
   * split-K partial tiles) is summed in a fixed order that does not depend on which workgroup
   * runs which tile, so a plan gives the same bits on the same inputs call after call and under
   * any schedule (ifnso_plan_set_config). The flag is accepted and changes nothing. */
  IFNSO_FLAG_DETERMINISTIC = 2,
  /* Gram basis with bf16 compute and at least one squaring: P = sum_{k>=1} c_k B^(e_k) is
   * carried into the final product as a split pair P_hi + P_lo of bf16 values (P_hi = bf16(P),
   * P_lo = bf16(P - P_hi)) and the product forms P_hi A + P_lo A (Algorithm 1's Y = Y' A with Y'
   * held to about 16 significant bits instead of 8). Worth it when the coefficients are large
   * with alternating signs, so that P is much larger than the result. Costs 2x the product work
   * and one more hp x hp level slot of workspace. Needs fixed coefficients and problems that take
   * the 256-tile kernels (as IFNSO_FLAG_SPLIT_BF16; otherwise a call returns
   * IFNSO_ERR_UNSUPPORTED). */
  IFNSO_FLAG_SPLIT_P = 4,
  /* Complement basis with bf16 compute: carry every squaring operand and P as a split pair
   * X = X_hi + X_lo of bf16 values (X_hi = bf16(X), X_lo = bf16(X - X_hi)), so a squaring forms
   * X_hi X_hi + X_hi X_lo + X_lo X_hi (three bf16 products, float32 accumulation) and the
   * product P M as P_hi M + P_lo M. The shifted powers D_l = T^(2^(l-1)) - I of the paper's
   * form (Sec. 2.4, Algorithm 1) are then held to about 16 significant bits instead of 8, which
   * the large alternating coefficients of a depth-14 polynomial need. Costs about 3x the
   * squaring and 2x the product work. Needs fixed coefficients and problems that take the
   * 256-tile kernels (16-byte aligned rows, a multiple of 8 columns; otherwise a call returns
   * IFNSO_ERR_UNSUPPORTED). */
  IFNSO_FLAG_SPLIT_BF16 = 8
};

/* Polynomial descriptor. Arrays are read during ifnso_plan() only (copied). */
typedef struct {
  int32_t num_terms;          /* K, 1..16 */
  const int32_t *exponents;   /* [K] strictly increasing; each 0 or 2^j with j <= 15 */
  const double *coeffs;       /* [K] finite */
  int32_t basis;              /* ifnso_basis */
  int32_t norm;               /* ifnso_norm */
  int32_t compute;            /* ifnso_compute */
  int32_t coeff_mode;         /* ifnso_coeff_mode */
  const float *mlp_params;    /* LEARNED only: host array of IFNSO_MLP_NUM_PARAMS floats (copied) */
  size_t mlp_params_len;      /* must equal IFNSO_MLP_NUM_PARAMS when LEARNED */
  uint32_t flags;             /* IFNSO_FLAG_* */
} ifnso_poly_desc;

typedef struct ifnso_plan_s *ifnso_plan_t;

/* Creates a plan for num_problems matrices of shapes rows[i] x cols[i] (host arrays).
 * The plan validates the descriptor, fixes the orientation of each problem, builds the
 * tile schedules, uploads them and the coefficients to `device`, and sizes the
 * workspace. It owns those device buffers until ifnso_plan_destroy().
 * Errors: INVALID_ARGUMENT (null pointers, num_problems < 1, a dimension < 1,
 * bad exponents/coefficients/enums, LEARNED without a parameter blob of the right
 * length), UNSUPPORTED (dtype/compute combination not implemented), HIP. */
ifnso_status ifnso_plan(const ifnso_poly_desc *desc, int32_t num_problems, const int64_t *rows,
                        const int64_t *cols, int32_t in_dtype, int32_t out_dtype, int32_t device,
                        ifnso_plan_t *out_plan);

/* Bytes of device workspace one call of this plan needs (256-byte aligned base). */
ifnso_status ifnso_plan_workspace_bytes(ifnso_plan_t plan, size_t *bytes);

/* Frees the plan and its device buffers. The caller must make sure no enqueued call of
 * the plan is still running. NULL is accepted. */
ifnso_status ifnso_plan_destroy(ifnso_plan_t plan);

/* Orthogonalises the single problem of a plan made with num_problems == 1.
 * M: device, rows x cols, leading dimension ldm; Y: device, same shape, ldy.
 * Y must not overlap M. Errors: INVALID_ARGUMENT (plan has more than one problem, null
 * or overlapping pointers, ld < cols), WORKSPACE_TOO_SMALL, HIP. */
ifnso_status ifnso_orthogonalize(ifnso_plan_t plan, const void *M, int64_t ldm, void *Y, int64_t ldy,
                                 void *workspace, size_t workspace_bytes, void *stream);

/* ifnso_orthogonalize without a workspace argument, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that forbid allocation).
 * The workspace is a fixed scratch area inside the library, IFNSO_STATIC_SCRATCH_BYTES
 * (64 MiB) on each GPU, held from the library's first use of that GPU until the process ends;
 * the call allocates nothing. Same arguments, layout and result as ifnso_orthogonalize
 * (bitwise), for a plan with num_problems == 1 whose ifnso_plan_workspace_bytes is at most
 * IFNSO_STATIC_SCRATCH_BYTES. Every call on one GPU shares that GPU's area and leaves its
 * contents behind (nothing in it needs to start at zero): calls that overlap on one GPU (on
 * different streams, or from several threads without ordering) race and must be serialised
 * by the caller. Errors: INVALID_ARGUMENT as ifnso_orthogonalize, WORKSPACE_TOO_SMALL when
 * the plan needs more than the area holds, HIP. */
#define IFNSO_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
ifnso_status ifnso_orthogonalize_static(ifnso_plan_t plan, const void *M, int64_t ldm, void *Y, int64_t ldy,
                                        void *stream);

/* Orthogonalises every problem of the plan in one grouped schedule: one persistent
 * launch per stage (Gram, each squaring level, product) over the tiles of all
 * problems, replayed as a HIP graph. M, ldm, Y, ldy are host arrays of length
 * num_problems holding device pointers and leading dimensions.
 * The call's problem table (pointers, leading dimensions, workspace offsets) goes to one of
 * four plan-owned device slots: a call whose table equals a slot's reuses that slot and its
 * captured graph as they are; otherwise the least recently filled slot is refilled in stream
 * order, after a device-side wait for the calls that last read it. The host never blocks. */
ifnso_status ifnso_orthogonalize_batched(ifnso_plan_t plan, const void *const *M, const int64_t *ldm,
                                         void *const *Y, const int64_t *ldy, void *workspace,
                                         size_t workspace_bytes, void *stream);

/* Launch slots of one call of this plan, in order: preparation (in FP8_E4M3 plans the pre-pass
 * (||A||_F and amax) with the e4m3 quantisation of A; empty in other plans), Gram for the
 * problems with rows <= cols, Gram for the
 * transposed (rows > cols) problems, one squaring per level, the aggregation of the weighted
 * powers, then the
 * product for the two groups in the same order: J + 6 slots where 2^J is the largest exponent.
 * A slot with no work in a call launches nothing. The aggregation slot runs only in learned
 * plans and in FP8_E4M3 plans without squarings; the other bfloat16 and FP8_E4M3 Gram-basis
 * plans form the weighted sum in their last squaring, and the remaining plans accumulate it in
 * every squaring. Returns the count, or a negative status for NULL. */
int32_t ifnso_plan_num_launches(ifnso_plan_t plan);

/* Stage of launch slot i (0 Gram, 1 squaring, 2 product, 3 aggregation, 4 preparation, with
 * 0 flops) and its algorithmic
 * flop count: h^2 w per problem for the Gram (symmetric), h^3 per problem for a squaring
 * (symmetric), 2 h^2 w per problem for the product, 0 for the (memory-bound) aggregation.
 * Errors: INVALID_ARGUMENT. */
ifnso_status ifnso_plan_launch_info(ifnso_plan_t plan, int32_t i, int32_t *stage, double *flops);

/* Schedule of a 256-tile stage (bf16 and FP8_E4M3 plans; other plans ignore it). Tiles are
 * ordered in panel-sharing blocks of block_rows x block_cols tiles; with xcd_sched, groups of
 * `group` consecutive tiles are dealt to the 8 XCDs in turn (workgroup b runs on XCD b % 8, so
 * tiles that share operand panels meet in one XCD's L2), and each XCD runs wg_per_xcd
 * workgroups. Defaults: 1, 32, 4, 8, 32. */
typedef struct {
  int32_t xcd_sched;   /* 0 or 1 */
  int32_t group;       /* 1..4096 */
  int32_t block_rows;  /* 1..64 */
  int32_t block_cols;  /* 1..64 */
  int32_t wg_per_xcd;  /* 1..1024 (capped at the XCD's CU count) */
} ifnso_stage_config;

/* Reads / replaces the schedule of stage 0 (Gram), 1 (squaring) or 2 (product). Setting a
 * config synchronises the plan's device, rebuilds the task lists and drops the plan's captured
 * graphs; results are unchanged (every tile is computed the same way whatever the order). For
 * a tuner that times candidate schedules (see the package's tune module).
 * Errors: INVALID_ARGUMENT, HIP. */
ifnso_status ifnso_plan_get_config(ifnso_plan_t plan, int32_t stage, ifnso_stage_config *cfg);
ifnso_status ifnso_plan_set_config(ifnso_plan_t plan, int32_t stage, const ifnso_stage_config *cfg);

/* Measurement hook: the next ifnso_orthogonalize / ifnso_orthogonalize_batched call of this
 * plan records events[i] (hipEvent_t handles created by the caller with timing enabled) on its
 * stream just before launch slot i, and events[num_launches] after the last slot; that call
 * enqueues its kernels directly instead of replaying the graph. count must equal
 * ifnso_plan_num_launches(plan) + 1; count 0 cancels a pending request.
 * Errors: INVALID_ARGUMENT. */
ifnso_status ifnso_plan_launch_events(ifnso_plan_t plan, void *const *events, int32_t count);

/* One Muon optimizer step over the plan's problems, with the plan's polynomial as the
 * orthogonalisation (the paper's setting: Muon orthogonalises momentum updates, Sec. 1; the
 * paper does not restate Muon's update, so this is the reading used):
 *   B <- momentum B + G
 *   U <- G + momentum B   (nesterov = 1)   or   U <- B   (nesterov = 0)
 *   O <- the plan's result for U (U rounded to the plan's input type)
 *   W <- (1 - lr weight_decay) W - lr sqrt(max(1, rows / cols)) O
 * W (weights) and B (momentum) are device float32 matrices of each problem's shape, updated in
 * place; G (gradients) is in the plan's input type. Leading dimensions >= cols. W, B and G must
 * not overlap. The workspace (ifnso_muon_workspace_bytes, 256-byte aligned) holds the plan's
 * workspace followed by U, O and a problem table; concurrent steps need their own workspaces.
 * Enqueued on `stream`; the call returns when the work is queued.
 * Errors: INVALID_ARGUMENT, WORKSPACE_TOO_SMALL, UNSUPPORTED (as for the plan's calls), HIP. */
typedef struct {
  double lr;            /* learning rate */
  double momentum;      /* momentum coefficient */
  double weight_decay;  /* decoupled weight decay */
  int32_t nesterov;     /* 0 or 1 */
} ifnso_muon_params;

ifnso_status ifnso_muon_workspace_bytes(ifnso_plan_t plan, size_t *bytes);
ifnso_status ifnso_muon_step(ifnso_plan_t plan, const ifnso_muon_params *params, float *const *W,
                             const int64_t *ldw, const void *const *G, const int64_t *ldg, float *const *B,
                             const int64_t *ldb, void *workspace, size_t workspace_bytes, void *stream);

/* Classical Newton-Schulz with one odd quintic per step, Eq. (iteration_jordan):
 *   X_0 = A / ||A||_F,  X_{k+1} = a X_k + (b G_k + c G_k^2) X_k,  G_k = X_k X_k^T,
 * for `steps` steps (abc = {a, b, c}; {1.5, -0.5, 0} is the cubic of
 * Eq. (one_iteration_matrix)). M: device rows x cols (ldm), dtype `dtype` (F32 with
 * compute F32, BF16 with compute BF16); Y: device, same shape and dtype, ldy. workspace:
 * device, 256-byte aligned, ifnso_classical_ns_workspace_bytes bytes, owned by the caller; its
 * contents on entry do not matter (the call clears the counters it uses before its first
 * launch), and two calls that overlap in time must not share it.
 * Errors: INVALID_ARGUMENT, UNSUPPORTED, WORKSPACE_TOO_SMALL, HIP. */
ifnso_status ifnso_classical_ns(const void *M, int64_t rows, int64_t cols, int64_t ldm, int32_t dtype,
                                void *Y, int64_t ldy, int32_t steps, const double abc[3], int32_t compute,
                                void *workspace, size_t workspace_bytes, void *stream);

/* Workspace bytes for ifnso_classical_ns with these dimensions (0 on bad arguments). */
size_t ifnso_classical_ns_workspace_bytes(int64_t rows, int64_t cols, int32_t compute);

/* Most steps of one ifnso_ns_schedule call. */
#define IFNSO_NS_MAX_STEPS 16

/* Newton-Schulz with its own odd quintic at every step: the iterations the paper compares
 * against in Sec. 2 (Cesista's iteration-specific coefficients, CANS' minimax polynomials),
 * in the form of Eq. (iteration_jordan):
 *   X_0 = A / s,  X_{k+1} = a_k X_k + (b_k G_k + c_k G_k^2) X_k,  G_k = X_k X_k^T,
 * with A oriented as in Sec. 1 (h <= w) and the result returned in M's orientation.
 * s = ||A||_F (gelfand_q = 0, Eq. (constraint)), or Gelfand's bound of Eq. (gelfand_formula)
 * and Eq. (scale_formula_function), s = ||(A A^T)^q||_F^(1/(2q)), for q = gelfand_q = 1 or 2
 * (q = 2 adds one h x h squaring of the raw Gram at the first step, for its norm only).
 * abc: host array of `steps` triples {a_k, b_k, c_k}, read during the call; 1 <= steps <=
 * IFNSO_NS_MAX_STEPS. M, Y, dtype, compute, workspace (ifnso_classical_ns_workspace_bytes
 * bytes) and stream as for ifnso_classical_ns; a zero input gives a zero output.
 * Errors: INVALID_ARGUMENT (NULL pointers, bad shapes, steps out of range, gelfand_q < 0,
 * non-finite coefficients, Y overlapping M), UNSUPPORTED (gelfand_q > 2, dtype/compute
 * pairs other than F32/F32 and BF16/BF16), WORKSPACE_TOO_SMALL, HIP. */
ifnso_status ifnso_ns_schedule(const void *M, int64_t rows, int64_t cols, int64_t ldm, int32_t dtype, void *Y,
                               int64_t ldy, int32_t steps, const double *abc, int32_t gelfand_q, int32_t compute,
                               void *workspace, size_t workspace_bytes, void *stream);

/* Newton-Schulz step schedules over a batch, on the batched path: step k,
 *   X_{k+1} = a_k X_k + b_k (X_k X_k^T) X_k + c_k (X_k X_k^T)^2 X_k   (Eq. (iteration_jordan)),
 * is a Gram-basis plan with exponents {0, 1, 2} ({0, 1} when c_k = 0) and coefficients
 * (a_k, b_k, c_k); the first step normalises by ||A||_F (gelfand_q = 0, Eq. (constraint)) or
 * ||A A^T||_F^(1/2) (gelfand_q = 1, Gelfand's bound of Eq. (scale_formula_function) with q = 1),
 * the others not at all. Steps with the same triple share one plan. The iterates between steps
 * are stored in `dtype` (as the single-matrix schedule of ifnso_ns_schedule stores them),
 * alternating between the workspace and Y so that the last step writes Y.
 * abc: host array of `steps` triples (copied), 1 <= steps <= IFNSO_NS_MAX_STEPS; rows, cols:
 * host arrays of num_problems shapes; dtype is the storage type of M, Y and the iterates
 * (F32 with COMPUTE_F32, BF16 with COMPUTE_BF16). Errors: INVALID_ARGUMENT (NULL pointers,
 * steps out of range, gelfand_q < 0, non-finite coefficients, bad shapes or dtype),
 * UNSUPPORTED (gelfand_q > 1, and what ifnso_plan refuses), HIP. */
typedef struct ifnso_schedule_plan_s *ifnso_schedule_plan_t;
ifnso_status ifnso_schedule_plan(const double *abc, int32_t steps, int32_t gelfand_q, int32_t num_problems,
                                 const int64_t *rows, const int64_t *cols, int32_t dtype, int32_t compute,
                                 int32_t device, ifnso_schedule_plan_t *out_plan);

/* Bytes of device workspace one call needs (256-byte aligned base): the largest step plan's
 * workspace, then (with more than one step) one iterate buffer per problem. */
ifnso_status ifnso_schedule_plan_workspace_bytes(ifnso_schedule_plan_t plan, size_t *bytes);

/* Frees the schedule plan and its step plans; no enqueued call may still be running. NULL is
 * accepted. */
ifnso_status ifnso_schedule_plan_destroy(ifnso_schedule_plan_t plan);

/* Runs the schedule on every problem: M, ldm, Y, ldy as for ifnso_orthogonalize_batched. Each
 * step is one batched call of its plan (stream-ordered on `stream`; the host never blocks). M
 * and Y must not overlap the workspace. Errors: INVALID_ARGUMENT, WORKSPACE_TOO_SMALL, HIP. */
ifnso_status ifnso_schedule_orthogonalize_batched(ifnso_schedule_plan_t plan, const void *const *M,
                                                  const int64_t *ldm, void *const *Y, const int64_t *ldy,
                                                  void *workspace, size_t workspace_bytes, void *stream);

/* The input side of the FP8_E4M3 mode on its own: A (= M, or M^T when rows > cols; h x w,
 * h <= w) quantised to OCP e4m3 with the per-tensor power-of-two scale of ifnso_compute,
 * Q[i][k] = e4m3(s A[i][k]) for k < w and 0 for w <= k < round_up(w, 16): the K-major operand
 * the e4m3 Gram reads. M: device BF16, rows x cols, ldm. Q: device, h rows of ldq bytes
 * (ldq >= round_up(w, 16), ldq % 16 == 0, 16-byte aligned). out3: device double[3] =
 * {||A||_F^2 (float64 sum), max |A|, s}. Workspace: device, 256-byte aligned,
 * ifnso_quantize_e4m3_workspace_bytes(rows, cols) bytes.
 * Errors: INVALID_ARGUMENT, UNSUPPORTED (h * ldq >= 2^31), WORKSPACE_TOO_SMALL, HIP. */
ifnso_status ifnso_quantize_e4m3(const void *M, int64_t rows, int64_t cols, int64_t ldm, void *Q, int64_t ldq,
                                 double *out3, void *workspace, size_t workspace_bytes, void *stream);
size_t ifnso_quantize_e4m3_workspace_bytes(int64_t rows, int64_t cols);

/* Orthogonality error of the Experiment section, e = ||Z Z^T - I||_F with Z = Y in the
 * h <= w orientation, computed on the device in float64 for `count` matrices (host arrays
 * of device pointers, shapes and leading dimensions; one dtype for all). Writes `count`
 * doubles to the device array `out`. Z Z^T is formed on the float64 matrix cores
 * (v_mfma_f64_16x16x4f64, upper 64 x 64 tiles, float64 accumulation throughout). The device
 * workspace must hold ifnso_orth_error_workspace_bytes(count) bytes (256-byte aligned). Evaluation helper,
 * not part of the timed path: it synchronises `stream` before returning.
 * Errors: INVALID_ARGUMENT, WORKSPACE_TOO_SMALL, HIP. */
ifnso_status ifnso_orth_error(int32_t count, const void *const *Y, const int64_t *rows, const int64_t *cols,
                              const int64_t *ldy, int32_t dtype, double *out, void *workspace,
                              size_t workspace_bytes, void *stream);
size_t ifnso_orth_error_workspace_bytes(int32_t count);

/* Per-problem statistics of the most recent call of a plan, copied to the host array
 * host_out[num_problems * IFNSO_STATS_PER_PROBLEM] after synchronising `stream`. Filled by
 * LEARNED plans: [0] ||A||_F^2, [1..8] log2 m_j for j = 0..7, [9..24] the coefficient slots used
 * (slot 0: exponent 0, slot 1 + j: exponent 2^j), [25] 1 if the network's coefficients were used,
 * 0 if the fixed fallback was. Zero for FIXED plans. Errors: INVALID_ARGUMENT, HIP. */
#define IFNSO_STATS_PER_PROBLEM 26
ifnso_status ifnso_plan_stats(ifnso_plan_t plan, double *host_out, void *stream);

/* ---- the coefficient network ---------------------------------------------------------------
 * phi_j = log2(m_j) / (8 * 2^j) (j = 0..7) -> 64 -> gelu -> 64 -> gelu -> 6 -> projection
 * c = z + (1 - sum z)/6 onto sum c = 1. gelu is the exact-erf form. Parameter layout (float32,
 * row-major, output-major weights): W1[64][8], b1[64], W2[64][64], b2[64], W3[6][64], b3[6]. */
#define IFNSO_MLP_NUM_PARAMS 5126

/* Features phi (device float[n][8]) of n spectra: sig is device float[n][smax] holding the
 * singular values of each matrix (any scale; zero-padded), nsig device int32[n] their counts
 * (= h). Evaluated in float64 log space. Errors: INVALID_ARGUMENT, HIP. */
ifnso_status ifnso_mlp_features(int32_t n, const float *sig, const int32_t *nsig, int32_t smax, float *feats_out,
                                void *stream);

/* Network outputs (device double[n][6], coefficients for exponents 0,1,2,4,8,16) for n feature
 * vectors (device float[n][8]) with parameters `params` (device). Errors: INVALID_ARGUMENT, HIP. */
ifnso_status ifnso_mlp_forward(int32_t n, const float *feats, const float *params, double *coeffs_out,
                               void *stream);

/* One training step on the device for a batch of n samples: forward, the spectral loss
 * (1/h) sum_i (s_i p(s_i^2) - 1)^2 over the normalised singular values s (the squared Frobenius
 * distance to the polar factor, over h), backward, a mean gradient reduced in sample order, and
 * one Adam update of params / adam_m / adam_v (device float[IFNSO_MLP_NUM_PARAMS], in place;
 * t >= 1 is the step number for bias correction). grad_out (device float[IFNSO_MLP_NUM_PARAMS])
 * and loss_out (device float[1]) are optional. Deterministic. Workspace: device,
 * ifnso_mlp_train_workspace_bytes(n) bytes. Errors: INVALID_ARGUMENT, WORKSPACE_TOO_SMALL, HIP. */
ifnso_status ifnso_mlp_train_step(int32_t n, const float *feats, const float *sig, const int32_t *nsig, int32_t smax,
                                  float *params, float *adam_m, float *adam_v, int32_t t, float lr, float beta1,
                                  float beta2, float eps, float *grad_out, float *loss_out, void *workspace,
                                  size_t workspace_bytes, void *stream);
size_t ifnso_mlp_train_workspace_bytes(int32_t n);

/* Thread-local message describing the last error returned on this thread. */
const char *ifnso_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* IFNSO_H */
