// Host side of libifnso: plans, argument checks, workspace layout, tile schedules,
// per-call problem tables, HIP-graph replay and the C ABI declared in ifnso.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ifnso.h"
#include "ifnso_common.hpp"
#include "ifnso_launch.hpp"

using namespace ifnso;

namespace {

thread_local std::string g_last_error;

ifnso_status fail(ifnso_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(IFNSO_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int kStatsPerProblem = 32;
constexpr int kSlotsRing = 4;  // per-call problem tables in flight per plan

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

size_t op_size(int op) { return op == kOpF32 ? 4 : (op == kOpBF16 ? 2 : 1); }

// Tile size of the symmetric stages and the product; every h x h buffer is padded to a
// multiple of kPad so that all stage kernels read it without bounds checks.
constexpr int kTS = 128;
constexpr int kPad = 256;

struct ProbLayout {
  int64_t rows, cols;
  int32_t h, w, trans, hp, nt;
  size_t off_opnd[2], off_accf, off_df[2], off_norm, off_lvl, off_diag, off_lsum, off_xbuf[2], off_lv;
  int64_t ldx, lv_stride;
  // the generic Gram split along K (ksplit chunks of kchunk columns) when it has few tiles
  int32_t ksplit, kchunk;
  size_t off_gpart, off_gnrm, off_gcnt;
  // e4m3 compute
  size_t off_q8, off_ql[2], off_qrmax, off_qrow_in, off_qpart, off_qamax, off_qscale;
  int32_t qnch;
  int64_t ldq;
  int32_t nq, rq;
  size_t bytes;
};

// e4m3 pre-pass chunks: about kQElems elements (whole storage rows) each
constexpr int64_t kQElems = 1 << 16;
constexpr int kQScaleFloats = 2 * (kMaxLevels + 1);

void e4m3_chunks(int64_t rows, int64_t cols, int32_t &rq, int32_t &nq) {
  rq = (int32_t)std::max<int64_t>(1, kQElems / cols);
  nq = (int32_t)((rows + rq - 1) / rq);
}

// K chunks of the generic Gram (Newton-Schulz, and single-problem plans on the generic kernels).
// A single problem with few 128-tiles leaves most CUs idle while each tile runs the whole long
// dimension, so the Gram is split into up to 16 chunks of at least 256 columns (a multiple of 128
// each), aiming at about one workgroup per CU.
static void gram_ksplit(int nt, int64_t w, int32_t &S, int32_t &kchunk) {
  const int64_t nsym = (int64_t)nt * (nt + 1) / 2;
  const int64_t want = std::min<int64_t>(16, std::min<int64_t>((256 + nsym - 1) / nsym, (w + 255) / 256));
  if (want <= 1) {
    S = 1;
    kchunk = (int32_t)w;
    return;
  }
  kchunk = (int32_t)round_up((w + want - 1) / want, 128);
  S = (int32_t)((w + kchunk - 1) / kchunk);
}

// Workspace layout of one problem. levels = J + 2 partial slots; the complement basis adds the
// float32 D ping-pong unless its operands are split; classical NS adds two h x w iterates.
ProbLayout layout_problem(int64_t rows, int64_t cols, int op, int J, bool complement, bool ns, bool agg = false,
                          bool e4m3 = false, bool split = false, bool gsplit = false, bool split_p = false) {
  ProbLayout L{};
  L.rows = rows;
  L.cols = cols;
  L.trans = rows > cols;
  L.h = (int32_t)std::min(rows, cols);
  L.w = (int32_t)std::max(rows, cols);
  L.hp = (int32_t)round_up(L.h, kPad);
  L.nt = L.hp / kTS;
  const size_t hh = (size_t)L.hp * L.hp;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes, kAlign);
    return at;
  };
  if (agg) {
    // level layout: J + 1 full symmetric bf16 levels; the first one doubles as the Gram
    // operand and, after the aggregate stage, as P. A split P (hp x 2hp) takes slots J and J + 1.
    L.lv_stride = (int64_t)align_up(hh * op_size(op), kAlign);
    L.off_lv = take((size_t)(J + (split_p ? 2 : 1)) * L.lv_stride);
    L.off_opnd[0] = L.off_lv;
    L.off_opnd[1] = L.off_lv;
    L.off_accf = L.off_lv;  // never written in the level layout
  } else {
    // split operands: hp x 2hp, [X_hi | X_lo] per row
    L.off_opnd[0] = take(hh * op_size(op) * (split ? 2 : 1));
    L.off_opnd[1] = take(hh * op_size(op) * (split ? 2 : 1));
    L.off_accf = take(hh * 4);
  }
  if (complement && !split) {  // split plans read D_l from its split operand
    L.off_df[0] = take(hh * 4);
    L.off_df[1] = take(hh * 4);
  }
  const int levels = J + 2;
  L.off_norm = take((size_t)L.nt * 8);
  L.off_lvl = take((size_t)levels * L.nt * L.nt * 8);
  L.off_diag = take((size_t)levels * L.nt * 8);
  L.off_lsum = take((size_t)(kMaxLevels + 1) * 8);
  if (ns) {
    L.ldx = round_up(L.w, 8);
    L.off_xbuf[0] = take((size_t)L.h * L.ldx * op_size(op));
    L.off_xbuf[1] = take((size_t)L.h * L.ldx * op_size(op));
  }
  if (ns || gsplit) {
    gram_ksplit(L.nt, L.w, L.ksplit, L.kchunk);
    if (L.ksplit > 1) {
      const size_t tiles = (size_t)L.nt * (L.nt + 1) / 2;
      L.off_gpart = take(tiles * L.ksplit * kTS * kTS * 4);
      L.off_gnrm = take(tiles * L.ksplit * kThreads * 8);
      L.off_gcnt = take(tiles * 4);
    }
  }
  if (e4m3) {
    // A (h x ldq) for the Gram; two level buffers (hp x hp), level l in slot l & 1 (a squaring
    // reads one slot and writes the other)
    L.ldq = round_up(L.w, 16);
    e4m3_chunks(rows, cols, L.rq, L.nq);
    L.off_q8 = take((size_t)L.h * L.ldq);
    for (int i = 0; i < 2; i++) L.off_ql[i] = take(hh);
    L.off_qrmax = take((size_t)(kMaxLevels + 1) * 8);
    L.qnch = (int32_t)(L.trans ? (L.ldq + 63) / 64 : (L.ldq / 16 + 63) / 64);  // see ProbDev::qrow_in
    L.off_qrow_in = take((size_t)L.h * L.qnch * 8);
    L.off_qpart = take((size_t)L.nq * 8);
    L.off_qamax = take((size_t)L.nq * 4);
    L.off_qscale = take(kQScaleFloats * 4);
  }
  L.bytes = o;
  return L;
}

void fill_dev(ProbDev &d, const ProbLayout &L, char *ws, const void *M, int64_t ldm, void *Y, int64_t ldy,
              int op, double *coef, double *stats) {
  std::memset(&d, 0, sizeof d);
  d.M = M;
  d.Y = Y;
  d.ldm = ldm;
  d.ldy = ldy;
  d.h = L.h;
  d.w = L.w;
  d.trans = L.trans;
  d.hp = L.hp;
  d.nt = L.nt;
  const size_t es = op_size(op);
  d.vecM = ((uintptr_t)M % 16 == 0) && ((size_t)ldm * es % 16 == 0);
  d.opnd[0] = ws + L.off_opnd[0];
  d.opnd[1] = ws + L.off_opnd[1];
  d.accf = (float *)(ws + L.off_accf);
  d.df[0] = L.off_df[0] ? (float *)(ws + L.off_df[0]) : nullptr;
  d.df[1] = L.off_df[1] ? (float *)(ws + L.off_df[1]) : nullptr;
  d.norm_part = (double *)(ws + L.off_norm);
  d.lvl_part = (double *)(ws + L.off_lvl);
  d.diag_part = (double *)(ws + L.off_diag);
  d.lvl_sum = (double *)(ws + L.off_lsum);
  d.coef = coef;
  d.stats = stats;
  d.xbuf[0] = L.off_xbuf[0] ? ws + L.off_xbuf[0] : nullptr;
  d.xbuf[1] = L.off_xbuf[1] ? ws + L.off_xbuf[1] : nullptr;
  d.ldx = L.ldx;
  d.gpart = L.off_gpart ? (float *)(ws + L.off_gpart) : nullptr;
  d.gnrm = L.off_gnrm ? (double *)(ws + L.off_gnrm) : nullptr;
  d.gcnt = L.off_gcnt ? (uint32_t *)(ws + L.off_gcnt) : nullptr;
  d.lv = L.lv_stride ? ws + L.off_lv : nullptr;
  d.lv_stride = L.lv_stride;
  if (L.ldq) {
    d.q8 = (uint8_t *)(ws + L.off_q8);
    d.ldq = L.ldq;
    d.q_part = (double *)(ws + L.off_qpart);
    d.q_amax = (float *)(ws + L.off_qamax);
    for (int i = 0; i < 2; i++) d.ql[i] = (uint8_t *)(ws + L.off_ql[i]);
    d.qrmax = (uint64_t *)(ws + L.off_qrmax);
    d.qrow_in = (double *)(ws + L.off_qrow_in);
    d.qnch = L.qnch;
    d.q_scale = (float *)(ws + L.off_qscale);
    d.nq = L.nq;
    d.rq = L.rq;
  }
}

bool ranges_overlap(const void *a, size_t na, const void *b, size_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

size_t matrix_bytes(int64_t rows, int64_t ld, int64_t cols, size_t es) {
  return ((size_t)(rows - 1) * ld + cols) * es;
}

int dev_cus(int device) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess) return 256;
  return p.multiProcessorCount;
}

int grid_for(int op, int stage, int ntasks, int cus) {
  int occ = 1;
  if (stage_occupancy(op, kTS, stage, &occ) != hipSuccess || occ < 1) occ = 1;
  return std::max(1, std::min(ntasks, occ * cus));
}



// Tiles of one problem in panel-sharing blocks of br x bc tiles (row-major inside a block,
// blocks row-major); `upper` keeps only tiles with tn >= tm.
constexpr int kXcds = 8;

void block_order(std::vector<Task> &out, int p, int rows, int cols, bool upper, int br_, int bc_) {
  for (int br = 0; br < rows; br += br_)
    for (int bc = upper ? (br / bc_) * bc_ : 0; bc < cols; bc += bc_)
      for (int tm = br; tm < std::min(rows, br + br_); tm++)
        for (int tn = bc; tn < std::min(cols, bc + bc_); tn++)
          if (!upper || tn >= tm) out.push_back(Task{p, tm, tn, 0});
}

// Deals groups of `group` consecutive tiles to the XCDs in turn; returns the tasks grouped
// by XCD with per-XCD offsets (relative to the start of the returned list) and counts.
std::vector<Task> xcd_queues(const std::vector<Task> &tiles, int group, int off[kXcds], int cnt[kXcds]) {
  std::vector<std::vector<Task>> q(kXcds);
  for (size_t g = 0; g * group < tiles.size(); g++) {
    const size_t b = g * group, e = std::min(tiles.size(), b + group);
    q[g % kXcds].insert(q[g % kXcds].end(), tiles.begin() + b, tiles.begin() + e);
  }
  std::vector<Task> out;
  for (int x = 0; x < kXcds; x++) {
    off[x] = (int)out.size();
    cnt[x] = (int)q[x].size();
    out.insert(out.end(), q[x].begin(), q[x].end());
  }
  return out;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------------------------

struct ifnso_plan_s {
  int device = 0;
  int num = 0;
  int K = 0;
  int32_t exps[kMaxTerms] = {};
  double coeffs[kMaxTerms] = {};
  double slots[kSlots] = {};
  int basis = 0, norm = 0, op = 0, coeff_mode = 0;
  uint32_t flags = 0;
  int in_dtype = 0, out_dtype = 0;
  int J = 0;
  bool p_empty = false;
  std::vector<ProbLayout> lay;
  std::vector<size_t> ws_off;  // per-problem offset into the workspace
  size_t ws_bytes = 0;
  // device schedule: generic (128 tiles) and fast (256 tiles, bfloat16) task lists
  Task *d_tasks = nullptr;
  int n_gram = 0, n_square = 0, n_prod = 0;
  size_t off_gram = 0, off_square = 0, off_prod = 0;
  bool fast = false;  // bfloat16 plan whose squarings use the fast kernels
  bool agg = false;   // level layout + aggregate stage (fast, Gram basis, J >= 1)
  bool learned = false;
  bool e4m3 = false;  // e4m3 Gram and squarings (level layout), bfloat16 aggregate and product
  bool split = false;  // complement basis: squaring and product operands as split bf16 pairs
  bool split_p = false;  // Gram basis: P carried into the product as a split bf16 pair
  bool fuse_agg = false;  // level layout with fixed coefficients: the last squaring forms P
  int q_grid[3] = {1, 1, 1};  // e4m3 passes: workgroups per problem (pre-pass, input, row maxima)
  int Jsq = 0;        // squaring launches: J, or J + 2 in learned mode (levels for m_6, m_7)
  float *d_params = nullptr;       // learned mode: network parameters
  double *d_fixed = nullptr;       // learned mode: fixed coefficient slots (fallback)
  int n_agg = 0;
  size_t off_agg = 0;
  int nf_gram[2] = {0, 0}, nf_square = 0, nf_prod[2] = {0, 0};  // [0] wide, [1] tall
  size_t offf_gram[2] = {0, 0}, offf_square = 0, offf_prod[2] = {0, 0};
  int xq_gram[2][2][kXcds] = {}, xq_square[2][kXcds] = {}, xq_prod[2][2][kXcds] = {};  // [off/cnt]
  double fl_gram[2] = {0, 0}, fl_square = 0, fl_prod[2] = {0, 0};  // algorithmic flops per launch
  ifnso_stage_config cfg[3];  // 256-tile schedule of the Gram, squaring and product stages
  std::vector<int> order;     // problems, largest first
  size_t n_all = 0;           // tasks in d_tasks
  double *d_coef = nullptr;   // [num][kSlots]
  double *d_stats = nullptr;  // [num][kStatsPerProblem]
  int grid[3] = {1, 1, 1};
  int cus = 256;
  // per-call tables
  // Each slot's device table and the host copy of what it holds; a call whose table equals a
  // slot's reuses it (and that slot's captured graph) without an upload.
  ProbDev *d_table[kSlotsRing] = {};
  std::vector<ProbDev> h_table[kSlotsRing];
  // task counters of the 256-tile launches of one call, 8 per launch slot, per table slot: calls
  // that share a table slot share its workspace too, which concurrent calls must not
  uint32_t *d_qctr = nullptr;
  hipEvent_t ev[kSlotsRing] = {};
  bool ev_used[kSlotsRing] = {};
  int next_slot = 0;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec[2 * kSlotsRing] = {};  // per table slot, generic / fast I/O
  std::vector<hipEvent_t> stage_events;  // pending measurement request (one call)
  std::mutex mu;
};

static ifnso_stage_config default_config(int stage) {
  ifnso_stage_config c;
  c.xcd_sched = 1;
  c.group = 32;
  c.block_rows = 4;
  c.block_cols = 8;
  c.wg_per_xcd = 32;
  return c;
}

// Host task list of a plan: the generic 128-tile lists, then the 256-tile lists (Gram and
// product split by orientation, each dealt into per-XCD queues as the stage's config says),
// then the aggregation chunks. Offsets and counts are stored in the plan.
static std::vector<Task> build_schedule(ifnso_plan_s *p) {
  std::vector<Task> gram, square, prod;
  for (int i : p->order) {
    const ProbLayout &L = p->lay[i];
    for (int tm = 0; tm < L.nt; tm++)
      for (int tn = tm; tn < L.nt; tn++) {
        gram.push_back(Task{i, tm, tn, 0});
        square.push_back(Task{i, tm, tn, 0});
      }
    const int rt = ((L.trans ? L.w : L.h) + kTS - 1) / kTS, ct = ((L.trans ? L.h : L.w) + kTS - 1) / kTS;
    for (int tm = 0; tm < rt; tm++)
      for (int tn = 0; tn < ct; tn++) prod.push_back(Task{i, tm, tn, 0});
  }
  p->n_gram = (int)gram.size();
  p->n_square = (int)square.size();
  p->n_prod = (int)prod.size();
  std::vector<Task> all;
  p->off_gram = 0;
  all.insert(all.end(), gram.begin(), gram.end());
  p->off_square = all.size();
  all.insert(all.end(), square.begin(), square.end());
  p->off_prod = all.size();
  all.insert(all.end(), prod.begin(), prod.end());
  if (!p->fast) return all;
  const ifnso_stage_config &cg = p->cfg[kStageGram], &cs = p->cfg[kStageSquare], &cp = p->cfg[kStageProduct];
  std::vector<Task> fg[2], fs, fp[2];
  for (int i : p->order) {
    const ProbLayout &L = p->lay[i];
    const int nt = L.hp / kFastTS, tr = L.trans;
    block_order(fg[tr], i, nt, nt, true, cg.block_rows, cg.block_cols);
    block_order(fs, i, nt, nt, true, cs.block_rows, cs.block_cols);
    const int rt = ((tr ? L.w : L.h) + kFastTS - 1) / kFastTS, ct = ((tr ? L.h : L.w) + kFastTS - 1) / kFastTS;
    block_order(fp[tr], i, rt, ct, false, cp.block_rows, cp.block_cols);
  }
  for (int t = 0; t < 2; t++) {
    p->offf_gram[t] = all.size();
    p->nf_gram[t] = (int)fg[t].size();
    const std::vector<Task> qg = xcd_queues(fg[t], cg.group, p->xq_gram[t][0], p->xq_gram[t][1]);
    all.insert(all.end(), qg.begin(), qg.end());
    p->offf_prod[t] = all.size();
    p->nf_prod[t] = (int)fp[t].size();
    const std::vector<Task> qp = xcd_queues(fp[t], cp.group, p->xq_prod[t][0], p->xq_prod[t][1]);
    all.insert(all.end(), qp.begin(), qp.end());
  }
  p->offf_square = all.size();
  p->nf_square = (int)fs.size();
  const std::vector<Task> qs = xcd_queues(fs, cs.group, p->xq_square[0], p->xq_square[1]);
  all.insert(all.end(), qs.begin(), qs.end());
  if (p->agg) {
    p->off_agg = all.size();
    for (int i : p->order) {
      const int64_t n = (int64_t)p->lay[i].hp * p->lay[i].hp;
      for (int64_t c = 0; c * kAggChunk < n; c++) all.push_back(Task{i, (int)c, 0, 0});
    }
    p->n_agg = (int)(all.size() - p->off_agg);
  }
  return all;
}

static ifnso_status validate_desc(const ifnso_poly_desc *d) {
  if (!d) return fail(IFNSO_ERR_INVALID_ARGUMENT, "descriptor is NULL");
  if (d->num_terms < 1 || d->num_terms > kMaxTerms)
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "num_terms %d outside 1..%d", d->num_terms, kMaxTerms);
  if (!d->exponents || !d->coeffs) return fail(IFNSO_ERR_INVALID_ARGUMENT, "exponents/coeffs is NULL");
  for (int k = 0; k < d->num_terms; k++) {
    const int32_t e = d->exponents[k];
    if (e < 0 || e > (1 << 15) || (e != 0 && (e & (e - 1)) != 0))
      return fail(IFNSO_ERR_INVALID_ARGUMENT, "exponent %d is not 0 or 2^j with j <= 15", e);
    if (k && e <= d->exponents[k - 1])
      return fail(IFNSO_ERR_INVALID_ARGUMENT, "exponents must be strictly increasing");
    if (!std::isfinite(d->coeffs[k])) return fail(IFNSO_ERR_INVALID_ARGUMENT, "coefficient %d is not finite", k);
  }
  if (d->basis != IFNSO_BASIS_GRAM && d->basis != IFNSO_BASIS_COMPLEMENT)
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "bad basis %d", d->basis);
  if (d->norm < IFNSO_NORM_FROBENIUS || d->norm > IFNSO_NORM_NONE)
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "bad norm %d", d->norm);
  if (d->compute < IFNSO_COMPUTE_F32 || d->compute > IFNSO_COMPUTE_FP8_E4M3)
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "bad compute %d", d->compute);
  if (d->coeff_mode != IFNSO_COEFF_FIXED && d->coeff_mode != IFNSO_COEFF_LEARNED)
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "bad coeff_mode %d", d->coeff_mode);
  if (d->flags & ~(uint32_t)(IFNSO_FLAG_ENFORCE_SUM_ONE | IFNSO_FLAG_DETERMINISTIC | IFNSO_FLAG_SPLIT_P |
                             IFNSO_FLAG_SPLIT_BF16))
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "unknown flags");
  if ((d->flags & IFNSO_FLAG_SPLIT_P) &&
      (d->compute != IFNSO_COMPUTE_BF16 || d->basis != IFNSO_BASIS_GRAM || d->coeff_mode != IFNSO_COEFF_FIXED))
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "IFNSO_FLAG_SPLIT_P needs bf16 compute, the Gram basis and fixed "
                                            "coefficients");
  if ((d->flags & IFNSO_FLAG_SPLIT_P) && d->exponents[d->num_terms - 1] < 2)
    return fail(IFNSO_ERR_UNSUPPORTED, "IFNSO_FLAG_SPLIT_P needs at least one squaring (an exponent >= 2)");
  if ((d->flags & IFNSO_FLAG_SPLIT_BF16) &&
      (d->compute != IFNSO_COMPUTE_BF16 || d->basis != IFNSO_BASIS_COMPLEMENT || d->coeff_mode != IFNSO_COEFF_FIXED))
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "IFNSO_FLAG_SPLIT_BF16 needs bf16 compute, the complement basis and fixed "
                                            "coefficients");
  if (d->flags & IFNSO_FLAG_ENFORCE_SUM_ONE) {
    double s = 0;
    for (int k = 0; k < d->num_terms; k++) s += d->coeffs[k];
    if (std::fabs(s - 1.0) > 1e-12) return fail(IFNSO_ERR_INVALID_ARGUMENT, "coefficients sum to %.17g, not 1", s);
  }
  if (d->coeff_mode == IFNSO_COEFF_LEARNED) {
    if (!d->mlp_params || d->mlp_params_len != (size_t)kMlpParams)
      return fail(IFNSO_ERR_INVALID_ARGUMENT, "learned mode needs %d network parameters", kMlpParams);
    static const int32_t want[6] = {0, 1, 2, 4, 8, 16};
    bool ok = d->num_terms == 6;
    for (int k = 0; ok && k < 6; k++) ok = d->exponents[k] == want[k];
    if (!ok) return fail(IFNSO_ERR_UNSUPPORTED, "learned mode predicts exponents {0,1,2,4,8,16} only");
    if (d->basis != IFNSO_BASIS_GRAM || d->norm != IFNSO_NORM_FROBENIUS || d->compute != IFNSO_COMPUTE_BF16)
      return fail(IFNSO_ERR_UNSUPPORTED, "learned mode needs the Gram basis, the Frobenius norm and bf16 compute");
    for (size_t i = 0; i < d->mlp_params_len; i++)
      if (!std::isfinite(d->mlp_params[i])) return fail(IFNSO_ERR_INVALID_ARGUMENT, "parameter %zu is not finite", i);
  }
  if (d->compute == IFNSO_COMPUTE_FP8_E4M3 && d->basis != IFNSO_BASIS_GRAM)
    return fail(IFNSO_ERR_UNSUPPORTED, "FP8 compute is built for the Gram basis only");
  return IFNSO_OK;
}

static bool fast_enabled_impl();
static bool fast_enabled() { return fast_enabled_impl(); }

static int slot_of_exponent(int e) {
  if (e == 0) return 0;
  int j = 0;
  while ((1 << j) < e) j++;
  return 1 + j;
}

static ifnso_status cleanup_early(ifnso_plan_s *p, ifnso_status st) {
  delete p;
  return st;
}

extern "C" ifnso_status ifnso_plan(const ifnso_poly_desc *desc, int32_t num_problems, const int64_t *rows,
                                   const int64_t *cols, int32_t in_dtype, int32_t out_dtype, int32_t device,
                                   ifnso_plan_t *out_plan) {
  if (!out_plan) return fail(IFNSO_ERR_INVALID_ARGUMENT, "out_plan is NULL");
  *out_plan = nullptr;
  ifnso_status st = validate_desc(desc);
  if (st != IFNSO_OK) return st;
  if (num_problems < 1) return fail(IFNSO_ERR_INVALID_ARGUMENT, "num_problems %d < 1", num_problems);
  if (!rows || !cols) return fail(IFNSO_ERR_INVALID_ARGUMENT, "rows/cols is NULL");
  if ((in_dtype != IFNSO_F32 && in_dtype != IFNSO_BF16) || (out_dtype != IFNSO_F32 && out_dtype != IFNSO_BF16))
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "bad dtype");
  for (int i = 0; i < num_problems; i++) {
    if (rows[i] < 1 || cols[i] < 1)
      return fail(IFNSO_ERR_INVALID_ARGUMENT, "problem %d has shape %lld x %lld", i, (long long)rows[i],
                  (long long)cols[i]);
    if (std::min(rows[i], cols[i]) > 65536 || std::max(rows[i], cols[i]) > (1LL << 30))
      return fail(IFNSO_ERR_UNSUPPORTED, "problem %d is larger than the library supports", i);
  }
  // the e4m3 mode keeps bfloat16 levels, P and product operands; only the Gram and squaring
  // GEMMs read e4m3
  const bool e4m3 = desc->compute == IFNSO_COMPUTE_FP8_E4M3;
  const int op = desc->compute == IFNSO_COMPUTE_F32 ? kOpF32 : kOpBF16;
  if ((op == kOpF32 && in_dtype != IFNSO_F32) || (op == kOpBF16 && in_dtype != IFNSO_BF16))
    return fail(IFNSO_ERR_UNSUPPORTED,
                "compute type must match the input dtype (F32 with F32, BF16 or FP8_E4M3 with BF16)");
  if (e4m3) {
    if (!fast_enabled()) return fail(IFNSO_ERR_UNSUPPORTED, "FP8 compute needs the 256-tile kernels (IFNSO_FAST != 0)");
    for (int i = 0; i < num_problems; i++) {
      const int64_t h = std::min(rows[i], cols[i]), w = std::max(rows[i], cols[i]);
      if (round_up(h, kPad) > 32512 || h * round_up(w, 16) >= (1LL << 31))
        return fail(IFNSO_ERR_UNSUPPORTED, "problem %d is too large for the FP8 path (32-bit buffer offsets)", i);
    }
  }
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(IFNSO_ERR_INVALID_ARGUMENT, "device %d not present", device);

  ifnso_plan_s *p = new (std::nothrow) ifnso_plan_s;
  if (!p) return fail(IFNSO_ERR_INTERNAL, "out of host memory");
  p->device = device;
  p->num = num_problems;
  p->K = desc->num_terms;
  for (int k = 0; k < p->K; k++) {
    p->exps[k] = desc->exponents[k];
    p->coeffs[k] = desc->coeffs[k];
    p->slots[slot_of_exponent(p->exps[k])] = p->coeffs[k];
  }
  p->basis = desc->basis;
  p->norm = desc->norm;
  p->op = op;
  p->coeff_mode = desc->coeff_mode;
  p->flags = desc->flags;
  p->in_dtype = in_dtype;
  p->out_dtype = out_dtype;
  const int emax = p->exps[p->K - 1];
  p->J = emax <= 1 ? 0 : slot_of_exponent(emax) - 1;
  p->p_empty = emax == 0;
  p->fast = op == kOpBF16 && fast_enabled();
  for (int i = 0; i < num_problems; i++)
    if (round_up(std::min(rows[i], cols[i]), kPad) > 32512) p->fast = false;  // bf16 h x h below 2 GiB
  p->e4m3 = e4m3;
  p->agg = p->fast && p->basis == IFNSO_BASIS_GRAM && (p->J >= 1 || e4m3);
  p->learned = desc->coeff_mode == IFNSO_COEFF_LEARNED;
  p->split = (desc->flags & IFNSO_FLAG_SPLIT_BF16) != 0;
  if (p->split && !p->fast)
    return cleanup_early(p, fail(IFNSO_ERR_UNSUPPORTED, "split bf16 operands need the bf16 fast path (IFNSO_FAST != 0, "
                                                        "h below 32512)"));
  for (int i = 0; p->split && i < num_problems; i++)
    if (round_up(std::min(rows[i], cols[i]), kPad) > 23040)  // hp x 2hp bf16 pairs below 2 GiB
      return cleanup_early(p, fail(IFNSO_ERR_UNSUPPORTED, "split bf16 operands need min(rows, cols) <= 23040"));
  if (p->learned && !p->agg)
    return cleanup_early(p, fail(IFNSO_ERR_UNSUPPORTED, "learned mode needs the bf16 fast path (IFNSO_FAST != 0)"));
  p->Jsq = p->learned ? p->J + 2 : p->J;
  p->split_p = (desc->flags & IFNSO_FLAG_SPLIT_P) != 0;
  if (p->split_p && !p->agg)
    return cleanup_early(p, fail(IFNSO_ERR_UNSUPPORTED, "IFNSO_FLAG_SPLIT_P needs the bf16 fast path (IFNSO_FAST != 0, "
                                                        "h below 32512)"));
  // the aggregation needs the coefficients before the last squaring: not in learned mode (the
  // network reads the last levels)
  p->fuse_agg = p->agg && !p->learned && p->J >= 1;
  size_t off = 0;
  for (int i = 0; i < num_problems; i++) {
    // a single problem that always runs on the generic kernels may split its Gram along K
    const bool gsplit = num_problems == 1 && !p->fast && !p->agg && !e4m3;
    p->lay.push_back(layout_problem(rows[i], cols[i], op, p->Jsq, p->basis == IFNSO_BASIS_COMPLEMENT, false,
                                    p->agg, e4m3, p->split, gsplit, p->split_p));
    p->ws_off.push_back(off);
    off = align_up(off + p->lay.back().bytes, kAlign);
  }
  p->ws_bytes = off;

  // tile schedules: largest problems first (longest-processing-time order)
  p->order.resize(num_problems);
  for (int i = 0; i < num_problems; i++) p->order[i] = i;
  std::stable_sort(p->order.begin(), p->order.end(), [&](int a, int b) {
    const double fa = (double)p->lay[a].h * p->lay[a].h * p->lay[a].w;
    const double fb = (double)p->lay[b].h * p->lay[b].h * p->lay[b].w;
    return fa > fb;
  });
  for (int st = 0; st < 3; st++) p->cfg[st] = default_config(st);
  for (int i = 0; i < num_problems; i++) {
    const ProbLayout &L = p->lay[i];
    const int tr = p->fast ? L.trans : 0;
    const double h = L.h, w = L.w;
    p->fl_gram[tr] += h * h * w;
    p->fl_square += h * h * h;
    p->fl_prod[tr] += 2 * h * h * w;
  }
  std::vector<Task> all = build_schedule(p);

  auto cleanup = [&](ifnso_status s) {
    ifnso_plan_destroy(p);
    return s;
  };
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) prev = 0;
  if (hipSetDevice(device) != hipSuccess) return cleanup(fail(IFNSO_ERR_HIP, "hipSetDevice(%d) failed", device));
  hipError_t e = hipSuccess;
  std::vector<double> coef((size_t)num_problems * kSlots);
  for (int i = 0; i < num_problems; i++)
    for (int k = 0; k < kSlots; k++) coef[(size_t)i * kSlots + k] = p->slots[k];
  p->cus = dev_cus(device);
  if (e == hipSuccess) e = hipMalloc(&p->d_tasks, all.size() * sizeof(Task));
  if (e == hipSuccess) e = hipMemcpy(p->d_tasks, all.data(), all.size() * sizeof(Task), hipMemcpyHostToDevice);
  p->n_all = all.size();
  if (e == hipSuccess) e = hipMalloc(&p->d_coef, coef.size() * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&p->d_qctr, (size_t)kSlotsRing * (p->Jsq + 6) * kXcds * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemcpy(p->d_coef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&p->d_stats, (size_t)num_problems * kStatsPerProblem * sizeof(double));
  if (e == hipSuccess) e = hipMemset(p->d_stats, 0, (size_t)num_problems * kStatsPerProblem * sizeof(double));
  if (p->learned) {
    if (e == hipSuccess) e = hipMalloc(&p->d_params, kMlpParams * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(p->d_params, desc->mlp_params, kMlpParams * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&p->d_fixed, kSlots * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(p->d_fixed, p->slots, kSlots * sizeof(double), hipMemcpyHostToDevice);
  }
  for (int s = 0; s < kSlotsRing && e == hipSuccess; s++) {
    e = hipMalloc(&p->d_table[s], (size_t)num_problems * sizeof(ProbDev));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev[s], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
  hipSetDevice(prev);
  if (e != hipSuccess) return cleanup(fail(IFNSO_ERR_HIP, "plan allocation: %s", hipGetErrorString(e)));
  if (e4m3) {
    // workgroups per problem for the memory-bound passes: enough work for each, about 8 per
    // CU over the whole batch
    int need[3] = {1, 1, 1};
    for (const ProbLayout &L : p->lay) {
      need[0] = std::max(need[0], L.nq);
      // tall: 64 x 64 tiles; wide: row chunks, one per wave (kThreads / 64 per workgroup)
      const int64_t units_in = L.trans ? (int64_t)((L.h + 63) / 64) * ((L.ldq + 63) / 64)
                                       : ((int64_t)L.h * L.qnch + kThreads / 64 - 1) / (kThreads / 64);
      need[1] = (int)std::max<int64_t>(need[1], units_in);
      need[2] = std::max(need[2], (L.hp + kQRowsPerBlock - 1) / kQRowsPerBlock);  // row-maxima blocks
    }
    const int cap = std::max(1, (8 * p->cus + num_problems - 1) / num_problems);
    for (int k = 0; k < 3; k++) p->q_grid[k] = std::max(1, std::min(need[k], cap));
  }
  p->grid[kStageGram] = grid_for(op, kStageGram, p->n_gram, p->cus);
  p->grid[kStageSquare] = grid_for(op, kStageSquare, p->n_square, p->cus);
  p->grid[kStageProduct] = grid_for(op, kStageProduct, p->n_prod, p->cus);
  *out_plan = p;
  return IFNSO_OK;
}

extern "C" ifnso_status ifnso_plan_workspace_bytes(ifnso_plan_t p, size_t *bytes) {
  if (!p || !bytes) return fail(IFNSO_ERR_INVALID_ARGUMENT, "NULL argument");
  *bytes = p->ws_bytes;
  return IFNSO_OK;
}

extern "C" ifnso_status ifnso_plan_destroy(ifnso_plan_t p) {
  if (!p) return IFNSO_OK;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) prev = 0;
  (void)hipSetDevice(p->device);
  for (int g = 0; g < 2 * kSlotsRing; g++)
    if (p->gexec[g]) (void)hipGraphExecDestroy(p->gexec[g]);
  for (int s = 0; s < kSlotsRing; s++) {
    if (p->ev[s]) {
      (void)hipEventSynchronize(p->ev[s]);
      (void)hipEventDestroy(p->ev[s]);
    }
    if (p->d_table[s]) (void)hipFree(p->d_table[s]);
  }
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->d_tasks) (void)hipFree(p->d_tasks);
  if (p->d_coef) (void)hipFree(p->d_coef);
  if (p->d_qctr) (void)hipFree(p->d_qctr);
  if (p->d_stats) (void)hipFree(p->d_stats);
  if (p->d_params) (void)hipFree(p->d_params);
  if (p->d_fixed) (void)hipFree(p->d_fixed);
  (void)hipSetDevice(prev);
  delete p;
  return IFNSO_OK;
}

// ---------------------------------------------------------------------------------------------
// enqueueing the stages
// ---------------------------------------------------------------------------------------------
static StageArgs base_args(const ifnso_plan_s *p) {
  StageArgs a;
  std::memset(&a, 0, sizeof a);
  a.J = p->J;
  a.basis = p->basis;
  a.norm = p->norm;
  a.ns_step = -1;
  a.p_empty = p->p_empty;
  a.learned = 0;
  a.agg = p->agg ? 1 : 0;
  a.split = p->split ? 1 : 0;
  a.fuse_agg = p->fuse_agg ? 1 : 0;
  a.p_slot = p->fuse_agg ? p->J : 0;  // P lands in level slot J + 1 (index J), else in level 1
  a.split_p = p->split_p ? 1 : 0;
  return a;
}

// Launch slots of one call, in order: preparation (e4m3 pre-pass and input quantisation; empty
// in other plans), Gram (wide, tall), each squaring level (with its quantisation in e4m3
// plans), aggregate, product (wide, tall). A slot that has no work in a call is skipped; with
// `ev`, ev[i] is recorded before slot i and ev[num_slots] after the last one, so empty slots
// read as zero time.
static int num_slots(const ifnso_plan_s *p) { return p->Jsq + 6; }

// Problem-level check for the fast kernels: 16-byte aligned rows whose length is a multiple of
// 8 elements, and an input small enough for 32-bit buffer offsets.
static bool fast_io_ok(const ifnso_plan_s *p, const ProbDev &d, const ProbLayout &L) {
  const int64_t cols = L.cols;
  const size_t in_bytes = ((size_t)(L.rows - 1) * d.ldm + cols) * 2;
  const int oes = p->out_dtype == IFNSO_F32 ? 4 : 2;
  return cols % 8 == 0 && d.ldm % 8 == 0 && ((uintptr_t)d.M % 16) == 0 && in_bytes < (1ull << 31) &&
         ((size_t)d.ldy * oes) % 16 == 0 && ((uintptr_t)d.Y % 16) == 0;
}

static bool use_xcd_sched();
static bool use_dynamic_queues();

static void set_xcd(StageArgs &a, const int off[kXcds], const int cnt[kXcds], const ifnso_stage_config &c) {
  a.xcd_sched = (use_xcd_sched() && c.xcd_sched) ? 1 : 0;
  a.wg_per_xcd = c.wg_per_xcd;
  for (int x = 0; x < kXcds; x++) {
    a.xcd_off[x] = off[x];
    a.xcd_cnt[x] = cnt[x];
  }
}

// One workgroup per CU; with XCD queues, a multiple of 8 workgroups, no more than the
// longest queue needs.
// Launch parameters of a stage's config that apply to single-problem calls too.
static void apply_cfg(StageArgs &a, const ifnso_stage_config &c) {
  a.wg_per_xcd = c.wg_per_xcd;
}

static int fast_grid(const StageArgs &a, int cus) {
  const int per_xcd = std::max(1, std::min(cus / kXcds, a.wg_per_xcd > 0 ? a.wg_per_xcd : cus / kXcds));
  if (!a.xcd_sched) return std::max(1, std::min(a.ntasks, kXcds * per_xcd));
  int mx = 1;
  for (int x = 0; x < kXcds; x++) mx = std::max(mx, a.xcd_cnt[x]);
  return kXcds * std::max(1, std::min(per_xcd, mx));
}

// Enqueues every stage of a plan on `s`, reading problems from `table` (batched) or `one`.
static hipError_t enqueue_plan(const ifnso_plan_s *p, const ProbDev *table, const ProbDev *one, bool fast_io,
                               hipStream_t s, const hipEvent_t *ev = nullptr, uint32_t *qctr = nullptr) {
  StageArgs a = base_args(p);
  const int outbf = p->out_dtype == IFNSO_BF16;
  const int cus = p->cus;
  const bool fast = p->fast;
  hipError_t e;
  int slot = 0;
  auto mark = [&]() -> hipError_t { return ev ? hipEventRecord(ev[slot++], s) : hipSuccess; };
  if (one) {
    a.tasks = nullptr;
    a.one = *one;
  } else {
    a.probs = table;
  }
  const ProbLayout *L0 = one ? &p->lay[0] : nullptr;
  const int tr0 = L0 ? L0->trans : 0;
  auto ntiles_sym = [&](int ts) { return (L0->hp / ts) * (L0->hp / ts + 1) / 2; };
  auto ntiles_prod = [&](int ts) {
    return (((L0->trans ? L0->w : L0->h) + ts - 1) / ts) * (((L0->trans ? L0->h : L0->w) + ts - 1) / ts);
  };
  const int nprob = one ? 1 : p->num;
  int qi = 0;  // next counter set of this call
  if (qctr && (e = launch_zero_u32(qctr, (p->Jsq + 6) * kXcds, s)) != hipSuccess) return e;
  if ((e = mark()) != hipSuccess) return e;
  if (p->e4m3) {
    if ((e = launch_e4m3_pass(kE4m3Prepass, a, nprob, p->q_grid[0], s)) != hipSuccess) return e;
    if ((e = launch_e4m3_pass(kE4m3QuantInput, a, nprob, p->q_grid[1], s)) != hipSuccess) return e;
    a.level = 0;  // the largest row sum of Q(A): the scale of the Gram's stored power
    if ((e = launch_e4m3_pass(kE4m3RowMax, a, nprob, p->q_grid[2], s)) != hipSuccess) return e;
  }
  // Gram
  for (int t = 0; t < 2; t++) {
    if ((e = mark()) != hipSuccess) return e;
    if (p->e4m3) {
      // the e4m3 copy of A is K-major for both orientations; the two lists are kept apart only
      // so that the launch slots match the other modes
      a.ntasks = one ? (t == tr0 ? ntiles_sym(kFastTS) : 0) : p->nf_gram[t];
      if (!one) {
        a.tasks = p->d_tasks + p->offf_gram[t];
        set_xcd(a, p->xq_gram[t][0], p->xq_gram[t][1], p->cfg[kStageGram]);
        a.qctr = (qctr && a.xcd_sched) ? qctr + kXcds * (qi++) : nullptr;
      }
      apply_cfg(a, p->cfg[kStageGram]);
      e = launch_e4m3_gemm(kStageGram, a, fast_grid(a, cus), s);
      a.xcd_sched = 0;
      a.qctr = nullptr;
    } else if (fast && fast_io) {
      a.ntasks = one ? (t == tr0 ? ntiles_sym(kFastTS) : 0) : p->nf_gram[t];
      if (!one) {
        a.tasks = p->d_tasks + p->offf_gram[t];
        set_xcd(a, p->xq_gram[t][0], p->xq_gram[t][1], p->cfg[kStageGram]);
        a.qctr = (qctr && a.xcd_sched) ? qctr + kXcds * (qi++) : nullptr;
      }
      apply_cfg(a, p->cfg[kStageGram]);
      e = launch_fast_stage(kStageGram, t, a, fast_grid(a, cus), outbf, s);
      a.xcd_sched = 0;
      a.qctr = nullptr;
    } else if (t == 0) {
      a.ntasks = one ? ntiles_sym(kTS) : p->n_gram;
      if (!one) a.tasks = p->d_tasks + p->off_gram;
      // split along K on the direct single-problem path only (a captured graph would keep the
      // first call's counter address)
      const bool ks = one && L0->ksplit > 1;
      if (ks) {
        a.ksplit = L0->ksplit;
        a.kchunk = L0->kchunk;
        e = launch_zero_u32(a.one.gcnt, a.ntasks, s);  // the workspace arrives uninitialised
      }
      if (e == hipSuccess)
        e = launch_stage(p->op, kTS, kStageGram, a, grid_for(p->op, kStageGram, a.ntasks * (ks ? a.ksplit : 1), cus),
                         outbf, s);
      a.ksplit = 0;
      a.kchunk = 0;
    }
    if (e != hipSuccess) return e;
  }
  // the 256-tile kernels read per-problem totals of the partials (ProbDev::lvl_sum)
  const bool sums = fast || p->e4m3;
  if (sums && (e = launch_level_sums(a, nprob, 1, s)) != hipSuccess) return e;
  // e4m3: the largest row sum of a stored power's e4m3 copy gives the scale of the next one
  auto row_max = [&](int level) -> hipError_t {
    if (!p->e4m3 || level > p->Jsq) return hipSuccess;
    const int l0 = a.level;
    a.level = level;
    const hipError_t r = launch_e4m3_pass(kE4m3RowMax, a, nprob, p->q_grid[2], s);
    a.level = l0;
    return r;
  };
  if ((e = row_max(1)) != hipSuccess) return e;
  for (int lvl = 1; lvl <= p->Jsq; lvl++) {
    if ((e = mark()) != hipSuccess) return e;
    a.level = lvl;
    a.last = lvl == p->Jsq;
    if (p->e4m3) {
      a.ntasks = one ? ntiles_sym(kFastTS) : p->nf_square;
      if (!one) {
        a.tasks = p->d_tasks + p->offf_square;
        set_xcd(a, p->xq_square[0], p->xq_square[1], p->cfg[kStageSquare]);
        a.qctr = (qctr && a.xcd_sched) ? qctr + kXcds * (qi++) : nullptr;
      }
      apply_cfg(a, p->cfg[kStageSquare]);
      e = launch_e4m3_gemm(kStageSquare, a, fast_grid(a, cus), s);
      a.xcd_sched = 0;
      a.qctr = nullptr;
    } else if (fast) {
      a.ntasks = one ? ntiles_sym(kFastTS) : p->nf_square;
      if (!one) {
        a.tasks = p->d_tasks + p->offf_square;
        set_xcd(a, p->xq_square[0], p->xq_square[1], p->cfg[kStageSquare]);
        a.qctr = (qctr && a.xcd_sched) ? qctr + kXcds * (qi++) : nullptr;
      }
      apply_cfg(a, p->cfg[kStageSquare]);
      e = launch_fast_stage(kStageSquare, 0, a, fast_grid(a, cus), outbf, s);
      a.xcd_sched = 0;
      a.qctr = nullptr;
    } else {
      a.ntasks = one ? ntiles_sym(kTS) : p->n_square;
      if (!one) a.tasks = p->d_tasks + p->off_square;
      e = launch_stage(p->op, kTS, kStageSquare, a, grid_for(p->op, kStageSquare, a.ntasks, cus), outbf, s);
    }
    if (e != hipSuccess) return e;
    // level lvl + 1 is read by the next squaring and by the aggregate stage, never after the last
    if (sums && lvl < p->Jsq && (e = launch_level_sums(a, nprob, lvl + 1, s)) != hipSuccess) return e;
    if (lvl < p->Jsq && (e = row_max(lvl + 1)) != hipSuccess) return e;
  }
  a.level = 0;
  a.last = 0;
  if ((e = mark()) != hipSuccess) return e;
  if (p->learned) {
    StageArgs b = a;
    if (!one) b.tasks = p->d_tasks;  // non-null: problems come from the table
    e = launch_learned(b, p->num, p->d_params, p->d_fixed, s);
    if (e != hipSuccess) return e;
  }
  if (p->agg && !p->fuse_agg) {
    a.ntasks = one ? (int)(((int64_t)L0->hp * L0->hp + kAggChunk - 1) / kAggChunk) : p->n_agg;
    if (!one) a.tasks = p->d_tasks + p->off_agg;
    e = launch_aggregate(a, std::max(1, std::min(a.ntasks, 8 * cus)), s);
    if (e != hipSuccess) return e;
  }
  for (int t = 0; t < 2; t++) {
    if ((e = mark()) != hipSuccess) return e;
    if (fast && fast_io) {
      a.ntasks = one ? (t == tr0 ? ntiles_prod(kFastTS) : 0) : p->nf_prod[t];
      if (!one) {
        a.tasks = p->d_tasks + p->offf_prod[t];
        set_xcd(a, p->xq_prod[t][0], p->xq_prod[t][1], p->cfg[kStageProduct]);
        a.qctr = (qctr && a.xcd_sched) ? qctr + kXcds * (qi++) : nullptr;
      }
      apply_cfg(a, p->cfg[kStageProduct]);
      const int sp = a.split;
      a.split = p->split || p->split_p;  // a split P (either form) takes the split product
      e = launch_fast_stage(kStageProduct, t, a, fast_grid(a, cus), outbf, s);
      a.split = sp;
      a.xcd_sched = 0;
      a.qctr = nullptr;
    } else if (t == 0) {
      a.ntasks = one ? ntiles_prod(kTS) : p->n_prod;
      if (!one) a.tasks = p->d_tasks + p->off_prod;
      e = launch_stage(p->op, kTS, kStageProduct, a, grid_for(p->op, kStageProduct, a.ntasks, cus), outbf, s);
    }
    if (e != hipSuccess) return e;
  }
  return mark();
}

static ifnso_status check_matrix_args(const ifnso_plan_s *p, int i, const void *M, int64_t ldm, const void *Y,
                                      int64_t ldy) {
  const ProbLayout &L = p->lay[i];
  if (!M || !Y) return fail(IFNSO_ERR_INVALID_ARGUMENT, "problem %d: NULL matrix pointer", i);
  if (ldm < L.cols || ldy < L.cols)
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "problem %d: leading dimension smaller than cols (%lld)", i,
                (long long)L.cols);
  const size_t ies = p->in_dtype == IFNSO_F32 ? 4 : 2, oes = p->out_dtype == IFNSO_F32 ? 4 : 2;
  if (ranges_overlap(M, matrix_bytes(L.rows, ldm, L.cols, ies), Y, matrix_bytes(L.rows, ldy, L.cols, oes)))
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "problem %d: Y overlaps M", i);
  return IFNSO_OK;
}

static bool use_dynamic_queues() {
  const char *v = getenv("IFNSO_DYNAMIC_QUEUES");
  return !(v && v[0] == '0');
}

static bool use_xcd_sched() {
  const char *v = getenv("IFNSO_XCD_SCHED");
  return !(v && v[0] == '0');
}

static bool fast_enabled_impl() {
  const char *v = getenv("IFNSO_FAST");
  return !(v && v[0] == '0');
}

static bool use_graphs() {
  const char *v = getenv("IFNSO_NO_GRAPH");
  return !(v && v[0] == '1');
}

static ifnso_status run_batched(ifnso_plan_s *p, const void *const *M, const int64_t *ldm, void *const *Y,
                                const int64_t *ldy, void *ws, size_t ws_bytes, hipStream_t s, bool single) {
  if (!ws && p->ws_bytes) return fail(IFNSO_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (ws_bytes < p->ws_bytes)
    return fail(IFNSO_ERR_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, plan needs %zu", ws_bytes, p->ws_bytes);
  if ((uintptr_t)ws % kAlign) return fail(IFNSO_ERR_INVALID_ARGUMENT, "workspace must be %zu-byte aligned", kAlign);
  for (int i = 0; i < p->num; i++) {
    ifnso_status st = check_matrix_args(p, i, M[i], ldm[i], Y[i], ldy[i]);
    if (st != IFNSO_OK) return st;
    if (p->split || p->split_p) {  // only the 256-tile kernels know the split layouts
      ProbDev t{};
      t.M = M[i];
      t.ldm = ldm[i];
      t.Y = Y[i];
      t.ldy = ldy[i];
      if (!fast_io_ok(p, t, p->lay[i]))
        return fail(IFNSO_ERR_UNSUPPORTED, "problem %d: split bf16 plans need 16-byte aligned M and Y rows and a "
                                           "multiple of 8 columns", i);
    }
  }
  std::lock_guard<std::mutex> lock(p->mu);
  int prev = 0;
  HIP_TRY(hipGetDevice(&prev));
  if (prev != p->device) HIP_TRY(hipSetDevice(p->device));
  struct Restore {
    int d, cur;
    ~Restore() {
      if (d != cur) (void)hipSetDevice(d);
    }
  } restore{prev, p->device};
  char *base = (char *)ws;
  std::vector<hipEvent_t> ev;
  ev.swap(p->stage_events);
  const hipEvent_t *evp = ev.empty() ? nullptr : ev.data();
  if (single) {
    ProbDev one;
    fill_dev(one, p->lay[0], base + p->ws_off[0], M[0], ldm[0], Y[0], ldy[0], p->op, p->d_coef, p->d_stats);
    HIP_TRY(enqueue_plan(p, nullptr, &one, p->fast && fast_io_ok(p, one, p->lay[0]), s, evp));
    return IFNSO_OK;
  }
  // The problem table of this call. A slot that already holds the same table is reused as it
  // is (the usual case: the same buffers every step); otherwise the least recently filled slot
  // takes it, after the calls that read that slot (a device-side wait on their event, so the
  // host never blocks), uploaded in stream order.
  std::vector<ProbDev> ht(p->num);
  memset((void *)ht.data(), 0, (size_t)p->num * sizeof(ProbDev));  // padding compares equal
  for (int i = 0; i < p->num; i++)
    fill_dev(ht[i], p->lay[i], base + p->ws_off[i], M[i], ldm[i], Y[i], ldy[i], p->op,
             p->d_coef + (size_t)i * kSlots, p->d_stats + (size_t)i * kStatsPerProblem);
  const size_t tbytes = (size_t)p->num * sizeof(ProbDev);
  int slot = -1;
  for (int k = 0; k < kSlotsRing && slot < 0; k++)
    if (p->h_table[k].size() == ht.size() && memcmp(p->h_table[k].data(), ht.data(), tbytes) == 0) slot = k;
  if (slot < 0) {
    slot = p->next_slot;
    p->next_slot = (slot + 1) % kSlotsRing;
    if (p->ev_used[slot]) HIP_TRY(hipStreamWaitEvent(s, p->ev[slot], 0));
    HIP_TRY(upload_table(p->d_table[slot], ht.data(), tbytes, s));
    p->h_table[slot] = ht;
  }
  bool fast_io = p->fast;
  for (int i = 0; i < p->num && fast_io; i++) fast_io = fast_io_ok(p, ht[i], p->lay[i]);
  uint32_t *qctr = use_dynamic_queues() ? p->d_qctr + (size_t)slot * (p->Jsq + 6) * kXcds : nullptr;
  const int gi = slot * 2 + (fast_io ? 1 : 0);
  if (use_graphs() && !evp) {
    if (!p->gexec[gi]) {
      hipGraph_t g = nullptr;
      HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = enqueue_plan(p, p->d_table[slot], nullptr, fast_io, p->cap_stream, nullptr, qctr);
      hipError_t e2 = hipStreamEndCapture(p->cap_stream, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(IFNSO_ERR_HIP, "graph capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
      }
      hipError_t e3 = hipGraphInstantiate(&p->gexec[gi], g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e3 != hipSuccess) return fail(IFNSO_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e3));
    }
    HIP_TRY(hipGraphLaunch(p->gexec[gi], s));
  } else {
    HIP_TRY(enqueue_plan(p, p->d_table[slot], nullptr, fast_io, s, evp, qctr));
  }
  HIP_TRY(hipEventRecord(p->ev[slot], s));
  p->ev_used[slot] = true;
  return IFNSO_OK;
}

extern "C" int32_t ifnso_plan_num_launches(ifnso_plan_t p) {
  if (!p) return -IFNSO_ERR_INVALID_ARGUMENT;
  return num_slots(p);
}

extern "C" ifnso_status ifnso_plan_launch_info(ifnso_plan_t p, int32_t i, int32_t *stage, double *flops) {
  if (!p || !stage || !flops) return fail(IFNSO_ERR_INVALID_ARGUMENT, "NULL argument");
  const int n = num_slots(p);
  if (i < 0 || i >= n) return fail(IFNSO_ERR_INVALID_ARGUMENT, "launch slot %d outside 0..%d", i, n - 1);
  if (i == 0) {
    *stage = kStagePrep;
    *flops = 0.0;
    return IFNSO_OK;
  }
  i--;
  if (i < 2) {
    *stage = kStageGram;
    *flops = p->fl_gram[i];
  } else if (i < 2 + p->Jsq) {
    *stage = kStageSquare;
    *flops = p->fl_square;
  } else if (i == 2 + p->Jsq) {
    *stage = kStageAggregate;
    *flops = 0.0;
  } else {
    *stage = kStageProduct;
    *flops = p->fl_prod[i - 3 - p->Jsq];
  }
  return IFNSO_OK;
}

extern "C" ifnso_status ifnso_plan_get_config(ifnso_plan_t p, int32_t stage, ifnso_stage_config *cfg) {
  if (!p || !cfg) return fail(IFNSO_ERR_INVALID_ARGUMENT, "NULL argument");
  if (stage < kStageGram || stage > kStageProduct) return fail(IFNSO_ERR_INVALID_ARGUMENT, "bad stage %d", stage);
  std::lock_guard<std::mutex> lock(p->mu);
  *cfg = p->cfg[stage];
  return IFNSO_OK;
}

extern "C" ifnso_status ifnso_plan_set_config(ifnso_plan_t p, int32_t stage, const ifnso_stage_config *cfg) {
  if (!p || !cfg) return fail(IFNSO_ERR_INVALID_ARGUMENT, "NULL argument");
  if (stage < kStageGram || stage > kStageProduct) return fail(IFNSO_ERR_INVALID_ARGUMENT, "bad stage %d", stage);
  const ifnso_stage_config &c = *cfg;
  if ((c.xcd_sched != 0 && c.xcd_sched != 1) || c.group < 1 || c.group > 4096 || c.block_rows < 1 ||
      c.block_rows > 64 || c.block_cols < 1 || c.block_cols > 64 || c.wg_per_xcd < 1 || c.wg_per_xcd > 1024)
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "stage config out of range");
  std::lock_guard<std::mutex> lock(p->mu);
  int prev = 0;
  HIP_TRY(hipGetDevice(&prev));
  if (prev != p->device) HIP_TRY(hipSetDevice(p->device));
  struct Restore {
    int d, cur;
    ~Restore() {
      if (d != cur) (void)hipSetDevice(d);
    }
  } restore{prev, p->device};
  // the task list changes: wait for calls in flight, drop the captured graphs
  HIP_TRY(hipDeviceSynchronize());
  p->cfg[stage] = c;
  const std::vector<Task> all = build_schedule(p);
  if (all.size() != p->n_all) return fail(IFNSO_ERR_INTERNAL, "schedule size changed");
  HIP_TRY(hipMemcpy(p->d_tasks, all.data(), all.size() * sizeof(Task), hipMemcpyHostToDevice));
  for (int g = 0; g < 2 * kSlotsRing; g++)
    if (p->gexec[g]) {
      (void)hipGraphExecDestroy(p->gexec[g]);
      p->gexec[g] = nullptr;
    }
  return IFNSO_OK;
}

extern "C" ifnso_status ifnso_plan_launch_events(ifnso_plan_t p, void *const *events, int32_t count) {
  if (!p) return fail(IFNSO_ERR_INVALID_ARGUMENT, "plan is NULL");
  std::lock_guard<std::mutex> lock(p->mu);
  if (count == 0) {
    p->stage_events.clear();
    return IFNSO_OK;
  }
  const int need = num_slots(p) + 1;
  if (!events || count != need) return fail(IFNSO_ERR_INVALID_ARGUMENT, "need %d events, got %d", need, count);
  for (int i = 0; i < count; i++)
    if (!events[i]) return fail(IFNSO_ERR_INVALID_ARGUMENT, "event %d is NULL", i);
  p->stage_events.assign((hipEvent_t *)events, (hipEvent_t *)events + count);
  return IFNSO_OK;
}

extern "C" ifnso_status ifnso_orthogonalize(ifnso_plan_t p, const void *M, int64_t ldm, void *Y, int64_t ldy,
                                            void *workspace, size_t workspace_bytes, void *stream) {
  if (!p) return fail(IFNSO_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (p->num != 1) return fail(IFNSO_ERR_INVALID_ARGUMENT, "plan has %d problems; use the batched call", p->num);
  const void *Ms[1] = {M};
  void *Ys[1] = {Y};
  return run_batched(p, Ms, &ldm, Ys, &ldy, workspace, workspace_bytes, (hipStream_t)stream, true);
}

extern "C" ifnso_status ifnso_orthogonalize_static(ifnso_plan_t p, const void *M, int64_t ldm, void *Y, int64_t ldy,
                                                   void *stream) {
  if (!p) return fail(IFNSO_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (p->num != 1) return fail(IFNSO_ERR_INVALID_ARGUMENT, "plan has %d problems; use the batched call", p->num);
  if (p->ws_bytes > kStaticScratchBytes)
    return fail(IFNSO_ERR_WORKSPACE_TOO_SMALL, "plan needs %zu bytes of workspace; the static scratch area holds %zu",
                p->ws_bytes, kStaticScratchBytes);
  void *ws = nullptr;
  HIP_TRY(static_scratch(p->device, &ws));
  const void *Ms[1] = {M};
  void *Ys[1] = {Y};
  return run_batched(p, Ms, &ldm, Ys, &ldy, ws, kStaticScratchBytes, (hipStream_t)stream, true);
}

extern "C" ifnso_status ifnso_orthogonalize_batched(ifnso_plan_t p, const void *const *M, const int64_t *ldm,
                                                    void *const *Y, const int64_t *ldy, void *workspace,
                                                    size_t workspace_bytes, void *stream) {
  if (!p) return fail(IFNSO_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (!M || !ldm || !Y || !ldy) return fail(IFNSO_ERR_INVALID_ARGUMENT, "NULL pointer array");
  return run_batched(p, M, ldm, Y, ldy, workspace, workspace_bytes, (hipStream_t)stream, false);
}

// ---------------------------------------------------------------------------------------------
// Muon step
// ---------------------------------------------------------------------------------------------
// Workspace of a Muon step: the plan's own, then per problem the orthogonalisation input U and
// output Y (rows x round_up(cols, 8), the plan's input and output types), then the device table.
struct MuonLayout {
  std::vector<size_t> off_u, off_y;
  std::vector<int64_t> ld;
  size_t off_table = 0, bytes = 0;
};

static MuonLayout muon_layout(const ifnso_plan_s *p) {
  MuonLayout m;
  size_t o = align_up(p->ws_bytes, kAlign);
  const size_t ies = p->in_dtype == IFNSO_F32 ? 4 : 2, oes = p->out_dtype == IFNSO_F32 ? 4 : 2;
  for (int i = 0; i < p->num; i++) {
    const ProbLayout &L = p->lay[i];
    const int64_t ld = round_up(L.cols, 8);
    m.ld.push_back(ld);
    m.off_u.push_back(o);
    o = align_up(o + (size_t)L.rows * ld * ies, kAlign);
    m.off_y.push_back(o);
    o = align_up(o + (size_t)L.rows * ld * oes, kAlign);
  }
  m.off_table = o;
  m.bytes = align_up(o + (size_t)p->num * sizeof(MuonProb), kAlign);
  return m;
}

extern "C" ifnso_status ifnso_muon_workspace_bytes(ifnso_plan_t p, size_t *bytes) {
  if (!p || !bytes) return fail(IFNSO_ERR_INVALID_ARGUMENT, "NULL argument");
  *bytes = muon_layout(p).bytes;
  return IFNSO_OK;
}

extern "C" ifnso_status ifnso_muon_step(ifnso_plan_t p, const ifnso_muon_params *hp, float *const *W,
                                        const int64_t *ldw, const void *const *G, const int64_t *ldg,
                                        float *const *B, const int64_t *ldb, void *workspace,
                                        size_t workspace_bytes, void *stream) {
  if (!p || !hp) return fail(IFNSO_ERR_INVALID_ARGUMENT, "NULL argument");
  if (!W || !ldw || !G || !ldg || !B || !ldb) return fail(IFNSO_ERR_INVALID_ARGUMENT, "NULL pointer array");
  if (!std::isfinite(hp->lr) || !std::isfinite(hp->momentum) || !std::isfinite(hp->weight_decay) ||
      (hp->nesterov != 0 && hp->nesterov != 1))
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "Muon parameters must be finite, nesterov 0 or 1");
  const MuonLayout m = muon_layout(p);
  if (!workspace) return fail(IFNSO_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (workspace_bytes < m.bytes)
    return fail(IFNSO_ERR_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, a Muon step needs %zu", workspace_bytes,
                m.bytes);
  if ((uintptr_t)workspace % kAlign) return fail(IFNSO_ERR_INVALID_ARGUMENT, "workspace must be %zu-byte aligned", kAlign);
  const size_t ies = p->in_dtype == IFNSO_F32 ? 4 : 2;
  for (int i = 0; i < p->num; i++) {
    const ProbLayout &L = p->lay[i];
    if (!W[i] || !G[i] || !B[i]) return fail(IFNSO_ERR_INVALID_ARGUMENT, "problem %d: NULL matrix pointer", i);
    if (ldw[i] < L.cols || ldg[i] < L.cols || ldb[i] < L.cols)
      return fail(IFNSO_ERR_INVALID_ARGUMENT, "problem %d: leading dimension smaller than cols (%lld)", i,
                  (long long)L.cols);
    const size_t wb = matrix_bytes(L.rows, ldw[i], L.cols, 4), bb = matrix_bytes(L.rows, ldb[i], L.cols, 4),
                 gb = matrix_bytes(L.rows, ldg[i], L.cols, ies);
    if (ranges_overlap(W[i], wb, B[i], bb) || ranges_overlap(W[i], wb, G[i], gb) || ranges_overlap(B[i], bb, G[i], gb))
      return fail(IFNSO_ERR_INVALID_ARGUMENT, "problem %d: W, G and the momentum buffer must not overlap", i);
  }
  hipStream_t s = (hipStream_t)stream;
  char *base = (char *)workspace;
  std::vector<const void *> U(p->num);
  std::vector<void *> Y(p->num);
  struct DeviceGuard {  // makes the plan's device current for a scope
    int prev = 0, dev;
    hipError_t e;
    explicit DeviceGuard(int d) : dev(d) {
      e = hipGetDevice(&prev);
      if (e == hipSuccess && prev != dev) e = hipSetDevice(dev);
    }
    ~DeviceGuard() {
      if (prev != dev) (void)hipSetDevice(prev);
    }
  };
  MuonArgs a;
  int per = 1;
  {
    DeviceGuard dg(p->device);
    HIP_TRY(dg.e);
    const double lr = hp->lr;
    std::vector<MuonProb> mt(p->num);
    memset((void *)mt.data(), 0, (size_t)p->num * sizeof(MuonProb));
    for (int i = 0; i < p->num; i++) {
      const ProbLayout &L = p->lay[i];
      MuonProb &q = mt[i];
      q.W = W[i];
      q.G = G[i];
      q.B = B[i];
      q.U = base + m.off_u[i];
      q.Y = base + m.off_y[i];
      q.rows = L.rows;
      q.cols = L.cols;
      q.ldw = ldw[i];
      q.ldg = ldg[i];
      q.ldb = ldb[i];
      q.ldu = m.ld[i];
      q.ldy = m.ld[i];
      q.step = (float)(lr * std::sqrt(std::max(1.0, (double)L.rows / (double)L.cols)));
      const bool a16 = ((uintptr_t)W[i] % 16) == 0 && ((uintptr_t)B[i] % 16) == 0 && ((uintptr_t)G[i] % (4 * ies)) == 0;
      q.vec = (L.cols % 4 == 0 && ldw[i] % 4 == 0 && ldb[i] % 4 == 0 && ldg[i] % 4 == 0 && a16) ? 1 : 0;
      U[i] = q.U;
      Y[i] = const_cast<void *>(q.Y);
    }
    // the table lives in the caller's workspace: uploaded every step, in stream order
    MuonProb *d_table = (MuonProb *)(base + m.off_table);
    HIP_TRY(upload_table(d_table, mt.data(), (size_t)p->num * sizeof(MuonProb), s));
    a.probs = d_table;
    a.momentum = hp->momentum;
    a.decay = (float)(1.0 - lr * hp->weight_decay);
    a.nesterov = hp->nesterov;
    a.in_bf16 = p->in_dtype == IFNSO_BF16;
    a.out_bf16 = p->out_dtype == IFNSO_BF16;
    // one grid row per problem, sized for the largest (workgroups of smaller problems run out
    // of work and exit): about 8 resident workgroups per CU over the largest problem's span
    int64_t most = 1;
    for (const ProbLayout &L : p->lay) most = std::max<int64_t>(most, L.rows * L.cols);
    per = (int)std::max<int64_t>(1, std::min<int64_t>((most / 4 + kThreads - 1) / kThreads, 8 * p->cus));
    HIP_TRY(launch_muon_pre(a, p->num, per, s));
  }
  ifnso_status st = run_batched(p, U.data(), m.ld.data(), Y.data(), m.ld.data(), workspace, p->ws_bytes, s, false);
  if (st != IFNSO_OK) return st;
  DeviceGuard dg(p->device);
  HIP_TRY(dg.e);
  HIP_TRY(launch_muon_post(a, p->num, per, s));
  return IFNSO_OK;
}

// ---------------------------------------------------------------------------------------------
// classical Newton-Schulz
// ---------------------------------------------------------------------------------------------
static int ns_op(int32_t compute, int32_t dtype) {
  if (compute == IFNSO_COMPUTE_F32 && dtype == IFNSO_F32) return kOpF32;
  if (compute == IFNSO_COMPUTE_BF16 && dtype == IFNSO_BF16) return kOpBF16;
  return -1;
}

extern "C" size_t ifnso_classical_ns_workspace_bytes(int64_t rows, int64_t cols, int32_t compute) {
  if (rows < 1 || cols < 1) return 0;
  const int op = compute == IFNSO_COMPUTE_F32 ? kOpF32 : compute == IFNSO_COMPUTE_BF16 ? kOpBF16 : -1;
  if (op < 0) return 0;
  return layout_problem(rows, cols, op, 1, false, true).bytes;
}

// Shared by ifnso_classical_ns (one (a, b, c) for every step) and ifnso_ns_schedule (one per
// step): step k uses sched[min(k, nsched - 1)].
static ifnso_status run_ns(const void *M, int64_t rows, int64_t cols, int64_t ldm, int32_t dtype, void *Y,
                           int64_t ldy, int32_t steps, const double *sched, int32_t nsched, int32_t gelfand_q,
                           int32_t compute, void *workspace, size_t workspace_bytes, void *stream) {
  if (!M || !Y || !sched) return fail(IFNSO_ERR_INVALID_ARGUMENT, "NULL argument");
  if (rows < 1 || cols < 1) return fail(IFNSO_ERR_INVALID_ARGUMENT, "bad shape");
  if (ldm < cols || ldy < cols) return fail(IFNSO_ERR_INVALID_ARGUMENT, "leading dimension smaller than cols");
  if (steps < 1) return fail(IFNSO_ERR_INVALID_ARGUMENT, "steps must be >= 1");
  if (dtype != IFNSO_F32 && dtype != IFNSO_BF16) return fail(IFNSO_ERR_INVALID_ARGUMENT, "bad dtype");
  if (compute < IFNSO_COMPUTE_F32 || compute > IFNSO_COMPUTE_FP8_E4M3)
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "bad compute");
  if (gelfand_q < 0) return fail(IFNSO_ERR_INVALID_ARGUMENT, "gelfand_q must be >= 0");
  for (int i = 0; i < 3 * nsched; i++)
    if (!std::isfinite(sched[i])) return fail(IFNSO_ERR_INVALID_ARGUMENT, "coefficient not finite");
  if (gelfand_q > 2) return fail(IFNSO_ERR_UNSUPPORTED, "gelfand_q above 2 is not implemented");
  const int op = ns_op(compute, dtype);
  if (op < 0) return fail(IFNSO_ERR_UNSUPPORTED, "classical NS supports F32/F32 and BF16/BF16 (dtype/compute)");
  if (std::min(rows, cols) > 65536) return fail(IFNSO_ERR_UNSUPPORTED, "matrix too large");
  const ProbLayout L = layout_problem(rows, cols, op, 1, false, true);
  if (!workspace) return fail(IFNSO_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (workspace_bytes < L.bytes)
    return fail(IFNSO_ERR_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, needs %zu", workspace_bytes, L.bytes);
  if ((uintptr_t)workspace % kAlign) return fail(IFNSO_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
  const size_t es = op_size(op);
  if (ranges_overlap(M, matrix_bytes(rows, ldm, cols, es), Y, matrix_bytes(rows, ldy, cols, es)))
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "Y overlaps M");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  const int cus = dev_cus(dev);
  StageArgs a;
  std::memset(&a, 0, sizeof a);
  fill_dev(a.one, L, (char *)workspace, M, ldm, Y, ldy, op, nullptr, nullptr);
  a.J = 1;
  a.basis = kGram;
  a.norm = gelfand_q == 0 ? kFrob : gelfand_q == 1 ? kGramFrob : kGelfand2;
  a.ns_nsched = nsched;
  for (int k = 0; k < nsched; k++)
    for (int i = 0; i < 3; i++) a.ns_sched[k][i] = sched[3 * k + i];
  const int nsym = L.nt * (L.nt + 1) / 2;
  hipStream_t s = (hipStream_t)stream;
  if (L.ksplit > 1) {
    a.ksplit = L.ksplit;
    a.kchunk = L.kchunk;
    HIP_TRY(launch_zero_u32(a.one.gcnt, nsym, s));  // the workspace arrives uninitialised
  }
  a.ns_steps = steps;
  // h == 1: the product kernel runs the scalar recursion from the float64 norm in one pass
  const int passes = L.h == 1 ? 1 : steps;
  for (int k = 0; k < passes; k++) {
    const double *abc = sched + 3 * std::min(k, nsched - 1);
    for (int i = 0; i < 3; i++) a.ns_abc[i] = abc[i];
    a.ns_step = k;
    a.ns_last = k == passes - 1;
    a.ntasks = nsym;
    a.level = 1;
    a.last = 1;
    HIP_TRY(launch_stage(op, kTS, kStageGram, a, grid_for(op, kStageGram, nsym * std::max(1, a.ksplit), cus), 0, s));
    if (L.h > 1 && k == 0 && gelfand_q == 2) {
      // ||G_raw^2||_F^2 into level slot 2 before any consumer of the scale runs
      a.ns_norm_pass = 1;
      HIP_TRY(launch_stage(op, kTS, kStageSquare, a, grid_for(op, kStageSquare, nsym, cus), 0, s));
      a.ns_norm_pass = 0;
    }
    if (L.h > 1) HIP_TRY(launch_stage(op, kTS, kStageSquare, a, grid_for(op, kStageSquare, nsym, cus), 0, s));
    const bool tall_map = k == 0 && L.trans;
    const int rt = ((tall_map ? L.w : L.h) + kTS - 1) / kTS, ct = ((tall_map ? L.h : L.w) + kTS - 1) / kTS;
    a.ntasks = rt * ct;
    a.level = 0;
    a.last = 0;
    HIP_TRY(launch_stage(op, kTS, kStageProduct, a, grid_for(op, kStageProduct, rt * ct, cus),
                         dtype == IFNSO_BF16, s));
  }
  return IFNSO_OK;
}

extern "C" ifnso_status ifnso_classical_ns(const void *M, int64_t rows, int64_t cols, int64_t ldm, int32_t dtype,
                                           void *Y, int64_t ldy, int32_t steps, const double abc[3],
                                           int32_t compute, void *workspace, size_t workspace_bytes, void *stream) {
  return run_ns(M, rows, cols, ldm, dtype, Y, ldy, steps, abc, 1, 0, compute, workspace, workspace_bytes, stream);
}

extern "C" ifnso_status ifnso_ns_schedule(const void *M, int64_t rows, int64_t cols, int64_t ldm, int32_t dtype,
                                          void *Y, int64_t ldy, int32_t steps, const double *abc, int32_t gelfand_q,
                                          int32_t compute, void *workspace, size_t workspace_bytes, void *stream) {
  static_assert(IFNSO_NS_MAX_STEPS == kMaxNsSteps, "schedule bound of the header and the kernels");
  if (steps > kMaxNsSteps)
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "a schedule holds at most %d steps", kMaxNsSteps);
  return run_ns(M, rows, cols, ldm, dtype, Y, ldy, steps, abc, std::max(steps, 1), gelfand_q, compute, workspace,
                workspace_bytes, stream);
}

// ---------------------------------------------------------------------------------------------
// e4m3 quantisation of one input on its own
// ---------------------------------------------------------------------------------------------
namespace {
struct QuantLayout {
  int32_t rq, nq;
  size_t off_part, off_amax, off_norm, off_scale, bytes;
};

QuantLayout quant_layout(int64_t rows, int64_t cols) {
  QuantLayout q{};
  e4m3_chunks(rows, cols, q.rq, q.nq);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes, kAlign);
    return at;
  };
  q.off_part = take((size_t)q.nq * 8);
  q.off_amax = take((size_t)q.nq * 4);
  q.off_norm = take(8);
  q.off_scale = take(kQScaleFloats * 4);
  q.bytes = o;
  return q;
}
}  // namespace

extern "C" size_t ifnso_quantize_e4m3_workspace_bytes(int64_t rows, int64_t cols) {
  if (rows < 1 || cols < 1) return 0;
  return quant_layout(rows, cols).bytes;
}

extern "C" ifnso_status ifnso_quantize_e4m3(const void *M, int64_t rows, int64_t cols, int64_t ldm, void *Q,
                                            int64_t ldq, double *out3, void *workspace, size_t workspace_bytes,
                                            void *stream) {
  if (!M || !Q || !out3) return fail(IFNSO_ERR_INVALID_ARGUMENT, "NULL argument");
  if (rows < 1 || cols < 1 || ldm < cols) return fail(IFNSO_ERR_INVALID_ARGUMENT, "bad shape or leading dimension");
  const int64_t h = std::min(rows, cols), w = std::max(rows, cols);
  if (ldq < round_up(w, 16) || ldq % 16 != 0 || (uintptr_t)Q % 16 != 0)
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "Q needs ldq >= %lld, a multiple of 16, and 16-byte alignment",
                (long long)round_up(w, 16));
  if (h * ldq >= (1LL << 31)) return fail(IFNSO_ERR_UNSUPPORTED, "h * ldq must stay below 2^31");
  if (ranges_overlap(M, matrix_bytes(rows, ldm, cols, 2), Q, (size_t)h * ldq))
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "Q overlaps M");
  const QuantLayout ql = quant_layout(rows, cols);
  if (!workspace) return fail(IFNSO_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (workspace_bytes < ql.bytes)
    return fail(IFNSO_ERR_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, needs %zu", workspace_bytes, ql.bytes);
  if ((uintptr_t)workspace % kAlign) return fail(IFNSO_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
  char *ws = (char *)workspace;
  StageArgs a;
  std::memset(&a, 0, sizeof a);
  ProbDev &d = a.one;
  d.M = M;
  d.ldm = ldm;
  d.h = (int32_t)h;
  d.w = (int32_t)w;
  d.trans = rows > cols;
  d.nt = 1;
  d.vecM = ((uintptr_t)M % 16 == 0) && (ldm * 2 % 16 == 0);
  d.norm_part = (double *)(ws + ql.off_norm);
  d.q8 = (uint8_t *)Q;
  d.ldq = ldq;
  d.q_part = (double *)(ws + ql.off_part);
  d.q_amax = (float *)(ws + ql.off_amax);
  d.q_scale = (float *)(ws + ql.off_scale);
  d.nq = ql.nq;
  d.rq = ql.rq;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  const int cus = dev_cus(dev);
  const int64_t units_in = d.trans ? ((h + 63) / 64) * ((ldq + 63) / 64)
                                   : (h * ((ldq / 16 + 63) / 64) + kThreads / 64 - 1) / (kThreads / 64);
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_e4m3_pass(kE4m3Prepass, a, 1, std::max(1, std::min(ql.nq, 8 * cus)), s));
  HIP_TRY(launch_e4m3_pass(kE4m3QuantInput, a, 1, (int)std::max<int64_t>(1, std::min<int64_t>(units_in, 8 * cus)), s));
  HIP_TRY(launch_e4m3_export(a.one, out3, s));
  return IFNSO_OK;
}

// ---------------------------------------------------------------------------------------------
// evaluation helpers
// ---------------------------------------------------------------------------------------------
static constexpr int kOrthSplit = 64;

extern "C" size_t ifnso_orth_error_workspace_bytes(int32_t count) {
  if (count < 1) return 0;
  return align_up((size_t)count * sizeof(OrthEntry), kAlign) + (size_t)count * kOrthSplit * sizeof(double);
}

extern "C" ifnso_status ifnso_orth_error(int32_t count, const void *const *Y, const int64_t *rows,
                                         const int64_t *cols, const int64_t *ldy, int32_t dtype, double *out,
                                         void *workspace, size_t workspace_bytes, void *stream) {
  if (count < 1 || !Y || !rows || !cols || !ldy || !out) return fail(IFNSO_ERR_INVALID_ARGUMENT, "bad arguments");
  if (dtype != IFNSO_F32 && dtype != IFNSO_BF16) return fail(IFNSO_ERR_INVALID_ARGUMENT, "bad dtype");
  if (!workspace || workspace_bytes < ifnso_orth_error_workspace_bytes(count))
    return fail(IFNSO_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
  std::vector<OrthEntry> e(count);
  for (int i = 0; i < count; i++) {
    if (!Y[i] || rows[i] < 1 || cols[i] < 1 || ldy[i] < cols[i])
      return fail(IFNSO_ERR_INVALID_ARGUMENT, "matrix %d: bad pointer or shape", i);
    e[i] = OrthEntry{Y[i], rows[i], cols[i], ldy[i]};
  }
  hipStream_t s = (hipStream_t)stream;
  OrthArgs a;
  a.e = (const OrthEntry *)workspace;
  a.part = (double *)((char *)workspace + align_up((size_t)count * sizeof(OrthEntry), kAlign));
  a.out = out;
  a.nsplit = kOrthSplit;
  a.count = count;
  HIP_TRY(hipMemcpyAsync((void *)a.e, e.data(), (size_t)count * sizeof(OrthEntry), hipMemcpyHostToDevice, s));
  HIP_TRY(launch_orth_error(a, dtype == IFNSO_BF16, s));
  // the host array `e` must outlive the copy
  HIP_TRY(hipStreamSynchronize(s));
  return IFNSO_OK;
}

extern "C" ifnso_status ifnso_plan_stats(ifnso_plan_t p, double *host_out, void *stream) {
  if (!p || !host_out) return fail(IFNSO_ERR_INVALID_ARGUMENT, "NULL argument");
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  std::vector<double> buf((size_t)p->num * kStatsPerProblem);
  HIP_TRY(hipMemcpy(buf.data(), p->d_stats, buf.size() * sizeof(double), hipMemcpyDeviceToHost));
  for (int i = 0; i < p->num; i++)
    for (int k = 0; k < IFNSO_STATS_PER_PROBLEM; k++)
      host_out[(size_t)i * IFNSO_STATS_PER_PROBLEM + k] = buf[(size_t)i * kStatsPerProblem + k];
  return IFNSO_OK;
}

extern "C" ifnso_status ifnso_mlp_features(int32_t n, const float *sig, const int32_t *nsig, int32_t smax,
                                           float *feats_out, void *stream) {
  if (n < 1 || !sig || !nsig || smax < 1 || !feats_out) return fail(IFNSO_ERR_INVALID_ARGUMENT, "bad arguments");
  HIP_TRY(launch_mlp_features(n, sig, nsig, smax, feats_out, (hipStream_t)stream));
  return IFNSO_OK;
}

extern "C" ifnso_status ifnso_mlp_forward(int32_t n, const float *feats, const float *params, double *coeffs_out,
                                          void *stream) {
  if (n < 1 || !feats || !params || !coeffs_out) return fail(IFNSO_ERR_INVALID_ARGUMENT, "bad arguments");
  HIP_TRY(launch_mlp_forward(n, feats, params, coeffs_out, (hipStream_t)stream));
  return IFNSO_OK;
}

extern "C" size_t ifnso_mlp_train_workspace_bytes(int32_t n) {
  if (n < 1) return 0;
  return align_up((size_t)n * kMlpParams * sizeof(float), kAlign) + align_up((size_t)n * sizeof(float), kAlign);
}

extern "C" ifnso_status ifnso_mlp_train_step(int32_t n, const float *feats, const float *sig, const int32_t *nsig,
                                             int32_t smax, float *params, float *adam_m, float *adam_v, int32_t t,
                                             float lr, float beta1, float beta2, float eps, float *grad_out,
                                             float *loss_out, void *workspace, size_t workspace_bytes,
                                             void *stream) {
  if (n < 1 || !feats || !sig || !nsig || smax < 1 || !params || !adam_m || !adam_v || t < 1)
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "bad arguments");
  if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "bad optimiser hyper-parameters");
  if (!workspace || workspace_bytes < ifnso_mlp_train_workspace_bytes(n))
    return fail(IFNSO_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
  float *grads = (float *)workspace;
  float *losses = (float *)((char *)workspace + align_up((size_t)n * kMlpParams * sizeof(float), kAlign));
  HIP_TRY(launch_mlp_train(n, feats, sig, nsig, smax, params, adam_m, adam_v, t, lr, beta1, beta2, eps, grad_out,
                           loss_out, grads, losses, (hipStream_t)stream));
  return IFNSO_OK;
}

extern "C" const char *ifnso_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------------------------
// Newton-Schulz step schedules over a batch: one Gram-basis plan per distinct step, chained
// ---------------------------------------------------------------------------------------------
struct ifnso_schedule_plan_s {
  std::vector<ifnso_plan_t> plans;  // one per distinct (a, b, c, normalisation)
  std::vector<int> step_plan;       // plan index of each step
  int num = 0;
  int dtype = 0;
  std::vector<int64_t> rows, cols, ld_iter;
  std::vector<size_t> off_iter;     // per problem: the iterate buffer, after the plans' workspace
  size_t ws_bytes = 0;
};

extern "C" ifnso_status ifnso_schedule_plan_destroy(ifnso_schedule_plan_t sp) {
  if (!sp) return IFNSO_OK;
  for (ifnso_plan_t p : sp->plans) ifnso_plan_destroy(p);
  delete sp;
  return IFNSO_OK;
}

extern "C" ifnso_status ifnso_schedule_plan(const double *abc, int32_t steps, int32_t gelfand_q, int32_t num_problems,
                                            const int64_t *rows, const int64_t *cols, int32_t dtype, int32_t compute,
                                            int32_t device, ifnso_schedule_plan_t *out) {
  if (!abc || !rows || !cols || !out) return fail(IFNSO_ERR_INVALID_ARGUMENT, "NULL argument");
  *out = nullptr;
  if (steps < 1 || steps > kMaxNsSteps)
    return fail(IFNSO_ERR_INVALID_ARGUMENT, "steps %d outside 1..%d", steps, kMaxNsSteps);
  if (gelfand_q < 0) return fail(IFNSO_ERR_INVALID_ARGUMENT, "gelfand_q %d < 0", gelfand_q);
  if (gelfand_q > 1)
    return fail(IFNSO_ERR_UNSUPPORTED, "batched schedules scale by ||A||_F (q = 0) or ||AA^T||_F^(1/2) (q = 1)");
  if (num_problems < 1) return fail(IFNSO_ERR_INVALID_ARGUMENT, "num_problems %d < 1", num_problems);
  for (int k = 0; k < 3 * steps; k++)
    if (!std::isfinite(abc[k])) return fail(IFNSO_ERR_INVALID_ARGUMENT, "schedule entry %d is not finite", k);
  if (dtype != IFNSO_F32 && dtype != IFNSO_BF16) return fail(IFNSO_ERR_INVALID_ARGUMENT, "bad dtype %d", dtype);
  for (int i = 0; i < num_problems; i++)
    if (rows[i] < 1 || cols[i] < 1) return fail(IFNSO_ERR_INVALID_ARGUMENT, "problem %d: dimensions must be >= 1", i);
  ifnso_schedule_plan_s *sp = new (std::nothrow) ifnso_schedule_plan_s;
  if (!sp) return fail(IFNSO_ERR_INTERNAL, "out of host memory");
  sp->num = num_problems;
  sp->dtype = dtype;
  std::vector<double> keys;  // (a, b, c, norm) of each distinct plan
  size_t ws_plan = 0;
  for (int k = 0; k < steps; k++) {
    const double a = abc[3 * k], b = abc[3 * k + 1], c = abc[3 * k + 2];
    const int norm = k > 0 ? IFNSO_NORM_NONE : (gelfand_q == 0 ? IFNSO_NORM_FROBENIUS : IFNSO_NORM_GRAM_FROBENIUS);
    int found = -1;
    for (size_t q = 0; q < sp->plans.size() && found < 0; q++)
      if (keys[4 * q] == a && keys[4 * q + 1] == b && keys[4 * q + 2] == c && keys[4 * q + 3] == norm) found = (int)q;
    if (found < 0) {
      // X_{k+1} = a X_k + b (X_k X_k^T) X_k + c (X_k X_k^T)^2 X_k: exponents {0, 1, 2}, or {0, 1} without c
      const int32_t e3[3] = {0, 1, 2};
      const double c3[3] = {a, b, c};
      ifnso_poly_desc d;
      std::memset(&d, 0, sizeof d);
      d.num_terms = c == 0.0 ? 2 : 3;
      d.exponents = e3;
      d.coeffs = c3;
      d.basis = IFNSO_BASIS_GRAM;
      d.norm = norm;
      d.compute = compute;
      d.coeff_mode = IFNSO_COEFF_FIXED;
      ifnso_plan_t p = nullptr;
      const ifnso_status st = ifnso_plan(&d, num_problems, rows, cols, dtype, dtype, device, &p);
      if (st != IFNSO_OK) {
        ifnso_schedule_plan_destroy(sp);
        return st;  // the message of ifnso_plan stands
      }
      sp->plans.push_back(p);
      keys.insert(keys.end(), {a, b, c, (double)norm});
      found = (int)sp->plans.size() - 1;
      ws_plan = std::max(ws_plan, p->ws_bytes);
    }
    sp->step_plan.push_back(found);
  }
  // iterates between steps: one buffer per problem, rows 16-byte aligned for the 256-tile kernels
  size_t o = align_up(ws_plan, kAlign);
  const size_t es = dtype == IFNSO_F32 ? 4 : 2;
  for (int i = 0; i < num_problems; i++) {
    sp->rows.push_back(rows[i]);
    sp->cols.push_back(cols[i]);
    sp->ld_iter.push_back(round_up(cols[i], 8));
    sp->off_iter.push_back(o);
    o = align_up(o + (size_t)rows[i] * sp->ld_iter.back() * es, kAlign);
  }
  sp->ws_bytes = steps > 1 ? o : ws_plan;
  *out = sp;
  return IFNSO_OK;
}

extern "C" ifnso_status ifnso_schedule_plan_workspace_bytes(ifnso_schedule_plan_t sp, size_t *bytes) {
  if (!sp || !bytes) return fail(IFNSO_ERR_INVALID_ARGUMENT, "NULL argument");
  *bytes = sp->ws_bytes;
  return IFNSO_OK;
}

extern "C" ifnso_status ifnso_schedule_orthogonalize_batched(ifnso_schedule_plan_t sp, const void *const *M,
                                                             const int64_t *ldm, void *const *Y, const int64_t *ldy,
                                                             void *workspace, size_t workspace_bytes, void *stream) {
  if (!sp) return fail(IFNSO_ERR_INVALID_ARGUMENT, "schedule plan is NULL");
  if (!M || !ldm || !Y || !ldy) return fail(IFNSO_ERR_INVALID_ARGUMENT, "NULL pointer array");
  if (!workspace) return fail(IFNSO_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (workspace_bytes < sp->ws_bytes)
    return fail(IFNSO_ERR_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, the schedule needs %zu", workspace_bytes,
                sp->ws_bytes);
  const size_t es = sp->dtype == IFNSO_F32 ? 4 : 2;
  for (int i = 0; i < sp->num; i++) {
    ifnso_status st = check_matrix_args(sp->plans[0], i, M[i], ldm[i], Y[i], ldy[i]);
    if (st != IFNSO_OK) return st;
    const void *t = (const char *)workspace + sp->off_iter[i];
    if (sp->step_plan.size() > 1 &&
        (ranges_overlap(t, matrix_bytes(sp->rows[i], sp->ld_iter[i], sp->cols[i], es), M[i],
                        matrix_bytes(sp->rows[i], ldm[i], sp->cols[i], es)) ||
         ranges_overlap(t, matrix_bytes(sp->rows[i], sp->ld_iter[i], sp->cols[i], es), Y[i],
                        matrix_bytes(sp->rows[i], ldy[i], sp->cols[i], es))))
      return fail(IFNSO_ERR_INVALID_ARGUMENT, "problem %d: M or Y overlaps the workspace", i);
  }
  // the last step writes Y; earlier ones alternate between the iterate buffers and Y
  const int n = (int)sp->step_plan.size();
  std::vector<const void *> src(M, M + sp->num);
  std::vector<int64_t> lsrc(ldm, ldm + sp->num);
  std::vector<void *> tbuf(sp->num);
  for (int i = 0; i < sp->num; i++) tbuf[i] = (char *)workspace + sp->off_iter[i];
  for (int k = 0; k < n; k++) {
    const bool to_y = (n - 1 - k) % 2 == 0;
    std::vector<void *> dst = to_y ? std::vector<void *>(Y, Y + sp->num) : tbuf;
    const int64_t *ld = to_y ? ldy : sp->ld_iter.data();
    ifnso_plan_t p = sp->plans[sp->step_plan[k]];
    const ifnso_status st =
        ifnso_orthogonalize_batched(p, src.data(), lsrc.data(), dst.data(), ld, workspace, workspace_bytes, stream);
    if (st != IFNSO_OK) return st;
    for (int i = 0; i < sp->num; i++) src[i] = dst[i];
    lsrc.assign(ld, ld + sp->num);
  }
  return IFNSO_OK;
}
