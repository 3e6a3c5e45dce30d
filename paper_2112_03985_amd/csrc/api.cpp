// Host side of the JK-CALS library: argument validation, workspace layout,
// model tables, tiling choice and tuning, and the launch sequence of the
// concurrent ALS sweep (Alg. 3).  All device memory comes from the caller's
// workspace; nothing here allocates on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <fstream>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "jkc_internal.hpp"

using namespace jkc;

namespace {

thread_local std::string g_last_error;

jkc_status fail(jkc_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

#define JKC_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(JKC_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));      \
  } while (0)

#define JKC_TRY(expr)                  \
  do {                                 \
    jkc_status s_ = (expr);            \
    if (s_ != JKC_OK) return s_;       \
  } while (0)

constexpr int64_t kAlign = 256;
constexpr int kNumCU = 256;
constexpr int64_t kAllModeLds = 160 * 1024;   // LDS per compute unit on gfx950
constexpr int kSliceChunks = 256;
constexpr size_t kMaxTimedLaunches = 65536;

int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// K step of the split-precision kernels (one v_mfma_f32_16x16x32_bf16 deep).
constexpr int64_t kSplitStep = 32;

// Low mode of the split-precision unfolding of mode n (see Plan::split_low).
int split_low_mode(int N, const int64_t* dims, int n) {
  int best = -1;
  for (int m = 0; m < N; ++m) {
    if (m == n) continue;
    if (best < 0) {
      best = m;
      continue;
    }
    // waste: padded / actual, compared exactly by cross-multiplication
    const int64_t pm = align_up(dims[m], kSplitStep), pb = align_up(dims[best], kSplitStep);
    const int64_t lhs = pm * dims[best], rhs = pb * dims[m];
    if (lhs < rhs || (lhs == rhs && dims[m] > dims[best])) best = m;
  }
  return best;
}

// Sizes derived from a validated problem, shared by the size query and init.
struct Plan {
  int N = 0, nhat = 0, K = 0, C = 0, ldc = 0;
  int64_t dims[kMaxOrder] = {0, 0, 0, 0};
  int64_t strides[kMaxOrder] = {0, 0, 0, 0};
  int64_t P = 0, maxI = 0, gsize = 0;
  int tensor_f32 = 0, precision = 0, copy_tensor = 1;
  int del_d = 1;   // rows of the sampled mode left out per submodel
  int split_max[kMaxOrder] = {1, 1, 1, 1};
  int64_t partial_doubles = 0;
  int64_t tree_rows = 0;   // rows of W (3-way float64 sweeps), 0 when not held
  // one-pass all-mode MTTKRP of the gradient: fibers per step (0: not
  // available), chunks of the last mode, doubles of its split partials
  int allmode_bk = 0;
  int allmode_nchunks = 0;
  int64_t allmode_doubles = 0;

  struct Item {
    const char* name;
    int64_t bytes;
  };
  std::vector<Item> items;
  int64_t total = 0;

  // Split-precision layout of mode n: the unfolding's columns ordered low
  // mode first (the other mode whose size pads to a multiple of the 32-K
  // step with the least waste, the larger size on ties), index padded to
  // split_ilp(n), then the remaining modes ("wraps").
  int split_low(int n) const { return split_low_mode(N, dims, n); }
  int64_t split_ilp(int n) const { return align_up(dims[split_low(n)], kSplitStep); }
  int64_t split_wraps(int n) const { return P / (dims[n] * dims[split_low(n)]); }
  int64_t split_ld(int n) const { return split_ilp(n) * split_wraps(n); }

  void layout() {
    items.clear();
    const int64_t es = tensor_f32 ? 4 : 8;
    int64_t tbytes = 0;
    if (precision != JKC_FP64) {
      // one unfolded copy per mode (rows padded to 8 columns), nterm planes each
      const int nterm = precision == JKC_SPLIT_BF16X6 ? 3 : 2;
      for (int n = 0; n < N; ++n) tbytes += (int64_t)nterm * dims[n] * split_ld(n) * 2;
    } else if (copy_tensor) {
      tbytes = P * es;
    }
    items.push_back({"tensor", tbytes});
    for (int n = 0; n < N; ++n) items.push_back({"U", dims[n] * ldc * 8});
    for (int n = 0; n < N; ++n) items.push_back({"G", gsize * 8});
    for (int n = 0; n < N; ++n) items.push_back({"grad", dims[n] * ldc * 8});
    items.push_back({"M", maxI * ldc * 8});
    items.push_back({"partial", partial_doubles * 8});
    items.push_back({"lambda", (int64_t)ldc * 8});
    items.push_back({"normT2", (int64_t)K * 8});
    items.push_back({"err", (int64_t)K * 8});
    items.push_back({"fit", (int64_t)K * 8});
    items.push_back({"fit_prev", (int64_t)K * 8});
    items.push_back({"eta", (int64_t)K * 8});
    items.push_back({"status", (int64_t)K * 4});
    items.push_back({"iters", (int64_t)K * 4});
    items.push_back({"off", (int64_t)K * 4});
    items.push_back({"rank", (int64_t)K * 4});
    items.push_back({"lomask", dims[nhat] * (int64_t)K});
    items.push_back({"order", (int64_t)K * 4});
    items.push_back({"goff", (int64_t)K * 8});
    items.push_back({"colmodel", (int64_t)ldc * 4});
    items.push_back({"slice", dims[nhat] * 8});
    items.push_back({"slice_part", (int64_t)kSliceChunks * dims[nhat] * 8});
    items.push_back({"counter", 4});
    items.push_back({"upart", update_rows_scratch(maxI, gsize, K) * 8});
    // split paths: the low mode's factor in bfloat16 terms, transposed and
    // padded ([term][ldc][ilp]), refreshed before each MTTKRP
    int64_t usplit = 0;
    if (precision != JKC_FP64) {
      const int nterm = precision == JKC_SPLIT_BF16X6 ? 3 : 2;
      for (int n = 0; n < N; ++n) usplit = std::max(usplit, (int64_t)nterm * ldc * split_ilp(n) * 2);
    }
    items.push_back({"Usplit", usplit});
    // jackknife post-processing: matched components and signed inverse norms
    items.push_back({"jk_perm", (int64_t)ldc * 4});
    items.push_back({"jk_scale", (int64_t)N * ldc * 8});
    // convergence compaction: column map of a relayout
    items.push_back({"colmap", (int64_t)ldc * 4});
    // shared partial contraction of a 3-way sweep
    items.push_back({"tree", tree_rows * ldc * 8});
    items.push_back({"allmode", allmode_doubles * 8});
    total = 0;
    for (auto& it : items) total += align_up(std::max<int64_t>(it.bytes, 1), kAlign);
  }
};

// Upper bound on split-K chunks for a mode: enough to fill the chip twice
// over when the output is small, none when the output alone is large (its
// own tiles fill the chip), and partials bounded to 128 MB or four output
// planes.
int split_cap(int64_t rows, int64_t ldc, int64_t J) {
  const int64_t plane = rows * ldc * 8;
  const int64_t budget = std::max<int64_t>(128ll << 20, 4 * plane);
  int64_t s = budget / std::max<int64_t>(plane, 1);
  // (16-column problems: small planes, and the narrow variant needs more
  // chunks to fill the chip, each of at least 16 fibers)
  s = std::min<int64_t>(s, ldc <= 16 ? 512 : 128);
  s = std::min<int64_t>(s, std::max<int64_t>(1, J / (ldc <= 16 ? 16 : 64)));
  return (int)std::max<int64_t>(s, 1);
}

jkc_status make_plan(const jkc_problem* prob, Plan* pl) {
  if (!prob) return fail(JKC_EINVAL, "problem is NULL");
  if (prob->order < 2 || prob->order > kMaxOrder)
    return fail(JKC_EINVAL, "order must be in 2..4");
  if (!prob->dims) return fail(JKC_EINVAL, "dims is NULL");
  pl->N = prob->order;
  int64_t P = 1;
  for (int n = 0; n < pl->N; ++n) {
    const int64_t d = prob->dims[n];
    if (d < 1 || d > (1ll << 30)) return fail(JKC_EINVAL, "dims must be in 1..2^30");
    pl->dims[n] = d;
    pl->strides[n] = P;
    P *= d;
    if (P > (1ll << 40)) return fail(JKC_EINVAL, "tensor larger than 2^40 elements");
  }
  pl->P = P;
  for (int n = 0; n < pl->N; ++n)
    if (P / pl->dims[n] >= (1ll << 31))
      return fail(JKC_EINVAL, "an unfolding has 2^31 or more columns");
  if (prob->sampled_mode < 0 || prob->sampled_mode >= pl->N)
    return fail(JKC_EINVAL, "sampled_mode out of range");
  pl->nhat = prob->sampled_mode;
  if (prob->num_models < 1) return fail(JKC_EINVAL, "num_models must be >= 1");
  if (!prob->ranks || !prob->left_out) return fail(JKC_EINVAL, "ranks/left_out is NULL");
  pl->K = prob->num_models;
  int64_t C = 0, gsize = 0;
  const int64_t Ih = pl->dims[pl->nhat];
  if (prob->delete_d < 0) return fail(JKC_EINVAL, "delete_d must be >= 0");
  const int d = prob->delete_d > 1 ? prob->delete_d : 1;
  if (d > 1 && d >= Ih) return fail(JKC_EINVAL, "delete_d must leave at least one sample");
  pl->del_d = d;
  std::vector<int64_t> seen(Ih, -1);
  for (int k = 0; k < pl->K; ++k) {
    const int R = prob->ranks[k];
    if (R < 1 || R > kMaxRank) return fail(JKC_EINVAL, "rank must be in 1..32 (model " + std::to_string(k) + ")");
    const int32_t* rows = prob->left_out + (int64_t)k * d;
    const bool full = rows[0] == -1;
    for (int j = 0; j < d; ++j) {
      const int p = rows[j];
      const std::string mk = " (model " + std::to_string(k) + ")";
      if (p < -1 || p >= Ih) return fail(JKC_EINVAL, "left_out out of range" + mk);
      if ((p == -1) != full) return fail(JKC_EINVAL, "left_out mixes -1 and sample indices" + mk);
      if (p >= 0 && Ih < 2) return fail(JKC_EINVAL, "cannot leave out the only sample");
      if (p >= 0) {
        if (seen[p] == k) return fail(JKC_EINVAL, "left_out repeats a sample" + mk);
        seen[p] = k;
      }
    }
    C += R;
    gsize += (int64_t)R * R;
  }
  if (C > (1ll << 28)) return fail(JKC_EINVAL, "too many columns");
  pl->C = (int)C;
  pl->ldc = (int)align_up(C, kColAlign);
  pl->gsize = gsize;
  if (prob->tensor_dtype != JKC_TENSOR_F64 && prob->tensor_dtype != JKC_TENSOR_F32)
    return fail(JKC_EINVAL, "tensor_dtype must be 0 (f64) or 1 (f32)");
  pl->tensor_f32 = prob->tensor_dtype == JKC_TENSOR_F32;
  if (prob->precision != JKC_FP64 && prob->precision != JKC_SPLIT_BF16X3 &&
      prob->precision != JKC_SPLIT_BF16X6)
    return fail(JKC_EINVAL, "precision must be 0 (fp64), 1 (split bf16x3) or 2 (split bf16x6)");
  pl->precision = prob->precision;
  if (prob->copy_tensor != 0 && prob->copy_tensor != 1)
    return fail(JKC_EINVAL, "copy_tensor must be 0 or 1");
  pl->copy_tensor = prob->copy_tensor;
  if (!pl->copy_tensor && pl->precision != JKC_FP64)
    return fail(JKC_EINVAL, "copy_tensor = 0 needs precision JKC_FP64");
  if (pl->precision != JKC_FP64)
    for (int n = 0; n < pl->N; ++n)
      if (pl->dims[n] * pl->split_ld(n) >= (1ll << 31) ||
          pl->dims[n] * (int64_t)pl->ldc >= (1ll << 31) ||
          pl->split_ilp(n) * (int64_t)pl->ldc >= (1ll << 31))
        return fail(JKC_EINVAL, "split precision needs every unfolding and factor below 2^31 elements");
  pl->maxI = 0;
  pl->partial_doubles = 0;
  for (int n = 0; n < pl->N; ++n) {
    pl->maxI = std::max(pl->maxI, pl->dims[n]);
    // split paths cut K at whole wraps
    const int64_t J = pl->precision != JKC_FP64 ? pl->split_wraps(n) * 64 : P / pl->dims[n];
    pl->split_max[n] = split_cap(pl->dims[n], pl->ldc, J);
    if (pl->split_max[n] > 1)
      pl->partial_doubles =
          std::max(pl->partial_doubles, (int64_t)pl->split_max[n] * pl->dims[n] * pl->ldc);
  }
  // W = T x_2 U_2 for 3-way float64 problems, when it takes at most
  // tree_max_gib GiB of the workspace (default 64; its rows i + I_0 j, fewer
  // than 2^31 of them: 32-bit row index in the kernel), with I_0, I_1 at
  // most 100000
  pl->tree_rows = 0;
  const int64_t tree_cap = prob->tree_max_gib == 0 ? (int64_t(64) << 30)
                           : prob->tree_max_gib < 0 ? -1
                                                    : (int64_t)prob->tree_max_gib << 30;
  if (pl->N == 3 && pl->precision == JKC_FP64 && pl->dims[0] <= 100000 && pl->dims[1] <= 100000 &&
      pl->dims[0] * pl->dims[1] < (int64_t(1) << 31) &&   // W's rows are 32-bit in the kernel
      pl->dims[0] * pl->dims[1] * (int64_t)pl->ldc * 8 <= tree_cap)
    pl->tree_rows = pl->dims[0] * pl->dims[1];
  // one-pass all-mode MTTKRP: 3- and 4-way float64 problems with at most 256
  // rows in mode 0 whose block fits in LDS; enough chunks of the last mode to
  // give the chip about one block per compute unit
  pl->allmode_bk = 0;
  if ((pl->N == 3 || pl->N == 4) && pl->precision == JKC_FP64 && pl->dims[0] <= 256 &&
      pl->dims[1] <= 65536 && pl->dims[2] <= 65536 &&
      P * (pl->tensor_f32 ? 4 : 8) < (int64_t(1) << 31)) {   // 32-bit buffer offsets
    const int nt = allmode_row_tiles((int)pl->dims[0]);
    for (int bk : {16, 8})
      if (allmode_has_kernel(nt, bk) &&
          allmode_lds_bytes(nt * 16, bk, (int)pl->dims[1], (int)pl->dims[2], pl->N) <= kAllModeLds) {
        pl->allmode_bk = bk;
        break;
      }
    if (pl->allmode_bk > 0) {
      const int64_t ntiles = (pl->ldc + kAllModeCols - 1) / kAllModeCols;
      const int64_t last = pl->dims[pl->N - 1];
      // (one block per compute unit at most: a second round of blocks
      // would double the time)
      const int64_t want = std::max<int64_t>(1, kNumCU / ntiles);
      pl->allmode_nchunks = (int)std::min<int64_t>(last, want);
      int64_t rows = 0;
      for (int m = 0; m + 1 < pl->N; ++m) rows += pl->dims[m];
      pl->allmode_doubles = pl->allmode_nchunks * rows * pl->ldc;
    }
  }
  pl->layout();
  return JKC_OK;
}

// ---------------------------------------------------------------------------
// Tiling choice.
// ---------------------------------------------------------------------------
struct ModeShape {
  int64_t M, J;
  int ncols, ldc, split_max;
  bool buf_ok;   // tensor and factors addressable with 32-bit byte offsets
  int64_t i0 = 0;       // size of mode 0 (the fibers the narrow variant walks)
  bool mode0 = false;   // the output mode is mode 0 (rows contiguous)
  int order = 0;        // N
};

// The narrow variant's fibers (all of them for mode 0, one output row's
// otherwise) and the fewest K chunks that hold them.
int64_t narrow_fibers(const ModeShape& s) { return s.mode0 ? s.J : s.J / std::max<int64_t>(s.i0, 1); }
int64_t narrow_min_splits(const ModeShape& s) {
  const int64_t cap = narrow_max_chunk_fibers((int)s.i0, s.ncols, s.mode0, s.order);
  return (narrow_fibers(s) + cap - 1) / cap;
}

// Float64 kernels with buffer loads (instr bit 16) address the tensor and
// the factors with 32-bit byte offsets: usable when each is below 2^31
// bytes (with room for the walk past the end of the last K chunk).
constexpr int64_t kBufLimit = (int64_t(1) << 31) - (int64_t(1) << 24);
bool usable(const MttkrpVariant& x, const ModeShape& s) {
  if (x.instr & kNarrowInstr)
    return s.ldc == 16 && s.i0 > 0 && narrow_supports((int)std::min<int64_t>(s.i0, 1 << 20), s.ncols) &&
           (s.mode0 ? s.M == s.i0 : true) && narrow_min_splits(s) <= s.split_max;
  return !(x.instr & 16) || s.buf_ok;
}

Tiling make_tiling(const std::vector<MttkrpVariant>& vars, int v, const ModeShape& s, int splits) {
  Tiling t;
  const auto& x = vars[v];
  t.variant = v;
  t.wm = x.wm; t.wn = x.wn; t.tm = x.tm; t.tn = x.tn; t.bk = x.bk; t.instr = x.instr;
  t.splits = std::max(1, std::min(splits, s.split_max));
  return t;
}

int default_splits(const Tiling& t, const ModeShape& s) {
  if (t.instr & kNarrowInstr) {
    // the largest chunks (the fewest partials; a mode > 0 row in one block
    // where it fits), with at least one block per compute unit for modes
    // n > 0 (two chunks per row on the 200-row modes of the benchmark: the
    // update sums two partials itself, so no reduction pass follows)
    int64_t sp = narrow_min_splits(s);
    if (!s.mode0 && s.M < kNumCU)
      sp = std::max(sp, std::min(narrow_fibers(s), (kNumCU + s.M - 1) / s.M));
    return (int)std::max<int64_t>(1, std::min<int64_t>(sp, s.split_max));
  }
  const int64_t tiles = ((s.M + t.bm() - 1) / t.bm()) * ((s.ncols + t.bn() - 1) / t.bn());
  // aim for two resident blocks per compute unit (one of 8 wavefronts)
  const int64_t want_blocks = (t.wm * t.wn >= 8 ? 1 : 2) * kNumCU;
  int64_t s_ = (want_blocks + tiles - 1) / tiles;
  s_ = std::min<int64_t>(s_, std::max<int64_t>(1, s.J / (8 * t.bk)));
  return (int)std::max<int64_t>(1, std::min<int64_t>(s_, s.split_max));
}

// Relative time estimate of a tiling (lower is better): padded matrix-core
// work, divided by how well one step's MFMA work hides its fixed load/barrier
// cost and by how well the grid fills the chip, plus split-K partial traffic.
double model_cost(const Tiling& t, const ModeShape& s) {
  // the narrow variant streams the tensor once at the HBM rate; the
  // matrix-core tilings pad 16 columns to their tile width
  if (t.instr & kNarrowInstr) return 0.5;
  const int64_t mt = (s.M + t.bm() - 1) / t.bm();
  const int64_t nt = (s.ncols + t.bn() - 1) / t.bn();
  const double useful = (double)s.M * s.ncols;
  const double padded = (double)mt * t.bm() * nt * t.bn();
  const int fam = t.instr & 7;
  const double per_step = (double)t.tm * t.tn * (t.bk / 4) * (fam == 0 ? 1.45 : fam == 2 ? 0.25 : 1.0);
  // the interleaved schedule hides more of the fixed cost; an 8-wavefront
  // block keeps two wavefronts on every SIMD
  const double hide =
      per_step / (per_step + ((t.instr & 16) ? 2.0 : (t.instr & 8) ? 3.0 : 6.0));
  const double blocks = (double)mt * nt * t.splits;
  const double per_cu = t.wm * t.wn >= 8 ? 1.0 : 2.0;
  const double fill = std::min(1.0, blocks / (per_cu * kNumCU)) * std::min(1.0, (double)(t.wm * t.wn) / 4.0) *
                      (t.wm * t.wn >= 8 ? 1.1 : 1.0);
  double cost = (padded / useful) / (hide * std::max(fill, 1e-3));
  if (t.splits > 1) cost *= 1.0 + 96.0 * t.splits / (double)s.J;
  return cost;
}

Tiling choose_tiling(const std::vector<MttkrpVariant>& vars, const ModeShape& s) {
  Tiling best;
  double best_cost = std::numeric_limits<double>::infinity();
  for (int v = 0; v < (int)vars.size(); ++v) {
    if (!usable(vars[v], s)) continue;
    Tiling t = make_tiling(vars, v, s, 1);
    t.splits = default_splits(t, s);
    const double c = model_cost(t, s);
    if (c < best_cost) {
      best_cost = c;
      best = t;
    }
  }
  return best;
}

ModeShape mode_shape(const jkc_ctx* ctx, int n, int split_max) {
  ModeShape s;
  s.M = ctx->dims[n];
  s.J = ctx->nterm > 0 ? (int64_t)ctx->tp_ilp[n] * (ctx->P / (ctx->dims[n] * ctx->dims[ctx->tp_low[n]]))
                       : ctx->P / ctx->dims[n];
  s.ncols = ctx->C;
  s.ldc = ctx->ldc;
  s.split_max = split_max;
  bool ok = ctx->P * (ctx->tensor_f32 ? 4 : 8) < kBufLimit;
  for (int m = 0; m < ctx->N; ++m) ok = ok && ctx->dims[m] * ctx->ldc * 8 < kBufLimit;
  s.buf_ok = ok;
  s.i0 = ctx->nterm > 0 ? 0 : ctx->dims[0];   // float64 path only
  s.mode0 = n == 0;
  s.order = ctx->N;
  return s;
}

// W = T x_2 U_2 as the MTTKRP of the two-way view of T (rows i + I_0 j,
// contraction over k): no split-K (its output alone fills the chip).
ModeShape tree_shape(const jkc_ctx* ctx) {
  ModeShape s;
  s.M = ctx->dims[0] * ctx->dims[1];
  s.J = ctx->dims[2];
  s.ncols = ctx->C;
  s.ldc = ctx->ldc;
  s.split_max = 1;
  s.buf_ok = ctx->P * (ctx->tensor_f32 ? 4 : 8) < kBufLimit && ctx->dims[2] * ctx->ldc * 8 < kBufLimit;
  return s;
}

std::string describe_tiling(const Tiling& t, int precision) {
  char buf[128];
  const int fam = t.instr & 7;
  snprintf(buf, sizeof(buf), "%s v%d wm%d wn%d tm%d tn%d bk%d s%d %s%s%s",
           precision == JKC_SPLIT_BF16X3 ? "bf16x3" : precision == JKC_SPLIT_BF16X6 ? "bf16x6" : "f64",
           t.variant, t.wm, t.wn, t.tm, t.tn, t.bk, t.splits,
           precision != JKC_FP64 ? "mfma16x16x32bf16"
           : (t.instr & kNarrowInstr) ? "valu-narrow"
           : fam == 2            ? "mfma4x4x4-strips"
           : fam == 1            ? "mfma4x4x4-diagonal"
                                 : "mfma16x16x4",
           (precision == JKC_FP64 && (t.instr & 8)) ? "-interleaved" : "",
           (precision == JKC_FP64 && (t.instr & 16)) ? "-buffer" : "");
  return buf;
}

// ---------------------------------------------------------------------------
// Tuning cache: the tiling jk_cals_tune found for a (precision, shape, mode),
// kept for the life of the process and, when JKC_TUNE_CACHE names a file,
// stored there as text ("key|variant geometry|splits" per line).
// ---------------------------------------------------------------------------
struct TuneEntry {
  int wm, wn, tm, tn, bk, instr, splits;
};
std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune;
bool g_tune_loaded = false;

// tuning-cache slot of the shared partial contraction's tiling
constexpr int kTreeSlot = 99;

std::string tune_key(const jkc_ctx* c, int n) {
  std::ostringstream o;
  o << "gfx950 p" << c->precision << " f32_" << c->tensor_f32 << " N" << c->N << " d";
  for (int m = 0; m < c->N; ++m) o << (m ? "x" : "") << c->dims[m];
  o << " ldc" << c->ldc;
  if (n == kTreeSlot) o << " tree";
  else o << " mode" << n;
  return o.str();
}

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("JKC_TUNE_CACHE");
  if (!path || !*path) return;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t a = line.find('|');
    if (a == std::string::npos) continue;
    TuneEntry e{};
    if (sscanf(line.c_str() + a + 1, "%d %d %d %d %d %d|%d", &e.wm, &e.wn, &e.tm, &e.tn, &e.bk,
               &e.instr, &e.splits) == 7)
      g_tune[line.substr(0, a)] = e;
  }
}

void tune_save_locked() {
  const char* path = std::getenv("JKC_TUNE_CACHE");
  if (!path || !*path) return;
  std::ofstream f(path, std::ios::trunc);
  for (const auto& kv : g_tune) {
    const TuneEntry& e = kv.second;
    f << kv.first << "|" << e.wm << " " << e.wn << " " << e.tm << " " << e.tn << " " << e.bk << " "
      << e.instr << "|" << e.splits << "\n";
  }
}

// Cached tiling for (ctx, mode) if one exists and still names a compiled
// kernel; returns false otherwise.
bool tune_lookup(const jkc_ctx* c, int n, const std::vector<MttkrpVariant>& vars,
                 const ModeShape& shape, Tiling* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  auto it = g_tune.find(tune_key(c, n));
  if (it == g_tune.end()) return false;
  const TuneEntry& e = it->second;
  for (int v = 0; v < (int)vars.size(); ++v) {
    const auto& x = vars[v];
    if (x.wm == e.wm && x.wn == e.wn && x.tm == e.tm && x.tn == e.tn && x.bk == e.bk &&
        x.instr == e.instr && usable(x, shape)) {
      *out = make_tiling(vars, v, shape, e.splits);
      return true;
    }
  }
  return false;
}

void tune_store(const jkc_ctx* c, int n, const Tiling& t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  g_tune[tune_key(c, n)] = TuneEntry{t.wm, t.wn, t.tm, t.tn, t.bk, t.instr, t.splits};
  tune_save_locked();
}

// ---------------------------------------------------------------------------
// Launch helpers.
// ---------------------------------------------------------------------------
// Float64 tilings: the matrix-core variants, then the narrow vector-ALU one.
const std::vector<MttkrpVariant>& f64_variants_all() {
  static const std::vector<MttkrpVariant> v = [] {
    std::vector<MttkrpVariant> x = mttkrp_f64_variants();
    x.push_back(mttkrp_narrow_variant());
    return x;
  }();
  return v;
}

const std::vector<MttkrpVariant>& variants_for(const jkc_ctx* ctx) {
  if (ctx->precision == JKC_SPLIT_BF16X3) return mttkrp_split_variants();
  if (ctx->precision == JKC_SPLIT_BF16X6) return mttkrp_split3_variants();
  return f64_variants_all();
}

jkc_status launch_mttkrp_timed(jkc_ctx* ctx, const MttkrpArgs& a, const Tiling& t, int slot,
                               bool reduce_follows);

// K chunking of mode n's MTTKRP under tiling t: K elements per split and
// the number of splits (split paths: whole wraps of the low mode).
void chunking(const jkc_ctx* ctx, int n, const Tiling& t, int64_t* kchunk, int* splits) {
  int64_t J, step;
  if (ctx->nterm > 0) {
    J = ctx->P / (ctx->dims[n] * ctx->dims[ctx->tp_low[n]]);   // wraps
    step = 1;
  } else if (t.instr & kNarrowInstr) {
    // the narrow variant: chunks of whole mode-0 fibers (of one output row
    // for n > 0), at most what one block takes
    const int64_t I0 = ctx->dims[0];
    const int64_t fib = n == 0 ? ctx->P / I0 : ctx->P / (I0 * ctx->dims[n]);
    const int64_t cap =
        narrow_max_chunk_fibers((int)std::min<int64_t>(I0, 1 << 20), ctx->C_act, n == 0, ctx->N);
    const int64_t kcf = std::min<int64_t>(std::max<int64_t>(1, (fib + t.splits - 1) / t.splits), cap);
    *kchunk = n == 0 ? kcf : kcf * I0;
    *splits = (int)((fib + kcf - 1) / kcf);
    return;
  } else {
    J = ctx->P / ctx->dims[n];
    step = t.bk;
  }
  int64_t kc = align_up((J + t.splits - 1) / t.splits, step);
  *kchunk = kc;
  *splits = (int)((J + kc - 1) / kc);
}

// Enqueue the fused MTTKRP of mode n.  Result: split-K partials in
// ctx->partial (t.splits > 1) or the product itself in ctx->Mbuf; with fin
// (the narrow tiling only), the reduced product in fin->out instead.  When
// reduce_follows, the reduction launched next (launch_reduce_timed) closes
// the launch's timing window.
// Reduced output of an MTTKRP whose kernels sum their own split-K partials
// (the narrow tiling): out (ld ldo, ncols columns), Case I rows cleared when
// zero_rows.
struct FinOut {
  double* out;
  int32_t ldo, ncols, zero_rows;
};

jkc_status enqueue_mttkrp(jkc_ctx* ctx, int n, const Tiling& t, bool reduce_follows = false,
                          const FinOut* fin = nullptr) {
  const auto& vars = variants_for(ctx);
  if (t.variant < 0 || t.variant >= (int)vars.size()) return fail(JKC_ESTATE, "no tiling");
  MttkrpArgs a{};
  a.t_is_f32 = ctx->tensor_f32;
  int q = 0;
  for (int m = 0; m < ctx->N; ++m) {
    if (m == n) continue;
    a.oU[q] = ctx->U[m];
    a.odim[q] = (int32_t)ctx->dims[m];
    a.ostride[q] = ctx->strides[m];
    ++q;
  }
  for (; q < kMaxOrder - 1; ++q) {
    a.oU[q] = nullptr;
    a.odim[q] = 1;
    a.ostride[q] = 0;
  }
  a.nother = ctx->N - 1;
  a.stride_n = ctx->strides[n];
  a.M = (int32_t)ctx->dims[n];
  a.J = ctx->P / ctx->dims[n];
  if (ctx->nterm > 0) {
    // the low mode's factor split into bfloat16 terms, transposed and padded
    const int low = ctx->tp_low[n];
    a.il = (int32_t)ctx->dims[low];
    a.ilp = ctx->tp_ilp[n];
    a.wraps = ctx->P / (ctx->dims[n] * ctx->dims[low]);
    a.ldt = (int64_t)a.ilp * a.wraps;
    a.J = a.ldt;
    a.T = ctx->T_planes + ctx->tp_off[n];
    a.plane = ctx->dims[n] * a.ldt;
    a.ut = ctx->Usplit;
    a.ut_plane = (int64_t)ctx->ldc * a.ilp;
    JKC_HIP(launch_split_factor_t(ctx->U[low], a.il, ctx->ldc, a.ilp, ctx->nterm, ctx->Usplit,
                                  ctx->stream));
    a.nh = 0;
    for (int m = 0; m < ctx->N; ++m) {
      if (m == n || m == low) continue;
      a.hU[a.nh] = ctx->U[m];
      a.hdim[a.nh] = (int32_t)ctx->dims[m];
      ++a.nh;
    }
    for (int h = a.nh; h < kMaxOrder - 2; ++h) {
      a.hU[h] = nullptr;
      a.hdim[h] = 1;
    }
  } else {
    a.T = ctx->T;
    a.plane = 0;
  }
  a.ldc = ctx->ldc;
  a.ncols = ctx->C_act;
  a.mtiles = (int32_t)((a.M + t.bm() - 1) / t.bm());
  a.ntiles = (int32_t)((a.ncols + t.bn() - 1) / t.bn());
  int64_t kchunk = 0;
  int splits = 1;
  chunking(ctx, n, t, &kchunk, &splits);
  a.kchunk = kchunk;
  a.splits = splits;
  if (splits > 1) {
    if ((int64_t)splits * a.M * a.ldc > ctx->partial_doubles)
      return fail(JKC_ESTATE, "split-K partial buffer too small");
    a.partial = ctx->partial;
  } else {
    a.partial = ctx->Mbuf;
  }
  if (fin) {
    if (!(t.instr & kNarrowInstr)) return fail(JKC_ESTATE, "tiling has no split-K finish");
    a.fin_out = fin->out;
    a.fin_ldo = fin->ldo;
    a.fin_ncols = fin->ncols;
    a.fin_zero = fin->zero_rows;
    a.fin_lo = ctx->left_out();
  }
  return launch_mttkrp_timed(ctx, a, t, n, reduce_follows);
}

// Launch a filled MTTKRP, timed in profiling slot `slot` while
// jk_cals_profile is on (slots 0..N-1: the fused MTTKRP of that mode with
// its split-K reduction; slot N: the shared contraction W).  The dispatch
// stamps the start event; the stop event is stamped by this dispatch, or,
// when reduce_follows, by the reduction's.
jkc_status launch_mttkrp_timed(jkc_ctx* ctx, const MttkrpArgs& a, const Tiling& t, int slot,
                               bool reduce_follows) {
  const auto& vars = variants_for(ctx);
  const int n = slot;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (ctx->prof_on && ctx->prof_used < kMaxTimedLaunches) {
    const size_t i = ctx->prof_used;
    if (ctx->prof_ev.size() < 2 * (i + 1)) {
      hipEvent_t a0, a1;
      JKC_HIP(hipEventCreate(&a0));
      if (hipEventCreate(&a1) != hipSuccess) {
        (void)hipEventDestroy(a0);
        return fail(JKC_EDEVICE, "hipEventCreate failed");
      }
      ctx->prof_ev.push_back(a0);
      ctx->prof_ev.push_back(a1);
      ctx->prof_mode.push_back(n);
    }
    ctx->prof_mode[i] = n;
    ev0 = ctx->prof_ev[2 * i];
    ev1 = ctx->prof_ev[2 * i + 1];
    ++ctx->prof_used;
  }
  ctx->prof_pending_stop = nullptr;
  if (reduce_follows) {
    ctx->prof_pending_stop = ev1;
    ev1 = nullptr;
  }
  JKC_HIP(vars[t.variant].launch(a, ctx->stream, ev0, ev1));
  return JKC_OK;
}

// The split-K reduction of the MTTKRP launched just before (stamps that
// launch's pending stop event, if any).
jkc_status launch_reduce_timed(jkc_ctx* ctx, const double* partial, int32_t splits, int32_t rows,
                               int32_t ncols, int32_t zero_rows, double* out, int32_t ldo) {
  hipEvent_t stop = ctx->prof_pending_stop;
  ctx->prof_pending_stop = nullptr;
  JKC_HIP(launch_reduce(partial, splits, rows, ctx->ldc, ncols, ctx->left_out(), zero_rows, out, ldo,
                        ctx->stream, stop));
  return JKC_OK;
}

int effective_splits(const jkc_ctx* ctx, int n, const Tiling& t) {
  int64_t kchunk = 0;
  int splits = 1;
  chunking(ctx, n, t, &kchunk, &splits);
  return splits;
}

// Whether the reduced MTTKRP of mode n under tiling t into out has the Case
// I rows cleared: always, except for an unsplit product left in Mbuf by a
// kernel without its own finish (the consumer clears them).
bool reduced_clears_rows(const jkc_ctx* ctx, int n, const Tiling& t, const double* out) {
  if (t.instr & kNarrowInstr) return true;
  return !(effective_splits(ctx, n, t) == 1 && out == ctx->Mbuf);
}

// MTTKRP of mode n under tiling t reduced into out (ld ldo, ncols columns),
// with the Case I row removal when n is the sampled mode (see
// reduced_clears_rows for the one exception).
jkc_status enqueue_mttkrp_reduced(jkc_ctx* ctx, int n, const Tiling& t, double* out, int ldo,
                                  int ncols) {
  const int zero = n == ctx->nhat ? 1 : 0;
  if (t.instr & kNarrowInstr) {   // the kernels sum their own partials
    const FinOut fin{out, ldo, ncols, zero};
    return enqueue_mttkrp(ctx, n, t, false, &fin);
  }
  const int splits = effective_splits(ctx, n, t);
  const bool reduce = reduced_clears_rows(ctx, n, t, out);
  JKC_TRY(enqueue_mttkrp(ctx, n, t, reduce));
  if (!reduce) return JKC_OK;
  const double* src = splits > 1 ? ctx->partial : ctx->Mbuf;
  return launch_reduce_timed(ctx, src, splits, (int32_t)ctx->dims[n], ncols, zero, out, ldo);
}

jkc_status enqueue_mttkrp_reduced(jkc_ctx* ctx, int n, double* out, int ldo, int ncols) {
  return enqueue_mttkrp_reduced(ctx, n, ctx->tiling[n], out, ldo, ncols);
}

// W = T x_2 U_2 over the active columns (tree.hip explains the scheme):
// the fused MTTKRP kernel on the two-way view of T, rows i + I_0 j (stride
// 1), contraction over k (stride I_0 I_1); timed as mode 0's MTTKRP.
jkc_status enqueue_tree_w(jkc_ctx* ctx) {
  const Tiling& t = ctx->tree_tiling;
  const auto& vars = variants_for(ctx);
  if (t.variant < 0 || t.variant >= (int)vars.size()) return fail(JKC_ESTATE, "no tiling");
  MttkrpArgs a{};
  a.T = ctx->T;
  a.plane = 0;
  a.t_is_f32 = ctx->tensor_f32;
  a.oU[0] = ctx->U[2];
  a.odim[0] = (int32_t)ctx->dims[2];
  a.ostride[0] = ctx->strides[2];
  for (int q = 1; q < kMaxOrder - 1; ++q) {
    a.oU[q] = nullptr;
    a.odim[q] = 1;
    a.ostride[q] = 0;
  }
  a.nother = 1;
  a.stride_n = 1;
  a.M = (int32_t)(ctx->dims[0] * ctx->dims[1]);
  a.J = ctx->dims[2];
  a.ldc = ctx->ldc;
  a.ncols = ctx->C_act;
  a.mtiles = (int32_t)((a.M + t.bm() - 1) / t.bm());
  a.ntiles = (int32_t)((a.ncols + t.bn() - 1) / t.bn());
  a.kchunk = align_up(a.J, t.bk);
  a.splits = 1;
  a.partial = ctx->Wtree;
  JKC_TRY(launch_mttkrp_timed(ctx, a, t, ctx->N, false));
  ctx->tree_fresh = true;
  return JKC_OK;
}

// M_n for n = 0 or 1 from W into out ([I_n][ldc]; rows of the left-out
// samples are cleared by the consumer, as for the fused kernel).
jkc_status enqueue_tree_pass(jkc_ctx* ctx, int n, double* out) {
  const int64_t I0 = ctx->dims[0], I1 = ctx->dims[1];
  if (n == 0)   // M_0(i, c) = sum_j W(i + I_0 j, c) U_1(j, c)
    JKC_HIP(launch_tree_pass(ctx->Wtree, ctx->U[1], (int32_t)I1, 1, I0, (int32_t)I0, ctx->ldc,
                             ctx->C_act, out, ctx->stream));
  else          // M_1(j, c) = sum_i W(i + I_0 j, c) U_0(i, c)
    JKC_HIP(launch_tree_pass(ctx->Wtree, ctx->U[0], (int32_t)I0, I0, 1, (int32_t)I1, ctx->ldc,
                             ctx->C_act, out, ctx->stream));
  return JKC_OK;
}

jkc_status enqueue_update(jkc_ctx* ctx, int n, double tol, int check_conv) {
  constexpr int64_t kLdsBudget = 64 * 1024;
  constexpr int kFuseMaxSplits = 2;
  const int64_t lds = update_lds_doubles(ctx->rmax, (int)ctx->dims[n]);
  const bool staged = ctx->update_kernel == 0 && lds * 8 <= kLdsBudget;
  // modes 0 and 1 of a 3-way sweep from the shared contraction W (mode 1
  // only right after mode 0 has formed it)
  const bool tree = ctx->use_tree && (n == 0 || (n == 1 && ctx->tree_fresh));
  if (n != 0) ctx->tree_fresh = false;
  const int splits = tree ? 1 : effective_splits(ctx, n, ctx->tiling[n]);
  UpdateArgs a{};
  if (tree) {
    if (n == 0) JKC_TRY(enqueue_tree_w(ctx));
    JKC_TRY(enqueue_tree_pass(ctx, n, ctx->Mbuf));
    a.partial = ctx->Mbuf;
    a.splits = 1;
    if (ctx->update_kernel == 2) {
      a.scratch = ctx->upart;
      a.Utmp = ctx->Mbuf;
      a.nch = (int32_t)((ctx->maxI + kUpdRows - 1) / kUpdRows);
    } else if (staged) {
      a.lds_doubles = lds;
    } else {
      a.partial = nullptr;
      a.lds_doubles = 0;
    }
  } else if (ctx->update_kernel == 2) {
    // row-parallel: the solve kernel sums the split-K partials itself
    JKC_TRY(enqueue_mttkrp(ctx, n, ctx->tiling[n]));
    a.partial = splits > 1 ? ctx->partial : ctx->Mbuf;
    a.splits = splits;
    a.scratch = ctx->upart;
    // staging for the unnormalised rows: Mbuf (when it holds the MTTKRP
    // itself, each element is read and then overwritten by the same block)
    a.Utmp = ctx->Mbuf;
    a.nch = (int32_t)((ctx->maxI + kUpdRows - 1) / kUpdRows);
  } else if (staged && splits <= kFuseMaxSplits) {
    // few partials: the update sums them itself while staging M in LDS
    JKC_TRY(enqueue_mttkrp(ctx, n, ctx->tiling[n]));
    a.partial = splits > 1 ? ctx->partial : ctx->Mbuf;
    a.splits = splits;
    a.lds_doubles = lds;
  } else if (staged) {
    // many partials: a full-chip reduction first, then the staged update
    JKC_TRY(enqueue_mttkrp_reduced(ctx, n, ctx->Mbuf, ctx->ldc, ctx->ldc));
    a.partial = ctx->Mbuf;
    a.splits = 1;
    a.lds_doubles = lds;
  } else {
    JKC_TRY(enqueue_mttkrp_reduced(ctx, n, ctx->Mbuf, ctx->ldc, ctx->ldc));
    a.partial = nullptr;
    a.splits = 1;
    a.lds_doubles = 0;
  }
  a.mt = ctx->table();
  a.N = ctx->N;
  a.n = n;
  a.nhat = ctx->nhat;
  a.In = (int32_t)ctx->dims[n];
  a.ldc = ctx->ldc;
  a.Mout = ctx->Mbuf;
  a.U = ctx->U[n];
  for (int m = 0; m < kMaxOrder; ++m) a.G[m] = ctx->G[m];
  a.lambda = ctx->lambda;
  a.normT2 = ctx->normT2;
  a.err = ctx->err;
  a.fit = ctx->fit;
  a.fit_prev = ctx->fit_prev;
  a.status = ctx->status;
  a.iters = ctx->iters;
  a.last_mode = (n == ctx->N - 1) ? 1 : 0;
  a.tol = tol;
  a.check_conv = check_conv;
  a.rmax = ctx->rmax;
  a.uniform_rank = (ctx->uniform_rank > 0 && ctx->h_off == ctx->h_off_canon) ? ctx->uniform_rank : 0;
  if (ctx->update_kernel == 2)
    JKC_HIP(launch_update_rows(a, ctx->stream));
  else
    JKC_HIP(launch_update(a, ctx->stream));
  return JKC_OK;
}

void drop_graph(jkc_ctx* ctx) {
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  ctx->graph_exec = nullptr;
}

// One sweep (all modes: MTTKRP, reduction, update) captured once into a HIP
// graph on a private stream, then replayed on the context's stream: the
// sweep is a fixed chain of kernels whose arguments never change for the
// life of the context (buffers live in the workspace; tilings only change
// through calls that drop the graph).  The graph holds kernel nodes only.
jkc_status build_sweep_graph(jkc_ctx* ctx) {
  if (ctx->graph_exec) return JKC_OK;
  hipStream_t cap = nullptr;
  JKC_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipStream_t user = ctx->stream;
  ctx->stream = cap;
  jkc_status st = JKC_OK;
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    st = fail(JKC_EDEVICE, "hipStreamBeginCapture failed");
  } else {
    for (int n = 0; n < ctx->N && st == JKC_OK; ++n) st = enqueue_update(ctx, n, 0.0, 0);
    const hipError_t e = hipStreamEndCapture(cap, &graph);
    if (st == JKC_OK && e != hipSuccess) st = fail(JKC_EDEVICE, "hipStreamEndCapture failed");
  }
  ctx->stream = user;
  if (st == JKC_OK && hipGraphInstantiate(&ctx->graph_exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    ctx->graph_exec = nullptr;
    st = fail(JKC_EDEVICE, "hipGraphInstantiate failed");
  }
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(cap);
  return st;
}

jkc_status enqueue_sweeps(jkc_ctx* ctx, int nsweeps, double tol, int check_conv) {
  const bool graph = ctx->use_graph && !ctx->prof_on && !check_conv && nsweeps > 1;
  if (graph) {
    JKC_TRY(build_sweep_graph(ctx));
    for (int s = 0; s < nsweeps; ++s) JKC_HIP(hipGraphLaunch(ctx->graph_exec, ctx->stream));
  } else {
    for (int s = 0; s < nsweeps; ++s)
      for (int n = 0; n < ctx->N; ++n) JKC_TRY(enqueue_update(ctx, n, tol, check_conv));
  }
  if (nsweeps > 0) ctx->lambda_is_one = false;
  return JKC_OK;
}

// Gram blocks of modes n0 .. n1-1 in one launch; with eta, each mode's
// factor first takes the gradient step U_n -= eta_k grad_n (same launch).
jkc_status enqueue_grams(jkc_ctx* ctx, int n0, int n1, const double* eta = nullptr) {
  GramArgs g{};
  g.mt = ctx->table();
  g.ldc = ctx->ldc;
  g.nmodes = n1 - n0;
  for (int q = 0; q < g.nmodes; ++q) {
    g.rows[q] = (int32_t)ctx->dims[n0 + q];
    g.U[q] = ctx->U[n0 + q];
    g.G[q] = ctx->G[n0 + q];
    g.grad[q] = ctx->grad[n0 + q];
  }
  g.eta = eta;
  g.uniform_rank = (ctx->uniform_rank > 0 && ctx->h_off == ctx->h_off_canon) ? ctx->uniform_rank : 0;
  JKC_HIP(launch_gram(g, ctx->stream));
  return JKC_OK;
}

jkc_status enqueue_gram(jkc_ctx* ctx, int n) { return enqueue_grams(ctx, n, n + 1); }

jkc_status enqueue_fold_lambda(jkc_ctx* ctx) {
  if (ctx->lambda_is_one) return JKC_OK;
  const int n = ctx->N - 1;
  JKC_HIP(launch_fold_lambda(ctx->U[n], (int32_t)ctx->dims[n], ctx->ldc, ctx->C, ctx->lambda,
                             ctx->stream));
  JKC_TRY(enqueue_gram(ctx, n));
  ctx->lambda_is_one = true;
  return JKC_OK;
}

// All-mode gradient at the current factors (lambda folded), loss optional.
// Loss and gradient assembly of every mode, in one launch, from the MTTKRPs
// held in ctx->grad[n] (in place: the gradient overwrites its MTTKRP).
jkc_status enqueue_grad_assemble(jkc_ctx* ctx, double* loss) {
  GradArgs g{};
  g.mt = ctx->table();
  g.N = ctx->N;
  g.nhat = ctx->nhat;
  g.n0 = 0;
  g.nmodes = ctx->N;
  g.ldc = ctx->ldc;
  for (int m = 0; m < kMaxOrder; ++m) {
    g.In[m] = m < ctx->N ? (int32_t)ctx->dims[m] : 0;
    g.Mfull[m] = m < ctx->N ? ctx->grad[m] : nullptr;
    g.U[m] = m < ctx->N ? ctx->U[m] : nullptr;
    g.Gp[m] = ctx->G[m];
    g.grad[m] = m < ctx->N ? ctx->grad[m] : nullptr;
  }
  g.normT2 = ctx->normT2;
  g.loss = loss;
  g.uniform_rank = (ctx->uniform_rank > 0 && ctx->h_off == ctx->h_off_canon) ? ctx->uniform_rank : 0;
  JKC_HIP(launch_grad_assemble(g, ctx->stream));
  return JKC_OK;
}

// All-mode MTTKRP in one pass over T (allmode.hip) into ctx->grad[n]: the
// last mode written directly, modes 0 .. N-2 reduced from their per-chunk
// partials in a fixed order.  Rows of the sampled mode's left-out samples
// are left as computed: the gradient assembly holds them at 0 and their
// factor rows are 0.
jkc_status enqueue_allmode(jkc_ctx* ctx) {
  AllModeArgs a{};
  a.T = ctx->T;
  a.tbytes = ctx->P * (ctx->tensor_f32 ? 4 : 8);
  a.t_is_f32 = ctx->tensor_f32;
  a.N = ctx->N;
  for (int m = 0; m < kMaxOrder; ++m) {
    a.dims[m] = m < ctx->N ? (int32_t)ctx->dims[m] : 1;
    a.U[m] = m < ctx->N ? ctx->U[m] : nullptr;
  }
  a.ldc = ctx->ldc;
  a.i0p = 16 * allmode_row_tiles((int)ctx->dims[0]);
  a.bk = ctx->allmode_bk;
  const int64_t last = ctx->dims[ctx->N - 1];
  a.nchunks = ctx->allmode_nchunks;
  a.chunk = (int32_t)((last + a.nchunks - 1) / a.nchunks);
  a.nchunks = (int32_t)((last + a.chunk - 1) / a.chunk);
  a.ntiles = (ctx->ldc + kAllModeCols - 1) / kAllModeCols;
  int64_t off = 0;
  for (int m = 0; m + 1 < ctx->N; ++m) {
    a.part[m] = ctx->allmode_part + off;
    off += (int64_t)a.nchunks * ctx->dims[m] * ctx->ldc;
  }
  a.out_last = ctx->grad[ctx->N - 1];
  JKC_HIP(launch_allmode(a, ctx->stream));
  for (int m = 0; m + 1 < ctx->N; ++m)
    JKC_HIP(launch_reduce(a.part[m], a.nchunks, (int32_t)ctx->dims[m], ctx->ldc, ctx->ldc,
                          ctx->left_out(), 0, ctx->grad[m], ctx->ldc, ctx->stream, nullptr));
  return JKC_OK;
}

jkc_status enqueue_loss_grad(jkc_ctx* ctx, double* loss) {
  JKC_TRY(enqueue_fold_lambda(ctx));
  if (ctx->use_allmode) {
    ctx->tree_fresh = false;
    JKC_TRY(enqueue_allmode(ctx));
    return enqueue_grad_assemble(ctx, loss);
  }
  // all-mode MTTKRP with the factors fixed: for 3-way float64 problems one
  // shared contraction W = T x_2 U_2 serves modes 0 and 1 (the tensor is read
  // twice instead of three times, two thirds of the matrix-core flops)
  const bool tree = ctx->use_tree;
  if (tree) JKC_TRY(enqueue_tree_w(ctx));
  ctx->tree_fresh = false;
  // each mode's MTTKRP into its own gradient buffer, then one assembly launch.
  // A pass from W leaves the left-out rows of the sampled mode as computed:
  // the assembly writes 0 there and those factor rows are 0, so they add
  // nothing to the loss (as in the one-pass all-mode path).
  for (int n = 0; n < ctx->N; ++n) {
    double* Mn = ctx->grad[n];
    if (tree && n < 2)
      JKC_TRY(enqueue_tree_pass(ctx, n, Mn));
    else
      JKC_TRY(enqueue_mttkrp_reduced(ctx, n, Mn, ctx->ldc, ctx->ldc));
  }
  return enqueue_grad_assemble(ctx, loss);
}

// ---------------------------------------------------------------------------
// Fixed device scratch of jk_cals_mttkrp_static, for callers that cannot
// allocate.  In host code the array's name is only a host-side stand-in:
// its device address comes from hipGetSymbolAddress, taken once per device
// with that device current, and only that address is handed to kernels and
// copies.
// ---------------------------------------------------------------------------
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char g_static_scratch[JKC_STATIC_SCRATCH_BYTES];

namespace {

// Device address of the fixed scratch on the current device.
jkc_status static_scratch_address(void** out) {
  int dev = -1;
  JKC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(JKC_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    JKC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(g_static_scratch)));
    if (!p) return fail(JKC_EDEVICE, "hipGetSymbolAddress returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return JKC_OK;
}

jkc_status check_ctx(const jkc_ctx* ctx) {
  if (!ctx) return fail(JKC_EINVAL, "context is NULL");
  return JKC_OK;
}

jkc_status check_mode(const jkc_ctx* ctx, int mode) {
  if (mode < 0 || mode >= ctx->N) return fail(JKC_EINVAL, "mode out of range");
  return JKC_OK;
}

}  // namespace

// ===========================================================================
// Exported C ABI.
// ===========================================================================
extern "C" {

const char* jk_cals_last_error(void) { return g_last_error.c_str(); }

jkc_status jk_cals_workspace_size(const jkc_problem* prob, size_t* bytes) {
  if (!bytes) return fail(JKC_EINVAL, "bytes is NULL");
  Plan pl;
  JKC_TRY(make_plan(prob, &pl));
  *bytes = (size_t)pl.total;
  g_last_error.clear();
  return JKC_OK;
}

jkc_status jk_cals_init(const jkc_problem* prob, const void* tensor, const double* const* init,
                        void* workspace, size_t ws_bytes, jkc_ctx** out) {
  if (!out) return fail(JKC_EINVAL, "out is NULL");
  *out = nullptr;
  Plan pl;
  JKC_TRY(make_plan(prob, &pl));
  if (!tensor) return fail(JKC_EINVAL, "tensor is NULL");
  if (!init) return fail(JKC_EINVAL, "init is NULL");
  for (int n = 0; n < pl.N; ++n)
    if (!init[n]) return fail(JKC_EINVAL, "init[" + std::to_string(n) + "] is NULL");
  if (!workspace) return fail(JKC_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(JKC_EINVAL, "workspace must be 256-byte aligned");
  if ((int64_t)ws_bytes < pl.total)
    return fail(JKC_ENOMEM, "workspace too small: need " + std::to_string(pl.total) + " bytes");

  std::unique_ptr<jkc_ctx> ctx(new (std::nothrow) jkc_ctx());
  if (!ctx) return fail(JKC_ENOMEM, "host allocation failed");
  jkc_ctx& c = *ctx;
  c.N = pl.N;
  c.nhat = pl.nhat;
  c.K = pl.K;
  c.C = pl.C;
  c.ldc = pl.ldc;
  c.P = pl.P;
  for (int n = 0; n < kMaxOrder; ++n) {
    c.dims[n] = pl.dims[n];
    c.strides[n] = pl.strides[n];
  }
  c.tensor_f32 = pl.tensor_f32;
  c.precision = pl.precision;
  c.stream = static_cast<hipStream_t>(prob->stream);
  c.gsize = pl.gsize;
  c.partial_doubles = pl.partial_doubles;
  c.maxI = pl.maxI;
  c.rmax = 0;
  for (int k = 0; k < pl.K; ++k) c.rmax = std::max(c.rmax, prob->ranks[k]);
  c.h_rank.assign(prob->ranks, prob->ranks + pl.K);
  c.del_d = pl.del_d;
  c.h_left.resize(pl.K);
  c.h_lomask.assign(pl.dims[pl.nhat] * pl.K, 0);
  for (int k = 0; k < pl.K; ++k) {
    const int32_t* rows = prob->left_out + (int64_t)k * pl.del_d;
    c.h_left[k] = rows[0];
    for (int j = 0; j < pl.del_d; ++j)
      if (rows[j] >= 0) c.h_lomask[(int64_t)rows[j] * pl.K + k] = 1;
  }
  c.h_off.resize(pl.K);
  c.h_goff.resize(pl.K);
  c.h_colmodel.assign(pl.ldc, -1);
  int32_t off = 0;
  int64_t goff = 0;
  for (int k = 0; k < pl.K; ++k) {
    c.h_off[k] = off;
    c.h_goff[k] = goff;
    for (int r = 0; r < c.h_rank[k]; ++r) c.h_colmodel[off + r] = k;
    off += c.h_rank[k];
    goff += (int64_t)c.h_rank[k] * c.h_rank[k];
  }
  c.h_off_canon = c.h_off;
  c.uniform_rank = c.h_rank.empty() ? 0 : c.h_rank[0];
  for (int k = 1; k < pl.K; ++k)
    if (c.h_rank[k] != c.uniform_rank) c.uniform_rank = 0;
  c.C_act = pl.C;
  // most expensive models first (rank^2 work per row), stable by index
  c.h_order.resize(pl.K);
  std::iota(c.h_order.begin(), c.h_order.end(), 0);
  std::stable_sort(c.h_order.begin(), c.h_order.end(),
                   [&](int a, int b) { return c.h_rank[a] > c.h_rank[b]; });

  // carve the workspace
  char* base = static_cast<char*>(workspace);
  int64_t pos = 0;
  auto take = [&](size_t idx) -> void* {
    void* p = base + pos;
    pos += align_up(std::max<int64_t>(pl.items[idx].bytes, 1), kAlign);
    return p;
  };
  size_t it = 0;
  void* tbuf = take(it++);
  for (int n = 0; n < pl.N; ++n) c.U[n] = static_cast<double*>(take(it++));
  for (int n = 0; n < pl.N; ++n) c.G[n] = static_cast<double*>(take(it++));
  for (int n = 0; n < pl.N; ++n) c.grad[n] = static_cast<double*>(take(it++));
  c.Mbuf = static_cast<double*>(take(it++));
  c.partial = static_cast<double*>(take(it++));
  c.lambda = static_cast<double*>(take(it++));
  c.normT2 = static_cast<double*>(take(it++));
  c.err = static_cast<double*>(take(it++));
  c.fit = static_cast<double*>(take(it++));
  c.fit_prev = static_cast<double*>(take(it++));
  c.eta = static_cast<double*>(take(it++));
  c.status = static_cast<int32_t*>(take(it++));
  c.iters = static_cast<int32_t*>(take(it++));
  c.d_off = static_cast<int32_t*>(take(it++));
  c.d_rank = static_cast<int32_t*>(take(it++));
  c.d_lomask = static_cast<uint8_t*>(take(it++));
  c.d_order = static_cast<int32_t*>(take(it++));
  c.d_goff = static_cast<int64_t*>(take(it++));
  c.d_colmodel = static_cast<int32_t*>(take(it++));
  c.slice = static_cast<double*>(take(it++));
  c.slice_part = static_cast<double*>(take(it++));
  c.counter = static_cast<int32_t*>(take(it++));
  c.upart = static_cast<double*>(take(it++));
  c.Usplit = static_cast<uint16_t*>(take(it++));
  c.jk_perm = static_cast<int32_t*>(take(it++));
  c.jk_scale = static_cast<double*>(take(it++));
  c.d_colmap = static_cast<int32_t*>(take(it++));
  c.Wtree = static_cast<double*>(take(it++));
  c.tree_avail = pl.tree_rows > 0;
  c.use_tree = c.tree_avail;
  c.allmode_part = static_cast<double*>(take(it++));
  c.allmode_avail = pl.allmode_bk > 0;
  // default where no shared contraction is held (4-way problems, 3-way
  // problems whose W does not fit): measured faster than the per-mode fused
  // MTTKRPs there, slower than the shared contraction for 3-way tensors
  c.use_allmode = c.allmode_avail && !c.tree_avail;
  c.allmode_bk = pl.allmode_bk;
  c.allmode_nchunks = pl.allmode_nchunks;

  hipStream_t st = c.stream;
  // model tables (host vectors live in the context, so the copies are safe)
  JKC_HIP(hipMemcpyAsync(c.d_off, c.h_off.data(), pl.K * 4, hipMemcpyHostToDevice, st));
  JKC_HIP(hipMemcpyAsync(c.d_rank, c.h_rank.data(), pl.K * 4, hipMemcpyHostToDevice, st));
  JKC_HIP(hipMemcpyAsync(c.d_lomask, c.h_lomask.data(), c.h_lomask.size(), hipMemcpyHostToDevice, st));
  JKC_HIP(hipMemcpyAsync(c.d_order, c.h_order.data(), pl.K * 4, hipMemcpyHostToDevice, st));
  JKC_HIP(hipMemcpyAsync(c.d_goff, c.h_goff.data(), pl.K * 8, hipMemcpyHostToDevice, st));
  JKC_HIP(hipMemcpyAsync(c.d_colmodel, c.h_colmodel.data(), pl.ldc * 4, hipMemcpyHostToDevice, st));

  // tensor residency
  if (pl.precision != JKC_FP64) {
    c.nterm = pl.precision == JKC_SPLIT_BF16X6 ? 3 : 2;
    c.T_planes = static_cast<uint16_t*>(tbuf);
    int64_t off = 0;
    for (int n = 0; n < pl.N; ++n) {
      c.tp_off[n] = off;
      c.tp_ld[n] = pl.split_ld(n);
      c.tp_low[n] = pl.split_low(n);
      c.tp_ilp[n] = (int32_t)pl.split_ilp(n);
      JKC_HIP(launch_split_unfold(tensor, pl.tensor_f32, pl.N, pl.dims, n, c.tp_low[n], c.tp_ilp[n],
                                  c.nterm, c.T_planes + off, st));
      off += (int64_t)c.nterm * pl.dims[n] * c.tp_ld[n];
    }
  } else if (pl.copy_tensor) {
    JKC_HIP(launch_copy_tensor(tensor, pl.tensor_f32, tbuf, pl.P, st));
    c.T = tbuf;
  } else {
    c.T = tensor;
  }
  // slice norms of the sampled mode, from the caller's tensor (exact values)
  {
    const int64_t I = pl.dims[pl.nhat];
    const int64_t inner = pl.strides[pl.nhat];
    const int64_t outer = pl.P / (inner * I);
    const int chunks = (int)std::min<int64_t>(kSliceChunks, outer);
    JKC_HIP(launch_slice_norms(tensor, pl.tensor_f32, inner, (int32_t)I, outer, c.slice_part,
                               chunks, c.slice, st));
    JKC_HIP(launch_model_norms(c.slice, (int32_t)I, c.d_lomask, pl.K, c.normT2, st));
  }
  // multi-factors with the inserted zero rows, then Grams
  for (int n = 0; n < pl.N; ++n) {
    JKC_HIP(launch_pack_factor(init[n], pl.C, (int32_t)pl.dims[n], pl.C, pl.ldc, c.left_out(),
                               n == pl.nhat ? 1 : 0, c.U[n], st));
  }
  JKC_TRY(enqueue_grams(&c, 0, pl.N));
  JKC_HIP(launch_fill(c.lambda, pl.ldc, 1.0, st));
  JKC_HIP(launch_fill(c.err, pl.K, 0.0, st));
  JKC_HIP(launch_fill(c.fit, pl.K, 0.0, st));
  JKC_HIP(launch_fill(c.fit_prev, pl.K, 0.0, st));
  JKC_HIP(launch_fill_i32(c.status, pl.K, 0, st));
  JKC_HIP(launch_fill_i32(c.iters, pl.K, 0, st));
  c.lambda_is_one = true;

  // tilings
  const auto& vars = variants_for(&c);
  if (vars.empty()) return fail(JKC_EUNSUPPORTED, "no MTTKRP kernels for this precision");
  for (int n = 0; n < pl.N; ++n) {
    c.split_max[n] = pl.split_max[n];
    const ModeShape shape = mode_shape(&c, n, pl.split_max[n]);
    if (!tune_lookup(&c, n, vars, shape, &c.tiling[n])) c.tiling[n] = choose_tiling(vars, shape);
    c.describe[n] = describe_tiling(c.tiling[n], c.precision);
  }
  if (c.tree_avail) {
    const ModeShape shape = tree_shape(&c);
    if (!tune_lookup(&c, kTreeSlot, vars, shape, &c.tree_tiling)) {
      // untuned: the 16x16x4 tiling of 112 x 128 with four wavefronts, the
      // tuner's choice on 300x250x200 at C = 82,500 (on 100x200x200 at
      // C = 500 the tuner prefers 80 x 128 by about 3 %), else the cost model
      c.tree_tiling = choose_tiling(vars, shape);
      for (int v = 0; v < (int)vars.size(); ++v) {
        const auto& x = vars[v];
        if (x.wm == 1 && x.wn == 4 && x.tm == 7 && x.tn == 2 && x.bk == 16 && x.instr == 24 &&
            usable(x, shape)) {
          c.tree_tiling = make_tiling(vars, v, shape, 1);
          break;
        }
      }
    }
  }
  *out = ctx.release();
  g_last_error.clear();
  return JKC_OK;
}

void jk_cals_destroy(jkc_ctx* ctx) { delete ctx; }

jkc_status jk_cals_mttkrp(jkc_ctx* ctx, int32_t mode, double* out) {
  JKC_TRY(check_ctx(ctx));
  JKC_TRY(check_mode(ctx, mode));
  if (!out) return fail(JKC_EINVAL, "out is NULL");
  JKC_TRY(enqueue_mttkrp_reduced(ctx, mode, out, ctx->C, ctx->C));
  g_last_error.clear();
  return JKC_OK;
}

jkc_status jk_cals_mttkrp_static(const jkc_problem* prob, const void* tensor,
                                 const double* const* factors, int32_t mode, double* out) {
  Plan pl;
  JKC_TRY(make_plan(prob, &pl));
  if (pl.precision != JKC_FP64)
    return fail(JKC_EUNSUPPORTED, "jk_cals_mttkrp_static computes in float64 only (precision 0)");
  if (!tensor) return fail(JKC_EINVAL, "tensor is NULL");
  if (!factors) return fail(JKC_EINVAL, "factors is NULL");
  if (mode < 0 || mode >= pl.N) return fail(JKC_EINVAL, "mode out of range");
  for (int m = 0; m < pl.N; ++m)
    if (m != mode && !factors[m])
      return fail(JKC_EINVAL, "factors[" + std::to_string(m) + "] is NULL");
  if (!out) return fail(JKC_EINVAL, "out is NULL");

  // Scratch layout: column -> model map, left-out row mask, the other
  // modes' factors padded to ldc columns (left-out rows zeroed), then the
  // split-K partials (at least one plane: the unsplit product).
  const int64_t Ih = pl.dims[pl.nhat];
  int64_t pos = 0;
  const int64_t off_colmodel = pos;
  pos += align_up((int64_t)pl.ldc * 4, kAlign);
  const int64_t off_lomask = pos;
  pos += align_up(Ih * pl.K, kAlign);
  int64_t off_u[kMaxOrder] = {0, 0, 0, 0};
  for (int m = 0; m < pl.N; ++m) {
    if (m == mode) continue;
    off_u[m] = pos;
    pos += align_up(pl.dims[m] * pl.ldc * 8, kAlign);
  }
  const int64_t plane = pl.dims[mode] * pl.ldc * 8;
  const int64_t off_part = pos;
  if (pos + plane > (int64_t)JKC_STATIC_SCRATCH_BYTES)
    return fail(JKC_EINVAL, "problem needs " + std::to_string(pos + plane) +
                                " bytes of scratch; the fixed scratch holds " +
                                std::to_string((int64_t)JKC_STATIC_SCRATCH_BYTES));
  const int split_room = (int)std::min<int64_t>(((int64_t)JKC_STATIC_SCRATCH_BYTES - pos) / plane,
                                                1 << 20);

  // A host-side context over the scratch: the launch path of jk_cals_mttkrp.
  jkc_ctx c;
  c.N = pl.N;
  c.nhat = pl.nhat;
  c.K = pl.K;
  c.C = pl.C;
  c.C_act = pl.C;
  c.ldc = pl.ldc;
  c.P = pl.P;
  for (int n = 0; n < kMaxOrder; ++n) {
    c.dims[n] = pl.dims[n];
    c.strides[n] = pl.strides[n];
  }
  c.tensor_f32 = pl.tensor_f32;
  c.precision = pl.precision;
  c.stream = static_cast<hipStream_t>(prob->stream);
  c.T = tensor;
  c.split_max[mode] = std::max(1, std::min(pl.split_max[mode], split_room));
  const auto& vars = variants_for(&c);
  const ModeShape shape = mode_shape(&c, mode, c.split_max[mode]);
  Tiling t;
  if (!tune_lookup(&c, mode, vars, shape, &t)) t = choose_tiling(vars, shape);
  if (t.variant < 0) return fail(JKC_EUNSUPPORTED, "no MTTKRP tiling for this shape");
  const int splits = effective_splits(&c, mode, t);
  c.partial_doubles = (int64_t)split_room * pl.dims[mode] * pl.ldc;
  if (splits > split_room) return fail(JKC_ESTATE, "split-K partials exceed the fixed scratch");

  std::vector<int32_t> colmodel(pl.ldc, -1);
  std::vector<uint8_t> lomask(Ih * pl.K, 0);
  for (int k = 0, off = 0; k < pl.K; ++k) {
    for (int r = 0; r < prob->ranks[k]; ++r) colmodel[off + r] = k;
    off += prob->ranks[k];
    const int32_t* rows = prob->left_out + (int64_t)k * pl.del_d;
    for (int j = 0; j < pl.del_d; ++j)
      if (rows[j] >= 0) lomask[(int64_t)rows[j] * pl.K + k] = 1;
  }

  // every check done: device work from here on
  void* sp = nullptr;
  JKC_TRY(static_scratch_address(&sp));
  char* base = static_cast<char*>(sp);
  c.d_colmodel = reinterpret_cast<int32_t*>(base + off_colmodel);
  c.d_lomask = reinterpret_cast<uint8_t*>(base + off_lomask);
  for (int m = 0; m < pl.N; ++m)
    if (m != mode) c.U[m] = reinterpret_cast<double*>(base + off_u[m]);
  c.partial = reinterpret_cast<double*>(base + off_part);
  c.Mbuf = c.partial;
  hipStream_t st = c.stream;
  // pageable host sources: these copies complete before the calls return
  JKC_HIP(hipMemcpyAsync(c.d_colmodel, colmodel.data(), colmodel.size() * 4,
                         hipMemcpyHostToDevice, st));
  JKC_HIP(hipMemcpyAsync(c.d_lomask, lomask.data(), lomask.size(), hipMemcpyHostToDevice, st));
  for (int m = 0; m < pl.N; ++m)
    if (m != mode)
      JKC_HIP(launch_pack_factor(factors[m], pl.C, (int32_t)pl.dims[m], pl.C, pl.ldc, c.left_out(),
                                 m == pl.nhat ? 1 : 0, c.U[m], st));
  JKC_TRY(enqueue_mttkrp(&c, mode, t, true));
  JKC_TRY(launch_reduce_timed(&c, c.partial, splits, (int32_t)pl.dims[mode], pl.C,
                              mode == pl.nhat ? 1 : 0, out, pl.C));
  g_last_error.clear();
  return JKC_OK;
}

jkc_status jk_cals_sweep(jkc_ctx* ctx, int32_t nsweeps, double* fit) {
  JKC_TRY(check_ctx(ctx));
  if (nsweeps < 0) return fail(JKC_EINVAL, "nsweeps must be >= 0");
  JKC_TRY(enqueue_sweeps(ctx, nsweeps, 0.0, 0));
  if (fit)
    JKC_HIP(hipMemcpyAsync(fit, ctx->fit, ctx->K * 8, hipMemcpyDeviceToDevice, ctx->stream));
  g_last_error.clear();
  return JKC_OK;
}

// Move every model's columns to the offsets new_off (a permutation of whole
// column blocks; Gram blocks, flags and masks are indexed by model and do
// not move): factors and lambda are gathered through a column map, the model
// table is updated, and the MTTKRP then covers the first c_act columns.
// Synchronises the stream (the host tables are rewritten).
static jkc_status relayout(jkc_ctx* ctx, const std::vector<int32_t>& new_off, int32_t c_act) {
  ctx->tree_fresh = false;
  ctx->h_colmap.assign(ctx->C, 0);
  for (int k = 0; k < ctx->K; ++k)
    for (int r = 0; r < ctx->h_rank[k]; ++r) ctx->h_colmap[new_off[k] + r] = ctx->h_off[k] + r;
  hipStream_t st = ctx->stream;
  JKC_HIP(hipMemcpyAsync(ctx->d_colmap, ctx->h_colmap.data(), (size_t)ctx->C * 4,
                         hipMemcpyHostToDevice, st));
  for (int n = 0; n < ctx->N; ++n) {
    const int32_t rows = (int32_t)ctx->dims[n];
    JKC_HIP(launch_gather_cols(ctx->U[n], rows, ctx->ldc, ctx->C, ctx->d_colmap, ctx->Mbuf, st));
    JKC_HIP(hipMemcpyAsync(ctx->U[n], ctx->Mbuf, (size_t)rows * ctx->ldc * 8,
                           hipMemcpyDeviceToDevice, st));
  }
  JKC_HIP(launch_gather_cols(ctx->lambda, 1, ctx->ldc, ctx->C, ctx->d_colmap, ctx->Mbuf, st));
  JKC_HIP(hipMemcpyAsync(ctx->lambda, ctx->Mbuf, (size_t)ctx->ldc * 8, hipMemcpyDeviceToDevice, st));
  ctx->h_off = new_off;
  ctx->h_colmodel.assign(ctx->ldc, -1);
  for (int k = 0; k < ctx->K; ++k)
    for (int r = 0; r < ctx->h_rank[k]; ++r) ctx->h_colmodel[ctx->h_off[k] + r] = k;
  JKC_HIP(hipMemcpyAsync(ctx->d_off, ctx->h_off.data(), (size_t)ctx->K * 4, hipMemcpyHostToDevice, st));
  JKC_HIP(hipMemcpyAsync(ctx->d_colmodel, ctx->h_colmodel.data(), (size_t)ctx->ldc * 4,
                         hipMemcpyHostToDevice, st));
  JKC_HIP(hipStreamSynchronize(st));
  ctx->C_act = c_act;
  drop_graph(ctx);
  return JKC_OK;
}

jkc_status jk_cals_fit(jkc_ctx* ctx, int32_t max_iters, double tol, int32_t* iters, double* fit,
                       int32_t* status) {
  JKC_TRY(check_ctx(ctx));
  if (max_iters < 0) return fail(JKC_EINVAL, "max_iters must be >= 0");
  const int check_every = 5;
  const int conv = tol > 0.0 ? 1 : 0;
  std::vector<int32_t> st_host;
  jkc_status result = JKC_OK;
  for (int t = 0; t < max_iters && result == JKC_OK; ++t) {
    for (int n = 0; n < ctx->N && result == JKC_OK; ++n) result = enqueue_update(ctx, n, tol, conv);
    if (result != JKC_OK) break;
    ctx->lambda_is_one = false;
    if (conv && ((t + 1) % check_every == 0 || t + 1 == max_iters)) {
      int32_t active = 0;
      if (launch_count_active(ctx->status, ctx->K, ctx->counter, ctx->stream) != hipSuccess ||
          hipMemcpyAsync(&active, ctx->counter, 4, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
          hipStreamSynchronize(ctx->stream) != hipSuccess) {
        result = fail(JKC_EDEVICE, "convergence check failed");
        break;
      }
      if (active == 0) break;
      // no copy of the status words while the active models alone could
      // still fill more than four fifths of the computed columns
      if (!ctx->compaction || (int64_t)active * ctx->rmax * 5 > (int64_t)ctx->C_act * 4) continue;
      // compaction: once a fifth of the computed columns belong to frozen
      // models, move the models still being fitted to the front (in model
      // order) so that the fused MTTKRP covers only their columns
      st_host.resize(ctx->K);
      if (hipMemcpy(st_host.data(), ctx->status, (size_t)ctx->K * 4, hipMemcpyDeviceToHost) != hipSuccess) {
        result = fail(JKC_EDEVICE, "hipMemcpy of the status words failed");
        break;
      }
      int32_t act_cols = 0;
      for (int k = 0; k < ctx->K; ++k)
        if (!(st_host[k] & (JKC_ST_CONVERGED | JKC_ST_NONFINITE))) act_cols += ctx->h_rank[k];
      if (act_cols * 5 <= ctx->C_act * 4) {
        std::vector<int32_t> new_off(ctx->K);
        int32_t pos = 0;
        for (int pass = 0; pass < 2; ++pass)
          for (int k = 0; k < ctx->K; ++k) {
            const bool frozen = st_host[k] & (JKC_ST_CONVERGED | JKC_ST_NONFINITE);
            if (frozen == (pass == 1)) {
              new_off[k] = pos;
              pos += ctx->h_rank[k];
            }
          }
        result = relayout(ctx, new_off, act_cols);
      }
    }
  }
  // back to the canonical layout, whatever happened above
  if (ctx->h_off != ctx->h_off_canon) {
    const jkc_status r2 = relayout(ctx, ctx->h_off_canon, ctx->C);
    if (result == JKC_OK) result = r2;
  }
  if (result != JKC_OK) return result;
  if (iters) JKC_HIP(hipMemcpyAsync(iters, ctx->iters, ctx->K * 4, hipMemcpyDeviceToHost, ctx->stream));
  if (fit) JKC_HIP(hipMemcpyAsync(fit, ctx->fit, ctx->K * 8, hipMemcpyDeviceToHost, ctx->stream));
  if (status)
    JKC_HIP(hipMemcpyAsync(status, ctx->status, ctx->K * 4, hipMemcpyDeviceToHost, ctx->stream));
  JKC_HIP(hipStreamSynchronize(ctx->stream));
  g_last_error.clear();
  return JKC_OK;
}

jkc_status jk_cals_get_factors(jkc_ctx* ctx, int32_t mode, double* out, double* lambda) {
  JKC_TRY(check_ctx(ctx));
  JKC_TRY(check_mode(ctx, mode));
  if (!out) return fail(JKC_EINVAL, "out is NULL");
  JKC_HIP(launch_unpack(ctx->U[mode], ctx->ldc, (int32_t)ctx->dims[mode], ctx->C, out, ctx->stream));
  if (lambda)
    JKC_HIP(hipMemcpyAsync(lambda, ctx->lambda, ctx->C * 8, hipMemcpyDeviceToDevice, ctx->stream));
  g_last_error.clear();
  return JKC_OK;
}

jkc_status jk_cals_set_factors(jkc_ctx* ctx, int32_t mode, const double* in, const double* lambda) {
  JKC_TRY(check_ctx(ctx));
  JKC_TRY(check_mode(ctx, mode));
  if (!in) return fail(JKC_EINVAL, "in is NULL");
  JKC_HIP(launch_pack_factor(in, ctx->C, (int32_t)ctx->dims[mode], ctx->C, ctx->ldc, ctx->left_out(),
                             mode == ctx->nhat ? 1 : 0, ctx->U[mode], ctx->stream));
  JKC_TRY(enqueue_gram(ctx, mode));
  ctx->tree_fresh = false;
  if (lambda) {
    JKC_HIP(hipMemcpyAsync(ctx->lambda, lambda, ctx->C * 8, hipMemcpyDeviceToDevice, ctx->stream));
    ctx->lambda_is_one = false;
  }
  g_last_error.clear();
  return JKC_OK;
}

jkc_status jk_cals_get_status(jkc_ctx* ctx, double* err, double* fit, int32_t* status,
                              int32_t* iters) {
  JKC_TRY(check_ctx(ctx));
  hipStream_t s = ctx->stream;
  if (err) JKC_HIP(hipMemcpyAsync(err, ctx->err, ctx->K * 8, hipMemcpyDeviceToDevice, s));
  if (fit) JKC_HIP(hipMemcpyAsync(fit, ctx->fit, ctx->K * 8, hipMemcpyDeviceToDevice, s));
  if (status) JKC_HIP(hipMemcpyAsync(status, ctx->status, ctx->K * 4, hipMemcpyDeviceToDevice, s));
  if (iters) JKC_HIP(hipMemcpyAsync(iters, ctx->iters, ctx->K * 4, hipMemcpyDeviceToDevice, s));
  g_last_error.clear();
  return JKC_OK;
}

jkc_status jk_cals_loss_grad(jkc_ctx* ctx, double* loss) {
  JKC_TRY(check_ctx(ctx));
  JKC_TRY(enqueue_loss_grad(ctx, loss));
  g_last_error.clear();
  return JKC_OK;
}

jkc_status jk_cals_get_grad(jkc_ctx* ctx, int32_t mode, const double* weights, double* out) {
  JKC_TRY(check_ctx(ctx));
  JKC_TRY(check_mode(ctx, mode));
  if (!out) return fail(JKC_EINVAL, "out is NULL");
  JKC_HIP(launch_scale_cols_by_model(ctx->table(), weights, ctx->grad[mode],
                                     (int32_t)ctx->dims[mode], ctx->ldc, out, ctx->C,
                                     ctx->stream));
  g_last_error.clear();
  return JKC_OK;
}

jkc_status jk_cals_scale_columns(jkc_ctx* ctx, int32_t rows, const double* src,
                                 const double* weights, double* out) {
  JKC_TRY(check_ctx(ctx));
  if (rows < 0) return fail(JKC_EINVAL, "rows must be >= 0");
  if (rows > 0 && (!src || !out)) return fail(JKC_EINVAL, "src/out is NULL");
  if (rows == 0) {
    g_last_error.clear();
    return JKC_OK;
  }
  JKC_HIP(launch_scale_cols_by_model(ctx->table(), weights, src, rows, ctx->C, out, ctx->C,
                                     ctx->stream));
  g_last_error.clear();
  return JKC_OK;
}

jkc_status jk_cals_refine(jkc_ctx* ctx, int32_t steps, double* loss) {
  JKC_TRY(check_ctx(ctx));
  if (steps < 0) return fail(JKC_EINVAL, "steps must be >= 0");
  JKC_TRY(enqueue_fold_lambda(ctx));
  const double* G[kMaxOrder] = {ctx->G[0], ctx->G[1], ctx->G[2], ctx->G[3]};
  JKC_HIP(launch_gd_eta(ctx->table(), ctx->N, G, ctx->eta, ctx->stream));
  // every mode's step and Gram blocks in one launch (the gradients are all
  // taken at the same point)
  for (int s = 0; s < steps; ++s) {
    JKC_TRY(enqueue_loss_grad(ctx, nullptr));
    JKC_TRY(enqueue_grams(ctx, 0, ctx->N, ctx->eta));
  }
  if (loss) JKC_TRY(enqueue_loss_grad(ctx, loss));
  g_last_error.clear();
  return JKC_OK;
}

jkc_status jk_cals_jackknife_std(jkc_ctx* ctx, int32_t ref, int32_t first, int32_t count,
                                 double* const* std_out, int32_t* perm, double* sign) {
  JKC_TRY(check_ctx(ctx));
  if (ref < 0 || ref >= ctx->K) return fail(JKC_EINVAL, "ref out of range");
  if (count < 1 || first < 0 || first > ctx->K - count)
    return fail(JKC_EINVAL, "models first .. first+count-1 out of range");
  if (!std_out) return fail(JKC_EINVAL, "std is NULL");
  const int R = ctx->h_rank[ref];
  for (int k = first; k < first + count; ++k)
    if (ctx->h_rank[k] != R)
      return fail(JKC_EINVAL, "model " + std::to_string(k) + " has another rank than the reference");
  for (int n = 0; n < ctx->N; ++n)
    if (n != ctx->nhat && !std_out[n]) return fail(JKC_EINVAL, "std[n] is NULL for a non-sampled mode");
  JkArgs a{};
  a.N = ctx->N;
  a.nhat = ctx->nhat;
  a.R = R;
  a.ref_off = ctx->h_off[ref];
  a.first_off = ctx->h_off[first];
  a.count = count;
  a.ldc = ctx->ldc;
  for (int n = 0; n < kMaxOrder; ++n) {
    a.dims[n] = n < ctx->N ? (int32_t)ctx->dims[n] : 0;
    a.U[n] = n < ctx->N ? ctx->U[n] : nullptr;
    a.std_out[n] = n < ctx->N && n != ctx->nhat ? std_out[n] : nullptr;
  }
  a.perm = ctx->jk_perm;
  a.scale = ctx->jk_scale;
  JKC_HIP(launch_jk(a, ctx->stream));
  if (perm)
    JKC_HIP(hipMemcpyAsync(perm, ctx->jk_perm + a.first_off, (size_t)count * R * 4,
                           hipMemcpyDeviceToDevice, ctx->stream));
  if (sign)
    JKC_HIP(launch_jk_signs(ctx->jk_scale, ctx->ldc, ctx->N, a.first_off, count * R, sign,
                            ctx->stream));
  g_last_error.clear();
  return JKC_OK;
}

jkc_status jk_cals_set_compaction(jkc_ctx* ctx, int32_t enable) {
  JKC_TRY(check_ctx(ctx));
  if (enable != 0 && enable != 1) return fail(JKC_EINVAL, "enable must be 0 or 1");
  ctx->compaction = enable != 0;
  g_last_error.clear();
  return JKC_OK;
}

jkc_status jk_cals_tune(jkc_ctx* ctx, int32_t reps) {
  JKC_TRY(check_ctx(ctx));
  if (reps < 1) return fail(JKC_EINVAL, "reps must be >= 1");
  const auto& vars = variants_for(ctx);
  hipEvent_t e0, e1;
  JKC_HIP(hipEventCreate(&e0));
  JKC_HIP(hipEventCreate(&e1));
  jkc_status result = JKC_OK;
  // bring the clocks up before the first timing: the current tiling of mode
  // 0, repeated for about 20 ms
  {
    const auto t0 = std::chrono::steady_clock::now();
    for (int r = 0; r < 1000 && result == JKC_OK; ++r) {
      result = enqueue_mttkrp(ctx, 0, ctx->tiling[0]);
      if (result == JKC_OK && hipStreamSynchronize(ctx->stream) != hipSuccess)
        result = fail(JKC_EDEVICE, "hipStreamSynchronize failed");
      if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(20)) break;
    }
  }
  // modes 0..N-1, then (slot N) the shared partial contraction if held
  for (int n = 0; n <= ctx->N && result == JKC_OK; ++n) {
    const bool is_tree = n == ctx->N;
    if (is_tree && !ctx->tree_avail) break;
    const ModeShape shape = is_tree ? tree_shape(ctx) : mode_shape(ctx, n, ctx->split_max[n]);
    Tiling best = is_tree ? ctx->tree_tiling : ctx->tiling[n];
    float best_ms = std::numeric_limits<float>::infinity();
    for (int v = 0; v < (int)vars.size() && result == JKC_OK; ++v) {
      if (!usable(vars[v], shape)) continue;
      Tiling base = make_tiling(vars, v, shape, 1);
      const int s0 = default_splits(base, shape);
      const int cands[3] = {s0, std::max(1, s0 / 2), std::min(shape.split_max, s0 * 2)};
      for (int ci = 0; ci < 3; ++ci) {
        if (ci > 0 && cands[ci] == cands[0]) continue;
        if (ci == 2 && cands[2] == cands[1]) continue;
        Tiling t = base;
        t.splits = cands[ci];
        // warm-up, then timed repetitions of MTTKRP + reduction
        auto run = [&]() -> jkc_status {
          if (is_tree) {
            const Tiling keep = ctx->tree_tiling;
            ctx->tree_tiling = t;
            const jkc_status r = enqueue_tree_w(ctx);
            ctx->tree_tiling = keep;
            return r;
          }
          return enqueue_mttkrp_reduced(ctx, n, t, ctx->Mbuf, ctx->ldc, ctx->ldc);
        };
        result = run();
        if (result != JKC_OK) break;
        // the faster of two timed windows (clock and cache noise)
        float ms = std::numeric_limits<float>::infinity();
        for (int w = 0; w < 2 && result == JKC_OK; ++w) {
          if (hipEventRecord(e0, ctx->stream) != hipSuccess) { result = fail(JKC_EDEVICE, "event"); break; }
          for (int r = 0; r < reps && result == JKC_OK; ++r) result = run();
          if (result != JKC_OK) break;
          if (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            result = fail(JKC_EDEVICE, "event sync");
            break;
          }
          float wms = 0.f;
          (void)hipEventElapsedTime(&wms, e0, e1);
          ms = std::min(ms, wms);
        }
        if (result != JKC_OK) break;
        if (ms < best_ms) {
          best_ms = ms;
          best = t;
        }
      }
    }
    if (is_tree) {
      ctx->tree_tiling = best;
      drop_graph(ctx);
      if (result == JKC_OK) tune_store(ctx, kTreeSlot, best);
      break;
    }
    ctx->tiling[n] = best;
    ctx->describe[n] = describe_tiling(best, ctx->precision);
    drop_graph(ctx);
    if (result == JKC_OK) tune_store(ctx, n, best);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (result == JKC_OK) g_last_error.clear();
  return result;
}

const char* jk_cals_describe(jkc_ctx* ctx, int32_t mode) {
  if (!ctx || mode < 0 || mode > ctx->N) return "";
  if (mode == ctx->N) {
    // the shared partial contraction, when sweeps use it
    if (!ctx->use_tree) return "";
    ctx->tree_describe = "tree " + describe_tiling(ctx->tree_tiling, ctx->precision);
    return ctx->tree_describe.c_str();
  }
  return ctx->describe[mode].c_str();
}

jkc_status jk_cals_set_update_kernel(jkc_ctx* ctx, int32_t which) {
  JKC_TRY(check_ctx(ctx));
  if (which < 0 || which > 2) return fail(JKC_EINVAL, "which must be 0, 1 or 2");
  ctx->update_kernel = which;
  drop_graph(ctx);
  g_last_error.clear();
  return JKC_OK;
}

jkc_status jk_cals_set_mttkrp_tree(jkc_ctx* ctx, int32_t enable) {
  JKC_TRY(check_ctx(ctx));
  if (enable != 0 && enable != 1) return fail(JKC_EINVAL, "enable must be 0 or 1");
  if (enable && !ctx->tree_avail)
    return fail(JKC_EUNSUPPORTED, "the shared contraction needs a 3-way float64 problem whose W fits");
  if (ctx->use_tree != (enable != 0)) drop_graph(ctx);
  ctx->use_tree = enable != 0;
  ctx->tree_fresh = false;
  g_last_error.clear();
  return JKC_OK;
}

jkc_status jk_cals_set_allmode(jkc_ctx* ctx, int32_t enable) {
  JKC_TRY(check_ctx(ctx));
  if (enable != 0 && enable != 1) return fail(JKC_EINVAL, "enable must be 0 or 1");
  if (enable && !ctx->allmode_avail)
    return fail(JKC_EUNSUPPORTED,
                "the one-pass all-mode MTTKRP needs a 3- or 4-way float64 problem with at most 256 "
                "rows in mode 0 whose block fits in LDS");
  ctx->use_allmode = enable != 0;
  g_last_error.clear();
  return JKC_OK;
}

jkc_status jk_cals_set_sweep_graph(jkc_ctx* ctx, int32_t enable) {
  JKC_TRY(check_ctx(ctx));
  ctx->use_graph = enable != 0;
  drop_graph(ctx);
  g_last_error.clear();
  return JKC_OK;
}

int32_t jk_cals_num_tilings(jkc_ctx* ctx) {
  if (!ctx) return 0;
  return (int32_t)variants_for(ctx).size();
}

jkc_status jk_cals_set_tiling(jkc_ctx* ctx, int32_t mode, int32_t variant, int32_t splits) {
  JKC_TRY(check_ctx(ctx));
  const bool is_tree = ctx && mode == ctx->N;
  if (!is_tree) JKC_TRY(check_mode(ctx, mode));
  if (is_tree && !ctx->tree_avail)
    return fail(JKC_EINVAL, "this context holds no shared partial contraction");
  const auto& vars = variants_for(ctx);
  if (variant < 0 || variant >= (int)vars.size()) return fail(JKC_EINVAL, "variant out of range");
  if (splits < 1) return fail(JKC_EINVAL, "splits must be >= 1");
  if (is_tree && splits != 1)
    return fail(JKC_EINVAL, "the shared partial contraction takes one K chunk (splits = 1)");
  const ModeShape shape = is_tree ? tree_shape(ctx) : mode_shape(ctx, mode, ctx->split_max[mode]);
  if (!usable(vars[variant], shape))
    return fail(JKC_EINVAL, (vars[variant].instr & kNarrowInstr)
                                ? "the narrow tiling needs at most 16 columns (ldc 16) and mode 0 of "
                                  "at most 256 rows (128 with more than 8 columns), float64 path"
                                : "this tiling needs the tensor and every factor below 2^31 bytes");
  if (is_tree) {
    ctx->tree_tiling = make_tiling(vars, variant, shape, 1);
  } else {
    ctx->tiling[mode] = make_tiling(vars, variant, shape, splits);
    ctx->describe[mode] = describe_tiling(ctx->tiling[mode], ctx->precision);
  }
  drop_graph(ctx);
  g_last_error.clear();
  return JKC_OK;
}

jkc_status jk_cals_profile(jkc_ctx* ctx, int32_t enable) {
  JKC_TRY(check_ctx(ctx));
  ctx->prof_on = enable != 0;
  g_last_error.clear();
  return JKC_OK;
}

jkc_status jk_cals_profile_read(jkc_ctx* ctx, int64_t* launches, double* ms) {
  JKC_TRY(check_ctx(ctx));
  JKC_HIP(hipStreamSynchronize(ctx->stream));
  std::vector<int64_t> cnt(ctx->N + 1, 0);
  std::vector<double> tot(ctx->N + 1, 0.0);
  for (size_t i = 0; i < ctx->prof_used; ++i) {
    float t = 0.f;
    JKC_HIP(hipEventElapsedTime(&t, ctx->prof_ev[2 * i], ctx->prof_ev[2 * i + 1]));
    cnt[ctx->prof_mode[i]] += 1;
    tot[ctx->prof_mode[i]] += t;
  }
  ctx->prof_used = 0;
  for (int n = 0; n <= ctx->N; ++n) {
    if (launches) launches[n] = cnt[n];
    if (ms) ms[n] = tot[n];
  }
  g_last_error.clear();
  return JKC_OK;
}

jkc_status jk_cals_remove_slice(const jkc_problem* prob, const void* tensor, int32_t p, void* out) {
  if (!prob) return fail(JKC_EINVAL, "problem is NULL");
  if (prob->order < 2 || prob->order > kMaxOrder || !prob->dims)
    return fail(JKC_EINVAL, "bad order/dims");
  if (prob->sampled_mode < 0 || prob->sampled_mode >= prob->order)
    return fail(JKC_EINVAL, "sampled_mode out of range");
  if (!tensor || !out) return fail(JKC_EINVAL, "tensor/out is NULL");
  if (prob->tensor_dtype != JKC_TENSOR_F64 && prob->tensor_dtype != JKC_TENSOR_F32)
    return fail(JKC_EINVAL, "bad tensor_dtype");
  int64_t inner = 1, outer = 1;
  for (int n = 0; n < prob->order; ++n) {
    if (prob->dims[n] < 1) return fail(JKC_EINVAL, "dims must be >= 1");
    if (n < prob->sampled_mode) inner *= prob->dims[n];
    if (n > prob->sampled_mode) outer *= prob->dims[n];
  }
  const int64_t I = prob->dims[prob->sampled_mode];
  if (I < 2) return fail(JKC_EINVAL, "cannot remove the only slice");
  if (p < 0 || p >= I) return fail(JKC_EINVAL, "p out of range");
  JKC_HIP(launch_remove_slice(tensor, prob->tensor_dtype == JKC_TENSOR_F32 ? 4 : 8, inner,
                              (int32_t)I, outer, p, out, static_cast<hipStream_t>(prob->stream)));
  g_last_error.clear();
  return JKC_OK;
}

}  // extern "C"
