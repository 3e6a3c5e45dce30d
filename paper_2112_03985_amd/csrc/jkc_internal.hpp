// Internal declarations of the JK-CALS library: the context, the launch
// parameter blocks of every kernel and the launchers.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/jk_cals.h"

namespace jkc {

constexpr int kMaxOrder = JKC_MAX_ORDER;
constexpr int kMaxRank = JKC_MAX_RANK;
constexpr int kColAlign = 16;          // MFMA tile width: factor ld is a multiple

// Relative pivot / eigenvalue cutoff of the normal-equation solve, times R:
// H counts as positive definite when every Cholesky pivot exceeds
// tau * max_j H_jj, tau = 64 * R * eps (the same reading on every path).
constexpr double kPivotTolPerRank = 64.0 * 2.220446049250313e-16;

// ---------------------------------------------------------------------------
// MTTKRP tiling.  A block has WM x WN wavefronts; each wavefront owns a
// (TM*16) x (TN*16) tile of the output made of 16x16 MFMA tiles ((TM*4) x
// (TN*16) of 4x16 strips for the row-strip float64 instruction); the block
// walks the K dimension (columns of the unfolding) in steps of BK.  The K
// range is cut into S contiguous chunks, one per grid row, whose partial
// products are summed afterwards in a fixed order.
// ---------------------------------------------------------------------------
struct Tiling {
  int variant = -1;   // index into the kernel table (precision specific)
  int wm = 0, wn = 0, tm = 0, tn = 0, bk = 0, instr = 0;
  int splits = 1;
  // rows per block (the narrow variant: one output row for modes other
  // than 0)
  int bm() const { return (instr & 32) ? 1 : wm * tm * ((instr & 7) == 2 ? 4 : 16); }
  int bn() const { return wn * tn * 16; }
};

// Left-out rows of the sampled mode: column c belongs to model colmodel[c]
// (-1: padding), and row i is left out of model k when lomask[i * K + k].
struct LeftOut {
  const int32_t* colmodel;
  const uint8_t* lomask;
  int32_t K;
};

struct MttkrpArgs {
  const void* T;            // tensor (f64/f32), or the first bf16 plane (split paths)
  int64_t plane;            // split paths: elements between bf16 planes
  int32_t t_is_f32;         // FP64 path: tensor stored as float32
  const double* oU[kMaxOrder - 1];   // factors of the other modes, ascending
  int32_t odim[kMaxOrder - 1];       // their sizes
  int64_t ostride[kMaxOrder - 1];    // their tensor strides (elements)
  int32_t nother;           // N - 1
  int64_t stride_n;         // tensor stride of the output mode
  int32_t M;                // I_n (output rows)
  int64_t J;                // columns of the unfolding
  int64_t kchunk;           // K elements per split (multiple of BK); split paths: wraps
  // Split paths.  The unfolding's columns are ordered (low, higher modes
  // ascending) with the low mode's index padded to ilp (a multiple of the
  // kernel's K step): column jl + ilp * w for wrap w of the higher modes.
  int64_t ldt;              // row pitch of the unfolded planes (ilp * wraps)
  const uint16_t* ut;       // low mode's factor in bfloat16 terms, [term][ilp/32][ldc][32]
  int64_t ut_plane;         // elements between the terms of ut
  int32_t il, ilp;          // low mode size and its padded size
  int32_t nh;               // number of higher modes (N - 2)
  const double* hU[kMaxOrder - 2];   // higher modes' float64 factors, ascending
  int32_t hdim[kMaxOrder - 2];       // their sizes
  int64_t wraps;            // product of the higher modes' sizes
  int32_t ldc;              // leading dimension of factors and partials
  int32_t ncols;            // columns to produce (<= ldc)
  int32_t mtiles, ntiles;
  int32_t splits;
  double* partial;          // [splits][M][ldc]
  // Reduced output (kernels that sum their own split-K partials; null: the
  // partials are left for a separate reduction): out[i * fin_ldo + c] for
  // c < fin_ncols (columns at or past ncols are 0), rows left out of column
  // c's model 0 when fin_zero.
  double* fin_out;
  int32_t fin_ldo, fin_ncols, fin_zero;
  LeftOut fin_lo;
  // Narrow variant (set by its launcher): fibers of an output row (all
  // fibers for mode 0) and per K chunk.
  int32_t nfib, kcf;
};

// Kernel table entries (defined in the .hip files).
struct MttkrpVariant {
  int wm, wn, tm, tn, bk;
  // start/stop events (may be null) are stamped by the dispatch itself
  hipError_t (*launch)(const MttkrpArgs&, hipStream_t, hipEvent_t, hipEvent_t);
  int instr;   // matrix instruction family (kernel specific, low 3 bits) |
               // 8 when the step uses the interleaved instruction schedule
};
const std::vector<MttkrpVariant>& mttkrp_f64_variants();
// The narrow vector-ALU variant (mttkrp_narrow.hip), listed after the
// matrix-core float64 variants: one 16-column tile (ldc == 16), mode 0 of at most 256
// rows (at most 128 with more than 8 columns), K chunks of whole mode-0
// fibers for the other modes.  With fin_out set it produces the reduced
// product itself.  A K chunk holds at most narrow_max_chunk_fibers fibers
// (all fibers for mode 0, those of one output row otherwise).
constexpr int kNarrowInstr = 32;
bool narrow_supports(int I0, int ncols);
int64_t narrow_max_chunk_fibers(int I0, int ncols, bool mode0, int order);
const MttkrpVariant& mttkrp_narrow_variant();
const std::vector<MttkrpVariant>& mttkrp_split_variants();    // two bf16 terms
const std::vector<MttkrpVariant>& mttkrp_split3_variants();   // three bf16 terms

// ---------------------------------------------------------------------------
// Per-model batched kernels.
// ---------------------------------------------------------------------------
struct ModelTable {
  const int32_t* off;     // [K] first column
  const int32_t* rank;    // [K]
  const uint8_t* lomask;  // [I_nhat][K]: 1 where row i of the sampled mode is left out of model k
  const int64_t* goff;    // [K] offset of the model's R x R blocks in a Gram plane
  const int32_t* order;   // [K] models sorted by decreasing cost
  int32_t K;
};

// Row i of the sampled mode is left out of model k.
__device__ inline bool left_out_row(const ModelTable& mt, int64_t i, int k) {
  return mt.lomask[i * mt.K + k] != 0;
}

struct UpdateArgs {
  ModelTable mt;
  int32_t N, n, nhat;
  int32_t In;                     // rows of the updated mode
  int32_t ldc;
  const double* partial;          // [splits][In][ldc] MTTKRP partials (LDS kernel)
  int32_t splits;
  double* Mout;                   // [In][ldc] reduced MTTKRP (global kernel)
  double* U;                      // [In][ldc] factor of mode n (output)
  double* G[kMaxOrder];           // Gram planes, one per mode
  double* lambda;                 // [ldc]
  const double* normT2;           // [K] ||T_{-p}||^2
  double* err;                    // [K]
  double* fit;                    // [K]
  double* fit_prev;               // [K]
  int32_t* status;                // [K]
  int32_t* iters;                 // [K]
  int32_t last_mode;              // 1 when n == N-1: evaluate the error
  double tol;                     // convergence tolerance (<= 0: off)
  int32_t check_conv;             // 1: update convergence flags
  int32_t rmax;                   // largest rank (LDS sizing)
  int32_t uniform_rank;           // > 0: every model has this rank, model k at column k*R and
                                  // Gram offset k*R*R (canonical layout; LDS-staged kernel)
  int64_t lds_doubles;            // > 0: LDS-staged kernel with this much dynamic LDS
  double* scratch;                // row-parallel update: per (model, chunk) sums
  double* Utmp;                   // row-parallel update: [In][ldc] unnormalised U
  int32_t nch;                    // row-parallel update: chunks per model
};

// Jackknife post-processing of a set of `count` models of rank R with
// contiguous columns (model j of the set at first_off + j * R).
struct JkArgs {
  int32_t N, nhat;
  int32_t R;
  int32_t ref_off;            // first column of the reference model
  int32_t first_off;          // first column of the set
  int32_t count;
  int32_t ldc;
  int32_t dims[kMaxOrder];
  const double* U[kMaxOrder];
  int32_t* perm;              // [ldc]: at column first_off + j*R + s, the component of model j matched to s
  double* scale;              // [N][ldc]: signed inverse norms of the matched columns (0 for the sampled mode)
  double* std_out[kMaxOrder]; // I_n x R row-major; unused for the sampled mode
};
hipError_t launch_jk(const JkArgs& a, hipStream_t s);
hipError_t launch_jk_signs(const double* scale, int32_t ldc, int32_t N, int32_t first_off,
                           int32_t cols, double* sign, hipStream_t s);

// Rows per block of the row-parallel update, and its scratch (doubles).
constexpr int kUpdRows = 64;
inline int64_t update_rows_scratch(int64_t maxI, int64_t gsize, int64_t K) {
  return ((maxI + kUpdRows - 1) / kUpdRows) * (gsize + 2 * K);
}
hipError_t launch_update_rows(const UpdateArgs& a, hipStream_t s);

// Dynamic LDS (doubles) of the LDS-staged update for a mode with `rows` rows.
int64_t update_lds_doubles(int rmax, int rows);
hipError_t launch_update(const UpdateArgs& a, hipStream_t s);

// Gram blocks of one or more modes in one launch (grid y: the modes).
struct GramArgs {
  ModelTable mt;
  int32_t ldc;
  int32_t nmodes;                    // modes in this launch (1..N)
  int32_t rows[kMaxOrder];           // per launched mode
  double* U[kMaxOrder];              // [rows][ldc] factor per launched mode
  double* G[kMaxOrder];              // its Gram plane
  int32_t uniform_rank;   // > 0: every model has this rank, canonical layout (see UpdateArgs)
  // gradient step before the Gram blocks when eta is not null:
  // U -= eta[k] * grad on model k's columns (grad [rows][ldc] per mode)
  const double* eta;                 // [K]
  const double* grad[kMaxOrder];
};
hipError_t launch_gram(const GramArgs& a, hipStream_t s);

// Left-out rows of the sampled mode, as the kernels that clear them see
// them: the owning model of every column ([ldc], -1 for padding) and the
// row mask of the model table.
hipError_t launch_tree_pass(const double* W, const double* F, int32_t S, int64_t ostep,
                            int64_t sstep, int32_t nout, int32_t ldc, int32_t ncols, double* out,
                            hipStream_t s);
// (stop: when not null, an event the dispatch stamps at its end)
hipError_t launch_reduce(const double* partial, int32_t splits, int32_t rows,
                         int32_t ldc, int32_t ncols, LeftOut lo,
                         int32_t zero_rows, double* out, int32_t ldo,
                         hipStream_t s, hipEvent_t stop);

// Preparation kernels.
hipError_t launch_copy_tensor(const void* src, int32_t src_f32, void* dst,
                              int64_t count, hipStream_t s);
// Split-precision tensor copy of one mode: the mode-n unfolding with its
// columns ordered low mode first (index padded to ilp with zeros), then the
// other modes ascending (lowest fastest), in K blocks of 32 (element (i, k)
// at ((k / 32) * I_n + i) * 32 + k % 32), as nterm bfloat16 planes of
// I_n * ilp * wraps elements.
hipError_t launch_split_unfold(const void* src, int32_t src_f32, int32_t N, const int64_t* dims,
                               int32_t n, int32_t low, int32_t ilp, int32_t nterm,
                               uint16_t* planes, hipStream_t s);
// The low mode's factor (rows x ldc float64) as nterm bfloat16 terms in K
// blocks of 32 rows: term t of U(j, c) at out + t * ldc * ilp +
// ((j / 32) * ldc + c) * 32 + j % 32 (0 for rows <= j < ilp).
hipError_t launch_split_factor_t(const double* U, int32_t rows, int32_t ldc, int32_t ilp,
                                 int32_t nterm, uint16_t* out, hipStream_t s);
hipError_t launch_slice_norms(const void* T, int32_t t_f32, int64_t inner,
                              int32_t I, int64_t outer, double* partial,
                              int32_t chunks, double* s_out, hipStream_t s);
hipError_t launch_model_norms(const double* s, int32_t I, const uint8_t* lomask,
                              int32_t K, double* normT2, hipStream_t st);
hipError_t launch_pack_factor(const double* src, int32_t lds, int32_t rows,
                              int32_t C, int32_t ldc, LeftOut lo,
                              int32_t zero_rows, double* dst, hipStream_t s);
hipError_t launch_gather_cols(const double* src, int32_t rows, int32_t ldc, int32_t C,
                              const int32_t* map, double* dst, hipStream_t s);
hipError_t launch_unpack(const double* src, int32_t ldc, int32_t rows,
                         int32_t C, double* dst, hipStream_t s);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_remove_slice(const void* src, int32_t elem_bytes,
                               int64_t inner, int32_t I, int64_t outer,
                               int32_t p, void* dst, hipStream_t s);
hipError_t launch_count_active(const int32_t* status, int32_t K, int32_t* out,
                               hipStream_t s);

// One-pass all-mode MTTKRP (allmode.hip): 3- and 4-way float64 problems
// whose mode 0 has at most 256 rows.  Block (column tile of 32, chunk of
// consecutive last-mode indices); modes 0 .. N-2 as split partials over the
// chunks, the last mode written directly.
struct AllModeArgs {
  const void* T;
  int64_t tbytes;           // bytes of T (below 2^31: 32-bit buffer offsets)
  int32_t t_is_f32;
  int32_t N;
  int32_t dims[kMaxOrder];
  const double* U[kMaxOrder];
  int32_t ldc;
  int32_t i0p;              // mode-0 rows padded to 16 * allmode_row_tiles(I0)
  int32_t bk;               // fibers per step: 8 or 16
  int32_t chunk;            // last-mode indices per chunk
  int32_t nchunks;
  int32_t ntiles;           // 32-column tiles
  double* part[kMaxOrder - 1];   // [nchunks][I_m][ldc] for m = 0 .. N-2
  double* out_last;         // [I_{N-1}][ldc]
};
constexpr int kAllModeCols = 32;
int64_t allmode_lds_bytes(int i0p, int bk, int I1, int I2, int N);
// Row tiles the compiled kernels offer for a mode-0 size I0 (0: none), and
// whether a (row tiles, fibers per step) pair is compiled.
int allmode_row_tiles(int I0);
bool allmode_has_kernel(int nt, int bk);
hipError_t launch_allmode(const AllModeArgs& a, hipStream_t s);

// Gradient assembly of modes n0 .. n0 + nmodes - 1 in one launch (grid y:
// the mode, n = n0 + blockIdx.y); entry q of the per-mode arrays belongs to
// mode n0 + q.  Mfull[q] may equal grad[q] (assembled in place).
struct GradArgs {
  ModelTable mt;
  int32_t N, nhat;
  int32_t n0, nmodes, ldc;
  int32_t In[kMaxOrder];
  const double* Mfull[kMaxOrder];  // [In][ldc] MTTKRP of the mode
  const double* U[kMaxOrder];      // [In][ldc] factor of the mode
  const double* Gp[kMaxOrder];     // Gram planes of every mode
  double* grad[kMaxOrder];         // [In][ldc] gradient of the mode (out)
  const double* normT2;    // [K]
  double* loss;            // [K]: written by the blocks of mode N - 1 when not null
  int32_t uniform_rank;    // > 0: every model has this rank, canonical layout (see UpdateArgs)
};
hipError_t launch_grad_assemble(const GradArgs& a, hipStream_t s);
hipError_t launch_scale_cols_by_model(const ModelTable& mt, const double* w,
                                      const double* src, int32_t rows,
                                      int32_t ldc, double* dst, int32_t ldd,
                                      hipStream_t s);
hipError_t launch_fold_lambda(double* U, int32_t rows, int32_t ldc, int32_t C,
                              double* lambda, hipStream_t s);
hipError_t launch_gd_eta(const ModelTable& mt, int32_t N, const double* const* G,
                         double* eta, hipStream_t s);

}  // namespace jkc

// The context (opaque to callers).
struct jkc_ctx {
  // problem
  int32_t N = 0, nhat = 0, K = 0, C = 0, ldc = 0;
  int64_t dims[jkc::kMaxOrder] = {0, 0, 0, 0};
  int64_t strides[jkc::kMaxOrder] = {0, 0, 0, 0};
  int64_t P = 0;
  int32_t tensor_f32 = 0, precision = 0;
  hipStream_t stream = nullptr;
  std::vector<int32_t> h_rank, h_left, h_off, h_order, h_colmodel;
  std::vector<uint8_t> h_lomask;  // [I_nhat][K]
  int32_t del_d = 1;              // rows left out per submodel
  std::vector<int64_t> h_goff;
  int64_t gsize = 0;  // doubles per Gram plane
  int32_t rmax = 0;   // largest model rank
  int64_t maxI = 0;   // largest mode size

  // device buffers (all inside the caller's workspace)
  const void* T = nullptr;       // FP64 path tensor (f64 or f32)
  uint16_t* T_planes = nullptr;  // split paths: per mode, nterm bf16 planes
  int32_t nterm = 0;
  int64_t tp_off[jkc::kMaxOrder] = {0, 0, 0, 0};   // element offset of mode n's planes
  int64_t tp_ld[jkc::kMaxOrder] = {0, 0, 0, 0};    // their row pitch
  double* U[jkc::kMaxOrder] = {nullptr, nullptr, nullptr, nullptr};
  uint16_t* Usplit = nullptr;    // split paths: the low mode's factor in bf16 terms
  int32_t tp_low[jkc::kMaxOrder] = {0, 0, 0, 0};   // split paths: low mode of each mode
  int32_t tp_ilp[jkc::kMaxOrder] = {0, 0, 0, 0};   // and its padded size
  double* G[jkc::kMaxOrder] = {nullptr, nullptr, nullptr, nullptr};
  double* Mbuf = nullptr;        // [max I_n][ldc]
  double* partial = nullptr;     // split-K partials
  int64_t partial_doubles = 0;
  double* lambda = nullptr;
  double* normT2 = nullptr;
  double* err = nullptr;
  double* fit = nullptr;
  double* fit_prev = nullptr;
  int32_t* status = nullptr;
  int32_t* iters = nullptr;
  int32_t* d_off = nullptr;
  int32_t* d_rank = nullptr;
  uint8_t* d_lomask = nullptr;
  int32_t* d_order = nullptr;
  int32_t* d_colmodel = nullptr;
  int64_t* d_goff = nullptr;
  double* slice = nullptr;       // [I_nhat] slice norms
  double* slice_part = nullptr;  // [chunks][I_nhat]
  int32_t* counter = nullptr;    // [1] active-model count
  double* grad[jkc::kMaxOrder] = {nullptr, nullptr, nullptr, nullptr};
  double* eta = nullptr;         // [K]

  jkc::Tiling tiling[jkc::kMaxOrder];
  int split_max[jkc::kMaxOrder] = {1, 1, 1, 1};
  std::string describe[jkc::kMaxOrder];
  bool lambda_is_one = true;     // lambda folded into the last factor
  // Convergence compaction (jk_cals_fit): the models still being fitted
  // occupy the first C_act columns; C_act == C in the canonical layout.
  int32_t C_act = 0;
  bool compaction = true;
  std::vector<int32_t> h_off_canon;   // offsets of the canonical layout
  int32_t uniform_rank = 0;           // the rank of every model when all are equal, else 0
  std::vector<int32_t> h_colmap;      // last relayout map, [C]
  int32_t* d_colmap = nullptr;        // [ldc]
  int update_kernel = 0;         // 0 LDS-staged, 1 global, 2 row-parallel
  double* upart = nullptr;       // row-parallel update scratch
  int32_t* jk_perm = nullptr;     // jackknife matching: [ldc]
  double* jk_scale = nullptr;     // jackknife matching: [N][ldc]
  bool use_graph = false;        // replay sweeps from a captured HIP graph
  // Shared partial contraction of a 3-way float64 sweep (tree.hip):
  // W = T x_2 U_2, [I_0 I_1][ldc], computed at mode 0 and used by modes 0, 1
  double* Wtree = nullptr;
  // One-pass all-mode MTTKRP of the loss gradient (allmode.hip)
  bool allmode_avail = false;
  bool use_allmode = false;
  int32_t allmode_bk = 16;
  int32_t allmode_nchunks = 1;
  double* allmode_part = nullptr;
  bool tree_avail = false;       // the workspace holds W
  bool use_tree = false;
  bool tree_fresh = false;       // W matches U_2 of this sweep (host-side order)
  jkc::Tiling tree_tiling;
  std::string tree_describe;
  hipGraphExec_t graph_exec = nullptr;

  // MTTKRP kernel timing (jk_cals_profile)
  bool prof_on = false;
  std::vector<hipEvent_t> prof_ev;     // pairs: [2i] start, [2i+1] stop
  std::vector<int> prof_mode;          // slot of each timed pair (mode, or N for W)
  size_t prof_used = 0;
  hipEvent_t prof_pending_stop = nullptr;   // stop event for the next reduction
  ~jkc_ctx() {
    for (hipEvent_t e : prof_ev) (void)hipEventDestroy(e);
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
  }

  jkc::ModelTable table() const {
    return jkc::ModelTable{d_off, d_rank, d_lomask, d_goff, d_order, K};
  }
  jkc::LeftOut left_out() const { return jkc::LeftOut{d_colmodel, d_lomask, K}; }
};
