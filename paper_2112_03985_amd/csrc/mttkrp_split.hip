// Split-precision fused MTTKRP: the same product as the float64 kernel
// (Alg. 3, MTTKRP step, over the full tensor, column-concatenated over all
// models; Eq. (1) per model), computed on the bfloat16 matrix cores.
//
// Factorisation of the Khatri-Rao product.  Pick one other mode L (the
// "low" mode) and write the remaining other modes' multi-index as a wrap w.
// Then
//   M_n(i, c) = sum_w s(w, c) * sum_jl T_(n)(i, jl, w) * U_L(jl, c),
//   s(w, c)   = prod_{m != n, L} U_m(w_m, c),
// so within one wrap the product is a plain GEMM of a tensor slab with U_L
// (the same B operand for every wrap), and the remaining Khatri-Rao factor
// is one float64 scale per (wrap, column), applied when the wrap's float32
// accumulators are added into the float64 ones.  Nothing is formed per
// Khatri-Rao entry in the inner loop: both operands are copied to LDS as
// loaded.  (The same multilinear identity as Eq. (1); only the evaluation
// order of the sums differs.)
//
// Operands as sums of NTERM bfloat16 terms, each the round-to-nearest-even
// of what the previous terms leave (x1 = bf16(x), x2 = bf16(x - x1), ...):
// the tensor once at init, U_L before each launch, both from float64.
// Products keep every term pair whose magnitude is at least 2^-8(NTERM-1)
// of the leading one:
//   NTERM = 2: a1 b1 + a1 b2 + a2 b1                       (3 MFMA products)
//   NTERM = 3: the above + a1 b3 + a2 b2 + a3 b1           (6 MFMA products)
// smallest terms first.  Products of bfloat16 are exact in float32; the
// float32 accumulators hold one wrap (at most 2048 K) before they are scaled
// and added into float64 ones; split-K partials are float64.
//
// Layout (written by the prep kernels).  For the split paths the tensor is
// held once per mode as that mode's unfolding with its columns ordered
// jl + ilp * w (jl padded with zeros to ilp, a multiple of the 32-K step),
// one plane per term, in K blocks of 32: the 32-K slice of all rows is one
// contiguous run, so a step's A operand (BM rows x 32 K) spans one or two
// pages whatever the tensor size (a row-major unfolding puts every row of
// the tile megabytes apart).  U_L is held the same way ([term][K block][c]
// [32], padded with zero rows).  Both operands arrive as aligned 16-byte
// runs of 8 consecutive K, the register layout of the
// v_mfma_f32_16x16x32_bf16 operands, and are copied to LDS unchanged.
//
// Tiles are BM x BN, BM = 16 WM TM; a block walks whole wraps of one K
// chunk; blocks are dealt to the XCDs in contiguous runs of column tiles
// (they share the tensor slab in L2).  Loads of a step are issued two steps
// before it is stored (two register stages); the store of step s+1 runs
// interleaved with the matrix instructions of step s (double-buffered LDS,
// one barrier per step).
#include <type_traits>

#include <hip/hip_ext.h>

#include "jkc_internal.hpp"

namespace jkc {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kBK = 32;           // one v_mfma_f32_16x16x32_bf16 deep
constexpr int kFlushSteps = 64;   // float32 accumulation span within a long wrap (2048 K)
constexpr int kXcds = 8;

// LDS rows of 32 bf16 (four 16-byte chunks) with the chunk index XOR-ed by
// g(row) = ((row >> 2) ^ (row >> 1)) mod 4: the fragment reads (lane l: row
// l mod 16 of a 16-row tile, chunk l / 16) and the staging writes (4
// consecutive lanes per row, all four chunks) then hit distinct banks for
// 16 and for 32 consecutive lanes (checked on the host), and the LDS
// bank-conflict counter reads zero for both on gfx950, where the earlier
// g(row) = ((row >> 1) mod 4) ^ ((row >> 3) mod 2), distinct only within
// groups of 16 lanes, measured two-way conflicts on the fragment reads.
// (g depends on row mod 16 only, so a fragment row's chunk follows from its lane.)
__device__ __forceinline__ int swz(int row) { return ((row >> 2) ^ (row >> 1)) & 3; }

// BRES: the block's B operand (its columns of U_L, all ilp rows) is loaded
// into dynamic LDS once and stays there (U_L is the same for every wrap), so
// a step streams only the tensor slab; otherwise B is staged per step like A.
template <int WM, int WN, int TM, int TN, int NTERM, int NH, bool BRES>
__global__ void __launch_bounds__(64 * WM * WN)
k_mttkrp_bf(const MttkrpArgs a) {
  constexpr int NT = 64 * WM * WN;
  constexpr int BM = WM * TM * 16;
  constexpr int BN = WN * TN * 16;
  constexpr int BK = kBK;
  constexpr int CH = BK / 8;                         // 8-K runs per row per step
  constexpr int AI = (BM * CH + NT - 1) / NT;        // A runs per thread
  constexpr int BI = (BN * CH + NT - 1) / NT;        // B runs per thread
  static_assert(NTERM == 2 || NTERM == 3, "terms");
  static_assert(NH >= 0 && NH <= kMaxOrder - 2, "higher modes");
  static_assert(NT >= BN, "one wrap scale per column and thread");

  __shared__ __attribute__((aligned(16))) uint16_t As[2][NTERM][BM][kBK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BRES ? 1 : 2][NTERM][BRES ? 1 : BN][kBK];
  __shared__ double Ss[2][BN];   // wrap scales s(w, c) of the step's columns
  // resident B: [term][K block of the wrap][column][32], swizzled chunks
  extern __shared__ __attribute__((aligned(16))) uint16_t Bres[];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM;
  const int wn = wave / WM;

  // Block -> (column tile, row tile, K chunk), XCD-aware as in the float64
  // kernel: each XCD receives a contiguous run of logical blocks, column
  // tile fastest, so the blocks sharing one tensor slab share an L2.
  const int total = gridDim.x;
  int logical = blockIdx.x;
  const int per_xcd = total / kXcds;
  if (logical < per_xcd * kXcds) logical = (logical % kXcds) * per_xcd + logical / kXcds;
  const int nt = logical % a.ntiles;
  const int mt = (logical / a.ntiles) % a.mtiles;
  const int split = logical / (a.ntiles * a.mtiles);
  const int i0 = mt * BM;
  const int c0 = nt * BN;
  // K chunk: whole wraps [wbeg, wend); steps of BK within each wrap
  const int64_t wbeg = (int64_t)split * a.kchunk;
  const int64_t wend = min(wbeg + a.kchunk, a.wraps);
  const int sw = a.ilp / BK;                                  // steps per wrap
  const int nsteps = wend > wbeg ? (int)((wend - wbeg) * sw) : 0;
  const uint32_t kbase = (uint32_t)(wbeg * a.ilp);            // first padded K of the chunk

  const uint16_t* __restrict__ Tp = static_cast<const uint16_t*>(a.T);
  const uint16_t* __restrict__ Up = a.ut;

  // A runs: item e = tid + NT*u -> row e / CH, run e % CH (CH threads cover
  // one row's 64 contiguous bytes per term).  B runs likewise: column e / CH,
  // run e % CH.  Items outside the tile, and steps past the chunk, read a
  // clamped address: rows past I_n and columns past ldc produce outputs that
  // are never stored, and steps past the chunk are never computed.  Element
  // offsets within a plane are below 2^31 (checked at init).

  u32x4 ra[2][AI][NTERM];
  u32x4 rb[2][BI][NTERM];
  double rs[2][NH > 0 ? NH : 1];   // higher modes' entries of the step's wrap, one column per thread
  using S0_t = std::integral_constant<int, 0>;
  using S1_t = std::integral_constant<int, 1>;

  // Wrap of the next step to load (loads run in step order): its index lw,
  // the step within it lin, and its multi-index over the higher modes
  // (lowest fastest), all uniform.
  int64_t lw = wbeg;
  int lin = 0;
  uint32_t hidx[NH > 0 ? NH : 1];
  {
    uint32_t rem = (uint32_t)min(wbeg, a.wraps);
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      hidx[h] = rem % (uint32_t)a.hdim[h];
      rem /= (uint32_t)a.hdim[h];
    }
  }
  // column whose wrap scale this thread fetches (every thread loads, so the
  // loads of a step are unconditional and their count is fixed)
  const int scl = tid % BN;
  const uint32_t scol = c0 + scl < a.ldc ? (uint32_t)(c0 + scl) : 0u;

  // Every load of a step is unconditional (no branch around a load), so the
  // wait before a step's store covers only that step's loads.
  auto load_step = [&](auto P, int s) __attribute__((always_inline)) {
    constexpr int p = decltype(P)::value;
    const bool sok = s < nsteps;
    // K blocks of 32: the step's slice of every row is contiguous
    const uint32_t kb = kbase / BK + (uint32_t)s;                    // K block of the step
    const uint32_t jb = (uint32_t)lin;                               // its low-mode block
#pragma unroll
    for (int u = 0; u < AI; ++u) {
      const int e = tid + NT * u;
      const int row = e / CH, run = e % CH;
      const bool ok = sok && e < BM * CH && i0 + row < a.M;
      const uint32_t at = ok ? (kb * (uint32_t)a.M + (uint32_t)(i0 + row)) * BK + 8u * run : 0u;
#pragma unroll
      for (int t = 0; t < NTERM; ++t)
        ra[p][u][t] = *reinterpret_cast<const u32x4*>(Tp + (int64_t)t * a.plane + at);
    }
    if constexpr (!BRES) {
#pragma unroll
      for (int u = 0; u < BI; ++u) {
        const int e = tid + NT * u;
        const int cl = e / CH, run = e % CH;
        const bool ok = sok && e < BN * CH && c0 + cl < a.ldc;
        const uint32_t at = ok ? (jb * (uint32_t)a.ldc + (uint32_t)(c0 + cl)) * BK + 8u * run : 0u;
#pragma unroll
        for (int t = 0; t < NTERM; ++t)
          rb[p][u][t] = *reinterpret_cast<const u32x4*>(Up + (int64_t)t * a.ut_plane + at);
      }
    }
    const bool wok = sok && lw < a.wraps;
#pragma unroll
    for (int h = 0; h < NH; ++h)
      rs[p][h] = a.hU[h][(wok ? hidx[h] : 0u) * (uint32_t)a.ldc + scol];
    if (++lin == sw) {
      lin = 0;
      ++lw;
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        if (++hidx[h] < (uint32_t)a.hdim[h]) break;
        hidx[h] = 0;
      }
    }
  };

  // The store of a step: both operands copied to LDS as loaded (swizzled
  // chunks), and the step's wrap scales s(w, c) = product of the higher
  // modes' entries, highest mode first (the order of Eq. (1)).
  auto store_step = [&](auto P, int buf) __attribute__((always_inline)) {
    constexpr int p = decltype(P)::value;
#pragma unroll
    for (int u = 0; u < AI; ++u) {
      const int e = tid + NT * u;
      if (AI * NT == BM * CH || e < BM * CH) {
        const int row = e / CH, run = e % CH;
#pragma unroll
        for (int t = 0; t < NTERM; ++t)
          *reinterpret_cast<u32x4*>(&As[buf][t][row][8 * (run ^ swz(row))]) = ra[p][u][t];
      }
    }
    if constexpr (!BRES) {
#pragma unroll
      for (int u = 0; u < BI; ++u) {
        const int e = tid + NT * u;
        if (BI * NT == BN * CH || e < BN * CH) {
          const int cl = e / CH, run = e % CH;
#pragma unroll
          for (int t = 0; t < NTERM; ++t)
            *reinterpret_cast<u32x4*>(&Bs[buf][t][cl][8 * (run ^ swz(cl))]) = rb[p][u][t];
        }
      }
    }
    double v = 1.0;
#pragma unroll
    for (int h = NH - 1; h >= 0; --h) v = (h == NH - 1) ? rs[p][h] : v * rs[p][h];
    Ss[buf][scl] = v;
  };

  v4f accf[TM][TN];
  v4d acc[TM][TN];
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y) {
      accf[x][y] = v4f{0.f, 0.f, 0.f, 0.f};
      acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};
    }

  // Pipeline: at the start of step s, LDS buffer s&1 holds step s, the
  // stage of parity (s+1)&1 holds step s+1 and the other stage step s+2
  // (loads possibly in flight).  Step s computes from LDS, stores step s+1
  // into the other buffer, synchronises, and reuses the freed stage for the
  // loads of step s+3.
  if constexpr (BRES) {
    // every K block of the wrap, this block's columns (past ldc: clamped,
    // their outputs are never stored)
    const int items = sw * BN * CH;
    for (int it = tid; it < items; it += NT) {
      const int jb = it / (BN * CH);
      const int rem = it - jb * (BN * CH);
      const int cl = rem / CH, run = rem % CH;
      const uint32_t at = c0 + cl < a.ldc ? ((uint32_t)jb * (uint32_t)a.ldc + (uint32_t)(c0 + cl)) * BK + 8u * run : 0u;
#pragma unroll
      for (int t = 0; t < NTERM; ++t)
        *reinterpret_cast<u32x4*>(&Bres[(((int64_t)t * sw + jb) * BN + cl) * BK + 8 * (run ^ swz(cl))]) =
            *reinterpret_cast<const u32x4*>(Up + (int64_t)t * a.ut_plane + at);
    }
  }
  load_step(S0_t{}, 0);
  store_step(S0_t{}, 0);
  __syncthreads();
  load_step(S1_t{}, 1);
  load_step(S0_t{}, 2);

  const int arow = wm * TM * 16 + (lane & 15);
  const int bcol = wn * TN * 16 + (lane & 15);
  const int kq = 8 * ((lane >> 4) ^ swz(lane & 15));   // fragment rows are 16-aligned
  int in_wrap = 0;        // steps of the current wrap done
  int since_flush = 0;    // steps accumulated in float32
  constexpr int NPROD = NTERM == 3 ? 6 : 3;
  constexpr int NMF = TM * TN * NPROD;            // matrix instructions per step
  constexpr int NRD = NTERM * (TN + TM);          // fragment reads per step
  constexpr int NWR = NTERM * (AI + (BRES ? 0 : BI));   // LDS writes of the store
  auto step = [&](int s, auto P) __attribute__((always_inline)) {
    const int buf = s & 1;
    __builtin_amdgcn_sched_barrier(0);
    bf16x8 bfr[NTERM][TN];
#pragma unroll
    for (int t = 0; t < NTERM; ++t)
#pragma unroll
      for (int y = 0; y < TN; ++y)
        bfr[t][y] = BRES ? *reinterpret_cast<const bf16x8*>(&Bres[(((int64_t)t * sw + in_wrap) * BN + bcol + y * 16) * BK + kq])
                         : *reinterpret_cast<const bf16x8*>(&Bs[buf][t][bcol + y * 16][kq]);
#pragma unroll
    for (int x = 0; x < TM; ++x) {
      bf16x8 af[NTERM];
#pragma unroll
      for (int t = 0; t < NTERM; ++t)
        af[t] = *reinterpret_cast<const bf16x8*>(&As[buf][t][arow + x * 16][kq]);
#pragma unroll
      for (int y = 0; y < TN; ++y) {
        v4f c = accf[x][y];
        if constexpr (NTERM == 3) {
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[2], bfr[0][y], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1], bfr[1][y], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0], bfr[2][y], c, 0, 0, 0);
        }
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1], bfr[0][y], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0], bfr[1][y], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0], bfr[0][y], c, 0, 0, 0);
        accf[x][y] = c;
      }
    }
    // the next step's store (the other LDS buffer, free since the last
    // barrier) interleaved with the matrix instructions
    store_step(P, buf ^ 1);
    __builtin_amdgcn_sched_group_barrier(0x100, NRD, 0);       // fragment reads
#pragma unroll
    for (int i = 0; i < NMF; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);       // matrix
      if (i % (NMF / NWR > 0 ? NMF / NWR : 1) == 0)
        __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);     // LDS write
    }
    __builtin_amdgcn_sched_barrier(0);
    ++in_wrap;
    ++since_flush;
    const bool wrap_end = in_wrap == sw;
    if (wrap_end || since_flush == kFlushSteps) {
      // the wrap's float32 sums, scaled by its Khatri-Rao factor, into float64
      double sc[TN];
#pragma unroll
      for (int y = 0; y < TN; ++y) sc[y] = Ss[buf][bcol + y * 16];
#pragma unroll
      for (int x = 0; x < TM; ++x)
#pragma unroll
        for (int y = 0; y < TN; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            acc[x][y][r] += sc[y] * (double)accf[x][y][r];
            accf[x][y][r] = 0.f;
          }
      since_flush = 0;
    }
    if (wrap_end) in_wrap = 0;
    __syncthreads();
    load_step(P, s + 3);
  };
  // Pairs of steps (stage parity is a compile-time constant) with no
  // conditional step inside the loop, so the load count between a step's
  // loads and its store is the same on every iteration; an odd last step
  // runs after the loop.
  int s = 0;
  for (; s + 1 < nsteps; s += 2) {
    step(s, S1_t{});
    step(s + 1, S0_t{});
  }
  if (s < nsteps) step(s, S1_t{});

  // Epilogue: v_mfma_f32_16x16x32_bf16 leaves row 4*(l/16)+r, column l%16
  // of its 16x16 tile in lane l, element r.  (Every chunk ends on a wrap
  // boundary, so the float32 accumulators are empty here.)
  double* __restrict__ out = a.partial + (int64_t)split * a.M * a.ldc;
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + wm * TM * 16 + x * 16 + 4 * (lane >> 4) + r;
        const int col = c0 + wn * TN * 16 + y * 16 + (lane & 15);
        if (row < a.M && col < a.ldc) out[(int64_t)row * a.ldc + col] = acc[x][y][r];
      }
}

constexpr size_t kLdsBytes = 160 * 1024;   // LDS per compute unit on gfx950

template <int WM, int WN, int TM, int TN, int NTERM>
hipError_t launch_bf(const MttkrpArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (a.ilp <= 0 || a.ilp % kBK != 0 || a.nh != a.nother - 1) return hipErrorInvalidValue;
  constexpr int BM = WM * TM * 16, BN = WN * TN * 16;
  const dim3 grid(a.mtiles * a.ntiles * a.splits);
  const dim3 block(64 * WM * WN);
  // B resident when it fits next to the static tiles
  constexpr size_t fixed = (size_t)2 * NTERM * BM * kBK * 2 + (size_t)2 * BN * 8 + NTERM * kBK * 2;
  const size_t bres = (size_t)NTERM * BN * a.ilp * 2;
  const bool resident = fixed + bres <= kLdsBytes;
  // with events, the dispatch stamps them itself
  auto go = [&](auto kernel, size_t dyn) -> hipError_t {
    if (dyn > 0) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
      if (e != hipSuccess) return e;
    }
    if (e0 || e1)
      hipExtLaunchKernelGGL(kernel, grid, block, dyn, s, e0, e1, 0, a);
    else
      hipLaunchKernelGGL(kernel, grid, block, dyn, s, a);
    return hipSuccess;
  };
  hipError_t e = hipErrorInvalidValue;
  switch (a.nh * 2 + (resident ? 1 : 0)) {
    case 0: e = go(k_mttkrp_bf<WM, WN, TM, TN, NTERM, 0, false>, 0); break;
    case 1: e = go(k_mttkrp_bf<WM, WN, TM, TN, NTERM, 0, true>, bres); break;
    case 2: e = go(k_mttkrp_bf<WM, WN, TM, TN, NTERM, 1, false>, 0); break;
    case 3: e = go(k_mttkrp_bf<WM, WN, TM, TN, NTERM, 1, true>, bres); break;
    case 4: e = go(k_mttkrp_bf<WM, WN, TM, TN, NTERM, 2, false>, 0); break;
    case 5: e = go(k_mttkrp_bf<WM, WN, TM, TN, NTERM, 2, true>, bres); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace

// instr = 0: tiles of 16-row matrix-core blocks (the host derives the row
// tile as wm * tm * 16 from it); the term count is fixed by the table.
#define JKC_BF_VARIANT(WM, WN, TM, TN, NTERM) \
  { WM, WN, TM, TN, kBK, &launch_bf<WM, WN, TM, TN, NTERM>, 0 }

const std::vector<MttkrpVariant>& mttkrp_split_variants() {
  static const std::vector<MttkrpVariant> v = {
      JKC_BF_VARIANT(2, 2, 7, 2, 2),   // 224 x 64
      JKC_BF_VARIANT(2, 2, 4, 2, 2),   // 128 x 64
      JKC_BF_VARIANT(2, 2, 4, 4, 2),   // 128 x 128
      JKC_BF_VARIANT(1, 4, 7, 2, 2),   // 112 x 128
      JKC_BF_VARIANT(1, 4, 5, 2, 2),   // 80 x 128
      JKC_BF_VARIANT(2, 2, 2, 2, 2),   // 64 x 64
      JKC_BF_VARIANT(2, 4, 4, 2, 2),   // 128 x 128, 8 wavefronts
      JKC_BF_VARIANT(4, 2, 4, 2, 2),   // 256 x 64, 8 wavefronts
  };
  return v;
}

const std::vector<MttkrpVariant>& mttkrp_split3_variants() {
  static const std::vector<MttkrpVariant> v = {
      JKC_BF_VARIANT(2, 2, 7, 2, 3),   // 224 x 64
      JKC_BF_VARIANT(2, 2, 4, 2, 3),   // 128 x 64
      JKC_BF_VARIANT(1, 4, 7, 2, 3),   // 112 x 128
      JKC_BF_VARIANT(1, 4, 5, 2, 3),   // 80 x 128
      JKC_BF_VARIANT(2, 2, 2, 2, 3),   // 64 x 64
      JKC_BF_VARIANT(2, 4, 4, 2, 3),   // 128 x 128, 8 wavefronts
      JKC_BF_VARIANT(4, 2, 4, 2, 3),   // 256 x 64, 8 wavefronts
      JKC_BF_VARIANT(1, 4, 8, 2, 3),   // 128 x 128 (a 120-row mode in one row tile)
  };
  return v;
}

}  // namespace jkc
