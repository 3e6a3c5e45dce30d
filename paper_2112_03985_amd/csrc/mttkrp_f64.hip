// Fused concurrent MTTKRP in float64 on the CDNA4 matrix cores.
//
// Computes, for one mode n, the partial products
//   P_s(i, c) = sum_{j in chunk s} T_(n)(i, j) * KRP(j, c)
// of the fused MTTKRP of JK-CALS (Alg. 3, MTTKRP step; Eq. (1) for one
// model, column-concatenated over all models), where T_(n) is the mode-n
// unfolding of the full tensor (index map Eq. (3)) and
//   KRP(j, c) = prod_{m != n} Ubar_m(i_m(j), c)
// is the Khatri-Rao product of the other modes' multi-factors, generated on
// the fly: it never exists in HBM.  The unfolding is never formed either:
// column j of T_(n) is addressed through the tensor strides of the other
// modes.  Leave-one-out submodels need nothing extra here: their zero row in
// the sampled mode's multi-factor (Case II) makes the KRP entries of the
// left-out slice exactly zero, and the sampled mode's own output row is
// cleared downstream (Case I).
//
// Structure: a block of WM x WN wavefronts owns a BM x BN output tile
// (BM = WM*TM*16, BN = WN*TN*16) and one contiguous chunk of the K range,
// walked in steps of BK columns.  Each step is software-pipelined: the
// global loads of step t+1 (a BM x BK slice of the unfolding and the factor
// rows of a BK x BN Khatri-Rao slice) are in flight while the matrix cores
// work on step t out of LDS; the KRP products are formed and written to the
// other LDS buffer afterwards, so one barrier per step suffices.  Each thread
// owns one column of the A slice and one column of the B slice and walks its
// column's multi-index incrementally (no divisions in the loop).
//
// Matrix instruction (INSTR):
//   0: v_mfma_f64_16x16x4 -- one 16x16 tile per instruction;
//   1: v_mfma_f64_4x4x4 (4 independent 4x4 blocks per instruction): four
//      instructions q = 0..3 cover a 16x16x4 step, block b producing rows
//      4b..4b+3 and columns 4((b+q) mod 4)..+3 (a diagonal schedule, so the
//      A operand is loaded once and four B operands are rotated);
//   2: v_mfma_f64_4x4x4 in row strips: all four blocks take the same 4 rows
//      of A and block b columns 4b..4b+3 of a 16-column group, so one
//      instruction is a 4 x 16 x 4 step and tiles need only multiples of 4
//      rows (no padding of 100- or 200-row modes to 16).
// Partials of the K chunks are summed later in a fixed order, so results are
// bitwise repeatable for a fixed tiling.
#include <type_traits>

#include "jkc_internal.hpp"

namespace jkc {

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {

constexpr int kPad = 8;  // LDS row padding (doubles)
constexpr int kXcds = 8;  // accelerator complex dies on MI355X

// Lane layout of v_mfma_f64_4x4x4 (4 blocks), measured on gfx950: lane l
// belongs to block b = (l >> 2) & 3 and holds, with e = l & 3, kq = l >> 4,
//   A(i = e, k = kq),  B(k = kq, j = e),  D(i = kq, j = e)
// of that block's 4x4x4 product.

// Incremental walk over columns j of the unfolding: the multi-index of the
// other modes (lowest mode fastest, Eq. (3)), the tensor offset of the
// column and the row offsets into the other modes' multi-factors.
struct ColWalker {
  uint32_t idx[kMaxOrder - 1];
  int64_t j;

  __device__ void init(const MttkrpArgs& a, int64_t j0) {
    j = j0;
    uint32_t rem = (uint32_t)min(j0, a.J);
#pragma unroll
    for (int q = 0; q < kMaxOrder - 1; ++q) {
      const uint32_t d = (uint32_t)a.odim[q];
      idx[q] = rem % d;
      rem /= d;
    }
  }
  __device__ void advance(const MttkrpArgs& a, int step) {
    j += step;
    idx[0] += step;
    while (idx[0] >= (uint32_t)a.odim[0]) {
      idx[0] -= a.odim[0];
      if (++idx[1] >= (uint32_t)a.odim[1]) {
        idx[1] = 0;
        ++idx[2];
      }
    }
  }
  __device__ int64_t toff(const MttkrpArgs& a) const {
    return (int64_t)idx[0] * a.ostride[0] + (int64_t)idx[1] * a.ostride[1] +
           (int64_t)idx[2] * a.ostride[2];
  }
};

template <int WM, int WN, int TM, int TN, int BK, int INSTR>
__global__ void __launch_bounds__(64 * WM * WN)
k_mttkrp_f64(const MttkrpArgs a) {
  constexpr int NT = 64 * WM * WN;
  constexpr int RPT = INSTR == 2 ? 4 : 16;   // rows per matrix-core tile
  constexpr int BM = WM * TM * RPT;
  constexpr int BMP = (BM + 15) / 16 * 16;    // rows staged in LDS
  constexpr int BN = WN * TN * 16;
  constexpr int LDA = BMP + kPad;
  constexpr int LDB = BN + kPad;
  constexpr int VA = BMP * BK / NT;  // A elements per thread per step (one column)
  constexpr int VB = BN * BK / NT;   // B elements per thread per step (one column)
  static_assert(BK % 4 == 0, "BK");
  static_assert(VA >= 1 && VA * NT == BMP * BK, "A tile must split evenly over threads");
  static_assert(VB >= 1 && VB * NT == BN * BK, "B tile must split evenly over threads");
  static_assert(BMP % VA == 0 && BN % VB == 0, "vector width");
  using AccT = typename std::conditional<INSTR == 2, double, v4d>::type;

  __shared__ __attribute__((aligned(16))) double As[2][BK][LDA];
  __shared__ __attribute__((aligned(16))) double Bs[2][BK][LDB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM;
  const int wn = wave / WM;

  // Block -> (column tile, row tile, K chunk).  Work-groups are dealt to the
  // 8 XCDs round-robin; remapping so that each XCD receives a contiguous
  // run of logical blocks (column tile fastest) keeps the blocks that share
  // one slice of the unfolding on the same XCD, where it stays in L2.
  const int total = gridDim.x;
  int logical = blockIdx.x;
  const int per_xcd = total / kXcds;
  if (logical < per_xcd * kXcds) logical = (logical % kXcds) * per_xcd + logical / kXcds;
  const int nt = logical % a.ntiles;
  const int mt = (logical / a.ntiles) % a.mtiles;
  const int split = logical / (a.ntiles * a.mtiles);
  const int i0 = mt * BM;
  const int c0 = nt * BN;
  const int64_t kbeg = (int64_t)split * a.kchunk;
  const int64_t kend = min(kbeg + a.kchunk, a.J);
  const int nsteps = kend > kbeg ? (int)((kend - kbeg + BK - 1) / BK) : 0;

  // Thread roles.  A: mode with unit stride (rows contiguous in memory) ->
  // threads run along the rows of one column; otherwise along the columns.
  const bool m_fast = a.stride_n == 1;
  const int kA = m_fast ? tid / (BMP / VA) : tid % BK;
  const int iA = m_fast ? (tid % (BMP / VA)) * VA : (tid / BK) * VA;
  const int kB = tid % BK;
  const int cB = (tid / BK) * VB;

  ColWalker wA, wB;
  wA.init(a, kbeg + kA);
  wB.init(a, kbeg + kB);

  const double* __restrict__ Tf64 = static_cast<const double*>(a.T);
  const float* __restrict__ Tf32 = static_cast<const float*>(a.T);

  double ra[VA];
  double rb[kMaxOrder - 1][VB];

  auto load_step = [&]() {
    const bool va = wA.j < kend;
    const int64_t toffA = wA.toff(a);
#pragma unroll
    for (int v = 0; v < VA; ++v) {
      const int row = i0 + iA + v;
      double x = 0.0;
      if (va && iA + v < BM && row < a.M) {
        const int64_t addr = toffA + (int64_t)row * a.stride_n;
        x = a.t_is_f32 ? (double)Tf32[addr] : Tf64[addr];
      }
      ra[v] = x;
    }
    const bool vb = wB.j < kend;
#pragma unroll
    for (int q = 0; q < kMaxOrder - 1; ++q) {
      if (q < a.nother) {
        const double* __restrict__ urow = a.oU[q] + (int64_t)wB.idx[q] * a.ldc;
#pragma unroll
        for (int v = 0; v < VB; ++v) {
          const int col = c0 + cB + v;
          rb[q][v] = (vb && col < a.ncols) ? urow[col] : 0.0;
        }
      }
    }
  };
  auto store_step = [&](int buf) {
#pragma unroll
    for (int v = 0; v < VA; ++v) As[buf][kA][iA + v] = ra[v];
#pragma unroll
    for (int v = 0; v < VB; ++v) {
      // product from the highest mode down (the listing order of Eq. (1))
      double x = 0.0;
      bool first = true;
#pragma unroll
      for (int q = kMaxOrder - 2; q >= 0; --q)
        if (q < a.nother) {
          x = first ? rb[q][v] : x * rb[q][v];
          first = false;
        }
      Bs[buf][kB][cB + v] = x;
    }
  };

  AccT acc[TM][TN];
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y) acc[x][y] = AccT{};

  if (nsteps > 0) {
    load_step();
    store_step(0);
  }
  __syncthreads();

  const int o16 = lane & 15;
  const int blk = lane >> 4;
  const int b4 = (lane >> 2) & 3;   // 4x4x4 block of this lane
  const int e4 = lane & 3;
  const int kq4 = lane >> 4;
  for (int s = 0; s < nsteps; ++s) {
    const int buf = s & 1;
    const bool more = s + 1 < nsteps;
    if (more) {
      wA.advance(a, BK);
      wB.advance(a, BK);
      load_step();
    }
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double av[TM], bv[TN];
      if constexpr (INSTR == 2) {
        // row strips: every block gets the same 4 rows of A (same LDS
        // addresses), block b the columns 4b..4b+3 of each 16-column group
#pragma unroll
        for (int x = 0; x < TM; ++x) av[x] = As[buf][kk + kq4][wm * TM * 4 + x * 4 + e4];
#pragma unroll
        for (int y = 0; y < TN; ++y) bv[y] = Bs[buf][kk + kq4][wn * TN * 16 + y * 16 + 4 * b4 + e4];
#pragma unroll
        for (int x = 0; x < TM; ++x)
#pragma unroll
          for (int y = 0; y < TN; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[x], bv[y], acc[x][y], 0, 0, 0);
      } else if constexpr (INSTR == 0) {
#pragma unroll
        for (int x = 0; x < TM; ++x) av[x] = As[buf][kk + blk][wm * TM * 16 + x * 16 + o16];
#pragma unroll
        for (int y = 0; y < TN; ++y) bv[y] = Bs[buf][kk + blk][wn * TN * 16 + y * 16 + o16];
#pragma unroll
        for (int x = 0; x < TM; ++x)
#pragma unroll
          for (int y = 0; y < TN; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv[y], acc[x][y], 0, 0, 0);
      } else {
        double bq[TN][4];
#pragma unroll
        for (int x = 0; x < TM; ++x)
          av[x] = As[buf][kk + kq4][wm * TM * 16 + x * 16 + 4 * b4 + e4];
#pragma unroll
        for (int y = 0; y < TN; ++y)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            bq[y][q] = Bs[buf][kk + kq4][wn * TN * 16 + y * 16 + 4 * ((b4 + q) & 3) + e4];
#pragma unroll
        for (int x = 0; x < TM; ++x)
#pragma unroll
          for (int y = 0; y < TN; ++y)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              acc[x][y][q] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[x], bq[y][q], acc[x][y][q], 0, 0, 0);
        (void)bv;
      }
    }
    if (more) store_step(buf ^ 1);
    __syncthreads();
  }

  // Epilogue.  16x16x4: lane l holds, in element r, row 4*r + l/16 and
  // column l%16 of its tile.  4x4x4: element q holds row 4*b + l/16 and
  // column 4*((b+q) mod 4) + (l mod 4), b = (l/4) mod 4.
  double* __restrict__ out = a.partial + (int64_t)split * a.M * a.ldc;
  if constexpr (INSTR == 2) {
    // row strip x, group y: lane holds row 4x + l/16, column 16y + 4b + l%4
#pragma unroll
    for (int x = 0; x < TM; ++x)
#pragma unroll
      for (int y = 0; y < TN; ++y) {
        const int row = i0 + wm * TM * 4 + x * 4 + kq4;
        const int col = c0 + wn * TN * 16 + y * 16 + 4 * b4 + e4;
        if (row < a.M && col < a.ldc) out[(int64_t)row * a.ldc + col] = acc[x][y];
      }
    return;
  } else {
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int rr, cc;
        if (INSTR == 0) {
          rr = 4 * r + blk;
          cc = o16;
        } else {
          rr = 4 * b4 + kq4;
          cc = 4 * ((b4 + r) & 3) + e4;
        }
        const int row = i0 + wm * TM * 16 + x * 16 + rr;
        const int col = c0 + wn * TN * 16 + y * 16 + cc;
        if (row < a.M && col < a.ldc) out[(int64_t)row * a.ldc + col] = acc[x][y][r];
      }
  }
}

template <int WM, int WN, int TM, int TN, int BK, int INSTR>
hipError_t launch_f64(const MttkrpArgs& a, hipStream_t s) {
  dim3 grid(a.mtiles * a.ntiles * a.splits);
  hipLaunchKernelGGL((k_mttkrp_f64<WM, WN, TM, TN, BK, INSTR>), grid, dim3(64 * WM * WN), 0, s, a);
  return hipGetLastError();
}

#define JKC_F64_VARIANT(WM, WN, TM, TN, BK, I) \
  { WM, WN, TM, TN, BK, &launch_f64<WM, WN, TM, TN, BK, I>, I }

}  // namespace

const std::vector<MttkrpVariant>& mttkrp_f64_variants() {
  static const std::vector<MttkrpVariant> v = {
      JKC_F64_VARIANT(1, 4, 25, 2, 16, 2),  // 100 x 128, 4x4x4 row strips
      JKC_F64_VARIANT(2, 2, 25, 2, 16, 2),  // 200 x 64
      JKC_F64_VARIANT(2, 2, 25, 1, 16, 2),  // 200 x 32
      JKC_F64_VARIANT(1, 4, 25, 1, 16, 2),  // 100 x 64
      JKC_F64_VARIANT(2, 2, 13, 2, 16, 2),  // 104 x 64
      JKC_F64_VARIANT(2, 2, 13, 4, 16, 2),  // 104 x 128
      JKC_F64_VARIANT(1, 4, 13, 4, 16, 2),  // 52 x 256
      JKC_F64_VARIANT(2, 2, 25, 4, 16, 2),  // 200 x 128
      JKC_F64_VARIANT(1, 4, 16, 2, 16, 2),  // 64 x 128
      JKC_F64_VARIANT(2, 2, 32, 1, 16, 2),  // 256 x 32
      JKC_F64_VARIANT(2, 2, 2, 2, 16, 1),   // 64 x 64, 4x4x4 diagonal
      JKC_F64_VARIANT(2, 2, 2, 4, 16, 1),   // 64 x 128
      JKC_F64_VARIANT(2, 2, 4, 2, 16, 1),   // 128 x 64
      JKC_F64_VARIANT(1, 4, 7, 2, 16, 1),   // 112 x 128
      JKC_F64_VARIANT(2, 2, 1, 1, 32, 1),   // 32 x 32
      JKC_F64_VARIANT(4, 1, 1, 1, 32, 1),   // 64 x 16
      JKC_F64_VARIANT(4, 1, 2, 1, 32, 1),   // 128 x 16
      JKC_F64_VARIANT(2, 2, 2, 2, 16, 0),   // 64 x 64, 16x16x4
      JKC_F64_VARIANT(2, 2, 4, 2, 16, 0),   // 128 x 64
      JKC_F64_VARIANT(1, 4, 7, 2, 16, 0),   // 112 x 128
  };
  return v;
}

}  // namespace jkc
