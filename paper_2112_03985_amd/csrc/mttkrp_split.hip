// Split-precision fused MTTKRP: the same product as the float64 kernel
// (Alg. 3, MTTKRP step, over the full tensor with on-the-fly Khatri-Rao
// tiles), computed on the bfloat16 matrix cores.
//
// Every operand x is written as a sum of NTERM bfloat16 terms, each the
// round-to-nearest-even of what the previous terms leave (x1 = bf16(x),
// x2 = bf16(x - x1), ...): the tensor once at init, directly from float64;
// the Khatri-Rao entries as they are generated, from a float32 product of the
// factor entries (read from float32 copies of the factors made before each
// launch).  Products keep every term pair whose magnitude is at least
// 2^-8(NTERM-1) of the leading one:
//   NTERM = 2: a1 b1 + a1 b2 + a2 b1                       (3 MFMA products)
//   NTERM = 3: the above + a1 b3 + a2 b2 + a3 b1           (6 MFMA products)
// smallest terms first.  Products of bfloat16 are exact in float32; the
// float32 accumulators are added into float64 ones after at most 2048
// columns of K, and split-K partials are float64.
//
// Accuracy: with two terms each operand carries ~17 bits and the result's
// normwise relative error is ~2^-17 times the ratio sum|T||KRP| / |M| (the
// cancellation in the MTTKRP sums), i.e. a few 1e-6 on data without
// cancellation and about 1e-5 when the sums cancel by half; with three
// terms it is ~2^-23 times that ratio.
//
// Layout.  For the split paths the tensor is held once per mode as that
// mode's unfolding (Eq. (3)) stored row-major, rows padded to a multiple of
// 8 columns, one plane per term.  A row of the unfolding is then contiguous,
// so the A operand of a step (BM rows x 32 columns) arrives as aligned
// 16-byte loads of 8 consecutive K for one row -- exactly the register
// layout of the v_mfma_f32_16x16x32_bf16 operands -- and is copied to LDS
// unchanged.
//
// Khatri-Rao generation.  A thread owns one column c of the tile and a run
// of 8 consecutive K (columns j of the unfolding).  Within the run the
// lowest other mode's index advances and the higher modes' indices stay
// fixed unless the run wraps; the product of the higher modes' entries is
// formed once per run and multiplied by the 8 entries of the lowest mode
// (the order highest mode first, as in Eq. (1)).  Runs that wrap take a
// per-entry path.  Each entry is split into its bfloat16 terms with the
// hardware round-to-nearest-even conversion and 8 terms are written to LDS
// as one 16-byte store, again in the operand's register layout.
//
// Tiles are BM x BN with BM = 16 WM TM covering all rows of small modes, so
// each Khatri-Rao entry is generated once per column tile; blocks are dealt
// to the XCDs in contiguous runs of column tiles (they share the tensor
// slice in L2).  The loads of a step are issued two steps before it is
// stored (two register stages), the store runs after the matrix-core work of
// the step before it (double-buffered LDS, one barrier per step).
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
constexpr int kLdk = kBK + 8;     // LDS row pitch in bf16 elements (80 bytes)
constexpr int kFlushK = 2048;     // float32 accumulation span before a float64 flush
constexpr int kXcds = 8;

// Multi-index of the other modes for column j of the unfolding (lowest
// other mode fastest, Eq. (3)), advanced incrementally.
struct Walk {
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
};


template <int WM, int WN, int TM, int TN, int NTERM, int NO>
__global__ void __launch_bounds__(64 * WM * WN)
k_mttkrp_bf(const MttkrpArgs a) {
  constexpr int NT = 64 * WM * WN;
  constexpr int BM = WM * TM * 16;
  constexpr int BN = WN * TN * 16;
  constexpr int BK = kBK;
  constexpr int CH = BK / 8;                         // 8-column runs per row per step
  constexpr int AI = (BM * CH + NT - 1) / NT;        // A runs per thread
  constexpr int BI = (BN * CH + NT - 1) / NT;        // B runs per thread
  static_assert(NTERM == 2 || NTERM == 3, "terms");
  static_assert(NO >= 1 && NO <= kMaxOrder - 1, "other modes");

  __shared__ __attribute__((aligned(16))) uint16_t As[2][NTERM][BM][kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][NTERM][BN][kLdk];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM;
  const int wn = wave / WM;

  // Block -> (column tile, row tile, K chunk), XCD-aware as in the float64
  // kernel: each XCD receives a contiguous run of logical blocks, column
  // tile fastest, so the blocks sharing one tensor slice share an L2.
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

  const uint16_t* __restrict__ Tp = static_cast<const uint16_t*>(a.T);

  // A runs: item e = tid + NT*u -> row e / CH, run e % CH (CH threads cover
  // one row's 64 contiguous bytes per term).  Runs outside the tile or past
  // the chunk read a clamped address and are not masked: past the chunk they
  // meet zero Khatri-Rao entries, and rows past I_n produce output rows that
  // are never stored (a non-finite tensor entry therefore only affects its
  // own output row, which is non-finite in the exact product too).
  const uint16_t* __restrict__ Tt[NTERM];
#pragma unroll
  for (int t = 0; t < NTERM; ++t) Tt[t] = Tp + (int64_t)t * a.plane;
  // B runs: item e -> column e % BN (consecutive threads, consecutive
  // columns: coalesced factor loads), run e / BN.
  Walk wb[BI];
#pragma unroll
  for (int u = 0; u < BI; ++u) wb[u].init(a, kbeg + 8 * ((tid + NT * u) / BN));
  const uint32_t ldc = (uint32_t)a.ldc;

  // Registers of the steps in flight, two stages indexed by a compile-time
  // stage number: the loads of a step are issued two steps before its store
  // (one wavefront per SIMD hides no latency by switching, so the distance
  // has to come from the schedule).
  u32x4 ra[2][AI][NTERM];
  float rlow[2][BI][8];        // the lowest other mode's 8 entries
  float rhigh[2][BI][NO];      // the higher modes' entries (fast path)
  bool bfast[2][BI], bok[2][BI];
  using S0_t = std::integral_constant<int, 0>;
  using S1_t = std::integral_constant<int, 1>;

  auto load_step = [&](auto P, int s) __attribute__((always_inline)) {
    constexpr int p = decltype(P)::value;
    const int64_t j0 = kbeg + (int64_t)s * BK;
#pragma unroll
    for (int u = 0; u < AI; ++u) {
      const int e = tid + NT * u;
      const int row = e / CH, run = e % CH;
      const int64_t j = j0 + 8 * run;
      const bool ok = e < BM * CH && i0 + row < a.M && j < kend;
      // element offset within a plane: below 2^31 (checked at init)
      const uint32_t at = ok ? (uint32_t)(i0 + row) * (uint32_t)a.ldt + (uint32_t)j : 0u;
#pragma unroll
      for (int t = 0; t < NTERM; ++t) ra[p][u][t] = *reinterpret_cast<const u32x4*>(Tt[t] + at);
    }
#pragma unroll
    for (int u = 0; u < BI; ++u) {
      const int e = tid + NT * u;
      const int col = c0 + e % BN;
      const Walk& w = wb[u];
      const bool ok = e < BN * CH && col < a.ldc && w.j < kend;
      bok[p][u] = ok;
      // fast path: the run neither wraps the lowest mode nor crosses kend
      const bool fast = ok && w.idx[0] + 8 <= (uint32_t)a.odim[0] && w.j + 8 <= kend;
      bfast[p][u] = fast;
      // float32 factor copies, 32-bit element offsets (below 2^31, checked
      // at init); rows i_low .. i_low+7 exist on the fast path, row 0 is read
      // eight times otherwise
      const uint32_t cc = ok ? (uint32_t)col : 0u;
      const uint32_t step = fast ? ldc : 0u;
      uint32_t o0 = (fast ? w.idx[0] : 0u) * ldc + cc;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        rlow[p][u][v] = a.oUf[0][o0];
        o0 += step;
      }
#pragma unroll
      for (int q = 1; q < NO; ++q) rhigh[p][u][q] = a.oUf[q][(ok ? w.idx[q] : 0u) * ldc + cc];
    }
  };

  // The store of a step, in two parts.  store_main writes the tensor runs
  // and every Khatri-Rao run by the run formula (the higher modes' product
  // times the 8 entries of the lowest mode), branch-free so that it can be
  // interleaved with the matrix instructions; store_fix then rewrites, entry
  // by entry, the runs the formula does not cover (runs that wrap the lowest
  // mode, end the chunk or lie outside the tile) -- the same thread's later
  // LDS write wins.
  auto store_run = [&](float (&f)[8], int buf, int cl, int run) __attribute__((always_inline)) {
#pragma unroll
    for (int t = 0; t < NTERM; ++t) {
      uint32_t wds[4];
#pragma unroll
      for (int v = 0; v < 8; v += 2) {
        // round-to-nearest-even conversion of two entries; the remainders
        // are exact in float32
        const __bf16 h0 = (__bf16)f[v];
        const __bf16 h1 = (__bf16)f[v + 1];
        wds[v / 2] = (uint32_t)__builtin_bit_cast(uint16_t, h0) |
                     ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
        f[v] -= (float)h0;
        f[v + 1] -= (float)h1;
      }
      *reinterpret_cast<u32x4*>(&Bs[buf][t][cl][8 * run]) = u32x4{wds[0], wds[1], wds[2], wds[3]};
    }
  };
  auto store_main = [&](auto P, int buf) __attribute__((always_inline)) {
    constexpr int p = decltype(P)::value;
#pragma unroll
    for (int u = 0; u < AI; ++u) {
      const int e = tid + NT * u;
      if (AI * NT == BM * CH || e < BM * CH) {
        const int row = e / CH, run = e % CH;
#pragma unroll
        for (int t = 0; t < NTERM; ++t) *reinterpret_cast<u32x4*>(&As[buf][t][row][8 * run]) = ra[p][u][t];
      }
    }
#pragma unroll
    for (int u = 0; u < BI; ++u) {
      const int e = tid + NT * u;
      if (BI * NT == BN * CH || e < BN * CH) {
        const int cl = e % BN, run = e / BN;
        float f[8];
        float hi = 1.f;
#pragma unroll
        for (int q = NO - 1; q >= 1; --q) hi = (q == NO - 1) ? rhigh[p][u][q] : hi * rhigh[p][u][q];
#pragma unroll
        for (int v = 0; v < 8; ++v) f[v] = NO == 1 ? rlow[p][u][v] : hi * rlow[p][u][v];
        store_run(f, buf, cl, run);
      }
    }
  };
  auto store_fix = [&](auto P, int buf, int sdata) __attribute__((always_inline)) {
    constexpr int p = decltype(P)::value;
#pragma unroll
    for (int u = 0; u < BI; ++u) {
      const int e = tid + NT * u;
      if (e >= BN * CH || bfast[p][u]) continue;
      const int cl = e % BN, run = e / BN;
      float f[8];
      Walk w;
      w.init(a, kbeg + (int64_t)sdata * BK + 8 * run);
      const int col = c0 + cl;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        float x = 0.f;
        if (bok[p][u] && w.j < kend) {
#pragma unroll
          for (int q = NO - 1; q >= 0; --q) {
            const float y = a.oUf[q][w.idx[q] * ldc + (uint32_t)col];
            x = (q == NO - 1) ? y : x * y;
          }
        }
        f[v] = x;
        w.advance(a, 1);
      }
      store_run(f, buf, cl, run);
    }
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
  // loads of step s+3.  Loads past the chunk fetch clamped addresses and are
  // masked (zero Khatri-Rao entries), so they are issued unconditionally.
  if (nsteps > 0) {
    load_step(S0_t{}, 0);
    store_main(S0_t{}, 0);
    store_fix(S0_t{}, 0, 0);
  }
  __syncthreads();
  auto advance_all = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < BI; ++u) wb[u].advance(a, BK);
  };
  advance_all();
  load_step(S1_t{}, 1);
  advance_all();
  load_step(S0_t{}, 2);

  const int arow = wm * TM * 16 + (lane & 15);
  const int bcol = wn * TN * 16 + (lane & 15);
  const int kq = 8 * (lane >> 4);
  int since_flush = 0;
  // one step; stage P holds step s+1 and receives step s+3 afterwards
  constexpr int NPROD = NTERM == 3 ? 6 : 3;
  constexpr int NMF = TM * TN * NPROD;            // matrix instructions per step
  constexpr int NRD = NTERM * (TN + TM);          // fragment reads per step
  constexpr int NWR = NTERM * (AI + BI);          // LDS writes of the store
  auto step = [&](int s, auto P) __attribute__((always_inline)) {
    const int buf = s & 1;
    __builtin_amdgcn_sched_barrier(0);
    bf16x8 bfr[NTERM][TN];
#pragma unroll
    for (int t = 0; t < NTERM; ++t)
#pragma unroll
      for (int y = 0; y < TN; ++y)
        bfr[t][y] = *reinterpret_cast<const bf16x8*>(&Bs[buf][t][bcol + y * 16][kq]);
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
    // barrier) interleaved with the matrix instructions: the fragment reads
    // first, then each matrix instruction followed by a few vector
    // instructions, the LDS writes spread over the step
    store_main(P, buf ^ 1);
    __builtin_amdgcn_sched_group_barrier(0x100, NRD, 0);       // fragment reads
#pragma unroll
    for (int i = 0; i < NMF; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);       // matrix
      __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);       // vector ALU
      if (i % (NMF / NWR > 0 ? NMF / NWR : 1) == 0)
        __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);     // LDS write
    }
    __builtin_amdgcn_sched_barrier(0);
    store_fix(P, buf ^ 1, s + 1);
    since_flush += BK;
    if (since_flush >= kFlushK) {
#pragma unroll
      for (int x = 0; x < TM; ++x)
#pragma unroll
        for (int y = 0; y < TN; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            acc[x][y][r] += (double)accf[x][y][r];
            accf[x][y][r] = 0.f;
          }
      since_flush = 0;
    }
    __syncthreads();
    advance_all();
    load_step(P, s + 3);
  };
  for (int s = 0; s < nsteps; s += 2) {
    step(s, S1_t{});
    if (s + 1 < nsteps) step(s + 1, S0_t{});
  }

  // Epilogue: v_mfma_f32_16x16x32_bf16 leaves row 4*(l/16)+r, column l%16
  // of its 16x16 tile in lane l, element r.
  double* __restrict__ out = a.partial + (int64_t)split * a.M * a.ldc;
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + wm * TM * 16 + x * 16 + 4 * (lane >> 4) + r;
        const int col = c0 + wn * TN * 16 + y * 16 + (lane & 15);
        const double v = acc[x][y][r] + (double)accf[x][y][r];
        if (row < a.M && col < a.ldc) out[(int64_t)row * a.ldc + col] = v;
      }
}

template <int WM, int WN, int TM, int TN, int NTERM>
hipError_t launch_bf(const MttkrpArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const dim3 grid(a.mtiles * a.ntiles * a.splits);
  const dim3 block(64 * WM * WN);
  // with events, the dispatch stamps them itself
  auto go = [&](auto kernel) {
    if (e0 || e1)
      hipExtLaunchKernelGGL(kernel, grid, block, 0, s, e0, e1, 0, a);
    else
      hipLaunchKernelGGL(kernel, grid, block, 0, s, a);
  };
  switch (a.nother) {
    case 1: go(k_mttkrp_bf<WM, WN, TM, TN, NTERM, 1>); break;
    case 2: go(k_mttkrp_bf<WM, WN, TM, TN, NTERM, 2>); break;
    case 3: go(k_mttkrp_bf<WM, WN, TM, TN, NTERM, 3>); break;
    default: return hipErrorInvalidValue;
  }
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
  };
  return v;
}

}  // namespace jkc
