// Split-precision fused MTTKRP: the same product as the float64 kernel
// (Alg. 3, MTTKRP step, over the full tensor with on-the-fly Khatri-Rao
// tiles), computed on the bfloat16 matrix cores.
//
// Every operand x is written as a sum of NTERM bfloat16 terms, each the
// round-to-nearest-even of what the previous terms leave (x1 = bf16(x),
// x2 = bf16(x - x1), ...): the tensor once at init, directly from float64;
// the Khatri-Rao entries as they are generated, from a float32 product of the
// factor entries.  Products keep every term pair whose magnitude is at least
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
#include "jkc_internal.hpp"

namespace jkc {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int kBK = 32;           // one v_mfma_f32_16x16x32_bf16 deep
constexpr int kLdk = kBK + 8;     // LDS row pitch in bf16 elements (80 bytes)
constexpr int kFlushK = 2048;     // float32 accumulation span before a float64 flush

// Incremental walk over columns j of the unfolding (lowest other mode
// fastest, Eq. (3)); no divisions once initialised.
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
  __device__ int64_t toff(const MttkrpArgs& a) const {
    return (int64_t)idx[0] * a.ostride[0] + (int64_t)idx[1] * a.ostride[1] +
           (int64_t)idx[2] * a.ostride[2];
  }
};

__device__ inline uint16_t bf16_bits(__bf16 x) { return __builtin_bit_cast(uint16_t, x); }

__device__ inline uint4 pack8(const uint16_t* v) {
  uint4 r;
  r.x = v[0] | ((uint32_t)v[1] << 16);
  r.y = v[2] | ((uint32_t)v[3] << 16);
  r.z = v[4] | ((uint32_t)v[5] << 16);
  r.w = v[6] | ((uint32_t)v[7] << 16);
  return r;
}

template <int WM, int WN, int TM, int TN, int NTERM>
__global__ void __launch_bounds__(64 * WM * WN)
k_mttkrp_split(const MttkrpArgs a) {
  constexpr int NT = 64 * WM * WN;
  constexpr int BM = WM * TM * 16;
  constexpr int BN = WN * TN * 16;
  constexpr int BK = kBK;
  constexpr int VA = BM * BK / NT;     // A values per thread per step
  constexpr int VB = BN * BK / NT;     // B values per thread per step
  static_assert(VA % 8 == 0 && VB % 8 == 0 && VA <= BK && VB <= BK, "vector widths");
  static_assert(NTERM == 2 || NTERM == 3, "terms");

  __shared__ __attribute__((aligned(16))) uint16_t As[2][NTERM][BM][kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][NTERM][BN][kLdk];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM;
  const int wn = wave / WM;

  const int tile = blockIdx.x;
  const int split = blockIdx.y;
  const int mt = tile % a.mtiles;
  const int nt = tile / a.mtiles;
  const int i0 = mt * BM;
  const int c0 = nt * BN;
  const int64_t kbeg = (int64_t)split * a.kchunk;
  const int64_t kend = min(kbeg + a.kchunk, a.J);
  const int nsteps = kend > kbeg ? (int)((kend - kbeg + BK - 1) / BK) : 0;

  // A roles.  Unit-stride mode: a thread owns one row and a run of VA
  // consecutive columns (row-contiguous global loads, 16-byte LDS writes).
  // Otherwise: a thread owns one column and VA rows (column-contiguous loads).
  const bool m_fast = a.stride_n == 1;
  const int aRow = m_fast ? tid % BM : (tid / BK) * VA;
  const int aK = m_fast ? (tid / BM) * VA : tid % BK;
  // B roles: a thread owns one Khatri-Rao column and VB consecutive k.
  const int bCol = tid % BN;
  const int bK = (tid / BN) * VB;

  Walk wA, wB;
  wA.init(a, kbeg + aK);
  wB.init(a, kbeg + bK);

  const uint16_t* __restrict__ Tp = static_cast<const uint16_t*>(a.T);

  uint16_t ra[NTERM][VA];
  float rb[kMaxOrder - 1][VB];   // factor entries, rounded to float32 on load

  auto load_step = [&]() {
    if (m_fast) {
      Walk w = wA;
      const int row = i0 + aRow;
#pragma unroll
      for (int v = 0; v < VA; ++v) {
        const bool ok = w.j < kend && row < a.M;
        const int64_t addr = w.toff(a) + row;
#pragma unroll
        for (int t = 0; t < NTERM; ++t) ra[t][v] = ok ? Tp[t * a.plane + addr] : (uint16_t)0;
        w.advance(a, 1);
      }
    } else {
      const bool ok = wA.j < kend;
      const int64_t toff = wA.toff(a);
#pragma unroll
      for (int v = 0; v < VA; ++v) {
        const int row = i0 + aRow + v;
        const bool okr = ok && row < a.M;
        const int64_t addr = toff + (int64_t)row * a.stride_n;
#pragma unroll
        for (int t = 0; t < NTERM; ++t) ra[t][v] = okr ? Tp[t * a.plane + addr] : (uint16_t)0;
      }
    }
    Walk w = wB;
    const int col = c0 + bCol;
#pragma unroll
    for (int v = 0; v < VB; ++v) {
      const bool ok = w.j < kend && col < a.ncols;
#pragma unroll
      for (int q = 0; q < kMaxOrder - 1; ++q)
        if (q < a.nother) rb[q][v] = ok ? (float)a.oU[q][(int64_t)w.idx[q] * a.ldc + col] : 0.f;
      w.advance(a, 1);
    }
  };
  auto store_step = [&](int buf) {
#pragma unroll
    for (int t = 0; t < NTERM; ++t) {
      if (m_fast) {
#pragma unroll
        for (int v = 0; v < VA; v += 8)
          *reinterpret_cast<uint4*>(&As[buf][t][aRow][aK + v]) = pack8(&ra[t][v]);
      } else {
#pragma unroll
        for (int v = 0; v < VA; ++v) As[buf][t][aRow + v][aK] = ra[t][v];
      }
    }
    uint16_t bt[NTERM][VB];
#pragma unroll
    for (int v = 0; v < VB; ++v) {
      // Khatri-Rao entry in float32 (highest mode first, Eq. (1) order),
      // split into bfloat16 terms with the hardware round-to-nearest-even
      // conversion; each remainder is exact in float32.
      float f = 0.f;
      bool first = true;
#pragma unroll
      for (int q = kMaxOrder - 2; q >= 0; --q)
        if (q < a.nother) {
          f = first ? rb[q][v] : f * rb[q][v];
          first = false;
        }
#pragma unroll
      for (int t = 0; t < NTERM; ++t) {
        const __bf16 h = (__bf16)f;
        bt[t][v] = bf16_bits(h);
        f = f - (float)h;
      }
    }
#pragma unroll
    for (int t = 0; t < NTERM; ++t)
#pragma unroll
      for (int v = 0; v < VB; v += 8)
        *reinterpret_cast<uint4*>(&Bs[buf][t][bCol][bK + v]) = pack8(&bt[t][v]);
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

  if (nsteps > 0) {
    load_step();
    store_step(0);
  }
  __syncthreads();

  const int arow = wm * TM * 16 + (lane & 15);
  const int bcol = wn * TN * 16 + (lane & 15);
  const int kq = 8 * (lane >> 4);
  int since_flush = 0;
  for (int s = 0; s < nsteps; ++s) {
    const int buf = s & 1;
    const bool more = s + 1 < nsteps;
    if (more) {
      wA.advance(a, BK);
      wB.advance(a, BK);
      load_step();
    }
    bf16x8 af[NTERM][TM], bfr[NTERM][TN];
#pragma unroll
    for (int t = 0; t < NTERM; ++t) {
#pragma unroll
      for (int x = 0; x < TM; ++x)
        af[t][x] = *reinterpret_cast<const bf16x8*>(&As[buf][t][arow + x * 16][kq]);
#pragma unroll
      for (int y = 0; y < TN; ++y)
        bfr[t][y] = *reinterpret_cast<const bf16x8*>(&Bs[buf][t][bcol + y * 16][kq]);
    }
#pragma unroll
    for (int x = 0; x < TM; ++x)
#pragma unroll
      for (int y = 0; y < TN; ++y) {
        v4f c = accf[x][y];
        if constexpr (NTERM == 3) {
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[2][x], bfr[0][y], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][x], bfr[1][y], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][x], bfr[2][y], c, 0, 0, 0);
        }
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][x], bfr[0][y], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][x], bfr[1][y], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][x], bfr[0][y], c, 0, 0, 0);
        accf[x][y] = c;
      }
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
    if (more) store_step(buf ^ 1);
    __syncthreads();
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
hipError_t launch_split(const MttkrpArgs& a, hipStream_t s) {
  dim3 grid(a.mtiles * a.ntiles, a.splits);
  hipLaunchKernelGGL((k_mttkrp_split<WM, WN, TM, TN, NTERM>), grid, dim3(64 * WM * WN), 0, s, a);
  return hipGetLastError();
}

}  // namespace

const std::vector<MttkrpVariant>& mttkrp_split_variants() {
  static const std::vector<MttkrpVariant> v = {
      {2, 2, 2, 2, kBK, &launch_split<2, 2, 2, 2, 2>, 2},   // 64 x 64
      {2, 2, 4, 2, kBK, &launch_split<2, 2, 4, 2, 2>, 2},   // 128 x 64
      {2, 2, 2, 4, kBK, &launch_split<2, 2, 2, 4, 2>, 2},   // 64 x 128
      {2, 2, 4, 4, kBK, &launch_split<2, 2, 4, 4, 2>, 2},   // 128 x 128
  };
  return v;
}

const std::vector<MttkrpVariant>& mttkrp_split3_variants() {
  static const std::vector<MttkrpVariant> v = {
      {2, 2, 2, 2, kBK, &launch_split<2, 2, 2, 2, 3>, 3},   // 64 x 64
      {2, 2, 4, 2, kBK, &launch_split<2, 2, 4, 2, 3>, 3},   // 128 x 64
      {2, 2, 2, 4, kBK, &launch_split<2, 2, 2, 4, 3>, 3},   // 64 x 128
  };
  return v;
}

}  // namespace jkc
