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
// (BM = WM*TM*16, BN = WN*TN*16) and one contiguous chunk of the K range.
// Per K step of BK columns it stages the A tile (BM x BK slice of the
// unfolding) and the generated B tile (BK x BN KRP slice) in LDS; each
// wavefront then issues TM x TN v_mfma_f64_16x16x4 per 4 columns of K.
// Partials of the K chunks are summed later in a fixed order, so results are
// bitwise repeatable for a fixed tiling.
#include "jkc_internal.hpp"

namespace jkc {

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {

constexpr int kPad = 8;  // LDS row padding (doubles)

template <int WM, int WN, int TM, int TN, int BK>
__global__ void __launch_bounds__(64 * WM * WN)
k_mttkrp_f64(const MttkrpArgs a) {
  constexpr int NT = 64 * WM * WN;
  constexpr int BM = WM * TM * 16;
  constexpr int BN = WN * TN * 16;
  constexpr int LDA = BM + kPad;
  constexpr int LDB = BN + kPad;
  static_assert(BK % 4 == 0 && BK <= NT, "BK");

  __shared__ double As[BK][LDA];
  __shared__ double Bs[BK][LDB];
  __shared__ int64_t s_toff[BK];
  __shared__ int32_t s_roff[kMaxOrder - 1][BK];

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

  v4d acc[TM][TN];
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y) acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};

  const double* __restrict__ Tf64 = static_cast<const double*>(a.T);
  const float* __restrict__ Tf32 = static_cast<const float*>(a.T);

  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    // Column decode: j -> indices of the other modes (lowest fastest, Eq. (3)).
    if (tid < BK) {
      const int64_t j = k0 + tid;
      if (j < kend) {
        uint32_t rem = (uint32_t)j;
        int64_t toff = 0;
#pragma unroll
        for (int q = 0; q < kMaxOrder - 1; ++q) {
          if (q < a.nother) {
            const uint32_t d = (uint32_t)a.odim[q];
            const uint32_t idx = rem % d;
            rem /= d;
            toff += (int64_t)idx * a.ostride[q];
            s_roff[q][tid] = (int32_t)idx * a.ldc;
          }
        }
        s_toff[tid] = toff;
      } else {
        s_toff[tid] = -1;
      }
    }
    __syncthreads();

    // A tile: As[k][i] = T_(n)(i0 + i, k0 + k), zero outside the matrix.
    if (a.stride_n == 1) {
      for (int e = tid; e < BM * BK; e += NT) {
        const int i = e % BM, k = e / BM;
        const int64_t toff = s_toff[k];
        double v = 0.0;
        if (toff >= 0 && i0 + i < a.M) {
          const int64_t addr = toff + (int64_t)(i0 + i);
          v = a.t_is_f32 ? (double)Tf32[addr] : Tf64[addr];
        }
        As[k][i] = v;
      }
    } else {
      for (int e = tid; e < BM * BK; e += NT) {
        const int k = e % BK, i = e / BK;
        const int64_t toff = s_toff[k];
        double v = 0.0;
        if (toff >= 0 && i0 + i < a.M) {
          const int64_t addr = toff + (int64_t)(i0 + i) * a.stride_n;
          v = a.t_is_f32 ? (double)Tf32[addr] : Tf64[addr];
        }
        As[k][i] = v;
      }
    }
    // B tile: Bs[k][c] = KRP(k0 + k, c0 + c), multiplied from the highest
    // mode down (the listing order of Eq. (1)).
    for (int e = tid; e < BK * BN; e += NT) {
      const int c = e % BN, k = e / BN;
      const int col = c0 + c;
      double v = 0.0;
      if (s_toff[k] >= 0 && col < a.ncols) {
        const int q0 = a.nother - 1;
        v = a.oU[q0][s_roff[q0][k] + col];
        for (int q = q0 - 1; q >= 0; --q) v *= a.oU[q][s_roff[q][k] + col];
      }
      Bs[k][c] = v;
    }
    __syncthreads();

    const int arow = wm * TM * 16 + (lane & 15);
    const int bcol = wn * TN * 16 + (lane & 15);
    const int kq = lane >> 4;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double av[TM], bv[TN];
#pragma unroll
      for (int x = 0; x < TM; ++x) av[x] = As[kk + kq][arow + x * 16];
#pragma unroll
      for (int y = 0; y < TN; ++y) bv[y] = Bs[kk + kq][bcol + y * 16];
#pragma unroll
      for (int x = 0; x < TM; ++x)
#pragma unroll
        for (int y = 0; y < TN; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }

  // Epilogue: for v_mfma_f64_16x16x4 lane l holds, in accumulator element r,
  // row 4*r + l/16 and column l%16 of its 16x16 tile.
  double* __restrict__ out = a.partial + (int64_t)split * a.M * a.ldc;
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + wm * TM * 16 + x * 16 + 4 * r + (lane >> 4);
        const int col = c0 + wn * TN * 16 + y * 16 + (lane & 15);
        if (row < a.M && col < a.ldc) out[(int64_t)row * a.ldc + col] = acc[x][y][r];
      }
}

template <int WM, int WN, int TM, int TN, int BK>
hipError_t launch_f64(const MttkrpArgs& a, hipStream_t s) {
  dim3 grid(a.mtiles * a.ntiles, a.splits);
  hipLaunchKernelGGL((k_mttkrp_f64<WM, WN, TM, TN, BK>), grid, dim3(64 * WM * WN), 0, s, a);
  return hipGetLastError();
}

}  // namespace

const std::vector<MttkrpVariant>& mttkrp_f64_variants() {
  static const std::vector<MttkrpVariant> v = {
      {2, 2, 2, 2, 16, &launch_f64<2, 2, 2, 2, 16>},   // 64 x 64
      {2, 2, 2, 4, 16, &launch_f64<2, 2, 2, 4, 16>},   // 64 x 128
      {1, 4, 4, 2, 16, &launch_f64<1, 4, 4, 2, 16>},   // 64 x 128
      {1, 4, 7, 2, 16, &launch_f64<1, 4, 7, 2, 16>},   // 112 x 128
      {2, 2, 4, 2, 16, &launch_f64<2, 2, 4, 2, 16>},   // 128 x 64
      {2, 2, 1, 1, 32, &launch_f64<2, 2, 1, 1, 32>},   // 32 x 32
      {4, 1, 1, 1, 32, &launch_f64<4, 1, 1, 1, 32>},   // 64 x 16
      {4, 1, 2, 1, 32, &launch_f64<4, 1, 2, 1, 32>},   // 128 x 16
      {1, 4, 1, 1, 32, &launch_f64<1, 4, 1, 1, 32>},   // 16 x 64
  };
  return v;
}

}  // namespace jkc
