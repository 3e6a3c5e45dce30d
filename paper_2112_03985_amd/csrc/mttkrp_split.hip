// Split-precision fused MTTKRP: the same product as the float64 kernel
// (Alg. 3, MTTKRP step, over the full tensor with on-the-fly Khatri-Rao
// tiles), computed on the bfloat16 matrix cores.
//
// Every float64 operand x is represented as hi + lo with hi = bf16(x) and
// lo = bf16(x - hi), both rounded to nearest even (the tensor once at init,
// the Khatri-Rao entries as they are generated).  The product of two such
// operands is approximated by three bfloat16 MFMA products
//   a*b ~ a_hi*b_hi + a_hi*b_lo + a_lo*b_hi
// (the dropped a_lo*b_lo term is below 2^-16 relative), each exact in the
// float32 accumulator's precision.  The float32 accumulators are added into
// float64 ones after at most 2048 columns of K, and split-K partials are
// float64, so accumulation error stays far below the representation error.
#include "jkc_internal.hpp"

namespace jkc {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int kBK = 32;           // one v_mfma_f32_16x16x32_bf16 deep
constexpr int kLdk = kBK + 8;     // LDS row pitch in bf16 elements (80 bytes)
constexpr int kFlushK = 2048;     // float32 accumulation span before a float64 flush

__device__ inline uint16_t bf16_rne_d(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t sign = (uint32_t)(b >> 63) << 15;
  const int e = (int)((b >> 52) & 0x7ff);
  const uint64_t m = b & ((1ull << 52) - 1);
  if (e == 0x7ff) return (uint16_t)(sign | 0x7f80u | (m ? 0x40u : 0u));
  const int eb = e - 1023 + 127;
  if (eb >= 255) return (uint16_t)(sign | 0x7f80u);
  if (eb <= 0) {
    if (e == 0) return (uint16_t)sign;
    const int drop = 45 + (1 - eb);
    if (drop > 62) return (uint16_t)sign;
    const uint64_t full = (1ull << 52) | m;
    uint64_t q = full >> drop;
    const uint64_t rem = full & ((1ull << drop) - 1);
    const uint64_t half = 1ull << (drop - 1);
    if (rem > half || (rem == half && (q & 1))) ++q;
    return (uint16_t)(sign | (uint32_t)q);
  }
  uint32_t r = ((uint32_t)eb << 7) | (uint32_t)(m >> 45);
  const uint64_t rem = m & ((1ull << 45) - 1);
  const uint64_t half = 1ull << 44;
  if (rem > half || (rem == half && (r & 1))) ++r;
  return (uint16_t)(sign | r);
}

__device__ inline double bf16_as_double(uint16_t h) {
  return (double)__uint_as_float((uint32_t)h << 16);
}

template <int WM, int WN, int TM, int TN>
__global__ void __launch_bounds__(64 * WM * WN)
k_mttkrp_split(const MttkrpArgs a) {
  constexpr int NT = 64 * WM * WN;
  constexpr int BM = WM * TM * 16;
  constexpr int BN = WN * TN * 16;
  constexpr int BK = kBK;

  __shared__ __attribute__((aligned(16))) uint16_t Ah[BM][kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t Al[BM][kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t Bh[BN][kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t Bl[BN][kLdk];
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

  v4f accf[TM][TN];
  v4d acc[TM][TN];
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y) {
      accf[x][y] = v4f{0.f, 0.f, 0.f, 0.f};
      acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};
    }

  const uint16_t* __restrict__ Thi = static_cast<const uint16_t*>(a.T);
  const uint16_t* __restrict__ Tlo = static_cast<const uint16_t*>(a.T_lo);
  int since_flush = 0;

  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
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

    // A tile (tensor planes), stored k-contiguous per row.
    if (a.stride_n == 1) {
      for (int e = tid; e < BM * BK; e += NT) {
        const int i = e % BM, k = e / BM;
        const int64_t toff = s_toff[k];
        uint16_t h = 0, l = 0;
        if (toff >= 0 && i0 + i < a.M) {
          const int64_t addr = toff + (int64_t)(i0 + i);
          h = Thi[addr];
          l = Tlo[addr];
        }
        Ah[i][k] = h;
        Al[i][k] = l;
      }
    } else {
      for (int e = tid; e < BM * BK; e += NT) {
        const int k = e % BK, i = e / BK;
        const int64_t toff = s_toff[k];
        uint16_t h = 0, l = 0;
        if (toff >= 0 && i0 + i < a.M) {
          const int64_t addr = toff + (int64_t)(i0 + i) * a.stride_n;
          h = Thi[addr];
          l = Tlo[addr];
        }
        Ah[i][k] = h;
        Al[i][k] = l;
      }
    }
    // B tile: float64 Khatri-Rao entries, split into bf16 hi + lo.
    for (int e = tid; e < BK * BN; e += NT) {
      const int c = e % BN, k = e / BN;
      const int col = c0 + c;
      uint16_t h = 0, l = 0;
      if (s_toff[k] >= 0 && col < a.ncols) {
        const int q0 = a.nother - 1;
        double v = a.oU[q0][s_roff[q0][k] + col];
        for (int q = q0 - 1; q >= 0; --q) v *= a.oU[q][s_roff[q][k] + col];
        h = bf16_rne_d(v);
        l = bf16_rne_d(v - bf16_as_double(h));
      }
      Bh[c][k] = h;
      Bl[c][k] = l;
    }
    __syncthreads();

    const int arow = wm * TM * 16 + (lane & 15);
    const int bcol = wn * TN * 16 + (lane & 15);
    const int kq = 8 * (lane >> 4);
    bf16x8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
    for (int x = 0; x < TM; ++x) {
      ah[x] = *reinterpret_cast<const bf16x8*>(&Ah[arow + x * 16][kq]);
      al[x] = *reinterpret_cast<const bf16x8*>(&Al[arow + x * 16][kq]);
    }
#pragma unroll
    for (int y = 0; y < TN; ++y) {
      bh[y] = *reinterpret_cast<const bf16x8*>(&Bh[bcol + y * 16][kq]);
      bl[y] = *reinterpret_cast<const bf16x8*>(&Bl[bcol + y * 16][kq]);
    }
#pragma unroll
    for (int x = 0; x < TM; ++x)
#pragma unroll
      for (int y = 0; y < TN; ++y) {
        accf[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[x], bh[y], accf[x][y], 0, 0, 0);
        accf[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[x], bl[y], accf[x][y], 0, 0, 0);
        accf[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[x], bh[y], accf[x][y], 0, 0, 0);
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

template <int WM, int WN, int TM, int TN>
hipError_t launch_split(const MttkrpArgs& a, hipStream_t s) {
  dim3 grid(a.mtiles * a.ntiles, a.splits);
  hipLaunchKernelGGL((k_mttkrp_split<WM, WN, TM, TN>), grid, dim3(64 * WM * WN), 0, s, a);
  return hipGetLastError();
}

}  // namespace

const std::vector<MttkrpVariant>& mttkrp_split_variants() {
  static const std::vector<MttkrpVariant> v = {
      {2, 2, 2, 2, kBK, &launch_split<2, 2, 2, 2>, 2},   // 64 x 64
      {2, 2, 4, 2, kBK, &launch_split<2, 2, 4, 2>, 2},   // 128 x 64
      {2, 2, 2, 4, kBK, &launch_split<2, 2, 2, 4>, 2},   // 64 x 128
      {2, 2, 4, 4, kBK, &launch_split<2, 2, 4, 4>, 2},   // 128 x 128
      {2, 2, 1, 1, kBK, &launch_split<2, 2, 1, 1>, 2},   // 32 x 32
      {4, 1, 1, 1, kBK, &launch_split<4, 1, 1, 1>, 2},   // 64 x 16
  };
  return v;
}

}  // namespace jkc
