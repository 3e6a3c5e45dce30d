// Narrow fused MTTKRP on the vector ALUs, for problems of at most 16
// columns (a single model of small rank: the plain per-submodel ALS of
// Alg. 2, or a jackknife of few columns).  Same product and the same split-K
// partials as the matrix-core kernels (Alg. 3, MTTKRP step; Eq. (1) per
// model), computed as one streaming pass over the tensor: at 2 flops per
// 8-byte element and column the product is bound by HBM, not arithmetic,
// and the matrix-core kernels would pad the columns to their tile width.
//
// The tensor is walked as mode-0 fibers (contiguous in the column-major
// layout of Eq. (3)); the lanes of a wavefront cover the fiber's index k_0
// (SLOTS x 64 >= I_0), so every load is coalesced, and the Khatri-Rao
// factor of the other modes is the same for the whole fiber (wavefront
// uniform):
//   mode 0:    M_0(i, c) += T(i, f) h_f(c),   h_f = prod_{m >= 1} U_m(k_m(f), c)
//              (lanes are the output rows; the four wavefronts of a block
//              take every fourth fiber of its chunk and are summed in order);
//   mode n>0:  M_n(r, c) = sum_{k_0} U_0(k_0, c) sum_f T(k_0, r, f) h_f(c),
//              h_f = prod_{m != 0, n} U_m(k_m(f), c)
//              (a wavefront per output row r; U_0 is applied once per lane
//              after the fiber sum, then the lanes are summed in order).
// K chunks (split-K) are whole fibers; partials are summed afterwards in a
// fixed order, as for the matrix-core kernels.
#include <type_traits>

#include <hip/hip_ext.h>

#include "jkc_internal.hpp"

namespace jkc {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int UF = 8;   // fibers whose loads are in flight together

// Offsets of fiber index q over a set of modes (ascending, lowest fastest):
// tensor offset and each mode's index, advanced incrementally.
template <int NW>
struct FiberWalk {
  uint32_t idx[NW > 0 ? NW : 1];
  __device__ void init(const int32_t* dim, int64_t q) {
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      idx[w] = (uint32_t)(q % dim[w]);
      q /= dim[w];
    }
  }
  __device__ void advance(const int32_t* dim, int step) {
    if constexpr (NW > 0) {
      idx[0] += step;
#pragma unroll
      for (int w = 0; w + 1 < NW; ++w) {
        while (idx[w] >= (uint32_t)dim[w]) {
          idx[w] -= dim[w];
          ++idx[w + 1];
        }
      }
    }
  }
};

// NO: other modes of the output mode (N - 1); NC: columns computed (the
// rest of the 16-column pitch are zero padding); SLOTS: lanes x slots cover
// I_0; MODE0: the output mode is mode 0.
template <int NO, int NC, int SLOTS, bool MODE0, bool F32>
__global__ void __launch_bounds__(kThreads) k_mttkrp_narrow(const MttkrpArgs a) {
  using TT = typename std::conditional<F32, float, double>::type;
  const TT* __restrict__ T = static_cast<const TT*>(a.T);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int ldc = a.ldc;
  // walked modes: mode 0 excluded always, and the output mode; for MODE0
  // they are the other modes 0..NO-1 of the arguments (ascending, mode 1
  // first); otherwise the other modes except the first (mode 0)
  constexpr int NW = MODE0 ? NO : NO - 1;
  const int wofs = MODE0 ? 0 : 1;
  int32_t wdim[NW > 0 ? NW : 1];
  int64_t wstride[NW > 0 ? NW : 1];
  const double* wU[NW > 0 ? NW : 1];
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    wdim[w] = a.odim[w + wofs];
    wstride[w] = a.ostride[w + wofs];
    wU[w] = a.oU[w + wofs];
  }
  const int I0 = MODE0 ? a.M : a.odim[0];

  double acc[SLOTS][NC];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[s][c] = 0.0;

  // uniform Khatri-Rao factor of the fiber at the walker's position,
  // highest mode first (the order of Eq. (1))
  auto kr = [&](const FiberWalk<NW>& fw, double (&h)[NC]) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < NC; ++c) h[c] = 1.0;
#pragma unroll
    for (int w = NW - 1; w >= 0; --w) {
      const double* row = wU[w] + (int64_t)fw.idx[w] * ldc;
#pragma unroll
      for (int c = 0; c < NC; ++c) h[c] = (w == NW - 1) ? row[c] : h[c] * row[c];
    }
  };
  auto toff = [&](const FiberWalk<NW>& fw) __attribute__((always_inline)) {
    int64_t o = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) o += (int64_t)fw.idx[w] * wstride[w];
    return o;
  };

  if constexpr (MODE0) {
    // block = one K chunk (fibers [kbeg, kend)); wavefront w takes fibers
    // kbeg + w, kbeg + w + 4, ...; lanes and slots are the rows i
    const int split = blockIdx.x;
    const int64_t kbeg = (int64_t)split * a.kchunk;
    const int64_t kend = min(kbeg + a.kchunk, a.J);
    FiberWalk<NW> fw;
    fw.init(wdim, kbeg + wave);
    // batches of UF fibers: every load of a batch is issued before its
    // products, so a wavefront has UF fibers' loads in flight at once
    for (int64_t f0 = kbeg + wave; f0 < kend; f0 += (int64_t)kWaves * UF) {
      TT tv[UF][SLOTS];
      int64_t base[UF];
      bool fok[UF];
      FiberWalk<NW> fb = fw;
#pragma unroll
      for (int u = 0; u < UF; ++u) {
        // fibers past the chunk and lanes past I_0 load from offset 0 (in
        // bounds) and are masked afterwards; the walker is only read in range
        fok[u] = f0 + (int64_t)kWaves * u < kend;
        base[u] = fok[u] ? toff(fb) : 0;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
          const int i = lane + 64 * s;
          const bool ok = fok[u] && i < I0;
          const TT x = T[ok ? base[u] + i : 0];
          tv[u][s] = ok ? x : (TT)0;
        }
        if (fok[u]) fb.advance(wdim, kWaves);
      }
#pragma unroll
      for (int u = 0; u < UF; ++u) {
        if (fok[u]) {   // uniform
          double h[NC];
          kr(fw, h);
#pragma unroll
          for (int s = 0; s < SLOTS; ++s)
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[s][c] += (double)tv[u][s] * h[c];
          fw.advance(wdim, kWaves);
        }
      }
    }
    // the four wavefronts' sums, in wavefront order
    __shared__ double red[kWaves][64][NC + 1];
    double* out = a.partial + (int64_t)split * a.M * ldc;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
#pragma unroll
      for (int c = 0; c < NC; ++c) red[wave][lane][c] = acc[s][c];
      __syncthreads();
      const int i = lane + 64 * s;
      if (wave == 0 && i < a.M) {
        for (int c = 0; c < ldc; ++c) {
          double v = 0.0;
          if (c < NC) {
            v = red[0][lane][c];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) v += red[w][lane][c];
          }
          out[(int64_t)i * ldc + c] = v;
        }
      }
      __syncthreads();
    }
  } else {
    // block = 4 output rows (a wavefront each) x one K chunk of whole
    // fibers; lanes and slots are k_0
    const int rtiles = (a.M + kWaves - 1) / kWaves;
    const int rt = blockIdx.x % rtiles;
    const int split = blockIdx.x / rtiles;
    const int r = rt * kWaves + wave;
    const bool rok = r < a.M;
    const int64_t fbeg = (int64_t)split * (a.kchunk / I0);
    const int64_t fend = min(fbeg + a.kchunk / I0, a.J / I0);
    FiberWalk<NW> fw;
    fw.init(wdim, fbeg);
    const int64_t rbase = (int64_t)(rok ? r : 0) * a.stride_n;
    for (int64_t f0 = fbeg; f0 < fend; f0 += UF) {
      TT tv[UF][SLOTS];
      FiberWalk<NW> fb = fw;
      bool fok[UF];
#pragma unroll
      for (int u = 0; u < UF; ++u) {
        // as for mode 0: clamped offsets, masked values, walker in range
        fok[u] = f0 + u < fend;
        const int64_t base = fok[u] ? rbase + toff(fb) : 0;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
          const int k0 = lane + 64 * s;
          const bool ok = fok[u] && k0 < I0;
          const TT x = T[ok ? base + k0 : 0];
          tv[u][s] = ok ? x : (TT)0;
        }
        if (fok[u]) fb.advance(wdim, 1);
      }
#pragma unroll
      for (int u = 0; u < UF; ++u) {
        if (!fok[u]) continue;   // uniform
        double h[NC];
        kr(fw, h);
#pragma unroll
        for (int s = 0; s < SLOTS; ++s)
#pragma unroll
          for (int c = 0; c < NC; ++c) acc[s][c] += (double)tv[u][s] * h[c];
        fw.advance(wdim, 1);
      }
    }
    // U_0 once per lane, then the lanes in a fixed butterfly order
    double v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = 0.0;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int k0 = lane + 64 * s;
      const double* u0 = a.oU[0] + (int64_t)(k0 < I0 ? k0 : 0) * ldc;
#pragma unroll
      for (int c = 0; c < NC; ++c) v[c] += (k0 < I0 ? u0[c] : 0.0) * acc[s][c];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double x = v[c];
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m);
      v[c] = x;
    }
    if (rok && lane < ldc) {
      double o = 0.0;
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (lane == c) o = v[c];
      a.partial[(int64_t)split * a.M * ldc + (int64_t)r * ldc + lane] = o;
    }
  }
}

template <int NO, int NC, int SLOTS, bool F32>
hipError_t launch_nar4(const MttkrpArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const bool mode0 = a.stride_n == 1;
  const int rtiles = (a.M + kWaves - 1) / kWaves;
  const dim3 grid(mode0 ? a.splits : rtiles * a.splits), block(kThreads);
  auto go = [&](auto kernel) {
    if (e0 || e1)
      hipExtLaunchKernelGGL(kernel, grid, block, 0, s, e0, e1, 0, a);
    else
      hipLaunchKernelGGL(kernel, grid, block, 0, s, a);
  };
  if (mode0)
    go(k_mttkrp_narrow<NO, NC, SLOTS, true, F32>);
  else
    go(k_mttkrp_narrow<NO, NC, SLOTS, false, F32>);
  return hipGetLastError();
}

template <int NO>
hipError_t launch_nar3(const MttkrpArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const int I0 = a.stride_n == 1 ? a.M : a.odim[0];
  const int slots = (I0 + 63) / 64;
  const bool nc8 = a.ncols <= 8;
  const bool f32 = a.t_is_f32 != 0;
#define JKC_NAR(SL, NC)                                                               \
  return f32 ? launch_nar4<NO, NC, SL, true>(a, s, e0, e1) : launch_nar4<NO, NC, SL, false>(a, s, e0, e1)
  if (slots <= 1) {
    if (nc8) JKC_NAR(1, 8);
    JKC_NAR(1, 16);
  }
  if (slots <= 2) {
    if (nc8) JKC_NAR(2, 8);
    JKC_NAR(2, 16);
  }
  if (slots <= 4 && nc8) JKC_NAR(4, 8);
#undef JKC_NAR
  return hipErrorInvalidValue;
}

hipError_t launch_narrow(const MttkrpArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (a.ldc != 16 || a.ntiles != 1) return hipErrorInvalidValue;
  const int I0 = a.stride_n == 1 ? a.M : a.odim[0];
  if (!narrow_supports(I0, a.ncols)) return hipErrorInvalidValue;
  if (a.stride_n != 1 && a.kchunk % I0 != 0) return hipErrorInvalidValue;
  switch (a.nother) {
    case 1: return launch_nar3<1>(a, s, e0, e1);
    case 2: return launch_nar3<2>(a, s, e0, e1);
    case 3: return launch_nar3<3>(a, s, e0, e1);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool narrow_supports(int I0, int ncols) {
  const int slots = (I0 + 63) / 64;
  return ncols <= 16 && (slots <= 2 || (slots <= 4 && ncols <= 8));
}

const MttkrpVariant& mttkrp_narrow_variant() {
  // wm = wn = 1, one 16-column tile, 4 output rows per block (modes > 0),
  // instruction family kNarrowInstr (vector ALUs)
  static const MttkrpVariant v = {1, 1, 1, 1, 16, &launch_narrow, kNarrowInstr};
  return v;
}

}  // namespace jkc
