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
//              (lanes are the output rows);
//   mode n>0:  M_n(r, c) = sum_{k_0} U_0(k_0, c) sum_f T(k_0, r, f) h_f(c),
//              h_f = prod_{m != 0, n} U_m(k_m(f), c)
//              (U_0 is applied once per lane after the fiber sum, then the
//              lanes are summed in a fixed butterfly).
// Each wavefront takes a run of at most UF consecutive fibers and issues all
// of their loads before its first product (one round trip to memory per
// wavefront; the grid keeps the chip's loads in flight).  A block is a run
// of wavefronts over consecutive fibers: for modes n > 0 all of them belong
// to one output row, so a row whose fibers fit one block (at most 16 x UF
// for three-way tensors) is summed inside the block and written finished; otherwise (mode 0, whose
// rows are the lanes, and long rows) the blocks write split-K partials that
// a short full-chip pass adds in ascending chunk order.  Every sum runs in a
// fixed order, so the result is bitwise repeatable.
#include <type_traits>

#include <hip/hip_ext.h>

#include "jkc_internal.hpp"
#include "wave_ops.hpp"

namespace jkc {

namespace {

// Wavefronts per block: 16 for modes n > 0 of three-way tensors; 8 where a
// second accumulator set (the factored inner sums) or mode 0's per-row block
// sum needs the registers or the LDS of a 512-thread block.
constexpr int max_waves(bool mode0, int nw) { return (mode0 || nw >= 2) ? 8 : 16; }
constexpr int kMaxWavesAll = 16;

// fibers per wavefront for NC columns and SLOTS lane slots (register budget:
// loads in flight plus accumulators)
constexpr int fibers_per_wave(int nc, int slots) { return nc * slots > 16 ? 4 : 16; }

int slots_for(int I0) { return (I0 + 63) / 64; }
int nc_for(int ncols) { return ncols <= 8 ? 8 : 16; }

// Row i of column c's model is left out (padding columns own no rows).
__device__ inline bool left_out_row(const LeftOut& lo, int64_t i, int c) {
  const int k = lo.colmodel[c];
  return k >= 0 && lo.lomask[i * lo.K + k] != 0;
}

// Position of a fiber among the walked modes (ascending, lowest fastest):
// each mode's index, the tensor offset of the fiber's first element and the
// walked modes' factor rows, all advanced incrementally (wavefront uniform,
// so they live in scalar registers).
template <int NW>
struct FiberPos {
  static constexpr int K = NW > 0 ? NW : 1;
  uint32_t idx[K];
  int64_t off;
  const double* row[K];
  // q below the product of the dims (the highest index takes no modulo)
  __device__ void init(const int32_t* dim, const int64_t* stride, const double* const* U, int ldc,
                       uint32_t q) {
    off = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      if (w + 1 < NW) {
        idx[w] = q % (uint32_t)dim[w];
        q /= (uint32_t)dim[w];
      } else {
        idx[w] = q;
      }
      off += (int64_t)idx[w] * stride[w];
      row[w] = U[w] + (int64_t)idx[w] * ldc;
    }
  }
  __device__ void advance(const int32_t* dim, const int64_t* stride, const double* const* U,
                          int ldc) {
    if constexpr (NW > 0) {
      ++idx[0];
      off += stride[0];
      row[0] += ldc;
#pragma unroll
      for (int w = 0; w + 1 < NW; ++w) {
        if (idx[w] >= (uint32_t)dim[w]) {
          idx[w] = 0;
          off += stride[w + 1] - (int64_t)dim[w] * stride[w];
          row[w] = U[w];
          ++idx[w + 1];
          row[w + 1] += ldc;
        }
      }
    }
  }
};

// NO: other modes of the output mode (N - 1); NC: columns computed (the
// rest of the 16-column pitch are zero padding); SLOTS: lanes x slots cover
// I_0; MODE0: the output mode is mode 0.  Block: blockDim.x / 64 wavefronts
// over consecutive fibers; grid: splits (mode 0) or M x splits (x: the
// output row, y: the chunk).
template <int NO, int NC, int SLOTS, bool MODE0, bool F32>
__global__ void __launch_bounds__(64 * max_waves(MODE0, MODE0 ? NO : NO - 1))
k_mttkrp_narrow(const MttkrpArgs a) {
  using TT = typename std::conditional<F32, float, double>::type;
  constexpr int UF = fibers_per_wave(NC, SLOTS);
  const TT* __restrict__ T = static_cast<const TT*>(a.T);
  const int lane = threadIdx.x & 63;
  // wavefront index as a scalar: everything derived from it (fiber walk,
  // Khatri-Rao rows) stays in scalar registers and scalar loads
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nwaves = blockDim.x >> 6;
  const int ldc = a.ldc;
  // walked modes: for MODE0 the other modes 0..NO-1 of the arguments
  // (ascending, mode 1 first); otherwise the other modes except mode 0
  constexpr int NW = MODE0 ? NO : NO - 1;
  constexpr int wofs = MODE0 ? 0 : 1;
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
  // fibers: all of them (mode 0) or those of one output row (n > 0), fewer
  // than 2^31 (checked by the launcher); a block's chunk of kcf fibers, this
  // wavefront's run [f0, f0 + nf)
  const uint32_t nfib = (uint32_t)a.nfib;
  const uint32_t kcf = (uint32_t)a.kcf;
  const int r = MODE0 ? 0 : (int)blockIdx.x;
  const int split = MODE0 ? (int)blockIdx.x : (int)blockIdx.y;
  const uint32_t cend = min((uint32_t)(split + 1) * kcf, nfib);
  const uint32_t f0 = min((uint32_t)split * kcf + (uint32_t)(wave * UF), cend);
  const int nf = (int)min((uint32_t)UF, cend - f0);
  const TT* __restrict__ Tr = T + (MODE0 ? 0 : (int64_t)r * a.stride_n);

  // every load of the run first: a scalar fiber pointer plus the lane's
  // offset.  Lanes past I_0 (only in the last slot) read the fiber's first
  // element: for mode 0 their rows are never written, for n > 0 they are
  // masked to 0 where the products use them (a mask here, inside the
  // fiber's branch, would make each load wait for its data).
  // modes n > 0: U_0 staged in LDS by the block (rows past I_0 zero), its
  // first 2 x blockDim entries loaded before the tensor so that the LDS
  // stores below wait for these loads only
  constexpr int kU0 = MODE0 ? 1 : SLOTS * 64 * NC;
  __shared__ double u0s[kU0];
  [[maybe_unused]] double u0v[2];
  if constexpr (!MODE0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = threadIdx.x + q * blockDim.x;
      const int k0 = e / NC, c = e % NC;
      u0v[q] = (e < kU0 && k0 < I0) ? a.oU[0][(int64_t)k0 * ldc + c] : 0.0;
    }
  }
  FiberPos<NW> start;
  start.init(wdim, wstride, wU, ldc, nf > 0 ? f0 : 0);
  TT tv[UF][SLOTS];
  {
    FiberPos<NW> fp = start;
#pragma unroll
    for (int u = 0; u < UF; ++u) {
      // unconditional (past the run: the tensor's first elements, unused),
      // so that each product waits for its own loads only
      const TT* p = u < nf ? Tr + fp.off : T;
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        const int i = lane + 64 * s;
        tv[u][s] = p[(s + 1 < SLOTS || i < I0) ? i : 0];
      }
      if (u + 1 < nf) fp.advance(wdim, wstride, wU, ldc);
    }
  }
  if constexpr (!MODE0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = threadIdx.x + q * blockDim.x;
      if (e < kU0) u0s[e] = u0v[q];
    }
    for (int e = threadIdx.x + 2 * blockDim.x; e < kU0; e += blockDim.x) {   // small blocks
      const int k0 = e / NC, c = e % NC;
      u0s[e] = k0 < I0 ? a.oU[0][(int64_t)k0 * ldc + c] : 0.0;
    }
  }
  // a fiber's value in slot s, masked past I_0 for modes n > 0
  const bool last_ok = MODE0 || lane + 64 * (SLOTS - 1) < I0;
  auto val = [&](int u, int s) __attribute__((always_inline)) {
    const double x = (double)tv[u][s];
    return (s + 1 < SLOTS || last_ok) ? x : 0.0;
  };
  // the products, fiber by fiber as their data arrive.  With two or more
  // walked modes the lowest one's factor is applied per fiber into inner
  // sums, and the product of the higher modes' rows (highest first, the
  // order of Eq. (1)) once per run of equal higher indices
  double acc[SLOTS][NC];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[s][c] = 0.0;
  {
    FiberPos<NW> fp = start;
    [[maybe_unused]] double ain[NW >= 2 ? SLOTS : 1][NW >= 2 ? NC : 1];
    if constexpr (NW >= 2) {
#pragma unroll
      for (int s = 0; s < SLOTS; ++s)
#pragma unroll
        for (int c = 0; c < NC; ++c) ain[s][c] = 0.0;
    }
#pragma unroll
    for (int u = 0; u < UF; ++u) {
      if (u < nf) {   // uniform
        if constexpr (NW == 0) {
#pragma unroll
          for (int s = 0; s < SLOTS; ++s)
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[s][c] += val(u, s);
        } else if constexpr (NW == 1) {
          const double* r0 = fp.row[0];
#pragma unroll
          for (int s = 0; s < SLOTS; ++s)
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[s][c] += val(u, s) * r0[c];
        } else {
          const double* r0 = fp.row[0];
#pragma unroll
          for (int s = 0; s < SLOTS; ++s)
#pragma unroll
            for (int c = 0; c < NC; ++c) ain[s][c] += val(u, s) * r0[c];
          // the higher indices change after this fiber, or the run ends
          if (u + 1 == nf || fp.idx[0] + 1 == (uint32_t)wdim[0]) {   // uniform
            double hh[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) hh[c] = fp.row[NW - 1][c];
#pragma unroll
            for (int w = NW - 2; w >= 1; --w)
#pragma unroll
              for (int c = 0; c < NC; ++c) hh[c] *= fp.row[w][c];
#pragma unroll
            for (int s = 0; s < SLOTS; ++s)
#pragma unroll
              for (int c = 0; c < NC; ++c) {
                acc[s][c] += hh[c] * ain[s][c];
                ain[s][c] = 0.0;
              }
          }
        }
        if (u + 1 < nf) fp.advance(wdim, wstride, wU, ldc);
      }
    }
  }

  if constexpr (MODE0) {
    // the block's wavefronts summed in wavefront order, one slot of rows at
    // a time; the partial of this chunk written by the whole block (the
    // zero padding columns only when a separate reduction reads all ldc)
    __shared__ double red[max_waves(true, NW)][64][NC + 1];
    double* out = a.partial + (int64_t)split * a.M * ldc;
    const int wc = a.fin_out ? NC : ldc;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
#pragma unroll
      for (int c = 0; c < NC; ++c) red[wave][lane][c] = acc[s][c];
      __syncthreads();
      for (int e = threadIdx.x; e < 64 * wc; e += blockDim.x) {
        const int l = e / wc, c = e % wc;
        const int i = l + 64 * s;
        if (i < a.M) {
          double v = 0.0;
          if (c < NC) {
            v = red[0][l][c];
            for (int w = 1; w < nwaves; ++w) v += red[w][l][c];
          }
          out[(int64_t)i * ldc + c] = v;
        }
      }
      __syncthreads();
    }
  } else {
    // U_0 once per lane (from LDS; zero rows past I_0), then the lanes in
    // the fixed order of wave_sum (every lane ends with the wavefront's sums)
    __syncthreads();
    double v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = 0.0;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const double* u0 = u0s + (lane + 64 * s) * NC;
#pragma unroll
      for (int c = 0; c < NC; ++c) v[c] += u0[c] * acc[s][c];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = wave_sum(v[c]);
    // the block's wavefronts in wavefront order
    __shared__ double red[kMaxWavesAll][NC];
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < NC; ++c) red[wave][c] = v[c];
    }
    __syncthreads();
    const int c = threadIdx.x;
    if (c < ldc) {
      double o = 0.0;
      if (c < NC) {
        o = red[0][c];
        for (int w = 1; w < nwaves; ++w) o += red[w][c];
      }
      if (a.fin_out && a.splits == 1) {
        // the row is finished: reduced output, Case I rows cleared
        if (c < a.fin_ncols) {
          if (c >= a.ncols || (a.fin_zero && left_out_row(a.fin_lo, r, c))) o = 0.0;
          a.fin_out[(int64_t)r * a.fin_ldo + c] = o;
        }
      } else {
        a.partial[((int64_t)split * a.M + r) * ldc + c] = o;
      }
    }
  }
}

// Reduced product from the narrow kernel's split-K partials: a block covers
// kFinElems consecutive elements (i, c) of the M x fin_ncols output; its
// threads are kFinElems elements x kFinParts contiguous shares of the
// chunks, each share summed in ascending order, then the shares added in
// ascending order (a fixed order).
constexpr int kFinElems = 16;
constexpr int kFinParts = 64;
__global__ void __launch_bounds__(kFinElems * kFinParts) k_narrow_finish(const MttkrpArgs a) {
  __shared__ double part[kFinParts][kFinElems];
  const int t = threadIdx.x;
  const int el = t % kFinElems, q = t / kFinElems;
  const int64_t n = (int64_t)a.M * a.fin_ncols;
  const int64_t e = (int64_t)blockIdx.x * kFinElems + el;
  const bool ok = e < n;
  const int64_t i = ok ? e / a.fin_ncols : 0;
  const int c = ok ? (int)(e % a.fin_ncols) : 0;
  const int per = (a.splits + kFinParts - 1) / kFinParts;
  const int sb = min(a.splits, q * per), se = min(a.splits, sb + per);
  const int64_t plane = (int64_t)a.M * a.ldc;
  double s = 0.0;
  if (ok && c < a.ncols) {
    const double* src = a.partial + i * a.ldc + c;
    constexpr int kBatch = 8;
    int sp = sb;
    for (; sp + kBatch <= se; sp += kBatch) {
      double v[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) v[u] = src[(int64_t)(sp + u) * plane];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) s += v[u];
    }
    for (; sp < se; ++sp) s += src[(int64_t)sp * plane];
  }
  part[q][el] = s;
  __syncthreads();
  if (q == 0 && ok) {
    double o = part[0][el];
    for (int g = 1; g < kFinParts; ++g) o += part[g][el];
    if (a.fin_zero && left_out_row(a.fin_lo, i, c)) o = 0.0;
    a.fin_out[i * a.fin_ldo + c] = o;
  }
}

template <int NO, int NC, int SLOTS, bool F32>
hipError_t launch_nar4(const MttkrpArgs& args, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  constexpr int UF = fibers_per_wave(NC, SLOTS);
  MttkrpArgs a = args;
  const bool mode0 = a.stride_n == 1;
  const int I0 = mode0 ? a.M : a.odim[0];
  const int64_t nfib = mode0 ? a.J : a.J / I0;
  const int64_t kcf = mode0 ? a.kchunk : a.kchunk / I0;
  const int64_t waves = (kcf + UF - 1) / UF;
  if (waves < 1 || waves > max_waves(mode0, mode0 ? NO : NO - 1)) return hipErrorInvalidValue;
  if (nfib < 1 || nfib >= (int64_t(1) << 31) || (int64_t)a.splits * kcf < nfib) return hipErrorInvalidValue;
  if (!mode0 && a.splits > 65535) return hipErrorInvalidValue;
  a.nfib = (int32_t)nfib;
  a.kcf = (int32_t)kcf;
  const dim3 grid = mode0 ? dim3((unsigned)a.splits) : dim3((unsigned)a.M, (unsigned)a.splits);
  const dim3 block((unsigned)(64 * waves));
  // a finishing pass follows when the output is asked for and the blocks
  // leave partials: it stamps the stop event then
  const bool fin = a.fin_out && (mode0 || a.splits > 1);
  auto go = [&](auto kernel, hipEvent_t stop) {
    if (e0 || stop)
      hipExtLaunchKernelGGL(kernel, grid, block, 0, s, e0, stop, 0, a);
    else
      hipLaunchKernelGGL(kernel, grid, block, 0, s, a);
  };
  if (mode0)
    go(k_mttkrp_narrow<NO, NC, SLOTS, true, F32>, fin ? nullptr : e1);
  else
    go(k_mttkrp_narrow<NO, NC, SLOTS, false, F32>, fin ? nullptr : e1);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess || !fin) return err;
  const dim3 fgrid((unsigned)(((int64_t)a.M * a.fin_ncols + kFinElems - 1) / kFinElems));
  const dim3 fblock(kFinElems * kFinParts);
  if (e1)
    hipExtLaunchKernelGGL(k_narrow_finish, fgrid, fblock, 0, s, nullptr, e1, 0, a);
  else
    hipLaunchKernelGGL(k_narrow_finish, fgrid, fblock, 0, s, a);
  return hipGetLastError();
}

template <int NO>
hipError_t launch_nar3(const MttkrpArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const int I0 = a.stride_n == 1 ? a.M : a.odim[0];
  const int slots = slots_for(I0);
  const bool nc8 = nc_for(a.ncols) == 8;
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
  if (a.fin_out && (a.fin_ncols < 1 || a.fin_ncols > a.ldc || a.fin_ldo < a.fin_ncols))
    return hipErrorInvalidValue;
  switch (a.nother) {
    case 1: return launch_nar3<1>(a, s, e0, e1);
    case 2: return launch_nar3<2>(a, s, e0, e1);
    case 3: return launch_nar3<3>(a, s, e0, e1);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool narrow_supports(int I0, int ncols) {
  const int slots = slots_for(I0);
  return ncols <= 16 && (slots <= 2 || (slots <= 4 && ncols <= 8));
}

int64_t narrow_max_chunk_fibers(int I0, int ncols, bool mode0, int order) {
  return (int64_t)max_waves(mode0, mode0 ? order - 1 : order - 2) *
         fibers_per_wave(nc_for(ncols), slots_for(I0));
}

const MttkrpVariant& mttkrp_narrow_variant() {
  // wm = wn = 1, one 16-column tile, 1 output row per block (modes > 0),
  // instruction family kNarrowInstr (vector ALUs)
  static const MttkrpVariant v = {1, 1, 1, 1, 16, &launch_narrow, kNarrowInstr};
  return v;
}

}  // namespace jkc
