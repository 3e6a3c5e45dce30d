// All-mode MTTKRP in one pass over the tensor (3- and 4-way, float64 matrix
// cores): for factors held fixed, every mode's fused MTTKRP
//   M_n(i_n, c) = sum_{i_m, m != n} T(i) prod_{m != n} Ubar_m(i_m, c)
// (Alg. 3, MTTKRP step, for all n at the same factors -- the gradient of the
// all-at-once CP loss the paper cites in Sec. 2 needs exactly this).
//
// The tensor is read as mode-0 fibers f = (j_1, j_2[, j_3]) (contiguous in
// the column-major layout of Eq. (3)).  A tile of T (all rows i of mode 0 x
// BK fibers of one (j_2[, j_3]) slab) is staged in LDS once and feeds two
// matrix-core products:
//   X(i, c) += sum_f T(i, f) KR(f, c),  KR(f, c) = prod_{m >= 1} U_m(j_m, c)
//            -> mode 0 (the fused MTTKRP of mode 0);
//   Z(f, c)  = sum_i T(i, f) U_0(i, c)
//            -> the mode-0-contracted tensor, from which the other modes
//               follow by per-column products (multilinearity of Eq. (1)):
//   M_1(j_1, c) += Z(f, c) U_2(j_2, c) [U_3(j_3, c)]
//   M_2(j_2, c) += sum_{j_1} Z(f, c) U_1(j_1, c) [U_3(j_3, c)]
//   M_3(j_3, c) += sum_{j_1, j_2} Z(f, c) U_1(j_1, c) U_2(j_2, c)       (4-way)
// So every output costs one pass over T and 4 C P matrix-core flops in all
// (against 2 N C P for N separate MTTKRPs).
//
// Work split.  A block owns a 32-column tile and a chunk of consecutive
// last-mode indices (all fibers of those slabs), so the last mode's rows are
// complete within the block and are written directly; modes 0 .. N-2 are
// partial over chunks: their per-chunk results go to split partials that a
// fixed-order reduction sums (bitwise repeatable).  Mode-1 (and mode-2)
// accumulators live in LDS, the mode-0 accumulators in the X wavefronts'
// registers.  Of the four wavefronts, two form Z (one 16-column group each,
// contraction over all rows) and two form X (one column group each, every
// 16-row tile): both products cost I0p * 32 * BK / 2 flops per step, so the
// halves are balanced.  A step's fibers never straddle two slabs: the j_1
// range is walked in blocks of BK with the tail masked to zero.
#include <type_traits>

#include <hip/hip_ext.h>

#include "jkc_internal.hpp"

namespace jkc {

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {

constexpr int kThreads = 256;
constexpr int kBN = 32;           // columns per block (two 16-column groups)
constexpr int kXcds = 8;

// Row pitch (doubles) of the staged tensor tile, 2 (mod 32): the Z
// product's operand reads (16 lanes on 16 fibers of one row) then start on
// 16 distinct bank pairs, and the X product's (16 consecutive rows of one
// fiber) are contiguous.
__host__ __device__ inline int tile_pitch(int i0p) { return i0p + ((i0p % 32) == 0 ? 2 : 18); }

// Dynamic LDS layout (doubles), shared by the kernel and the host check.
struct AllModeLds {
  int64_t ts, u1s, hs, u0s, m1, m2, total;
  __host__ __device__ AllModeLds(int i0p, int bk, int I1, int I2, int N) {
    const int ldt = tile_pitch(i0p);
    ts = 0;                                  // [2][bk][ldt]   T tile (fiber-major)
    u1s = ts + 2 * (int64_t)bk * ldt;        // [2][bk][kBN]   U_1 rows of the step
    hs = u1s + 2 * (int64_t)bk * kBN;        // [2][2][kBN]    U_2(j_2, :), U_3(j_3, :)
    u0s = hs + 4 * kBN;                      // [i0p][kBN]     U_0 (fixed)
    m1 = u0s + (int64_t)i0p * kBN;           // [I1 padded to bk][kBN] mode-1 accumulators
    m2 = m1 + (int64_t)((I1 + bk - 1) / bk * bk) * kBN;   // [I2][kBN] mode-2 accumulators (4-way)
    total = m2 + (N == 4 ? (int64_t)I2 * kBN : 0);
  }
};

// NT: 16-row tiles of mode 0 (rows padded with zeros to NT * 16), a
// compile-time count so every accumulator of the X product stays in place.
template <int BK, int NO, bool F32, int NT>
__global__ void __launch_bounds__(kThreads) k_allmode(const AllModeArgs a) {
  extern __shared__ double lds[];
  constexpr bool FOUR = NO == 3;
  const int I0 = a.dims[0], I1 = a.dims[1], I2 = a.dims[2];
  const int I3 = FOUR ? a.dims[3] : 1;
  constexpr int i0p = NT * 16;
  const int ldt = tile_pitch(i0p);
  const AllModeLds L(i0p, BK, I1, I2, NO + 1);
  double* Ts = lds + L.ts;
  double* U1s = lds + L.u1s;
  double* Hs = lds + L.hs;
  double* U0s = lds + L.u0s;
  double* M1 = lds + L.m1;
  double* M2 = lds + L.m2;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int o16 = lane & 15;
  const int blk = lane >> 4;

  // block -> (column tile, chunk), XCD-aware: each XCD gets a contiguous
  // run of logical blocks, column tile fastest (blocks of one chunk read the
  // same slabs of T and share an L2)
  const int total = gridDim.x;
  int logical = blockIdx.x;
  const int per_xcd = total / kXcds;
  if (logical < per_xcd * kXcds) logical = (logical % kXcds) * per_xcd + logical / kXcds;
  const int ct = logical % a.ntiles;
  const int chunk = logical / a.ntiles;
  const int c0 = ct * kBN;
  const int last_dim = FOUR ? I3 : I2;
  const int e0 = chunk * a.chunk;
  const int e1 = min(e0 + a.chunk, last_dim);
  const int nj1 = (I1 + BK - 1) / BK;               // j_1 blocks per slab
  const int nslab = FOUR ? I2 : 1;                  // slabs (j_2) per last-mode index (4-way)
  const int nsteps = e1 > e0 ? (e1 - e0) * nslab * nj1 : 0;

  const int ldc = a.ldc;

  // fixed operands and accumulators
  for (int e = tid; e < i0p * kBN; e += kThreads) {
    const int i = e / kBN, c = e % kBN;
    U0s[e] = (i < I0 && c0 + c < ldc) ? a.U[0][(int64_t)i * ldc + c0 + c] : 0.0;
  }
  const int i1p = (I1 + BK - 1) / BK * BK;          // mode-1 rows padded to whole steps
  for (int e = tid; e < (FOUR ? i1p + I2 : i1p) * kBN; e += kThreads) M1[e] = 0.0;

  // step s -> (last-mode index, slab, j_1 block); loads of the next step are
  // issued before the current step computes
  constexpr int tile = i0p * BK;                    // T elements per step
  auto step_index = [&](int s, int& e, int& j2, int& jb) {
    jb = s % nj1;
    const int q = s / nj1;
    if (FOUR) {
      j2 = q % nslab;
      e = e0 + q / nslab;
    } else {
      j2 = e0 + q;
      e = j2;
    }
  };
  // registers of the step in flight: T elements (strided over threads), the
  // U_1 entries of the step and the per-column entries U_2(j_2), U_3(j_3).
  // Every load is unconditional at a clamped address and keeps its raw
  // value until the store (where masks and the float32 conversion apply),
  // so no load is waited for before the step's matrix-core work.
  using TT = typename std::conditional<F32, float, double>::type;
  constexpr int VT = (tile + kThreads - 1) / kThreads;   // T elements per thread
  constexpr int VU = (BK * kBN + kThreads - 1) / kThreads;
  TT rt[2][VT];
  // this thread's tile elements, fixed for the launch: byte offset of
  // (i, f) within the step's fibers, and the fiber f (past the tile or
  // past I0: f = BK, never valid).  The tensor is read through a buffer
  // resource: offsets of masked elements point past its end, and the
  // hardware range check returns zeros for them.
  uint32_t toff[VT];
  int tfib[VT];
#pragma unroll
  for (int v = 0; v < VT; ++v) {
    const int idx = tid + kThreads * v;
    const int f = idx / i0p, i = idx % i0p;
    const bool in = idx < tile && i < I0;
    toff[v] = (uint32_t)(i + I0 * f) * (uint32_t)sizeof(TT);
    tfib[v] = in ? f : BK;
  }
  constexpr int kRsrcWord3 = 0x00020000;   // raw buffer, range checked
  const __amdgpu_buffer_rsrc_t rT = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(a.T), (short)0, (int)(a.tbytes), kRsrcWord3);
  double ru1[2][VU];
  uint32_t umask[2] = {0, 0};
  double rh[2] = {0.0, 0.0};
  bool hok[2] = {false, false};
  using S0_t = std::integral_constant<int, 0>;
  using S1_t = std::integral_constant<int, 1>;
  // load step s into register stage P (a compile-time index)
  auto load = [&](auto P, int s) __attribute__((always_inline)) {
    constexpr int p = decltype(P)::value;
    int e, j2, jb;
    step_index(s < nsteps ? s : 0, e, j2, jb);
    const bool sok = s < nsteps;
    const int j3 = e;                               // 4-way: last mode index
    const int64_t slab = FOUR ? ((int64_t)j3 * I2 + j2) : (int64_t)j2;
    // uniform byte offset of the step's first fiber; fibers past I_1 (the
    // slab's tail) and steps past the chunk read zeros
    const uint32_t base = (uint32_t)I0 * (uint32_t)(jb * BK + I1 * slab) * (uint32_t)sizeof(TT);
    const int flim = sok ? I1 - jb * BK : 0;
#pragma unroll
    for (int v = 0; v < VT; ++v) {
      const uint32_t off = tfib[v] < flim ? base + toff[v] : 0x80000000u;
      if constexpr (F32)
        rt[p][v] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rT, off, 0, 0));
      else
        rt[p][v] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rT, off, 0, 0));
    }
    umask[p] = 0;
#pragma unroll
    for (int v = 0; v < VU; ++v) {
      const int idx = tid + kThreads * v;
      const int f = idx / kBN, c = idx % kBN;
      const int j1 = jb * BK + f;
      const bool ok = idx < BK * kBN && sok && j1 < I1 && c0 + c < ldc;
      ru1[p][v] = a.U[1][ok ? (int64_t)j1 * ldc + c0 + c : 0];
      umask[p] |= (uint32_t)ok << v;
    }
    // per-column entries: threads 0..31 U_2(j_2, :), 32..63 U_3(j_3, :)
    {
      const int c = tid % kBN;
      const bool third = FOUR && tid >= kBN && tid < 2 * kBN;
      hok[p] = sok && tid < (FOUR ? 2 : 1) * kBN && c0 + c < ldc;
      const double* src = third ? a.U[3] : a.U[2];
      const int64_t row = third ? j3 : j2;
      rh[p] = src[hok[p] ? row * ldc + c0 + c : 0];
    }
  };
  auto store = [&](auto P, int buf) __attribute__((always_inline)) {
    constexpr int p = decltype(P)::value;
#pragma unroll
    for (int v = 0; v < VT; ++v) {
      const int idx = tid + kThreads * v;
      if (VT * kThreads == tile || idx < tile) {
        const int f = idx / i0p, i = idx % i0p;
        Ts[(buf * BK + f) * ldt + i] = (double)rt[p][v];
      }
    }
#pragma unroll
    for (int v = 0; v < VU; ++v) {
      const int idx = tid + kThreads * v;
      if (idx < BK * kBN) U1s[(int64_t)buf * BK * kBN + idx] = ((umask[p] >> v) & 1u) ? ru1[p][v] : 0.0;
    }
    if (tid < 2 * kBN) Hs[buf * 2 * kBN + tid] = hok[p] ? rh[p] : 0.0;
  };

  const int g = wave & 1;                 // 16-column group of this wavefront
  const int cg = g * 16;
  const bool zwave = wave < 2;
  v4d acc[NT];                            // X wavefronts: one per row tile
#pragma unroll
  for (int x = 0; x < NT; ++x) acc[x] = v4d{0.0, 0.0, 0.0, 0.0};
  double mlast = 0.0;                     // Z wavefronts: last-mode sum of this lane's column

  // Pipeline (as in the split-precision kernel): at the start of step s,
  // LDS buffer s&1 holds step s, register stage (s+1)&1 step s+1 and the
  // other stage step s+2 (loads possibly in flight).  Step s computes from
  // LDS, stores step s+1 into the other buffer (last read in step s-1,
  // which every wavefront finished at the barrier ending it), synchronises,
  // and loads step s+3 into the freed stage; loads of steps past the chunk
  // read zeros and their stores are never used.
  load(S0_t{}, 0);
  store(S0_t{}, 0);
  __syncthreads();
  load(S1_t{}, 1);
  load(S0_t{}, 2);
  auto step = [&](int s, auto P) __attribute__((always_inline)) {
    const int buf = s & 1;
    int e, j2, jb;
    step_index(s, e, j2, jb);
    const double* Tb = Ts + (int64_t)buf * BK * ldt;
    const double* Ub = U1s + (int64_t)buf * BK * kBN;
    const double* Hb = Hs + buf * 2 * kBN;
    if (!zwave) {
      // X(i, c) += T(i, f) KR(f, c): A = T tile (rows i), B = KR formed from
      // the staged entries, highest mode first (the order of Eq. (1))
      const double h = FOUR ? Hb[kBN + cg + o16] * Hb[cg + o16] : Hb[cg + o16];
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        const double b = h * Ub[(kk + blk) * kBN + cg + o16];
#pragma unroll
        for (int x = 0; x < NT; ++x)
          acc[x] = __builtin_amdgcn_mfma_f64_16x16x4f64(Tb[(kk + blk) * ldt + x * 16 + o16], b, acc[x], 0, 0, 0);
      }
    } else {
      // Z(f, c) = sum_i T(i, f) U_0(i, c): A = T tile transposed (rows f),
      // contraction over every row of mode 0
      // four independent accumulation chains (rows ii mod 16 = 0, 4, 8, 12),
      // added in a fixed order
      v4d zq[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) zq[q] = v4d{0.0, 0.0, 0.0, 0.0};
      const double* Tf = Tb + (o16 < BK ? o16 : 0) * ldt + blk;
      const double amask = o16 < BK ? 1.0 : 0.0;
#pragma unroll
      for (int ii = 0; ii < i0p; ii += 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          zq[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(amask * Tf[ii + 4 * q],
                                                       U0s[(ii + 4 * q + blk) * kBN + cg + o16], zq[q], 0, 0, 0);
      }
      const v4d z = (zq[0] + zq[1]) + (zq[2] + zq[3]);
      // lane holds Z(f = 4r + blk, c = cg + o16), r = 0..3
      const int c = cg + o16;
      const double u2 = Hb[c];
      const double u3 = FOUR ? Hb[kBN + c] : 1.0;
      double s2 = 0.0, s3 = 0.0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int f = 4 * r + blk;
        if (f < BK) {
          const int j1 = jb * BK + f;                 // < i1p; z is 0 past I_1
          const double zv = z[r];
          const double u1 = Ub[f * kBN + c];
          M1[j1 * kBN + c] += FOUR ? zv * (u3 * u2) : zv * u2;   // distinct (j_1, c) per lane
          if (FOUR) {
            s2 += zv * (u3 * u1);
            s3 += zv * (u2 * u1);
          } else {
            s2 += zv * u1;
          }
        }
      }
      // sums over the step's fibers: lanes o16, o16+16, o16+32, o16+48
      s2 += __shfl_xor(s2, 16);
      s2 += __shfl_xor(s2, 32);
      if (FOUR) {
        s3 += __shfl_xor(s3, 16);
        s3 += __shfl_xor(s3, 32);
        if (blk == 0) M2[j2 * kBN + c] += s2;
        mlast += s3;
      } else {
        mlast += s2;
      }
      // the last-mode row is complete after its final step in this block
      const bool row_end = FOUR ? (jb == nj1 - 1 && j2 == nslab - 1) : (jb == nj1 - 1);
      if (row_end) {
        if (blk == 0 && c0 + c < ldc) a.out_last[(int64_t)e * ldc + c0 + c] = mlast;
        mlast = 0.0;
      }
    }
    store(P, buf ^ 1);
    __syncthreads();
    load(P, s + 3);
  };
  int s = 0;
  for (; s + 1 < nsteps; s += 2) {
    step(s, S1_t{});
    step(s + 1, S0_t{});
  }
  if (s < nsteps) step(s, S1_t{});

  // split partials of modes 0 .. N-2 for this chunk (every row; zeros where
  // the chunk contributed nothing)
  double* p0 = a.part[0] + (int64_t)chunk * I0 * ldc;
  if (!zwave) {
#pragma unroll
    for (int x = 0; x < NT; ++x)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
          const int i = x * 16 + 4 * r + blk;
          const int c = c0 + cg + o16;
          if (i < I0 && c < ldc) p0[(int64_t)i * ldc + c] = acc[x][r];
        }
  }
  double* p1 = a.part[1] + (int64_t)chunk * I1 * ldc;
  for (int e = tid; e < I1 * kBN; e += kThreads) {
    const int j = e / kBN, c = e % kBN;
    if (c0 + c < ldc) p1[(int64_t)j * ldc + c0 + c] = M1[e];
  }
  if (FOUR) {
    double* p2 = a.part[2] + (int64_t)chunk * I2 * ldc;
    for (int e = tid; e < I2 * kBN; e += kThreads) {
      const int j = e / kBN, c = e % kBN;
      if (c0 + c < ldc) p2[(int64_t)j * ldc + c0 + c] = M2[e];
    }
  }
}

template <int BK, int NO, int NT>
hipError_t launch_nt(const AllModeArgs& a, size_t lds, hipStream_t s) {
  auto go = [&](auto kernel) -> hipError_t {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kernel, dim3(a.ntiles * a.nchunks), dim3(kThreads), lds, s, a);
    return hipGetLastError();
  };
  return a.t_is_f32 ? go(k_allmode<BK, NO, true, NT>) : go(k_allmode<BK, NO, false, NT>);
}

template <int NO>
hipError_t launch_no(const AllModeArgs& a, size_t lds, hipStream_t s) {
  const int nt = a.i0p / 16;
  if (a.bk == 16) {
    switch (nt) {
      case 2: return launch_nt<16, NO, 2>(a, lds, s);
      case 4: return launch_nt<16, NO, 4>(a, lds, s);
      case 7: return launch_nt<16, NO, 7>(a, lds, s);
      case 8: return launch_nt<16, NO, 8>(a, lds, s);
      case 13: return launch_nt<16, NO, 13>(a, lds, s);
      case 16: return launch_nt<16, NO, 16>(a, lds, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (a.bk == 8) {
    if (nt == 13) return launch_nt<8, NO, 13>(a, lds, s);
    if (nt == 16) return launch_nt<8, NO, 16>(a, lds, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

int64_t allmode_lds_bytes(int i0p, int bk, int I1, int I2, int N) {
  return AllModeLds(i0p, bk, I1, I2, N).total * 8;
}

int allmode_row_tiles(int I0) {
  for (int nt : {2, 4, 7, 8, 13, 16})
    if (nt * 16 >= I0) return nt;
  return 0;
}

bool allmode_has_kernel(int nt, int bk) {
  return bk == 16 ? allmode_row_tiles(nt * 16) == nt : (bk == 8 && (nt == 13 || nt == 16));
}

hipError_t launch_allmode(const AllModeArgs& a, hipStream_t s) {
  if (a.N != 3 && a.N != 4) return hipErrorInvalidValue;
  if (a.i0p % 16 != 0 || a.i0p < a.dims[0] || !allmode_has_kernel(a.i0p / 16, a.bk))
    return hipErrorInvalidValue;
  const size_t lds = (size_t)allmode_lds_bytes(a.i0p, a.bk, a.dims[1], a.dims[2], a.N);
  return a.N == 3 ? launch_no<2>(a, lds, s) : launch_no<3>(a, lds, s);
}

}  // namespace jkc
