// Shared partial contraction of a 3-way sweep: an extension beyond Alg. 3
// (which computes each mode's MTTKRP separately).  The MTTKRPs of Alg. 1
// inside the concurrent sweep are evaluated as a two-level dimension tree,
// the reuse of partial MTTKRPs of Phan et al. (the paper's reference for the
// error identity).  Modes are numbered from 0 here.  Before mode 0 of a
// sweep the tensor is contracted once with the last factor,
//   W(i, j, c) = sum_k T(i, j, k) U_2(k, c)         (all C columns at once),
// by the fused MTTKRP kernel on the two-way view of T (rows i + I_0 j,
// contraction over k), and W serves two MTTKRPs of the sweep:
//   M_0(i, c) = sum_j W(i, j, c) U_1(j, c)          (U_1 of the last sweep)
//   M_1(j, c) = sum_i W(i, j, c) U_0(i, c)          (U_0 just updated)
// U_2 changes only at the last mode, so both equal the MTTKRP of Alg. 1 up
// to rounding; mode 2 keeps the fused MTTKRP.  Case II needs nothing more
// (a model's zero rows of the sampled factor zero its terms in W or in the
// pass), and Case I is applied by the update as for the fused kernel.
//
// This file holds the pass kernel: out(o, c) = sum_{s < S} W(row(o, s), c)
// F(s, c) with row(o, s) = o ostep + s sstep (rows of W, pitch ldc).  It is
// bound by reading W once.  A block covers 64 columns (one per lane) and
// kPassOut outputs; its kPassWaves wavefronts each sum a contiguous range
// of s in ascending order, and the ranges are combined in ascending order,
// so results are bitwise repeatable.
#include <algorithm>

#include "jkc_internal.hpp"

namespace jkc {

namespace {

constexpr int kPassWaves = 8;
constexpr int kPassOut = 4;

__global__ void __launch_bounds__(64 * kPassWaves)
    k_tree_pass(const double* __restrict__ W, const double* __restrict__ F, int32_t S, int64_t ostep,
                int64_t sstep, int32_t nout, int32_t ldc, int32_t ncols, double* __restrict__ out) {
  __shared__ double part[kPassWaves][kPassOut][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  const int o0 = blockIdx.y * kPassOut;
  const int qs = (S + kPassWaves - 1) / kPassWaves;
  const int s0 = std::min(S, wave * qs), s1 = std::min(S, s0 + qs);
  double acc[kPassOut];
#pragma unroll
  for (int u = 0; u < kPassOut; ++u) acc[u] = 0.0;
  if (c < ncols) {
    const double* w[kPassOut];
#pragma unroll
    for (int u = 0; u < kPassOut; ++u)   // rows past the last output repeat it (discarded)
      w[u] = W + (int64_t)std::min(o0 + u, nout - 1) * ostep * ldc + c;
    const int64_t wstep = sstep * ldc;
    // one s per iteration (kPassOut + 1 loads in flight per wavefront): with
    // thousands of wavefronts resident this keeps the memory system busiest
    // (on the benchmark's two passes over an 82 MB W, 12.6 us per pass
    // against 12.9 with two s per iteration, 13.5 with four, 13.5 with eight)
#pragma unroll 1
    for (int s = s0; s < s1; ++s) {
      const double f = F[(int64_t)s * ldc + c];
#pragma unroll
      for (int u = 0; u < kPassOut; ++u) acc[u] += w[u][(int64_t)s * wstep] * f;
    }
  }
#pragma unroll
  for (int u = 0; u < kPassOut; ++u) part[wave][u][lane] = acc[u];
  __syncthreads();
  if (wave < kPassOut && c < ncols && o0 + wave < nout) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kPassWaves; ++q) t += part[q][wave][lane];
    out[(int64_t)(o0 + wave) * ldc + c] = t;
  }
}

}  // namespace

hipError_t launch_tree_pass(const double* W, const double* F, int32_t S, int64_t ostep, int64_t sstep,
                            int32_t nout, int32_t ldc, int32_t ncols, double* out, hipStream_t s) {
  if (nout <= 0 || ncols <= 0) return hipSuccess;
  const dim3 grid((unsigned)((ncols + 63) / 64), (unsigned)((nout + kPassOut - 1) / kPassOut));
  hipLaunchKernelGGL(k_tree_pass, grid, dim3(64 * kPassWaves), 0, s, W, F, S, ostep, sstep, nout, ldc,
                     ncols, out);
  return hipGetLastError();
}

}  // namespace jkc
