// Jackknife post-processing (Alg. 2, the permutation and scale adjustment
// of every fitted submodel and the standard deviation of the factor
// matrices over the submodels), for a set of `count` models of one rank R
// whose columns are contiguous in the multi-factors, against a reference
// model of the same rank (normally the model fitted to all of T).
//
// Matching: the congruence of submodel component r with reference component
// s is the product over the non-sampled modes, in ascending mode order, of
// the cosines of their loading vectors; the assignment maximising the sum
// of absolute congruences is solved exactly (shortest augmenting paths with
// dual potentials, O(R^3), one thread per model: R <= 32).
// Scale adjustment: every non-sampled loading vector is scaled to unit norm
// with the sign that makes its inner product with the matched reference
// vector non-negative; the sampled mode absorbs scales and signs and gets no
// deviation (Alg. 2 reports the other modes).
// Deviation: S = sqrt((count - 1) / count * sum_j (theta_j - mean)^2) per
// element, sums in ascending model order (bitwise repeatable).
#include <cmath>

#include "jkc_internal.hpp"

namespace jkc {

namespace {

constexpr int kThreads = 256;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Minimum-cost perfect assignment of an n x n cost matrix (rows: submodel
// components, columns: reference components) by successive shortest
// augmenting paths with row/column potentials.  col_row[j] receives the row
// assigned to column j.  Single thread; every cost must be finite, which
// bounds each augmentation to n + 1 column scans.
__device__ void assign_min_cost(const double (*cost)[kMaxRank + 1], int n, double* u, double* v,
                                int* colrow, int* way, double* minv, int* used, int* col_row) {
  const double kInf = 1e300;
  for (int j = 0; j <= n; ++j) {
    u[j] = 0.0;
    v[j] = 0.0;
    colrow[j] = 0;
    way[j] = 0;
  }
  for (int i = 1; i <= n; ++i) {
    colrow[0] = i;
    int j0 = 0;
    for (int j = 0; j <= n; ++j) {
      minv[j] = kInf;
      used[j] = 0;
    }
    for (int guard = 0; guard <= n; ++guard) {
      used[j0] = 1;
      const int i0 = colrow[j0];
      double delta = kInf;
      int j1 = 0;
      for (int j = 1; j <= n; ++j) {
        if (used[j]) continue;
        const double cur = cost[i0 - 1][j - 1] - u[i0] - v[j];
        if (cur < minv[j]) {
          minv[j] = cur;
          way[j] = j0;
        }
        if (minv[j] < delta) {
          delta = minv[j];
          j1 = j;
        }
      }
      for (int j = 0; j <= n; ++j) {
        if (used[j]) {
          u[colrow[j]] += delta;
          v[j] -= delta;
        } else {
          minv[j] -= delta;
        }
      }
      j0 = j1;
      if (colrow[j0] == 0) break;
    }
    // augment along the path back to column 0
    for (int guard = 0; guard <= n && j0 != 0; ++guard) {
      const int j1 = way[j0];
      colrow[j0] = colrow[j1];
      j0 = j1;
    }
  }
  // a column left unassigned (impossible with finite costs) keeps its own
  // index, so every later access stays inside the model's columns
  for (int j = 1; j <= n; ++j) {
    const int r = colrow[j] - 1;
    col_row[j - 1] = (r >= 0 && r < n) ? r : j - 1;
  }
}

__global__ void __launch_bounds__(kThreads) k_jk_match(const JkArgs a) {
  __shared__ double D[kMaxOrder][kMaxRank][kMaxRank + 1];
  __shared__ double nk[kMaxOrder][kMaxRank], nr[kMaxOrder][kMaxRank];
  __shared__ double cost[kMaxRank][kMaxRank + 1];
  __shared__ double hu[kMaxRank + 1], hv[kMaxRank + 1], hminv[kMaxRank + 1];
  __shared__ int hcolrow[kMaxRank + 1], hway[kMaxRank + 1], hused[kMaxRank + 1];
  __shared__ int match[kMaxRank];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, nw = blockDim.x >> 6;
  const int R = a.R;
  const int j = blockIdx.x;
  const int off = a.first_off + j * R;
  // inner products and squared norms, one wavefront per task
  for (int n = 0; n < a.N; ++n) {
    if (n == a.nhat) continue;
    const double* U = a.U[n];
    const int I = a.dims[n];
    const int tasks = R * R + 2 * R;
    for (int task = wave; task < tasks; task += nw) {
      int c0, c1;
      if (task < R * R) {
        c0 = off + task / R;
        c1 = a.ref_off + task % R;
      } else if (task < R * R + R) {
        c0 = c1 = off + (task - R * R);
      } else {
        c0 = c1 = a.ref_off + (task - R * R - R);
      }
      double acc = 0.0;
      for (int i = lane; i < I; i += 64) acc += U[(int64_t)i * a.ldc + c0] * U[(int64_t)i * a.ldc + c1];
      acc = wave_sum(acc);
      if (lane == 0) {
        if (task < R * R) D[n][task / R][task % R] = acc;
        else if (task < R * R + R) nk[n][task - R * R] = acc;
        else nr[n][task - R * R - R] = acc;
      }
    }
  }
  __syncthreads();
  // congruences (product over the non-sampled modes, ascending) -> costs
  for (int e = t; e < R * R; e += blockDim.x) {
    const int r = e / R, s = e % R;
    double phi = 1.0;
    for (int n = 0; n < a.N; ++n) {
      if (n == a.nhat) continue;
      const double den = sqrt(nk[n][r]) * sqrt(nr[n][s]);
      phi *= den > 0.0 ? D[n][r][s] / den : 0.0;
    }
    cost[r][s] = isfinite(phi) ? -fabs(phi) : 0.0;
  }
  __syncthreads();
  if (t == 0) assign_min_cost(cost, R, hu, hv, hcolrow, hway, hminv, hused, match);
  __syncthreads();
  // permutation and signed inverse norms of the matched columns
  for (int e = t; e < a.N * R; e += blockDim.x) {
    const int n = e / R, s = e % R;
    const int r = match[s];
    if (n == 0) a.perm[off + s] = r;
    double sc = 0.0;
    if (n != a.nhat && nk[n][r] > 0.0) {
      const double inv = 1.0 / sqrt(nk[n][r]);
      sc = D[n][r][s] < 0.0 ? -inv : inv;
    }
    a.scale[(int64_t)n * a.ldc + off + s] = sc;
  }
}

__global__ void __launch_bounds__(kThreads) k_jk_std(const JkArgs a, int n) {
  const double* U = a.U[n];
  const int R = a.R;
  const int64_t total = (int64_t)a.dims[n] * R;
  const double* sc = a.scale + (int64_t)n * a.ldc;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / R;
    const int s = (int)(e % R);
    const double* row = U + i * a.ldc;
    double sum = 0.0;
    for (int jj = 0; jj < a.count; ++jj) {
      const int c = a.first_off + jj * R;
      sum += row[c + a.perm[c + s]] * sc[c + s];
    }
    const double mean = sum / a.count;
    double ss = 0.0;
    for (int jj = 0; jj < a.count; ++jj) {
      const int c = a.first_off + jj * R;
      const double d = row[c + a.perm[c + s]] * sc[c + s] - mean;
      ss += d * d;
    }
    a.std_out[n][e] = sqrt((double)(a.count - 1) / a.count * ss);
  }
}

// sign[n * cols + c] = +1 / -1 from the signed inverse norms (+1 for a zero
// column and for the sampled mode)
__global__ void k_jk_signs(const double* scale, int32_t ldc, int32_t N, int32_t first_off,
                           int32_t cols, double* sign) {
  const int64_t total = (int64_t)N * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = e / cols;
    const int c = (int)(e % cols);
    sign[e] = scale[n * ldc + first_off + c] < 0.0 ? -1.0 : 1.0;
  }
}

}  // namespace

hipError_t launch_jk_signs(const double* scale, int32_t ldc, int32_t N, int32_t first_off,
                           int32_t cols, double* sign, hipStream_t s) {
  const int64_t total = (int64_t)N * cols;
  int64_t blocks = (total + kThreads - 1) / kThreads;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(k_jk_signs, dim3((unsigned)blocks), dim3(kThreads), 0, s, scale, ldc, N,
                     first_off, cols, sign);
  return hipGetLastError();
}

hipError_t launch_jk(const JkArgs& a, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_jk_match, dim3(a.count), dim3(kThreads), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int n = 0; n < a.N; ++n) {
    if (n == a.nhat) continue;
    const int64_t total = (int64_t)a.dims[n] * a.R;
    int64_t blocks = (total + kThreads - 1) / kThreads;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_jk_std, dim3((unsigned)blocks), dim3(kThreads), 0, s, a, n);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace jkc
