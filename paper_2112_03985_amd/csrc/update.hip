// Per-model batched kernels of JK-CALS: everything after the fused MTTKRP
// that stays separate for each submodel (Alg. 3, the per-p loop inside the
// mode loop, and the error step).
//
// One 256-thread block handles one model at a time and strides over the
// models in decreasing-cost order (a persistent grid), so batches of
// uneven ranks keep every block busy.  For model k of rank R (<= 32) the
// update of mode n is:
//   H = *_{m != n} G_m|k                        (Hadamard of Gramians)
//   H = L L^T                                    (Cholesky; eigen
//                                                 pseudoinverse fallback)
//   U_n|k(i,:) = M_n|k(i,:) H^{-1}  for all rows (normal equations)
//   the model's left-out rows of M (one, or d for delete-d) are taken as 0
//   when n is the sampled mode (Case I; the re-zeroing step of Alg. 3 then
//   holds automatically: 0 H^{-1} = 0)
//   lambda_r = ||U(:,r)||, U(:,r) /= lambda_r    (normalisation)
//   G_n|k = U^T U, upper triangle mirrored       (exactly symmetric)
// and after the last mode the submodel error with ||T_{-P}||^2 (Alg. 3
// error step, with the identity's Gram term read with a plus sign).
// Every reduction runs in a fixed order, so results are bitwise repeatable.
#include "jkc_internal.hpp"
#include "wave_ops.hpp"

namespace jkc {

namespace {

constexpr int kThreads = 256;
// block size of the LDS-staged update: its row phases (U = M H^{-1}, column
// norms, Gram pairs) are spread over more wavefronts
constexpr int kUpdThreads = 512;
constexpr int kLd = kMaxRank + 1;   // LDS row pitch of R x R matrices

// Orders LDS accesses of the lanes of one wavefront: a wavefront's LDS
// operations execute in issue order, so keeping the compiler from moving
// them across this point is enough (no block barrier).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cholesky H = L L^T and the columns of L^{-1} for R <= RB <= 32, by the 64
// lanes of one wavefront, in registers: lane r holds row r of H and then of
// L; each right-looking step broadcasts the pivot and the new column with
// readlane, so there are no LDS round trips and no barriers.  Every entry
// gets the same operations in the same order as in the left-looking form
// (products with the earlier columns subtracted in ascending column order,
// then the division by the pivot), hence the same bits.  A pivot that is
// not finite or not above 64 eps R max_j H_jj fails the factorisation
// (return false, X untouched).  Otherwise lane j forms column j of L^{-1}
// (forward substitution against rows of L broadcast the same way) and stores
// it to X (LDS, pitch ld).  Loops run to the compile-time bound RB with
// uniform guards, so the row arrays stay in registers.
template <int RB>
__device__ __attribute__((always_inline)) inline bool chol_inv_regs(const double* H, double* X,
                                                                    int ld, int R, int t) {
  double arow[RB];
#pragma unroll
  for (int c = 0; c < RB; ++c) arow[c] = (c < R && t < R) ? H[t * ld + c] : 0.0;
  double maxdiag = 0.0;
#pragma unroll
  for (int j = 0; j < RB; ++j)
    if (j < R) maxdiag = fmax(maxdiag, lane_f64(arow[j], j));
  const double thresh = kPivotTolPerRank * R * maxdiag;
  bool all_ok = true;
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    if (j < R) {
      const double d = lane_f64(arow[j], j);
      const bool ok = isfinite(d) && d > thresh && maxdiag > 0.0 && isfinite(maxdiag);
      all_ok = all_ok && ok;
      const double ljj = ok ? sqrt(d) : 1.0;
      const double lj = t > j ? arow[j] / ljj : ljj;     // L[t][j] for t >= j
      arow[j] = lj;
#pragma unroll
      for (int c = j + 1; c < RB; ++c) {
        if (c < R) {
          const double lc = lane_f64(lj, c);               // L[c][j]
          if (t >= c) arow[c] -= lj * lc;
        }
      }
    }
  }
  if (!all_ok) return false;
  double x[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    if (r < R) {
      double v = (r == t) ? 1.0 : 0.0;
#pragma unroll
      for (int q = 0; q < r; ++q) {
        const double lrq = lane_f64(arow[q], r);           // L[r][q]
        if (q >= t) v -= lrq * x[q];
      }
      x[r] = (r < t) ? 0.0 : v / lane_f64(arow[r], r);
    }
  }
  if (t < R) {
#pragma unroll
    for (int r = 0; r < RB; ++r)
      if (r < R) X[r * ld + t] = x[r];
  }
  return true;
}

// Sum of one value per thread in a fixed order: butterfly within each
// wavefront, then the wavefront sums in ascending order; every thread gets
// the result.  scratch needs blockDim.x / 64 doubles; the call synchronises
// the block (and leaves scratch free again).
__device__ inline double block_sum(double v, double* scratch) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += scratch[q];
  __syncthreads();
  return s;
}

// H for model k: product of the other modes' Gram blocks in ascending mode
// order (the oracle's order).
__device__ void build_h(const double* G0, const double* G1, const double* G2, const double* G3,
                        int N, int n, int64_t goff, int R, double (*H)[kLd]) {
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
    const int r = e / R, s = e % R;
    const int64_t at = goff + r * R + s;
    double h = 0.0;
    bool first = true;
#pragma unroll
    for (int m = 0; m < kMaxOrder; ++m) {
      if (m >= N || m == n) continue;
      const double* Gm = m == 0 ? G0 : m == 1 ? G1 : m == 2 ? G2 : G3;
      const double g = Gm[at];
      h = first ? g : h * g;
      first = false;
    }
    H[r][s] = h;
  }
}

// Cholesky H = L L^T (lower).  Returns false (block-uniform) when a pivot is
// not finite or at or below tau * max_j H_jj.
__device__ bool cholesky(const double (*H)[kLd], double (*L)[kLd], int R, int* s_flag) {
  if (threadIdx.x == 0) *s_flag = 1;
  __syncthreads();
  double maxdiag = 0.0;
  for (int j = 0; j < R; ++j) maxdiag = fmax(maxdiag, H[j][j]);
  const double thresh = kPivotTolPerRank * R * maxdiag;
  for (int j = 0; j < R; ++j) {
    if (threadIdx.x == 0) {
      double d = H[j][j];
      for (int q = 0; q < j; ++q) d -= L[j][q] * L[j][q];
      const bool ok = isfinite(d) && d > thresh && maxdiag > 0.0 && isfinite(maxdiag);
      if (!ok) *s_flag = 0;
      L[j][j] = ok ? sqrt(d) : 1.0;
    }
    __syncthreads();
    const int i = threadIdx.x;
    if (i > j && i < R) {
      double v = H[i][j];
      for (int q = 0; q < j; ++q) v -= L[i][q] * L[j][q];
      L[i][j] = v / L[j][j];
    }
    __syncthreads();
  }
  const bool ok = *s_flag != 0;
  __syncthreads();
  return ok;
}

// Eigen pseudoinverse of symmetric H by cyclic Jacobi rotations (fallback
// only).  Writes Hp = V diag(w^+) V^T with eigenvalues at or below
// tau * w_max treated as zero.  W and V are LDS scratch.
__device__ void jacobi_pinv(const double (*H)[kLd], double (*W)[kLd], double (*V)[kLd],
                            double (*Hp)[kLd], int R, double* s_cs) {
  const int t = threadIdx.x;
  for (int e = t; e < R * R; e += blockDim.x) {
    const int r = e / R, s = e % R;
    W[r][s] = H[r][s];
    V[r][s] = (r == s) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    // off-diagonal mass, computed by one thread in a fixed order
    if (t == 0) {
      double off = 0.0, tot = 0.0;
      for (int r = 0; r < R; ++r)
        for (int s = 0; s < R; ++s) {
          tot += W[r][s] * W[r][s];
          if (r != s) off += W[r][s] * W[r][s];
        }
      s_cs[2] = (off <= 1e-30 * tot || !isfinite(off)) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (s_cs[2] != 0.0) break;
    for (int p = 0; p < R - 1; ++p)
      for (int q = p + 1; q < R; ++q) {
        if (t == 0) {
          const double apq = W[p][q];
          double c = 1.0, s = 0.0;
          if (apq != 0.0) {
            const double theta = (W[q][q] - W[p][p]) / (2.0 * apq);
            const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(tt * tt + 1.0);
            s = tt * c;
          }
          s_cs[0] = c;
          s_cs[1] = s;
        }
        __syncthreads();
        const double c = s_cs[0], s = s_cs[1];
        if (s != 0.0) {
          // columns p, q of W and V
          if (t < R) {
            const double wp = W[t][p], wq = W[t][q];
            W[t][p] = c * wp - s * wq;
            W[t][q] = s * wp + c * wq;
            const double vp = V[t][p], vq = V[t][q];
            V[t][p] = c * vp - s * vq;
            V[t][q] = s * vp + c * vq;
          }
          __syncthreads();
          // rows p, q of W
          if (t < R) {
            const double wp = W[p][t], wq = W[q][t];
            W[p][t] = c * wp - s * wq;
            W[q][t] = s * wp + c * wq;
          }
        }
        __syncthreads();
      }
  }
  if (t == 0) {
    double wmax = 0.0;
    for (int r = 0; r < R; ++r) wmax = fmax(wmax, W[r][r]);
    s_cs[3] = kPivotTolPerRank * R * wmax;
  }
  __syncthreads();
  const double cutoff = s_cs[3];
  for (int e = t; e < R * R; e += blockDim.x) {
    const int r = e / R, s = e % R;
    double acc = 0.0;
    for (int q = 0; q < R; ++q) {
      const double w = W[q][q];
      if (w > cutoff) acc += V[r][q] * (1.0 / w) * V[s][q];
    }
    Hp[r][s] = acc;
  }
  __syncthreads();
}

// Inverse of H from its Cholesky factor: Linv = L^{-1} by forward
// substitution (one column per thread), then H^{-1} = Linv^T Linv with the
// upper triangle mirrored (exactly symmetric).
__device__ void cholesky_inverse(const double (*L)[kLd], double (*Linv)[kLd],
                                 double (*Hinv)[kLd], int R) {
  const int j = threadIdx.x;
  if (j < R) {
    for (int r = 0; r < R; ++r) {
      double v = (r == j) ? 1.0 : 0.0;
      for (int q = j; q < r; ++q) v -= L[r][q] * Linv[q][j];
      Linv[r][j] = (r < j) ? 0.0 : v / L[r][r];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
    const int r = e / R, s = e % R;
    if (r <= s) {
      double acc = 0.0;
      for (int q = s; q < R; ++q) acc += Linv[q][r] * Linv[q][s];
      Hinv[r][s] = acc;
      Hinv[s][r] = acc;
    }
  }
  __syncthreads();
}

// Row pass: U(i,:) = M(i,:) H^{-1} for every row i of the model's block (the
// model's left-out rows of M taken as 0 when `zero`); returns this thread's
// share of sum_i U(i,:) . M(i,:) (for the error identity).
__device__ double row_pass(const double* __restrict__ M, double* __restrict__ U, int rows,
                           int ldc, int off, int R, bool zero, const ModelTable& mt, int k,
                           const double (*Hinv)[kLd]) {
  double inner = 0.0;
  for (int e = threadIdx.x; e < rows * R; e += blockDim.x) {
    const int i = e / R, r = e % R;
    const double* mrow = M + (int64_t)i * ldc + off;
    double u = 0.0, m = 0.0;
    if (!(zero && left_out_row(mt, i, k))) {
      for (int q = 0; q < R; ++q) u += mrow[q] * Hinv[q][r];
      m = mrow[r];
    }
    U[(int64_t)i * ldc + off + r] = u;
    inner += u * m;
  }
  return inner;
}

// Column sums of squares of the model's block of U, one column per wave
// round, lanes striding rows; then a fixed butterfly.
__device__ void column_norms(const double* U, int rows, int ldc, int off, int R, double* lam) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = blockDim.x >> 6;
  for (int r = wave; r < R; r += nw) {
    double s = 0.0;
    for (int i = lane; i < rows; i += 64) {
      const double v = U[(int64_t)i * ldc + off + r];
      s += v * v;
    }
    s = wave_sum(s);
    if (lane == 0) lam[r] = sqrt(s);
  }
}

// G = U^T U on the model's block, upper triangle computed, then mirrored.
__device__ void gram_block(const double* U, int rows, int ldc, int off, int R, double* G,
                           double (*Gs)[kLd]) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = blockDim.x >> 6;
  const int npairs = R * (R + 1) / 2;
  for (int pr = wave; pr < npairs; pr += nw) {
    // pair index -> (r, s), r <= s, row-major over the upper triangle
    int r = 0, rem = pr;
    while (rem >= R - r) {
      rem -= R - r;
      ++r;
    }
    const int s = r + rem;
    double acc = 0.0;
    for (int i = lane; i < rows; i += 64) {
      const double* row = U + (int64_t)i * ldc + off;
      acc += row[r] * row[s];
    }
    acc = wave_sum(acc);
    if (lane == 0) {
      G[r * R + s] = acc;
      G[s * R + r] = acc;
      if (Gs) {
        Gs[r][s] = acc;
        Gs[s][r] = acc;
      }
    }
  }
}

__global__ void __launch_bounds__(kThreads) k_update(const UpdateArgs a) {
  __shared__ double H[kMaxRank][kLd];
  __shared__ double L[kMaxRank][kLd];
  __shared__ double Hp[kMaxRank][kLd];
  __shared__ double Wj[kMaxRank][kLd];
  __shared__ double Vj[kMaxRank][kLd];
  __shared__ double Gs[kMaxRank][kLd];
  __shared__ double s_lam[kMaxRank];
  __shared__ double s_red[kThreads];
  __shared__ double s_cs[4];
  __shared__ int s_flag;

  for (int idx = blockIdx.x; idx < a.mt.K; idx += gridDim.x) {
    const int k = a.mt.order[idx];
    const int32_t st = a.status[k];
    if (st & (JKC_ST_CONVERGED | JKC_ST_NONFINITE)) continue;  // frozen (block-uniform)
    const int R = a.mt.rank[k];
    const int off = a.mt.off[k];
    const int64_t goff = a.mt.goff[k];
    const bool zero = a.n == a.nhat;

    build_h(a.G[0], a.G[1], a.G[2], a.G[3], a.N, a.n, goff, R, H);
    __syncthreads();
    const bool chol_ok = cholesky(H, L, R, &s_flag);
    if (chol_ok)
      cholesky_inverse(L, Wj, Hp, R);
    else
      jacobi_pinv(H, Wj, Vj, Hp, R, s_cs);

    const double inner = row_pass(a.Mout, a.U, a.In, a.ldc, off, R, zero, a.mt, k, Hp);
    const double in_all = block_sum(inner, s_red);

    column_norms(a.U, a.In, a.ldc, off, R, s_lam);
    __syncthreads();
    for (int e = threadIdx.x; e < a.In * R; e += blockDim.x) {
      const int i = e / R, r = e % R;
      const double l = s_lam[r];
      if (l > 0.0) {
        double* u = a.U + (int64_t)i * a.ldc + off + r;
        *u = *u / l;
      }
    }
    __syncthreads();
    double* Gn = a.n == 0 ? a.G[0] : a.n == 1 ? a.G[1] : a.n == 2 ? a.G[2] : a.G[3];
    gram_block(a.U, a.In, a.ldc, off, R, Gn + goff, Gs);
    if (threadIdx.x < R) a.lambda[off + threadIdx.x] = s_lam[threadIdx.x];
    __syncthreads();

    if (threadIdx.x == 0) {
      int32_t nst = st | (chol_ok ? 0 : JKC_ST_FALLBACK);
      if (a.last_mode) {
        const double in = in_all;
        double quad = 0.0;
        for (int r = 0; r < R; ++r)
          for (int s = 0; s < R; ++s) quad += s_lam[r] * H[r][s] * Gs[r][s] * s_lam[s];
        const double nt2 = a.normT2[k];
        const double e = nt2 + quad - 2.0 * in;
        const double f = 1.0 - sqrt(fmax(e, 0.0)) / sqrt(nt2);
        const int it = a.iters[k] + 1;
        a.iters[k] = it;
        a.err[k] = e;
        if (!isfinite(e)) nst |= JKC_ST_NONFINITE;
        if (a.check_conv && a.tol > 0.0 && it >= 2 && fabs(f - a.fit_prev[k]) < a.tol)
          nst |= JKC_ST_CONVERGED;
        a.fit_prev[k] = f;
        a.fit[k] = f;
      }
      a.status[k] = nst;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// LDS-staged update with the split-K reduction fused in.  Same mathematics
// and the same summation orders as k_update (so the same bits for U, lambda
// and the Gram matrices), but the model's block of M is summed over the
// split-K partials (ascending split order, the order of the stand-alone
// reduction) straight into LDS, and U is formed, normalised and reduced in
// LDS, so global memory is touched once for reading and once for writing.
// Used when the model's rows fit in the dynamic LDS budget.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kUpdThreads) k_update_lds(const UpdateArgs a) {
  extern __shared__ double smem[];
  const int Rp = a.rmax;
  const int ld = Rp + 1;
  double* H = smem;
  double* L = H + Rp * ld;             // Cholesky factor, then H^{-1}
  double* X = L + Rp * ld;             // L^{-1}, or Jacobi W
  double* V = X + Rp * ld;             // Jacobi eigenvectors
  double* Gs = V + Rp * ld;            // new Gram block
  double* lam = Gs + Rp * ld;
  double* misc = lam + Rp;             // [0] c, [1] s, [2] done, [3] cutoff
  double* red = misc + 8;              // per-wavefront sums (block_sum)
  double* Ms = red + kUpdThreads / 64; // In x ld: reduced M block
  double* Us = Ms + (size_t)a.In * ld; // In x ld: U block
  __shared__ int s_flag;
  const int t = threadIdx.x;
  const int64_t plane = (int64_t)a.In * a.ldc;

  // launch_update never gives this kernel more blocks than models, so every
  // block has a first model: no bounds check (and no wait for the model
  // count) before its loads are issued
  int idx = blockIdx.x;
  do {
    // one model per block when the grid covers them all (the cost order only
    // matters for a persistent grid): saves a dependent load
    const int k = (int)gridDim.x >= a.mt.K ? idx : a.mt.order[idx];
    // every per-model scalar in one round of loads; with one rank for every
    // model in the canonical column layout the model's columns and Gram
    // blocks follow from k, so the loads of H and M need no table lookup and
    // go out with the status in a single round
    const int32_t st = a.status[k];
    int R, off;
    int64_t goff;
    if (a.uniform_rank > 0) {
      R = a.uniform_rank;
      off = k * R;
      goff = (int64_t)k * R * R;
    } else {
      R = a.mt.rank[k];
      off = a.mt.off[k];
      goff = a.mt.goff[k];
    }
    // per-model scalars of the error step, fetched now (by every thread, with
    // no branch: a branch would make the compiler wait for them here) so that
    // their latency overlaps the update
    const double pre_nt2 = a.normT2[k];
    const double pre_fprev = a.fit_prev[k];
    const int32_t pre_it = a.iters[k];
    // a frozen model (converged or non-finite) is skipped once H and M are
    // staged (block-uniform; the loads are in bounds and nothing is written
    // to global memory before the check), so the status wait overlaps them
    const bool frozen = (st & (JKC_ST_CONVERGED | JKC_ST_NONFINITE)) != 0;
    const bool zero = a.n == a.nhat;
    const int RR = R * R;

    // The Gram factors of H, loaded before M's first round (every mode's
    // plane is read, a present one standing in for the skipped modes, so no
    // load sits behind a branch; 1.0 replaces the skipped modes' values, and
    // x * 1.0 == x exactly, so the product keeps the ascending-mode order and
    // bits of the oracle's).  For R <= 8 wavefront 0 forms H, factors it and
    // forms H^{-1} as soon as these arrive, while the other wavefronts load
    // and stage M; larger ranks factor after M is stored.
    constexpr int kHPer = (kMaxRank * kMaxRank + kUpdThreads - 1) / kUpdThreads;
    const bool early = R <= 8;
    double hg[kHPer][kMaxOrder];
    {
      const int present = a.n == 0 ? 1 : 0;
#pragma unroll
      for (int u = 0; u < kHPer; ++u) {
        const int e = t + u * kUpdThreads;
        const int64_t ge = goff + (e < RR ? e : 0);
#pragma unroll
        for (int mm = 0; mm < kMaxOrder; ++mm) {
          const bool use = mm < a.N && mm != a.n;
          // the plane by selects between the four pointers (an index into
          // the argument array would re-read the kernel arguments at a
          // computed offset, one more dependent round before the loads)
          const double* gp = mm == 0 ? a.G[0] : mm == 1 ? a.G[1] : mm == 2 ? a.G[2] : a.G[3];
          const double g = (use ? gp : (present ? a.G[1] : a.G[0]))[ge];
          hg[u][mm] = use ? g : 1.0;
        }
      }
    }
    auto form_h = [&]() __attribute__((always_inline)) {
#pragma unroll
      for (int u = 0; u < kHPer; ++u) {
        const int e = t + u * kUpdThreads;
        if (e < RR) {
          double h = hg[u][0];
#pragma unroll
          for (int m = 1; m < kMaxOrder; ++m) h *= hg[u][m];
          H[(e / R) * ld + e % R] = h;
        }
      }
    };
    if (early && t < 64) {
      // wavefront 0 (R^2 <= 64 entries): H, its Cholesky factor and L^{-1}
      // in registers (chol_inv_regs), then H^{-1} = L^{-T} L^{-1} with the
      // upper triangle mirrored, ordered by wavefront-local syncs; the
      // other wavefronts load and stage M meanwhile
      form_h();
      wave_lds_sync();
      const bool all_ok = chol_inv_regs<8>(H, X, ld, R, t);
      if (t == 0) s_flag = all_ok ? 1 : 0;
      wave_lds_sync();
      if (all_ok && t < RR) {
        const int r = t / R, c = t % R;
        if (r <= c) {
          double acc = 0.0;
          for (int q = c; q < R; ++q) acc += X[q * ld + r] * X[q * ld + c];
          L[r * ld + c] = acc;
          L[c * ld + r] = acc;
        }
      }
    }
    // M: kStage elements per thread per round (by the wavefronts other than
    // 0 when wavefront 0 factors H meanwhile), their loads (and the
    // left-out row flags) issued before any of them is stored (one memory
    // latency per round); partials summed in ascending split order
    const int tw = early ? t - 64 : t;
    const int nw = early ? kUpdThreads - 64 : kUpdThreads;
    if (tw >= 0) {
      constexpr int kStage = 4;
      const int nel = a.In * R;
      for (int e0 = 0; e0 == 0 || e0 < nel; e0 += kStage * nw) {
        double m[kStage];
        bool lo[kStage];
        if (a.splits == 1 && nel > 0) {
#pragma unroll
          for (int u = 0; u < kStage; ++u) {
            const int e = e0 + u * nw + tw;
            const int ec = e < nel ? e : 0;
            const int i = ec / R, r = ec - (ec / R) * R;
            m[u] = a.partial[(int64_t)i * a.ldc + off + r];
            // the flag is loaded unconditionally (row 0 when this is not the
            // sampled mode, whose rows may outnumber the flag table's) so no
            // branch waits for it before the next element's loads
            lo[u] = left_out_row(a.mt, zero ? i : 0, k) && zero;
          }
        } else {
#pragma unroll
          for (int u = 0; u < kStage; ++u) {
            const int e = e0 + u * nw + tw;
            m[u] = 0.0;
            lo[u] = false;
            if (e < nel) {
              const int i = e / R, r = e - (e / R) * R;
              const double* src = a.partial + (int64_t)i * a.ldc + off + r;
              for (int sp = 0; sp < a.splits; ++sp) m[u] += src[sp * plane];
              lo[u] = zero && left_out_row(a.mt, i, k);
            }
          }
        }
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
          const int e = e0 + u * nw + tw;
          if (e < nel) {
            const int i = e / R, r = e - (e / R) * R;
            Ms[i * ld + r] = lo[u] ? 0.0 : m[u];
          }
        }
      }
    }
    if (!early) form_h();
    __syncthreads();
    if (frozen) continue;

    // R > 8: Cholesky and L^{-1} in wavefront 0, in LDS with its steps
    // ordered by wavefront-local syncs: pivots by lane 0, the column below
    // by lanes i > j; then, if every pivot passed, lane j forms column j of
    // L^{-1}
    if (!early && t < 64) {
      double maxdiag = 0.0;
      for (int j = 0; j < R; ++j) maxdiag = fmax(maxdiag, H[j * ld + j]);
      const double thresh = kPivotTolPerRank * R * maxdiag;
      bool all_ok = true;
      for (int j = 0; j < R; ++j) {
        if (t == 0) {
          double d = H[j * ld + j];
          for (int q = 0; q < j; ++q) d -= L[j * ld + q] * L[j * ld + q];
          const bool ok = isfinite(d) && d > thresh && maxdiag > 0.0 && isfinite(maxdiag);
          all_ok = all_ok && ok;
          L[j * ld + j] = ok ? sqrt(d) : 1.0;
        }
        wave_lds_sync();
        if (t > j && t < R) {
          double v = H[t * ld + j];
          for (int q = 0; q < j; ++q) v -= L[t * ld + q] * L[j * ld + q];
          L[t * ld + j] = v / L[j * ld + j];
        }
        wave_lds_sync();
      }
      if (t == 0) s_flag = all_ok ? 1 : 0;
      wave_lds_sync();
      if (s_flag != 0 && t < R) {
        const int j = t;
        for (int r = 0; r < R; ++r) {
          double v = (r == j) ? 1.0 : 0.0;
          for (int q = j; q < r; ++q) v -= L[r * ld + q] * X[q * ld + j];
          X[r * ld + j] = (r < j) ? 0.0 : v / L[r * ld + r];
        }
      }
    }
    __syncthreads();
    const bool chol_ok = s_flag != 0;

    if (chol_ok) {
      if (!early) {   // (R <= 8: H^{-1} formed by wavefront 0 above)
        for (int e = t; e < R * R; e += blockDim.x) {
          const int r = e / R, c = e % R;
          if (r <= c) {
            double acc = 0.0;
            for (int q = c; q < R; ++q) acc += X[q * ld + r] * X[q * ld + c];
            L[r * ld + c] = acc;
            L[c * ld + r] = acc;
          }
        }
        __syncthreads();
      }
    } else {
      for (int e = t; e < R * R; e += blockDim.x) {
        const int r = e / R, c = e % R;
        X[r * ld + c] = H[r * ld + c];
        V[r * ld + c] = (r == c) ? 1.0 : 0.0;
      }
      __syncthreads();
      for (int sweep = 0; sweep < 40; ++sweep) {
        if (t == 0) {
          double offd = 0.0, tot = 0.0;
          for (int r = 0; r < R; ++r)
            for (int c = 0; c < R; ++c) {
              const double w = X[r * ld + c];
              tot += w * w;
              if (r != c) offd += w * w;
            }
          misc[2] = (offd <= 1e-30 * tot || !isfinite(offd)) ? 1.0 : 0.0;
        }
        __syncthreads();
        if (misc[2] != 0.0) break;
        for (int pp = 0; pp < R - 1; ++pp)
          for (int qq = pp + 1; qq < R; ++qq) {
            if (t == 0) {
              const double apq = X[pp * ld + qq];
              double c = 1.0, sn = 0.0;
              if (apq != 0.0) {
                const double theta = (X[qq * ld + qq] - X[pp * ld + pp]) / (2.0 * apq);
                const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                c = 1.0 / sqrt(tt * tt + 1.0);
                sn = tt * c;
              }
              misc[0] = c;
              misc[1] = sn;
            }
            __syncthreads();
            const double c = misc[0], sn = misc[1];
            if (sn != 0.0) {
              if (t < R) {
                const double wp = X[t * ld + pp], wq = X[t * ld + qq];
                X[t * ld + pp] = c * wp - sn * wq;
                X[t * ld + qq] = sn * wp + c * wq;
                const double vp = V[t * ld + pp], vq = V[t * ld + qq];
                V[t * ld + pp] = c * vp - sn * vq;
                V[t * ld + qq] = sn * vp + c * vq;
              }
              __syncthreads();
              if (t < R) {
                const double wp = X[pp * ld + t], wq = X[qq * ld + t];
                X[pp * ld + t] = c * wp - sn * wq;
                X[qq * ld + t] = sn * wp + c * wq;
              }
            }
            __syncthreads();
          }
      }
      if (t == 0) {
        double wmax = 0.0;
        for (int r = 0; r < R; ++r) wmax = fmax(wmax, X[r * ld + r]);
        misc[3] = kPivotTolPerRank * R * wmax;
      }
      __syncthreads();
      const double cutoff = misc[3];
      for (int e = t; e < R * R; e += blockDim.x) {
        const int r = e / R, c = e % R;
        double acc = 0.0;
        for (int q = 0; q < R; ++q) {
          const double w = X[q * ld + q];
          if (w > cutoff) acc += V[r * ld + q] * (1.0 / w) * V[c * ld + q];
        }
        L[r * ld + c] = acc;
      }
      __syncthreads();
    }

    // U = M H^{-1} in LDS, and this thread's share of sum U .* M
    double inner = 0.0;
    for (int e = t; e < a.In * R; e += blockDim.x) {
      const int i = e / R, r = e % R;
      const double* mrow = Ms + i * ld;
      double u = 0.0;
      for (int q = 0; q < R; ++q) u += mrow[q] * L[q * ld + r];
      Us[i * ld + r] = u;
      inner += u * mrow[r];
    }
    const double in_all = block_sum(inner, red);
    // column norms: one wave per column, lanes stride rows, fixed butterfly
    {
      const int wave = t >> 6, lane = t & 63, nw = blockDim.x >> 6;
      for (int r = wave; r < R; r += nw) {
        double sq = 0.0;
        for (int i = lane; i < a.In; i += 64) {
          const double v = Us[i * ld + r];
          sq += v * v;
        }
        sq = wave_sum(sq);
        if (lane == 0) lam[r] = sqrt(sq);
      }
    }
    __syncthreads();
    for (int e = t; e < a.In * R; e += blockDim.x) {
      const int i = e / R, r = e % R;
      const double l = lam[r];
      double v = Us[i * ld + r];
      if (l > 0.0) v = v / l;
      Us[i * ld + r] = v;
      a.U[(int64_t)i * a.ldc + off + r] = v;
    }
    __syncthreads();
    // Gram of the normalised block: one wave per upper-triangle pair
    double* Gn = a.n == 0 ? a.G[0] : a.n == 1 ? a.G[1] : a.n == 2 ? a.G[2] : a.G[3];
    {
      const int wave = t >> 6, lane = t & 63, nw = blockDim.x >> 6;
      const int npairs = R * (R + 1) / 2;
      for (int pr = wave; pr < npairs; pr += nw) {
        int r = 0, rem = pr;
        while (rem >= R - r) {
          rem -= R - r;
          ++r;
        }
        const int c = r + rem;
        double acc = 0.0;
        for (int i = lane; i < a.In; i += 64) acc += Us[i * ld + r] * Us[i * ld + c];
        acc = wave_sum(acc);
        if (lane == 0) {
          Gn[goff + r * R + c] = acc;
          Gn[goff + c * R + r] = acc;
          Gs[r * ld + c] = acc;
          Gs[c * ld + r] = acc;
        }
      }
    }
    if (t < R) a.lambda[off + t] = lam[t];
    __syncthreads();
    // the error's quadratic form lambda^T (H * G) lambda: wavefront 0, lanes
    // over the R^2 terms, fixed butterfly
    double quad = 0.0;
    if (a.last_mode && t < 64) {
      for (int e = t; e < R * R; e += 64) {
        const int r = e / R, c = e % R;
        quad += lam[r] * H[r * ld + c] * Gs[r * ld + c] * lam[c];
      }
      quad = wave_sum(quad);
    }
    if (t == 0) {
      int32_t nst = st | (chol_ok ? 0 : JKC_ST_FALLBACK);
      if (a.last_mode) {
        const double in = in_all;
        const double nt2 = pre_nt2;
        const double e = nt2 + quad - 2.0 * in;
        const double f = 1.0 - sqrt(fmax(e, 0.0)) / sqrt(nt2);
        const int it = pre_it + 1;
        a.iters[k] = it;
        a.err[k] = e;
        if (!isfinite(e)) nst |= JKC_ST_NONFINITE;
        if (a.check_conv && a.tol > 0.0 && it >= 2 && fabs(f - pre_fprev) < a.tol)
          nst |= JKC_ST_CONVERGED;
        a.fit_prev[k] = f;
        a.fit[k] = f;
      }
      a.status[k] = nst;
    }
    __syncthreads();
  } while ((idx += gridDim.x) < a.mt.K);
}

// Gram blocks of the models' columns of U.  A model's rows x R block is
// staged in LDS first, every load of it issued in one round (gram_block reads
// global memory again for each of the R(R+1)/2 pairs, one dependent round
// per pair and wavefront), then the pairs are formed from LDS with the same
// per-lane order and wavefront sums as gram_block, so the bits are the same.
// Blocks larger than the staging buffer use gram_block itself.  With a
// step (eta not null) each element of the block first becomes
// U - eta_k grad, written back to U, and the Gram block is that of the
// stepped factor: every mode's gradient step and Gram blocks in one launch.
constexpr int kGramStage = 6144;   // doubles (48 KB)
constexpr int kGramThreads = 512;  // eight wavefronts share the R(R+1)/2 pairs
__global__ void __launch_bounds__(kGramThreads) k_gram(const GramArgs a) {
  __shared__ double Bs[kGramStage];
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;
  constexpr int nw = kGramThreads / 64;
  // the launched mode of this block row (pointers by selects: an index into
  // the argument arrays would re-read the kernel arguments)
  const int mi = blockIdx.y;
  const int rows = mi == 0 ? a.rows[0] : mi == 1 ? a.rows[1] : mi == 2 ? a.rows[2] : a.rows[3];
  double* Um = mi == 0 ? a.U[0] : mi == 1 ? a.U[1] : mi == 2 ? a.U[2] : a.U[3];
  double* Gm = mi == 0 ? a.G[0] : mi == 1 ? a.G[1] : mi == 2 ? a.G[2] : a.G[3];
  const double* gm =
      mi == 0 ? a.grad[0] : mi == 1 ? a.grad[1] : mi == 2 ? a.grad[2] : a.grad[3];
  const bool step = a.eta != nullptr;
  for (int idx = blockIdx.x; idx < a.mt.K; idx += gridDim.x) {
    // models are independent here: with a block per model no cost order is
    // needed, and one rank in the canonical layout gives the offsets from k
    // (no dependent table round before the loads of U)
    const int k = (int)gridDim.x >= a.mt.K ? idx : a.mt.order[idx];
    int R, off;
    int64_t goff;
    if (a.uniform_rank > 0) {
      R = a.uniform_rank;
      off = k * R;
      goff = (int64_t)k * R * R;
    } else {
      R = a.mt.rank[k];
      off = a.mt.off[k];
      goff = a.mt.goff[k];
    }
    double* G = Gm + goff;
    if ((int64_t)rows * R > kGramStage) {
      if (step) {
        const double eta = a.eta[k];
        for (int e = t; e < rows * R; e += kGramThreads) {
          const int i = e / R, r = e - (e / R) * R;
          const int64_t at = (int64_t)i * a.ldc + off + r;
          Um[at] = Um[at] - eta * gm[at];
        }
        __syncthreads();   // the block's own writes, read back by gram_block
      }
      gram_block(Um, rows, a.ldc, off, R, G, nullptr);
    } else {
      const int n = rows * R;
      const double eta = step ? a.eta[k] : 0.0;
      for (int e0 = 0; e0 < n; e0 += 8 * kGramThreads) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + u * kGramThreads + t;
          const int ec = e < n ? e : 0;
          const int i = ec / R, r = ec - (ec / R) * R;
          v[u] = Um[(int64_t)i * a.ldc + off + r];
        }
        if (step) {
          double g[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * kGramThreads + t;
            const int ec = e < n ? e : 0;
            const int i = ec / R, r = ec - (ec / R) * R;
            g[u] = gm[(int64_t)i * a.ldc + off + r];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * kGramThreads + t;
            v[u] = v[u] - eta * g[u];
            if (e < n) {
              const int i = e / R, r = e - (e / R) * R;
              Um[(int64_t)i * a.ldc + off + r] = v[u];
            }
          }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + u * kGramThreads + t;
          if (e < n) Bs[e] = v[u];
        }
      }
      __syncthreads();
      const int npairs = R * (R + 1) / 2;
      for (int pr = wave; pr < npairs; pr += nw) {
        int r = 0, rem = pr;
        while (rem >= R - r) {
          rem -= R - r;
          ++r;
        }
        const int c = r + rem;
        double acc = 0.0;
        for (int i = lane; i < rows; i += 64) acc += Bs[i * R + r] * Bs[i * R + c];
        acc = wave_sum(acc);
        if (lane == 0) {
          G[r * R + c] = acc;
          G[c * R + r] = acc;
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Row-parallel update (default).  The model's update (Alg. 1 inner step for
// each submodel of Alg. 3) is split over blocks of kUpdRows rows:
//   k_solve_rows:    per (model, row chunk): H and H^{-1} (recomputed per
//                    chunk, R <= 32), the chunk's rows of M summed from the
//                    split-K partials in ascending split order (left-out
//                    rows zero for Case I), U = M H^{-1} (unnormalised) written to a staging
//                    buffer, and the chunk's U^T U (upper triangle) and
//                    sum U .* M stored;
//   k_finalize_rows: per (model, row chunk): the chunk sums added in chunk
//                    order give lambda_r = sqrt((U^T U)_rr); the chunk's rows
//                    are written normalised to the factor; chunk 0 writes
//                    lambda, the Gram of the normalised block and, on the last
//                    mode, the error and fit.
// Scratch per (model k, chunk c): R^2 + 2 doubles at nch * (goff_k + 2k) +
// c * (R^2 + 2); slot R^2 holds sum U .* M, slot R^2 + 1 the solve flag
// (1 Cholesky, 0 pseudoinverse, -1 model frozen), so the finalize kernel
// never reads the status it may rewrite.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_solve_rows(const UpdateArgs a) {
  __shared__ double H[kMaxRank][kLd], L[kMaxRank][kLd], Wj[kMaxRank][kLd], Vj[kMaxRank][kLd];
  __shared__ double Hp[kMaxRank][kLd];
  __shared__ double Ms[kUpdRows][kLd], Us[kUpdRows][kLd];
  __shared__ double s_cs[4];
  __shared__ double s_red[kThreads / 64];
  __shared__ int s_flag;
  const int t = threadIdx.x;
  const int nch = a.nch;
  const int64_t plane = (int64_t)a.In * a.ldc;
  for (int idx = blockIdx.x; idx < a.mt.K * nch; idx += gridDim.x) {
    const int k = a.mt.order[idx / nch];
    const int ch = idx % nch;
    const int r0 = ch * kUpdRows;
    if (r0 >= a.In) continue;                                     // block-uniform
    const int R = a.mt.rank[k];
    const int64_t goff = a.mt.goff[k];
    double* sc = a.scratch + (int64_t)nch * (goff + 2 * k) + (int64_t)ch * (R * R + 2);
    const int32_t st = a.status[k];
    if (st & (JKC_ST_CONVERGED | JKC_ST_NONFINITE)) {            // frozen
      if (t == 0) sc[R * R + 1] = -1.0;
      continue;
    }
    const int off = a.mt.off[k];
    const int rows = min(kUpdRows, a.In - r0);
    const bool zero = a.n == a.nhat;
    // H (other modes' Grams) and the chunk's rows of M: loads issued together
    build_h(a.G[0], a.G[1], a.G[2], a.G[3], a.N, a.n, goff, R, H);
    for (int e = t; e < rows * R; e += blockDim.x) {
      const int i = e / R, r = e % R;
      const double* src = a.partial + (int64_t)(r0 + i) * a.ldc + off + r;
      constexpr int kBatch = 16;
      double m = 0.0;
      int sp = 0;
      for (; sp + kBatch <= a.splits; sp += kBatch) {
        double v[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) v[u] = src[(int64_t)(sp + u) * plane];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) m += v[u];
      }
      for (; sp < a.splits; ++sp) m += src[(int64_t)sp * plane];
      Ms[i][r] = (zero && left_out_row(a.mt, r0 + i, k)) ? 0.0 : m;
    }
    __syncthreads();
    const bool chol_ok = cholesky(H, L, R, &s_flag);
    if (chol_ok)
      cholesky_inverse(L, Wj, Hp, R);
    else
      jacobi_pinv(H, Wj, Vj, Hp, R, s_cs);
    double inner = 0.0;
    for (int e = t; e < rows * R; e += blockDim.x) {
      const int i = e / R, r = e % R;
      double u = 0.0;
      for (int q = 0; q < R; ++q) u += Ms[i][q] * Hp[q][r];
      Us[i][r] = u;
      a.Utmp[(int64_t)(r0 + i) * a.ldc + off + r] = u;
      inner += u * Ms[i][r];
    }
    const double in_all = block_sum(inner, s_red);   // also makes Us visible
    // U^T U over the chunk's rows (<= 64: one lane per row), upper triangle
    {
      const int wave = t >> 6, lane = t & 63, nw = blockDim.x >> 6;
      const int npairs = R * (R + 1) / 2;
      for (int pr = wave; pr < npairs; pr += nw) {
        int r = 0, rem = pr;
        while (rem >= R - r) {
          rem -= R - r;
          ++r;
        }
        const int c = r + rem;
        double v = lane < rows ? Us[lane][r] * Us[lane][c] : 0.0;
        v = wave_sum(v);
        if (lane == 0) sc[r * R + c] = v;
      }
    }
    if (t == 0) {
      sc[R * R] = in_all;
      sc[R * R + 1] = chol_ok ? 1.0 : 0.0;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kThreads) k_finalize_rows(const UpdateArgs a) {
  __shared__ double S[kMaxRank][kLd], Hs[kMaxRank][kLd], Gs[kMaxRank][kLd];
  __shared__ double lam[kMaxRank];
  __shared__ double s_in;
  const int t = threadIdx.x;
  const int nch = a.nch;
  const int nchk = (a.In + kUpdRows - 1) / kUpdRows;
  for (int idx = blockIdx.x; idx < a.mt.K * nch; idx += gridDim.x) {
    const int k = a.mt.order[idx / nch];
    const int ch = idx % nch;
    const int r0 = ch * kUpdRows;
    if (r0 >= a.In) continue;                                     // block-uniform
    const int R = a.mt.rank[k];
    const int64_t goff = a.mt.goff[k];
    const double* sc0 = a.scratch + (int64_t)nch * (goff + 2 * k);
    const int stride = R * R + 2;
    const double flag = sc0[(int64_t)ch * stride + R * R + 1];
    if (flag < 0.0) continue;                                     // frozen (block-uniform)
    const int off = a.mt.off[k];
    const int rows = min(kUpdRows, a.In - r0);
    // chunk sums in chunk order; the upper triangle of U^T U, then sum U .* M
    for (int e = t; e <= R * R; e += blockDim.x) {
      const int r = e / R, c = e % R;
      if (e < R * R && r > c) continue;
      double v = 0.0;
      for (int q = 0; q < nchk; ++q) v += sc0[(int64_t)q * stride + e];
      if (e == R * R)
        s_in = v;
      else
        S[r][c] = v;
    }
    __syncthreads();
    if (t < R) lam[t] = sqrt(S[t][t]);
    __syncthreads();
    for (int e = t; e < rows * R; e += blockDim.x) {
      const int i = e / R, r = e % R;
      const int64_t at = (int64_t)(r0 + i) * a.ldc + off + r;
      const double u = a.Utmp[at];
      a.U[at] = lam[r] > 0.0 ? u / lam[r] : u;
    }
    if (ch == 0) {
      // Gram of the normalised block over all rows, formed exactly as the
      // Gram kernel forms it from stored factors (one wavefront per pair,
      // lanes striding rows, fixed butterfly), so a context restarted from
      // the factors continues bit for bit.
      double* Gn = a.n == 0 ? a.G[0] : a.n == 1 ? a.G[1] : a.n == 2 ? a.G[2] : a.G[3];
      const int wave = t >> 6, lane = t & 63, nw = blockDim.x >> 6;
      const int npairs = R * (R + 1) / 2;
      for (int pr = wave; pr < npairs; pr += nw) {
        int r = 0, rem = pr;
        while (rem >= R - r) {
          rem -= R - r;
          ++r;
        }
        const int c = r + rem;
        double acc = 0.0;
        for (int i = lane; i < a.In; i += 64) {
          const double* row = a.Utmp + (int64_t)i * a.ldc + off;
          const double ur = lam[r] > 0.0 ? row[r] / lam[r] : row[r];
          const double uc = lam[c] > 0.0 ? row[c] / lam[c] : row[c];
          acc += ur * uc;
        }
        acc = wave_sum(acc);
        if (lane == 0) {
          Gn[goff + r * R + c] = acc;
          Gn[goff + c * R + r] = acc;
          Gs[r][c] = acc;
          Gs[c][r] = acc;
        }
      }
      if (t < R) a.lambda[off + t] = lam[t];
      if (a.last_mode) build_h(a.G[0], a.G[1], a.G[2], a.G[3], a.N, a.n, goff, R, Hs);
      __syncthreads();
      if (t == 0) {
        const int32_t st = a.status[k];
        int32_t nst = st | (flag > 0.0 ? 0 : JKC_ST_FALLBACK);
        if (a.last_mode) {
          double quad = 0.0;
          for (int r = 0; r < R; ++r)
            for (int c = 0; c < R; ++c) quad += lam[r] * Hs[r][c] * Gs[r][c] * lam[c];
          const double nt2 = a.normT2[k];
          const double e = nt2 + quad - 2.0 * s_in;
          const double f = 1.0 - sqrt(fmax(e, 0.0)) / sqrt(nt2);
          const int it = a.iters[k] + 1;
          a.iters[k] = it;
          a.err[k] = e;
          if (!isfinite(e)) nst |= JKC_ST_NONFINITE;
          if (a.check_conv && a.tol > 0.0 && it >= 2 && fabs(f - a.fit_prev[k]) < a.tol)
            nst |= JKC_ST_CONVERGED;
          a.fit_prev[k] = f;
          a.fit[k] = f;
        }
        a.status[k] = nst;
      }
    }
    __syncthreads();
  }
}

int persistent_grid(int K) {
  // enough resident blocks to cover all 256 compute units a few times over
  return K < 1024 ? K : 1024;
}

// Gradient of the CP loss (all-at-once CP) per model and mode, every mode
// of the launch at once (grid y: the mode):
// grad = U H - M with H = *_{m != n} G_m; the left-out rows of the sampled
// mode are 0.  The blocks of the last mode also give the loss
// 1/2 (||T_{-P}||^2 + sum(H*G) - 2 sum(U*M)).
// The model's rows x R blocks of U and M are staged in LDS when they fit
// (their loads in flight while H is formed), so each element's row of U is
// read from LDS rather than with one dependent global round per element; the
// element-to-thread assignment and every sum keep their order, so the bits
// are those of the unstaged path.
constexpr int kGradStage = 3072;   // doubles per block (U and M: 48 KB)
constexpr int kGradThreads = 512;
__global__ void __launch_bounds__(kGradThreads) k_grad(const GradArgs a) {
  __shared__ double H[kMaxRank][kLd];
  __shared__ double s_red[kGradThreads / 64];
  __shared__ double Us[kGradStage], Ms[kGradStage];
  const int t = threadIdx.x;
  // this block row's mode, its arrays chosen by selects (no dynamic index
  // into the argument block)
  const int mq = blockIdx.y;
  const int n = a.n0 + mq;
  const int In = mq == 0 ? a.In[0] : mq == 1 ? a.In[1] : mq == 2 ? a.In[2] : a.In[3];
  const double* Mq = mq == 0 ? a.Mfull[0] : mq == 1 ? a.Mfull[1] : mq == 2 ? a.Mfull[2] : a.Mfull[3];
  const double* Uq = mq == 0 ? a.U[0] : mq == 1 ? a.U[1] : mq == 2 ? a.U[2] : a.U[3];
  double* gq = mq == 0 ? a.grad[0] : mq == 1 ? a.grad[1] : mq == 2 ? a.grad[2] : a.grad[3];
  const bool last_mode = a.loss != nullptr && n == a.N - 1;
  for (int idx = blockIdx.x; idx < a.mt.K; idx += gridDim.x) {
    const int k = (int)gridDim.x >= a.mt.K ? idx : a.mt.order[idx];
    int R, off;
    int64_t goff;
    if (a.uniform_rank > 0) {
      R = a.uniform_rank;
      off = k * R;
      goff = (int64_t)k * R * R;
    } else {
      R = a.mt.rank[k];
      off = a.mt.off[k];
      goff = a.mt.goff[k];
    }
    const int nel = In * R;
    const bool staged = nel <= kGradStage;
    if (staged) {
      for (int e0 = 0; e0 < nel; e0 += 4 * kGradThreads) {
        double vu[4], vm[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = e0 + u * kGradThreads + t;
          const int ec = e < nel ? e : 0;
          const int i = ec / R, r = ec - (ec / R) * R;
          const int64_t at = (int64_t)i * a.ldc + off + r;
          vu[u] = Uq[at];
          vm[u] = Mq[at];
        }
        if (e0 == 0) build_h(a.Gp[0], a.Gp[1], a.Gp[2], a.Gp[3], a.N, n, goff, R, H);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = e0 + u * kGradThreads + t;
          if (e < nel) {
            Us[e] = vu[u];
            Ms[e] = vm[u];
          }
        }
      }
    } else {
      build_h(a.Gp[0], a.Gp[1], a.Gp[2], a.Gp[3], a.N, n, goff, R, H);
    }
    __syncthreads();
    double inner = 0.0;
    for (int e = t; e < nel; e += blockDim.x) {
      const int i = e / R, r = e % R;
      const double* urow = staged ? Us + i * R : Uq + (int64_t)i * a.ldc + off;
      double g = 0.0;
      const double m = staged ? Ms[e] : Mq[(int64_t)i * a.ldc + off + r];
      if (!(n == a.nhat && left_out_row(a.mt, i, k))) {
        double uh = 0.0;
        for (int q = 0; q < R; ++q) uh += urow[q] * H[q][r];
        g = uh - m;
      }
      gq[(int64_t)i * a.ldc + off + r] = g;
      inner += urow[r] * m;
    }
    const double in_all = block_sum(inner, s_red);
    if (last_mode && threadIdx.x == 0) {
      const double in = in_all;
      const double* Gn = (n == 0 ? a.Gp[0] : n == 1 ? a.Gp[1] : n == 2 ? a.Gp[2] : a.Gp[3]) + goff;
      double quad = 0.0;
      for (int r = 0; r < R; ++r)
        for (int s = 0; s < R; ++s) quad += H[r][s] * Gn[r * R + s];
      a.loss[k] = 0.5 * (a.normT2[k] + quad - 2.0 * in);
    }
    __syncthreads();
  }
}

__global__ void k_scale_cols(const ModelTable mt, const double* w, const double* src,
                             int32_t rows, int32_t ldc, double* dst, int32_t ldd) {
  for (int idx = blockIdx.x; idx < mt.K; idx += gridDim.x) {
    const int R = mt.rank[idx], off = mt.off[idx];
    const double s = w ? w[idx] : 1.0;
    for (int e = threadIdx.x; e < rows * R; e += blockDim.x) {
      const int i = e / R, r = e % R;
      dst[(int64_t)i * ldd + off + r] = s * src[(int64_t)i * ldc + off + r];
    }
  }
}

__global__ void k_fold_lambda(double* U, int32_t rows, int32_t ldc, int32_t C, double* lambda) {
  const int64_t n = (int64_t)rows * C;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / C;
    const int c = (int)(e % C);
    U[i * ldc + c] *= lambda[c];
  }
}

__global__ void k_reset_lambda(double* lambda, int32_t C) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < C; c += gridDim.x * blockDim.x)
    lambda[c] = 1.0;
}

// eta_k = 1 / sum_n ||H_n|k||_F from the current Gram planes.
__global__ void k_gd_eta(const ModelTable mt, int32_t N, const double* G0, const double* G1,
                         const double* G2, const double* G3, double* eta) {
  const double* G[kMaxOrder] = {G0, G1, G2, G3};
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < mt.K; k += gridDim.x * blockDim.x) {
    const int R = mt.rank[k];
    const int64_t goff = mt.goff[k];
    double tot = 0.0;
    for (int n = 0; n < N; ++n) {
      double f2 = 0.0;
      for (int r = 0; r < R; ++r)
        for (int s = 0; s < R; ++s) {
          double h = 0.0;
          bool first = true;
          for (int m = 0; m < N; ++m) {
            if (m == n) continue;
            const double g = G[m][goff + r * R + s];
            h = first ? g : h * g;
            first = false;
          }
          f2 += h * h;
        }
      tot += sqrt(f2);
    }
    eta[k] = 1.0 / tot;
  }
}

__global__ void k_count_active(const int32_t* status, int32_t K, int32_t* out) {
  __shared__ int s[256];
  int c = 0;
  for (int k = threadIdx.x; k < K; k += blockDim.x)
    c += (status[k] & (JKC_ST_CONVERGED | JKC_ST_NONFINITE)) ? 0 : 1;
  s[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int i = 0; i < (int)blockDim.x; ++i) t += s[i];
    out[0] = t;
  }
}

int grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (int)b;
}

}  // namespace

int64_t update_lds_doubles(int rmax, int rows) {
  const int64_t ld = rmax + 1;
  return 5 * rmax * ld + rmax + 8 + kUpdThreads / 64 + 2 * (int64_t)rows * ld;
}

hipError_t launch_update(const UpdateArgs& a, hipStream_t s) {
  if (a.mt.K <= 0) return hipSuccess;
  if (a.lds_doubles > 0) {
    int blocks = a.mt.K < 2048 ? a.mt.K : 2048;
    hipLaunchKernelGGL(k_update_lds, dim3(blocks), dim3(kUpdThreads),
                       (size_t)a.lds_doubles * sizeof(double), s, a);
  } else {
    hipLaunchKernelGGL(k_update, dim3(persistent_grid(a.mt.K)), dim3(kThreads), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_update_rows(const UpdateArgs& a, hipStream_t s) {
  if (a.mt.K <= 0) return hipSuccess;
  const int64_t work = (int64_t)a.mt.K * a.nch;
  const int blocks = (int)(work < 4096 ? work : 4096);
  hipLaunchKernelGGL(k_solve_rows, dim3(blocks), dim3(kThreads), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_finalize_rows, dim3(blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gram(const GramArgs& a, hipStream_t s) {
  if (a.mt.K <= 0) return hipSuccess;
  if (a.nmodes < 1 || a.nmodes > kMaxOrder) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gram, dim3(persistent_grid(a.mt.K), a.nmodes), dim3(kGramThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_grad_assemble(const GradArgs& a, hipStream_t s) {
  if (a.nmodes < 1 || a.nmodes > kMaxOrder) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_grad, dim3(persistent_grid(a.mt.K), a.nmodes), dim3(kGradThreads), 0, s,
                     a);
  return hipGetLastError();
}

hipError_t launch_scale_cols_by_model(const ModelTable& mt, const double* w, const double* src,
                                      int32_t rows, int32_t ldc, double* dst, int32_t ldd,
                                      hipStream_t s) {
  hipLaunchKernelGGL(k_scale_cols, dim3(persistent_grid(mt.K)), dim3(kThreads), 0, s, mt, w,
                     src, rows, ldc, dst, ldd);
  return hipGetLastError();
}

hipError_t launch_fold_lambda(double* U, int32_t rows, int32_t ldc, int32_t C, double* lambda,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_fold_lambda, dim3(grid_for((int64_t)rows * C)), dim3(256), 0, s, U, rows,
                     ldc, C, lambda);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reset_lambda, dim3(grid_for(C)), dim3(256), 0, s, lambda, C);
  return hipGetLastError();
}

hipError_t launch_gd_eta(const ModelTable& mt, int32_t N, const double* const* G, double* eta,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_gd_eta, dim3(grid_for(mt.K)), dim3(256), 0, s, mt, N, G[0], G[1],
                     N > 2 ? G[2] : nullptr, N > 3 ? G[3] : nullptr, eta);
  return hipGetLastError();
}

hipError_t launch_count_active(const int32_t* status, int32_t K, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_count_active, dim3(1), dim3(256), 0, s, status, K, out);
  return hipGetLastError();
}

}  // namespace jkc
