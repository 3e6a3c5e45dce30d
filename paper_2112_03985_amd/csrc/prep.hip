// Preparation and bookkeeping kernels: tensor residency (copy or bfloat16
// hi/lo split), slice norms ||T(p,:,...)||^2 and the submodel norms
// ||T_{-p}||^2 of the error step of Alg. 3, multi-factor packing with the
// inserted zero row of Alg. 3's initialisation, the fixed-order reduction of
// split-K MTTKRP partials with the Case I row removal, and the explicit
// slice removal of Alg. 2 (used by the plain per-submodel baseline).
#include <algorithm>

#include <hip/hip_ext.h>

#include "jkc_internal.hpp"

namespace jkc {

namespace {

int grid_for(int64_t n, int per = 256) {
  int64_t b = (n + per - 1) / per;
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  return (int)b;
}

__global__ void k_copy_tensor(const void* src, int32_t src_f32, void* dst, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (src_f32)
      static_cast<float*>(dst)[e] = static_cast<const float*>(src)[e];
    else
      static_cast<double*>(dst)[e] = static_cast<const double*>(src)[e];
  }
}

// Round a float64 to bfloat16 with round-to-nearest-even, directly from the
// float64 bits (no intermediate float32 rounding).
__device__ uint16_t bf16_rne(double x) {
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

__device__ inline double bf16_to_double(uint16_t h) {
  return (double)__uint_as_float((uint32_t)h << 16);
}

// x = t_1 + t_2 + ... : t_1 = bf16(x), t_2 = bf16(x - t_1), ... (each
// remainder exact in float64), term t at planes + t * (plane size).
// The mode-n unfolding with its columns ordered k = jl + ilp * w (low-mode
// index jl, zero for jl >= I_low; wrap w over the other modes, lowest
// fastest), stored in K blocks of 32: element (i, k) at
// ((k / 32) * I_n + i) * 32 + k % 32, so the 32-K slice of every row is
// one contiguous run of I_n * 64 bytes.  One thread per element.  IT is the
// type of the index arithmetic: 32-bit when every element index fits (the
// multi-index of each element costs a few integer divisions, about five
// times cheaper in 32 bits than in 64), 64-bit otherwise.
template <typename IT>
__global__ void k_split_unfold(const void* src, int32_t src_f32, int32_t N, int64_t d0,
                               int64_t d1, int64_t d2, int64_t d3, int32_t n, int32_t low,
                               int32_t ilp, int32_t nterm, uint16_t* planes) {
  const IT dims[4] = {(IT)d0, (IT)d1, (IT)d2, (IT)d3};
  IT stride[4];
  IT P = 1;
  for (int m = 0; m < 4; ++m) {
    stride[m] = P;
    if (m < N) P *= dims[m];
  }
  const IT I = dims[n];
  const IT ilpT = (IT)ilp;
  const IT wraps = P / (I * dims[low]);
  const int64_t total = (int64_t)I * ilp * (int64_t)wraps;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const IT ee = (IT)e;
    const IT kk = ee & 31;
    const IT q = ee >> 5;
    const IT kb = q / I;
    const IT i = q - kb * I;
    const IT k = kb * 32 + kk;
    const IT w = k / ilpT;
    const IT jl = k - w * ilpT;
    double x = 0.0;
    if (jl < dims[low]) {
      IT rem = w, off = i * stride[n] + jl * stride[low];
      for (int m = 0; m < N; ++m) {
        if (m == n || m == low) continue;
        off += (rem % dims[m]) * stride[m];
        rem /= dims[m];
      }
      x = src_f32 ? (double)static_cast<const float*>(src)[off] : static_cast<const double*>(src)[off];
    }
    for (int t = 0; t < nterm; ++t) {
      const uint16_t h = bf16_rne(x);
      planes[(int64_t)t * total + e] = h;
      x -= bf16_to_double(h);
    }
  }
}

// The low mode's factor U (rows x ldc float64) as nterm bfloat16 terms, in
// K blocks of 32 rows: term t of U(j, c) at out + t * ldc * ilp +
// ((j / 32) * ldc + c) * 32 + j % 32, zero for rows <= j < ilp.
__global__ void k_split_factor_t(const double* U, int32_t rows, int32_t ldc, int32_t ilp,
                                 int32_t nterm, uint16_t* out) {
  const int64_t total = (int64_t)ldc * ilp;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t jj = e & 31;
    const int64_t q = e >> 5;
    const int64_t jb = q / ldc;
    const int64_t c = q - jb * ldc;
    const int64_t j = jb * 32 + jj;
    double x = j < rows ? U[j * ldc + c] : 0.0;
    for (int t = 0; t < nterm; ++t) {
      const uint16_t h = bf16_rne(x);
      out[(int64_t)t * total + e] = h;
      x -= bf16_to_double(h);
    }
  }
}

// Tensor viewed as (inner, I, outer): element (a, p, b) at a + inner*(p + I*b).
// Block `chunk` sums outer indices b = chunk, chunk + chunks, ...; thread
// handles slices p; each partial is one sequential sum.
__global__ void k_slice_partial(const void* T, int32_t t_f32, int64_t inner, int32_t I,
                                int64_t outer, int32_t chunks, double* part) {
  const int chunk = blockIdx.x;
  auto at = [&](int64_t e) -> double {
    return t_f32 ? (double)static_cast<const float*>(T)[e] : static_cast<const double*>(T)[e];
  };
  for (int p = threadIdx.x; p < I; p += blockDim.x) {
    double s = 0.0;
    int64_t b = chunk;
    if (inner == 1) {
      // the sampled mode is mode 0: four slabs' loads issued together,
      // added in the same ascending order
      for (; b + 3 * (int64_t)chunks < outer; b += 4 * (int64_t)chunks) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = at((int64_t)p + (int64_t)I * (b + u * (int64_t)chunks));
#pragma unroll
        for (int u = 0; u < 4; ++u) s += v[u] * v[u];
      }
    }
    for (; b < outer; b += chunks) {
      const int64_t base = inner * ((int64_t)p + (int64_t)I * b);
      for (int64_t a = 0; a < inner; ++a) {
        const double v = at(base + a);
        s += v * v;
      }
    }
    part[(int64_t)chunk * I + p] = s;
  }
}

// One block per slice p: thread t holds the chunk partials t, t + blockDim,
// ... (ascending), then a pairwise tree over the threads in a fixed order.
constexpr int kSliceFinalThreads = 256;
__global__ void __launch_bounds__(kSliceFinalThreads)
k_slice_final(const double* part, int32_t chunks, int32_t I, double* s_out) {
  __shared__ double red[kSliceFinalThreads];
  const int t = threadIdx.x;
  for (int p = blockIdx.x; p < I; p += gridDim.x) {
    double s = 0.0;
    for (int c = t; c < chunks; c += kSliceFinalThreads) s += part[(int64_t)c * I + p];
    red[t] = s;
    __syncthreads();
    for (int w = kSliceFinalThreads / 2; w > 0; w >>= 1) {
      if (t < w) red[t] += red[t + w];
      __syncthreads();
    }
    if (t == 0) s_out[p] = red[0];
    __syncthreads();
  }
}

// ||T_{-P}||^2 = sum of s_i over the rows i not left out of the model,
// ascending i (the full norm for a model that leaves out nothing).
// A left-out row adds +0.0, which leaves the (non-negative) running sum
// unchanged bit for bit, so the loads carry no branch and go out four at a
// time.
__global__ void k_model_norms(const double* s, int32_t I, const uint8_t* lomask, int32_t K,
                              double* normT2) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x) {
    double t = 0.0;
    int i = 0;
    for (; i + 4 <= I; i += 4) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = lomask[(int64_t)(i + u) * K + k] ? 0.0 : s[i + u];
#pragma unroll
      for (int u = 0; u < 4; ++u) t += v[u];
    }
    for (; i < I; ++i) t += lomask[(int64_t)i * K + k] ? 0.0 : s[i];
    normT2[k] = t;
  }
}

// Row i of column c's model is left out (padding columns own no rows).
__device__ inline bool row_left_out(const LeftOut& lo, int64_t i, int c) {
  const int k = lo.colmodel[c];
  return k >= 0 && lo.lomask[i * lo.K + k] != 0;
}

// dst[i][c] (ld ldc) = src[i][c] (ld lds) for c < C, 0 for C <= c < ldc;
// the left-out rows of column c's model are zeroed when zero_rows (the
// inserted zero rows, Alg. 3).
__global__ void k_pack(const double* src, int32_t lds, int32_t rows, int32_t C, int32_t ldc,
                       LeftOut lo, int32_t zero_rows, double* dst) {
  const int64_t n = (int64_t)rows * ldc;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / ldc;
    const int c = (int)(e % ldc);
    double v = 0.0;
    if (c < C) {
      v = src[i * lds + c];
      if (zero_rows && row_left_out(lo, i, c)) v = 0.0;
    }
    dst[e] = v;
  }
}

// dst[i][c] = src[i][map[c]] for c < C, 0 for C <= c < ldc (column
// relayout of a multi-factor; rows x ldc, both leading dimension ldc).
__global__ void k_gather_cols(const double* src, int32_t rows, int32_t ldc, int32_t C,
                              const int32_t* map, double* dst) {
  const int64_t n = (int64_t)rows * ldc;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / ldc;
    const int c = (int)(e % ldc);
    dst[e] = c < C ? src[i * ldc + map[c]] : 0.0;
  }
}

__global__ void k_unpack(const double* src, int32_t ldc, int32_t rows, int32_t C, double* dst) {
  const int64_t n = (int64_t)rows * C;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / C;
    const int c = (int)(e % C);
    dst[e] = src[i * ldc + c];
  }
}

__global__ void k_fill(double* p, int64_t n, double v) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

// out[i][c] = sum_s partial[s][i][c]; the left-out rows of column c's model
// set to 0 when zero_rows (Case I: the left-out rows of the sampled mode's
// MTTKRP).  A block covers
// 64 consecutive elements with kReduceGroups wavefronts: with many partials
// wavefront q sums its contiguous quarter of the splits in ascending order
// and the quarter sums are added in ascending q; with few partials
// (splits < kReduceQuarterMin) wavefront 0 sums them all in ascending order.
// Either order is fixed, so the result is bitwise repeatable.
constexpr int kReduceGroups = 4;
constexpr int kReduceQuarterMin = 16;
__global__ void __launch_bounds__(64 * kReduceGroups)
k_reduce(const double* partial, int32_t splits, int32_t rows, int32_t ldc, int32_t ncols,
         LeftOut lo, int32_t zero_rows, double* out, int32_t ldo) {
  __shared__ double part[kReduceGroups][64];
  const int64_t n = (int64_t)rows * ncols;
  const int64_t plane = (int64_t)rows * ldc;
  const int lane = threadIdx.x & 63;
  const int q = threadIdx.x >> 6;
  const int groups = splits >= kReduceQuarterMin ? kReduceGroups : 1;
  const int per = (splits + groups - 1) / groups;
  const int sb = q * per;
  const int se = min(splits, sb + per);
  for (int64_t e0 = (int64_t)blockIdx.x * 64; e0 < n; e0 += (int64_t)gridDim.x * 64) {
    const int64_t e = e0 + lane;
    const bool ok = e < n;
    const int64_t i = ok ? e / ncols : 0;
    const int c = ok ? (int)(e % ncols) : 0;
    const double* src = partial + i * ldc + c;
    double s = 0.0;
    if (ok && q < groups) {
      // loads of kBatch partials issued together, additions in ascending
      // order; with thousands of wavefronts resident, short batches keep the
      // memory system busiest (the reductions of the 100x200x200 benchmark,
      // 32 to 128 splits of 100 or 200 x 500 outputs, 8.7 us on average
      // with batches of 2, 8.9 with 4, 9.7 with 8, 12.9 with 16)
      constexpr int kBatch = 2;
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
    part[q][lane] = s;
    __syncthreads();
    if (q == 0 && ok) {
      double t = part[0][lane];
      for (int g = 1; g < groups; ++g) t += part[g][lane];
      if (zero_rows && row_left_out(lo, i, c)) t = 0.0;
      out[i * ldo + c] = t;
    }
    __syncthreads();
  }
}

template <typename E>
__global__ void k_remove_slice(const E* src, int64_t inner, int32_t I, int64_t outer, int32_t p,
                               E* dst) {
  const int64_t n = inner * (int64_t)(I - 1) * outer;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = e % inner;
    const int64_t rest = e / inner;
    const int64_t q = rest % (I - 1);
    const int64_t b = rest / (I - 1);
    const int64_t qs = q < p ? q : q + 1;
    dst[e] = src[a + inner * (qs + (int64_t)I * b)];
  }
}

}  // namespace

hipError_t launch_copy_tensor(const void* src, int32_t src_f32, void* dst, int64_t count,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_copy_tensor, dim3(grid_for(count)), dim3(256), 0, s, src, src_f32, dst,
                     count);
  return hipGetLastError();
}

hipError_t launch_split_unfold(const void* src, int32_t src_f32, int32_t N, const int64_t* dims,
                               int32_t n, int32_t low, int32_t ilp, int32_t nterm,
                               uint16_t* planes, hipStream_t s) {
  int64_t P = 1;
  for (int m = 0; m < N; ++m) P *= dims[m];
  const int64_t total = dims[n] * (int64_t)ilp * (P / (dims[n] * dims[low]));
  // every element index (and every tensor offset, < P <= total) below 2^31
  if (total < (int64_t(1) << 31))
    hipLaunchKernelGGL(k_split_unfold<uint32_t>, dim3(grid_for(total)), dim3(256), 0, s, src,
                       src_f32, N, dims[0], N > 1 ? dims[1] : 1, N > 2 ? dims[2] : 1,
                       N > 3 ? dims[3] : 1, n, low, ilp, nterm, planes);
  else
    hipLaunchKernelGGL(k_split_unfold<int64_t>, dim3(grid_for(total)), dim3(256), 0, s, src,
                       src_f32, N, dims[0], N > 1 ? dims[1] : 1, N > 2 ? dims[2] : 1,
                       N > 3 ? dims[3] : 1, n, low, ilp, nterm, planes);
  return hipGetLastError();
}

hipError_t launch_split_factor_t(const double* U, int32_t rows, int32_t ldc, int32_t ilp,
                                 int32_t nterm, uint16_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_split_factor_t, dim3(grid_for((int64_t)ldc * ilp)), dim3(256), 0, s, U,
                     rows, ldc, ilp, nterm, out);
  return hipGetLastError();
}

hipError_t launch_slice_norms(const void* T, int32_t t_f32, int64_t inner, int32_t I,
                              int64_t outer, double* partial, int32_t chunks, double* s_out,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_slice_partial, dim3(chunks), dim3(256), 0, s, T, t_f32, inner, I, outer,
                     chunks, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int fblocks = I < 1 ? 1 : I < 4096 ? (int)I : 4096;
  hipLaunchKernelGGL(k_slice_final, dim3(fblocks), dim3(kSliceFinalThreads), 0, s, partial, chunks,
                     I, s_out);
  return hipGetLastError();
}

hipError_t launch_model_norms(const double* s, int32_t I, const uint8_t* lomask, int32_t K,
                              double* normT2, hipStream_t st) {
  hipLaunchKernelGGL(k_model_norms, dim3(grid_for(K)), dim3(256), 0, st, s, I, lomask, K, normT2);
  return hipGetLastError();
}

hipError_t launch_pack_factor(const double* src, int32_t lds, int32_t rows, int32_t C,
                              int32_t ldc, LeftOut lo, int32_t zero_rows, double* dst,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3(grid_for((int64_t)rows * ldc)), dim3(256), 0, s, src, lds,
                     rows, C, ldc, lo, zero_rows, dst);
  return hipGetLastError();
}

hipError_t launch_gather_cols(const double* src, int32_t rows, int32_t ldc, int32_t C,
                              const int32_t* map, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_cols, dim3(grid_for((int64_t)rows * ldc)), dim3(256), 0, s, src,
                     rows, ldc, C, map, dst);
  return hipGetLastError();
}

hipError_t launch_unpack(const double* src, int32_t ldc, int32_t rows, int32_t C, double* dst,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_unpack, dim3(grid_for((int64_t)rows * C)), dim3(256), 0, s, src, ldc,
                     rows, C, dst);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partial, int32_t splits, int32_t rows, int32_t ldc,
                         int32_t ncols, LeftOut lo, int32_t zero_rows, double* out,
                         int32_t ldo, hipStream_t s, hipEvent_t stop) {
  const int64_t n = (int64_t)rows * ncols;
  if (n <= 0) return stop ? hipEventRecord(stop, s) : hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 63) / 64, 16384);
  if (stop)
    hipExtLaunchKernelGGL(k_reduce, dim3((unsigned)blocks), dim3(64 * kReduceGroups), 0, s, nullptr,
                          stop, 0, partial, splits, rows, ldc, ncols, lo, zero_rows, out, ldo);
  else
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)blocks), dim3(64 * kReduceGroups), 0, s, partial,
                       splits, rows, ldc, ncols, lo, zero_rows, out, ldo);
  return hipGetLastError();
}

hipError_t launch_remove_slice(const void* src, int32_t elem_bytes, int64_t inner, int32_t I,
                               int64_t outer, int32_t p, void* dst, hipStream_t s) {
  const int64_t n = inner * (int64_t)(I - 1) * outer;
  if (n <= 0) return hipSuccess;
  if (elem_bytes == 4)
    hipLaunchKernelGGL(k_remove_slice<float>, dim3(grid_for(n)), dim3(256), 0, s,
                       static_cast<const float*>(src), inner, I, outer, p,
                       static_cast<float*>(dst));
  else
    hipLaunchKernelGGL(k_remove_slice<double>, dim3(grid_for(n)), dim3(256), 0, s,
                       static_cast<const double*>(src), inner, I, outer, p,
                       static_cast<double*>(dst));
  return hipGetLastError();
}

}  // namespace jkc
