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
// (BM = WM*TM*16, BN = WN*TN*16) and one contiguous chunk of the K range,
// walked in steps of BK columns.  Each step is software-pipelined: the
// global loads of step t+1 (a BM x BK slice of the unfolding and the factor
// rows of a BK x BN Khatri-Rao slice) are in flight while the matrix cores
// work on step t out of LDS; the KRP products are formed and written to the
// other LDS buffer afterwards, so one barrier per step suffices.  Each thread
// owns one column of the A slice and one column of the B slice and walks its
// column's multi-index incrementally (no divisions in the loop).
//
// Matrix instruction (INSTR):
//   0: v_mfma_f64_16x16x4 -- one 16x16 tile per instruction;
//   1: v_mfma_f64_4x4x4 (4 independent 4x4 blocks per instruction): four
//      instructions q = 0..3 cover a 16x16x4 step, block b producing rows
//      4b..4b+3 and columns 4((b+q) mod 4)..+3 (a diagonal schedule, so the
//      A operand is loaded once and four B operands are rotated);
//   2: v_mfma_f64_4x4x4 in row strips: all four blocks take the same 4 rows
//      of A and block b columns 4b..4b+3 of a 16-column group, so one
//      instruction is a 4 x 16 x 4 step and tiles need only multiples of 4
//      rows (no padding of 100- or 200-row modes to 16).
// INSTR + 8 selects the interleaved step schedule (see the main loop).
// INSTR + 16 loads through buffer resources with 32-bit byte offsets (the
// tensor and every factor below 2^31 bytes): the hardware range check
// returns zeros past the end, so the chunk end is enforced by pointing the
// Khatri-Rao loads of out-of-range K indices past their buffer, and tile
// rows and columns past the matrix read clamped-free (their results are
// never stored).  Row offsets are scalar and immediate, so a step spends
// almost no vector instructions on addressing and masking: on gfx950 every
// vector ALU instruction issued between matrix instructions costs matrix
// throughput.
// Partials of the K chunks are summed later in a fixed order, so results are
// bitwise repeatable for a fixed tiling.
#include <type_traits>

#include <hip/hip_ext.h>

#include "jkc_internal.hpp"

namespace jkc {

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {

constexpr int kXcds = 8;  // accelerator complex dies on MI355X

// Lane layout of v_mfma_f64_4x4x4 (4 blocks), measured on gfx950: lane l
// belongs to block b = (l >> 2) & 3 and holds, with e = l & 3, kq = l >> 4,
//   A(i = e, k = kq),  B(k = kq, j = e),  D(i = kq, j = e)
// of that block's 4x4x4 product.

// Incremental walk over columns j of the unfolding: the multi-index of the
// other modes (lowest mode fastest, Eq. (3)), the tensor offset of the
// column and the row offsets into the other modes' multi-factors.
struct ColWalker {
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
  // the same offset in 32-bit arithmetic (tensors below 2^31 bytes)
  __device__ uint32_t toff32(const MttkrpArgs& a) const {
    return idx[0] * (uint32_t)a.ostride[0] + idx[1] * (uint32_t)a.ostride[1] +
           idx[2] * (uint32_t)a.ostride[2];
  }
};

template <int WM, int WN, int TM, int TN, int BK, int INSTR, int NO, bool F32>
__global__ void __launch_bounds__(64 * WM * WN)
k_mttkrp_f64(const MttkrpArgs a) {
  constexpr int NT = 64 * WM * WN;
  constexpr int FAM = INSTR & 7;             // matrix instruction family
  constexpr bool SCHED = (INSTR & 8) != 0;   // interleaved step schedule
  constexpr bool BUF = (INSTR & 16) != 0;    // buffer loads, 32-bit offsets
  constexpr int RPT = FAM == 2 ? 4 : 16;     // rows per matrix-core tile
  constexpr int BM = WM * TM * RPT;
  // rows staged in LDS: a multiple of 16, and of the rows one K index of a
  // step spreads over the block's threads
  constexpr int RQ = NT / BK > 16 ? NT / BK : 16;
  constexpr int BMP = (BM + RQ - 1) / RQ * RQ;
  constexpr int BN = WN * TN * 16;
  // Row pitches in LDS (doubles).  Measured on gfx950: paired fragment reads
  // (two doubles per lane) are free of bank conflicts at any pitch; a
  // column-walk staging write (16 or 32 consecutive K rows of one column per
  // wavefront, the layout of modes without unit stride) is free of them only
  // at an odd pitch (4-way at 20 mod 32); a single strip read (4 doubles of
  // each of 2 rows per half-wavefront) needs the pitch in [4, 28] mod 32; a
  // single read of 16 doubles of each of 2 rows is 2-way at any pitch but 16
  // (mod 32), which would make the column walk 16-way.  A rows therefore sit
  // at 21 (mod 32) for every family; B rows, read in pairs and written along
  // rows, at 8.
  constexpr int LDA = BMP + (21 - BMP % 32 + 32) % 32;
  constexpr int LDB = BN + (8 - BN % 32 + 32) % 32;
  constexpr int VA = BMP * BK / NT;  // A elements per thread per step (one column)
  constexpr int VB = BN * BK / NT;   // B elements per thread per step (one column)
  static_assert(BK % 4 == 0, "BK");
  static_assert(VA >= 1 && VA * NT == BMP * BK, "A tile must split evenly over threads");
  static_assert(VB >= 1 && VB * NT == BN * BK, "B tile must split evenly over threads");
  static_assert(BMP % VA == 0 && BN % VB == 0, "vector width");
  static_assert(VB == 1 || VB % 2 == 0, "B is staged in pairs of columns");
  using AccT = typename std::conditional<FAM == 2, double, v4d>::type;

  __shared__ __attribute__((aligned(16))) double As[2][BK][LDA];
  __shared__ __attribute__((aligned(16))) double Bs[2][BK][LDB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM;
  const int wn = wave / WM;

  // Block -> (column tile, row tile, K chunk).  Work-groups are dealt to the
  // 8 XCDs round-robin; remapping so that each XCD receives a contiguous
  // run of logical blocks (column tile fastest) keeps the blocks that share
  // one slice of the unfolding on the same XCD, where it stays in L2.
  const int total = gridDim.x;
  int logical = blockIdx.x;
  const int per_xcd = total / kXcds;
  if (logical < per_xcd * kXcds) logical = (logical % kXcds) * per_xcd + logical / kXcds;
  const int nt = logical % a.ntiles;
  const int mt = (logical / a.ntiles) % a.mtiles;
  const int split = logical / (a.ntiles * a.mtiles);
  const int i0 = mt * BM;
  const int c0 = nt * BN;
  const int64_t kbeg = (int64_t)split * a.kchunk;
  const int64_t kend = min(kbeg + a.kchunk, a.J);
  const int nsteps = kend > kbeg ? (int)((kend - kbeg + BK - 1) / BK) : 0;

  // Thread roles.  A (BMP x BK slice of the unfolding): for a mode with unit
  // stride (rows contiguous in memory) threads run along the rows of one
  // column, otherwise along the columns of one row; a thread's VA elements
  // are interleaved with its neighbours' (row gA + sA * v), so each load and
  // each LDS write of a wavefront covers contiguous addresses.  B (BK x BN
  // Khatri-Rao slice): threads run along the columns of one K index, in
  // pairs of columns interleaved the same way (column 2 gB + 2 GB u).
  const bool m_fast = a.stride_n == 1;
  constexpr int GA = BMP / VA;      // threads per A column when m_fast
  constexpr int GK = NT / BK;       // threads per A row otherwise
  const int kA = m_fast ? tid / GA : tid % BK;
  const int gA = m_fast ? tid % GA : tid / BK;
  const int sA = m_fast ? GA : GK;
  constexpr int PB = VB == 1 ? 1 : 2;  // columns per B chunk
  constexpr int GB = BN / VB;          // threads per K index of B
  const int kB = tid / GB;
  const int gB = tid % GB;

  ColWalker wA, wB;
  wA.init(a, kbeg + kA);
  wB.init(a, kbeg + kB);

  const double* __restrict__ Tf64 = static_cast<const double*>(a.T);
  const float* __restrict__ Tf32 = static_cast<const float*>(a.T);

  // Registers of the step in flight.  Loads are unconditional at a clamped
  // address; which values are real is kept in amask / bmask and applied when
  // the step is stored, so no load result is consumed (waited for) before
  // the matrix-core work of the current step has been issued.
  using TT = typename std::conditional<F32, float, double>::type;
  using TTyp = TT;
  TT ra[VA];
  double rb[NO][VB];
  uint32_t amask = 0;
  uint32_t bmask = 0;

  // Buffer resources (word 3: the gfx9 raw-buffer format, range checked).
  constexpr int kRsrcWord3 = 0x00020000;
  const __amdgpu_buffer_rsrc_t rT = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(a.T), (short)0, BUF ? (int)((int64_t)a.M * a.J * (int64_t)sizeof(TTyp)) : 0,
      kRsrcWord3);
  __amdgpu_buffer_rsrc_t rU[NO];
#pragma unroll
  for (int q = 0; q < NO; ++q)
    rU[q] = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(a.oU[q]), (short)0,
                                              BUF ? a.odim[q] * a.ldc * 8 : 0, kRsrcWord3);
  // byte distance between a thread's consecutive A rows (scalar)
  const int sA_bytes = (int)(sA * a.stride_n * (int64_t)sizeof(TTyp));

  auto load_step = [&]() {
    if constexpr (BUF) {
      const uint32_t voffA = (wA.toff32(a) + (uint32_t)(i0 + gA) * (uint32_t)a.stride_n) *
                             (uint32_t)sizeof(TTyp);
#pragma unroll
      for (int v = 0; v < VA; ++v) {
        if constexpr (F32)
          ra[v] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rT, voffA, v * sA_bytes, 0));
        else
          ra[v] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rT, voffA, v * sA_bytes, 0));
      }
      // K indices past the chunk read past the factor buffers (zeros)
      const bool kok = wB.j < kend;
#pragma unroll
      for (int q = 0; q < NO; ++q) {
        const uint32_t vb = kok ? (wB.idx[q] * (uint32_t)a.ldc + (uint32_t)(c0 + PB * gB)) * 8u
                                : 0x80000000u;
#pragma unroll
        for (int u = 0; u < VB / PB; ++u) {
          const uint32_t o = vb + (uint32_t)(8 * PB * GB * u);
          if constexpr (PB == 2) {
            const double2 x = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rU[q], o, 0, 0));
            rb[q][2 * u] = x.x;
            rb[q][2 * u + 1] = x.y;
          } else {
            rb[q][u] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rU[q], o, 0, 0));
          }
        }
      }
      return;
    }
    const bool va = wA.j < kend;
    const int64_t toffA = va ? wA.toff(a) : 0;
    amask = 0;
#pragma unroll
    for (int v = 0; v < VA; ++v) {
      const int r = gA + sA * v;
      const int row = i0 + r;
      const bool ok = va && r < BM && row < a.M;
      amask |= (uint32_t)ok << v;
      const int64_t addr = ok ? toffA + (int64_t)row * a.stride_n : 0;
      ra[v] = F32 ? Tf32[addr] : Tf64[addr];
    }
    // Columns come in pairs (ldc is even), each pair wholly inside the
    // factor rows or wholly past them; the columns between ncols and ldc
    // hold zeros.
    const bool kok = wB.j < kend;
    bmask = 0;
#pragma unroll
    for (int u = 0; u < VB / PB; ++u) {
      const int col = c0 + PB * (gB + GB * u);
      bmask |= (uint32_t)(kok && col < a.ldc) << u;
    }
#pragma unroll
    for (int q = 0; q < NO; ++q) {
      const double* __restrict__ urow = a.oU[q] + (int64_t)(kok ? wB.idx[q] : 0u) * a.ldc;
#pragma unroll
      for (int u = 0; u < VB / PB; ++u) {
        const int col = c0 + PB * (gB + GB * u);
        const int cc = (bmask >> u) & 1u ? col : 0;
        if constexpr (PB == 2) {
          const double2 x = *reinterpret_cast<const double2*>(urow + cc);
          rb[q][2 * u] = x.x;
          rb[q][2 * u + 1] = x.y;
        } else {
          rb[q][u] = urow[cc];
        }
      }
    }
  };
  auto store_step = [&](int buf) {
    // Empty asm statements pin the first use of the loaded registers here:
    // the wait on global memory and every product come after this point.
#pragma unroll
    for (int v = 0; v < VA; ++v) asm volatile("" : "+v"(ra[v]));
#pragma unroll
    for (int q = 0; q < NO; ++q)
#pragma unroll
      for (int v = 0; v < VB; ++v) asm volatile("" : "+v"(rb[q][v]));
#pragma unroll
    for (int v = 0; v < VA; ++v)
      As[buf][kA][gA + sA * v] = (BUF || ((amask >> v) & 1u)) ? (double)ra[v] : 0.0;
#pragma unroll
    for (int u = 0; u < VB / PB; ++u) {
      double x[PB];
#pragma unroll
      for (int p = 0; p < PB; ++p) {
        // product from the highest mode down (the listing order of Eq. (1))
        double y = rb[NO - 1][PB * u + p];
#pragma unroll
        for (int q = NO - 2; q >= 0; --q) y *= rb[q][PB * u + p];
        x[p] = (BUF || ((bmask >> u) & 1u)) ? y : 0.0;
      }
      double* dst = &Bs[buf][kB][PB * (gB + GB * u)];
      if constexpr (PB == 2)
        *reinterpret_cast<double2*>(dst) = make_double2(x[0], x[1]);
      else
        dst[0] = x[0];
    }
  };

  AccT acc[TM][TN];
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y) acc[x][y] = AccT{};

  if (nsteps > 0) {
    load_step();
    store_step(0);
  }
  __syncthreads();

  const int o16 = lane & 15;
  const int blk = lane >> 4;
  const int b4 = (lane >> 2) & 3;   // 4x4x4 block of this lane
  const int e4 = lane & 3;
  const int kq4 = lane >> 4;

  // Matrix-core operand fragments, double-buffered in registers: the
  // fragments of group g+1 are read from LDS while the matrix cores work on
  // group g.
  constexpr int FB = FAM == 1 ? 4 * TN : TN;
  constexpr int G = BK / 4;                        // groups of 4 K per step
  constexpr int NMF = TM * TN * (FAM == 1 ? 4 : 1);
  constexpr int NRD = TM + FB;
  double fa[2][TM], fb[2][FB];
  auto read_frag = [&](int buf, int kk, int slot) {
    if constexpr (FAM == 2) {
      // row strips: every block gets the same 4 rows of A (same LDS
      // addresses), block b the columns 4b..4b+3 of each 16-column group.
      // B first, then A in the order the matrix instructions use them, so
      // the first instructions of a group wait only for the earliest reads.
#pragma unroll
      for (int y = 0; y < TN; ++y)
        fb[slot][y] = Bs[buf][kk + kq4][wn * TN * 16 + y * 16 + 4 * b4 + e4];
#pragma unroll
      for (int x = 0; x < TM; ++x) fa[slot][x] = As[buf][kk + kq4][wm * TM * 4 + x * 4 + e4];
    } else if constexpr (FAM == 0) {
#pragma unroll
      for (int x = 0; x < TM; ++x) fa[slot][x] = As[buf][kk + blk][wm * TM * 16 + x * 16 + o16];
#pragma unroll
      for (int y = 0; y < TN; ++y) fb[slot][y] = Bs[buf][kk + blk][wn * TN * 16 + y * 16 + o16];
    } else {
#pragma unroll
      for (int x = 0; x < TM; ++x)
        fa[slot][x] = As[buf][kk + kq4][wm * TM * 16 + x * 16 + 4 * b4 + e4];
#pragma unroll
      for (int y = 0; y < TN; ++y)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          fb[slot][4 * y + q] = Bs[buf][kk + kq4][wn * TN * 16 + y * 16 + 4 * ((b4 + q) & 3) + e4];
    }
  };
  auto mfma_group = [&](int slot) {
#pragma unroll
    for (int x = 0; x < TM; ++x)
#pragma unroll
      for (int y = 0; y < TN; ++y) {
        if constexpr (FAM == 2)
          acc[x][y] = __builtin_amdgcn_mfma_f64_4x4x4f64(fa[slot][x], fb[slot][y], acc[x][y], 0, 0, 0);
        else if constexpr (FAM == 0)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[slot][x], fb[slot][y], acc[x][y], 0, 0, 0);
        else
#pragma unroll
          for (int q = 0; q < 4; ++q)
            acc[x][y][q] = __builtin_amdgcn_mfma_f64_4x4x4f64(fa[slot][x], fb[slot][4 * y + q],
                                                              acc[x][y][q], 0, 0, 0);
      }
  };

  // One K step = G groups of matrix-core work.  Loads and the store of the
  // next step run unconditionally (past the end of the chunk they fetch
  // clamped addresses and store zeros into the idle buffer), which keeps the
  // step free of branches.
  //
  // Interleaved schedule (SCHED): each group is a scheduling region of its
  // own in which the step's memory work is interleaved with the matrix
  // instructions by scheduling-group directives (one global load, one LDS
  // read, or one LDS write with its arithmetic between matrix instructions)
  // and the fragments of group g+1 are read while group g computes.  The
  // next step is stored into the other LDS buffer during group G-2 and the
  // step's barrier sits before the last group, whose fragments are already
  // in registers: the first fragments of the next step are read from the
  // other buffer while the last group computes, so no wavefront waits on
  // LDS right after the barrier.
  // Otherwise the compiler schedules each group; scheduling barriers only
  // keep the loads at the head of the step and the store before the last
  // group, and the barrier ends the step.
  static_assert(!SCHED || (G >= 4 && G % 2 == 0), "interleaved schedule needs BK % 16 == 0");
  if constexpr (SCHED) {
    if (nsteps > 0) read_frag(0, 0, 0);
  }
  for (int s = 0; s < nsteps; ++s) {
    const int buf = s & 1;
    if constexpr (SCHED) {
      wA.advance(a, BK);
      wB.advance(a, BK);
      load_step();
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int cur = g & 1;
        if (g == G - 1) {
          __syncthreads();
          read_frag(buf ^ 1, 0, cur ^ 1);
        } else {
          read_frag(buf, 4 * (g + 1), cur ^ 1);
          if (g == G - 2) store_step(buf ^ 1);
        }
        mfma_group(cur);
        if (g == 0) {
#pragma unroll
          for (int i = 0; i < VA + NO * (VB / PB); ++i) {
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);   // global load
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // matrix
          }
        }
        if (g == G - 2) {
#pragma unroll
          for (int i = 0; i < NRD; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // LDS read
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // matrix
          }
#pragma unroll
          for (int i = 0; i < VA + VB / PB; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x002, 2 * NO, 0);   // products, selects
            __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);       // LDS write
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);       // matrix
          }
        } else {
#pragma unroll
          for (int i = 0; i < NRD; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // LDS read
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);   // matrix
          }
        }
        __builtin_amdgcn_sched_group_barrier(0x008, NMF, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
      wA.advance(a, BK);
      wB.advance(a, BK);
      load_step();
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if (g == G - 1) {
          __builtin_amdgcn_sched_barrier(0);
          store_step(buf ^ 1);
          __builtin_amdgcn_sched_barrier(0);
        }
        read_frag(buf, 4 * g, 0);
        mfma_group(0);
      }
      __syncthreads();
    }
  }

  // Epilogue.  16x16x4: lane l holds, in element r, row 4*r + l/16 and
  // column l%16 of its tile.  4x4x4: element q holds row 4*b + l/16 and
  // column 4*((b+q) mod 4) + (l mod 4), b = (l/4) mod 4.
  double* __restrict__ out = a.partial + (int64_t)split * a.M * a.ldc;
  if constexpr (FAM == 2) {
    // row strip x, group y: lane holds row 4x + l/16, column 16y + 4b + l%4
#pragma unroll
    for (int x = 0; x < TM; ++x)
#pragma unroll
      for (int y = 0; y < TN; ++y) {
        const int row = i0 + wm * TM * 4 + x * 4 + kq4;
        const int col = c0 + wn * TN * 16 + y * 16 + 4 * b4 + e4;
        if (row < a.M && col < a.ldc) out[(int64_t)row * a.ldc + col] = acc[x][y];
      }
    return;
  } else {
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int rr, cc;
        if (FAM == 0) {
          rr = 4 * r + blk;
          cc = o16;
        } else {
          rr = 4 * b4 + kq4;
          cc = 4 * ((b4 + r) & 3) + e4;
        }
        const int row = i0 + wm * TM * 16 + x * 16 + rr;
        const int col = c0 + wn * TN * 16 + y * 16 + cc;
        if (row < a.M && col < a.ldc) out[(int64_t)row * a.ldc + col] = acc[x][y][r];
      }
  }
}

// With events, the dispatch stamps them itself (no separate event packets
// between kernels).
template <int WM, int WN, int TM, int TN, int BK, int INSTR, int NO, bool F32>
void launch_one(const MttkrpArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const dim3 grid(a.mtiles * a.ntiles * a.splits), block(64 * WM * WN);
  if (e0 || e1)
    hipExtLaunchKernelGGL((k_mttkrp_f64<WM, WN, TM, TN, BK, INSTR, NO, F32>), grid, block, 0, s, e0, e1,
                          0, a);
  else
    hipLaunchKernelGGL((k_mttkrp_f64<WM, WN, TM, TN, BK, INSTR, NO, F32>), grid, block, 0, s, a);
}

// One instantiation per (number of other modes, tensor element type), so
// that the load and product loops are fully unrolled without branches.
template <int WM, int WN, int TM, int TN, int BK, int INSTR>
hipError_t launch_f64(const MttkrpArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  switch (a.nother * 2 + (a.t_is_f32 ? 1 : 0)) {
    case 2: launch_one<WM, WN, TM, TN, BK, INSTR, 1, false>(a, s, e0, e1); break;
    case 3: launch_one<WM, WN, TM, TN, BK, INSTR, 1, true>(a, s, e0, e1); break;
    case 4: launch_one<WM, WN, TM, TN, BK, INSTR, 2, false>(a, s, e0, e1); break;
    case 5: launch_one<WM, WN, TM, TN, BK, INSTR, 2, true>(a, s, e0, e1); break;
    case 6: launch_one<WM, WN, TM, TN, BK, INSTR, 3, false>(a, s, e0, e1); break;
    case 7: launch_one<WM, WN, TM, TN, BK, INSTR, 3, true>(a, s, e0, e1); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define JKC_F64_VARIANT(WM, WN, TM, TN, BK, I) \
  { WM, WN, TM, TN, BK, &launch_f64<WM, WN, TM, TN, BK, I>, I }

}  // namespace

const std::vector<MttkrpVariant>& mttkrp_f64_variants() {
  static const std::vector<MttkrpVariant> v = {
      JKC_F64_VARIANT(1, 4, 25, 2, 16, 2),  // 100 x 128, 4x4x4 row strips
      JKC_F64_VARIANT(2, 2, 25, 2, 16, 2),  // 200 x 64
      JKC_F64_VARIANT(2, 2, 25, 1, 16, 2),  // 200 x 32
      JKC_F64_VARIANT(1, 4, 25, 1, 16, 2),  // 100 x 64
      JKC_F64_VARIANT(2, 2, 13, 2, 16, 2),  // 104 x 64
      JKC_F64_VARIANT(2, 2, 13, 4, 16, 2),  // 104 x 128
      JKC_F64_VARIANT(1, 4, 13, 4, 16, 2),  // 52 x 256
      JKC_F64_VARIANT(2, 2, 25, 4, 16, 2),  // 200 x 128
      JKC_F64_VARIANT(1, 4, 16, 2, 16, 2),  // 64 x 128
      JKC_F64_VARIANT(2, 2, 32, 1, 16, 2),  // 256 x 32
      JKC_F64_VARIANT(2, 2, 2, 2, 16, 1),   // 64 x 64, 4x4x4 diagonal
      JKC_F64_VARIANT(2, 2, 4, 2, 16, 1),   // 128 x 64
      JKC_F64_VARIANT(2, 2, 2, 2, 16, 0),   // 64 x 64, 16x16x4
      JKC_F64_VARIANT(2, 2, 4, 2, 16, 0),   // 128 x 64
      JKC_F64_VARIANT(1, 4, 7, 2, 16, 0),   // 112 x 128
      JKC_F64_VARIANT(2, 4, 13, 2, 32, 2),  // 104 x 128, 8 wavefronts, BK 32
      JKC_F64_VARIANT(2, 2, 13, 4, 32, 2),  // 104 x 128, BK 32
      // interleaved schedule
      JKC_F64_VARIANT(1, 4, 7, 2, 16, 8),   // 112 x 128, 16x16x4
      JKC_F64_VARIANT(2, 2, 4, 2, 16, 8),   // 128 x 64, 16x16x4
      JKC_F64_VARIANT(2, 2, 13, 4, 16, 10), // 104 x 128, strips
      JKC_F64_VARIANT(2, 2, 13, 2, 16, 10), // 104 x 64, strips
      JKC_F64_VARIANT(2, 4, 13, 2, 32, 10), // 104 x 128, 8 wavefronts, BK 32
      JKC_F64_VARIANT(2, 4, 13, 2, 16, 10), // 104 x 128, 8 wavefronts
      JKC_F64_VARIANT(4, 2, 7, 4, 32, 10),  // 112 x 128, 8 wavefronts, BK 32
      JKC_F64_VARIANT(4, 2, 13, 2, 32, 10), // 208 x 64, 8 wavefronts, BK 32
      JKC_F64_VARIANT(2, 4, 13, 4, 16, 10), // 104 x 256, 8 wavefronts
      JKC_F64_VARIANT(2, 4, 4, 2, 16, 8),   // 128 x 128, 8 wavefronts, 16x16x4
      // interleaved schedule, buffer loads
      JKC_F64_VARIANT(2, 4, 13, 2, 32, 26), // 104 x 128, 8 wavefronts, BK 32
      JKC_F64_VARIANT(2, 4, 13, 2, 16, 26), // 104 x 128, 8 wavefronts
      JKC_F64_VARIANT(2, 2, 13, 4, 16, 26), // 104 x 128
      JKC_F64_VARIANT(2, 2, 13, 2, 16, 26), // 104 x 64
      JKC_F64_VARIANT(4, 2, 7, 4, 32, 26),  // 112 x 128, 8 wavefronts, BK 32
      JKC_F64_VARIANT(4, 2, 13, 2, 32, 26), // 208 x 64, 8 wavefronts, BK 32
      JKC_F64_VARIANT(2, 4, 13, 4, 16, 26), // 104 x 256, 8 wavefronts
      JKC_F64_VARIANT(1, 4, 7, 2, 16, 24),  // 112 x 128, 16x16x4
      JKC_F64_VARIANT(2, 4, 4, 2, 16, 24),  // 128 x 128, 8 wavefronts, 16x16x4
      JKC_F64_VARIANT(1, 4, 5, 2, 16, 24),  // 80 x 128, 16x16x4 (W on 20,000 rows: 1,000 blocks)
  };
  return v;
}

}  // namespace jkc
