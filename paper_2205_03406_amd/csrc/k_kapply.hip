// On-the-fly kernel-matrix apply Y = K X on the MFMA units (the built-in
// black box standing in for the fast matvecs of the experiments section:
// K(x, y) = log|x - y| in 1D/2D, 1/|x - y| in 3D, 0 where x = y).
//
// Design (gfx950): a workgroup of 4 waves owns 64 rows of Y and BN = 16*NT
// columns.  Each wave owns 16 rows.  The K(rows, k-block) operand is never
// stored: every lane evaluates one kernel entry per 4-deep MFMA step in
// registers, in exactly the A-operand layout of the 16x16x4 MFMA (lane l
// holds row l%16, depth l/16), so K costs one VALU evaluation per entry per
// column tile while the matrix core does 2*BN flops with it.  X k-blocks and
// the matching point coordinates are staged through LDS, double-buffered.
// The contraction over all N points is the whole cost: 2 N^2 ncols flops
// against N*ncols*8 bytes of X per row block, far above the FP64 ridge.
#include <algorithm>
#include <type_traits>

#include "device_common.h"
#include "kernels.h"

namespace hm {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// k-block (points per LDS stage): 16 in FP64 (49.7 TFLOP/s against 44.8 at
// 32 on the log kernel, N = 16384, 576 columns), 32 in FP32 (92.8 against
// 83.0 at 16 and 87.2 at 64: half the barriers per point, still two
// workgroups per CU)
#ifndef HM_KAPPLY_BK32
#define HM_KAPPLY_BK32 32
#endif
#ifndef HM_KAPPLY_BK64
#define HM_KAPPLY_BK64 16
#endif
#ifndef HM_KAPPLY_PAD
#define HM_KAPPLY_PAD 2      // LDS row padding of the X k-block (elements)
#endif

// Natural logarithm of a positive finite x, written from the series
//   x = 2^e m,  m in [1/sqrt2, sqrt2),  log m = 2 atanh(s) = 2 s sum_k s^(2k)/(2k+1),
//   s = (m - 1) / (m + 1),  |s| <= 0.1716,
// truncated after s^22 (next term below 2^-55 relative).  m - 1 is exact;
// the quotient is refined once from the hardware reciprocal; e ln2 is added
// in two parts.  About 30 straight-line FP64 instructions, a few ulp.
__device__ __forceinline__ double log_pos(double x) {
  int e = __builtin_amdgcn_frexp_exp(x);
  double m = __builtin_amdgcn_frexp_mant(x);  // [0.5, 1)
  const bool lo = m < 0.70710678118654752440;
  m = lo ? 2.0 * m : m;
  e = lo ? e - 1 : e;
  const double num = m - 1.0;
  const double den = m + 1.0;
  double rc = __builtin_amdgcn_rcp(den);
  rc = fma(fma(-den, rc, 1.0), rc, rc);
  rc = fma(fma(-den, rc, 1.0), rc, rc);
  double s = num * rc;
  s = fma(fma(-s, den, num), rc, s);
  const double t = s * s;
  double p = 1.0 / 23.0;
  p = fma(p, t, 1.0 / 21.0);
  p = fma(p, t, 1.0 / 19.0);
  p = fma(p, t, 1.0 / 17.0);
  p = fma(p, t, 1.0 / 15.0);
  p = fma(p, t, 1.0 / 13.0);
  p = fma(p, t, 1.0 / 11.0);
  p = fma(p, t, 1.0 / 9.0);
  p = fma(p, t, 1.0 / 7.0);
  p = fma(p, t, 1.0 / 5.0);
  p = fma(p, t, 1.0 / 3.0);
  const double lm = 2.0 * s + (2.0 * s) * (t * p);
  const double fe = (double)e;
  const double ln2_hi = 0.6931471526622772216796875;  // ln2 rounded to 24 bits
  const double ln2_lo = 2.7897668087737545e-08;       // ln2 - ln2_hi
  return fe * ln2_hi + (fe * ln2_lo + lm);
}

// 1/sqrt(x) for x > 0 from the hardware estimate y (relative error e0):
// with e = 1 - x y^2, (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + O(e^3), so
// y (1 + e/2 + 3e^2/8) has relative error O(e0^3), below an ulp.  x = 0
// gives inf or NaN here; the caller replaces it.
__device__ __forceinline__ double rsqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}

template <int KER>
__device__ __forceinline__ double kval64(double r2) {
  if (KER == 1) {
    const double v = rsqrt_pos(r2);
    return r2 > 0.0 ? v : 0.0;
  }
  const double v = 0.5 * log_pos(r2 > 0.0 ? r2 : 1.0);
  return r2 > 0.0 ? v : 0.0;
}

template <int KER>
__device__ __forceinline__ float kval32(float r2) {
  const float safe = r2 > 0.0f ? r2 : 1.0f;
  const float v = KER == 0 ? 0.34657359027997264f * __log2f(safe)  // 0.5 ln(2) log2(r2)
                           : rsqrtf(safe);
  return r2 > 0.0f ? v : 0.0f;
}

// SEG = false: the whole operator, grid (row blocks, column tiles), the
// row blocks counted from aux (a slice of the rows: aux = its first block).
// SEG = true: block-diagonal (forest) form, a 1-D grid over (item, column
// tile) pairs, column tile fastest; all indices below are relative to the
// item's instance (rows, depth and point coordinates start at its base row),
// and n stays the stride of the point coordinates; aux = split (the second
// live column range, < 0: none).
template <typename T, int NT, int KER, int DIM, bool SEG>
__global__ void __launch_bounds__(256)
kapply_kernel(int64_t n, const double *__restrict__ pts_all, int64_t ncols,
              const T *__restrict__ X_all, int64_t ldx, T *__restrict__ Y_all, int64_t ldy,
              const KItem *__restrict__ items, int64_t aux) {
  constexpr int BK = sizeof(T) == 4 ? HM_KAPPLY_BK32 : HM_KAPPLY_BK64;  // points per LDS buffer
  constexpr int BN = 16 * NT;
  constexpr int LDT = BN + HM_KAPPLY_PAD;
  __shared__ T Xs[2][BK][LDT];
  __shared__ double Ps[2][DIM][BK];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  int64_t row_blk, col0, base = 0, nloc = n;
  bool live = true;
  if constexpr (SEG) {
    const int64_t nct = (ncols + BN - 1) / BN;
    const KItem it = items[blockIdx.x / nct];
    col0 = (int64_t)(blockIdx.x % nct) * BN;
    row_blk = it.rblk;
    base = it.base;
    nloc = it.nloc;
    live = col0 < it.width || (aux >= 0 && col0 + BN > aux && col0 < aux + it.width);
  } else {
    row_blk = ((int64_t)blockIdx.x + aux) * 64;
    col0 = (int64_t)blockIdx.y * BN;
  }
  const double *__restrict__ pts = pts_all + base;
  const T *__restrict__ X = X_all + base;
  T *__restrict__ Y = Y_all + base;
  const int64_t my_row = row_blk + wave * 16 + (lane & 15);
  const int kq = lane >> 4;  // depth index of this lane inside an MFMA step

  double pr[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) pr[d] = my_row < nloc ? pts[(int64_t)d * n + my_row] : 0.0;

  typedef typename std::conditional<sizeof(T) == 8, d4, f4>::type acc_t;
  acc_t acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = (acc_t){0, 0, 0, 0};
  // FP32: the matrix core accumulates one chunk of KCH k-blocks (64
  // points) into a fresh accumulator; chunk sums are added into (sum, cmp)
  // with Kahan's compensated summation, so the rounding error of the
  // accumulation stays near that of one chunk instead of growing with N
  // (plain FP32 accumulation over N = 32768 points loses about 1e-4 of a
  // row's magnitude)
  constexpr int NS = sizeof(T) == 4 ? NT : 1;
  constexpr int KCH = 64 / BK;  // k-blocks per 64-point chunk
  f4 sum[NS], cmp[NS];
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    sum[t] = (f4){0, 0, 0, 0};
    cmp[t] = (f4){0, 0, 0, 0};
  }

  // X k-block and point coordinates: fetched into registers one block ahead
  // (global latency overlaps the MFMA work), written to LDS after compute.
  constexpr int PER = (BK * BN) / 256;  // elements per thread (NT)
  T xr[PER];
  double pk = 0.0;
  // Out-of-range elements load from a clamped (valid, finite) address: the
  // kernel value of a depth beyond n is set to zero, and columns beyond
  // ncols are never stored, so nothing needs masking and the loads stay in
  // flight across the MFMA work of the current block.
  // Element q of a thread is X(k0 + tid % BK, col0 + tid / BK + q * 256 / BK)
  // (256 is a multiple of BK): the row is clamped once per fetch, each column
  // in 32 bits, and the address is one 32 x 32 -> 64-bit multiply-add
  // (column counts and leading dimensions are below 2^31).  Computed in
  // place, so no per-element offsets stay live across the k loop.
  static_assert(256 % BK == 0, "a thread's elements share one row");
  const int ldx32 = (int)ldx, nc32 = (int)ncols;
  auto fetch = [&](int64_t k0) {
    const int64_t gk = k0 + tid % BK;
    const T *__restrict__ xk = X + (gk < nloc ? gk : nloc - 1);
    const int cb = (int)col0 + tid / BK;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int gc = cb + q * (256 / BK);
      xr[q] = xk[(int64_t)(gc < nc32 ? gc : nc32 - 1) * ldx32];
    }
    {  // every thread loads (a clamped coordinate), so no branch splits the
       // block of instructions the loads are scheduled into; the first BK * DIM
       // keep theirs
      const int64_t gk = k0 + tid % BK;
      const int d = tid / BK < DIM ? tid / BK : DIM - 1;
      pk = pts[(int64_t)d * n + (gk < nloc ? gk : nloc - 1)];
    }
  };
  auto store_x = [&](int buf) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q;
      Xs[buf][e % BK][e / BK] = xr[q];
    }
  };

  // a dead tile (zero columns of X) skips the contraction and stores zeros
  const int64_t nk = live ? (nloc + BK - 1) / BK : 0;
  constexpr int KS = BK / 4;  // MFMA depth steps per k-block
  static_assert(KS >= 2, "the loads of the first step and the stores of the last are apart");

  // One k-block into the accumulators c.  The B fragments of the first
  // depth step and the block's coordinates are read from LDS before the
  // kernel values are computed, and each later step's fragments are read
  // between the previous step's MFMAs, so LDS latency hides under VALU
  // and matrix work.  The KS kernel evaluations are straight-line code (no
  // per-lane branches) so their dependency chains interleave; depths
  // beyond the instance are zeroed on the tail block only (a wave-uniform
  // branch).
  //   Where the next block's global loads and LDS stores go.  FP64 (4 depth
  // steps per block): the loads between the first step's MFMAs, the stores
  // between the last step's (62.2 TFLOP/s on the sphere against 57.0 with
  // the loads at the top of the block and the stores in a burst after the
  // MFMAs).  FP32 (8 steps, twice the elements per thread): at the top and
  // in a burst (83.4 against 79.1 TFLOP/s spread as in FP64, 79.5 spread
  // over two steps each).  After the last block the loads are issued too:
  // clamped addresses, and what they load goes to the idle buffer and is
  // never read, so no branch splits the instructions they are placed among.
  constexpr bool kSpread = sizeof(T) == 8;
  auto kblock = [&](int64_t kb, int buf, acc_t *c) {
    if constexpr (!kSpread) fetch((kb + 1) * BK);
    T bq[2][NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) bq[0][t] = Xs[buf][kq][t * 16 + (lane & 15)];
    double pk4[KS][DIM];
#pragma unroll
    for (int s4 = 0; s4 < KS; ++s4)
#pragma unroll
      for (int d = 0; d < DIM; ++d) pk4[s4][d] = Ps[buf][d][4 * s4 + kq];
    // keep the reads above the VALU work (the scheduler would otherwise
    // sink each read next to its use and expose the LDS latency)
    __builtin_amdgcn_sched_barrier(0);
    T av[KS];
#pragma unroll
    for (int s4 = 0; s4 < KS; ++s4) {
      double r2 = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const double df = pr[d] - pk4[s4][d];
        r2 += df * df;
      }
      if constexpr (sizeof(T) == 8)
        av[s4] = kval64<KER>(r2);
      else
        av[s4] = kval32<KER>((float)r2);
    }
    if ((kb + 1) * BK > nloc) {
#pragma unroll
      for (int s4 = 0; s4 < KS; ++s4)
        if (kb * BK + 4 * s4 + kq >= nloc) av[s4] = (T)0;
    }
#pragma unroll
    for (int s4 = 0; s4 < KS; ++s4) {
      if (s4 + 1 < KS) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
          bq[(s4 + 1) & 1][t] = Xs[buf][4 * (s4 + 1) + kq][t * 16 + (lane & 15)];
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if constexpr (sizeof(T) == 8)
          c[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s4], bq[s4 & 1][t], c[t], 0, 0, 0);
        else
          c[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s4], bq[s4 & 1][t], c[t], 0, 0, 0);
      }
      // the next step's reads spread over this step's MFMAs, one LDS read
      // (a pair of fragments) between every two, instead of in one burst
      // ahead of them: the LDS serves the four waves' reads while the matrix
      // cores run, not all at once (2 % faster in FP64, 1 % in FP32)
      if (kSpread && s4 == 0) {
        fetch((kb + 1) * BK);
#pragma unroll
        for (int i = 0; i < NT / 2; ++i) {
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
          __builtin_amdgcn_sched_group_barrier(0x020, 2, 0);  // two global loads
          __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);  // two MFMAs
        }
      } else if (s4 + 1 < KS) {
#pragma unroll
        for (int i = 0; i < NT / 2; ++i) {
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
          __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);  // two MFMAs
        }
      } else if (kSpread) {
        store_x(buf ^ 1);
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // one LDS store
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (!kSpread) store_x(buf ^ 1);
    if (kb + 1 < nk && tid < BK * DIM) Ps[buf ^ 1][tid / BK][tid % BK] = pk;
    __syncthreads();
  };

  fetch(0);
  store_x(0);
  if (tid < BK * DIM) Ps[0][tid / BK][tid % BK] = pk;
  __syncthreads();
  if constexpr (sizeof(T) == 8) {
    for (int64_t kb = 0; kb < nk; ++kb) kblock(kb, (int)(kb & 1), acc);
  } else {
    for (int64_t kc = 0; kc < nk; kc += KCH) {
      acc_t c[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) c[t] = (acc_t){0, 0, 0, 0};
#pragma unroll
      for (int u = 0; u < KCH; ++u)
        if (kc + u < nk) kblock(kc + u, u & 1, c);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float y = c[t][i] - cmp[t][i];
          const float u = sum[t][i] + y;
          cmp[t][i] = (u - sum[t][i]) - y;
          sum[t][i] = u;
        }
      }
    }
  }
  // D layout of the 16x16 tiles, column l%16 for lane l:
  //   FP32 16x16x4: item i -> row 4*(l/16) + i
  //   FP64 16x16x4: item i -> row 4*i + l/16   (rows interleaved by item)
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int64_t c = col0 + t * 16 + (lane & 15);
    if (c >= ncols) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rin = sizeof(T) == 8 ? 4 * i + kq : 4 * kq + i;
      const int64_t rr = row_blk + wave * 16 + rin;
      if constexpr (sizeof(T) == 8) {
        if (rr < nloc) Y[c * ldy + rr] = acc[t][i];
      } else {
        if (rr < nloc) Y[c * ldy + rr] = sum[t][i];
      }
    }
  }
}

template <typename T, int NT, int KER, int DIM>
void launch_nt(int64_t n, const double *pts, int64_t ncols, const T *X, int64_t ldx, T *Y,
               int64_t ldy, int32_t nitems, const KItem *items, int64_t split, hipStream_t s) {
  const int64_t bn = 16 * NT;
  const int64_t nct = (ncols + bn - 1) / bn;
  if (items) {
    kapply_kernel<T, NT, KER, DIM, true><<<(unsigned)(nitems * nct), 256, 0, s>>>(
        n, pts, ncols, X, ldx, Y, ldy, items, split);
  } else {
    // row blocks [split, split + nitems) (a slice), nitems <= 0: to the end
    const int64_t nb = (n + 63) / 64;
    const int64_t b0 = split > 0 ? split : 0;
    const int64_t cnt = nitems > 0 ? std::min<int64_t>(nitems, nb - b0) : nb - b0;
    if (cnt <= 0) return;
    dim3 g((unsigned)cnt, (unsigned)nct);
    kapply_kernel<T, NT, KER, DIM, false><<<g, 256, 0, s>>>(n, pts, ncols, X, ldx, Y, ldy,
                                                             nullptr, b0);
  }
}

template <typename T, int KER, int DIM>
void launch_dim(int nt, int64_t n, const double *pts, int64_t ncols, const T *X, int64_t ldx,
                T *Y, int64_t ldy, int32_t nitems, const KItem *items, int64_t split,
                hipStream_t s) {
#define HM_KAPPLY_NT(V)                                                              \
  case V:                                                                           \
    launch_nt<T, V, KER, DIM>(n, pts, ncols, X, ldx, Y, ldy, nitems, items, split, s); \
    break;
  switch (nt) {
    HM_KAPPLY_NT(2)
    HM_KAPPLY_NT(4)
    HM_KAPPLY_NT(6)
    HM_KAPPLY_NT(8)
    HM_KAPPLY_NT(10)
    HM_KAPPLY_NT(12)
    HM_KAPPLY_NT(14)
    default:
      launch_nt<T, 16, KER, DIM>(n, pts, ncols, X, ldx, Y, ldy, nitems, items, split, s);
  }
#undef HM_KAPPLY_NT
}

template <typename T, int KER>
void launch_ker(int nt, int dim, int64_t n, const double *pts, int64_t ncols, const T *X,
                int64_t ldx, T *Y, int64_t ldy, int32_t nitems, const KItem *items,
                int64_t split, hipStream_t s) {
  if (dim == 1)
    launch_dim<T, KER, 1>(nt, n, pts, ncols, X, ldx, Y, ldy, nitems, items, split, s);
  else if (dim == 2)
    launch_dim<T, KER, 2>(nt, n, pts, ncols, X, ldx, Y, ldy, nitems, items, split, s);
  else
    launch_dim<T, KER, 3>(nt, n, pts, ncols, X, ldx, Y, ldy, nitems, items, split, s);
}

void launch_any(int kernel, int nt, int dim, int64_t n, const double *pts, int64_t ncols,
                bool f32, const void *X, int64_t ldx, void *Y, int64_t ldy, int32_t nitems,
                const KItem *items, int64_t split, hipStream_t s) {
  if (nt <= 0) nt = kapply_default_nt(ncols, f32, nitems > 0 ? nitems : (n + 63) / 64);
  if (f32) {
    if (kernel == 0)
      launch_ker<float, 0>(nt, dim, n, pts, ncols, (const float *)X, ldx, (float *)Y, ldy, nitems,
                           items, split, s);
    else
      launch_ker<float, 1>(nt, dim, n, pts, ncols, (const float *)X, ldx, (float *)Y, ldy, nitems,
                           items, split, s);
  } else {
    if (kernel == 0)
      launch_ker<double, 0>(nt, dim, n, pts, ncols, (const double *)X, ldx, (double *)Y, ldy,
                            nitems, items, split, s);
    else
      launch_ker<double, 1>(nt, dim, n, pts, ncols, (const double *)X, ldx, (double *)Y, ldy,
                            nitems, items, split, s);
  }
}

}  // namespace

// Tile width without timing: columns come in 16-wide fragments; a tile of
// nt fragments evaluates the kernel once for its nt fragments of MFMA work,
// which costs about as much as two more fragments, so a launch costs about
// tiles * (nt + 2); a grid of fewer than two workgroups per CU (512) leaves
// CUs idle and is charged for it.  nt is capped where the accumulators
// would drop the occupancy to one wave per SIMD (FP64: 12, FP32 with its
// compensated sums and 32-point k-blocks: 6).
int kapply_default_nt(int64_t ncols, bool f32, int64_t units) {
  const int cap = f32 ? 6 : 12;
  const int64_t frags = (ncols + 15) / 16;
  int best = 2;
  double best_cost = 1e300;
  for (int nt = 2; nt <= cap; nt += 2) {
    const int64_t tiles = (frags + nt - 1) / nt;
    const double fill = std::min(1.0, (double)(std::max<int64_t>(units, 1) * tiles) / 512.0);
    const double cost = (double)tiles * (nt + 2) / fill;
    if (cost <= best_cost) {
      best_cost = cost;
      best = nt;
    }
  }
  return best;
}

void launch_kapply(int kernel, int dim, int64_t n, const double *pts, int64_t ncols, int nt,
                   bool f32, const void *X, int64_t ldx, void *Y, int64_t ldy, hipStream_t s,
                   int64_t rows, int64_t row0) {
  if (n <= 0 || ncols <= 0 || row0 < 0 || row0 >= n) return;
  // rows of a slice start on a 64-row block
  const int64_t b0 = row0 / 64;
  const int32_t nblk = rows > 0 ? (int32_t)((std::min(rows, n - b0 * 64) + 63) / 64) : 0;
  launch_any(kernel, nt, dim, n, pts, ncols, f32, X, ldx, Y, ldy, nblk, nullptr, b0, s);
}

void launch_kapply_forest(int kernel, int dim, int64_t n, const double *pts, int32_t nitems,
                          const KItem *items, int64_t ncols, int64_t split, int nt, bool f32,
                          const void *X, int64_t ldx, void *Y, int64_t ldy, hipStream_t s) {
  if (n <= 0 || ncols <= 0 || nitems <= 0) return;
  launch_any(kernel, nt, dim, n, pts, ncols, f32, X, ldx, Y, ldy, nitems, items, split, s);
}

}  // namespace hm
