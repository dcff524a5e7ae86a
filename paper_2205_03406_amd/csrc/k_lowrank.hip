// Grouped low-rank products for the peeling subtraction and the H^1 apply:
//   project  T_p = R_p^T X(col box)            (one job per admissible pair)
//   expand   Y(row chunk) += sign * sum_p L_p(chunk rows) T_p
//   near     Y(row chunk) += sum_q D_q(chunk rows) X(col box of q)
// and the dense FP64 GEMM behind the dense test black box.
//
// Every output row chunk is owned by one workgroup, which sums all of its
// contributions in registers before a single read-modify-write of Y: the
// result is deterministic (no atomics) and each Y element is written once
// per call.  Tiles are 64 rows x 64 columns, K staged through LDS in chunks
// of 32; FP64 (or FP32 in the mixed path) on the vector ALUs.
#include "device_common.h"
#include "kernels.h"

namespace hm {

namespace {

constexpr int TC = 64;  // columns per workgroup
constexpr int KC = 32;  // contraction chunk

template <typename T>
__global__ void __launch_bounds__(256)
lr_project_kernel(const ProjItem *__restrict__ items, const ProjPair *__restrict__ pairs,
                  int32_t kmax, int64_t tstride, const int32_t *__restrict__ ranks,
                  const T *__restrict__ R, const T *__restrict__ X, int64_t ldx, int64_t ncols,
                  T *__restrict__ Tout) {
  __shared__ T Rs[2][KC][64 + 1];   // [row][pair*kmax + kk]
  __shared__ T Xs[2][KC][TC + 1];   // [row][col]
  __shared__ int64_t rsl[64];
  __shared__ int kk_of[64];
  const ProjItem it = items[blockIdx.x];
  const int64_t c0 = (int64_t)blockIdx.y * TC;
  const int tid = threadIdx.x;
  const int col = tid & 63, g = tid >> 6;
  const int nout = it.npairs * kmax;  // output rows of this group (<= 64)
  if (tid < 64) {
    const int j = tid / kmax, kk = tid % kmax;
    int k = 0;
    int64_t rs = 0;
    if (j < it.npairs) {
      const ProjPair pp = pairs[it.first + j];
      k = ranks[pp.kidx];
      rs = pp.rslot + it.seg_off;
    }
    rsl[tid] = rs;
    kk_of[tid] = (j < it.npairs && kk < k) ? kk : -1;
  }
  __syncthreads();
  T acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0;
  T rr_[8], xr_[8];
  auto fetch = [&](int r0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + 256 * q;
      const int rr = e % KC, o = e / KC;
      const int row = r0 + rr;
      const int kk = kk_of[o];
      rr_[q] = (row < it.nrows && kk >= 0) ? R[rsl[o] + (int64_t)kk * it.m + row] : (T)0;
      const int64_t gc = c0 + o;
      xr_[q] = (row < it.nrows && gc < ncols) ? X[gc * ldx + it.row0 + row] : (T)0;
    }
  };
  auto commit = [&](int b) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + 256 * q;
      Rs[b][e % KC][e / KC] = rr_[q];
      Xs[b][e % KC][e / KC] = xr_[q];
    }
  };
  fetch(0);
  commit(0);
  __syncthreads();
  int b = 0;
  for (int r0 = 0; r0 < it.nrows; r0 += KC) {
    const bool more = r0 + KC < it.nrows;
    if (more) fetch(r0 + KC);
#pragma unroll 4
    for (int rr = 0; rr < KC; ++rr) {
      const T xv = Xs[b][rr][col];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] += Rs[b][rr][g + 4 * q] * xv;
    }
    if (more) commit(b ^ 1);
    __syncthreads();
    b ^= 1;
  }
  const int64_t gc = c0 + col;
  if (gc < ncols) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int o = g + 4 * q;
      if (o < nout && kk_of[o] >= 0) {
        const ProjPair pp = pairs[it.first + o / kmax];
        Tout[(int64_t)pp.tslot * tstride + gc * kmax + kk_of[o]] = acc[q];
      }
    }
  }
}

// All entries of a chunk form one contraction: their rank columns are laid
// end to end (prefix sums in LDS), so a 32-deep stage mixes several pairs and
// no stage waits on a single entry's descriptor.  The next stage is fetched
// into registers while the current one is multiplied.
constexpr int EMAX = 256;  // entries handled per pass over a chunk

template <typename T>
__global__ void __launch_bounds__(256)
lr_expand_kernel(const ExpandChunk *__restrict__ chunks, const ExpandEntry *__restrict__ entries,
                 int32_t kmax, int64_t tstride, const int32_t *__restrict__ ranks,
                 const T *__restrict__ L, const T *__restrict__ Tin, int64_t ncols, T sign,
                 T *__restrict__ Y, int64_t ldy) {
  __shared__ T Ls[2][KC][64 + 1];   // [kk][row]
  __shared__ T Ts[2][KC][TC + 1];   // [kk][col]
  __shared__ int64_t e_l[EMAX];      // lslot + off
  __shared__ int32_t e_mq[EMAX], e_k[EMAX], e_ts[EMAX], e_ns[EMAX], e_ko[EMAX + 1];
  const ExpandChunk ch = chunks[blockIdx.x];
  const int64_t c0 = (int64_t)blockIdx.y * TC;
  const int tid = threadIdx.x;
  const int col = tid & 63, g = tid >> 6;
  T acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0;

  for (int e0 = ch.first; e0 < ch.last; e0 += EMAX) {
    const int ne = min(EMAX, ch.last - e0);
    if (tid < ne) {
      const ExpandEntry en = entries[e0 + tid];
      e_l[tid] = en.lslot + en.off;
      e_mq[tid] = en.mq;
      e_k[tid] = ranks[en.kidx];
      e_ts[tid] = en.tslot;
      e_ns[tid] = en.nseg;
    }
    __syncthreads();
    if (tid == 0) {
      int acc_k = 0;
      for (int i = 0; i < ne; ++i) {
        e_ko[i] = acc_k;
        acc_k += e_k[i];
      }
      e_ko[ne] = acc_k;
    }
    __syncthreads();
    const int ktot = e_ko[ne];
    // stage element ownership: 8 L elements and 8 T elements per thread
    T lr[8], tr[8];
    auto fetch = [&](int k0) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int e = tid + 256 * q;
        // L: (row rr, depth kk); T: (depth kt, column cc)
        const int rr = e % 64, kk = e / 64;
        const int kt = e % KC, cc = e / KC;
        lr[q] = 0;
        tr[q] = 0;
        int kg = k0 + kk;
        if (kg < ktot && rr < ch.nrows) {
          int lo = 0, hi = ne - 1;  // entry holding depth kg
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (e_ko[mid] <= kg) lo = mid; else hi = mid - 1;
          }
          lr[q] = L[e_l[lo] + (int64_t)(kg - e_ko[lo]) * e_mq[lo] + rr];
        }
        kg = k0 + kt;
        const int64_t gc = c0 + cc;
        if (kg < ktot && gc < ncols) {
          int lo = 0, hi = ne - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (e_ko[mid] <= kg) lo = mid; else hi = mid - 1;
          }
          const T *tp = Tin + (int64_t)e_ts[lo] * tstride + gc * kmax + (kg - e_ko[lo]);
          T t = 0;
          for (int sg = 0; sg < e_ns[lo]; ++sg) t += tp[(int64_t)sg * tstride];
          tr[q] = t;
        }
      }
    };
    auto commit = [&](int b) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int e = tid + 256 * q;
        Ls[b][e / 64][e % 64] = lr[q];
        Ts[b][e % KC][e / KC] = tr[q];
      }
    };
    if (ktot > 0) {
      fetch(0);
      commit(0);
      __syncthreads();
      int b = 0;
      for (int k0 = 0; k0 < ktot; k0 += KC) {
        const bool more = k0 + KC < ktot;
        if (more) fetch(k0 + KC);
#pragma unroll 4
        for (int kk = 0; kk < KC; ++kk) {
          const T tv = Ts[b][kk][col];
#pragma unroll
          for (int q = 0; q < 16; ++q) acc[q] += Ls[b][kk][g + 4 * q] * tv;
        }
        if (more) commit(b ^ 1);
        __syncthreads();
        b ^= 1;
      }
    }
  }
  const int64_t gc = c0 + col;
  if (gc < ncols) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int rr = g + 4 * q;
      if (rr < ch.nrows) {
        T *y = Y + gc * ldy + ch.row0 + rr;
        *y += sign * acc[q];
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
near_kernel(const ExpandChunk *__restrict__ chunks, const NearEntry *__restrict__ entries,
            const double *__restrict__ D, const T *__restrict__ X, int64_t ldx, int64_t ncols,
            T *__restrict__ Y, int64_t ldy) {
  __shared__ T Ds[KC][64 + 1];   // [kk][row]
  __shared__ T Xs[KC][TC + 1];   // [kk][col]
  const ExpandChunk ch = chunks[blockIdx.x];
  const int64_t c0 = (int64_t)blockIdx.y * TC;
  const int tid = threadIdx.x;
  const int col = tid & 63, g = tid >> 6;
  T acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0;
  for (int ei = ch.first; ei < ch.last; ++ei) {
    const NearEntry en = entries[ei];
    const double *Dp = D + en.dslot;
    for (int k0 = 0; k0 < en.mb; k0 += KC) {
      for (int e = tid; e < KC * 64; e += 256) {
        const int rr = e % 64, kk = e / 64;
        Ds[kk][rr] = (rr < ch.nrows && k0 + kk < en.mb)
                         ? (T)Dp[(int64_t)(k0 + kk) * en.ma + en.off + rr] : (T)0;
        const int kt = e % KC, cc = e / KC;
        const int64_t gc = c0 + cc;
        Xs[kt][cc] = (k0 + kt < en.mb && gc < ncols) ? X[gc * ldx + en.xrow0 + k0 + kt] : (T)0;
      }
      __syncthreads();
#pragma unroll 4
      for (int kk = 0; kk < KC; ++kk) {
        const T xv = Xs[kk][col];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] += Ds[kk][g + 4 * q] * xv;
      }
      __syncthreads();
    }
  }
  const int64_t gc = c0 + col;
  if (gc < ncols) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int rr = g + 4 * q;
      if (rr < ch.nrows) Y[gc * ldy + ch.row0 + rr] += acc[q];
    }
  }
}

// Y = op(A) X, 64 x 64 output tiles, A FP64 column-major
__global__ void __launch_bounds__(256)
dense_gemm_kernel(int64_t n, const double *__restrict__ A, int64_t lda, int trans, int64_t ncols,
                  const double *__restrict__ X, int64_t ldx, double *__restrict__ Y, int64_t ldy) {
  __shared__ double As[KC][64 + 1];  // [kk][row]
  __shared__ double Xs[KC][TC + 1];  // [kk][col]
  const int64_t r0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * TC;
  const int tid = threadIdx.x;
  const int col = tid & 63, g = tid >> 6;
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0;
  for (int64_t k0 = 0; k0 < n; k0 += KC) {
    for (int e = tid; e < KC * 64; e += 256) {
      int rr, kk;
      if (trans) {
        kk = e % KC;
        rr = e / KC;
      } else {
        rr = e % 64;
        kk = e / 64;
      }
      const int64_t gr = r0 + rr, gk = k0 + kk;
      double v = 0.0;
      if (gr < n && gk < n) v = trans ? A[gr * lda + gk] : A[gk * lda + gr];
      As[kk][rr] = v;
      const int kt = e % KC, cc = e / KC;
      const int64_t gc = c0 + cc;
      Xs[kt][cc] = (k0 + kt < n && gc < ncols) ? X[gc * ldx + k0 + kt] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < KC; ++kk) {
      const double xv = Xs[kk][col];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] += As[kk][g + 4 * q] * xv;
    }
    __syncthreads();
  }
  const int64_t gc = c0 + col;
  if (gc < ncols) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int64_t gr = r0 + g + 4 * q;
      if (gr < n) Y[gc * ldy + gr] = acc[q];
    }
  }
}

inline unsigned col_tiles(int64_t ncols) { return (unsigned)((ncols + TC - 1) / TC); }

}  // namespace

void launch_lr_project(int32_t nitems, const ProjItem *items, const ProjPair *pairs, int32_t kmax,
                       int64_t tstride, const int32_t *ranks, bool f32, const void *R,
                       const void *X, int64_t ldx, int64_t ncols, void *T, hipStream_t s) {
  if (nitems <= 0 || ncols <= 0) return;
  dim3 g(nitems, col_tiles(ncols));
  if (f32)
    lr_project_kernel<float><<<g, 256, 0, s>>>(items, pairs, kmax, tstride, ranks,
                                               (const float *)R, (const float *)X, ldx, ncols,
                                               (float *)T);
  else
    lr_project_kernel<double><<<g, 256, 0, s>>>(items, pairs, kmax, tstride, ranks,
                                                (const double *)R, (const double *)X, ldx, ncols,
                                                (double *)T);
}

void launch_lr_expand(int32_t nchunks, const ExpandChunk *chunks, const ExpandEntry *entries,
                      int32_t kmax, int64_t tstride, const int32_t *ranks, bool f32,
                      const void *L, const void *T, int64_t ncols, double sign, void *Y,
                      int64_t ldy, hipStream_t s) {
  if (nchunks <= 0 || ncols <= 0) return;
  dim3 g(nchunks, col_tiles(ncols));
  if (f32)
    lr_expand_kernel<float><<<g, 256, 0, s>>>(chunks, entries, kmax, tstride, ranks,
                                              (const float *)L, (const float *)T, ncols,
                                              (float)sign, (float *)Y, ldy);
  else
    lr_expand_kernel<double><<<g, 256, 0, s>>>(chunks, entries, kmax, tstride, ranks,
                                               (const double *)L, (const double *)T, ncols, sign,
                                               (double *)Y, ldy);
}

void launch_near_apply(int32_t nchunks, const ExpandChunk *chunks, const NearEntry *entries,
                       bool f32, const void *D, const void *X, int64_t ldx, int64_t ncols,
                       void *Y, int64_t ldy, hipStream_t s) {
  if (nchunks <= 0 || ncols <= 0) return;
  dim3 g(nchunks, col_tiles(ncols));
  if (f32)
    near_kernel<float><<<g, 256, 0, s>>>(chunks, entries, (const double *)D, (const float *)X, ldx,
                                         ncols, (float *)Y, ldy);
  else
    near_kernel<double><<<g, 256, 0, s>>>(chunks, entries, (const double *)D, (const double *)X,
                                          ldx, ncols, (double *)Y, ldy);
}

void launch_dense_gemm(int64_t n, const double *A, int64_t lda, bool trans, int64_t ncols,
                       const double *X, int64_t ldx, double *Y, int64_t ldy, hipStream_t s) {
  if (n <= 0 || ncols <= 0) return;
  dim3 g((unsigned)((n + 63) / 64), col_tiles(ncols));
  dense_gemm_kernel<<<g, 256, 0, s>>>(n, A, lda, trans ? 1 : 0, ncols, X, ldx, Y, ldy);
}

}  // namespace hm
