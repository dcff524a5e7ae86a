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
lr_project_kernel(const ProjJob *__restrict__ jobs, int32_t kmax, int64_t tstride,
                  const int32_t *__restrict__ ranks, const T *__restrict__ R,
                  const T *__restrict__ X, int64_t ldx, int64_t ncols, T *__restrict__ Tout) {
  __shared__ T Rs[KC][TC + 1];
  __shared__ T Xs[KC][TC + 1];
  const ProjJob job = jobs[blockIdx.x];
  const int k = ranks[job.kidx], m = job.m;
  if (k <= 0) return;
  const int64_t c0 = (int64_t)blockIdx.y * TC;
  const int tid = threadIdx.x;
  const int col = tid & 63, g = tid >> 6;
  T acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0;
  const T *Rp = R + job.rslot;
  for (int r0 = 0; r0 < m; r0 += KC) {
    for (int e = tid; e < KC * TC; e += 256) {
      const int rr = e % KC, cc = e / KC;
      const int row = r0 + rr;
      Rs[rr][cc] = (row < m && cc < k) ? Rp[(int64_t)cc * m + row] : (T)0;
      const int64_t gc = c0 + cc;
      Xs[rr][cc] = (row < m && gc < ncols) ? X[gc * ldx + job.row0 + row] : (T)0;
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < KC; ++rr) {
      const T xv = Xs[rr][col];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] += Rs[rr][g + 4 * q] * xv;
    }
    __syncthreads();
  }
  const int64_t gc = c0 + col;
  if (gc < ncols) {
    T *Tp = Tout + (int64_t)job.tidx * tstride + gc * kmax;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int kk = g + 4 * q;
      if (kk < k) Tp[kk] = acc[q];
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
lr_expand_kernel(const ExpandChunk *__restrict__ chunks, const ExpandEntry *__restrict__ entries,
                 int32_t kmax, int64_t tstride, const int32_t *__restrict__ ranks,
                 const T *__restrict__ L, const T *__restrict__ Tin, int64_t ncols, T sign,
                 T *__restrict__ Y, int64_t ldy) {
  __shared__ T Ls[KC][64 + 1];   // [kk][row]
  __shared__ T Ts[KC][TC + 1];   // [kk][col]
  const ExpandChunk ch = chunks[blockIdx.x];
  const int64_t c0 = (int64_t)blockIdx.y * TC;
  const int tid = threadIdx.x;
  const int col = tid & 63, g = tid >> 6;
  T acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0;
  for (int ei = ch.first; ei < ch.last; ++ei) {
    const ExpandEntry en = entries[ei];
    const T *Lp = L + en.lslot;
    const T *Tp = Tin + (int64_t)en.tidx * tstride;
    const int kq = ranks[en.kidx];
    for (int k0 = 0; k0 < kq; k0 += KC) {
      for (int e = tid; e < KC * 64; e += 256) {
        const int rr = e % 64, kk = e / 64;
        Ls[kk][rr] = (rr < ch.nrows && k0 + kk < kq)
                         ? Lp[(int64_t)(k0 + kk) * en.mq + en.off + rr] : (T)0;
        const int kt = e % KC, cc = e / KC;
        const int64_t gc = c0 + cc;
        Ts[kt][cc] = (k0 + kt < kq && gc < ncols) ? Tp[gc * kmax + k0 + kt] : (T)0;
      }
      __syncthreads();
#pragma unroll 4
      for (int kk = 0; kk < KC; ++kk) {
        const T tv = Ts[kk][col];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] += Ls[kk][g + 4 * q] * tv;
      }
      __syncthreads();
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

void launch_lr_project(int32_t njobs, const ProjJob *jobs, int32_t kmax, int64_t tstride,
                       const int32_t *ranks, bool f32, const void *R, const void *X, int64_t ldx,
                       int64_t ncols, void *T, hipStream_t s) {
  if (njobs <= 0 || ncols <= 0) return;
  dim3 g(njobs, col_tiles(ncols));
  if (f32)
    lr_project_kernel<float><<<g, 256, 0, s>>>(jobs, kmax, tstride, ranks, (const float *)R,
                                               (const float *)X, ldx, ncols, (float *)T);
  else
    lr_project_kernel<double><<<g, 256, 0, s>>>(jobs, kmax, tstride, ranks, (const double *)R,
                                                (const double *)X, ldx, ncols, (double *)T);
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
