// H^2 apply (alg:apply_h2_level_truncated): outgoing expansions of the
// boxes that hold long bases (q = V* x on their rows), the upward pass
// through the transfer matrices, the couplings and the downward pass
// (u_a = sum_b B_ab q_b + T_a u_parent), and the expansion y += U u on the
// rows of the boxes with long bases.  Expansions are FP64, kmax x ncols per
// box (ld kmax), at QH / UH + box * kmax * ldq; X and Y are FP64 or FP32.
// Every output element is owned by one thread: no atomics, deterministic.
#include "device_common.h"
#include "kernels.h"

namespace hm {

namespace {

constexpr int HC = 64;  // columns per workgroup

// q_b(0:k, c) = sum_{i < m} V_b(i, 0:k) x(row0 + i, c): one workgroup per
// (box, 64-column tile); rows staged 64 at a time through LDS.
template <typename T>
__global__ void __launch_bounds__(256)
h2_project_kernel(const H2Leaf *__restrict__ jobs, int32_t kmax, const int32_t *__restrict__ rank,
                  const double *__restrict__ VB, const T *__restrict__ X, int64_t ldx,
                  int64_t ncols, double *__restrict__ QH, int64_t ldq) {
  __shared__ double Vs[64][65];  // [row][basis column]
  __shared__ double Xs[64][HC + 1];
  const H2Leaf job = jobs[blockIdx.x];
  const int64_t c0 = (int64_t)blockIdx.y * HC;
  const int tid = threadIdx.x;
  const int k = rank[job.g];
  const int cc = tid & 63, ig = tid >> 6;  // column, basis-column group
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  for (int r0 = 0; r0 < job.m; r0 += 64) {
    const int rows = job.m - r0 < 64 ? job.m - r0 : 64;
    for (int e = tid; e < 64 * 64; e += 256) {
      const int i = e % 64, j = e / 64;
      Vs[i][j] = (i < rows && j < k) ? VB[job.boff + (int64_t)j * job.m + r0 + i] : 0.0;
      const int64_t gc = c0 + j;
      Xs[i][j] = (i < rows && gc < ncols) ? (double)X[gc * ldx + job.row0 + r0 + i] : 0.0;
    }
    __syncthreads();
    for (int i = 0; i < rows; ++i) {
      const double xv = Xs[i][cc];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] += Vs[i][ig + 4 * q] * xv;
    }
    __syncthreads();
  }
  const int64_t gc = c0 + cc;
  if (gc < ncols) {
    double *o = QH + (int64_t)job.g * kmax * ldq + gc * kmax;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int j = ig + 4 * q;
      if (j < kmax) o[j] = j < k ? acc[q] : 0.0;
    }
  }
}

// Small sums of products: out(0:ko, c) = sum_t M_t(0:ko, 0:kt) in_t(0:kt, c),
// M_t stored k x k (ld kmax) or transposed (trans), for the terms of one job:
// the transfers of the upward pass, or the couplings and the parent term of
// the downward pass.  Ranks: ko from rank_o, kt from rank_i (rank_o for a
// parent term, whose input is an incoming expansion).  One thread per
// (row, column).
__global__ void __launch_bounds__(256)
h2_sum_kernel(const H2Sum *__restrict__ jobs, const H2Term *__restrict__ terms, int32_t kmax,
              const int32_t *__restrict__ rank_o, const int32_t *__restrict__ rank_i,
              const double *__restrict__ Mpool, const double *__restrict__ Mpar,
              const double *__restrict__ IN, const double *__restrict__ PAR,
              double *__restrict__ OUT, int64_t ldq, int64_t ncols) {
  const H2Sum job = jobs[blockIdx.x];
  const int64_t c0 = (int64_t)blockIdx.y * HC;
  const int ko = rank_o[job.g];
  for (int e = threadIdx.x; e < kmax * HC; e += 256) {
    const int i = e % kmax, cl = e / kmax;
    const int64_t gc = c0 + cl;
    if (gc >= ncols) continue;
    double s = 0.0;
    if (i < ko) {
      for (int t = job.t0; t < job.t1; ++t) {
        const H2Term tm = terms[t];
        const int kt = tm.parent ? rank_o[tm.src] : rank_i[tm.src];
        const double *M = (tm.parent ? Mpar : Mpool) + tm.moff;
        const double *in = (tm.parent ? PAR : IN) + (int64_t)tm.src * kmax * ldq + gc * kmax;
        if (tm.trans)
          for (int j = 0; j < kt; ++j) s += M[(int64_t)i * kmax + j] * in[j];
        else
          for (int j = 0; j < kt; ++j) s += M[(int64_t)j * kmax + i] * in[j];
      }
    }
    OUT[(int64_t)job.g * kmax * ldq + gc * kmax + i] = s;
  }
}

// y(row0 + r, c) (+)= sum_j U_a(r, j) u_a(j, c) for one 64-row chunk of a box.
template <typename T>
__global__ void __launch_bounds__(256)
h2_expand_kernel(const H2Leaf *__restrict__ jobs, int32_t kmax, const int32_t *__restrict__ rank,
                 const double *__restrict__ UB, const double *__restrict__ UH, int64_t ldq,
                 int64_t ncols, T *__restrict__ Y, int64_t ldy) {
  __shared__ double Us[64][65];   // [row][j]
  __shared__ double Hs[64][HC + 1];  // [j][column]
  const H2Leaf job = jobs[blockIdx.x];
  const int64_t c0 = (int64_t)blockIdx.y * HC;
  const int tid = threadIdx.x;
  const int k = rank[job.g];
  const int rows = job.m - job.r0 < 64 ? job.m - job.r0 : 64;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int i = e % 64, j = e / 64;
    Us[i][j] = (i < rows && j < k) ? UB[job.boff + (int64_t)j * job.m + job.r0 + i] : 0.0;
    const int64_t gc = c0 + i;  // i as the column here
    Hs[j][i] = (j < k && gc < ncols) ? UH[(int64_t)job.g * kmax * ldq + gc * kmax + j] : 0.0;
  }
  __syncthreads();
  const int cc = tid & 63, rg = tid >> 6;
  const int64_t gc = c0 + cc;
  if (gc >= ncols) return;
  for (int q = 0; q < 16; ++q) {
    const int r = rg + 4 * q;
    if (r >= rows) break;
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += Us[r][j] * Hs[j][cc];
    T *y = Y + gc * ldy + job.row0 + job.r0 + r;
    *y = (T)((double)*y + s);
  }
}

}  // namespace

void launch_h2_project(int32_t njobs, const H2Leaf *jobs, int32_t kmax, const int32_t *rank,
                       const double *VB, bool f32, const void *X, int64_t ldx, int64_t ncols,
                       double *QH, int64_t ldq, hipStream_t s) {
  if (njobs <= 0 || ncols <= 0 || kmax > 64) return;
  dim3 g(njobs, (unsigned)((ncols + HC - 1) / HC));
  if (f32)
    h2_project_kernel<float><<<g, 256, 0, s>>>(jobs, kmax, rank, VB, (const float *)X, ldx, ncols,
                                               QH, ldq);
  else
    h2_project_kernel<double><<<g, 256, 0, s>>>(jobs, kmax, rank, VB, (const double *)X, ldx,
                                                ncols, QH, ldq);
}

void launch_h2_sum(int32_t njobs, const H2Sum *jobs, const H2Term *terms, int32_t kmax,
                   const int32_t *rank_o, const int32_t *rank_i, const double *Mpool,
                   const double *Mpar, const double *IN, const double *PAR, double *OUT,
                   int64_t ldq, int64_t ncols, hipStream_t s) {
  if (njobs <= 0 || ncols <= 0) return;
  dim3 g(njobs, (unsigned)((ncols + HC - 1) / HC));
  h2_sum_kernel<<<g, 256, 0, s>>>(jobs, terms, kmax, rank_o, rank_i, Mpool, Mpar, IN, PAR, OUT,
                                  ldq, ncols);
}

void launch_h2_expand(int32_t njobs, const H2Leaf *jobs, int32_t kmax, const int32_t *rank,
                      const double *UB, const double *UH, int64_t ldq, bool f32, int64_t ncols,
                      void *Y, int64_t ldy, hipStream_t s) {
  if (njobs <= 0 || ncols <= 0 || kmax > 64) return;
  dim3 g(njobs, (unsigned)((ncols + HC - 1) / HC));
  if (f32)
    h2_expand_kernel<float><<<g, 256, 0, s>>>(jobs, kmax, rank, UB, UH, ldq, ncols, (float *)Y,
                                              ldy);
  else
    h2_expand_kernel<double><<<g, 256, 0, s>>>(jobs, kmax, rank, UB, UH, ldq, ncols,
                                               (double *)Y, ldy);
}

}  // namespace hm
