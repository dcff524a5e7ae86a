// Uniform H^1 kernels (section on uniform H^1 compression): the stage-2
// test matrix assembled from the stage-1 column bases, and the randomized
// combination of a box's sample blocks whose basis is the box's row basis.
// Both are HBM-bound and coalesced along the column-major row index.
#include "device_common.h"
#include "kernels.h"

namespace hm {

namespace {

template <typename T>
__global__ void __launch_bounds__(256)
basis_testmat_kernel(int64_t n, const int32_t *__restrict__ rowbox,
                     const int64_t *__restrict__ box_start, const int32_t *__restrict__ slot,
                     int32_t ncolors, int32_t kmax, const double *__restrict__ UB,
                     const int64_t *__restrict__ uoff, const int32_t *__restrict__ urank,
                     T *__restrict__ out, int64_t ld) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t col = blockIdx.y;
  const int c = (int)(col / kmax), j = (int)(col % kmax);
  double v = 0.0;
  if (c < ncolors) {
    const int b = rowbox[i];
    const int u = slot[(int64_t)b * ncolors + c] - 1;
    if (u >= 0 && j < urank[u]) {
      const int64_t s0 = box_start[b], m = box_start[b + 1] - s0;
      v = UB[uoff[u] + (int64_t)j * m + (i - s0)];
    }
  }
  out[col * ld + i] = (T)v;
}

// One workgroup per job (a chunk of <= 256 rows of one box), one row per
// thread, kmax accumulators per thread.  Per term, Gamma is drawn into LDS
// by the whole workgroup (kmax * ceil(kmax/2) Philox draws), then every row
// takes its kmax x kmax product with the term's Z block.
template <typename T>
__global__ void __launch_bounds__(256)
mix_sum_kernel(const MixJob *__restrict__ jobs, const MixTerm *__restrict__ terms, int32_t kmax,
               int32_t level, uint64_t seed, const T *__restrict__ Z, int64_t ldz,
               double *__restrict__ S, int64_t lds) {
  __shared__ double G[64 * 64];
  const MixJob job = jobs[blockIdx.x];
  const int tid = threadIdx.x;
  const int npair = (kmax + 1) / 2;
  double acc[64];
#pragma unroll
  for (int j = 0; j < 64; ++j) acc[j] = 0.0;
  for (int t = job.t0; t < job.t1; ++t) {
    const MixTerm tm = terms[t];
    const uint64_t key = seed + (uint64_t)tm.inst;
    for (int e = tid; e < kmax * npair; e += 256) {
      const int i = e / npair, jj = e % npair;
      dev::U4 ctr{tm.grow, (uint32_t)jj, (uint32_t)i, (uint32_t)(4 * level + 3)};
      double z0, z1;
      dev::normal_pair(dev::philox10(ctr, (uint32_t)key, (uint32_t)(key >> 32)), z0, z1);
      G[i * 64 + 2 * jj] = z0;
      if (2 * jj + 1 < kmax) G[i * 64 + 2 * jj + 1] = z1;
    }
    __syncthreads();
    if (tid < job.m) {
      const T *zr = Z + tm.zcol0 * ldz + job.row0 + tid;
      for (int i = 0; i < kmax; ++i) {
        const double z = (double)zr[(int64_t)i * ldz];
#pragma unroll
        for (int j = 0; j < 64; ++j)
          if (j < kmax) acc[j] += z * G[i * 64 + j];
      }
    }
    __syncthreads();
  }
  if (tid < job.m) {
#pragma unroll
    for (int j = 0; j < 64; ++j)
      if (j < kmax) S[(int64_t)j * lds + job.row0 + tid] = acc[j];
  }
}

}  // namespace

void launch_basis_testmat(int64_t n, const int32_t *rowbox, const int64_t *box_start,
                          const int32_t *slot, int32_t ncolors, int32_t kmax, const double *UB,
                          const int64_t *uoff, const int32_t *urank, bool f32, void *out,
                          int64_t ld, int64_t ncols_pad, hipStream_t s) {
  if (n <= 0 || ncols_pad <= 0 || kmax <= 0) return;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)ncols_pad);
  if (f32)
    basis_testmat_kernel<float><<<grid, 256, 0, s>>>(n, rowbox, box_start, slot, ncolors, kmax,
                                                     UB, uoff, urank, (float *)out, ld);
  else
    basis_testmat_kernel<double><<<grid, 256, 0, s>>>(n, rowbox, box_start, slot, ncolors, kmax,
                                                      UB, uoff, urank, (double *)out, ld);
}

void launch_mix_sum(int32_t njobs, const MixJob *jobs, const MixTerm *terms, int32_t kmax,
                    int32_t level, uint64_t seed, bool f32, const void *Z, int64_t ldz, double *S,
                    int64_t lds, hipStream_t s) {
  if (njobs <= 0 || kmax <= 0 || kmax > 64) return;
  if (f32)
    mix_sum_kernel<float><<<njobs, 256, 0, s>>>(jobs, terms, kmax, level, seed, (const float *)Z,
                                                ldz, S, lds);
  else
    mix_sum_kernel<double><<<njobs, 256, 0, s>>>(jobs, terms, kmax, level, seed,
                                                 (const double *)Z, ldz, S, lds);
}

}  // namespace hm
