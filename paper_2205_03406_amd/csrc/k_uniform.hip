// Uniform H^1 and H^2 kernels (sections on uniform H^1 and on H^2
// compression): the stage-2 test matrix assembled from the stage-1 column
// bases, the sum of a box's sample blocks whose basis is the box's row
// basis (or, as an extension, a Gaussian-weighted combination), the parent
// augmentation of H^2 samples and the
// nesting of bases through transfer matrices.  All are row-parallel (one
// row per thread, coalesced along the column-major row index).
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

// Row-basis sample of a box: the sum of the box's Z blocks over its
// interaction list (alg:h2_pseudocode, "sum samples"), in term order.  One
// workgroup per job (a chunk of <= 256 rows of one box), one row per
// thread, kmax FP64 accumulators per thread.
template <typename T>
__global__ void __launch_bounds__(256)
sum_blocks_kernel(const MixJob *__restrict__ jobs, const MixTerm *__restrict__ terms,
                  int32_t kmax, const T *__restrict__ Z, int64_t ldz, double *__restrict__ S,
                  int64_t lds) {
  const MixJob job = jobs[blockIdx.x];
  const int tid = threadIdx.x;
  if (tid >= job.m) return;
  double acc[64];
#pragma unroll
  for (int j = 0; j < 64; ++j) acc[j] = 0.0;
  for (int t = job.t0; t < job.t1; ++t) {
    const T *zr = Z + terms[t].zcol0 * ldz + job.row0 + tid;
#pragma unroll
    for (int j = 0; j < 64; ++j)
      if (j < kmax) acc[j] += (double)zr[(int64_t)j * ldz];
  }
#pragma unroll
  for (int j = 0; j < 64; ++j)
    if (j < kmax) S[(int64_t)j * lds + job.row0 + tid] = acc[j];
}

// The Gaussian-weighted combination (an extension, HM_FLAG_MIX_GAMMA): each
// term is multiplied by Gamma_a before the sum.  Same jobs and layout as
// sum_blocks_kernel.  Per term, Gamma is drawn into LDS by the whole
// workgroup (kmax * ceil(kmax/2) Philox draws), then every row takes its
// kmax x kmax product with the term's Z block.
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

// Augmented sample of one chunk of a box (one row per thread, ncols FP64
// accumulators); the parent term's G, scaled by the parent's singular
// values, is drawn into LDS by the whole workgroup.
template <typename T>
__global__ void __launch_bounds__(256)
h2_sample_kernel(const AugJob *__restrict__ jobs, int32_t ncols, int32_t level, int32_t pass,
                 uint64_t seed, const T *__restrict__ src, int64_t lds,
                 const double *__restrict__ UBp, const int32_t *__restrict__ prank,
                 const double *__restrict__ psigma, int32_t kmax, double *__restrict__ dst,
                 int64_t ldd) {
  __shared__ double G[64 * 64];
  const AugJob job = jobs[blockIdx.x];
  const int tid = threadIdx.x;
  const int kp = job.par_off >= 0 ? prank[job.par_idx] : 0;
  const int npair = (ncols + 1) / 2;
  const uint64_t key = seed + (uint64_t)job.inst;
  for (int e = tid; e < kp * npair; e += 256) {
    const int i = e / npair, jj = e % npair;
    dev::U4 ctr{job.grow, (uint32_t)jj, 0x80000000u + (uint32_t)i, (uint32_t)(4 * level + pass)};
    double z0, z1;
    dev::normal_pair(dev::philox10(ctr, (uint32_t)key, (uint32_t)(key >> 32)), z0, z1);
    const double sgm = psigma[(int64_t)job.par_idx * kmax + i];
    G[i * 64 + 2 * jj] = sgm * z0;
    if (2 * jj + 1 < ncols) G[i * 64 + 2 * jj + 1] = sgm * z1;
  }
  __syncthreads();
  if (tid >= job.m) return;
  double acc[64];
#pragma unroll
  for (int j = 0; j < 64; ++j) acc[j] = 0.0;
  if (job.src_col0 >= 0) {
    const T *sr = src + job.src_col0 * lds + job.row0 + tid;
#pragma unroll
    for (int j = 0; j < 64; ++j)
      if (j < ncols) acc[j] = (double)sr[(int64_t)j * lds];
  }
  if (kp > 0) {
    const double *pr = UBp + job.par_off + tid;
    for (int i = 0; i < kp; ++i) {
      const double u = pr[(int64_t)i * job.par_ld];
#pragma unroll
      for (int j = 0; j < 64; ++j)
        if (j < ncols) acc[j] += u * G[i * 64 + j];
    }
  }
#pragma unroll
  for (int j = 0; j < 64; ++j)
    if (j < ncols) dst[(int64_t)j * ldd + job.row0 + tid] = acc[j];
}

// One chunk of nested rows: out(row, 0:kp) = U_a(row, 0:kc) Tr (one row per thread).
__global__ void __launch_bounds__(256)
nest_kernel(const NestJob *__restrict__ jobs, int32_t kmax, const double *__restrict__ UBin,
            const double *__restrict__ Tr, const int32_t *__restrict__ rank,
            double *__restrict__ UBout) {
  __shared__ double Ts[64 * 64];
  const NestJob job = jobs[blockIdx.x];
  const int tid = threadIdx.x;
  const int kc = rank[job.cidx], kp = rank[job.pidx];
  for (int e = tid; e < kc * kp; e += 256) {
    const int i = e % kc, j = e / kc;
    Ts[i * 64 + j] = Tr[job.t_off + (int64_t)j * kmax + i];
  }
  __syncthreads();
  if (tid >= job.m) return;
  double acc[64];
#pragma unroll
  for (int j = 0; j < 64; ++j) acc[j] = 0.0;
  const double *ur = UBin + job.in_off + tid;
  for (int i = 0; i < kc; ++i) {
    const double u = ur[(int64_t)i * job.ldi];
#pragma unroll
    for (int j = 0; j < 64; ++j)
      if (j < kp) acc[j] += u * Ts[i * 64 + j];
  }
  double *o = UBout + job.out_off + tid;
#pragma unroll
  for (int j = 0; j < 64; ++j)
    if (j < kp) o[(int64_t)j * job.ldo] = acc[j];
}

}  // namespace

void launch_h2_sample(int32_t njobs, const AugJob *jobs, int32_t ncols, int32_t level,
                      int32_t pass, uint64_t seed, bool src_f32, const void *src, int64_t lds,
                      const double *UBp, const int32_t *prank, const double *psigma,
                      int32_t kmax, double *dst, int64_t ldd, hipStream_t s) {
  if (njobs <= 0 || ncols <= 0 || ncols > 64 || kmax > 64) return;
  if (src_f32)
    h2_sample_kernel<float><<<njobs, 256, 0, s>>>(jobs, ncols, level, pass, seed,
                                                  (const float *)src, lds, UBp, prank, psigma,
                                                  kmax, dst, ldd);
  else
    h2_sample_kernel<double><<<njobs, 256, 0, s>>>(jobs, ncols, level, pass, seed,
                                                   (const double *)src, lds, UBp, prank, psigma,
                                                   kmax, dst, ldd);
}

void launch_nest(int32_t njobs, const NestJob *jobs, int32_t kmax, const double *UBin,
                 const double *Tr, const int32_t *rank, double *UBout, hipStream_t s) {
  if (njobs <= 0 || kmax <= 0 || kmax > 64) return;
  nest_kernel<<<njobs, 256, 0, s>>>(jobs, kmax, UBin, Tr, rank, UBout);
}

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
                    int32_t level, uint64_t seed, bool gamma, bool f32, const void *Z,
                    int64_t ldz, double *S, int64_t lds, hipStream_t s) {
  if (njobs <= 0 || kmax <= 0 || kmax > 64) return;
  if (!gamma) {
    if (f32)
      sum_blocks_kernel<float><<<njobs, 256, 0, s>>>(jobs, terms, kmax, (const float *)Z, ldz, S,
                                                     lds);
    else
      sum_blocks_kernel<double><<<njobs, 256, 0, s>>>(jobs, terms, kmax, (const double *)Z, ldz,
                                                      S, lds);
    return;
  }
  if (f32)
    mix_sum_kernel<float><<<njobs, 256, 0, s>>>(jobs, terms, kmax, level, seed, (const float *)Z,
                                                ldz, S, lds);
  else
    mix_sum_kernel<double><<<njobs, 256, 0, s>>>(jobs, terms, kmax, level, seed,
                                                 (const double *)Z, ldz, S, lds);
}

}  // namespace hm
