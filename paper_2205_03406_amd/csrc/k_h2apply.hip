// H^2 apply (alg:apply_h2_level_truncated): outgoing expansions of the
// boxes that hold long bases (q = V* x on their rows), the upward pass
// through the transfer matrices, the couplings and the downward pass
// (u_a = sum_b B_ab q_b + T_a u_parent), and the expansion y += U u on the
// rows of the boxes with long bases.  Expansions are FP64, kmax x ncols per
// box (ld kmax), at QH / UH + box * kmax * ldq; X and Y are FP64 or FP32.
// Every output element is owned by one thread: no atomics, deterministic.
#include <algorithm>
#include <stdexcept>

#include "device_common.h"
#include "kernels.h"

namespace hm {

namespace {

constexpr int HC = 64;  // columns per workgroup (projection, expansion)

// The partial q_b(0:k, c) = sum_i V_b(i, 0:k) x(row0 + i, c) over one
// 64-row chunk of a box: one workgroup per (chunk, 64-column tile), written
// to PART at the chunk's index; the chunks of a large box run in parallel
// (one workgroup walking a box of thousands of rows is latency-bound).
// Thread (column cc, group ig) accumulates rows j = ig + 4 q (q < NQ,
// 4 NQ >= kmax) of the expansion; rows past kmax read row kmax - 1 and are
// dropped.
template <typename T, int NQ>
__global__ void __launch_bounds__(256)
h2_project_kernel(const H2Leaf *__restrict__ jobs, int32_t kmax, const int32_t *__restrict__ rank,
                  const double *__restrict__ VB, const T *__restrict__ X, int64_t ldx,
                  int64_t ncols, double *__restrict__ PART, int64_t ldq) {
  extern __shared__ double sm[];
  const int ldv = kmax + 1;
  double *Xs = sm;                  // [row][column], ld HC + 1
  double *Vs = sm + 64 * (HC + 1);  // [row][basis column], ld kmax + 1
  const H2Leaf job = jobs[blockIdx.x];
  const int64_t c0 = (int64_t)blockIdx.y * HC;
  const int tid = threadIdx.x;
  const int k = rank[job.g];
  const int cc = tid & 63, ig = tid >> 6;
  double acc[NQ];
  int jr[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    acc[q] = 0.0;
    jr[q] = ig + 4 * q < kmax ? ig + 4 * q : kmax - 1;
  }
  {
    const int r0 = job.r0;
    const int rows = job.m - r0 < 64 ? job.m - r0 : 64;
    const bool rin = cc < rows;
    const T *xr = X + job.row0 + r0 + cc;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = ig + 4 * q;
      Xs[cc * (HC + 1) + c] = (rin && c0 + c < ncols) ? (double)xr[(c0 + c) * ldx] : 0.0;
    }
    const double *vr = VB + job.boff + r0 + cc;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int j = ig + 4 * q;
      if (j < kmax) Vs[cc * ldv + j] = (rin && j < k) ? vr[(int64_t)j * job.m] : 0.0;
    }
    __syncthreads();
    for (int i = 0; i < rows; ++i) {
      const double xv = Xs[i * (HC + 1) + cc];
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc[q] += Vs[i * ldv + jr[q]] * xv;
    }
  }
  // through LDS so that the stores are contiguous
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int j = ig + 4 * q;
    if (j < kmax) Xs[cc * ldv + j] = j < k ? acc[q] : 0.0;
  }
  __syncthreads();
  double *o = PART + (int64_t)blockIdx.x * kmax * ldq + c0 * kmax;
  const int64_t left = ncols - c0;
  const int ne = kmax * (int)(left < HC ? left : HC);
  for (int e = tid; e < ne; e += 256) {
    const int c = e / kmax, j = e - c * kmax;
    o[e] = Xs[c * ldv + j];
  }
}

// QH[g] = the sum of the partials of box g's chunks, in chunk order
// (deterministic); one workgroup per (box, 64-column tile).
__global__ void __launch_bounds__(256)
h2_reduce_kernel(const H2Leaf *__restrict__ leaf, int32_t kmax, const double *__restrict__ PART,
                 double *__restrict__ QH, int64_t ldq, int64_t ncols) {
  const H2Leaf job = leaf[blockIdx.x];
  const int64_t c0 = (int64_t)blockIdx.y * HC;
  const int64_t left = ncols - c0;
  const int ne = kmax * (int)(left < HC ? left : HC);
  const int nch = (job.m + 63) / 64;
  const double *p = PART + (int64_t)job.c0 * kmax * ldq + c0 * kmax;
  double *o = QH + (int64_t)job.g * kmax * ldq + c0 * kmax;
  for (int e = threadIdx.x; e < ne; e += 256) {
    double acc = 0.0;
    for (int t = 0; t < nch; ++t) acc += p[(int64_t)t * kmax * ldq + e];
    o[e] = acc;
  }
}

// Small sums of products: out(0:ko, c) = sum_t M_t(0:ko, 0:kt) in_t(0:kt, c),
// M_t stored kmax x kmax (ld kmax) or transposed (trans), for the terms of
// one job: the transfers of the upward pass, or the couplings and the parent
// term of the downward pass.  Ranks: ko from rank_o, kt from rank_i (rank_o
// for a parent term, whose input is an incoming expansion).  One workgroup
// per (job, HCT-column tile); the terms' descriptors go to LDS 256 at a
// time, the terms themselves tb at a time (a wave per term): each M_t as
// stored, its input tile with the column stride padded to ldk (odd).  Thread (column cc,
// group ig) owns rows i = ig + NG q (q < NQ, NG NQ >= kmax); rows past kmax
// read row kmax - 1 and are dropped.
template <int HCT, int NQ>
__global__ void __launch_bounds__(256)
h2_sum_kernel(const H2Sum *__restrict__ jobs, const H2Term *__restrict__ terms, int32_t kmax,
              const int32_t *__restrict__ rank_o, const int32_t *__restrict__ rank_i,
              const double *__restrict__ Mpool, const double *__restrict__ Mpar,
              const double *IN, const double *PAR, double *OUT, int64_t ldq, int64_t ncols,
              int32_t tb) {
  constexpr int NG = 256 / HCT;
  extern __shared__ double sm[];
  __shared__ int64_t t_off[256], t_in[256];
  __shared__ int32_t t_kt[256], t_fl[256];  // fl: parent | trans << 1
  const int ldk = kmax | 1;
  const int pm = kmax * kmax;
  const int ps = pm + HCT * ldk;  // LDS doubles per term
  const H2Sum job = jobs[blockIdx.x];
  const int64_t c0 = (int64_t)blockIdx.y * HCT;
  const int64_t left = ncols - c0;
  const int wc = (int)(left < HCT ? left : HCT);  // columns of this tile
  const int pi = kmax * wc;                       // input elements per term
  const int tid = threadIdx.x, cc = tid % HCT, ig = tid / HCT;
  const int wv = tid >> 6, lane = tid & 63;
  const int dc = 64 / kmax, dj = 64 - dc * kmax;  // a 64-element step in (column, row)
  const int ko = rank_o[job.g];
  double acc[NQ];
  int ir[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    acc[q] = 0.0;
    ir[q] = ig + NG * q < kmax ? ig + NG * q : kmax - 1;
  }
  for (int s0 = job.t0; s0 < job.t1; s0 += 256) {
    const int ns = job.t1 - s0 < 256 ? job.t1 - s0 : 256;
    __syncthreads();
    if (tid < ns) {
      const H2Term tm = terms[s0 + tid];
      t_off[tid] = tm.moff;
      t_in[tid] = (int64_t)tm.src * kmax * ldq + c0 * kmax;
      t_kt[tid] = tm.parent ? rank_o[tm.src] : rank_i[tm.src];
      t_fl[tid] = (tm.parent ? 1 : 0) | (tm.trans ? 2 : 0);
    }
    for (int b0 = 0; b0 < ns; b0 += tb) {
      const int nb = tb < ns - b0 ? tb : ns - b0;
      __syncthreads();
      // one wave per term: descriptors read once, loads independent
      for (int u = wv; u < nb; u += 4) {
        const int t = b0 + u;
        const bool par = (t_fl[t] & 1) != 0;
        const double *Mg = (par ? Mpar : Mpool) + t_off[t];
        const double *Ig = (par ? PAR : IN) + t_in[t];
        double *d = sm + u * ps;
#pragma unroll 4
        for (int r = lane; r < pm; r += 64) d[r] = Mg[r];
        int c = lane / kmax, j = lane - c * kmax;
#pragma unroll 4
        for (int r = lane; r < pi; r += 64) {
          d[pm + c * ldk + j] = Ig[r];
          c += dc;
          j += dj;
          if (j >= kmax) {
            j -= kmax;
            ++c;
          }
        }
      }
      __syncthreads();
      if (cc < wc) {
        for (int u = 0; u < nb; ++u) {
          const int t = b0 + u;
          const int kt = t_kt[t];
          const bool tr = (t_fl[t] & 2) != 0;
          const int si = tr ? kmax : 1, sj = tr ? 1 : kmax;  // M(i, j) at i si + j sj
          const double *Ms = sm + u * ps;
          const double *Is = Ms + pm + cc * ldk;
          for (int j = 0; j < kt; ++j) {
            const double xv = Is[j];
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[q] += Ms[ir[q] * si + j * sj] * xv;
          }
        }
      }
    }
  }
  // through LDS so that the stores are contiguous
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = ig + NG * q;
    if (i < kmax) sm[cc * ldk + i] = i < ko ? acc[q] : 0.0;
  }
  __syncthreads();
  double *o = OUT + (int64_t)job.g * kmax * ldq + c0 * kmax;
  for (int e = tid; e < pi; e += 256) {
    const int c = e / kmax, i = e - c * kmax;
    o[e] = sm[c * ldk + i];
  }
}

// y(row0 + r, c) += sign sum_j U_a(r, j) u_a(j, c) for one 64-row chunk of a
// box: lanes along the rows (coalesced read-modify-write of y), thread
// (row r, group cg) owns columns cg + 4 q.
template <typename T>
__global__ void __launch_bounds__(256)
h2_expand_kernel(const H2Leaf *__restrict__ jobs, int32_t kmax, const int32_t *__restrict__ rank,
                 const double *__restrict__ UB, const double *__restrict__ UH, int64_t ldq,
                 int64_t ncols, T *__restrict__ Y, int64_t ldy, double sign) {
  extern __shared__ double sm[];
  double *Us = sm;              // [j][row], ld 65
  double *Hs = sm + kmax * 65;  // [j][column], ld HC + 1
  const H2Leaf job = jobs[blockIdx.x];
  const int64_t c0 = (int64_t)blockIdx.y * HC;
  const int tid = threadIdx.x;
  const int k = rank[job.g];
  const int rows = job.m - job.r0 < 64 ? job.m - job.r0 : 64;
  const int r = tid & 63, cg = tid >> 6;
  const bool rin = r < rows;
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
#pragma unroll 4
  for (int j = cg; j < kmax; j += 4)
    Us[j * 65 + r] = (rin && j < k) ? UB[job.boff + (int64_t)j * job.m + job.r0 + r] : 0.0;
  const double *uh = UH + (int64_t)job.g * kmax * ldq + c0 * kmax;
  const int64_t left = ncols - c0;
  const int wc = (int)(left < HC ? left : HC);
  for (int e = tid; e < kmax * HC; e += 256) {
    const int c = e / kmax, j = e - c * kmax;
    Hs[j * (HC + 1) + c] = (j < k && c < wc) ? uh[e] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    const double u = Us[j * 65 + r];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] += u * Hs[j * (HC + 1) + cg + 4 * q];
  }
  if (!rin) return;
  T *y = Y + job.row0 + job.r0 + r;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int c = cg + 4 * q;
    if (c < wc) y[(c0 + c) * ldy] = (T)((double)y[(c0 + c) * ldy] + sign * acc[q]);
  }
}

template <typename T>
void project_nq(dim3 g, size_t lds, hipStream_t s, const H2Leaf *jobs, int32_t kmax,
                const int32_t *rank, const double *VB, const T *X, int64_t ldx, int64_t ncols,
                double *PART, int64_t ldq) {
  if (kmax <= 16)
    h2_project_kernel<T, 4><<<g, 256, lds, s>>>(jobs, kmax, rank, VB, X, ldx, ncols, PART, ldq);
  else if (kmax <= 32)
    h2_project_kernel<T, 8><<<g, 256, lds, s>>>(jobs, kmax, rank, VB, X, ldx, ncols, PART, ldq);
  else
    h2_project_kernel<T, 16><<<g, 256, lds, s>>>(jobs, kmax, rank, VB, X, ldx, ncols, PART, ldq);
}

template <int HCT, int NQ>
void sum_launch(dim3 g, size_t lds, hipStream_t s, const H2Sum *jobs, const H2Term *terms,
                int32_t kmax, const int32_t *rank_o, const int32_t *rank_i, const double *Mpool,
                const double *Mpar, const double *IN, const double *PAR, double *OUT, int64_t ldq,
                int64_t ncols, int32_t tb) {
  h2_sum_kernel<HCT, NQ><<<g, 256, lds, s>>>(jobs, terms, kmax, rank_o, rank_i, Mpool, Mpar, IN,
                                             PAR, OUT, ldq, ncols, tb);
}

}  // namespace

void launch_h2_project(int32_t nchunks, const H2Leaf *chunks, int32_t kmax, const int32_t *rank,
                       const double *VB, bool f32, const void *X, int64_t ldx, int64_t ncols,
                       double *PART, int64_t ldq, hipStream_t s) {
  if (nchunks <= 0 || ncols <= 0 || kmax <= 0) return;
  if (kmax > 64) throw std::runtime_error("h2 apply: rank above 64");
  dim3 g(nchunks, (unsigned)((ncols + HC - 1) / HC));
  const size_t lds = (size_t)(64 * (HC + 1) + 64 * (kmax + 1)) * sizeof(double);
  if (f32)
    project_nq<float>(g, lds, s, chunks, kmax, rank, VB, (const float *)X, ldx, ncols, PART, ldq);
  else
    project_nq<double>(g, lds, s, chunks, kmax, rank, VB, (const double *)X, ldx, ncols, PART,
                       ldq);
}

void launch_h2_reduce(int32_t nleaf, const H2Leaf *leaf, int32_t kmax, const double *PART,
                      double *QH, int64_t ldq, int64_t ncols, hipStream_t s) {
  if (nleaf <= 0 || ncols <= 0 || kmax <= 0) return;
  dim3 g(nleaf, (unsigned)((ncols + HC - 1) / HC));
  h2_reduce_kernel<<<g, 256, 0, s>>>(leaf, kmax, PART, QH, ldq, ncols);
}

void launch_h2_sum(int32_t njobs, const H2Sum *jobs, const H2Term *terms, int32_t kmax,
                   const int32_t *rank_o, const int32_t *rank_i, const double *Mpool,
                   const double *Mpar, const double *IN, const double *PAR, double *OUT,
                   int64_t ldq, int64_t ncols, hipStream_t s) {
  if (njobs <= 0 || ncols <= 0 || kmax <= 0) return;
  if (kmax > 64) throw std::runtime_error("h2 apply: rank above 64");
  // 64-column tiles for wide right-hand sides while one term fits 56 KB of
  // LDS, else 32; batches of up to 8 terms within 40 KB
  const int ldk = kmax | 1;
  const int hct = (ncols > 32 && kmax * kmax + 64 * ldk <= 7168) ? 64 : 32;
  const int ps = kmax * kmax + hct * ldk;
  const int tb = std::max(1, std::min(8, 5120 / ps));
  const size_t lds = (size_t)std::max(tb * ps, hct * ldk) * sizeof(double);
  dim3 g(njobs, (unsigned)((ncols + hct - 1) / hct));
  if (hct == 64) {
    if (kmax <= 16)
      sum_launch<64, 4>(g, lds, s, jobs, terms, kmax, rank_o, rank_i, Mpool, Mpar, IN, PAR, OUT,
                        ldq, ncols, tb);
    else if (kmax <= 32)
      sum_launch<64, 8>(g, lds, s, jobs, terms, kmax, rank_o, rank_i, Mpool, Mpar, IN, PAR, OUT,
                        ldq, ncols, tb);
    else
      sum_launch<64, 16>(g, lds, s, jobs, terms, kmax, rank_o, rank_i, Mpool, Mpar, IN, PAR,
                         OUT, ldq, ncols, tb);
  } else {
    if (kmax <= 32)
      sum_launch<32, 4>(g, lds, s, jobs, terms, kmax, rank_o, rank_i, Mpool, Mpar, IN, PAR, OUT,
                        ldq, ncols, tb);
    else
      sum_launch<32, 8>(g, lds, s, jobs, terms, kmax, rank_o, rank_i, Mpool, Mpar, IN, PAR, OUT,
                        ldq, ncols, tb);
  }
}

void launch_h2_expand(int32_t njobs, const H2Leaf *jobs, int32_t kmax, const int32_t *rank,
                      const double *UB, const double *UH, int64_t ldq, bool f32, int64_t ncols,
                      void *Y, int64_t ldy, double sign, hipStream_t s) {
  if (njobs <= 0 || ncols <= 0 || kmax <= 0) return;
  if (kmax > 64) throw std::runtime_error("h2 apply: rank above 64");
  dim3 g(njobs, (unsigned)((ncols + HC - 1) / HC));
  const size_t lds = (size_t)(kmax * 65 + kmax * (HC + 1)) * sizeof(double);
  if (f32)
    h2_expand_kernel<float><<<g, 256, lds, s>>>(jobs, kmax, rank, UB, UH, ldq, ncols, (float *)Y,
                                                ldy, sign);
  else
    h2_expand_kernel<double><<<g, 256, lds, s>>>(jobs, kmax, rank, UB, UH, ldq, ncols,
                                                 (double *)Y, ldy, sign);
}

}  // namespace hm
