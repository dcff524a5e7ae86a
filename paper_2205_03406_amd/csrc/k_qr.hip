// Per-pair recovery of alg:compress_double_random, batched over all
// admissible pairs of a level, one workgroup (4 waves) per pair:
//
//   pivqr     U = qr(S, k): column-pivoted Householder QR of the sample block
//             S (m x r) in an FP64 workspace, stopped at the fixed rank or at
//             the first |R_jj| <= tol |R_00| (eq:QR, partial QR), then the
//             explicit Q[:, 0:k] by backward accumulation of the reflectors.
//   core      C = G2^T S (r x r), the sketch of the block seen from both sides.
//   coupling  B = (G2^T U)^+ C (V^T G1)^+ through two small Householder
//             least-squares solves in LDS, and W = U B for the apply.
//
// All of this stays in FP64 in every precision mode.  Reductions over rows
// are wave-wide shuffles; every column update is owned by one wave.
#include <algorithm>
#include <atomic>

#include "device_common.h"
#include "kernels.h"

namespace hm {

namespace {

using dev::wave_sum;

// ------------------------------------------------------------------ lane loops
// A lane's share of a column operation over rows i0, i0 + 64, ... < m, four
// rows in flight at a time (independent partial sums, every load of a group
// issued before its results are used or stored): a loop with one row per
// step waits on each load in turn, and these blocks run to thousands of rows.
__device__ __forceinline__ double lane_dot(const double *x, const double *y, int i0, int m) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int i = i0;
  for (; i + 192 < m; i += 256) {
    const double x0 = x[i], x1 = x[i + 64], x2 = x[i + 128], x3 = x[i + 192];
    const double y0 = y[i], y1 = y[i + 64], y2 = y[i + 128], y3 = y[i + 192];
    a0 += x0 * y0;
    a1 += x1 * y1;
    a2 += x2 * y2;
    a3 += x3 * y3;
  }
  for (; i < m; i += 64) a0 += x[i] * y[i];
  return (a0 + a1) + (a2 + a3);
}

// y(i) -= f x(i) over the lane's rows; returns the lane's sum of the new y(i)^2
__device__ __forceinline__ double lane_axpy(double *y, const double *x, double f, int i0, int m) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int i = i0;
  for (; i + 192 < m; i += 256) {
    const double x0 = x[i], x1 = x[i + 64], x2 = x[i + 128], x3 = x[i + 192];
    const double y0 = y[i], y1 = y[i + 64], y2 = y[i + 128], y3 = y[i + 192];
    const double v0 = y0 - f * x0, v1 = y1 - f * x1, v2 = y2 - f * x2, v3 = y3 - f * x3;
    y[i] = v0;
    y[i + 64] = v1;
    y[i + 128] = v2;
    y[i + 192] = v3;
    s0 += v0 * v0;
    s1 += v1 * v1;
    s2 += v2 * v2;
    s3 += v3 * v3;
  }
  for (; i < m; i += 64) {
    const double v = y[i] - f * x[i];
    y[i] = v;
    s0 += v * v;
  }
  return (s0 + s1) + (s2 + s3);
}

// ------------------------------------------------------------------ block norms
// out[j] = scale * ||S(rows, cols) of job j||_F (FP64 accumulation).
template <typename T>
__global__ void __launch_bounds__(256)
block_norm_kernel(const QrJob *__restrict__ jobs, int32_t r, double scale,
                  const T *__restrict__ S, int64_t lds, double *__restrict__ out) {
  __shared__ double part[4];
  const QrJob job = jobs[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const T *A = S + job.col0 * lds + job.row0;
  double s2 = 0.0;
  for (int c = wave; c < r; c += 4)
    for (int i = lane; i < job.m; i += 64) {
      const double v = (double)A[(int64_t)c * lds + i];
      s2 += v * v;
    }
  s2 = wave_sum(s2);
  if (lane == 0) part[wave] = s2;
  __syncthreads();
  if (tid == 0) out[blockIdx.x] = scale * sqrt(part[0] + part[1] + part[2] + part[3]);
}

// ------------------------------------------------------------------ pivqr
// Rows of a QR block held in LDS: 4096 / r (128 at r = 32), fewer when the
// device's per-workgroup LDS is smaller than 64 KB plus `other` bytes.  The
// working copy and the explicit basis each take rows x r FP64 there (64 KB
// per workgroup at most; the QR kernels' registers allow two workgroups per
// compute unit, which then use 128 of the 160 KB).
int32_t qr_lds_rows(int32_t r, size_t other) {
  if (r <= 0) return 0;
  static std::atomic<int> cap[64];  // per device, 0 until queried
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    return 0;
  }
  int c = cap[dev].load();
  if (c == 0) {
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      c = 65536;
    (void)hipGetLastError();
    cap[dev].store(c);
  }
  const int64_t room = ((int64_t)c - (int64_t)other - 2048) / (2 * 8 * (int64_t)r);
  return (int32_t)std::max<int64_t>(0, std::min<int64_t>(4096 / r, room));
}

// One block (job index jx): the body of pivqr_kernel and of the fused
// recovery kernel.  The FP64 working copy of the block and the explicit
// basis are built in LDS (lws: room for 2 lws_rows x r) when the block has
// at most lws_rows rows, else in the global workspace and in U: every step
// of the factorization and of the basis formation reads and writes them,
// and from LDS those round trips take a fraction of the time.
template <typename T>
__device__ void pivqr_body(const QrJob &job, int jx, int32_t r, int32_t rank_fixed, double tol,
                           int32_t cap, const double *__restrict__ floor_abs,
                           const T *__restrict__ S, int64_t lds, double *__restrict__ Wk,
                           double *__restrict__ U, int32_t *__restrict__ ranks,
                           int32_t *__restrict__ sat, double *lws, int32_t lws_rows) {
  __shared__ double nrm2[64];
  __shared__ int piv[64];
  __shared__ double tau[64];
  __shared__ double bcast[4];
  __shared__ int stop_s;
  const int m = job.m;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const T *A = S + job.col0 * lds + job.row0;
  const bool in_lds = lws && m <= lws_rows;
  double *W = in_lds ? lws : Wk + job.wslot;  // m x r, ld = m
  const int kmax_here = m < r ? m : r;
  const int kcap = rank_fixed > 0 ? (rank_fixed < kmax_here ? rank_fixed : kmax_here)
                                  : (cap < kmax_here ? cap : kmax_here);
  // absolute floor under the relative threshold (the rounding noise of a
  // reduced-precision sample), 0 when none
  const double fl = floor_abs ? floor_abs[jx] : 0.0;

  // copy to the FP64 workspace and take squared column norms
  for (int c = wave; c < r; c += 4) {
    double s2 = 0.0;
    for (int i = lane; i < m; i += 64) {
      const double v = (double)A[(int64_t)c * lds + i];
      W[(int64_t)c * m + i] = v;
      s2 += v * v;
    }
    s2 = wave_sum(s2);
    if (lane == 0) nrm2[c] = s2;
  }
  if (tid < 64) piv[tid] = tid;
  __syncthreads();

  int rank = 0;
  int saturated = 0;
  double r00 = 0.0;
  for (int j = 0; j < kcap; ++j) {
    if (tid == 0) {
      // largest remaining column (first one on ties)
      int p = j;
      for (int c = j + 1; c < r; ++c)
        if (nrm2[c] > nrm2[p]) p = c;
      const double tn = nrm2[j];
      nrm2[j] = nrm2[p];
      nrm2[p] = tn;
      const int tp = piv[j];
      piv[j] = piv[p];
      piv[p] = tp;
    }
    __syncthreads();
    const int pc = piv[j];
    double *x = W + (int64_t)pc * m;
    if (wave == 0) {
      double s2 = lane_dot(x, x, j + lane, m);
      s2 = wave_sum(s2);
      if (lane == 0) {
        const double nrm = sqrt(s2);
        if (j == 0) bcast[1] = nrm;
        const double ref = j == 0 ? nrm : bcast[1];
        int stop = !(nrm > 0.0);
        if (rank_fixed <= 0 && !(nrm > fmax(tol * ref, fl))) stop = 1;
        stop_s = stop;
        if (!stop) {
          const double alpha = x[j];
          const double beta = alpha >= 0.0 ? -nrm : nrm;
          tau[j] = (beta - alpha) / beta;
          bcast[0] = 1.0 / (alpha - beta);
          x[j] = beta;
        }
      }
    }
    __syncthreads();
    r00 = bcast[1];
    if (stop_s) break;
    rank = j + 1;
    const double sc = bcast[0];
    for (int i = j + 1 + tid; i < m; i += 256) x[i] *= sc;
    __syncthreads();
    const double tj = tau[j];
    for (int c = j + 1 + wave; c < r; c += 4) {
      double *y = W + (int64_t)piv[c] * m;
      double w = lane_dot(x, y, j + 1 + lane, m);
      w = wave_sum(w) + y[j];
      const double f = tj * w;
      if (lane == 0) y[j] -= f;
      double s2 = lane_axpy(y, x, f, j + 1 + lane, m);
      s2 = wave_sum(s2);
      if (lane == 0) nrm2[c] = s2;
    }
    __syncthreads();
  }
  // tolerance mode: the cap was reached while a remaining column still
  // exceeds the threshold
  if (rank_fixed <= 0 && rank == kcap && kcap < kmax_here) {
    double mx = 0.0;
    for (int c = kcap; c < r; ++c) mx = nrm2[c] > mx ? nrm2[c] : mx;
    if (sqrt(mx) > fmax(tol * r00, fl)) saturated = 1;
  }

  // explicit basis: U = H_0 ... H_{rank-1} [I; 0], column-major (ld = m)
  double *Uo = U + job.uslot;
  double *Ub = in_lds ? lws + (int64_t)lws_rows * r : Uo;
  for (int c = wave; c < rank; c += 4)
    for (int i = lane; i < m; i += 64) Ub[(int64_t)c * m + i] = (i == c) ? 1.0 : 0.0;
  __syncthreads();
  for (int j = rank - 1; j >= 0; --j) {
    const double *x = W + (int64_t)piv[j] * m;
    const double tj = tau[j];
    for (int c = j + wave; c < rank; c += 4) {
      double *y = Ub + (int64_t)c * m;
      double w = lane_dot(x, y, j + 1 + lane, m);
      w = wave_sum(w) + y[j];
      const double f = tj * w;
      (void)lane_axpy(y, x, f, j + 1 + lane, m);
      if (lane == 0) y[j] -= f;
    }
    __syncthreads();
  }
  if (in_lds)
    for (int e = tid; e < m * rank; e += 256) Uo[e] = Ub[e];
  if (tid == 0) {
    ranks[jx] = rank;
    sat[jx] = saturated;
  }
  __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(256)
pivqr_kernel(const QrJob *__restrict__ jobs, int32_t r, int32_t rank_fixed, double tol,
             int32_t cap, const double *__restrict__ floor_abs, const T *__restrict__ S,
             int64_t lds, double *__restrict__ Wk, double *__restrict__ U,
             int32_t *__restrict__ ranks, int32_t *__restrict__ sat, int32_t lws_rows) {
  extern __shared__ double lws[];  // lws_rows x r
  pivqr_body<T>(jobs[blockIdx.x], blockIdx.x, r, rank_fixed, tol, cap, floor_abs, S, lds, Wk, U,
                ranks, sat, lws, lws_rows);
}

// ------------------------------------------------------------------ small dense helpers
// out(i, c) = sum_t X(t, i) Y(t, c), i < a, c < b (a*b <= 4096); X and Y are
// m-row column-major blocks; `stage` holds 32*(a+b) (+pad) doubles of LDS.
template <typename TX, typename TY>
__device__ void tn_gemm(int m, int a, int b, const TX *X, int64_t ldx, const TY *Y, int64_t ldy,
                        double *out, int ldo, double *stage) {
  const int tid = threadIdx.x;
  constexpr int SP = 33;
  double *sx = stage, *sy = stage + SP * a;
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  for (int t0 = 0; t0 < m; t0 += 32) {
    const int rows = m - t0 < 32 ? m - t0 : 32;
    for (int e = tid; e < 32 * a; e += 256) {
      const int tt = e % 32, i = e / 32;
      sx[i * SP + tt] = tt < rows ? (double)X[(int64_t)i * ldx + t0 + tt] : 0.0;
    }
    for (int e = tid; e < 32 * b; e += 256) {
      const int tt = e % 32, c = e / 32;
      sy[c * SP + tt] = tt < rows ? (double)Y[(int64_t)c * ldy + t0 + tt] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + 256 * q;
      if (e < a * b) {
        const int i = e % a, c = e / a;
        double s = 0.0;
#pragma unroll 8
        for (int tt = 0; tt < 32; ++tt) s += sx[i * SP + tt] * sy[c * SP + tt];
        acc[q] += s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q;
    if (e < a * b) out[(e / a) * ldo + (e % a)] = acc[q];
  }
  __syncthreads();
}

// Householder QR of M (rows x cols, ld, rows <= 64) in place: R in the upper
// triangle, reflector tails below it (leading 1 implicit), factors in tau.
__device__ void lds_qr(double *M, int ld, int rows, int cols, double *tau, double *bc) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = 0; j < cols; ++j) {
    if (wave == 0) {
      const double v = (lane >= j && lane < rows) ? M[j * ld + lane] : 0.0;
      const double s2 = wave_sum(v * v);
      if (lane == 0) {
        const double nrm = sqrt(s2);
        const double alpha = M[j * ld + j];
        if (nrm > 0.0) {
          const double beta = alpha >= 0.0 ? -nrm : nrm;
          tau[j] = (beta - alpha) / beta;
          bc[0] = 1.0 / (alpha - beta);
          M[j * ld + j] = beta;
        } else {
          tau[j] = 0.0;
          bc[0] = 0.0;
        }
      }
    }
    __syncthreads();
    if (tid > j && tid < rows) M[j * ld + tid] *= bc[0];
    __syncthreads();
    const double tj = tau[j];
    for (int c = j + 1 + wave; c < cols; c += 4) {
      const double v = (lane > j && lane < rows) ? M[j * ld + lane] : 0.0;
      const double y = (lane > j && lane < rows) ? M[c * ld + lane] : 0.0;
      const double w = wave_sum(v * y) + M[c * ld + j];
      const double f = tj * w;
      if (lane > j && lane < rows) M[c * ld + lane] = y - f * v;
      if (lane == 0) M[c * ld + j] -= f;
    }
    __syncthreads();
  }
}

// C <- Q^T C for the reflectors stored in M (rows x k); C is rows x nc (ldc)
__device__ void lds_apply_qt(const double *M, int ld, int rows, int k, const double *tau,
                             double *C, int ldc, int nc) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = 0; j < k; ++j) {
    const double tj = tau[j];
    for (int c = wave; c < nc; c += 4) {
      const double v = (lane > j && lane < rows) ? M[j * ld + lane] : 0.0;
      const double y = (lane > j && lane < rows) ? C[c * ldc + lane] : 0.0;
      const double w = wave_sum(v * y) + C[c * ldc + j];
      const double f = tj * w;
      if (lane > j && lane < rows) C[c * ldc + lane] = y - f * v;
      if (lane == 0) C[c * ldc + j] -= f;
    }
    __syncthreads();
  }
}

// Solve R X = C[0:k, :] in place (R upper k x k in M), one thread per column
__device__ void lds_backsolve(const double *M, int ld, int k, double *C, int ldc, int nc) {
  const int tid = threadIdx.x;
  for (int c = tid; c < nc; c += 256) {
    for (int i = k - 1; i >= 0; --i) {
      double s = C[c * ldc + i];
      for (int t = i + 1; t < k; ++t) s -= M[t * ld + i] * C[c * ldc + t];
      C[c * ldc + i] = s / M[i * ld + i];
    }
  }
  __syncthreads();
}

// ------------------------------------------------------------------ core
template <typename T>
__device__ void core_body(const CoreJob &job, int32_t r, const T *__restrict__ Psi, int64_t ldp,
                          const T *__restrict__ Y, int64_t ldy, double *__restrict__ core,
                          double *smem) {
  tn_gemm(job.ma, r, r, Psi + job.vcol0 * ldp + job.arow0, ldp, Y + job.ucol0 * ldy + job.arow0,
          ldy, core + job.cslot, r, smem);
}

// ------------------------------------------------------------------ coupling
template <typename T>
__device__ void coupling_body(const CoreJob &job, int32_t r, int32_t kmax,
                              const T *__restrict__ Omega, int64_t ldo, const T *__restrict__ Psi,
                              int64_t ldp, const double *__restrict__ U,
                              const double *__restrict__ V, const int32_t *__restrict__ ranks,
                              const double *__restrict__ core, double *__restrict__ scratch,
                              double *__restrict__ B, double *__restrict__ Wout, double *smem) {
  __shared__ double tau[64];
  __shared__ double bc[2];
  const int ku = ranks[job.pu], kv = ranks[job.pv];
  const int tid = threadIdx.x;
  double *Bs = B + job.bslot;
  double *W = Wout + job.wslot;
  if (ku == 0 || kv == 0) {
    // a zero block: B and W stay empty (ranks say so); clear for export
    for (int e = tid; e < kmax * kmax; e += 256) Bs[e] = 0.0;
    __syncthreads();
    return;
  }
  const int sa = (r * r > 33 * (r + kmax)) ? r * r : 33 * (r + kmax);
  double *A = smem;            // sa doubles: staging / C / X1
  double *M = smem + sa;       // r x kmax: M1 then M2^T
  const double *Ua = U + job.uslot;
  const double *Vb = V + job.vslot;
  // M1 = G2^T U  (r x ku), G2 = Psi(alpha rows, block of (b, a))
  tn_gemm(job.ma, r, ku, Psi + job.vcol0 * ldp + job.arow0, ldp, Ua, (int64_t)job.ma, M, r, A);
  lds_qr(M, r, r, ku, tau, bc);
  // X1 = R^{-1} (Q^T C)[0:ku, :]
  for (int e = tid; e < r * r; e += 256) A[e] = core[job.cslot + e];
  __syncthreads();
  lds_apply_qt(M, r, r, ku, tau, A, r, r);
  lds_backsolve(M, r, ku, A, r, r);
  double *X1 = scratch + job.cslot;  // ku x r, ld = r (rows 0..ku-1 of A)
  for (int e = tid; e < r * r; e += 256) X1[e] = A[e];
  __syncthreads();
  // M2^T = G1^T V  (r x kv), G1 = Omega(beta rows, block of (a, b))
  tn_gemm(job.mb, r, kv, Omega + job.ucol0 * ldo + job.brow0, ldo, Vb, (int64_t)job.mb, M, r, A);
  lds_qr(M, r, r, kv, tau, bc);
  // B^T = R^{-1} (Q^T X1^T)[0:kv, :] with X1^T (r x ku) in A (ld = r)
  for (int e = tid; e < r * ku; e += 256) {
    const int i = e % r, c = e / r;  // X1^T(i, c) = X1(c, i)
    A[c * r + i] = X1[i * r + c];
  }
  __syncthreads();
  lds_apply_qt(M, r, r, kv, tau, A, r, ku);
  lds_backsolve(M, r, kv, A, r, ku);
  // B(t, c) = B^T(c, t) = A[t * r + c], t < ku, c < kv; slot ld = kmax
  for (int e = tid; e < kmax * kmax; e += 256) {
    const int t = e % kmax, c = e / kmax;
    Bs[e] = (t < ku && c < kv) ? A[t * r + c] : 0.0;
  }
  __syncthreads();
  // W = U B  (ma x kv), ld = ma: eight columns of W per sweep over U, so a
  // thread reads each U entry of its row once per eight columns (B from LDS)
  for (int i = tid; i < job.ma; i += 256) {
    for (int c0 = 0; c0 < kv; c0 += 8) {
      double sacc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      for (int t = 0; t < ku; ++t) {
        const double u = Ua[(int64_t)t * job.ma + i];
#pragma unroll
        for (int cc = 0; cc < 8; ++cc)
          sacc[cc] += u * (c0 + cc < kv ? A[t * r + c0 + cc] : 0.0);
      }
#pragma unroll
      for (int cc = 0; cc < 8; ++cc)
        if (c0 + cc < kv) W[(int64_t)(c0 + cc) * job.ma + i] = sacc[cc];
    }
  }
  __syncthreads();
}

// Fused, persistent recovery of one level: a grid of up to 16 workgroups
// per compute unit (as many as fit stay resident), each pulling pairs from the level's work
// list (largest blocks first) through an atomic counter until the list is
// exhausted; per pair, in one workgroup, the core C = G2^T Y, the two
// pivoted QRs (U from the Y block, V from the Z block) and the coupling
// solve with W = U B: one launch per level, no workgroup idle while others
// finish the large blocks.  The counter must be zero at the launch.
template <typename T>
__global__ void __launch_bounds__(256)
recover_kernel(RecoverArgs a, const T *__restrict__ Om, const T *__restrict__ Ps,
               const T *__restrict__ Ys) {
  extern __shared__ double smem[];
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(a.counter, 1);
    __syncthreads();
    const int i = next;
    __syncthreads();
    if (i >= a.njobs) break;
    const int q = a.order[i];
    const CoreJob cj = a.jc[q];
    core_body<T>(cj, a.r, Ps, a.ld, Ys, a.ld, a.core, smem);
    pivqr_body<T>(a.ju[q], q, a.r, a.rank_fixed, a.tol, a.cap, a.floor_u, Ys, a.ld, a.work, a.U,
                  a.ranks_u, a.sat_u, smem, a.qr_rows);
    pivqr_body<T>(a.jv[q], q, a.r, a.rank_fixed, a.tol, a.cap, a.floor_v, Ys, a.ld, a.work, a.V,
                  a.ranks_v, a.sat_v, smem, a.qr_rows);
    coupling_body<T>(cj, a.r, a.kmax, Om, a.ld, Ps, a.ld, a.U, a.V, a.ranks, a.core, a.scratch,
                     a.B, a.W, smem);
  }
}

// ------------------------------------------------------------------ uniform coupling
// Per pair (a, b): ranks, copies of the shared bases into the pair's slots
// (when U and V are given), B = Z(I_b, block of (b, a))[:, :ku]^T V_b
// (slot ld = kmax) and, when Wout is given, W = U_a B.
template <typename T>
__global__ void __launch_bounds__(256)
ucoupling_kernel(const UCJob *__restrict__ jobs, int32_t kmax, const T *__restrict__ Z,
                 int64_t ldz, const double *__restrict__ UB, const double *__restrict__ VB,
                 const int32_t *__restrict__ urank, const int32_t *__restrict__ vrank,
                 double *__restrict__ U, double *__restrict__ V, double *__restrict__ B,
                 double *__restrict__ Wout, int32_t *__restrict__ ranks, int recompute) {
  extern __shared__ double smem[];  // tn_gemm staging, 33 * 2 kmax doubles
  const UCJob job = jobs[blockIdx.x];
  const int ku = urank[job.ua], kv = vrank[job.vb];
  const int tid = threadIdx.x;
  if (tid == 0) {
    ranks[job.pu] = ku;
    ranks[job.pv] = kv;
  }
  const double *Ua = UB + job.uboff;
  const double *Vb = VB + job.vboff;
  if (U)
    for (int64_t e = tid; e < (int64_t)job.ma * ku; e += 256) U[job.uslot + e] = Ua[e];
  if (V)
    for (int64_t e = tid; e < (int64_t)job.mb * kv; e += 256) V[job.vslot + e] = Vb[e];
  double *Bs = B + job.bslot;
  if (recompute) {
    for (int e = tid; e < kmax * kmax; e += 256) Bs[e] = 0.0;
    __syncthreads();
    if (ku == 0 || kv == 0) return;
    tn_gemm(job.mb, ku, kv, Z + job.zcol0 * ldz + job.zrow0, ldz, Vb, (int64_t)job.mb, Bs, kmax,
            smem);
  } else if (ku == 0 || kv == 0) {
    return;
  }
  if (!Wout) return;
  double *W = Wout + job.wslot;
  for (int i = tid; i < job.ma; i += 256) {
    for (int c = 0; c < kv; ++c) {
      double s = 0.0;
      for (int t = 0; t < ku; ++t) s += Ua[(int64_t)t * job.ma + i] * Bs[t + c * kmax];
      W[(int64_t)c * job.ma + i] = s;
    }
  }
}

// ------------------------------------------------------------------ SVD bases
// Left singular vectors of a sample block S (m x c, c <= 64) in FP64:
// Householder QR of S in the workspace (no pivoting), one-sided Jacobi
// (Hestenes) on the columns of R* in LDS until no pair is rotated, with the
// rotations accumulated in J; singular values = the column norms, sorted
// descending; U = Q [J ; 0] (the columns of J in that order) truncated to
// the rank (fixed, or the values above max(tol sigma_0,
// floor), at most cap), each column signed so that its largest entry is
// positive (the first on ties).  Singular values go to sigma (kmax per job).
__global__ void __launch_bounds__(256)
svd_basis_kernel(const QrJob *__restrict__ jobs, int32_t c, int32_t rank_fixed, double tol,
                 int32_t cap, const double *__restrict__ floor_abs, const double *__restrict__ S,
                 int64_t lds, double *__restrict__ Wk, double *__restrict__ U,
                 double *__restrict__ sigma, int32_t kmax, int32_t *__restrict__ ranks,
                 int32_t *__restrict__ sat) {
  __shared__ double Rs[64][65];  // R*: [column][row]
  __shared__ double Js[64][65];  // rotations: [column][row]
  __shared__ double tau[64];
  __shared__ double sg[64];
  __shared__ int ord[64];
  __shared__ double bc[2];
  __shared__ int flag, kk_s, sat_s;
  const QrJob job = jobs[blockIdx.x];
  const int m = job.m;
  const int kq = m < c ? m : c;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double *W = Wk + job.wslot;  // m x c, ld = m
  for (int j = wave; j < c; j += 4)
    for (int i = lane; i < m; i += 64)
      W[(int64_t)j * m + i] = S[(job.col0 + j) * lds + job.row0 + i];
  __syncthreads();
  // Householder QR: R in the upper triangle, reflector tails below it
  for (int j = 0; j < kq; ++j) {
    double *x = W + (int64_t)j * m;
    if (wave == 0) {
      double s2 = lane_dot(x, x, j + lane, m);
      s2 = wave_sum(s2);
      if (lane == 0) {
        const double nrm = sqrt(s2);
        const double alpha = x[j];
        if (nrm > 0.0) {
          const double beta = alpha >= 0.0 ? -nrm : nrm;
          tau[j] = (beta - alpha) / beta;
          bc[0] = 1.0 / (alpha - beta);
          x[j] = beta;
        } else {
          tau[j] = 0.0;
          bc[0] = 0.0;
        }
      }
    }
    __syncthreads();
    const double sc = bc[0];
    for (int i = j + 1 + tid; i < m; i += 256) x[i] *= sc;
    __syncthreads();
    const double tj = tau[j];
    for (int cc = j + 1 + wave; cc < c; cc += 4) {
      double *y = W + (int64_t)cc * m;
      double w = lane_dot(x, y, j + 1 + lane, m);
      w = wave_sum(w) + y[j];
      const double f = tj * w;
      (void)lane_axpy(y, x, f, j + 1 + lane, m);
      if (lane == 0) y[j] -= f;
    }
    __syncthreads();
  }
  // R* (c x kq: column j is row j of R) into LDS, zero elsewhere; J = I
  for (int e = tid; e < 64 * 64; e += 256) {
    const int i = e % 64, j = e / 64;
    Rs[j][i] = (j < kq && i < c && i >= j) ? W[(int64_t)i * m + j] : 0.0;
    Js[j][i] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  // One-sided Jacobi on R* over round-robin pairings of its kq columns,
  // accumulating the rotations in J: R* J = X Sigma, so R = J Sigma X* and
  // the left singular vectors of R are the columns of J (no division by
  // sigma).  R* converges in far fewer sweeps than R (about 8 against 13 to
  // 20 on kernel samples, and R itself stalls when m < c).  tpp threads per
  // pair (the most that 256 threads give every pair, a power of two from 8
  // to 32).  A pair is rotated while |p.q| > 2e-14 |p| |q|: rounding keeps
  // smaller products from vanishing.
  const int ce = kq + (kq & 1);
  const int tpp = ce <= 16 ? 32 : (ce <= 32 ? 16 : 8);
  const int pk = tid / tpp, lt = tid % tpp;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) flag = 0;
    __syncthreads();
    for (int rr = 0; rr < ce - 1; ++rr) {
      if (pk < ce / 2) {
        const int p = (rr + pk) % (ce - 1);
        const int q = pk == 0 ? ce - 1 : (rr - pk + ce - 1) % (ce - 1);
        double al = 0.0, be = 0.0, ga = 0.0;
        if (p < kq && q < kq)
          for (int i = lt; i < c; i += tpp) {
            const double u = Rs[p][i], v = Rs[q][i];
            al += u * u;
            be += v * v;
            ga += u * v;
          }
        for (int off = tpp >> 1; off > 0; off >>= 1) {
          al += __shfl_xor(al, off, tpp);
          be += __shfl_xor(be, off, tpp);
          ga += __shfl_xor(ga, off, tpp);
        }
        if (p < kq && q < kq && ga != 0.0 && fabs(ga) > 2e-14 * sqrt(al * be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double t = fabs(zeta) > 1e100
                               ? 0.5 / zeta
                               : (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
          for (int i = lt; i < c; i += tpp) {
            const double u = Rs[p][i], v = Rs[q][i];
            Rs[p][i] = cs * u - sn * v;
            Rs[q][i] = sn * u + cs * v;
          }
          for (int i = lt; i < kq; i += tpp) {
            const double u = Js[p][i], v = Js[q][i];
            Js[p][i] = cs * u - sn * v;
            Js[q][i] = sn * u + cs * v;
          }
          if (lt == 0) flag = 1;
        }
      }
      __syncthreads();
    }
    const int again = flag;
    __syncthreads();
    if (again == 0) break;
  }
  if (tid < kq) {
    double s2 = 0.0;
    for (int i = 0; i < c; ++i) s2 += Rs[tid][i] * Rs[tid][i];
    sg[tid] = sqrt(s2);
  }
  __syncthreads();
  if (tid < kq) {
    int rk = 0;
    for (int i = 0; i < kq; ++i) rk += (sg[i] > sg[tid] || (sg[i] == sg[tid] && i < tid)) ? 1 : 0;
    ord[rk] = tid;
  }
  __syncthreads();
  if (tid == 0) {
    const double s0 = kq > 0 ? sg[ord[0]] : 0.0;
    int kk, st = 0;
    if (!(s0 > 0.0)) {
      kk = 0;
    } else if (rank_fixed > 0) {
      kk = rank_fixed < kq ? rank_fixed : kq;
    } else {
      const double thr = fmax(tol * s0, floor_abs ? floor_abs[blockIdx.x] : 0.0);
      int cnt = 0;
      while (cnt < kq && sg[ord[cnt]] > thr) ++cnt;
      st = cnt > cap ? 1 : 0;
      kk = cnt < cap ? cnt : cap;
    }
    kk_s = kk;
    sat_s = st;
  }
  __syncthreads();
  const int kk = kk_s;
  // U = Q [J(:, order); 0]: the left singular vectors of R, then the reflectors
  double *Uo = U + job.uslot;
  for (int j = wave; j < kk; j += 4) {
    const int col = ord[j];
    for (int i = lane; i < m; i += 64) Uo[(int64_t)j * m + i] = i < kq ? Js[col][i] : 0.0;
  }
  __syncthreads();
  for (int j = kq - 1; j >= 0; --j) {
    const double *x = W + (int64_t)j * m;
    const double tj = tau[j];
    for (int cc = wave; cc < kk; cc += 4) {
      double *y = Uo + (int64_t)cc * m;
      double w = lane_dot(x, y, j + 1 + lane, m);
      w = wave_sum(w) + y[j];
      const double f = tj * w;
      (void)lane_axpy(y, x, f, j + 1 + lane, m);
      if (lane == 0) y[j] -= f;
    }
    __syncthreads();
  }
  // sign: the largest entry of every column positive (first on ties)
  for (int cc = wave; cc < kk; cc += 4) {
    double *y = Uo + (int64_t)cc * m;
    double best = -1.0;
    int bi = 0;
    for (int i = lane; i < m; i += 64) {
      const double a = fabs(y[i]);
      if (a > best) {
        best = a;
        bi = i;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (y[bi] < 0.0)
      for (int i = lane; i < m; i += 64) y[i] = -y[i];
  }
  if (tid < kmax) sigma[(int64_t)blockIdx.x * kmax + tid] = tid < kk ? sg[ord[tid]] : 0.0;
  if (tid == 0) {
    ranks[blockIdx.x] = kk;
    sat[blockIdx.x] = sat_s;
  }
}

// Transfer (short basis) of one child a of tau: out (k_a x k_tau, ld kmax)
// = U_a* U_tau(rows of a, :).
__global__ void __launch_bounds__(256)
transfer_kernel(const TransferJob *__restrict__ jobs, int32_t kmax, const double *__restrict__ UB,
                const int32_t *__restrict__ rank, double *__restrict__ out) {
  extern __shared__ double smem[];
  const TransferJob job = jobs[blockIdx.x];
  const int kc = rank[job.cidx], kp = rank[job.pidx];
  double *o = out + job.out_off;
  for (int e = threadIdx.x; e < kmax * kmax; e += 256) o[e] = 0.0;
  __syncthreads();
  if (kc == 0 || kp == 0) return;
  tn_gemm(job.mc, kc, kp, UB + job.child_off, (int64_t)job.mc, UB + job.par_off,
          (int64_t)job.ldp, o, kmax, smem);
}

}  // namespace

void launch_ucoupling(int32_t njobs, const UCJob *jobs, int32_t kmax, bool f32, const void *Z,
                      int64_t ldz, const double *UB, const double *VB, const int32_t *urank,
                      const int32_t *vrank, double *U, double *V, double *B, double *W,
                      int32_t *ranks, bool recompute, hipStream_t s) {
  if (njobs <= 0) return;
  const size_t sh = sizeof(double) * (33 * 2 * (size_t)kmax);
  if (f32)
    ucoupling_kernel<float><<<njobs, 256, sh, s>>>(jobs, kmax, (const float *)Z, ldz, UB, VB,
                                                   urank, vrank, U, V, B, W, ranks,
                                                   recompute ? 1 : 0);
  else
    ucoupling_kernel<double><<<njobs, 256, sh, s>>>(jobs, kmax, (const double *)Z, ldz, UB, VB,
                                                    urank, vrank, U, V, B, W, ranks,
                                                    recompute ? 1 : 0);
}

void launch_svd_basis(int32_t njobs, const QrJob *jobs, int32_t c, int32_t rank_fixed, double tol,
                      int32_t cap, const double *floor_abs, const double *S, int64_t lds,
                      double *Wk, double *U, double *sigma, int32_t kmax, int32_t *ranks,
                      int32_t *sat, hipStream_t s) {
  if (njobs <= 0 || c <= 0 || c > 64 || kmax > 64) return;
  svd_basis_kernel<<<njobs, 256, 0, s>>>(jobs, c, rank_fixed, tol, cap, floor_abs, S, lds, Wk, U,
                                         sigma, kmax, ranks, sat);
}

void launch_transfer(int32_t njobs, const TransferJob *jobs, int32_t kmax, const double *UB,
                     const int32_t *rank, double *out, hipStream_t s) {
  if (njobs <= 0) return;
  const size_t sh = sizeof(double) * (33 * 2 * (size_t)kmax);
  transfer_kernel<<<njobs, 256, sh, s>>>(jobs, kmax, UB, rank, out);
}

void launch_pivqr(int32_t njobs, const QrJob *jobs, int32_t r, int32_t rank_fixed, double tol,
                  int32_t cap, const double *floor_abs, bool f32, const void *S, int64_t lds,
                  double *Wk, double *U, int32_t *ranks, int32_t *sat, hipStream_t s) {
  if (njobs <= 0) return;
  const int32_t rows = qr_lds_rows(r, 0);
  const size_t sh = sizeof(double) * 2 * (size_t)rows * r;
  if (f32)
    pivqr_kernel<float><<<njobs, 256, sh, s>>>(jobs, r, rank_fixed, tol, cap, floor_abs,
                                               (const float *)S, lds, Wk, U, ranks, sat, rows);
  else
    pivqr_kernel<double><<<njobs, 256, sh, s>>>(jobs, r, rank_fixed, tol, cap, floor_abs,
                                                (const double *)S, lds, Wk, U, ranks, sat, rows);
}

void launch_block_norms(int32_t njobs, const QrJob *jobs, int32_t r, double scale, bool f32,
                        const void *S, int64_t lds, double *out, hipStream_t s) {
  if (njobs <= 0) return;
  if (f32)
    block_norm_kernel<float><<<njobs, 256, 0, s>>>(jobs, r, scale, (const float *)S, lds, out);
  else
    block_norm_kernel<double><<<njobs, 256, 0, s>>>(jobs, r, scale, (const double *)S, lds, out);
}

void launch_recover(const RecoverArgs &a, int grid, bool f32, const void *Omega, const void *Psi,
                    const void *Y, hipStream_t s) {
  if (a.njobs <= 0) return;
  const size_t core_sh = 33 * 2 * (size_t)a.r;
  const size_t sa = ((size_t)a.r * a.r > 33 * (size_t)(a.r + a.kmax)) ? (size_t)a.r * a.r
                                                                       : 33 * (size_t)(a.r + a.kmax);
  RecoverArgs b = a;
  b.qr_rows = qr_lds_rows(a.r, 0);
  const size_t qr_sh = 2 * (size_t)b.qr_rows * a.r;
  const size_t sh = sizeof(double) * std::max(std::max(core_sh, sa + (size_t)a.r * a.kmax), qr_sh);
  const unsigned g = (unsigned)std::max(1, std::min(grid, (int)a.njobs));
  if (f32)
    recover_kernel<float><<<g, 256, sh, s>>>(b, (const float *)Omega, (const float *)Psi,
                                             (const float *)Y);
  else
    recover_kernel<double><<<g, 256, sh, s>>>(b, (const double *)Omega, (const double *)Psi,
                                              (const double *)Y);
}

}  // namespace hm
