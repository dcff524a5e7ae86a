// Test-matrix draws and data-movement kernels (HBM-bound, coalesced along
// the column-major row index).
#include "device_common.h"
#include "kernels.h"

namespace hm {

namespace {

template <typename T>
__global__ void __launch_bounds__(256) testmat_kernel(int64_t n, const int32_t *__restrict__ rowbox,
                                                      const uint8_t *__restrict__ active,
                                                      int32_t ncolors, int32_t r, int32_t level,
                                                      int32_t pass, uint32_t k0, uint32_t k1,
                                                      const int64_t *__restrict__ inst_off,
                                                      int32_t ninst, T *__restrict__ out,
                                                      int64_t ld, int64_t ncols_pad) {
  // one thread per (row, column pair); consecutive threads walk rows
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t jp = blockIdx.y;          // (color, column pair) index
  const int npair = (r + 1) / 2;
  const int c = (int)(jp / npair);
  const int jj = (int)(jp % npair);
  double z0 = 0.0, z1 = 0.0;
  bool in0 = c < ncolors;
  if (in0 && active[(int64_t)rowbox[i] * ncolors + c]) {
    // forest: the row's instance (binary search over the row offsets)
    // supplies the key seed + instance and the row count restarts at 0
    int64_t row = i;
    uint32_t q0 = k0, q1 = k1;
    if (ninst > 1) {
      int lo = 0, hi = ninst;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (inst_off[mid] <= i)
          lo = mid;
        else
          hi = mid;
      }
      row = i - inst_off[lo];
      const uint64_t key = ((((uint64_t)k1) << 32) | k0) + (uint64_t)lo;
      q0 = (uint32_t)key;
      q1 = (uint32_t)(key >> 32);
    }
    dev::U4 ctr{(uint32_t)row, (uint32_t)jj, (uint32_t)c, (uint32_t)(4 * level + pass)};
    dev::normal_pair(dev::philox10(ctr, q0, q1), z0, z1);
  }
  // the pair (2jj, 2jj+1) lives in color block c; when r is odd the second
  // value of the last pair is dropped and the next block starts
  const int64_t c0 = (int64_t)c * r + 2 * jj;
  if (in0) {
    out[c0 * ld + i] = (T)z0;
    if (2 * jj + 1 < r) out[(c0 + 1) * ld + i] = (T)z1;
  }
}

// padding columns [ncolors*r, ncols_pad) are zeroed
template <typename T>
__global__ void zero_cols(int64_t n, int64_t c0, int64_t c1, T *out, int64_t ld) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t c = c0 + blockIdx.y; c < c1; c += gridDim.y) out[c * ld + i] = (T)0;
}

template <typename T>
__global__ void fill_kernel(T *p, int64_t count, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename T>
__global__ void leaf_ones(int32_t nitems, const int32_t *item_box, const int32_t *item_color,
                          const int64_t *box_start, int32_t m, T *out, int64_t ld) {
  const int it = blockIdx.x;
  if (it >= nitems) return;
  const int b = item_box[it];
  const int64_t s0 = box_start[b], s1 = box_start[b + 1];
  const int64_t cbase = (int64_t)item_color[it] * m;
  for (int64_t t = threadIdx.x; t < s1 - s0 && t < m; t += blockDim.x)
    out[(cbase + t) * ld + s0 + t] = (T)1;
}

template <typename T>
__global__ void permute_rows_kernel(int64_t n, int64_t ncols, const int64_t *idx, int scatter,
                                    const T *src, int64_t lds, T *dst, int64_t ldd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t j = idx[i];
  for (int64_t c = blockIdx.y; c < ncols; c += gridDim.y) {
    if (scatter)
      dst[c * ldd + j] = src[c * lds + i];
    else
      dst[c * ldd + i] = src[c * lds + j];
  }
}

template <typename S, typename D>
__global__ void convert_kernel(int64_t n, int64_t ncols, const S *src, int64_t lds, D *dst,
                               int64_t ldd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t c = blockIdx.y; c < ncols; c += gridDim.y) dst[c * ldd + i] = (D)src[c * lds + i];
}

__global__ void philox_raw_kernel(const uint32_t *ctr, int64_t count, uint32_t k0, uint32_t k1,
                                  uint32_t *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  dev::U4 c{ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
  dev::U4 r = dev::philox10(c, k0, k1);
  out[4 * i] = r.x;
  out[4 * i + 1] = r.y;
  out[4 * i + 2] = r.z;
  out[4 * i + 3] = r.w;
}

template <typename T>
__global__ void extract_near_kernel(const int64_t *row0, const int32_t *ma, const int64_t *col0,
                                    const int32_t *mb, const int64_t *dst_off, const T *Y,
                                    int64_t ldy, double *D) {
  const int p = blockIdx.x;
  const int64_t r0 = row0[p], c0 = col0[p];
  const int m = ma[p], w = mb[p];
  double *d = D + dst_off[p];
  for (int j = 0; j < w; ++j)
    for (int i = threadIdx.x; i < m; i += blockDim.x) d[(int64_t)j * m + i] = (double)Y[(c0 + j) * ldy + r0 + i];
}

template <typename T>
__global__ void finite_kernel(int64_t n, int64_t ncols, const T *Y, int64_t ldy, int32_t *flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int bad = 0;
  if (i < n)
    for (int64_t c = blockIdx.y; c < ncols; c += gridDim.y) {
      const double v = (double)Y[c * ldy + i];
      if (!(v - v == 0.0)) bad = 1;
    }
  if (bad) flag[0] = 1;
}

inline dim3 grid_rows(int64_t n, int64_t ycols) {
  int64_t gy = ycols < 1 ? 1 : (ycols > 65535 ? 65535 : ycols);
  return dim3((unsigned)((n + 255) / 256), (unsigned)gy);
}

}  // namespace

void launch_testmat(int64_t n, const int32_t *rowbox, const uint8_t *active, int32_t ncolors,
                    int32_t r, int32_t level, int32_t pass, uint64_t seed,
                    const int64_t *inst_off, int32_t ninst, bool f32, void *out, int64_t ld,
                    int64_t ncols_pad, hipStream_t s) {
  if (n <= 0) return;
  const int64_t npairs = (int64_t)ncolors * ((r + 1) / 2);
  const uint32_t k0 = (uint32_t)(seed & 0xFFFFFFFFu), k1 = (uint32_t)(seed >> 32);
  if (npairs > 0) {
    dim3 g((unsigned)((n + 255) / 256), (unsigned)npairs);
    if (f32)
      testmat_kernel<float><<<g, 256, 0, s>>>(n, rowbox, active, ncolors, r, level, pass, k0, k1,
                                              inst_off, ninst, (float *)out, ld, ncols_pad);
    else
      testmat_kernel<double><<<g, 256, 0, s>>>(n, rowbox, active, ncolors, r, level, pass, k0,
                                               k1, inst_off, ninst, (double *)out, ld, ncols_pad);
  }
  const int64_t c0 = (int64_t)ncolors * r;
  if (ncols_pad > c0) {
    dim3 g = grid_rows(n, ncols_pad - c0);
    if (f32)
      zero_cols<float><<<g, 256, 0, s>>>(n, c0, ncols_pad, (float *)out, ld);
    else
      zero_cols<double><<<g, 256, 0, s>>>(n, c0, ncols_pad, (double *)out, ld);
  }
}

void launch_fill(void *p, int64_t count, bool f32, double value, hipStream_t s) {
  if (count <= 0) return;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (f32)
    fill_kernel<float><<<(unsigned)blocks, 256, 0, s>>>((float *)p, count, (float)value);
  else
    fill_kernel<double><<<(unsigned)blocks, 256, 0, s>>>((double *)p, count, value);
}

void launch_fill_cols(void *p, int64_t n, int64_t ncols, int64_t ld, bool f32, hipStream_t s) {
  if (n <= 0 || ncols <= 0) return;
  dim3 g = grid_rows(n, ncols);
  if (f32)
    zero_cols<float><<<g, 256, 0, s>>>(n, 0, ncols, (float *)p, ld);
  else
    zero_cols<double><<<g, 256, 0, s>>>(n, 0, ncols, (double *)p, ld);
}

void launch_leaf_identity(int64_t n, int32_t nitems, const int32_t *item_box,
                          const int32_t *item_color, const int64_t *box_start, int32_t m,
                          bool f32, void *out, int64_t ld, int64_t ncols_pad, hipStream_t s) {
  launch_fill(out, ld * ncols_pad, f32, 0.0, s);
  if (nitems <= 0) return;
  if (f32)
    leaf_ones<float><<<nitems, 128, 0, s>>>(nitems, item_box, item_color, box_start, m,
                                            (float *)out, ld);
  else
    leaf_ones<double><<<nitems, 128, 0, s>>>(nitems, item_box, item_color, box_start, m,
                                             (double *)out, ld);
}

void launch_permute_rows(int64_t n, int64_t ncols, const int64_t *idx, bool scatter, bool f32,
                         const void *src, int64_t lds, void *dst, int64_t ldd, hipStream_t s) {
  if (n <= 0 || ncols <= 0) return;
  dim3 g = grid_rows(n, ncols);
  if (f32)
    permute_rows_kernel<float><<<g, 256, 0, s>>>(n, ncols, idx, scatter ? 1 : 0,
                                                 (const float *)src, lds, (float *)dst, ldd);
  else
    permute_rows_kernel<double><<<g, 256, 0, s>>>(n, ncols, idx, scatter ? 1 : 0,
                                                  (const double *)src, lds, (double *)dst, ldd);
}

void launch_convert(int64_t n, int64_t ncols, bool src_f32, const void *src, int64_t lds,
                    void *dst, int64_t ldd, hipStream_t s) {
  if (n <= 0 || ncols <= 0) return;
  dim3 g = grid_rows(n, ncols);
  if (src_f32)
    convert_kernel<float, double><<<g, 256, 0, s>>>(n, ncols, (const float *)src, lds,
                                                    (double *)dst, ldd);
  else
    convert_kernel<double, float><<<g, 256, 0, s>>>(n, ncols, (const double *)src, lds,
                                                    (float *)dst, ldd);
}

void launch_philox_raw(const uint32_t *ctr, int64_t count, uint32_t k0, uint32_t k1,
                       uint32_t *out, hipStream_t s) {
  if (count <= 0) return;
  philox_raw_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(ctr, count, k0, k1, out);
}

void launch_extract_near(int32_t np, const int64_t *row0, const int32_t *ma, const int64_t *col0,
                         const int32_t *mb, const int64_t *dst_off, bool f32, const void *Y,
                         int64_t ldy, double *D, hipStream_t s) {
  if (np <= 0) return;
  if (f32)
    extract_near_kernel<float><<<np, 128, 0, s>>>(row0, ma, col0, mb, dst_off, (const float *)Y,
                                                  ldy, D);
  else
    extract_near_kernel<double><<<np, 128, 0, s>>>(row0, ma, col0, mb, dst_off,
                                                   (const double *)Y, ldy, D);
}

void launch_check_finite(int64_t n, int64_t ncols, bool f32, const void *Y, int64_t ldy,
                         int32_t *flag, hipStream_t s) {
  if (n <= 0 || ncols <= 0) return;
  dim3 g = grid_rows(n, ncols < 64 ? ncols : 64);
  if (f32)
    finite_kernel<float><<<g, 256, 0, s>>>(n, ncols, (const float *)Y, ldy, flag);
  else
    finite_kernel<double><<<g, 256, 0, s>>>(n, ncols, (const double *)Y, ldy, flag);
}

}  // namespace hm
