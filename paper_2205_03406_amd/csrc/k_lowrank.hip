// Grouped low-rank products for the peeling subtraction and the H^1 apply:
//   project  T_p = R_p^T X(col box)            (one job per admissible pair)
//   expand   Y(row chunk) += sign * sum_p L_p(chunk rows) T_p
//   near     Y(row chunk) += sum_q D_q(chunk rows) X(col box of q)
// and the dense FP64 GEMM behind the dense test black box.
//
// Every output row chunk is owned by one workgroup, which sums all of its
// contributions in registers before a single read-modify-write of Y: the
// result is deterministic (no atomics) and each Y element is written once
// per call.  Tiles are 64 rows x 64 columns on the matrix cores (FP64, or
// FP32 in the mixed path), the contraction staged through LDS 16 (project,
// expand) or 32 (near) deep.
#include <algorithm>
#include <stdexcept>
#include <string>

#include "device_common.h"
#include "kernels.h"

namespace hm {

namespace {

constexpr int TC = 64;  // columns per workgroup
constexpr int KC = 32;  // contraction chunk

// Both kernels run on the matrix cores: a 64 x 64 output tile per
// workgroup, wave w owning rows [16w, 16w + 16) as four 16 x 16 MFMA tiles;
// the contraction is staged 32 deep through LDS (single buffer) with the next
// stage fetched into registers while the current one is multiplied.  MFMA is
// used for its issue efficiency on these skinny products (one instruction
// per 16x16x4 block instead of 16 FMAs and their operand reads).
typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
template <typename T>
struct Acc;
template <>
struct Acc<double> {
  typedef d4v type;
  static __device__ __forceinline__ void step(double a, double b, d4v &c) {
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of item i of lane l inside a 16 x 16 tile
  static __device__ __forceinline__ int row(int i, int lane) { return 4 * i + (lane >> 4); }
};
template <>
struct Acc<float> {
  typedef f4v type;
  static __device__ __forceinline__ void step(float a, float b, f4v &c) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int i, int lane) { return 4 * (lane >> 4) + i; }
};

constexpr int PMAX = 128;  // packed output rows of one projection item

// Projection: the pairs of one item share a column box; their rank columns
// are packed end to end (actual device ranks) into at most PMAX output rows,
// all of them accumulated in one sweep over the item's rows (NP passes of
// 64 output rows side by side), so each X tile is fetched once per item.
// Given the zero pattern of a colored X, the sweep covers only the rows of
// the sampled level's boxes that are active in a color of the column tile
// (their segments listed in LDS first); elsewhere X is zero in the tile.
// A box holds about one active color of the 50 to 100 of a level, so most
// tiles of most items have no rows to sweep at all: T is left unwritten
// and the tile flagged 0 for the expansion.
// (Walking several column tiles per workgroup, to set the packing up once
// and keep the prefetch running across tiles, measured slower at 2 and 4
// tiles: neighbouring workgroups then no longer share X rows in L2.)
template <typename T, int NTW, int KD>
__global__ void __launch_bounds__(256, 2)
lr_project_kernel(const ProjItem *__restrict__ items, const ProjPair *__restrict__ pairs,
                  int32_t kmax, int64_t tstride, const int32_t *__restrict__ ranks,
                  const T *__restrict__ R, const T *__restrict__ X, int64_t ldx, int64_t ncols,
                  T *__restrict__ Tout, ColorPattern pat, uint8_t *__restrict__ flags,
                  int32_t nitems, int32_t ntiles) {
  constexpr int NP = PMAX / 64;
  constexpr int MAXSEG = 256;  // boxes of the sampled level inside one item
  constexpr int QS = 256 / KD;              // output rows / columns per fetch round
  constexpr int NA = PMAX / QS, NB = 16 * NTW / QS;  // fetch rounds of R and X
  static_assert(KD % 4 == 0 && 256 % KD == 0 && PMAX % QS == 0 && (16 * NTW) % QS == 0,
                "fetch layout");
  __shared__ T As[KD][PMAX + 1];   // [depth][output row]
  __shared__ T Bs[KD][16 * NTW + 1];   // [depth][col]
  __shared__ int64_t o_r[PMAX];  // R element offset of output row (segment start)
  __shared__ int64_t o_t[PMAX];  // T element offset of output row
  __shared__ int p_k[PMAX], p_o[PMAX + 1];
  __shared__ int32_t sg_s[MAXSEG], sg_e[MAXSEG];  // live row segments [s, e) of the item
  __shared__ int32_t w_cnt[4], s_nseg;
  typedef typename Acc<T>::type acc_t;
  int64_t item, tile;
  dev::xcd_item_tile(nitems, ntiles, item, tile);
  const ProjItem it = items[item];
  const int64_t c0 = tile * (16 * NTW);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // packing of the pairs' rank columns: ranks read in parallel, offsets by
  // a short serial scan (at most PMAX pairs), rows filled per pair
  const int np = it.npairs < PMAX ? it.npairs : PMAX;
  if (tid < np) p_k[tid] = ranks[pairs[it.first + tid].kidx];
  __syncthreads();
  if (tid == 0) {
    int o = 0;
    for (int j = 0; j < np; ++j) {
      p_o[j] = o;
      o = min(o + p_k[j], PMAX);
    }
    p_o[np] = o;
  }
  __syncthreads();
  if (tid < np) {
    const ProjPair pp = pairs[it.first + tid];
    for (int o = p_o[tid], kk = 0; o < p_o[tid + 1]; ++o, ++kk) {
      o_r[o] = pp.rslot + it.seg_off + (int64_t)kk * it.m;
      o_t[o] = (int64_t)pp.tslot * tstride + kk;
    }
  }
  // live row segments for this tile's colors
  bool dense = pat.rowbox == nullptr || it.nrows <= 0;
  int b0 = 0, nb = 0;
  if (!dense) {
    b0 = pat.rowbox[it.row0];
    nb = pat.rowbox[it.row0 + it.nrows - 1] - b0 + 1;
    dense = nb > MAXSEG;
  }
  if (dense) {
    if (tid == 0) {
      sg_s[0] = 0;
      sg_e[0] = it.nrows;
      s_nseg = it.nrows > 0 ? 1 : 0;
    }
  } else {
    const int64_t cend = c0 + 16 * NTW < ncols ? c0 + 16 * NTW : ncols;
    const int ca = (int)((pat.col0 + c0) / pat.colw);
    const int cb =
        c0 < ncols ? (int)min<int64_t>((pat.col0 + cend - 1) / pat.colw, pat.ncolors - 1) : -1;
    bool live = false;
    int ss = 0, se = 0;
    if (tid < nb) {
      const int b = b0 + tid;
      ss = (int)(max(pat.bstart[b], it.row0) - it.row0);
      se = (int)(min(pat.bstart[b + 1], it.row0 + it.nrows) - it.row0);
      for (int c = ca; c <= cb && !live; ++c) live = pat.act[(int64_t)b * pat.ncolors + c] != 0;
      live = live && se > ss;
    }
    const uint64_t m = __ballot(live);
    if (lane == 0) w_cnt[wave] = __popcll(m);
    __syncthreads();
    int k = 0;
    for (int w = 0; w < wave; ++w) k += w_cnt[w];
    if (live) {
      k += __popcll(m & ((uint64_t(1) << lane) - 1));
      sg_s[k] = ss;
      sg_e[k] = se;
    }
    if (tid == 0) s_nseg = w_cnt[0] + w_cnt[1] + w_cnt[2] + w_cnt[3];
  }
  __syncthreads();
  const int nout = p_o[np];
  const int nseg = s_nseg;
  const bool any = nout > 0 && nseg > 0;
  if (flags && tid < np) flags[(int64_t)pairs[it.first + tid].tslot * ntiles + tile] = any ? 1 : 0;
  if (!any) return;  // uniform: nothing to project
  acc_t acc[NP][NTW];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int t = 0; t < NTW; ++t) acc[p][t] = (acc_t){0, 0, 0, 0};
  // thread operands: row r0 + (tid mod KD) (below re, the segment's end)
  // of output rows / columns tid / KD + QS q
  T av[NA], bv[NB];
  auto fetch = [&](int r0, int re) {
    const int row = r0 + (tid % KD);
    const bool rv = row < re;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int o = tid / KD + QS * q;
      av[q] = (rv && o < nout) ? R[o_r[o] + row] : (T)0;
    }
    const T *xr = X + it.row0 + row;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int64_t gc = c0 + tid / KD + QS * q;
      bv[q] = (rv && gc < ncols) ? xr[gc * ldx] : (T)0;
    }
  };
  // steps of KD rows through the live segments, the next one prefetched
  int cs = 0, cr = sg_s[0];
  fetch(cr, sg_e[0]);
  for (;;) {
#pragma unroll
    for (int q = 0; q < NA; ++q) As[tid % KD][tid / KD + QS * q] = av[q];
#pragma unroll
    for (int q = 0; q < NB; ++q) Bs[tid % KD][tid / KD + QS * q] = bv[q];
    __syncthreads();
    int ns = cs, nr = cr + KD;
    if (nr >= sg_e[ns]) {
      ++ns;
      nr = ns < nseg ? sg_s[ns] : 0;
    }
    const bool more = ns < nseg;
    if (more) fetch(nr, sg_e[ns]);
#pragma unroll
    for (int ks = 0; ks < KD; ks += 4) {
      T b[NTW];
#pragma unroll
      for (int t = 0; t < NTW; ++t) b[t] = Bs[ks + (lane >> 4)][16 * t + (lane & 15)];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        if (64 * p + 16 * wave < nout) {  // uniform across the wave: rows of the pass it holds
          const T a = As[ks + (lane >> 4)][64 * p + 16 * wave + (lane & 15)];
#pragma unroll
          for (int t = 0; t < NTW; ++t) Acc<T>::step(a, b[t], acc[p][t]);
        }
      }
    }
    __syncthreads();
    if (!more) break;
    cs = ns;
    cr = nr;
  }
#pragma unroll
  for (int p = 0; p < NP; ++p) {
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
      const int64_t gc = c0 + 16 * t + (lane & 15);
      if (gc >= ncols) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int o = 64 * p + 16 * wave + Acc<T>::row(i, lane);
        if (o < nout) Tout[o_t[o] + gc * kmax] = acc[p][t][i];
      }
    }
  }
}

// Expansion: the entries of a chunk form one contraction of depth
// sum_e rank_e (actual device ranks, packed end to end), taken in passes of
// up to EMAX entries and DMAX depths; per pass a depth -> (L offset, T
// offset) table in LDS, so that every operand fetch is one table read and
// one load.  The partial projections of pairs split over segments must be
// summed into their first slot beforehand (lr_reduce_kernel).
constexpr int EMAX = 32;
constexpr int DMAX = 384;

// four waves per SIMD (at most 128 VGPRs): 11 % faster than three at 288
// columns; the latency of the operand fetches needs the waves
template <typename T, int NTW, int KD>
__global__ void __launch_bounds__(256, 4)
lr_expand_kernel(const ExpandChunk *__restrict__ chunks, const ExpandEntry *__restrict__ entries,
                 int32_t kmax, int64_t tstride, const int32_t *__restrict__ ranks,
                 const T *__restrict__ L, const T *__restrict__ Tin, int64_t ncols, T sign,
                 T *__restrict__ Y, int64_t ldy, const uint8_t *__restrict__ flags,
                 int32_t nitems, int32_t ntiles) {
  constexpr int QS = 256 / KD;  // T columns per fetch round
  constexpr int NA = KD / 4, NB = 16 * NTW / QS;  // fetch rounds of L and T
  static_assert(KD % 4 == 0 && 256 % KD == 0 && (16 * NTW) % QS == 0, "fetch layout");
  __shared__ T As[KD][64 + 1];   // [depth][row]
  __shared__ T Bs[KD][16 * NTW + 1];   // [depth][col]
  __shared__ int64_t d_l[DMAX];  // L element offset of depth d at the chunk's first row
  __shared__ int64_t d_t[DMAX];  // T element offset of depth d at column 0
  __shared__ int32_t e_k[EMAX], e_ko[EMAX + 1];
  __shared__ int32_t s_ne;
  typedef typename Acc<T>::type acc_t;
  int64_t item, tile;
  dev::xcd_item_tile(nitems, ntiles, item, tile);
  const ExpandChunk ch = chunks[item];
  const int64_t c0 = tile * (16 * NTW);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // a wave whose 16 rows all lie past the chunk's end has nothing to add
  const bool rows_live = 16 * wave < ch.nrows;
  acc_t acc[NTW];
#pragma unroll
  for (int t = 0; t < NTW; ++t) acc[t] = (acc_t){0, 0, 0, 0};
  bool touched = false;  // any depth contracted (uniform across the workgroup)

  for (int e0 = ch.first; e0 < ch.last;) {
    const int avail = min(EMAX, ch.last - e0);
    __syncthreads();  // the previous pass is done with the tables
    if (tid < avail) {
      // an entry whose projection is zero in this tile (flag 0) adds nothing
      const ExpandEntry en = entries[e0 + tid];
      const bool z = flags && !flags[(int64_t)en.tslot * ntiles + tile];
      e_k[tid] = z ? 0 : ranks[en.kidx];
    }
    __syncthreads();
    if (tid == 0) {
      // entries while the depth fits (every rank <= kmax <= DMAX: at least one)
      int a = 0, i = 0;
      for (; i < avail && a + e_k[i] <= DMAX; ++i) {
        e_ko[i] = a;
        a += e_k[i];
      }
      e_ko[i] = a;
      s_ne = i;
    }
    __syncthreads();
    const int ne = s_ne;
    if (tid < ne) {
      const ExpandEntry en = entries[e0 + tid];
      const int64_t lb = en.lslot + en.off;
      const int64_t tb = (int64_t)en.tslot * tstride;
      for (int kk = 0, d = e_ko[tid]; kk < e_k[tid]; ++kk, ++d) {
        d_l[d] = lb + (int64_t)kk * en.mq;
        d_t[d] = tb + kk;
      }
    }
    __syncthreads();
    const int ktot = e_ko[ne];
    touched = touched || ktot > 0;
    T av[NA], bv[NB];
    auto fetch = [&](int k0) {
      // L: the lane's chunk row at depth k0 + wave + 4 q (one depth per wave)
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const int d = k0 + wave + 4 * q;
        av[q] = (d < ktot && lane < ch.nrows) ? L[d_l[d] + lane] : (T)0;
      }
      // T: depth k0 + (tid mod KD) at columns tid / KD + QS q
      const int d = k0 + tid % KD;
      const bool dv = d < ktot;
      const int64_t tb = dv ? d_t[d] : 0;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int64_t gc = c0 + tid / KD + QS * q;
        bv[q] = (dv && gc < ncols) ? Tin[tb + gc * kmax] : (T)0;
      }
    };
    if (ktot > 0) fetch(0);
    for (int k0 = 0; k0 < ktot; k0 += KD) {
#pragma unroll
      for (int q = 0; q < NA; ++q) As[wave + 4 * q][lane] = av[q];
#pragma unroll
      for (int q = 0; q < NB; ++q) Bs[tid % KD][tid / KD + QS * q] = bv[q];
      __syncthreads();
      if (k0 + KD < ktot) fetch(k0 + KD);
      if (rows_live) {
#pragma unroll
        for (int ks = 0; ks < KD; ks += 4) {
          const T a = As[ks + (lane >> 4)][16 * wave + (lane & 15)];
#pragma unroll
          for (int t = 0; t < NTW; ++t)
            Acc<T>::step(a, Bs[ks + (lane >> 4)][16 * t + (lane & 15)], acc[t]);
        }
      }
      __syncthreads();
    }
    e0 += ne;
  }
  if (!rows_live || !touched) return;  // nothing to add: Y is left as it is
#pragma unroll
  for (int t = 0; t < NTW; ++t) {
    const int64_t gc = c0 + 16 * t + (lane & 15);
    if (gc >= ncols) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rr = 16 * wave + Acc<T>::row(i, lane);
      if (rr < ch.nrows) {
        T *y = Y + gc * ldy + ch.row0 + rr;
        *y += sign * acc[t][i];
      }
    }
  }
}

// Near field on the matrix cores, laid out like the expansion: the entries
// of a chunk (neighbor boxes, at most 128 columns each) form one contraction
// of depth sum_e mb_e, staged 32 deep through LDS; a depth -> (entry,
// column) table is built per pass of up to NEMAX entries.  overwrite: the
// chunk's rows of Y are written instead of accumulated (the first term of an
// apply, so Y needs no clearing).
constexpr int NEMAX = 32;
constexpr int NKTAB = NEMAX * 128;

template <typename T, int NTW>
__global__ void __launch_bounds__(256, 2)
near_kernel(const ExpandChunk *__restrict__ chunks, const NearEntry *__restrict__ entries,
            const double *__restrict__ D, const T *__restrict__ X, int64_t ldx, int64_t ncols,
            T *__restrict__ Y, int64_t ldy, int overwrite, int32_t nitems, int32_t ntiles) {
  __shared__ T As[KC][64 + 1];   // [depth][row]
  __shared__ T Bs[KC][16 * NTW + 1];   // [depth][col]
  __shared__ int64_t e_d[NEMAX], e_x[NEMAX];
  __shared__ int32_t e_ma[NEMAX], e_mb[NEMAX], e_tr[NEMAX], e_ko[NEMAX + 1];
  __shared__ int16_t d_e[NKTAB];
  __shared__ uint8_t d_k[NKTAB];
  typedef typename Acc<T>::type acc_t;
  int64_t item, tile;
  dev::xcd_item_tile(nitems, ntiles, item, tile);
  const ExpandChunk ch = chunks[item];
  const int64_t c0 = tile * (16 * NTW);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  acc_t acc[NTW];
#pragma unroll
  for (int t = 0; t < NTW; ++t) acc[t] = (acc_t){0, 0, 0, 0};

  for (int e0 = ch.first; e0 < ch.last; e0 += NEMAX) {
    const int ne = min(NEMAX, ch.last - e0);
    __syncthreads();
    if (tid < ne) {
      const NearEntry en = entries[e0 + tid];
      // element (row i, column k) of the block: D[e_d + k ma + i], or
      // D[e_d + i ma + k] for a transposed entry
      e_d[tid] = en.dslot + (en.trans ? (int64_t)en.off * en.ma : (int64_t)en.off);
      e_x[tid] = en.xrow0;
      e_ma[tid] = en.ma;
      e_mb[tid] = en.mb;
      e_tr[tid] = en.trans;
    }
    __syncthreads();
    if (tid == 0) {
      int a = 0;
      for (int i = 0; i < ne; ++i) {
        e_ko[i] = a;
        a += e_mb[i];
      }
      e_ko[ne] = a;
    }
    __syncthreads();
    if (tid < ne)
      for (int kk = 0; kk < e_mb[tid]; ++kk) {
        d_e[e_ko[tid] + kk] = (int16_t)tid;
        d_k[e_ko[tid] + kk] = (uint8_t)kk;
      }
    __syncthreads();
    const int ktot = e_ko[ne];
    T av[8], bv[2 * NTW];
    auto fetch = [&](int k0) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int e = tid + 256 * q;
        {
          const int rr = e % 64, kk = e / 64;   // D (row, depth)
          const int d = k0 + kk;
          T v = 0;
          if (d < ktot && rr < ch.nrows) {
            const int j = d_e[d];
            const int k = d_k[d];
            v = (T)(e_tr[j] ? D[e_d[j] + (int64_t)rr * e_ma[j] + k]
                            : D[e_d[j] + (int64_t)k * e_ma[j] + rr]);
          }
          av[q] = v;
        }
      }
#pragma unroll
      for (int q = 0; q < 2 * NTW; ++q) {
        const int e = tid + 256 * q;
        const int kt = e % KC, cc = e / KC;   // X (depth, column)
        const int d = k0 + kt;
        const int64_t gc = c0 + cc;
        T v = 0;
        if (d < ktot && gc < ncols) v = X[gc * ldx + e_x[d_e[d]] + d_k[d]];
        bv[q] = v;
      }
    };
    if (ktot > 0) fetch(0);
    for (int k0 = 0; k0 < ktot; k0 += KC) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int e = tid + 256 * q;
        As[e / 64][e % 64] = av[q];
      }
#pragma unroll
      for (int q = 0; q < 2 * NTW; ++q) {
        const int e = tid + 256 * q;
        Bs[e % KC][e / KC] = bv[q];
      }
      __syncthreads();
      if (k0 + KC < ktot) fetch(k0 + KC);
#pragma unroll
      for (int ks = 0; ks < KC; ks += 4) {
        const T a = As[ks + (lane >> 4)][16 * wave + (lane & 15)];
#pragma unroll
        for (int t = 0; t < NTW; ++t)
          Acc<T>::step(a, Bs[ks + (lane >> 4)][16 * t + (lane & 15)], acc[t]);
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int t = 0; t < NTW; ++t) {
    const int64_t gc = c0 + 16 * t + (lane & 15);
    if (gc >= ncols) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rr = 16 * wave + Acc<T>::row(i, lane);
      if (rr < ch.nrows) {
        T *y = Y + gc * ldy + ch.row0 + rr;
        *y = overwrite ? acc[t][i] : *y + acc[t][i];
      }
    }
  }
}

// Partial projections of a pair split over several row segments, summed
// into the first segment's slot: T[s0] = T[s0] + T[s0 + 1] + ... (in order).
template <typename T>
__global__ void __launch_bounds__(256)
lr_reduce_kernel(const ReduceItem *__restrict__ items, int64_t tstride, int64_t elems,
                 T *__restrict__ Tb) {
  const ReduceItem it = items[blockIdx.y];
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < elems;
       e += (int64_t)gridDim.x * 256) {
    T *p = Tb + (int64_t)it.slot * tstride + e;
    T v = p[0];
    for (int sg = 1; sg < it.nseg; ++sg) v += p[(int64_t)sg * tstride];
    p[0] = v;
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

// Workgroups of 64 columns (4 MFMA column tiles per wave).  Wider tiles
// (8 per wave, 128 columns) measured slower for all three kernels at 288
// and 1024 columns: the kernels are bound by the latency of their operand
// fetches, and wider tiles halve the resident workgroups that hide it.
constexpr int kNTW = 4;
static_assert(16 * kNTW == kLowRankTile, "projection and expansion share the column tiling");
// contraction depth per LDS stage of the projection and the expansion: 16
// (half the LDS and prefetch registers of 32, four waves per SIMD instead
// of three for the projection) measured 6 % faster over the sphere's peel
constexpr int kProjDepth = 16;
constexpr int kExpandDepth = 16;

template <int NTW>
inline unsigned tiles_of(int64_t ncols) {
  return (unsigned)((ncols + 16 * NTW - 1) / (16 * NTW));
}

// workgroups of a 1-D (item, tile) grid; the work-items of one grid
// dimension must stay below 2^32
inline unsigned grid_of(int64_t nitems, unsigned ntiles) {
  const int64_t g = nitems * (int64_t)ntiles;
  if (g * 256 >= (int64_t(1) << 32))
    throw std::runtime_error("low-rank launch of " + std::to_string(g) + " workgroups is too large");
  return (unsigned)g;
}

template <typename T, int NTW>
void project_ntw(int32_t nitems, const ProjItem *items, const ProjPair *pairs, int32_t kmax,
                 int64_t tstride, const int32_t *ranks, const void *R, const void *X, int64_t ldx,
                 int64_t ncols, void *Tb, const ColorPattern *pat, uint8_t *flags,
                 hipStream_t s) {
  const unsigned nt = tiles_of<NTW>(ncols);
  const ColorPattern cp = pat ? *pat : ColorPattern{nullptr, nullptr, nullptr, 0, 1, 0};
  lr_project_kernel<T, NTW, kProjDepth><<<grid_of(nitems, nt), 256, 0, s>>>(
      items, pairs, kmax, tstride, ranks, (const T *)R, (const T *)X, ldx, ncols, (T *)Tb, cp,
      pat ? flags : nullptr, nitems, (int32_t)nt);
}

template <typename T, int NTW>
void expand_ntw(int32_t nchunks, const ExpandChunk *chunks, const ExpandEntry *entries,
                int32_t kmax, int64_t tstride, const int32_t *ranks, const void *L,
                const void *Tb, int64_t ncols, double sign, void *Y, int64_t ldy,
                const uint8_t *flags, hipStream_t s) {
  const unsigned nt = tiles_of<NTW>(ncols);
  lr_expand_kernel<T, NTW, kExpandDepth><<<grid_of(nchunks, nt), 256, 0, s>>>(
      chunks, entries, kmax, tstride, ranks, (const T *)L, (const T *)Tb, ncols, (T)sign, (T *)Y,
      ldy, flags, nchunks, (int32_t)nt);
}

template <typename T, int NTW>
void near_ntw(int32_t nchunks, const ExpandChunk *chunks, const NearEntry *entries,
              const void *D, const void *X, int64_t ldx, int64_t ncols, void *Y, int64_t ldy,
              bool overwrite, hipStream_t s) {
  const unsigned nt = tiles_of<NTW>(ncols);
  near_kernel<T, NTW><<<grid_of(nchunks, nt), 256, 0, s>>>(
      chunks, entries, (const double *)D, (const T *)X, ldx, ncols, (T *)Y, ldy,
      overwrite ? 1 : 0, nchunks, (int32_t)nt);
}

void launch_lr_project(int32_t nitems, const ProjItem *items, const ProjPair *pairs, int32_t kmax,
                       int64_t tstride, const int32_t *ranks, bool f32, const void *R,
                       const void *X, int64_t ldx, int64_t ncols, void *T,
                       const ColorPattern *pat, uint8_t *flags, hipStream_t s) {
  if (nitems <= 0 || ncols <= 0) return;
  if (pat && (!flags || pat->colw < 1 || pat->ncolors < 1))
    throw std::runtime_error("projection with a color pattern needs flags and colors");
  if (f32)
    project_ntw<float, kNTW>(nitems, items, pairs, kmax, tstride, ranks, R, X, ldx, ncols, T, pat,
                             flags, s);
  else
    project_ntw<double, kNTW>(nitems, items, pairs, kmax, tstride, ranks, R, X, ldx, ncols, T,
                              pat, flags, s);
}

void launch_lr_expand(int32_t nchunks, const ExpandChunk *chunks, const ExpandEntry *entries,
                      int32_t kmax, int64_t tstride, const int32_t *ranks, bool f32,
                      const void *L, const void *T, int64_t ncols, double sign, void *Y,
                      int64_t ldy, const uint8_t *flags, hipStream_t s) {
  if (nchunks <= 0 || ncols <= 0) return;
  if (f32)
    expand_ntw<float, kNTW>(nchunks, chunks, entries, kmax, tstride, ranks, L, T, ncols, sign, Y,
                            ldy, flags, s);
  else
    expand_ntw<double, kNTW>(nchunks, chunks, entries, kmax, tstride, ranks, L, T, ncols, sign, Y,
                             ldy, flags, s);
}

void launch_lr_reduce(int32_t nitems, const ReduceItem *items, int64_t tstride, int64_t elems,
                      bool f32, void *T, hipStream_t s) {
  if (nitems <= 0 || elems <= 0) return;
  dim3 g((unsigned)std::min<int64_t>((elems + 255) / 256, 64), (unsigned)nitems);
  if (f32)
    lr_reduce_kernel<float><<<g, 256, 0, s>>>(items, tstride, elems, (float *)T);
  else
    lr_reduce_kernel<double><<<g, 256, 0, s>>>(items, tstride, elems, (double *)T);
}

void launch_near_apply(int32_t nchunks, const ExpandChunk *chunks, const NearEntry *entries,
                       bool f32, const void *D, const void *X, int64_t ldx, int64_t ncols,
                       void *Y, int64_t ldy, bool overwrite, hipStream_t s) {
  if (nchunks <= 0 || ncols <= 0) return;
  if (f32)
    near_ntw<float, kNTW>(nchunks, chunks, entries, D, X, ldx, ncols, Y, ldy, overwrite, s);
  else
    near_ntw<double, kNTW>(nchunks, chunks, entries, D, X, ldx, ncols, Y, ldy, overwrite, s);
}

void launch_dense_gemm(int64_t n, const double *A, int64_t lda, bool trans, int64_t ncols,
                       const double *X, int64_t ldx, double *Y, int64_t ldy, hipStream_t s) {
  if (n <= 0 || ncols <= 0) return;
  dim3 g((unsigned)((n + 63) / 64), col_tiles(ncols));
  dense_gemm_kernel<<<g, 256, 0, s>>>(n, A, lda, trans ? 1 : 0, ncols, X, ldx, Y, ldy);
}

}  // namespace hm
