// Launchers of the libhm HIP kernels (host-callable, enqueue on `s`).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hm {

// ---- test matrices and data movement (k_misc.hip)
// Colored Gaussian test matrix of one level/pass: out (n x ncolors*r, ld)
// in tree order; row i of color block c is nonzero iff active[rowbox[i]*ncol + c].
// Forest (ninst > 1): row i of instance q (inst_off[q] <= i < inst_off[q+1],
// device array) draws with key seed + q and row number i - inst_off[q].
void launch_testmat(int64_t n, const int32_t *rowbox, const uint8_t *active, int32_t ncolors,
                    int32_t r, int32_t level, int32_t pass, uint64_t seed,
                    const int64_t *inst_off, int32_t ninst, bool f32, void *out, int64_t ld,
                    int64_t ncols_pad, hipStream_t s);
// Identity blocks of the leaf pass: out zeroed (n x ncols_pad), then
// out[start[b] + t, color*m + t] = 1 for each (b, color) item, t < size(b).
void launch_leaf_identity(int64_t n, int32_t nitems, const int32_t *item_box,
                          const int32_t *item_color, const int64_t *box_start, int32_t m,
                          bool f32, void *out, int64_t ld, int64_t ncols_pad, hipStream_t s);
void launch_fill(void *p, int64_t count, bool f32, double value, hipStream_t s);
// zeros in an n x ncols column-major block (leading dimension ld), one launch
void launch_fill_cols(void *p, int64_t n, int64_t ncols, int64_t ld, bool f32, hipStream_t s);
// Row permutation of a column-major block: dst[i, :] = src[idx[i], :] (gather)
// or dst[idx[i], :] = src[i, :] (scatter).
void launch_permute_rows(int64_t n, int64_t ncols, const int64_t *idx, bool scatter, bool f32,
                         const void *src, int64_t lds, void *dst, int64_t ldd, hipStream_t s);
// dtype conversion of a column-major block (FP64 <-> FP32).
void launch_convert(int64_t n, int64_t ncols, bool src_f32, const void *src, int64_t lds,
                    void *dst, int64_t ldd, hipStream_t s);
void launch_philox_raw(const uint32_t *ctr, int64_t count, uint32_t k0, uint32_t k1,
                       uint32_t *out, hipStream_t s);
// Leaf neighbor blocks: D_p = Y[a0:a0+ma, col0 : col0+mb] for each pair p.
void launch_extract_near(int32_t np, const int64_t *row0, const int32_t *ma, const int64_t *col0,
                         const int32_t *mb, const int64_t *dst_off, bool f32, const void *Y,
                         int64_t ldy, double *D, hipStream_t s);
// Sets *flag = 1 when the block holds a NaN or Inf (plain store, no atomics).
void launch_check_finite(int64_t n, int64_t ncols, bool f32, const void *Y, int64_t ldy,
                         int32_t *flag, hipStream_t s);

// ---- black-box applies (k_kapply.hip, k_lowrank.hip)
// Y = K X with K(i,j) = kernel(p_i, p_j) generated on the fly (points SoA,
// tree order), 0 where p_i == p_j.  kernel: 0 = log, 1 = 1/r.
// nt: column fragments (16 columns each) per workgroup, even, 2..16; 0 =
// kapply_default_nt.  Every nt computes the same values bit for bit.
// rows > 0: compute only Y rows [row0, row0 + rows) (row0 a multiple of
// 64): a slice of a launch, or a partial launch for timing (row0 = 0).
void launch_kapply(int kernel, int dim, int64_t n, const double *pts, int64_t ncols, int nt,
                   bool f32, const void *X, int64_t ldx, void *Y, int64_t ldy, hipStream_t s,
                   int64_t rows = 0, int64_t row0 = 0);
// Block-diagonal form for a forest: one work item per 64-row block of one
// instance.  Rows [base, base + nloc) of Y are K_inst X(base : base+nloc, :)
// where K_inst only couples points of the instance.  Columns outside
// [0, width) and [split, split + width) (split < 0: no second range) are
// known to be zero in the instance's rows of X: their tiles are not
// computed, and Y there is written 0.  Items are launched in the given
// order (put the long instances first).  nt: column fragments per
// workgroup (0 = chosen from ncols).
struct KItem {
  int64_t base;   // first row of the instance
  int32_t nloc;   // rows of the instance
  int32_t rblk;   // first row of the block, relative to base
  int32_t width;  // live columns of the instance
  int32_t pad;
};
void launch_kapply_forest(int kernel, int dim, int64_t n, const double *pts, int32_t nitems,
                          const KItem *items, int64_t ncols, int64_t split, int nt, bool f32,
                          const void *X, int64_t ldx, void *Y, int64_t ldy, hipStream_t s);
// Column fragments per workgroup chosen without timing, for ncols columns
// over `units` row blocks (or forest items).
int kapply_default_nt(int64_t ncols, bool f32, int64_t units);
// Dense Y = op(A) X, FP64.
void launch_dense_gemm(int64_t n, const double *A, int64_t lda, bool trans, int64_t ncols,
                       const double *X, int64_t ldx, double *Y, int64_t ldy, hipStream_t s);

// ---- low-rank products (k_lowrank.hip)
// Project: for one row segment of one column box and a group of pairs that
// share that column box, T_{p,s}[0:k_p, :] = R_p(segment rows)^T X(segment rows, :).
// The group holds at most 64 / kmax pairs; ranks are read from ranks[kidx];
// the partial T_{p,s} lives at T + tslot * tstride (kmax x ncols, ld = kmax).
struct ProjItem {
  int64_t row0;     // first X row of the segment
  int32_t nrows;    // rows in the segment
  int32_t seg_off;  // row offset of the segment inside the box
  int32_t m;        // rows of the box (leading dimension of R_p)
  int32_t npairs;   // pairs in the group
  int32_t first;    // first entry in the ProjPair list
  int32_t pad;
};
struct ProjPair {
  int64_t rslot;    // element offset of R_p (m x kmax, ld = m)
  int32_t kidx;     // index of the rank
  int32_t tslot;    // partial slot of this pair and segment
};
// Expand: Y[row0 : row0+nrows, :] += sign * sum_q L_q[off_q : off_q+nrows, 0:k_q] T_q
// with T_q = the sum of its nseg partial slots starting at tslot, held in
// the first of them when the expansion runs.
struct ExpandChunk {
  int64_t row0;
  int32_t nrows;
  int32_t first, last;  // range in the entry list
  int32_t pad;
};
struct ExpandEntry {
  int64_t lslot;   // element offset of L_q (ld = mq)
  int32_t mq;      // leading dimension of L_q (rows of its box)
  int32_t off;     // row offset of the chunk inside L_q
  int32_t kidx;
  int32_t tslot;   // first partial slot
  int32_t nseg;    // number of partial slots
  int32_t pad;
};
// Zero pattern of a colored test matrix X (the peel's right-hand side):
// column block c (columns [c colw, (c + 1) colw)) is zero on the rows of
// box b of the sampled level unless act[b * ncolors + c] != 0.  rowbox:
// that level's box of every row; bstart: its box row starts (nbox + 1);
// col0: the column of X where a launch's first column sits.
struct ColorPattern {
  const int32_t *rowbox;
  const int64_t *bstart;
  const uint8_t *act;
  int32_t ncolors, colw;
  int64_t col0;
};
// Column tile of the low-rank products (columns per workgroup).
constexpr int kLowRankTile = 64;
// With a pattern, the projection skips the rows of boxes whose blocks are
// zero in all colors of a column tile, and records per slot and tile
// whether T was written (flags[tslot * ntiles + tile], ntiles =
// ceil(ncols / kLowRankTile)); a tile with no live rows leaves T unwritten
// and flag 0.  The expansion given the flags skips the entries whose tile
// is flagged 0.  pat == nullptr: dense X, no flags.
void launch_lr_project(int32_t nitems, const ProjItem *items, const ProjPair *pairs, int32_t kmax,
                       int64_t tstride, const int32_t *ranks, bool f32, const void *R,
                       const void *X, int64_t ldx, int64_t ncols, void *T,
                       const ColorPattern *pat, uint8_t *flags, hipStream_t s);
// Every entry's partials must already be summed into its first slot
// (launch_lr_reduce): only that slot is read.
void launch_lr_expand(int32_t nchunks, const ExpandChunk *chunks, const ExpandEntry *entries,
                      int32_t kmax, int64_t tstride, const int32_t *ranks, bool f32,
                      const void *L, const void *T, int64_t ncols, double sign, void *Y,
                      int64_t ldy, const uint8_t *flags, hipStream_t s);
// T[slot] += T[slot + 1] + ... + T[slot + nseg - 1] (elems values per slot,
// slot s at T + s * tstride), one item per pair split over several segments.
struct ReduceItem {
  int32_t slot, nseg;
};
void launch_lr_reduce(int32_t nitems, const ReduceItem *items, int64_t tstride, int64_t elems,
                      bool f32, void *T, hipStream_t s);
// Near field: Y[rows] += sum D_q(off: off+nrows, 0:mb) X[b0 : b0+mb, :]
struct NearEntry {
  int64_t dslot;   // element offset of D_q (ld = ma)
  int64_t xrow0;   // first row of the column box in X
  int32_t ma;      // leading dimension
  int32_t mb;      // columns of the operator block (at most 128)
  int32_t off;     // row offset of the chunk inside the operator block
  int32_t trans;   // 1: the operator block is D_q^T (the adjoint's near field);
                   // element (i, k) = D_q[(off + i) * ma + k]
};
// overwrite: Y's chunk rows are set rather than accumulated.
void launch_near_apply(int32_t nchunks, const ExpandChunk *chunks, const NearEntry *entries,
                       bool f32, const void *D, const void *X, int64_t ldx, int64_t ncols,
                       void *Y, int64_t ldy, bool overwrite, hipStream_t s);

// ---- per-pair recovery (k_qr.hip)
struct QrJob {
  int64_t row0;    // first row of the block in the sample matrix
  int64_t col0;    // first column (color block)
  int64_t uslot;   // element offset of the output basis (m x kmax, ld = m)
  int64_t wslot;   // element offset of the FP64 workspace (m x r, ld = m)
  int32_t m;       // rows
  int32_t pad;
};
// Column-pivoted Householder QR of S (m x r) in place, truncated by rank /
// tolerance, and the explicit basis Q[:, 0:k] written to U.  ranks[j] = k,
// sat[j] = 1 when the tolerance was not met within `cap` columns.
// floor_abs (device, njobs, or NULL): tolerance mode stops at the first
// |R_jj| <= max(tol |R_00|, floor_abs[job]).
void launch_pivqr(int32_t njobs, const QrJob *jobs, int32_t r, int32_t rank_fixed, double tol,
                  int32_t cap, const double *floor_abs, bool f32, const void *S, int64_t lds,
                  double *Wk, double *U, int32_t *ranks, int32_t *sat, hipStream_t s);
// out[j] = scale * Frobenius norm of job j's block S(row0 : row0+m, col0 : col0+r).
void launch_block_norms(int32_t njobs, const QrJob *jobs, int32_t r, double scale, bool f32,
                        const void *S, int64_t lds, double *out, hipStream_t s);
// C_p = G2^T S_U (r x r) for every pair, into core (np x r x r).
struct CoreJob {
  int64_t arow0;   // rows of alpha in Psi / Y
  int64_t brow0;   // rows of beta in Omega / Z
  int64_t ucol0;   // Omega / Y color block of the pair
  int64_t vcol0;   // Psi / Z color block of the pair
  int64_t uslot, vslot, wslot, bslot, cslot;
  int32_t ma, mb;
  int32_t pu, pv;  // index of the pair's U / V rank
};
// The recovery of a whole level in one persistent launch (core, the two
// pivoted QRs and the coupling of every pair, pairs pulled through
// *counter in `order`, largest blocks first): C_p = G2^T S_U (r x r) into
// core, U and V by launch_pivqr's rule, B = (G2^T U)^+ C (V^T G1)^+ and
// W = U B.  *counter must be 0 at the launch.
struct RecoverArgs {
  const CoreJob *jc;
  const QrJob *ju, *jv;
  const int32_t *order;
  int32_t *counter;
  int32_t njobs, r, kmax, rank_fixed, cap;
  double tol;
  int64_t ld;                   // leading dimension of Omega, Psi, Y (= n)
  const double *floor_u, *floor_v;
  double *work, *U, *V, *core, *scratch, *B, *W;
  int32_t *ranks;               // all ranks (coupling: ranks[pu], ranks[pv])
  int32_t *ranks_u, *ranks_v, *sat_u, *sat_v;  // this level's, indexed by pair
  int32_t qr_rows;              // set by launch_recover: rows of a QR block held in LDS
};
void launch_recover(const RecoverArgs &a, int grid, bool f32, const void *Omega, const void *Psi,
                    const void *Y, hipStream_t s);

// ---- uniform H^1 (k_uniform.hip, k_qr.hip)
// Stage-2 test matrix assembled from the stage-1 column bases: out (n x
// ncols_pad, ld) with out[i, c*kmax + j] = U_u(i - start[b], j) for the row's
// box b at this level when u = slot[b*ncolors + c] - 1 >= 0 and j < urank[u]
// (U_u at UB + uoff[u], m_b x kmax, ld = m_b), else 0.
void launch_basis_testmat(int64_t n, const int32_t *rowbox, const int64_t *box_start,
                          const int32_t *slot, int32_t ncolors, int32_t kmax, const double *UB,
                          const int64_t *uoff, const int32_t *urank, bool f32, void *out,
                          int64_t ld, int64_t ncols_pad, hipStream_t s);
// One chunk (<= 256 rows) of box b's combination S_b = sum_t Z(rows, term t
// block) Gamma_t over the terms [t0, t1).
struct MixJob {
  int64_t row0;
  int32_t m;
  int32_t t0, t1;
  int32_t pad;
};
// Gamma_t (kmax x kmax): entry (i, j) is the Gaussian of counter (grow, j/2, i,
// 4*level + 3) under key seed + inst (the test-matrix generator).
struct MixTerm {
  int64_t zcol0;   // first column of the term's block in Z
  uint32_t grow;   // first tree row (instance-local) of the other box
  uint32_t inst;   // instance of the pair
};
void launch_mix_sum(int32_t njobs, const MixJob *jobs, const MixTerm *terms, int32_t kmax,
                    int32_t level, uint64_t seed, bool gamma, bool f32, const void *Z,
                    int64_t ldz, double *S, int64_t lds, hipStream_t s);
// Per admissible pair (a, b) of a uniform level: B = Z(I_b, block of (b, a))[:, :k_a]^T V_b,
// W = U_a B, and the per-pair copies of U_a and V_b with their ranks.
struct UCJob {
  int64_t zrow0, zcol0;        // rows of b, block of the pair (b, a) in Z
  int64_t uboff, vboff;        // U_a in UB (ma x kmax), V_b in VB (mb x kmax)
  int64_t uslot, vslot, wslot, bslot;
  int32_t ma, mb;
  int32_t ua, vb;              // basis indexes into urank / vrank
  int32_t pu, pv;              // rank slots of the pair
};
// recompute = false: keep the stored B (bases replaced by nested ones:
// copies and W = U_a B only).
void launch_ucoupling(int32_t njobs, const UCJob *jobs, int32_t kmax, bool f32, const void *Z,
                      int64_t ldz, const double *UB, const double *VB, const int32_t *urank,
                      const int32_t *vrank, double *U, double *V, double *B, double *W,
                      int32_t *ranks, bool recompute, hipStream_t s);

// ---- H^2 (k_qr.hip, k_uniform.hip)
// Left singular vectors of each job's sample S(row0 : row0+m, col0 : col0+c)
// (FP64, c <= 64) into U + uslot (m x k, ld m), k by the fixed rank or by
// max(tol sigma_0, floor_abs[job]) capped at cap (sat[job] = 1 when more
// values exceed it); the job's singular values into sigma + job * kmax.
// Workspace Wk + wslot: m x c.
void launch_svd_basis(int32_t njobs, const QrJob *jobs, int32_t c, int32_t rank_fixed, double tol,
                      int32_t cap, const double *floor_abs, const double *S, int64_t lds,
                      double *Wk, double *U, double *sigma, int32_t kmax, int32_t *ranks,
                      int32_t *sat, hipStream_t s);
struct TransferJob {
  int64_t child_off;   // U_a in UB (mc x k_a, ld mc)
  int64_t par_off;     // first row of a inside U_tau in UB (ld ldp)
  int64_t out_off;     // transfer slot (kmax x kmax, ld kmax)
  int32_t mc, ldp;
  int32_t cidx, pidx;  // rank indexes of a and tau
};
void launch_transfer(int32_t njobs, const TransferJob *jobs, int32_t kmax, const double *UB,
                     const int32_t *rank, double *out, hipStream_t s);
// Augmented samples, one job per chunk (<= 256 rows) of a box:
// dst(rows, 0:ncols) = src(rows, src_col0 : src_col0+ncols) (or 0 when
// src_col0 < 0) + P(rows, 0:kp) diag(sigma_p) G, P = the parent basis rows
// at UBp + par_off (ld par_ld; none when par_off < 0), kp = prank[par_idx],
// G (kp x ncols) from counter (grow, j/2, 2^31 + i, 4*level + pass) under key
// seed + inst.
struct AugJob {
  int64_t row0;
  int64_t src_col0;
  int64_t par_off;
  int32_t m, par_ld, par_idx;
  uint32_t grow, inst;
  int32_t pad;
};
void launch_h2_sample(int32_t njobs, const AugJob *jobs, int32_t ncols, int32_t level,
                      int32_t pass, uint64_t seed, bool src_f32, const void *src, int64_t lds,
                      const double *UBp, const int32_t *prank, const double *psigma,
                      int32_t kmax, double *dst, int64_t ldd, hipStream_t s);
// Nested bases: out rows (a chunk of child a inside tau) = U_a(chunk) Tr_a,
// Tr_a the transfer (k_a x k_tau, ld kmax).
struct NestJob {
  int64_t out_off;     // first output row in UB (ld ldo)
  int64_t in_off;      // first input row of U_a in UB (ld ldi)
  int64_t t_off;       // transfer slot
  int32_t m, ldo, ldi;
  int32_t cidx, pidx;  // rank indexes of a and tau
  int32_t pad;
};
void launch_nest(int32_t njobs, const NestJob *jobs, int32_t kmax, const double *UBin,
                 const double *Tr, const int32_t *rank, double *UBout, hipStream_t s);

// ---- H^2 apply (k_h2apply.hip).  Expansions QH / UH: FP64, kmax x ncols per
// basis box g at + g * kmax * ldq (ld kmax).
// A box holding long bases (or a 64-row chunk of it, for the expansion).
struct H2Leaf {
  int64_t row0;   // first row of the box
  int64_t boff;   // its basis in UB / VB (m x kmax, ld m)
  int32_t m;      // rows of the box
  int32_t g;      // global basis index (ranks, expansions)
  int32_t r0;     // first row of the chunk inside the box
  int32_t c0;     // box records: index of the box's first chunk record
};
// Outgoing expansions in two steps: every 64-row chunk (chunk list) its
// partial V* x into PART (chunk-indexed, kmax x ncols, ld kmax), then every
// box (leaf list; c0 = its first chunk) the sum of its chunks' partials in
// order into QH.
void launch_h2_project(int32_t nchunks, const H2Leaf *chunks, int32_t kmax, const int32_t *rank,
                       const double *VB, bool f32, const void *X, int64_t ldx, int64_t ncols,
                       double *PART, int64_t ldq, hipStream_t s);
void launch_h2_reduce(int32_t nleaf, const H2Leaf *leaf, int32_t kmax, const double *PART,
                      double *QH, int64_t ldq, int64_t ncols, hipStream_t s);
// OUT[g] = sum over the job's terms of M (x IN[src], or x PAR[src] for a parent term).
struct H2Sum {
  int32_t g, t0, t1, pad;
};
struct H2Term {
  int64_t moff;    // matrix in Mpool (or Mpar for a parent term), kmax x kmax
  int32_t src;     // global basis index of the input expansion
  int16_t parent;  // 1: Mpar and PAR, ranks from rank_o
  int16_t trans;   // 1: the matrix is applied transposed
};
void launch_h2_sum(int32_t njobs, const H2Sum *jobs, const H2Term *terms, int32_t kmax,
                   const int32_t *rank_o, const int32_t *rank_i, const double *Mpool,
                   const double *Mpar, const double *IN, const double *PAR, double *OUT,
                   int64_t ldq, int64_t ncols, hipStream_t s);
// Y(rows of the chunk) += U_g UH[g], one job per 64-row chunk of a box with long bases.
void launch_h2_expand(int32_t njobs, const H2Leaf *jobs, int32_t kmax, const int32_t *rank,
                      const double *UB, const double *UH, int64_t ldq, bool f32, int64_t ncols,
                      void *Y, int64_t ldy, double sign, hipStream_t s);

// Sustained TFLOP/s of the 16x16x4 matrix-core instruction of the kernel
// apply (FP32 or FP64), independent chains, no memory traffic; cus = the
// device's compute units.
double measure_mfma_rate(bool f32, int cus, hipStream_t s);

}  // namespace hm
