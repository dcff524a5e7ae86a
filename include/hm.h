/*
 * hm.h -- C ABI of the MI355X colored-peeling library (libhm.so).
 *
 * The library builds an H^1 representation of an N x N operator A that is
 * reachable only through products with A and A* (Levitt & Martinsson,
 * "Randomized compression of rank-structured matrices accelerated with graph
 * coloring", arXiv 2205.03406, introduction: the user can evaluate
 * Y = A Omega and Z = A* Psi; the partition comes from the geometry).
 *
 * Conventions for every entry point:
 *   - Return value: HM_OK (0) or a negative hm_status.  Nothing aborts; on
 *     error no handle is created and outputs are left untouched.  The
 *     thread-local message of the last error is hm_last_error().
 *   - Host pointers are marked "host", device pointers "device".  Device
 *     buffers are ordinary HIP device allocations on the current device.
 *   - Dense matrices are column-major with an explicit leading dimension.
 *   - "Tree order" is the point order after the tree's permutation
 *     (hm_tree_perm maps tree position -> original index); "original order"
 *     is the caller's order.
 *   - Streams are hipStream_t passed as void* (NULL = the default stream).
 *     Work is enqueued on that stream; a call returns after enqueueing
 *     unless stated otherwise.
 *   - Handles are not thread-safe; distinct handles may be used from
 *     distinct threads.
 */
#ifndef HM_H
#define HM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int hm_status;
#define HM_OK 0
#define HM_E_ARG (-1)       /* invalid argument (null pointer, bad size or enum) */
#define HM_E_NOMEM (-2)     /* host or device allocation failed */
#define HM_E_DEVICE (-3)    /* a HIP call failed */
#define HM_E_CALLBACK (-4)  /* the user black box returned nonzero */
#define HM_E_NUMERIC (-5)   /* NaN or Inf in the samples */
#define HM_E_STATE (-6)     /* handle not ready (e.g. tree not colored) */
#define HM_E_SATURATED (-7) /* tolerance not reached within r - p columns */

enum { HM_TREE_GEOMETRIC = 0, HM_TREE_INDEX_BINARY = 1 };
enum { HM_ADM_STRONG = 0, HM_ADM_WEAK = 1 };
enum { HM_F64 = 0, HM_F32 = 1 };
enum { HM_PREC_F64 = 0, HM_PREC_MIXED = 1 };
enum { HM_KERNEL_LOG = 0, HM_KERNEL_INV_R = 1 };
enum { HM_ORDER_ORIGINAL = 0, HM_ORDER_TREE = 1 };
enum { HM_LIST_NEIGHBOR = 0, HM_LIST_INTERACTION = 1 };

typedef struct hm_tree hm_tree;
typedef struct hm_hmatrix hm_hmatrix;

const char *hm_last_error(void);

/* ------------------------------------------------------------------ tree
 * hm_build_tree: the box tree of the section "Rank-structured matrices"
 * (every box bisected along each dimension, empty children omitted, boxes
 * with more than leaf_size points split; fig:tree for the index-halving
 * variant), its neighbor lists (same-level boxes whose closed cubes touch,
 * the box itself included) and interaction lists (children of the parent's
 * neighbors that are not neighbors), and the constraint incompatibility
 * graphs of every level (def:incompatibility_graph, eq:h1constraints) and of
 * the leaf level (section on extracting inadmissible blocks).
 *
 *   points     host, n x dim row-major FP64, copied (1 <= dim <= 8; the
 *              kernel black box and kernel apply take dim <= 3)
 *   leaf_size  m >= 1
 *   tree_kind  HM_TREE_GEOMETRIC: root = bounding cube of the points, integer
 *              cell c = min(2^b-1, floor(((x-lo)/s) 2^b)) with b = 21 bits for
 *              dim <= 3 and floor(63/dim) above (at most b levels), tree order =
 *              stable sort by the interleaved cell bits (x lowest); a box that
 *              stops splitting is carried unchanged to finer levels.
 *              HM_TREE_INDEX_BINARY: points stably sorted by x, ranges halved
 *              at lo + (hi-lo)/2 while longer than leaf_size (requires
 *              HM_ADM_WEAK).
 *   adm        HM_ADM_STRONG: interaction lists as above.  HM_ADM_WEAK
 *              (HODLR): neighbors = {box}, interaction list = the other
 *              children of the parent.
 *   out        receives the handle; free with hm_tree_free.
 */
hm_status hm_build_tree(const double *points, int64_t n, int dim, int leaf_size, int tree_kind,
                        int adm, hm_tree **out);
void hm_tree_free(hm_tree *tree);

/* hm_build_forest: `ninst` independent problems compressed together (the
 * batched form).  Instance i owns the counts[i] consecutive points of
 * `points` (host, row-major, sum(counts) x dim, copied) and gets its own tree,
 * lists and graphs exactly as hm_build_tree builds them.  The forest merges
 * them level by level: rows of instance i are [off_i, off_i + counts[i]) in
 * both the original and the tree order (off_i = counts[0] + ... +
 * counts[i-1]), its boxes precede those of instance i+1 at every level, a
 * tree shallower than the deepest one carries its leaves down unchanged,
 * and every graph is the disjoint union of the instances' graphs (vertex
 * ids instance-major).  No list or graph edge joins two instances, so a
 * compression of the forest is the compression of the block-diagonal
 * operator diag(A_0, ..., A_{ninst-1}); the built-in kernel black box
 * evaluates exactly that, and a user black box must too.  Instance i draws
 * its test matrices with seed opts->seed + i and its own row numbering, so
 * its factors are those of a compression of instance i alone (same tree,
 * colors, seed) up to floating-point summation order.
 *   counts  host, ninst entries, each >= 1;  ninst >= 1.
 * Other arguments as hm_build_tree; all instances share them. */
hm_status hm_build_forest(const double *points, const int64_t *counts, int32_t ninst, int dim,
                          int leaf_size, int tree_kind, int adm, hm_tree **out);
/* ninst (always written) and offsets (host, ninst+1, or NULL): row ranges of
 * the instances; a tree from hm_build_tree is a forest of one instance. */
hm_status hm_tree_instances(const hm_tree *tree, int32_t *ninst, int64_t *offsets);

/* levels are 0..nlevels-1; nlevels-1 is the leaf level L */
hm_status hm_tree_info(const hm_tree *tree, int32_t *nlevels, int64_t *n, int32_t *dim);
/* perm: host, n entries: perm[i] = original index of tree position i */
hm_status hm_tree_perm(const hm_tree *tree, int64_t *perm);
/* box ranges of one level: start (host, nbox+1; box b holds tree positions
 * [start[b], start[b+1])), parent (host, nbox; box id at level-1, -1 at
 * level 0), org (host, max(3, dim)*nbox; integer cube origin in 2^-b root
 * units, b as for hm_build_tree),
 * blev (host, nbox; level whose cube size the box has).  Any output may be
 * NULL; nbox is always written. */
hm_status hm_tree_level(const hm_tree *tree, int level, int32_t *nbox, int64_t *start,
                        int32_t *parent, int64_t *org, int32_t *blev);
/* CSR list of one level (which = HM_LIST_*): nnz always written; ptr (host,
 * nbox+1) and idx (host, nnz) written when non-NULL; lists ascending. */
hm_status hm_tree_list(const hm_tree *tree, int level, int which, int64_t *nnz, int32_t *ptr,
                       int32_t *idx);

/* ------------------------------------------------------------------ graphs
 * hm_incompat_graph: the constraint incompatibility graph of `level`
 * (level = -1: the leaf graph).  Vertices are distinct constraint sets
 * (active box beta, box set S) where the test matrix must equal a Gaussian
 * block on beta and vanish on S minus {beta}; for an admissible pair (a, b)
 * of the level, beta = b and S = children of the neighbors of a's parent
 * (= neighbors of a plus its interaction list); for a leaf pair, beta = b and
 * S = neighbors of a.  Two vertices are adjacent when the active box of one
 * lies in the zero set of the other.  Vertex order: parents ascending, then
 * active boxes ascending (leaf: row boxes ascending, then neighbors).
 *
 * Outputs point into memory owned by the tree (valid until hm_tree_free):
 *   xadj (nv+1), adj (nadj) CSR adjacency, ascending;  vbox (nv) active box;
 *   pair_a, pair_b (npairs) the pairs of the level (a ascending, then b
 *   ascending), pair_v (npairs) the vertex of each pair.
 */
hm_status hm_incompat_graph(const hm_tree *tree, int level, int64_t *nv, int64_t *nadj,
                            const int64_t **xadj, const int32_t **adj, const int32_t **vbox,
                            int64_t *npairs, const int32_t **pair_a, const int32_t **pair_b,
                            const int32_t **pair_v);

/* hm_uniform_graph: the stage-1 constraint incompatibility graph of uniform
 * H^1 compression at `level` (section on uniform H^1 compression,
 * eq:unifh1constraints), built and DSatur-colored on first use.  One vertex
 * per box a with a non-empty interaction list (boxes ascending): the test
 * matrix must be a Gaussian block on every box of a's interaction list and
 * vanish on a's neighbors; a and b are adjacent when a box active for one is
 * a neighbor of the other.  Outputs point into memory owned by the tree:
 * xadj (nv+1), adj (nadj, ascending), vbox (nv), color (nv). */
hm_status hm_uniform_graph(hm_tree *tree, int level, int64_t *nv, int64_t *nadj,
                           const int64_t **xadj, const int32_t **adj, const int32_t **vbox,
                           int32_t *ncolors, const int32_t **color);

/* hm_color: DSatur greedy coloring (alg:dsatur) of a CSR graph.  The next
 * vertex is the uncolored one with the largest saturation (number of
 * distinct colors among its neighbors), ties by larger degree, then lower
 * id; it gets the smallest color not used by a neighbor.
 *   xadj (host, nv+1), adj (host, xadj[nv]) symmetric adjacency
 *   color (host, nv) output; ncolors output. */
hm_status hm_color(int64_t nv, const int64_t *xadj, const int32_t *adj, int32_t *color,
                   int32_t *ncolors);
/* Colors every graph of the tree with hm_color and stores the result (in a
 * forest: each instance's component on its own, which gives the colors
 * hm_color gives on the whole graph; a level's color count is the largest
 * over the instances). */
hm_status hm_tree_color(hm_tree *tree);
/* Installs a caller-chosen coloring of one graph (checked for validity). */
hm_status hm_tree_set_colors(hm_tree *tree, int level, const int32_t *color);
/* The stored coloring (owned by the tree). */
hm_status hm_tree_colors(const hm_tree *tree, int level, int32_t *ncolors, const int32_t **color);

/* Decisions of the kernel-apply autotuner so far, one line per launch shape
 * (precision, kernel, dimension, columns, log2 of the point count, forest
 * form -> column-tile width, best and default times).  The first launch of
 * a shape times every tile width on the real operands (each computes the
 * same values bit for bit) and keeps the fastest; HM_AUTOTUNE=0 disables
 * tuning, HM_TUNE_FILE names a file that keeps decisions across processes.
 * The string is owned by the calling thread and valid until its next call. */
const char *hm_autotune_table(void);

/* ------------------------------------------------------------------ black box
 * The black box computes Y = A X (transpose = 0) or Y = A* X (transpose = 1)
 * for a device block X of ncols columns, enqueued on `stream`.
 *   dtype  HM_F64 or HM_F32 (X and Y element type)
 *   order  the point order of the rows of X and Y the box expects
 * It must not keep X or Y after returning; nonzero return = failure. */
typedef int (*hm_apply_fn)(void *ctx, int transpose, int64_t n, int64_t ncols, int dtype,
                           const void *X, int64_t ldx, void *Y, int64_t ldy, void *stream);

typedef struct {
  hm_apply_fn apply;
  void *ctx;
  int32_t order;     /* HM_ORDER_ORIGINAL or HM_ORDER_TREE */
  int32_t symmetric; /* nonzero when A* = A: one call may serve both passes */
  int32_t dtypes;    /* bit (1 << HM_F64) | (1 << HM_F32) of supported types */
} hm_blackbox;

/* Built-in black box: A(i,j) = K(x_i, x_j) generated on the fly from the
 * tree's points, K = log|x-y| (HM_KERNEL_LOG) or 1/|x-y| (HM_KERNEL_INV_R),
 * A(i,j) = 0 when x_i = x_j (the diagonal included).  Stands in for the fast
 * black boxes of the experiments section.  Tree order, symmetric, FP64 and
 * FP32 (FP32: kernel evaluated and accumulated on MFMA in FP32 from FP64
 * point differences).  The ctx is owned by the tree. */
hm_status hm_kernel_blackbox(hm_tree *tree, int kernel, hm_blackbox *out);
/* Direct call of the built-in kernel apply: Y = K X (rows in `order`). */
hm_status hm_kernel_apply(hm_tree *tree, int kernel, int64_t ncols, int dtype, const void *X,
                          int64_t ldx, void *Y, int64_t ldy, int order, void *stream);

/* Dense black box for tests and small operators: A is a device FP64 n x n
 * column-major matrix (lda >= n) in `order`, not copied (must outlive every
 * compression that uses it).  Y = A X or A* X by a tiled FP64 GEMM. */
hm_status hm_dense_blackbox(const double *A, int64_t n, int64_t lda, int order, hm_blackbox *out);
void hm_dense_blackbox_free(hm_blackbox *bb);

/* Black boxes built from compressed operators, for compressing products and
 * compositions whose factors have fast applies (the operator-multiplication
 * experiment of the experiments section; any black box with a fast apply
 * fits the problem statement of the introduction).
 * hm_hmatrix_blackbox: Y = H X, and Y = H* X for the adjoint (hm_matvec_op).
 *   FP64 and FP32.  H is borrowed (must outlive every use).  order =
 *   HM_ORDER_TREE is valid only when the compression runs on the tree H was
 *   built on (rows in that tree's order); HM_ORDER_ORIGINAL always is.
 * hm_product_blackbox: Y = A (B X), adjoint Y = B* (A* X), through a
 *   stream-ordered n x ncols intermediate.  A and B are copied (their ctx
 *   objects must outlive the product); both must take the same order; the
 *   product supports the dtypes both support and is symmetric when A and B
 *   are the same symmetric box.
 * hm_blackbox_free releases the ctx of a dense, H-matrix or product black
 * box (not of its factors); it ignores the kernel black box, which belongs
 * to its tree. */
hm_status hm_hmatrix_blackbox(const hm_hmatrix *H, int order, hm_blackbox *out);
hm_status hm_product_blackbox(const hm_blackbox *A, const hm_blackbox *B, hm_blackbox *out);
void hm_blackbox_free(hm_blackbox *bb);

/* ------------------------------------------------------------------ device memory
 * hm_allocator: a caller's device allocator (for instance the PyTorch
 * caching allocator), so that the caller owns every device block the
 * library uses.  alloc returns a block of at least `bytes` bytes on the
 * current device for work ordered on `stream` (a hipStream_t; NULL = the
 * null stream), or NULL when it cannot (the call then fails with
 * HM_E_NOMEM); free takes back a block alloc returned, with the stream it
 * was used on.  The library frees a block only once the work that used it
 * is complete or ordered on that stream (stream-ordered scratch).  Both
 * functions may be called from any thread the library runs on (the
 * server's workers included). */
typedef struct {
  void *ctx;
  void *(*alloc)(void *ctx, size_t bytes, void *stream);
  void (*free)(void *ctx, void *p, void *stream);
} hm_allocator;

/* ------------------------------------------------------------------ compression
 * hm_compress: alg:h1_pseudocode.  For each sampled level (coarsest first):
 * draw the colored Gaussian test matrices Omega, Psi (one N x r block per
 * color; eq:neartestmatrices), apply the black box, subtract the levels
 * already compressed (the level-truncated matrix), and recover every
 * admissible pair (a, b): U = qr(Y(I_a, block), k), V = qr(Z(I_b, block), k)
 * and B = (G2* U)^+ (G2* Y(I_a, block)) (V* G1)^+ (alg:compress_double_random).
 * Then extract the leaf neighbor blocks with identity test matrices.
 *
 * qr(., k) is column-pivoted Householder QR truncated to k columns; in
 * tolerance mode k = first j with |R_jj| <= tol |R_00|, capped at r - p
 * (each cap hit is counted as saturation in hm_stats; opts->max_retries and
 * HM_FLAG_STRICT say what happens then).  In the mixed form the threshold
 * has a floor at the FP32 rounding level of the raw sample block:
 * max(tol |R_00|, 8 u32 ||block||_F / sqrt(r)).
 *
 * Test-matrix entries: Philox4x32-10 keyed by seed, counter (tree row,
 * column/2, color, 4*level + pass), two 53-bit uniforms, Box-Muller.  In a
 * forest (hm_build_forest) instance i uses key seed + i and its tree row
 * counted from the instance's first row.
 *
 *   tree   colored (hm_tree_color) tree
 *   bb     black box; its columns are padded to a multiple of 16
 *   opts   see hm_compress_opts
 *   out    the H-matrix (device resident), free with hm_hmatrix_free.
 * The call synchronizes `stream` before returning.
 * Errors (out is then left unwritten, and every device block the call took
 * is released, through opts->allocator when one is given; only a tree
 * device copy the call made stays with the tree):
 *   HM_E_ARG        a null pointer, an empty tree, neither rank nor tol, r > 64
 *                   or r - p < 1 in tolerance mode, an unknown format, a black
 *                   box without an apply of the precision it needs;
 *   HM_E_STATE      the tree is not colored;
 *   HM_E_CALLBACK   the black box returned nonzero (it is not called again);
 *   HM_E_NUMERIC    a block of black-box samples holds a NaN or an Inf;
 *   HM_E_SATURATED  HM_FLAG_STRICT and a block still at the cap r - p;
 *   HM_E_NOMEM, HM_E_DEVICE  an allocation or a HIP call failed.
 */
typedef struct {
  int32_t rank;       /* fixed rank k > 0, or 0 for tolerance mode */
  double tol;         /* relative per-block tolerance (rank == 0) */
  int32_t oversample; /* p (default 10 when 0) */
  int32_t r;          /* columns per test matrix (0: rank + oversample) */
  int32_t prec;       /* HM_PREC_F64, or HM_PREC_MIXED: black box and peel in FP32,
                         QR and coupling solves in FP64 */
  int32_t flags;      /* HM_FLAG_TIMING: record stage times (HIP events);
                         HM_FLAG_STRICT: fail with HM_E_SATURATED when a block
                         still reaches the cap r - p after the retries */
  uint64_t seed;
  int32_t max_retries; /* tolerance mode: recompress with r + 8 (at most 64) while
                          some block reaches the cap, at most this many times */
  int32_t format;      /* HM_FORMAT_H1, HM_FORMAT_UNIFORM_H1 or HM_FORMAT_H2 (below) */
  const hm_allocator *allocator; /* NULL: the library allocates (hipMalloc, a block
                          cache of idle H-matrix blocks, hipMallocAsync scratch).
                          Else every device block of the call goes through it: the
                          compression's scratch, the H-matrix (which keeps a copy
                          of the struct, frees its blocks through it in
                          hm_hmatrix_free and takes its applies' scratch from it),
                          and the tree's device copy when this call makes it (the
                          first call that needs it makes it: a compression, with
                          its allocator, or hm_kernel_blackbox, hm_kernel_apply,
                          hm_test_matrix with the library's own; hm_tree_free
                          frees it there).  ctx must stay valid until all of
                          those are freed. */
} hm_compress_opts;
#define HM_FLAG_TIMING 1
#define HM_FLAG_STRICT 2
/* HM_FLAG_MIX_GAMMA (uniform H^1 and H^2 only; an extension, not the
 * paper's rule): form the row-basis sample of box b as
 * sum_a Z(I_b, block of (b, a)) Gamma_a with Gamma_a a kmax x kmax Gaussian
 * (pass 3 of the generator, counter (first tree row of a, column/2, row of
 * Gamma, 4*level + 3)) instead of the plain sum of the blocks. */
#define HM_FLAG_MIX_GAMMA 4
/* format = HM_FORMAT_UNIFORM_H1: uniform H^1 compression (section on
 * uniform H^1 compression), one column basis U_a and one row basis V_b per
 * box, shared by all admissible pairs: A(I_a, I_b) ~ U_a B_ab V_b*.  Per
 * sampled level, coarsest first:
 *   stage 1: test matrices from the coloring of hm_uniform_graph (pass 2 of
 *     the generator): a Gaussian block on every box of a's interaction list,
 *     zero on a's neighbors; Y = (A - A^(l)) Omega; U_a = qr(Y(I_a, block), k)
 *     with the rules (cap r - p, saturation, mixed floor) of hm_compress.
 *   stage 2: Psi = the level's pair-graph test matrix with U_a (k_a of kmax
 *     columns) in place of the Gaussian block on box a; Z = (A - A^(l))* Psi;
 *     V_b = qr(sum over a in int(b) of Z(I_b, block of (b, a)), k)
 *     (alg:h2_pseudocode, "sum samples and orthonormalize"; HM_FLAG_MIX_GAMMA
 *     selects the Gaussian-weighted extension); rank at most kmax, no cap.
 *     Stage 2 runs in FP64 in both precisions (the sum adds column j of
 *     every term, and where terms cancel, FP32 rounding of the samples
 *     would decide the directions V_b keeps); the black box therefore needs
 *     an FP64 apply in the mixed form too (HM_E_ARG otherwise).
 *   B_ab = Z(I_b, block of (b, a))[:, :k_a]* V_b.
 * kmax = rank (fixed rank) or r - p.  The leaf pass is that of hm_compress.
 * The result applies, exports and serves like any H-matrix (the per-pair
 * factors hold copies of the shared bases); hm_stats.nfloats counts each
 * basis once. */
/* format = HM_FORMAT_H2: H^2 compression (section on H^2 compression,
 * alg:h2_pseudocode): the uniform stages with three changes.  Every box of
 * the sampled levels whose far field is not empty (an interaction list, or
 * a parent with a basis) gets bases, from the SVD of its sample augmented
 * with its parent's:  U_a = svd(Y(I_a, block) + U_tau(rows of a) S_tau G, k)
 * (G: k_tau x r Gaussian, counter (first tree row of a, column/2, 2^31 + row
 * of G, 4*level + 2)), and V_b likewise from the sum of the uniform form
 * (G: k_tau x kmax, 4*level + 3); singular vectors are signed so that
 * their largest entry is positive.  After each level, the previous level's
 * bases become transfers U_a* U_tau(rows of a) (eq:nested_basis), and every
 * coarser level's bases are rebuilt from the finest ones through the
 * transfers, so the level-truncated matrix peeled from the next samples
 * and the final operator are the nested ones.  The sampled levels must be
 * consecutive (HM_E_ARG otherwise).  hm_stats.nfloats counts the finest
 * level's bases, the transfers, the couplings and the leaf blocks; the
 * device copy keeps the implied bases of every level for the applies. */
#define HM_FORMAT_H1 0
#define HM_FORMAT_UNIFORM_H1 1
#define HM_FORMAT_H2 2

hm_status hm_compress(hm_tree *tree, const hm_blackbox *bb, const hm_compress_opts *opts,
                      void *stream, hm_hmatrix **out);
void hm_hmatrix_free(hm_hmatrix *H);

/* Device memory planning (host computation only, no device work).
 * hm_compress_footprint: the most device bytes one hm_compress of `tree`
 * with `opts` and a black box in tree order holds at once, from the sizes
 * the compression computes (factor pools at the largest rank, sample and
 * scratch buffers, plans and work lists, and the tree's device copy when
 * the tree has none on the current device yet; the H-matrix's own blocks,
 * which stay after the call, are part of it), the retries of
 * opts->max_retries not included.  The server reserves it before it starts
 * a compression.  A black
 * box in the original order takes two more N x (widest sample) buffers.
 * HM_E_ARG for null pointers, r outside 1..64 or an unknown format;
 * HM_E_STATE when the tree is not colored.
 * hm_matvec_footprint: the device bytes one hm_matvec / hm_matvec_op of
 * nrhs right-hand sides of dtype takes as scratch (X and Y are the
 * caller's).  HM_E_ARG for bad arguments. */
hm_status hm_compress_footprint(hm_tree *tree, const hm_compress_opts *opts, int64_t *bytes);
hm_status hm_matvec_footprint(const hm_hmatrix *H, int64_t nrhs, int dtype, int64_t *bytes);

/* Plans: compress the same tree with the same black box and options many
 * times (for instance a black box whose device data change between calls),
 * with the whole device pipeline captured once into a HIP graph.
 * hm_compress_plan runs one compression eagerly on `stream` (which also
 * settles the kernel-apply autotuner), then captures the same launches on a
 * stream of its own and instantiates the graph.  hm_plan_execute replays it
 * on `stream` (the black box is applied again, the test matrices are the
 * same draws) and reads the ranks back; the result replaces the plan's
 * H-matrix, which hm_plan_hmatrix borrows (valid until the next execution or
 * hm_plan_free).  The black box must only enqueue device work on the stream
 * it is given (the built-in kernel and dense black boxes do); retries
 * (max_retries) do not apply.  graph_nodes (or NULL) receives the node
 * count of the captured graph. */
typedef struct hm_plan hm_plan;
hm_status hm_compress_plan(hm_tree *tree, const hm_blackbox *bb, const hm_compress_opts *opts,
                           void *stream, hm_plan **out);
hm_status hm_plan_execute(hm_plan *plan, void *stream);
hm_status hm_plan_hmatrix(const hm_plan *plan, const hm_hmatrix **H, int64_t *graph_nodes);
void hm_plan_free(hm_plan *plan);

/* hm_matvec: Y = H X, the apply of the H^1 representation (section on
 * rank-structured matrices: Y = sum over levels and admissible pairs of
 * U B V* X(I_b) plus the leaf neighbor blocks A(I_a, I_b) X(I_b); an H^2
 * matrix applies through its nested form, alg:apply_h2_level_truncated:
 * outgoing expansions, upward pass through the transfers, couplings and
 * downward pass, expansion).  X, Y device, n x nrhs column-major (ldx, ldy
 * >= n), dtype HM_F64 or HM_F32, rows in `order`; the caller owns both.
 * Enqueued on stream; scratch stream-ordered (through the H-matrix's
 * allocator when it was made with one).  HM_E_ARG for bad arguments,
 * HM_E_NOMEM when scratch cannot be had. */
hm_status hm_matvec(const hm_hmatrix *H, int64_t nrhs, int dtype, const void *X, int64_t ldx,
                    void *Y, int64_t ldy, int order, void *stream);
/* hm_matvec_op: hm_matvec (trans = 0) or the adjoint Y = H* X (trans = 1:
 * every admissible block V B* U*, the leaf blocks transposed; for H^2 the
 * passes with the two basis families swapped and the couplings
 * transposed). */
hm_status hm_matvec_op(const hm_hmatrix *H, int trans, int64_t nrhs, int dtype, const void *X,
                       int64_t ldx, void *Y, int64_t ldy, int order, void *stream);

/* hm_matvec_static: hm_matvec_op without any device allocation, for callers
 * that cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Its scratch (the order-conversion
 * copies and the low-rank expansions) is a static device array of
 * HM_STATIC_SCRATCH_BYTES, one per device, held from the library's load
 * until the process ends; the right-hand sides go through in blocks of as
 * many columns as fit.  Results equal hm_matvec_op's (every column is
 * computed the same way).  Arguments, layout and ownership as hm_matvec_op.
 * Errors: HM_E_ARG for bad arguments or when one right-hand side needs more
 * scratch than the array holds (the message gives the bytes needed: about
 * 2 n + (pair segments) kmax elements in the original order); HM_E_DEVICE
 * when the array's device address cannot be obtained.  Every call on one
 * device shares that device's array: calls that overlap on a device (on
 * several streams, or from several threads without ordering) race, and
 * must be serialized by the caller.  Nothing in the array needs to start
 * at zero (every byte a call reads it has written first). */
#define HM_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
hm_status hm_matvec_static(const hm_hmatrix *H, int trans, int64_t nrhs, int dtype, const void *X,
                           int64_t ldx, void *Y, int64_t ldy, int order, void *stream);

/* Device test matrix of one level and pass (0 = Omega, 1 = Psi, 2 = stage 1
 * of the uniform format, colored by hm_uniform_graph) exactly as hm_compress
 * draws it: out (device, n x ncolors*r, ld) in tree order. */
hm_status hm_test_matrix(const hm_tree *tree, int level, int pass, int32_t r, uint64_t seed,
                         int dtype, void *out, int64_t ld, void *stream);
/* Calibration of the kernel apply's roofline: the sustained TFLOP/s of the
 * 16x16x4 matrix-core instruction the kernel apply issues in dtype (HM_F64:
 * v_mfma_f64_16x16x4f64, HM_F32: v_mfma_f32_16x16x4f32), measured on the
 * current device with independent accumulator chains and no memory traffic
 * (best of 1, 2 and 4 workgroups per compute unit, 4 and 8 chains per wave;
 * about a second of device time).  tflops (host) written on success;
 * HM_E_ARG for a bad dtype or null pointer, HM_E_DEVICE on a failed launch.
 * Synchronizes the stream. */
hm_status hm_mfma_rate(int dtype, void *stream, double *tflops);
/* Raw Philox4x32-10: ctr (device, 4*count u32, counter i at 4i..4i+3),
 * out (device, 4*count u32). */
hm_status hm_philox4x32_10(const uint32_t *ctr, int64_t count, uint32_t key0, uint32_t key1,
                           uint32_t *out, void *stream);

typedef struct {
  int32_t nlevels;
  int32_t r;
  int64_t n;
  int64_t cols_A;            /* black-box columns through A */
  int64_t cols_At;           /* ... and through A* */
  int32_t colors[32];        /* colors per level (0: level not sampled); uniform
                                format: colors of the stage-2 (pair) graph */
  int32_t leaf_colors;
  int32_t leaf_width;        /* m: columns per leaf color */
  int32_t max_rank;
  int64_t npairs;            /* admissible pairs over all levels */
  int64_t nnear;             /* leaf neighbor pairs */
  int64_t saturated;         /* rank caps hit */
  int64_t nfloats;           /* stored values (U, B, V at their ranks, near blocks) */
  int32_t retries;           /* recompressions with a larger r (max_retries) */
  int32_t format;            /* HM_FORMAT_* of the compression */
  int32_t ucolors[32];       /* uniform format: stage-1 colors per level */
  double flops_blackbox;     /* 2 N^2 per black-box column */
  double flops_peel;         /* level-truncated products subtracted */
  double flops_qr;           /* pivoted QR + basis formation */
  double flops_solve;        /* coupling solves */
  double ms_total, ms_blackbox, ms_peel, ms_qr, ms_solve, ms_other; /* flags bit 0 */
  int64_t device_bytes;      /* device memory the H-matrix holds (factors, plans) */
  double bytes_peel;         /* algorithmic HBM bytes of the peel: per sampled level
                                (and the leaf pass) the samples read and written once
                                and the coarser levels' factors read once */
} hm_stats;
hm_status hm_hmatrix_stats(const hm_hmatrix *H, hm_stats *out);

/* Export for parity checks (host copies).  For `level`: npairs, then per
 * pair the two ranks and the factors U (|a| x kU), B (kU x kV), V (|b| x kV)
 * packed column-major one after another in pair order; sizes are returned
 * when the buffers are NULL. */
hm_status hm_hmatrix_export_level(const hm_hmatrix *H, int level, int64_t *npairs,
                                  int32_t *pair_a, int32_t *pair_b, int32_t *rank_u,
                                  int32_t *rank_v, int64_t *size_u, int64_t *size_b,
                                  int64_t *size_v, double *U, double *B, double *V);
/* Leaf neighbor blocks: pairs (a, b) in leaf-pair order, blocks packed
 * column-major |a| x |b|. */
hm_status hm_hmatrix_export_near(const hm_hmatrix *H, int64_t *npairs, int32_t *pair_a,
                                 int32_t *pair_b, int64_t *size, double *D);

/* ------------------------------------------------------------------ serving
 * A request loop on one GPU that keeps compressed H-matrices resident and
 * runs compressions and applies of different sizes side by side
 * (continuous batching).  nslots host workers, each with its own stream,
 * take pending requests in arrival order; a request starts as soon as a
 * worker is free and its device-memory footprint fits beside the resident
 * H-matrices and the work in flight (an apply also waits for its
 * H-matrix; a compression also waits while compress_slots others run).  Results do not depend on what else runs: every request
 * computes exactly what the same call made alone computes.
 *
 * Ownership: the server owns the H-matrices it makes (freed by
 * hm_server_release or hm_server_free).  Calls are thread-safe. */
typedef struct hm_server hm_server;

typedef struct {
  int64_t hbm_budget;     /* device bytes for residents + work in flight (<= 0: 90% of free) */
  int32_t nslots;         /* requests on the GPU at once, 1..64 */
  int32_t compress_slots; /* of which compressions, at most (<= 0: 1) */
  const hm_allocator *allocator; /* NULL, or the allocator of every device block of
                          every request (copied; ctx must outlive the server) */
} hm_server_opts;

typedef struct {
  int64_t id;       /* request id returned by the submit call */
  int32_t kind;     /* 0 compression, 1 apply */
  int32_t status;   /* hm_status of the request */
  int64_t hmatrix;  /* compression: id of the H-matrix it made (its request id);
                       apply: the H-matrix it used */
  double t_submit, t_admit, t_start, t_end; /* seconds on the server's clock */
  int64_t bytes;    /* device bytes reserved for the request */
  double device_ms; /* apply: device time between its first and last operation on
                       its stream (HIP events around the upload, the apply and the
                       download); 0 for a compression */
  double enqueue_ms; /* apply: host time from t_start until its last operation was
                       enqueued (staging into pinned memory and the enqueue calls);
                       the rest of t_end - t_start is spent waiting for the stream */
} hm_completion;

hm_status hm_server_create(const hm_server_opts *opts, hm_server **out);
/* Stops taking requests, waits for the running ones, frees every resident
 * H-matrix; pending requests are dropped. */
void hm_server_free(hm_server *srv);
/* Queue a compression: hm_build_tree(points, ...), hm_tree_color, the
 * built-in kernel black box `kernel`, hm_compress(opts).  points (host) are
 * copied.  The H-matrix id is the request id. */
hm_status hm_server_submit_compress(hm_server *srv, const double *points, int64_t n, int dim,
                                    int leaf_size, int tree_kind, int adm, int kernel,
                                    const hm_compress_opts *opts, int64_t *request_id);
/* Queue Y = H X for a resident (or queued) H-matrix: X, Y host, n x nrhs
 * column-major (ld = n), original point order, dtype HM_F64 or HM_F32.  X is
 * copied before the call returns; Y must stay valid until the completion is
 * returned by hm_server_poll. */
hm_status hm_server_submit_matvec(hm_server *srv, int64_t hmatrix, int64_t nrhs, int dtype,
                                  const void *X, void *Y, int64_t *request_id);
/* Up to max completions in completion order; waits up to wait_ms (0: no
 * wait, < 0: until one completes) when none is ready. */
hm_status hm_server_poll(hm_server *srv, int32_t max, int32_t wait_ms, hm_completion *out,
                         int32_t *count);
/* Borrow a resident H-matrix (valid until it is released). */
hm_status hm_server_hmatrix(hm_server *srv, int64_t hmatrix, const hm_hmatrix **H);
/* Evict a resident H-matrix (once its running applies finish). */
hm_status hm_server_release(hm_server *srv, int64_t hmatrix);
/* Server clock (seconds since creation), device bytes in use and budget,
 * pending and running requests, resident H-matrices; any may be NULL. */
hm_status hm_server_info(hm_server *srv, double *now, int64_t *in_use, int64_t *budget,
                         int32_t *pending, int32_t *running, int32_t *residents);

#ifdef __cplusplus
}
#endif
#endif /* HM_H */
