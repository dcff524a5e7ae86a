/*
 * Oracle (test infrastructure only): the combinatorial half of colored
 * peeling, in plain C, written for obviousness rather than speed.
 *
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg may load
 * this.  It shares no code with the GPU library.
 *
 * What it computes (Levitt & Martinsson, arXiv 2205.03406):
 *   - the box tree of section "Rank-structured matrices": each box is bisected
 *     along every dimension, empty children are dropped, boxes with more than
 *     m points are split (fig:tree for the index-halving variant);
 *   - neighbor lists (same-level boxes whose closed cubes touch, the box
 *     included) and interaction lists (children of the parent's neighbors that
 *     are not neighbors), same section;
 *   - the constraint sets of eq:h1constraints and the constraint
 *     incompatibility graph of def:incompatibility_graph, and the leaf graph
 *     of the section on extracting inadmissible blocks;
 *   - DSatur greedy coloring (alg:dsatur).
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - root cube = bounding cube of the points (the paper assumes [0,1]^d);
 *     integer coordinates c = min(2^b-1, floor(((x-lo)/s) * 2^b)) with
 *     b = 21 bits for d <= 3 and floor(63 / d) for 4 <= d <= 8 (the key of
 *     all d coordinates fits 64 bits; at most b levels);
 *   - a box that stops splitting is carried unchanged to every finer level,
 *     so each level partitions all N points;
 *   - box ids at a level are ranks of their first point in tree order;
 *   - tree order: stable sort by the interleaved key (x lowest bit);
 *   - weak admissibility (HODLR): neighbors = {box}, interaction list =
 *     the other children of the parent;
 *   - DSatur ties: larger saturation, then larger degree, then lower id;
 *     the smallest color not used by a neighbor is assigned.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>


typedef struct {
  int nv;
  int *vbox;              /* active box of each vertex */
  int *vset_ptr, *vset;   /* the box set whose complement-of-active is zeroed */
  int64_t *xadj; int *adj;
  int npairs;
  int *pair_a, *pair_b, *pair_v;  /* pair list and its vertex */
} ograph;

typedef struct {
  int n, dim, nlev, weak;
  int kb;          /* key bits per coordinate: 21 for dim <= 3, 63 / dim above */
  int os;          /* origin entries per box: max(3, dim) */
  int64_t *perm;
  int *nbox;
  int64_t **start;
  int **parent;
  int64_t **org;   /* integer cube origin, dim entries per box */
  int **blev;      /* level at which the cube was created */
  int **nei_ptr, **nei;
  int **int_ptr, **intl;
  ograph *graphs;  /* nlev admissible graphs + 1 leaf graph (index nlev) */
} otree;

/* ---------------------------------------------------------------- sort */
typedef struct { uint64_t key; int64_t idx; } kv_t;
/* memcpy of n bytes; nothing for n = 0 (the source of an empty array may be
 * a null pointer, which memcpy does not accept even for no bytes) */
static void copy_bytes(void *dst, const void *src, size_t n) {
  if (n) memcpy(dst, src, n);
}

static int kv_cmp(const void *a, const void *b) {
  const kv_t *x = (const kv_t *)a, *y = (const kv_t *)b;
  if (x->key < y->key) return -1;
  if (x->key > y->key) return 1;
  if (x->idx < y->idx) return -1;
  if (x->idx > y->idx) return 1;
  return 0;
}
typedef struct { double x; int64_t idx; } dv_t;
static int dv_cmp(const void *a, const void *b) {
  const dv_t *p = (const dv_t *)a, *q = (const dv_t *)b;
  if (p->x < q->x) return -1;
  if (p->x > q->x) return 1;
  if (p->idx < q->idx) return -1;
  if (p->idx > q->idx) return 1;
  return 0;
}
static int int_cmp(const void *a, const void *b) {
  int x = *(const int *)a, y = *(const int *)b;
  return (x > y) - (x < y);
}

/* --------------------------------------------------------- growable lists */
typedef struct { int64_t n, cap; int64_t *v; } vec64;
static void v64_push(vec64 *a, int64_t x) {
  if (a->n == a->cap) { a->cap = a->cap ? 2 * a->cap : 64; a->v = (int64_t *)realloc(a->v, a->cap * sizeof(int64_t)); }
  a->v[a->n++] = x;
}
typedef struct { int64_t n, cap; int *v; } vec32;
static void v32_push(vec32 *a, int x) {
  if (a->n == a->cap) { a->cap = a->cap ? 2 * a->cap : 64; a->v = (int *)realloc(a->v, a->cap * sizeof(int)); }
  a->v[a->n++] = x;
}

/* ------------------------------------------------------------ the tree */
static uint32_t coord_of(double x, double lo, double s, int kb) {
  double t = (x - lo) / s;
  t = t * ldexp(1.0, kb); /* 2^kb */
  double f = floor(t);
  const double top = ldexp(1.0, kb) - 1.0;
  uint32_t c = (f >= top) ? (uint32_t)top : (uint32_t)f;
  return c;
}

static uint64_t interleave(const uint32_t *c, int dim, int kb) {
  uint64_t key = 0;
  for (int b = 0; b < kb; ++b)
    for (int d = 0; d < dim; ++d)
      if ((c[d] >> b) & 1u) key |= (uint64_t)1 << (b * dim + d);
  return key;
}

/* One level under construction. */
typedef struct { vec64 start; vec32 parent; vec64 org; vec32 blev; } lvl_t;

static void push_level(otree *T, lvl_t *L, int64_t n) {
  int l = T->nlev;
  T->nbox = (int *)realloc(T->nbox, (l + 1) * sizeof(int));
  T->start = (int64_t **)realloc(T->start, (l + 1) * sizeof(int64_t *));
  T->parent = (int **)realloc(T->parent, (l + 1) * sizeof(int *));
  T->org = (int64_t **)realloc(T->org, (l + 1) * sizeof(int64_t *));
  T->blev = (int **)realloc(T->blev, (l + 1) * sizeof(int *));
  int nb = (int)L->start.n;
  T->nbox[l] = nb;
  T->start[l] = (int64_t *)malloc((nb + 1) * sizeof(int64_t));
  copy_bytes(T->start[l], L->start.v, nb * sizeof(int64_t));
  T->start[l][nb] = n;
  T->parent[l] = L->parent.v; L->parent.v = NULL;
  T->org[l] = L->org.v; L->org.v = NULL;
  T->blev[l] = L->blev.v; L->blev.v = NULL;
  free(L->start.v);
  memset(L, 0, sizeof(*L));
  T->nlev = l + 1;
}

static void build_geometric(otree *T, const double *pts, int64_t n, int dim, int m) {
  const int kb = T->kb, os = T->os;
  double lo[8] = {0}, hi[8] = {0};
  for (int d = 0; d < dim; ++d) { lo[d] = pts[d]; hi[d] = pts[d]; }
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < dim; ++d) {
      double x = pts[i * dim + d];
      if (x < lo[d]) lo[d] = x;
      if (x > hi[d]) hi[d] = x;
    }
  double s = 0;
  for (int d = 0; d < dim; ++d) if (hi[d] - lo[d] > s) s = hi[d] - lo[d];
  if (!(s > 0)) s = 1.0;
  uint32_t *c = (uint32_t *)malloc(n * dim * sizeof(uint32_t));
  kv_t *kv = (kv_t *)malloc(n * sizeof(kv_t));
  for (int64_t i = 0; i < n; ++i) {
    for (int d = 0; d < dim; ++d) c[i * dim + d] = coord_of(pts[i * dim + d], lo[d], s, kb);
    kv[i].key = interleave(&c[i * dim], dim, kb);
    kv[i].idx = i;
  }
  qsort(kv, n, sizeof(kv_t), kv_cmp);
  for (int64_t i = 0; i < n; ++i) T->perm[i] = kv[i].idx;
  /* coordinates in tree order */
  uint32_t *ct = (uint32_t *)malloc(n * dim * sizeof(uint32_t));
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < dim; ++d) ct[i * dim + d] = c[kv[i].idx * dim + d];
  free(c); free(kv);

  lvl_t L; memset(&L, 0, sizeof(L));
  v64_push(&L.start, 0); v32_push(&L.parent, -1);
  for (int d = 0; d < T->os; ++d) v64_push(&L.org, 0);
  v32_push(&L.blev, 0);
  push_level(T, &L, n);
  for (int l = 0; l < kb; ++l) {
    int nb = T->nbox[l], any = 0;
    for (int b = 0; b < nb; ++b) if (T->start[l][b + 1] - T->start[l][b] > m) any = 1;
    if (!any) break;
    for (int b = 0; b < nb; ++b) {
      int64_t s0 = T->start[l][b], s1 = T->start[l][b + 1];
      if (s1 - s0 <= m) {            /* carried leaf */
        v64_push(&L.start, s0); v32_push(&L.parent, b);
        for (int d = 0; d < os; ++d) v64_push(&L.org, T->org[l][b * os + d]);
        v32_push(&L.blev, T->blev[l][b]);
        continue;
      }
      int bit = kb - 1 - l;        /* the coordinate bit that picks the child */
      for (int ch = 0; ch < (1 << dim); ++ch) {
        int64_t first = -1;
        for (int64_t i = s0; i < s1; ++i) {
          int cc = 0;
          for (int d = 0; d < dim; ++d) cc |= (int)((ct[i * dim + d] >> bit) & 1u) << d;
          if (cc == ch) { first = i; break; }
        }
        if (first < 0) continue;     /* empty child omitted */
        v64_push(&L.start, first); v32_push(&L.parent, b);
        for (int d = 0; d < os; ++d) {
          int64_t o = T->org[l][b * os + d];
          if (d < dim && ((ch >> d) & 1)) o += (int64_t)1 << bit;
          v64_push(&L.org, o);
        }
        v32_push(&L.blev, l + 1);
      }
    }
    push_level(T, &L, n);
  }
  free(ct);
}

static void build_index_binary(otree *T, const double *pts, int64_t n, int dim, int m) {
  dv_t *dv = (dv_t *)malloc(n * sizeof(dv_t));
  for (int64_t i = 0; i < n; ++i) { dv[i].x = pts[i * dim]; dv[i].idx = i; }
  qsort(dv, n, sizeof(dv_t), dv_cmp);
  for (int64_t i = 0; i < n; ++i) T->perm[i] = dv[i].idx;
  free(dv);
  lvl_t L; memset(&L, 0, sizeof(L));
  v64_push(&L.start, 0); v32_push(&L.parent, -1);
  for (int d = 0; d < T->os; ++d) v64_push(&L.org, 0);
  v32_push(&L.blev, 0);
  push_level(T, &L, n);
  for (int l = 0; l < 62; ++l) {
    int nb = T->nbox[l], any = 0;
    for (int b = 0; b < nb; ++b) if (T->start[l][b + 1] - T->start[l][b] > m) any = 1;
    if (!any) break;
    for (int b = 0; b < nb; ++b) {
      int64_t s0 = T->start[l][b], s1 = T->start[l][b + 1];
      v64_push(&L.start, s0); v32_push(&L.parent, b);
      for (int d = 0; d < T->os; ++d) v64_push(&L.org, 0);
      v32_push(&L.blev, (s1 - s0 > m) ? l + 1 : T->blev[l][b]);
      if (s1 - s0 > m) {
        v64_push(&L.start, s0 + (s1 - s0) / 2); v32_push(&L.parent, b);
        for (int d = 0; d < T->os; ++d) v64_push(&L.org, 0);
        v32_push(&L.blev, l + 1);
      }
    }
    push_level(T, &L, n);
  }
}

/* closed cubes of boxes a and b at level l touch */
static int touch(const otree *T, int l, int a, int b) {
  for (int d = 0; d < T->dim; ++d) {
    int64_t oa = T->org[l][a * T->os + d], ob = T->org[l][b * T->os + d];
    int64_t sa = (int64_t)1 << (T->kb - T->blev[l][a]);
    int64_t sb = (int64_t)1 << (T->kb - T->blev[l][b]);
    if (!(oa <= ob + sb && ob <= oa + sa)) return 0;
  }
  return 1;
}

static int in_list(const int *a, int n, int x) {
  for (int i = 0; i < n; ++i) if (a[i] == x) return 1;
  return 0;
}

/* children of every box of level l-1, as lists of level-l boxes (ascending) */
static void child_lists(const otree *T, int l, int **ptr_out, int **idx_out) {
  int nbp = T->nbox[l - 1], nb = T->nbox[l];
  int *ptr = (int *)calloc(nbp + 1, sizeof(int));
  int *idx = (int *)malloc((nb > 0 ? nb : 1) * sizeof(int));
  for (int b = 0; b < nb; ++b) ptr[T->parent[l][b] + 1]++;
  for (int P = 0; P < nbp; ++P) ptr[P + 1] += ptr[P];
  int *fill = (int *)calloc((size_t)(nbp > 0 ? nbp : 1), sizeof(int));
  for (int b = 0; b < nb; ++b) { int P = T->parent[l][b]; idx[ptr[P] + fill[P]++] = b; }
  free(fill);
  *ptr_out = ptr; *idx_out = idx;
}

/* S(P) = children of the neighbors of P (level l-1), ascending; returns count */
static int children_of_neighbors(const otree *T, int l, const int *cptr, const int *cidx, int P, int *out) {
  int ns = 0;
  for (int t = T->nei_ptr[l - 1][P]; t < T->nei_ptr[l - 1][P + 1]; ++t) {
    int Q = T->nei[l - 1][t];
    for (int q = cptr[Q]; q < cptr[Q + 1]; ++q) out[ns++] = cidx[q];
  }
  qsort(out, ns, sizeof(int), int_cmp);
  return ns;
}

static void build_lists(otree *T) {
  T->nei_ptr = (int **)calloc(T->nlev, sizeof(int *));
  T->nei = (int **)calloc(T->nlev, sizeof(int *));
  T->int_ptr = (int **)calloc(T->nlev, sizeof(int *));
  T->intl = (int **)calloc(T->nlev, sizeof(int *));
  for (int l = 0; l < T->nlev; ++l) {
    int nb = T->nbox[l];
    vec32 ptr = {0}, idx = {0};
    v32_push(&ptr, 0);
    for (int a = 0; a < nb; ++a) {
      for (int b = 0; b < nb; ++b) {
        int is_nei = T->weak ? (a == b) : touch(T, l, a, b);
        if (is_nei) v32_push(&idx, b);
      }
      v32_push(&ptr, (int)idx.n);
    }
    T->nei_ptr[l] = ptr.v; T->nei[l] = idx.v;
    vec32 iptr = {0}, iidx = {0};
    v32_push(&iptr, 0);
    if (l > 0) {
      int *cptr, *cidx;
      child_lists(T, l, &cptr, &cidx);
      int *set = (int *)malloc((nb > 0 ? nb : 1) * sizeof(int));
      for (int a = 0; a < nb; ++a) {
        int ns = children_of_neighbors(T, l, cptr, cidx, T->parent[l][a], set);
        const int *na = &T->nei[l][T->nei_ptr[l][a]];
        int nna = T->nei_ptr[l][a + 1] - T->nei_ptr[l][a];
        for (int t = 0; t < ns; ++t)
          if (!in_list(na, nna, set[t])) v32_push(&iidx, set[t]);
        v32_push(&iptr, (int)iidx.n);
      }
      free(set); free(cptr); free(cidx);
    } else {
      for (int a = 0; a < nb; ++a) v32_push(&iptr, 0);
    }
    T->int_ptr[l] = iptr.v; T->intl[l] = iidx.v;
  }
}

/* ------------------------------------------------------------ the graphs */
/* Vertices are distinct constraint sets (active box, box set); `bybox` lists,
   for each box, the vertices whose active box it is, in creation order. */
typedef struct { vec32 vbox, sptr, sidx; vec32 *bybox; } vtab;

static int vt_find_or_add(vtab *V, int beta, const int *set, int nset) {
  vec32 *cand = &V->bybox[beta];
  for (int64_t q = 0; q < cand->n; ++q) {
    int v = cand->v[q];
    int n0 = V->sptr.v[v], n1 = V->sptr.v[v + 1];
    if (n1 - n0 == nset && memcmp(&V->sidx.v[n0], set, nset * sizeof(int)) == 0) return v;
  }
  int v = (int)V->vbox.n;
  v32_push(&V->vbox, beta);
  for (int q = 0; q < nset; ++q) v32_push(&V->sidx, set[q]);
  v32_push(&V->sptr, (int)V->sidx.n);
  v32_push(cand, v);
  return v;
}

static void finish_graph(ograph *G, vtab *V, int nboxes) {
  G->nv = (int)V->vbox.n;
  G->vbox = V->vbox.v ? V->vbox.v : (int *)malloc(sizeof(int));
  G->vset_ptr = V->sptr.v;
  G->vset = V->sidx.v ? V->sidx.v : (int *)malloc(sizeof(int));
  /* u ~ v when the active box of v lies in the zero set of u (its box set
     minus its own active box), or the other way round */
  vec32 *nb = (vec32 *)calloc(G->nv > 0 ? G->nv : 1, sizeof(vec32));
  for (int u = 0; u < G->nv; ++u) {
    for (int t = G->vset_ptr[u]; t < G->vset_ptr[u + 1]; ++t) {
      int g = G->vset[t];
      if (g == G->vbox[u]) continue;
      vec32 *cand = &V->bybox[g];
      for (int64_t q = 0; q < cand->n; ++q) {
        int v = cand->v[q];
        v32_push(&nb[u], v);
        v32_push(&nb[v], u);
      }
    }
  }
  G->xadj = (int64_t *)malloc((G->nv + 1) * sizeof(int64_t));
  G->xadj[0] = 0;
  vec32 adj = {0};
  for (int u = 0; u < G->nv; ++u) {
    if (nb[u].n > 1) qsort(nb[u].v, nb[u].n, sizeof(int), int_cmp);
    for (int64_t t = 0; t < nb[u].n; ++t)
      if (t == 0 || nb[u].v[t] != nb[u].v[t - 1]) v32_push(&adj, nb[u].v[t]);
    G->xadj[u + 1] = adj.n;
    free(nb[u].v);
  }
  G->adj = adj.v ? adj.v : (int *)malloc(sizeof(int));
  free(nb);
  for (int b = 0; b < nboxes; ++b) free(V->bybox[b].v);
  free(V->bybox);
}

static void build_level_graph(otree *T, int l, ograph *G) {
  memset(G, 0, sizeof(*G));
  int nb = T->nbox[l];
  vtab V; memset(&V, 0, sizeof(V));
  V.bybox = (vec32 *)calloc(nb > 0 ? nb : 1, sizeof(vec32));
  v32_push(&V.sptr, 0);
  vec32 pa = {0}, pb = {0}, pv = {0};
  if (l >= 1) {
    int nbp = T->nbox[l - 1];
    int *cptr, *cidx;
    child_lists(T, l, &cptr, &cidx);
    int *set = (int *)malloc((nb > 0 ? nb : 1) * sizeof(int));
    int *act = (int *)malloc((nb > 0 ? nb : 1) * sizeof(int));
    /* canonical vertex order: parents ascending, active boxes ascending */
    for (int P = 0; P < nbp; ++P) {
      int ns = children_of_neighbors(T, l, cptr, cidx, P, set);
      int na = 0;
      for (int q = cptr[P]; q < cptr[P + 1]; ++q) {
        int a = cidx[q];
        for (int t = T->int_ptr[l][a]; t < T->int_ptr[l][a + 1]; ++t)
          if (!in_list(act, na, T->intl[l][t])) act[na++] = T->intl[l][t];
      }
      qsort(act, na, sizeof(int), int_cmp);
      for (int t = 0; t < na; ++t) vt_find_or_add(&V, act[t], set, ns);
    }
    /* the pairs of the level: alpha ascending, then beta ascending */
    for (int a = 0; a < nb; ++a) {
      int ns = children_of_neighbors(T, l, cptr, cidx, T->parent[l][a], set);
      for (int t = T->int_ptr[l][a]; t < T->int_ptr[l][a + 1]; ++t) {
        int beta = T->intl[l][t];
        v32_push(&pa, a); v32_push(&pb, beta);
        v32_push(&pv, vt_find_or_add(&V, beta, set, ns));
      }
    }
    free(set); free(act); free(cptr); free(cidx);
  }
  G->npairs = (int)pa.n;
  G->pair_a = pa.v; G->pair_b = pb.v; G->pair_v = pv.v;
  finish_graph(G, &V, nb);
}

static void build_leaf_graph(otree *T, ograph *G) {
  memset(G, 0, sizeof(*G));
  int l = T->nlev - 1, nb = T->nbox[l];
  vtab V; memset(&V, 0, sizeof(V));
  V.bybox = (vec32 *)calloc(nb > 0 ? nb : 1, sizeof(vec32));
  v32_push(&V.sptr, 0);
  vec32 pa = {0}, pb = {0}, pv = {0};
  for (int a = 0; a < nb; ++a) {
    const int *set = &T->nei[l][T->nei_ptr[l][a]];
    int ns = T->nei_ptr[l][a + 1] - T->nei_ptr[l][a];
    for (int t = 0; t < ns; ++t) {
      v32_push(&pa, a); v32_push(&pb, set[t]);
      v32_push(&pv, vt_find_or_add(&V, set[t], set, ns));
    }
  }
  G->npairs = (int)pa.n;
  G->pair_a = pa.v; G->pair_b = pb.v; G->pair_v = pv.v;
  finish_graph(G, &V, nb);
}

/* ------------------------------------------------------------ DSatur */
int orc_dsatur(int nv, const int64_t *xadj, const int *adj, int *color) {
  if (nv <= 0) return 0;
  int maxdeg = 0;
  for (int v = 0; v < nv; ++v) if (xadj[v + 1] - xadj[v] > maxdeg) maxdeg = (int)(xadj[v + 1] - xadj[v]);
  int W = maxdeg + 2;
  unsigned char *seen = (unsigned char *)calloc((size_t)nv * W, 1);  /* seen[w][c]: c is on a neighbor of w */
  int *sat = (int *)calloc(nv, sizeof(int));
  int ncol = 0;
  for (int v = 0; v < nv; ++v) color[v] = -1;
  for (int step = 0; step < nv; ++step) {
    int best = -1;
    for (int v = 0; v < nv; ++v) {
      if (color[v] >= 0) continue;
      if (best < 0) { best = v; continue; }
      int64_t dv = xadj[v + 1] - xadj[v], db = xadj[best + 1] - xadj[best];
      if (sat[v] > sat[best] || (sat[v] == sat[best] && dv > db)) best = v;
    }
    int c = 0;
    while (seen[(size_t)best * W + c]) ++c;
    color[best] = c;
    if (c + 1 > ncol) ncol = c + 1;
    for (int64_t t = xadj[best]; t < xadj[best + 1]; ++t) {
      int w = adj[t];
      if (!seen[(size_t)w * W + c]) { seen[(size_t)w * W + c] = 1; sat[w]++; }
    }
  }
  free(seen); free(sat);
  return ncol;
}

/* ------------------------------------------------------------ public */
void *orc_build(const double *pts, int64_t n, int dim, int leaf, int index_binary, int weak) {
  otree *T = (otree *)calloc(1, sizeof(otree));
  T->n = (int)n; T->dim = dim; T->weak = weak;
  T->kb = dim <= 3 ? 21 : 63 / dim;
  T->os = dim > 3 ? dim : 3;
  T->perm = (int64_t *)malloc((n > 0 ? n : 1) * sizeof(int64_t));
  if (index_binary) build_index_binary(T, pts, n, dim, leaf);
  else build_geometric(T, pts, n, dim, leaf);
  build_lists(T);
  T->graphs = (ograph *)calloc(T->nlev + 1, sizeof(ograph));
  for (int l = 0; l < T->nlev; ++l) build_level_graph(T, l, &T->graphs[l]);
  build_leaf_graph(T, &T->graphs[T->nlev]);
  return T;
}

int orc_nlev(void *t) { return ((otree *)t)->nlev; }
int orc_nbox(void *t, int l) { return ((otree *)t)->nbox[l]; }
void orc_perm(void *t, int64_t *out) { otree *T = (otree *)t; copy_bytes(out, T->perm, T->n * sizeof(int64_t)); }
void orc_boxes(void *t, int l, int64_t *start, int *parent, int64_t *org, int *blev) {
  otree *T = (otree *)t; int nb = T->nbox[l];
  copy_bytes(start, T->start[l], (nb + 1) * sizeof(int64_t));
  copy_bytes(parent, T->parent[l], nb * sizeof(int));
  copy_bytes(org, T->org[l], (size_t)nb * T->os * sizeof(int64_t));
  copy_bytes(blev, T->blev[l], nb * sizeof(int));
}
int orc_list_len(void *t, int l, int which) {
  otree *T = (otree *)t; int nb = T->nbox[l];
  return which == 0 ? T->nei_ptr[l][nb] : T->int_ptr[l][nb];
}
void orc_list(void *t, int l, int which, int *ptr, int *idx) {
  otree *T = (otree *)t; int nb = T->nbox[l];
  int *p = which == 0 ? T->nei_ptr[l] : T->int_ptr[l];
  int *x = which == 0 ? T->nei[l] : T->intl[l];
  copy_bytes(ptr, p, (nb + 1) * sizeof(int));
  copy_bytes(idx, x, p[nb] * sizeof(int));
}
/* g = level for the admissible graph of that level, g = nlev for the leaf graph */
void orc_graph_sizes(void *t, int g, int *nv, int64_t *nadj, int *nset, int *npairs) {
  ograph *G = &((otree *)t)->graphs[g];
  *nv = G->nv; *nadj = G->xadj[G->nv]; *nset = G->vset_ptr[G->nv]; *npairs = G->npairs;
}
void orc_graph(void *t, int g, int *vbox, int *vset_ptr, int *vset, int64_t *xadj, int *adj,
               int *pair_a, int *pair_b, int *pair_v) {
  ograph *G = &((otree *)t)->graphs[g];
  copy_bytes(vbox, G->vbox, G->nv * sizeof(int));
  copy_bytes(vset_ptr, G->vset_ptr, (G->nv + 1) * sizeof(int));
  copy_bytes(vset, G->vset, G->vset_ptr[G->nv] * sizeof(int));
  copy_bytes(xadj, G->xadj, (G->nv + 1) * sizeof(int64_t));
  copy_bytes(adj, G->adj, G->xadj[G->nv] * sizeof(int));
  copy_bytes(pair_a, G->pair_a, G->npairs * sizeof(int));
  copy_bytes(pair_b, G->pair_b, G->npairs * sizeof(int));
  copy_bytes(pair_v, G->pair_v, G->npairs * sizeof(int));
}
void orc_free(void *t) {
  otree *T = (otree *)t;
  if (!T) return;
  for (int l = 0; l < T->nlev; ++l) {
    free(T->start[l]); free(T->parent[l]); free(T->org[l]); free(T->blev[l]);
    free(T->nei_ptr[l]); free(T->nei[l]); free(T->int_ptr[l]); free(T->intl[l]);
  }
  for (int g = 0; g <= T->nlev; ++g) {
    ograph *G = &T->graphs[g];
    free(G->vbox); free(G->vset_ptr); free(G->vset); free(G->xadj); free(G->adj);
    free(G->pair_a); free(G->pair_b); free(G->pair_v);
  }
  free(T->graphs); free(T->nbox); free(T->start); free(T->parent); free(T->org); free(T->blev);
  free(T->nei_ptr); free(T->nei); free(T->int_ptr); free(T->intl); free(T->perm); free(T);
}
