/*
 * oracle.c - plain single-threaded CPU reference of the exact-cover layout
 * decomposition path.  TEST INFRASTRUCTURE ONLY (see oracle.h): used by the
 * tests and the benchmark's CPU-baseline leg; the product library neither
 * links nor calls it, and the two share no code.
 *
 * Pipeline, in the paper's order (Sec. 2.2): layout -> layout graph ->
 * simplification -> sub-graphs -> exact-cover solve (Sec. 2.3, Algorithm 1,
 * Eq. 2) -> recovery of removed nodes -> stitch / conflict counts (Eq. 1).
 */
#include "oracle.h"

#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

void orc_free(void* p) { free(p); }

/* ------------------------------------------------------------------------
 * Layout graph (Sec. 2.1): one node per feature; a conflict edge joins two
 * features closer than the minimum coloring distance.  Reading: distance is
 * the Euclidean gap between the closed boxes, strict "<".  Stitch insertion
 * (Sec. 2.2; Fig. 1c splits features to break odd cliques) is realised as a
 * midpoint split of every rectangle longer than split_len: the two halves
 * are joined by a stitch edge and never by a conflict edge.
 * ---------------------------------------------------------------------- */

static int64_t gap2(const orc_rect* a, const orc_rect* b) {
  int64_t gx = 0, gy = 0;
  if ((int64_t)b->x0 - a->x1 > gx) gx = (int64_t)b->x0 - a->x1;
  if ((int64_t)a->x0 - b->x1 > gx) gx = (int64_t)a->x0 - b->x1;
  if ((int64_t)b->y0 - a->y1 > gy) gy = (int64_t)b->y0 - a->y1;
  if ((int64_t)a->y0 - b->y1 > gy) gy = (int64_t)a->y0 - b->y1;
  return gx * gx + gy * gy;
}

static const orc_rect* g_sort_nodes; /* qsort context (single-threaded use) */

static int cmp_by_x0(const void* pa, const void* pb) {
  int32_t a = *(const int32_t*)pa, b = *(const int32_t*)pb;
  if (g_sort_nodes[a].x0 != g_sort_nodes[b].x0)
    return g_sort_nodes[a].x0 < g_sort_nodes[b].x0 ? -1 : 1;
  return a < b ? -1 : (a > b);
}

static int cmp_pair(const void* pa, const void* pb) {
  const int32_t* a = (const int32_t*)pa;
  const int32_t* b = (const int32_t*)pb;
  if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
  return a[1] < b[1] ? -1 : (a[1] > b[1]);
}

static int cmp_i32(const void* pa, const void* pb) {
  int32_t a = *(const int32_t*)pa, b = *(const int32_t*)pb;
  return a < b ? -1 : (a > b);
}

int32_t orc_build_graph(const orc_rect* rects, int32_t n, int32_t dmin,
                        int32_t split_len, int32_t* num_nodes,
                        int64_t* num_ce, int32_t** ce, int64_t* num_se,
                        int32_t** se) {
  if (n < 0 || dmin < 0 || split_len < 0 || (n > 0 && !rects)) return -1;
  /* 1. nodes, with the midpoint split */
  orc_rect* nodes = (orc_rect*)malloc(sizeof(orc_rect) * 2 * (size_t)(n + 1));
  int32_t* partner = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(n + 1));
  int32_t* sep = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(n + 1));
  if (!nodes || !partner || !sep) { free(nodes); free(partner); free(sep); return -2; }
  int32_t nn = 0;
  int64_t ns = 0;
  for (int32_t i = 0; i < n; ++i) {
    orc_rect r = rects[i];
    int32_t w = r.x1 - r.x0, h = r.y1 - r.y0;
    int32_t len = w > h ? w : h;
    if (split_len > 0 && len > split_len) {
      orc_rect a = r, b = r;
      if (w >= h) { a.x1 = r.x0 + len / 2; b.x0 = a.x1; }   /* left half first */
      else        { a.y1 = r.y0 + len / 2; b.y0 = a.y1; }   /* lower half first */
      nodes[nn] = a; partner[nn] = nn + 1;
      nodes[nn + 1] = b; partner[nn + 1] = nn;
      sep[2 * ns] = nn; sep[2 * ns + 1] = nn + 1; ++ns;
      nn += 2;
    } else {
      nodes[nn] = r; partner[nn] = -1; ++nn;
    }
  }
  /* 2. conflict edges: sweep over nodes sorted by x0.  For x0_i <= x0_j the
   * horizontal gap is max(0, x0_j - x1_i); once it reaches dmin no later
   * node in the order can be closer than dmin. */
  int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nn + 1));
  int64_t cap = 1024, m = 0;
  int32_t* e = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)cap);
  if (!order || !e) { free(nodes); free(partner); free(sep); free(order); free(e); return -2; }
  for (int32_t i = 0; i < nn; ++i) order[i] = i;
  g_sort_nodes = nodes;
  qsort(order, (size_t)nn, sizeof(int32_t), cmp_by_x0);
  const int64_t d2 = (int64_t)dmin * dmin;
  for (int32_t a = 0; a < nn; ++a) {
    const int32_t i = order[a];
    for (int32_t b = a + 1; b < nn; ++b) {
      const int32_t j = order[b];
      if ((int64_t)nodes[j].x0 - nodes[i].x1 >= dmin) break;
      if (partner[i] == j) continue;              /* stitch pair: no conflict */
      if (gap2(&nodes[i], &nodes[j]) >= d2) continue;
      if (m == cap) {
        cap *= 2;
        int32_t* ne = (int32_t*)realloc(e, sizeof(int32_t) * 2 * (size_t)cap);
        if (!ne) { free(nodes); free(partner); free(sep); free(order); free(e); return -2; }
        e = ne;
      }
      e[2 * m] = i < j ? i : j;
      e[2 * m + 1] = i < j ? j : i;
      ++m;
    }
  }
  qsort(e, (size_t)m, 2 * sizeof(int32_t), cmp_pair);
  free(nodes); free(partner); free(order);
  *num_nodes = nn;
  *num_ce = m;
  *ce = e;
  *num_se = ns;
  *se = sep;
  return 0;
}

/* ------------------------------------------------------------------------
 * Exact-cover matrix (Sec. 2.3, Fig. 3 caption): one row per (node, color),
 * one primary column per node (each node gets exactly one color) and one
 * secondary column per (conflict edge, color) (two ends of a conflict edge
 * may not share a color: at most one 1 chosen per secondary column).  A set
 * of rows with exactly one 1 in every primary column and at most one in
 * every secondary column is a proper k-coloring of the no-stitch graph.
 * ---------------------------------------------------------------------- */

typedef struct {
  int32_t n, k;
  int64_t m;
  int32_t* edges;      /* sorted local pairs (u < w) */
  int64_t* inc_ptr;    /* incident edge ids per node, ascending */
  int32_t* inc;
} orc_comp_graph;

static int32_t make_comp_graph(int32_t n, int64_t m, const int32_t* edges,
                               int32_t k, orc_comp_graph* g) {
  g->n = n; g->k = k; g->m = m;
  g->edges = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(m + 1));
  g->inc_ptr = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  g->inc = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(m + 1));
  if (!g->edges || !g->inc_ptr || !g->inc) return -2;
  for (int64_t i = 0; i < m; ++i) {
    int32_t u = edges[2 * i], w = edges[2 * i + 1];
    if (u < 0 || w < 0 || u >= n || w >= n || u == w) return -1;
    g->edges[2 * i] = u < w ? u : w;
    g->edges[2 * i + 1] = u < w ? w : u;
  }
  qsort(g->edges, (size_t)m, 2 * sizeof(int32_t), cmp_pair);
  for (int64_t i = 1; i < m; ++i)
    if (g->edges[2 * i] == g->edges[2 * i - 2] && g->edges[2 * i + 1] == g->edges[2 * i - 1])
      return -1; /* duplicate edge */
  for (int64_t i = 0; i < m; ++i) {
    g->inc_ptr[g->edges[2 * i] + 1]++;
    g->inc_ptr[g->edges[2 * i + 1] + 1]++;
  }
  for (int32_t v = 0; v < n; ++v) g->inc_ptr[v + 1] += g->inc_ptr[v];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
  if (!fill) return -2;
  memcpy(fill, g->inc_ptr, sizeof(int64_t) * ((size_t)n + 1));
  for (int64_t i = 0; i < m; ++i) {   /* edge ids ascending per node */
    g->inc[fill[g->edges[2 * i]]++] = (int32_t)i;
    g->inc[fill[g->edges[2 * i + 1]]++] = (int32_t)i;
  }
  free(fill);
  return 0;
}

static void free_comp_graph(orc_comp_graph* g) {
  free(g->edges); free(g->inc_ptr); free(g->inc);
}

int32_t orc_ec_matrix(int32_t n, int64_t m, const int32_t* edges, int32_t k,
                      int64_t** row_ptr, int32_t** col_idx) {
  if (n < 0 || m < 0 || k < 1) return -1;
  orc_comp_graph g;
  int32_t rc = make_comp_graph(n, m, edges, k, &g);
  if (rc) { free_comp_graph(&g); return rc; }
  const int64_t rows = (int64_t)n * k;
  int64_t* rp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(rows + 1));
  int32_t* ci = (int32_t*)malloc(sizeof(int32_t) * (size_t)(rows + 2 * m * k + 1));
  if (!rp || !ci) { free(rp); free(ci); free_comp_graph(&g); return -2; }
  int64_t p = 0;
  for (int32_t v = 0; v < n; ++v)
    for (int32_t c = 0; c < k; ++c) {
      rp[(int64_t)v * k + c] = p;
      ci[p++] = v;
      for (int64_t t = g.inc_ptr[v]; t < g.inc_ptr[v + 1]; ++t)
        ci[p++] = n + g.inc[t] * k + c;
    }
  rp[rows] = p;
  free_comp_graph(&g);
  *row_ptr = rp;
  *col_idx = ci;
  return 0;
}

/* ------------------------------------------------------------------------
 * Dancing links (Knuth) on the exact-cover matrix.  Node 0 is the root;
 * nodes 1..C are column headers (column j -> header j+1); primary headers
 * sit on the root's horizontal ring in index order, secondary headers are
 * self-linked.  Each 1 of the matrix is a node linked into its row
 * (horizontal ring) and its column (vertical ring, rows in ascending order).
 * Cover/uncover are Eq. 2 applied to the header and to every node of every
 * row in the column.
 * ---------------------------------------------------------------------- */

typedef struct {
  int32_t *L, *R, *U, *D, *col, *row;
  int32_t* size;
  int32_t nprim;
  /* search state */
  int64_t budget, nodes;
  uint64_t hash;
  int32_t status; /* -1 while running */
  int32_t depth_at_stop;
  int32_t* sol;   /* row chosen at each depth */
  /* stitch-aware row order (NULL partner: rows ascending) */
  int32_t k;
  const int32_t* partner;   /* stitch partner of each node in the component, -1 none */
  int8_t* color;            /* color of each node on the current path, -1 none */
} orc_dlx;

static void dlx_cover(orc_dlx* x, int32_t c) {
  x->L[x->R[c]] = x->L[c];
  x->R[x->L[c]] = x->R[c];
  for (int32_t i = x->D[c]; i != c; i = x->D[i])
    for (int32_t j = x->R[i]; j != i; j = x->R[j]) {
      x->U[x->D[j]] = x->U[j];
      x->D[x->U[j]] = x->D[j];
      x->size[x->col[j]]--;
    }
}

static void dlx_uncover(orc_dlx* x, int32_t c) {
  for (int32_t i = x->U[c]; i != c; i = x->U[i])
    for (int32_t j = x->L[i]; j != i; j = x->L[j]) {
      x->size[x->col[j]]++;
      x->U[x->D[j]] = j;
      x->D[x->U[j]] = j;
    }
  x->L[x->R[c]] = c;
  x->R[x->L[c]] = c;
}

/* Trace fingerprint (our check of the search order; the method defines no
 * such value).  Each counted search node contributes x = FNV-1a 64
 * (Fowler/Noll/Vo) of its 16 bytes - depth, entering row, chosen column,
 * its size; each u32 little-endian (entering row 0xFFFFFFFF at the root,
 * column 0xFFFFFFFF at a solution) - started from the offset basis; the
 * fingerprint of N nodes in search order is the sum of x_i * B^(N-i) modulo
 * 2^64 with B the FNV prime, i.e. h = h * B + x per node from h = 0.  The
 * fingerprint of a trace S followed by a trace T is then h(S) * B^|T| +
 * h(T), so subtrees searched apart can be combined in search order. */
static uint64_t fnv_u32(uint64_t h, uint32_t v) {
  for (int b = 0; b < 4; ++b) {
    h ^= (v >> (8 * b)) & 0xffu;
    h *= 0x100000001b3ULL;
  }
  return h;
}

static void trace_node(orc_dlx* x, uint32_t depth, uint32_t row_in, uint32_t col,
                       uint32_t size) {
  uint64_t h = 0xcbf29ce484222325ULL;
  h = fnv_u32(h, depth);
  h = fnv_u32(h, row_in);
  h = fnv_u32(h, col);
  h = fnv_u32(h, size);
  x->hash = x->hash * 0x100000001b3ULL + h;
}

/* Algorithm X (Algorithm 1): stop when every primary column is covered (the
 * first solution ends the search); otherwise take the uncovered primary
 * column with the fewest rows, ties to the lowest index (our reading of
 * Algorithm 1's column rule, which prefers single-row columns and otherwise
 * follows BFS order: the index is the BFS position), cover it, and try its
 * rows in ascending order - include the
 * row, cover its other columns, recurse, uncover, exclude - then uncover the
 * column.  An empty column is a dead end (the hot path reports INFEASIBLE
 * instead of marking conflict candidates).  A search node is an entry that
 * passes the budget test; the budget is tested before counting. */
static void dlx_search(orc_dlx* x, int32_t depth, int32_t row_in) {
  if (x->nodes == x->budget) {
    x->status = ORC_BUDGET;
    x->depth_at_stop = depth;
    return;
  }
  x->nodes++;
  if (x->R[0] == 0) {
    trace_node(x, (uint32_t)depth, (uint32_t)row_in, 0xffffffffu, 0);
    x->status = ORC_FEASIBLE;
    x->depth_at_stop = depth;
    return;
  }
  int32_t c = x->R[0];
  for (int32_t j = x->R[c]; j != 0 && x->size[c] > 0; j = x->R[j])
    if (x->size[j] < x->size[c]) c = j;
  trace_node(x, (uint32_t)depth, (uint32_t)row_in, (uint32_t)(c - 1),
             (uint32_t)x->size[c]);
  if (x->size[c] == 0) return;
  dlx_cover(x, c);
  /* Rows in ascending order; with the stitch-aware order the row of the
   * color the column's stitch partner already has (if that row is still
   * there) goes first (Eq. 1: a pair of halves colored alike is no stitch). */
  int32_t first = -1;
  if (x->partner) {
    const int32_t v = c - 1, p = x->partner[v];
    if (p >= 0 && x->color[p] >= 0)
      for (int32_t r = x->D[c]; r != c; r = x->D[r])
        if (x->row[r] == v * x->k + x->color[p]) first = r;
  }
  for (int32_t pass = first >= 0 ? 0 : 1; pass < 2; ++pass)
    for (int32_t r = pass == 0 ? first : x->D[c]; r != c; r = pass == 0 ? c : x->D[r]) {
      if (pass == 1 && r == first) continue;
      x->sol[depth] = x->row[r];
      if (x->partner) x->color[x->row[r] / x->k] = (int8_t)(x->row[r] % x->k);
      for (int32_t j = x->R[r]; j != r; j = x->R[j]) dlx_cover(x, x->col[j]);
      dlx_search(x, depth + 1, x->row[r]);
      if (x->status >= 0) return;
      for (int32_t j = x->L[r]; j != r; j = x->L[j]) dlx_uncover(x, x->col[j]);
      if (x->partner) x->color[x->row[r] / x->k] = -1;
    }
  dlx_uncover(x, c);
}

/* Links the matrix (CSR over rows rp/ci) into x's arrays: root, headers
 * (primaries on the root ring in index order, secondaries self-linked),
 * then every 1 into its row ring and, rows ascending, its column. */
static void dlx_link(orc_dlx* x, int32_t n, int32_t ncols, int64_t rows, const int64_t* rp,
                     const int32_t* ci) {
  /* root and headers */
  for (int32_t h = 0; h <= ncols; ++h) {
    x->U[h] = x->D[h] = h;
    x->col[h] = h;
    x->row[h] = -1;
    x->L[h] = x->R[h] = h;
  }
  x->nprim = n;
  for (int32_t h = 1; h <= n; ++h) {  /* primary ring: root, 1, 2, ..., n */
    x->L[h] = h - 1;
    x->R[h - 1] = h;
  }
  if (n > 0) { x->R[n] = 0; x->L[0] = n; }
  /* rows, ascending */
  int32_t next = ncols + 1;
  for (int64_t r = 0; r < rows; ++r) {
    int32_t first = -1;
    for (int64_t p = rp[r]; p < rp[r + 1]; ++p) {
      const int32_t h = ci[p] + 1;
      const int32_t nd = next++;
      x->col[nd] = h;
      x->row[nd] = (int32_t)r;
      x->U[nd] = x->U[h]; x->D[nd] = h;
      x->D[x->U[h]] = nd; x->U[h] = nd;
      x->size[h]++;
      if (first < 0) { first = nd; x->L[nd] = x->R[nd] = nd; }
      else { x->L[nd] = x->L[first]; x->R[nd] = first; x->R[x->L[first]] = nd; x->L[first] = nd; }
    }
  }
}

/* Allocates the link arrays for `total` nodes and n rows of solution. */
static int32_t dlx_alloc(orc_dlx* x, int64_t total, int32_t n) {
  memset(x, 0, sizeof(*x));
  x->L = (int32_t*)malloc(sizeof(int32_t) * (size_t)total);
  x->R = (int32_t*)malloc(sizeof(int32_t) * (size_t)total);
  x->U = (int32_t*)malloc(sizeof(int32_t) * (size_t)total);
  x->D = (int32_t*)malloc(sizeof(int32_t) * (size_t)total);
  x->col = (int32_t*)malloc(sizeof(int32_t) * (size_t)total);
  x->row = (int32_t*)malloc(sizeof(int32_t) * (size_t)total);
  x->size = (int32_t*)calloc((size_t)total, sizeof(int32_t));
  x->sol = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  return (x->L && x->R && x->U && x->D && x->col && x->row && x->size && x->sol) ? 0 : -2;
}

static void dlx_free(orc_dlx* x) {
  free(x->L); free(x->R); free(x->U); free(x->D); free(x->col); free(x->row);
  free(x->size); free(x->sol);
}

int32_t orc_solve_component(int32_t n, int64_t m, const int32_t* edges,
                            int32_t k, int64_t budget, int8_t* colors,
                            int32_t* status, int64_t* nodes,
                            uint64_t* trace_hash, int32_t* depth_at_stop) {
  return orc_solve_component_stitch(n, m, edges, k, budget, NULL, colors, status, nodes,
                                    trace_hash, depth_at_stop);
}

int32_t orc_solve_component_stitch(int32_t n, int64_t m, const int32_t* edges,
                                   int32_t k, int64_t budget, const int32_t* partner,
                                   int8_t* colors, int32_t* status, int64_t* nodes,
                                   uint64_t* trace_hash, int32_t* depth_at_stop) {
  if (n < 0 || m < 0 || k < 1 || k > 127 || budget < 1) return -1;
  if (partner)
    for (int32_t v = 0; v < n; ++v)
      if (partner[v] >= n || partner[v] == v || (partner[v] >= 0 && partner[partner[v]] != v))
        return -1;
  if (m > 0 && !edges) return -1;
  orc_comp_graph g;
  int32_t rc = make_comp_graph(n, m, edges, k, &g);
  if (rc) { free_comp_graph(&g); return rc; }
  int64_t* rp = NULL;
  int32_t* ci = NULL;
  rc = orc_ec_matrix(n, m, g.edges, k, &rp, &ci);
  if (rc) { free_comp_graph(&g); return rc; }
  const int32_t ncols = (int32_t)(n + m * k);
  const int64_t rows = (int64_t)n * k;
  const int64_t ones = rp[rows];
  const int64_t total = 1 + (int64_t)ncols + ones;
  orc_dlx x;
  if (dlx_alloc(&x, total, n)) {
    rc = -2;
    goto done;
  }
  dlx_link(&x, n, ncols, rows, rp, ci);
  x.k = k;
  x.partner = partner;
  x.color = NULL;
  if (partner) {
    x.color = (int8_t*)malloc((size_t)n + 1);
    if (!x.color) { rc = -2; goto done; }
    for (int32_t v = 0; v < n; ++v) x.color[v] = -1;
  }
  x.budget = budget;
  x.nodes = 0;
  x.hash = 0;
  x.status = -1;
  x.depth_at_stop = 0;
  dlx_search(&x, 0, -1);
  if (x.status < 0) x.status = ORC_INFEASIBLE;
  for (int32_t v = 0; v < n; ++v) colors[v] = -1;
  if (x.status == ORC_FEASIBLE)
    for (int32_t d = 0; d < x.depth_at_stop; ++d)
      colors[x.sol[d] / k] = (int8_t)(x.sol[d] % k);
  *status = x.status;
  *nodes = x.nodes;
  *trace_hash = x.hash;
  if (depth_at_stop) *depth_at_stop = x.status == ORC_INFEASIBLE ? 0 : x.depth_at_stop;
  rc = 0;
done:
  free(x.color);
  dlx_free(&x);
  free(rp); free(ci);
  free_comp_graph(&g);
  return rc;
}

/* ------------------------------------------------------------------------
 * Conflict marking (Algorithm 1: a column left with no related row is
 * marked as a conflict candidate (cl, cl'), cl' being the column whose cover
 * removed cl's final row).  Reading: a component whose search ends without
 * a solution is still colored, by one descent of the same search that never
 * backtracks.  The column is chosen by the search's rule and its first
 * remaining row is included; a column with no row left is a conflict
 * candidate and takes its final removed row anyway: the column and those of
 * the row's secondary columns that are still uncovered are covered, and the
 * covered ones are the marked conflicts.  Every primary column ends covered,
 * so every node gets a color; the conflicts are the conflict edges whose
 * ends share a color (Eq. 1).
 * ---------------------------------------------------------------------- */

/* Eq. 2 cover that also records, for every primary column that loses a row,
 * the row it lost last. */
static void dlx_cover_track(orc_dlx* x, int32_t c, int32_t* last_row) {
  x->L[x->R[c]] = x->L[c];
  x->R[x->L[c]] = x->R[c];
  for (int32_t i = x->D[c]; i != c; i = x->D[i])
    for (int32_t j = x->R[i]; j != i; j = x->R[j]) {
      x->U[x->D[j]] = x->U[j];
      x->D[x->U[j]] = x->D[j];
      x->size[x->col[j]]--;
      if (x->col[j] <= x->nprim) last_row[x->col[j]] = x->row[j];
    }
}

int32_t orc_mark_conflicts(int32_t n, int64_t m, const int32_t* edges, int32_t k,
                           int8_t* colors) {
  if (n < 0 || m < 0 || k < 1 || k > 127) return -1;
  if (m > 0 && !edges) return -1;
  orc_comp_graph g;
  int32_t rc = make_comp_graph(n, m, edges, k, &g);
  if (rc) { free_comp_graph(&g); return rc; }
  int64_t* rp = NULL;
  int32_t* ci = NULL;
  rc = orc_ec_matrix(n, m, g.edges, k, &rp, &ci);
  if (rc) { free_comp_graph(&g); return rc; }
  const int32_t ncols = (int32_t)(n + m * k);
  const int64_t rows = (int64_t)n * k;
  const int64_t total = 1 + (int64_t)ncols + rp[rows];
  orc_dlx x;
  int32_t* last_row = (int32_t*)malloc(sizeof(int32_t) * ((size_t)ncols + 1));
  int32_t* row_node = (int32_t*)malloc(sizeof(int32_t) * ((size_t)rows + 1));
  char* covered = (char*)calloc((size_t)ncols + 1, 1);
  if (dlx_alloc(&x, total, n) || !last_row || !row_node || !covered) {
    rc = -2;
    goto done;
  }
  dlx_link(&x, n, ncols, rows, rp, ci);
  for (int32_t h = 0; h <= ncols; ++h) last_row[h] = -1;
  for (int64_t nd = ncols + 1; nd < total; ++nd)   /* each row's node in its primary column */
    if (x.col[nd] <= n) row_node[x.row[nd]] = (int32_t)nd;
  for (int32_t v = 0; v < n; ++v) colors[v] = -1;
  while (x.R[0] != 0) {
    int32_t c = x.R[0];
    for (int32_t j = x.R[c]; j != 0 && x.size[c] > 0; j = x.R[j])
      if (x.size[j] < x.size[c]) c = j;
    /* the first remaining row, or for a conflict candidate the final one removed */
    const int32_t rw = x.size[c] > 0 ? x.row[x.D[c]] : last_row[c];
    if (rw < 0) { rc = -6; goto done; }   /* impossible: every column starts with k rows */
    const int32_t nd = row_node[rw];
    dlx_cover_track(&x, c, last_row);
    covered[c] = 1;
    for (int32_t j = x.R[nd]; j != nd; j = x.R[j])
      if (!covered[x.col[j]]) {
        dlx_cover_track(&x, x.col[j], last_row);
        covered[x.col[j]] = 1;
      }
    colors[rw / k] = (int8_t)(rw % k);
  }
  rc = 0;
done:
  dlx_free(&x);
  free(last_row); free(row_node); free(covered);
  free(rp); free(ci);
  free_comp_graph(&g);
  return rc;
}

/* ------------------------------------------------------------------------
 * Eq. 1 minimisation (Sec. 2.1 objective with alpha = 0.1; Algorithm 1's
 * conflict candidates generalised).  Reading: the exact-cover search is
 * relaxed so that a row whose secondary columns are already covered may
 * still be taken, each such covered (edge, color) column counting one
 * conflict; a row (v, c) whose node's stitch partner already holds another
 * color counts one stitch.  Cost = 10 conflicts + stitches (Eq. 1 scaled by
 * 10, integers).  A depth-first branch and bound over the rows finds a
 * coloring of least cost, starting from an incumbent coloring (the first
 * solution, or the conflict-marking descent):
 *   - penalty p(u, c) of an uncolored node = 10 x (colored neighbours of
 *     color c) + 1 if its partner is colored with a color other than c;
 *   - lower bound = cost so far + sum over uncolored u of min_c p(u, c)
 *     (each term charges edges to colored nodes only, so the terms are
 *     disjoint and can only grow);
 *   - a node entry that passes the budget test counts one node; with every
 *     node colored it replaces the incumbent if cheaper; otherwise it
 *     returns when the bound reaches the incumbent's cost, else takes the
 *     uncolored node with the fewest conflict-free colors (lowest index on
 *     ties) and tries its colors in ascending order, skipping a color whose
 *     child bound (bound - min_c p(v, c) + p(v, c)) reaches the incumbent's
 *     cost at the moment it is tried.
 * ---------------------------------------------------------------------- */

typedef struct {
  int32_t n, k;
  const int64_t* ap;      /* adjacency (both directions) */
  const int32_t* adj;
  const int32_t* partner; /* stitch partner (-1 none) or NULL */
  int8_t* col;            /* current colors, -1 uncolored */
  int32_t* cnt;           /* cnt[u * k + c]: colored neighbours of u with color c */
  int8_t* pcol;           /* color of u's partner, -1 none or uncolored */
  int64_t budget, nodes;
  int32_t stopped;
  int32_t cost, best;
  int8_t* best_col;
} orc_bb;

static int32_t bb_pen(const orc_bb* b, int32_t u, int32_t c) {
  return 10 * b->cnt[(int64_t)u * b->k + c] + ((b->pcol[u] >= 0 && b->pcol[u] != c) ? 1 : 0);
}

static int32_t bb_minpen(const orc_bb* b, int32_t u) {
  int32_t m = bb_pen(b, u, 0);
  for (int32_t c = 1; c < b->k; ++c) {
    const int32_t p = bb_pen(b, u, c);
    if (p < m) m = p;
  }
  return m;
}

/* colors c with no colored neighbour of color c (the node's open rows) */
static int32_t bb_open(const orc_bb* b, int32_t u) {
  int32_t o = 0;
  for (int32_t c = 0; c < b->k; ++c) o += b->cnt[(int64_t)u * b->k + c] == 0;
  return o;
}

/* colors v with c (delta = +1) or takes that color back (delta = -1) */
static void bb_set(orc_bb* b, int32_t v, int32_t c, int32_t delta) {
  for (int64_t t = b->ap[v]; t < b->ap[v + 1]; ++t) b->cnt[(int64_t)b->adj[t] * b->k + c] += delta;
  if (b->partner && b->partner[v] >= 0) b->pcol[b->partner[v]] = (int8_t)(delta > 0 ? c : -1);
  b->col[v] = (int8_t)(delta > 0 ? c : -1);
}

static void bb_search(orc_bb* b) {
  if (b->nodes == b->budget) {
    b->stopped = 1;
    return;
  }
  b->nodes++;
  int32_t lb = b->cost, v = -1, vopen = b->k + 1;
  for (int32_t u = 0; u < b->n; ++u) {
    if (b->col[u] >= 0) continue;
    lb += bb_minpen(b, u);
    const int32_t o = bb_open(b, u);
    if (o < vopen) { vopen = o; v = u; }
  }
  if (v < 0) {   /* every node colored */
    if (b->cost < b->best) {
      b->best = b->cost;
      memcpy(b->best_col, b->col, (size_t)b->n);
    }
    return;
  }
  if (lb >= b->best) return;
  const int32_t mpv = bb_minpen(b, v);
  for (int32_t c = 0; c < b->k; ++c) {
    const int32_t pen = bb_pen(b, v, c);
    if (lb - mpv + pen >= b->best) continue;
    bb_set(b, v, c, +1);
    b->cost += pen;
    bb_search(b);
    b->cost -= pen;
    bb_set(b, v, c, -1);
    if (b->stopped) return;
  }
}

/* Eq. 1 cost of a complete coloring: 10 per conflict edge colored alike,
 * 1 per stitch pair colored differently (each pair once). */
static int32_t eq1_cost(int32_t n, int64_t m, const int32_t* edges, const int32_t* partner,
                        const int8_t* colors) {
  int32_t cost = 0;
  for (int64_t e = 0; e < m; ++e)
    if (colors[edges[2 * e]] == colors[edges[2 * e + 1]]) cost += 10;
  if (partner)
    for (int32_t v = 0; v < n; ++v)
      if (partner[v] > v && colors[v] != colors[partner[v]]) cost += 1;
  return cost;
}

int32_t orc_minimize_component(int32_t n, int64_t m, const int32_t* edges, int32_t k,
                               const int32_t* partner, int64_t budget, int8_t* colors,
                               int64_t* nodes, int32_t* stopped, int32_t* cost) {
  if (n < 0 || m < 0 || k < 1 || k > 127 || budget < 1 || (m > 0 && !edges)) return -1;
  for (int32_t v = 0; v < n; ++v) {
    if (colors[v] < 0 || colors[v] >= k) return -1;   /* the incumbent is complete */
    if (partner && (partner[v] >= n || partner[v] == v ||
                    (partner[v] >= 0 && partner[partner[v]] != v)))
      return -1;
  }
  *nodes = 0;
  *stopped = 0;
  *cost = eq1_cost(n, m, edges, partner, colors);
  if (*cost == 0) return 0;   /* nothing to improve: not run */
  int64_t* ap = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t* adj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
  int32_t* cnt = (int32_t*)calloc((size_t)n * (size_t)k + 1, sizeof(int32_t));
  int8_t* col = (int8_t*)malloc((size_t)n + 1);
  int8_t* pcol = (int8_t*)malloc((size_t)n + 1);
  int32_t rc = 0;
  if (!ap || !adj || !fill || !cnt || !col || !pcol) { rc = -2; goto done; }
  for (int64_t e = 0; e < m; ++e) {
    const int32_t u = edges[2 * e], w = edges[2 * e + 1];
    if (u < 0 || w < 0 || u >= n || w >= n || u == w) { rc = -1; goto done; }
    ap[u + 1]++; ap[w + 1]++;
  }
  for (int32_t v = 0; v < n; ++v) ap[v + 1] += ap[v];
  memcpy(fill, ap, sizeof(int64_t) * ((size_t)n + 1));
  for (int64_t e = 0; e < m; ++e) {
    adj[fill[edges[2 * e]]++] = edges[2 * e + 1];
    adj[fill[edges[2 * e + 1]]++] = edges[2 * e];
  }
  for (int32_t v = 0; v < n; ++v) { col[v] = -1; pcol[v] = -1; }
  orc_bb b;
  b.n = n; b.k = k; b.ap = ap; b.adj = adj; b.partner = partner;
  b.col = col; b.cnt = cnt; b.pcol = pcol;
  b.budget = budget; b.nodes = 0; b.stopped = 0;
  b.cost = 0; b.best = *cost; b.best_col = colors;
  bb_search(&b);
  *nodes = b.nodes;
  *stopped = b.stopped;
  *cost = b.best;
done:
  free(ap); free(adj); free(fill); free(cnt); free(col); free(pcol);
  return rc;
}

/* ------------------------------------------------------------------------
 * Whole flow (Sec. 2.2).
 * Simplification reading: iterative removal of nodes with conflict degree
 * < k, first-in first-out - seed the queue with every such node in
 * ascending id, then pop a node, remove it, lower its remaining
 * neighbours' degrees in ascending id and queue each one that drops below
 * k.  The removal order is kept for recovery.
 * Sub-graphs (Algorithm 1): connected components of the remaining nodes
 * over conflict edges, ordered by smallest id; local index = BFS order from
 * that node, neighbours in ascending id.
 * Recovery reading: in reverse removal order a node takes its stitch
 * partner's color when the partner is colored and no colored conflict
 * neighbour uses it, else the lowest color no colored conflict neighbour
 * uses.
 * ---------------------------------------------------------------------- */

/* Adjacency lists (ascending) and stitch partners; validates the input. */
static int32_t build_adjacency(int32_t n, int64_t num_ce, const int32_t* ce,
                               int64_t num_se, const int32_t* se, int64_t* ap,
                               int32_t* adj, int32_t* partner) {
  for (int32_t v = 0; v <= n; ++v) ap[v] = 0;
  for (int64_t i = 0; i < num_ce; ++i) {
    int32_t u = ce[2 * i], v = ce[2 * i + 1];
    if (u < 0 || v < 0 || u >= n || v >= n || u == v) return -1;
    ap[u + 1]++; ap[v + 1]++;
  }
  for (int32_t v = 0; v < n; ++v) ap[v + 1] += ap[v];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
  if (!fill) return -2;
  memcpy(fill, ap, sizeof(int64_t) * ((size_t)n + 1));
  for (int64_t i = 0; i < num_ce; ++i) {
    adj[fill[ce[2 * i]]++] = ce[2 * i + 1];
    adj[fill[ce[2 * i + 1]]++] = ce[2 * i];
  }
  free(fill);
  for (int32_t v = 0; v < n; ++v) {
    qsort(adj + ap[v], (size_t)(ap[v + 1] - ap[v]), sizeof(int32_t), cmp_i32);
    for (int64_t t = ap[v] + 1; t < ap[v + 1]; ++t)
      if (adj[t] == adj[t - 1]) return -1;   /* duplicate edge */
    partner[v] = -1;
  }
  for (int64_t i = 0; i < num_se; ++i) {
    int32_t u = se[2 * i], v = se[2 * i + 1];
    if (u < 0 || v < 0 || u >= n || v >= n || u == v) return -1;
    if (partner[u] >= 0 || partner[v] >= 0) return -1;  /* one partner per node */
    partner[u] = v; partner[v] = u;
  }
  for (int64_t i = 0; i < num_se; ++i) {           /* a stitch pair is no conflict pair */
    int32_t u = se[2 * i], v = se[2 * i + 1];
    for (int64_t t = ap[u]; t < ap[u + 1]; ++t)
      if (adj[t] == v) return -1;
  }
  return 0;
}

/* Simplification and sub-graphs.  removal[0 .. *nrem-1] = removal order;
 * comp_of[v] = component or -1; bfs = core nodes grouped by component, each
 * in local (BFS) order; comp_ptr[c] .. comp_ptr[c+1] delimits component c. */
static int32_t simplify_split(int32_t n, const int64_t* ap, const int32_t* adj,
                              int32_t k, uint32_t flags, int32_t* removal,
                              int32_t* nrem_out, int32_t* comp_of, int32_t* bfs,
                              int32_t* comp_ptr, int32_t* nc_out) {
  int32_t* deg = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  char* removed = (char*)calloc((size_t)n + 1, 1);
  char* queued = (char*)calloc((size_t)n + 1, 1);
  if (!deg || !removed || !queued) { free(deg); free(removed); free(queued); return -2; }
  for (int32_t v = 0; v < n; ++v) deg[v] = (int32_t)(ap[v + 1] - ap[v]);
  int32_t head = 0, tail = 0;
  if (flags & ORC_SIMPLIFY) {
    for (int32_t v = 0; v < n; ++v)
      if (deg[v] < k) { removal[tail++] = v; queued[v] = 1; }
    while (head < tail) {
      const int32_t u = removal[head++];
      removed[u] = 1;
      for (int64_t t = ap[u]; t < ap[u + 1]; ++t) {
        const int32_t w = adj[t];
        if (removed[w]) continue;
        deg[w]--;
        if (deg[w] < k && !queued[w]) { removal[tail++] = w; queued[w] = 1; }
      }
    }
  }
  *nrem_out = tail;
  int32_t nc = 0, pos = 0;
  for (int32_t v = 0; v < n; ++v) comp_of[v] = -1;
  comp_ptr[0] = 0;
  for (int32_t s = 0; s < n; ++s) {
    if (removed[s] || comp_of[s] >= 0) continue;
    int32_t h = pos;
    bfs[pos++] = s;
    comp_of[s] = nc;
    while (h < pos) {
      const int32_t x = bfs[h++];
      for (int64_t t = ap[x]; t < ap[x + 1]; ++t) {
        const int32_t w = adj[t];
        if (removed[w] || comp_of[w] >= 0) continue;
        comp_of[w] = nc;
        bfs[pos++] = w;
      }
    }
    comp_ptr[++nc] = pos;
  }
  *nc_out = nc;
  free(deg); free(removed); free(queued);
  return 0;
}

int32_t orc_simplify(int32_t num_nodes, int64_t num_ce, const int32_t* ce,
                     int32_t k, uint32_t flags, int32_t* removal_order,
                     int32_t* num_removed, int32_t* comp_of, int32_t* bfs_order,
                     int32_t* comp_ptr, int32_t* num_comps) {
  if (num_nodes < 0 || num_ce < 0 || k < 1) return -1;
  const int32_t n = num_nodes;
  int64_t* ap = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
  int32_t* adj = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(num_ce + 1));
  int32_t* partner = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  int32_t rc = -2;
  if (ap && adj && partner) {
    rc = build_adjacency(n, num_ce, ce, 0, NULL, ap, adj, partner);
    if (!rc)
      rc = simplify_split(n, ap, adj, k, flags, removal_order, num_removed,
                          comp_of, bfs_order, comp_ptr, num_comps);
  }
  free(ap); free(adj); free(partner);
  return rc;
}

int32_t orc_decompose(int32_t num_nodes, int64_t num_ce, const int32_t* ce,
                      int64_t num_se, const int32_t* se, int32_t k,
                      int64_t budget, int64_t min_budget, uint32_t flags, int8_t* colors,
                      int32_t* comp_of, int32_t* num_comps, orc_comp** comps,
                      int64_t* total_stitches, int64_t* total_conflicts,
                      int64_t* total_uncolored) {
  if (num_nodes < 0 || num_ce < 0 || num_se < 0 || k < 1 || k > 64 || budget < 1)
    return -1;
  if ((flags & ORC_MINIMIZE) && (min_budget < 1 || min_budget > INT32_MAX)) return -1;
  const int32_t n = num_nodes;
  int32_t rc = 0;
  int64_t* ap = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
  int32_t* adj = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(num_ce + 1));
  int32_t* partner = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  int32_t* removal = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  int32_t* bfs = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  int32_t* comp_ptr = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 2));
  int32_t* local = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  int32_t* ledges = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(num_ce + 1));
  int8_t* lcolors = (int8_t*)malloc((size_t)n + 1);
  int32_t* lpartner = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  orc_comp* cs = NULL;
  int32_t nrem = 0, nc = 0;
  if (!ap || !adj || !partner || !removal || !bfs || !comp_ptr || !local ||
      !ledges || !lcolors || !lpartner) { rc = -2; goto out; }
  rc = build_adjacency(n, num_ce, ce, num_se, se, ap, adj, partner);
  if (rc) goto out;
  rc = simplify_split(n, ap, adj, k, flags, removal, &nrem, comp_of, bfs,
                      comp_ptr, &nc);
  if (rc) goto out;
  cs = (orc_comp*)malloc(sizeof(orc_comp) * ((size_t)nc + 1));
  if (!cs) { rc = -2; goto out; }

  /* solve every sub-graph in its local numbering */
  for (int32_t v = 0; v < n; ++v) { colors[v] = -1; local[v] = -1; }
  for (int32_t c = 0; c < nc; ++c) {
    const int32_t* nodes = bfs + comp_ptr[c];
    const int32_t size = comp_ptr[c + 1] - comp_ptr[c];
    for (int32_t i = 0; i < size; ++i) local[nodes[i]] = i;
    int64_t lm = 0;
    for (int32_t i = 0; i < size; ++i) {
      const int32_t x = nodes[i];
      for (int64_t t = ap[x]; t < ap[x + 1]; ++t) {
        const int32_t w = adj[t];
        if (comp_of[w] != c || local[w] <= i) continue;
        ledges[2 * lm] = i;
        ledges[2 * lm + 1] = local[w];
        ++lm;
      }
    }
    orc_comp* r = &cs[c];
    r->size = size;
    r->first_node = nodes[0];
    r->num_edges = (int32_t)lm;
    if (flags & (ORC_STITCH | ORC_MINIMIZE))   /* stitch partners inside the component, local ids */
      for (int32_t i = 0; i < size; ++i) {
        const int32_t p = partner[nodes[i]];
        lpartner[i] = p >= 0 && comp_of[p] == c ? local[p] : -1;
      }
    rc = orc_solve_component_stitch(size, lm, ledges, k, budget,
                                    (flags & ORC_STITCH) ? lpartner : NULL, lcolors,
                                    &r->status, &r->nodes, &r->trace_hash, &r->depth_at_stop);
    if (rc) goto out;
    const int marked = r->status != ORC_FEASIBLE && (flags & (ORC_MARK | ORC_MINIMIZE));
    if (marked) {
      rc = orc_mark_conflicts(size, lm, ledges, k, lcolors);
      if (rc) goto out;
    }
    r->min_nodes = 0;
    if ((flags & ORC_MINIMIZE) && size <= ORC_MINIMIZE_MAX_N) {
      int64_t bn = 0;
      int32_t stopped = 0, cost = 0;
      rc = orc_minimize_component(size, lm, ledges, k, lpartner, min_budget, lcolors, &bn,
                                  &stopped, &cost);
      if (rc) goto out;
      r->min_nodes = (int32_t)(stopped ? -bn : bn);
    }
    for (int32_t i = 0; i < size; ++i) colors[nodes[i]] = lcolors[i];
    r->stitches = 0;
    for (int32_t i = 0; i < size; ++i) {
      const int32_t x = nodes[i], p = partner[x];
      if (p > x && comp_of[p] == c && colors[p] != colors[x]) r->stitches++;
    }
    if (r->status != ORC_FEASIBLE && !marked) r->stitches = -1;
    r->conflicts = 0;
    for (int64_t e = 0; e < lm; ++e)
      if (lcolors[ledges[2 * e]] >= 0 && lcolors[ledges[2 * e]] == lcolors[ledges[2 * e + 1]])
        r->conflicts++;
  }

  /* recovery, reverse removal order */
  for (int32_t i = nrem - 1; i >= 0; --i) {
    const int32_t x = removal[i];
    uint64_t used = 0;
    for (int64_t t = ap[x]; t < ap[x + 1]; ++t)
      if (colors[adj[t]] >= 0) used |= 1ULL << colors[adj[t]];
    const int32_t p = partner[x];
    if (p >= 0 && colors[p] >= 0 && !((used >> colors[p]) & 1)) {
      colors[x] = colors[p];
    } else {
      int32_t c = 0;
      while (c < k && ((used >> c) & 1)) ++c;
      if (c == k) { rc = -6; goto out; }   /* impossible: degree < k at removal */
      colors[x] = (int8_t)c;
    }
  }

  /* Eq. 1 tallies: stitches = stitch pairs colored differently, conflicts =
   * conflict pairs colored alike (uncolored nodes take part in neither) */
  {
    int64_t st = 0, cn = 0, un = 0;
    for (int32_t v = 0; v < n; ++v) {
      if (colors[v] < 0) ++un;
      if (partner[v] > v && colors[v] >= 0 && colors[partner[v]] >= 0 &&
          colors[v] != colors[partner[v]])
        ++st;
    }
    for (int64_t i = 0; i < num_ce; ++i) {
      const int8_t a = colors[ce[2 * i]], b = colors[ce[2 * i + 1]];
      if (a >= 0 && a == b) ++cn;
    }
    if (total_stitches) *total_stitches = st;
    if (total_conflicts) *total_conflicts = cn;
    if (total_uncolored) *total_uncolored = un;
  }
  *num_comps = nc;
  *comps = cs;
  cs = NULL;
out:
  free(ap); free(adj); free(partner); free(removal); free(bfs); free(comp_ptr);
  free(local); free(ledges); free(lcolors); free(lpartner); free(cs);
  return rc;
}

/* ------------------------------------------------------------------------
 * Many components on several host threads (timing only; per component the
 * result is orc_solve_component's).  The workers live for the whole call
 * and repeat the set `passes` times: task t is component t % count of pass
 * t / count, claimed in chunks from one atomic counter.  Pass 0 writes the
 * outputs; later passes solve into each worker's own scratch, so no two
 * threads write the same output.
 * ---------------------------------------------------------------------- */

enum { ORC_POOL_CHUNK = 4 };

typedef struct {
  int32_t count, k, passes, max_n;
  int64_t budget;
  const int32_t* sizes;
  const int64_t* edge_off;
  const int64_t* node_off;
  const int32_t* edges;
  int8_t* colors;
  int32_t* status;
  int64_t* nodes;
  uint64_t* hash;
  _Atomic int64_t next;        /* next task to claim */
  _Atomic int64_t total_nodes; /* search nodes over every pass */
  _Atomic int32_t err;
} orc_pool;

static void* pool_worker(void* arg) {
  orc_pool* p = (orc_pool*)arg;
  const int64_t tasks = (int64_t)p->count * p->passes;
  int8_t* scratch = (int8_t*)malloc((size_t)(p->max_n > 0 ? p->max_n : 1));
  if (!scratch) { atomic_store(&p->err, -2); return NULL; }
  int64_t mine = 0;
  for (;;) {
    const int64_t t0 = atomic_fetch_add(&p->next, (int64_t)ORC_POOL_CHUNK);
    if (t0 >= tasks) break;
    const int64_t t1 = t0 + ORC_POOL_CHUNK < tasks ? t0 + ORC_POOL_CHUNK : tasks;
    for (int64_t t = t0; t < t1; ++t) {
      const int32_t i = (int32_t)(t % p->count);
      const int first = t < p->count;
      const int64_t m = p->edge_off[i + 1] - p->edge_off[i];
      int32_t st;
      int64_t nd;
      uint64_t h;
      int32_t rc = orc_solve_component(p->sizes[i], m, p->edges + 2 * p->edge_off[i], p->k,
                                       p->budget, first ? p->colors + p->node_off[i] : scratch,
                                       &st, &nd, &h, NULL);
      if (rc) atomic_store(&p->err, rc);
      if (first) {
        p->status[i] = st;
        p->nodes[i] = nd;
        p->hash[i] = h;
      }
      mine += nd;
    }
  }
  atomic_fetch_add(&p->total_nodes, mine);
  free(scratch);
  return NULL;
}

int32_t orc_solve_many(int32_t count, const int32_t* sizes,
                       const int64_t* edge_counts, const int32_t* edges,
                       int32_t k, int64_t budget, int32_t threads, int32_t passes,
                       int8_t* colors, int32_t* status, int64_t* nodes,
                       uint64_t* trace_hash, int64_t* total_nodes) {
  if (count < 0 || threads < 1 || passes < 1) return -1;
  if (total_nodes) *total_nodes = 0;
  if (count == 0) return 0;
  int64_t* eo = (int64_t*)malloc(sizeof(int64_t) * ((size_t)count + 1));
  int64_t* no = (int64_t*)malloc(sizeof(int64_t) * ((size_t)count + 1));
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)threads);
  if (!eo || !no || !th) { free(eo); free(no); free(th); return -2; }
  eo[0] = 0; no[0] = 0;
  int32_t max_n = 0;
  for (int32_t i = 0; i < count; ++i) {
    if (sizes[i] < 0 || edge_counts[i] < 0) { free(eo); free(no); free(th); return -1; }
    eo[i + 1] = eo[i] + edge_counts[i];
    no[i + 1] = no[i] + sizes[i];
    if (sizes[i] > max_n) max_n = sizes[i];
  }
  orc_pool p;
  p.count = count; p.k = k; p.passes = passes; p.max_n = max_n; p.budget = budget;
  p.sizes = sizes; p.edge_off = eo; p.node_off = no; p.edges = edges;
  p.colors = colors; p.status = status; p.nodes = nodes; p.hash = trace_hash;
  atomic_init(&p.next, 0);
  atomic_init(&p.total_nodes, 0);
  atomic_init(&p.err, 0);
  if (threads == 1) {
    /* one thread: the caller's own (keeps any CPU affinity it has set) */
    pool_worker(&p);
  } else {
    int32_t started = 0;
    for (int32_t t = 0; t < threads; ++t)
      if (pthread_create(&th[started], NULL, pool_worker, &p) == 0) ++started;
    if (started == 0) pool_worker(&p);
    for (int32_t t = 0; t < started; ++t) pthread_join(th[t], NULL);
  }
  if (total_nodes) *total_nodes = atomic_load(&p.total_nodes);
  free(eo); free(no); free(th);
  return atomic_load(&p.err);
}
