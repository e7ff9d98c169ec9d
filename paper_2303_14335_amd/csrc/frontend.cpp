// frontend.cpp - host front-end of the decomposer: layout graph from
// rectangles, graph validation, simplification, sub-graph split, recovery
// and the Eq. 1 tallies (Sec. 2.1, 2.2 of the paper).
#include <algorithm>
#include <cstdlib>
#include <thread>

#include "internal.h"

namespace mpld {

static thread_local std::string g_last_error;

void set_last_error(const std::string& s) { g_last_error = s; }
const char* last_error_cstr() { return g_last_error.c_str(); }

[[noreturn]] void fail(int32_t code, const std::string& what) { throw Error{code, what}; }

int host_threads() {
  static int t = [] {
    if (const char* e = std::getenv("MPLD_HOST_THREADS")) {
      int v = std::atoi(e);
      if (v > 0) return v;
    }
    unsigned h = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(h ? h : 1u, 16u));
  }();
  return t;
}

Graph make_graph(const mpld_graph& in) {
  if (in.num_nodes < 0 || in.num_ce < 0 || in.num_se < 0)
    fail(MPLD_E_INVALID, "negative graph size");
  if ((in.num_ce > 0 && !in.ce) || (in.num_se > 0 && !in.se))
    fail(MPLD_E_INVALID, "null edge array");
  Graph g;
  const int32_t n = in.num_nodes;
  g.n = n;
  g.num_ce = in.num_ce;
  g.ptr.assign((size_t)n + 1, 0);
  for (int64_t i = 0; i < in.num_ce; ++i) {
    const int32_t u = in.ce[2 * i], v = in.ce[2 * i + 1];
    if (u < 0 || v < 0 || u >= n || v >= n)
      fail(MPLD_E_INVALID, "conflict edge " + std::to_string(i) + " has a node id out of range");
    if (u == v) fail(MPLD_E_INVALID, "conflict edge " + std::to_string(i) + " is a self loop");
    ++g.ptr[u + 1];
    ++g.ptr[v + 1];
  }
  for (int32_t v = 0; v < n; ++v) g.ptr[v + 1] += g.ptr[v];
  g.adj.resize((size_t)g.ptr[n]);
  {
    std::vector<int64_t> fill(g.ptr.begin(), g.ptr.end() - 1);
    for (int64_t i = 0; i < in.num_ce; ++i) {
      const int32_t u = in.ce[2 * i], v = in.ce[2 * i + 1];
      g.adj[fill[u]++] = v;
      g.adj[fill[v]++] = u;
    }
  }
  for (int32_t v = 0; v < n; ++v) {
    auto b = g.adj.begin() + g.ptr[v], e = g.adj.begin() + g.ptr[v + 1];
    std::sort(b, e);
    if (std::adjacent_find(b, e) != e)
      fail(MPLD_E_INVALID, "duplicate conflict edge at node " + std::to_string(v));
  }
  g.partner.assign((size_t)n, -1);
  for (int64_t i = 0; i < in.num_se; ++i) {
    const int32_t u = in.se[2 * i], v = in.se[2 * i + 1];
    if (u < 0 || v < 0 || u >= n || v >= n || u == v)
      fail(MPLD_E_INVALID, "stitch edge " + std::to_string(i) + " is out of range or a loop");
    if (g.partner[u] >= 0 || g.partner[v] >= 0)
      fail(MPLD_E_INVALID, "a node is in two stitch pairs (stitch edge " + std::to_string(i) + ")");
    g.partner[u] = v;
    g.partner[v] = u;
    if (std::binary_search(g.adj.begin() + g.ptr[u], g.adj.begin() + g.ptr[u + 1], v))
      fail(MPLD_E_INVALID, "pair is both stitch and conflict edge (stitch edge " + std::to_string(i) + ")");
  }
  return g;
}

Split simplify_and_split(const Graph& g, int32_t k, bool simplify) {
  const int32_t n = g.n;
  Split s;
  std::vector<int32_t> deg((size_t)n);
  std::vector<uint8_t> state((size_t)n, 0);  // bit0 queued, bit1 removed
  for (int32_t v = 0; v < n; ++v) deg[v] = (int32_t)(g.ptr[v + 1] - g.ptr[v]);
  s.removal.reserve((size_t)n);
  if (simplify) {
    // FIFO peeling: the removal vector doubles as the queue.
    for (int32_t v = 0; v < n; ++v)
      if (deg[v] < k) { s.removal.push_back(v); state[v] = 1; }
    for (size_t head = 0; head < s.removal.size(); ++head) {
      const int32_t u = s.removal[head];
      state[u] |= 2;
      for (int64_t t = g.ptr[u]; t < g.ptr[u + 1]; ++t) {
        const int32_t w = g.adj[t];
        if (state[w] & 2) continue;
        if (--deg[w] < k && !(state[w] & 1)) { state[w] |= 1; s.removal.push_back(w); }
      }
    }
  }
  s.comp_of.assign((size_t)n, -1);
  s.local.assign((size_t)n, -1);
  s.order.reserve((size_t)n - s.removal.size());
  s.comp_ptr.push_back(0);
  for (int32_t root = 0; root < n; ++root) {
    if ((state[root] & 2) || s.comp_of[root] >= 0) continue;
    const int32_t c = (int32_t)s.comp_ptr.size() - 1;
    const size_t base = s.order.size();
    s.order.push_back(root);
    s.comp_of[root] = c;
    for (size_t h = base; h < s.order.size(); ++h) {
      const int32_t x = s.order[h];
      s.local[x] = (int32_t)(h - base);
      for (int64_t t = g.ptr[x]; t < g.ptr[x + 1]; ++t) {
        const int32_t w = g.adj[t];
        if ((state[w] & 2) || s.comp_of[w] >= 0) continue;
        s.comp_of[w] = c;
        s.order.push_back(w);
      }
    }
    s.comp_ptr.push_back((int32_t)s.order.size());
  }
  return s;
}

void local_edges(const Graph& g, const Split& s, int32_t c, std::vector<int32_t>& out) {
  out.clear();
  for (int32_t p = s.comp_ptr[c]; p < s.comp_ptr[c + 1]; ++p) {
    const int32_t x = s.order[p];
    const int32_t i = p - s.comp_ptr[c];
    for (int64_t t = g.ptr[x]; t < g.ptr[x + 1]; ++t) {
      const int32_t j = s.local[g.adj[t]];
      if (s.comp_of[g.adj[t]] == c && j > i) {
        out.push_back(i);
        out.push_back(j);
      }
    }
  }
  // Neighbour order in the global numbering is not local order: sort pairs.
  const size_t m = out.size() / 2;
  std::vector<uint64_t> key(m);
  for (size_t e = 0; e < m; ++e) key[e] = ((uint64_t)(uint32_t)out[2 * e] << 32) | (uint32_t)out[2 * e + 1];
  std::sort(key.begin(), key.end());
  for (size_t e = 0; e < m; ++e) {
    out[2 * e] = (int32_t)(key[e] >> 32);
    out[2 * e + 1] = (int32_t)(key[e] & 0xffffffffu);
  }
}

void recover(const Graph& g, const Split& s, int32_t k, std::vector<int8_t>& colors) {
  for (size_t i = s.removal.size(); i-- > 0;) {
    const int32_t x = s.removal[i];
    uint32_t used = 0;
    for (int64_t t = g.ptr[x]; t < g.ptr[x + 1]; ++t) {
      const int8_t c = colors[g.adj[t]];
      if (c >= 0) used |= 1u << c;
    }
    const int32_t p = g.partner[x];
    if (p >= 0 && colors[p] >= 0 && !((used >> colors[p]) & 1u)) {
      colors[x] = colors[p];
    } else {
      const uint32_t free_mask = ~used & ((1u << k) - 1u);
      if (!free_mask) fail(MPLD_E_INTERNAL, "recovery found no free color");
      colors[x] = (int8_t)__builtin_ctz(free_mask);
    }
  }
}

void tallies(const Graph& g, const std::vector<int8_t>& colors, int64_t* stitches,
             int64_t* conflicts, int64_t* uncolored) {
  int64_t st = 0, cn = 0, un = 0;
  const int8_t* col = colors.data();
  const int32_t* adj = g.adj.data();
  for (int32_t v = 0; v < g.n; ++v) {
    const int8_t cv = col[v];
    if (cv < 0) { ++un; continue; }
    const int32_t p = g.partner[v];
    if (p > v) st += col[p] >= 0 && col[p] != cv;
    int64_t c = 0;   // branch-free: the pair test is unpredictable
    for (int64_t t = g.ptr[v], e = g.ptr[v + 1]; t < e; ++t) {
      const int32_t w = adj[t];
      c += (w > v) & (col[w] == cv);
    }
    cn += c;
  }
  *stitches = st;
  *conflicts = cn;
  *uncolored = un;
}

// --------------------------------------------------------------------------
// Layout graph from rectangles.  Nodes are binned by lower-left corner into
// square cells of side S = (largest extent) + dmin; two features closer than
// dmin have lower-left corners less than S apart on each axis, so only the
// 3x3 cells around a node hold its possible conflict partners.

void prepare_layout(const mpld_rect* rects, int32_t n, int32_t dmin, int32_t split_len,
                    LayoutPrep& lp) {
  if (n < 0 || dmin < 0 || split_len < 0) fail(MPLD_E_INVALID, "negative size, dmin or split length");
  if (n > 0 && !rects) fail(MPLD_E_INVALID, "null rectangle array");
  std::vector<mpld_rect>& nd = lp.nd;
  std::vector<int32_t>& partner = lp.partner;
  nd.clear();
  partner.clear();
  lp.se.clear();
  nd.reserve((size_t)n * (split_len > 0 ? 2 : 1));
  for (int32_t i = 0; i < n; ++i) {
    const mpld_rect r = rects[i];
    if (r.x1 < r.x0 || r.y1 < r.y0) fail(MPLD_E_INVALID, "rectangle " + std::to_string(i) + " has x1 < x0 or y1 < y0");
    const int32_t w = r.x1 - r.x0, h = r.y1 - r.y0, len = std::max(w, h);
    if (split_len > 0 && len > split_len) {
      mpld_rect a = r, b = r;
      if (w >= h) { a.x1 = r.x0 + len / 2; b.x0 = a.x1; }
      else { a.y1 = r.y0 + len / 2; b.y0 = a.y1; }
      const int32_t id = (int32_t)nd.size();
      lp.se.push_back(id);
      lp.se.push_back(id + 1);
      nd.push_back(a);
      nd.push_back(b);
      partner.push_back(id + 1);
      partner.push_back(id);
    } else {
      nd.push_back(r);
      partner.push_back(-1);
    }
  }
  const int32_t nn = (int32_t)nd.size();
  lp.minx = lp.miny = 0;
  lp.cell = 1;
  lp.gx = lp.gy = 1;
  if (nn == 0) return;
  int64_t minx = INT64_MAX, miny = INT64_MAX, maxx = INT64_MIN, maxy = INT64_MIN, ext = 1;
  for (const auto& r : nd) {
    minx = std::min<int64_t>(minx, r.x0);
    miny = std::min<int64_t>(miny, r.y0);
    maxx = std::max<int64_t>(maxx, r.x0);
    maxy = std::max<int64_t>(maxy, r.y0);
    ext = std::max<int64_t>(ext, std::max<int64_t>((int64_t)r.x1 - r.x0, (int64_t)r.y1 - r.y0));
  }
  // cells of side > largest extent + d_min: every conflict pair has its
  // lower-left corners in the same or adjacent cells
  int64_t cell = ext + dmin + 1;
  int64_t gx = (maxx - minx) / cell + 1, gy = (maxy - miny) / cell + 1;
  while (gx * gy > 4 * (int64_t)nn + 1024) {   // keep the grid O(n)
    cell *= 2;
    gx = (maxx - minx) / cell + 1;
    gy = (maxy - miny) / cell + 1;
  }
  lp.minx = minx;
  lp.miny = miny;
  lp.cell = cell;
  lp.gx = gx;
  lp.gy = gy;
}

void build_layout_graph(const mpld_rect* rects, int32_t n, int32_t dmin,
                        int32_t split_len, OwnedGraph& out, int threads) {
  LayoutPrep lp;
  prepare_layout(rects, n, dmin, split_len, lp);
  const std::vector<mpld_rect>& nd = lp.nd;
  const std::vector<int32_t>& partner = lp.partner;
  out.se = lp.se;
  const int32_t nn = (int32_t)nd.size();
  out.num_nodes = nn;
  out.ce.clear();
  if (nn == 0) return;
  const int64_t minx = lp.minx, miny = lp.miny, cell = lp.cell, gx = lp.gx, gy = lp.gy;
  // counting sort of the nodes by cell (ascending id within a cell), with a
  // copy of their boxes in that order so that the 3x3 neighbourhood scans
  // below read contiguous memory
  std::vector<int32_t> cell_of((size_t)nn), start((size_t)(gx * gy + 1), 0), sorted((size_t)nn);
  for (int32_t i = 0; i < nn; ++i) {
    const int64_t cx = (nd[i].x0 - minx) / cell, cy = (nd[i].y0 - miny) / cell;
    cell_of[i] = (int32_t)(cy * gx + cx);
    ++start[cell_of[i] + 1];
  }
  for (int64_t c = 0; c < gx * gy; ++c) start[c + 1] += start[c];
  {
    std::vector<int32_t> fill(start.begin(), start.end() - 1);
    for (int32_t i = 0; i < nn; ++i) sorted[fill[cell_of[i]]++] = i;
  }
  std::vector<mpld_rect> box((size_t)nn);
  std::vector<int32_t> mate((size_t)nn);   // stitch partner of the node at sorted position p
  for (int32_t p = 0; p < nn; ++p) {
    box[p] = nd[sorted[p]];
    mate[p] = partner[sorted[p]];
  }
  const int64_t d2 = (int64_t)dmin * dmin;
  const int64_t ncell = gx * gy;
  const int T = std::min(threads > 0 ? threads : host_threads(), std::max(1, nn / 4096));
  // Thread t scans cell rows [gy*t/T, gy*(t+1)/T).  Every unordered pair is
  // tested once: a node against the later nodes of its own cell and every
  // node of the four forward neighbour cells (right; below-left, below,
  // below-right).  Pairs are emitted as (min id, max id).
  std::vector<std::vector<uint64_t>> part((size_t)T);
  auto work = [&](int t) {
    const int64_t ylo = gy * t / T, yhi = gy * (t + 1) / T;
    std::vector<uint64_t>& e = part[t];
    auto test = [&](int32_t pa, const mpld_rect& ra, int32_t pb) {
      const mpld_rect& rb = box[pb];
      const int64_t dx = std::max<int64_t>({0, (int64_t)rb.x0 - ra.x1, (int64_t)ra.x0 - rb.x1});
      const int64_t dy = std::max<int64_t>({0, (int64_t)rb.y0 - ra.y1, (int64_t)ra.y0 - rb.y1});
      if (dx * dx + dy * dy < d2) {
        const int32_t a = sorted[pa], b = sorted[pb];
        if (mate[pa] == b) return;   // the two halves of a split feature
        const uint32_t lo = (uint32_t)std::min(a, b), hi = (uint32_t)std::max(a, b);
        e.push_back(((uint64_t)lo << 32) | hi);
      }
    };
    for (int64_t cy = ylo; cy < yhi; ++cy)
      for (int64_t cx = 0; cx < gx; ++cx) {
        const int64_t c = cy * gx + cx;
        for (int32_t pa = start[c]; pa < start[c + 1]; ++pa) {
          const mpld_rect ra = box[pa];
          for (int32_t pb = pa + 1; pb < start[c + 1]; ++pb) test(pa, ra, pb);
          if (cx + 1 < gx)
            for (int32_t pb = start[c + 1]; pb < start[c + 2]; ++pb) test(pa, ra, pb);
          if (cy + 1 < gy) {
            const int64_t c0 = (cy + 1) * gx + std::max<int64_t>(0, cx - 1);
            const int64_t c1 = (cy + 1) * gx + std::min(gx - 1, cx + 1);
            for (int32_t pb = start[c0]; pb < start[c1 + 1]; ++pb) test(pa, ra, pb);
          }
        }
      }
  };
  (void)ncell;
  if (T == 1) {
    work(0);
  } else {
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t) th.emplace_back(work, t);
    for (auto& x : th) x.join();
  }
  // pairs sorted by (a, b): counting sort by a, then each a's few b ascending
  size_t total = 0;
  for (auto& q : part) total += q.size();
  std::vector<int64_t> off((size_t)nn + 1, 0);
  for (auto& q : part)
    for (uint64_t x : q) ++off[(x >> 32) + 1];
  for (int32_t i = 0; i < nn; ++i) off[i + 1] += off[i];
  std::vector<int32_t> nb(total);
  {
    std::vector<int64_t> fill(off.begin(), off.end() - 1);
    for (auto& q : part)
      for (uint64_t x : q) nb[(size_t)fill[x >> 32]++] = (int32_t)(uint32_t)x;
  }
  out.ce.resize(2 * total);
  for (int32_t a = 0; a < nn; ++a) {
    std::sort(nb.begin() + off[a], nb.begin() + off[a + 1]);
    for (int64_t j = off[a]; j < off[a + 1]; ++j) {
      out.ce[2 * j] = a;
      out.ce[2 * j + 1] = nb[(size_t)j];
    }
  }
}

}  // namespace mpld
