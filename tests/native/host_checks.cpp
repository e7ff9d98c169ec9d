// host_checks.cpp - a driver for sanitizer builds (ASan + UBSan, TSan) of
// the library's host-only code: the layout-graph builder (several scan
// threads), graph validation, simplification and sub-graph split, local
// edge lists, recovery and the Eq. 1 tallies (csrc/frontend.cpp), and the
// first-fit range allocator of the server's admission (csrc/range_alloc.h).
// Built with g++ from those sources alone (no HIP); every check prints a
// line and the driver exits non-zero on the first failure.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "internal.h"
#include "layoutgen.h"
#include "range_alloc.h"

using namespace mpld;

static int g_fail = 0;
#define CHECK(cond, ...)                                       \
  do {                                                         \
    if (!(cond)) {                                             \
      std::fprintf(stderr, "FAILED %s:%d: ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);                       \
      std::fprintf(stderr, "\n");                              \
      g_fail = 1;                                              \
      return;                                                  \
    }                                                          \
  } while (0)

static std::vector<mpld_rect> layout(int32_t n, int32_t side, uint64_t seed) {
  lg_params p{n, side, 20, 40, 200, 1000};
  std::vector<lg_rect> r((size_t)std::max(n, 1));
  int32_t placed = 0, skipped = 0;
  if (lg_generate(&p, seed, r.data(), &placed, &skipped) != 0) std::abort();
  std::vector<mpld_rect> out((size_t)placed);
  for (int32_t i = 0; i < placed; ++i) out[i] = {r[i].x0, r[i].y0, r[i].x1, r[i].y1};
  return out;
}

// Conflict pairs by testing every pair of nodes (after the same split).
static std::vector<int32_t> brute_pairs(const LayoutPrep& lp, int32_t dmin) {
  std::vector<int32_t> out;
  const int32_t n = (int32_t)lp.nd.size();
  for (int32_t i = 0; i < n; ++i)
    for (int32_t j = i + 1; j < n; ++j) {
      if (lp.partner[i] == j) continue;
      const mpld_rect &a = lp.nd[i], &b = lp.nd[j];
      const int64_t gx = std::max<int64_t>({0, (int64_t)b.x0 - a.x1, (int64_t)a.x0 - b.x1});
      const int64_t gy = std::max<int64_t>({0, (int64_t)b.y0 - a.y1, (int64_t)a.y0 - b.y1});
      if (gx * gx + gy * gy < (int64_t)dmin * dmin) {
        out.push_back(i);
        out.push_back(j);
      }
    }
  return out;
}

static void check_graph_builder() {
  for (int trial = 0; trial < 6; ++trial) {
    const int32_t n = 400 + 300 * trial, split = trial % 2 ? 100 : 0, dmin = 80 + 20 * trial;
    const std::vector<mpld_rect> rects = layout(n, 2500 + 400 * trial, 11 + trial);
    LayoutPrep lp;
    prepare_layout(rects.data(), (int32_t)rects.size(), dmin, split, lp);
    const std::vector<int32_t> want = brute_pairs(lp, dmin);
    for (int threads : {1, 3, 8}) {
      OwnedGraph g;
      build_layout_graph(rects.data(), (int32_t)rects.size(), dmin, split, g, threads);
      CHECK(g.num_nodes == (int32_t)lp.nd.size(), "node count");
      CHECK(g.ce == want, "trial %d threads %d: %zu pairs against %zu", trial, threads,
            g.ce.size() / 2, want.size() / 2);
      CHECK(g.se == lp.se, "stitch pairs");
    }
  }
  std::printf("graph builder: all-pairs equal at 1, 3 and 8 threads\n");
}

static void check_split_and_recovery() {
  for (int32_t k = 2; k <= 4; ++k) {
    const std::vector<mpld_rect> rects = layout(3000, 6000, 100 + k);
    OwnedGraph og;
    build_layout_graph(rects.data(), (int32_t)rects.size(), 120, 120, og, 4);
    mpld_graph view{og.num_nodes, 0, (int64_t)og.ce.size() / 2, og.ce.data(),
                    (int64_t)og.se.size() / 2, og.se.data()};
    const Graph g = make_graph(view);
    const Split s = simplify_and_split(g, k, true);
    // every core node keeps at least k core neighbours; components are
    // connected over core edges and listed with their smallest id first
    int32_t core = 0;
    for (int32_t v = 0; v < g.n; ++v) {
      if (s.comp_of[v] < 0) continue;
      ++core;
      int32_t d = 0;
      for (int64_t t = g.ptr[v]; t < g.ptr[v + 1]; ++t) d += s.comp_of[g.adj[t]] >= 0;
      CHECK(d >= k, "core node %d has %d core neighbours (k = %d)", v, d, k);
    }
    CHECK((int32_t)s.removal.size() + core == g.n, "removed + core = n");
    const int32_t nc = (int32_t)s.comp_ptr.size() - 1;
    std::vector<int32_t> pairs;
    for (int32_t c = 0; c < nc; ++c) {
      const int32_t first = s.order[s.comp_ptr[c]];
      for (int32_t p = s.comp_ptr[c]; p < s.comp_ptr[c + 1]; ++p) {
        CHECK(s.comp_of[s.order[p]] == c, "component id");
        CHECK(s.order[p] >= first, "smallest id first");
      }
      local_edges(g, s, c, pairs);
      const int32_t size = s.comp_ptr[c + 1] - s.comp_ptr[c];
      for (size_t e = 0; e < pairs.size(); e += 2)
        CHECK(pairs[e] < pairs[e + 1] && pairs[e + 1] < size, "local pair");
    }
    // greedy colors for the core, then recovery: no removed node may end in
    // a conflict
    std::vector<int8_t> colors((size_t)g.n, -1);
    for (int32_t p = 0; p < (int32_t)s.order.size(); ++p) colors[s.order[p]] = (int8_t)(p % k);
    recover(g, s, k, colors);
    for (int32_t v : s.removal) {
      CHECK(colors[v] >= 0 && colors[v] < k, "recovered color");
      for (int64_t t = g.ptr[v]; t < g.ptr[v + 1]; ++t)
        CHECK(colors[g.adj[t]] != colors[v], "recovered node %d conflicts", v);
    }
    int64_t st = 0, cn = 0, un = 0;
    tallies(g, colors, &st, &cn, &un);
    CHECK(un == 0 && st >= 0 && cn >= 0, "tallies");
  }
  std::printf("split and recovery: invariants hold for k = 2..4\n");
}

static void check_validation() {
  const int32_t bad_ce[][2] = {{0, 0}, {0, 5}, {-1, 2}};
  for (const auto& e : bad_ce) {
    mpld_graph g{4, 0, 1, &e[0], 0, nullptr};
    bool thrown = false;
    try {
      (void)make_graph(g);
    } catch (const Error& err) {
      thrown = err.code == MPLD_E_INVALID;
    }
    CHECK(thrown, "bad edge (%d, %d) accepted", e[0], e[1]);
  }
  const int32_t dup[] = {0, 1, 1, 0};
  mpld_graph g{3, 0, 2, dup, 0, nullptr};
  bool thrown = false;
  try {
    (void)make_graph(g);
  } catch (const Error& err) {
    thrown = err.code == MPLD_E_INVALID;
  }
  CHECK(thrown, "duplicate accepted");
  std::printf("validation: bad graphs rejected\n");
}

static void check_range_alloc() {
  std::mt19937_64 rng(7);
  for (int64_t cap : {1, 4096, 1 << 20}) {
    RangeAlloc a;
    a.reset(cap);
    std::vector<std::pair<int64_t, int64_t>> live;
    std::vector<uint8_t> used((size_t)cap, 0);
    for (int step = 0; step < 20000; ++step) {
      if (live.empty() || rng() % 3 != 0) {
        const int64_t len = 1 + (int64_t)(rng() % (uint64_t)std::max<int64_t>(1, cap / 16));
        const int64_t align = int64_t(1) << (rng() % 9);
        const int64_t off = a.alloc(len, align);
        if (off < 0) continue;
        CHECK(off % align == 0 && off + len <= cap, "range in bounds and aligned");
        for (int64_t i = off; i < off + len; ++i) {
          CHECK(!used[(size_t)i], "overlap at %lld", (long long)i);
          used[(size_t)i] = 1;
        }
        live.push_back({off, len});
      } else {
        const size_t i = (size_t)(rng() % live.size());
        a.release(live[i].first, live[i].second);
        for (int64_t j = live[i].first; j < live[i].first + live[i].second; ++j) used[(size_t)j] = 0;
        live[i] = live.back();
        live.pop_back();
      }
      int64_t sum = 0;
      for (const auto& r : live) sum += r.second;
      CHECK(a.used() == sum, "used() bookkeeping");
    }
    for (const auto& r : live) a.release(r.first, r.second);
    CHECK(a.used() == 0 && a.alloc(cap, 1) == 0, "empty allocator is one free range");
  }
  std::printf("range allocator: no overlap, exact bookkeeping, full merge\n");
}

int main() {
  check_graph_builder();
  if (!g_fail) check_split_and_recovery();
  if (!g_fail) check_validation();
  if (!g_fail) check_range_alloc();
  if (g_fail) return 1;
  std::printf("host checks passed\n");
  return 0;
}
