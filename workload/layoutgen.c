/*
 * layoutgen.c - seeded synthetic layout and request-trace generator
 * (inputs only; the definitions are stated in layoutgen.h).
 */
#include "layoutgen.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

uint64_t lg_u64(uint64_t* state) {
  /* SplitMix64: golden-ratio increment, then the variant-13 mix. */
  uint64_t z = (*state += 0x9e3779b97f4a7c15ULL);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

static uint32_t draw32(uint64_t* s) { return (uint32_t)(lg_u64(s) >> 32); }

/* Uniform integer in [0, range) for 1 <= range <= 2^32-1 (Lemire 2019). */
static uint32_t bounded(uint64_t* s, uint32_t range) {
  uint64_t m = (uint64_t)draw32(s) * range;
  uint32_t low = (uint32_t)m;
  if (low < range) {
    uint32_t threshold = (uint32_t)(0u - range) % range;
    while (low < threshold) {
      m = (uint64_t)draw32(s) * range;
      low = (uint32_t)m;
    }
  }
  return (uint32_t)(m >> 32);
}

static int32_t uniform_int(uint64_t* s, int32_t lo, int32_t hi) {
  return lo + (int32_t)bounded(s, (uint32_t)(hi - lo) + 1u);
}

static double uniform_real(uint64_t* s) {
  return (double)(lg_u64(s) >> 11) * (1.0 / 9007199254740992.0);
}

/* closed boxes intersect or touch */
static int touches(const lg_rect* a, const lg_rect* b) {
  return a->x0 <= b->x1 && b->x0 <= a->x1 && a->y0 <= b->y1 && b->y0 <= a->y1;
}

int32_t lg_generate(const lg_params* p, uint64_t seed, lg_rect* out,
                    int32_t* placed, int32_t* skipped) {
  if (!p || !placed || !skipped) return -1;
  if (p->n < 0 || p->side < 1 || p->width < 0 || p->len_min < 0 ||
      p->len_min > p->len_max || p->max_attempts < 1)
    return -1;
  if (p->n > 0 && !out) return -1;
  *placed = 0;
  *skipped = 0;
  if (p->n == 0) return 0;

  /* Bucket grid over [0, side + maxlen]: every placed box is linked into
   * each cell it overlaps, so two touching boxes always share a cell. */
  const int64_t reach = (int64_t)p->side + (p->len_max > p->width ? p->len_max : p->width);
  int32_t cell = 256;
  while (cell <= p->len_max || cell <= p->width) cell *= 2;
  const int64_t g = reach / cell + 1;
  if (g > 65536) return -1;
  int32_t* head = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g * g));
  /* each box overlaps at most 2 cells per axis (cell > box extent) */
  int32_t* ent_box = (int32_t*)malloc(sizeof(int32_t) * 4 * (size_t)p->n);
  int32_t* ent_next = (int32_t*)malloc(sizeof(int32_t) * 4 * (size_t)p->n);
  if (!head || !ent_box || !ent_next) {
    free(head); free(ent_box); free(ent_next);
    return -2;
  }
  for (int64_t i = 0; i < g * g; ++i) head[i] = -1;
  int32_t nent = 0;

  uint64_t st = seed;
  int32_t np = 0, ns = 0;
  for (int32_t i = 0; i < p->n; ++i) {
    int ok = 0;
    lg_rect r;
    for (int32_t a = 0; a < p->max_attempts && !ok; ++a) {
      const int vertical = (int)(lg_u64(&st) >> 63);
      const int32_t len = uniform_int(&st, p->len_min, p->len_max);
      const int32_t x = uniform_int(&st, 0, p->side - 1);
      const int32_t y = uniform_int(&st, 0, p->side - 1);
      r.x0 = x;
      r.y0 = y;
      r.x1 = x + (vertical ? p->width : len);
      r.y1 = y + (vertical ? len : p->width);
      ok = 1;
      for (int64_t cy = r.y0 / cell; cy <= r.y1 / cell && ok; ++cy)
        for (int64_t cx = r.x0 / cell; cx <= r.x1 / cell && ok; ++cx)
          for (int32_t e = head[cy * g + cx]; e >= 0; e = ent_next[e])
            if (touches(&r, &out[ent_box[e]])) { ok = 0; break; }
    }
    if (!ok) { ++ns; continue; }
    out[np] = r;
    for (int64_t cy = r.y0 / cell; cy <= r.y1 / cell; ++cy)
      for (int64_t cx = r.x0 / cell; cx <= r.x1 / cell; ++cx) {
        ent_box[nent] = np;
        ent_next[nent] = head[cy * g + cx];
        head[cy * g + cx] = nent++;
      }
    ++np;
  }
  free(head); free(ent_box); free(ent_next);
  *placed = np;
  *skipped = ns;
  return 0;
}

int32_t lg_request_trace(uint64_t seed, int32_t count, double rate,
                         int32_t n_min, int32_t n_max, int32_t base_side,
                         int32_t base_n, double* arrival_s, int32_t* n_rects,
                         int32_t* side_nm, uint64_t* layout_seed) {
  if (count < 0 || !(rate > 0.0) || n_min < 1 || n_max < n_min ||
      base_side < 1 || base_n < 1)
    return -1;
  if (count > 0 && (!arrival_s || !n_rects || !side_nm || !layout_seed)) return -1;
  uint64_t st = seed;
  double t = 0.0;
  const double lmin = log((double)n_min), lspan = log((double)n_max / (double)n_min);
  for (int32_t i = 0; i < count; ++i) {
    t += -log(1.0 - uniform_real(&st)) / rate;
    const int32_t n = (int32_t)llround(exp(lmin + uniform_real(&st) * lspan));
    arrival_s[i] = t;
    n_rects[i] = n;
    side_nm[i] = (int32_t)llround((double)base_side * sqrt((double)n / (double)base_n));
    layout_seed[i] = lg_u64(&st);
  }
  return 0;
}
