/*
 * layoutgen.h - seeded synthetic layout and request-trace generator.
 *
 * This module produces INPUTS only: axis-aligned rectangles standing in for
 * the layout features of the paper's problem statement (Sec. 2.1; the flow
 * of Sec. 2.2 builds its layout graph from the layout's rectangles), and arrival
 * traces for a serving workload.  It holds none of the decomposition method's
 * arithmetic (no conflict test, no graph, no search) and is shared, as a
 * separate library, by the product library's callers and by the oracle's
 * tests.  The paper's own benchmark layouts (ISCAS, Sec. 3) are not
 * available; these seeded generators stand in for them.
 *
 * Random numbers:
 *   - SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
 *     number generators", OOPSLA 2014): state += 0x9e3779b97f4a7c15, then the
 *     variant-13 finaliser.  lg_u64() returns one output.
 *   - 32-bit draw      = top 32 bits of one lg_u64() output.
 *   - uniform integer in [lo, hi] = lo + Lemire's multiply-shift with
 *     rejection on the 32-bit draw (Lemire, "Fast random integer generation
 *     in an interval", ACM TOMACS 2019).
 *   - Bernoulli(1/2)  = top bit of one lg_u64() output.
 *   - uniform real in [0,1) = (lg_u64() >> 11) * 2^-53.
 *
 * Rectangle placement (one attempt draws, in this order): orientation
 * (1 = vertical), length L in [len_min, len_max], x in [0, side-1],
 * y in [0, side-1].  Horizontal: [x, x+L] x [y, y+width]; vertical:
 * [x, x+width] x [y, y+L].  Boxes are closed and may extend past the
 * window.  A placement that intersects or touches an already placed box is
 * redrawn (all four draws again), at most max_attempts times; after that the
 * rectangle is skipped and counted.
 *
 * Ownership: the caller owns every buffer; nothing is allocated for the
 * caller.  Errors: negative return, no partial guarantees on outputs.
 */
#ifndef LAYOUTGEN_H
#define LAYOUTGEN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { int32_t x0, y0, x1, y1; } lg_rect;

typedef struct {
  int32_t n;            /* rectangles to place                       */
  int32_t side;         /* window side, nm (corners drawn in [0,side)) */
  int32_t width;        /* short side, nm (20)                       */
  int32_t len_min;      /* long side range, nm (40)                  */
  int32_t len_max;      /* (200)                                     */
  int32_t max_attempts; /* redraw cap per rectangle (1000)           */
} lg_params;

/* One SplitMix64 step on *state; returns the output. */
uint64_t lg_u64(uint64_t* state);

/* Places up to p->n rectangles into out[0 .. p->n-1] (caller-allocated with
 * room for p->n).  *placed receives the count written (in placement order),
 * *skipped the count given up after max_attempts.  Returns 0, or -1 on bad
 * parameters (n < 0, side < 1, width < 0, len_min > len_max, len_min < 0,
 * max_attempts < 1) or -2 when scratch memory cannot be allocated. */
int32_t lg_generate(const lg_params* p, uint64_t seed, lg_rect* out,
                    int32_t* placed, int32_t* skipped);

/* Request trace for a serving workload: Poisson arrivals at `rate` per second
 * and feature counts log-uniform in [n_min, n_max]; the window side is
 * scaled as round(base_side * sqrt(N / base_n)) to keep the density of the
 * base window.  Per request, draws in this order: u1 (uniform real) ->
 * gap = -ln(1-u1)/rate added to the running time; u2 -> N =
 * round(exp(ln n_min + u2 * ln(n_max/n_min))); then one lg_u64() as the
 * request's layout seed.  Writes count entries to each output array.
 * Returns 0 or -1 on bad parameters. */
int32_t lg_request_trace(uint64_t seed, int32_t count, double rate,
                         int32_t n_min, int32_t n_max, int32_t base_side,
                         int32_t base_n, double* arrival_s, int32_t* n_rects,
                         int32_t* side_nm, uint64_t* layout_seed);

#ifdef __cplusplus
}
#endif
#endif
