// trace.h - the trace fingerprint, our check of the search order (the
// method defines no such value).  Each counted search node contributes
// x = FNV-1a 64 (Fowler/Noll/Vo) of its 16 bytes - depth, entering row,
// chosen column, its size; u32 little-endian each (entering row 0xFFFFFFFF
// at the root, column 0xFFFFFFFF at a solution) - started from the offset
// basis; a trace of N nodes has fingerprint sum x_i * B^(N-i) mod 2^64 with
// B the FNV prime, i.e. h = h * B + x per node from h = 0.  A trace S
// followed by a trace T then has h(S) * B^|T| + h(T), so subtrees searched
// apart combine exactly in search order.  The functions are constexpr, so
// host code and (implicitly host-device) device code share them.
#pragma once

#include <cstdint>

namespace mpld {

constexpr uint64_t kTraceBase = 0x100000001b3ull;   // the FNV prime
constexpr uint64_t kFnvBasis = 0xcbf29ce484222325ull;

constexpr uint64_t fnv_word(uint64_t h, uint32_t v) {
  for (int b = 0; b < 4; ++b) {
    h ^= (v >> (8 * b)) & 0xffu;
    h *= kTraceBase;
  }
  return h;
}

// The fingerprint h of a trace extended by one node.
constexpr uint64_t trace_node(uint64_t h, uint32_t depth, uint32_t row_in, uint32_t col,
                              uint32_t size) {
  return h * kTraceBase + fnv_word(fnv_word(fnv_word(fnv_word(kFnvBasis, depth), row_in), col), size);
}

// B^n mod 2^64.
constexpr uint64_t trace_pow(uint64_t n) {
  uint64_t r = 1, b = kTraceBase;
  while (n) {
    if (n & 1u) r *= b;
    b *= b;
    n >>= 1;
  }
  return r;
}

// Fingerprint of trace a followed by trace b of nb nodes.
constexpr uint64_t trace_concat(uint64_t a, uint64_t b, uint64_t nb) { return a * trace_pow(nb) + b; }

}  // namespace mpld
