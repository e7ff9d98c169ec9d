// device_types.h - layout of the packed exact-cover image in device memory,
// shared by the host packer/runtime and the HIP kernels.
#pragma once

#include <cstdint>

namespace mpld {

enum Tier : int32_t { kTierReg = 0, kTierLds = 1, kTierGlobal = 2, kTierDevice = 3 };

// One descriptor per component (32 bytes).  On the device the descriptors
// of each tier are stored contiguously in that tier's launch order (largest
// component first), so a wave's work item indexes them directly.
//   register tier: nbr_off indexes `masks` (one uint64 neighbour mask per
//                  local node, bit u set iff u is a conflict neighbour).
//   LDS / global tier: nbr_off indexes `adj32`: n+1 row offsets (relative to
//                  nbr_off + n + 1) followed by the local neighbour ids.
struct DevDesc {
  int32_t n;        // nodes
  int32_t k;        // colors
  int64_t budget;   // search-node budget
  int64_t nbr_off;
  int32_t out_off;  // first entry of the component in the colors output
  int32_t comp;     // component id: index of its record
};
static_assert(sizeof(DevDesc) == 32, "descriptor is 32 bytes");

// Register-tier work items (n <= 64), stored in launch order.  Item i is a
// 32-byte descriptor followed by `width` neighbour masks (mask v = the
// conflict neighbours of local node v; zero past n) at byte offset
// i * stride, stride = 32 + 8 * width (+ 8-byte-rounded partner bytes with
// the stitch-aware order).  One width per batch (the largest n
// of its items) keeps the address a function of the index, so a wave
// issues the descriptor and mask loads at once, and lanes at or past
// `width` load nothing.
struct RegItems {
  const uint8_t* base;
  uint32_t width;      // 1 .. 64
  uint32_t stride;     // 32 + 8 * width bytes (+ the partner bytes)
  uint32_t part_off;   // with the stitch-aware order: offset of `width` bytes
                       // of local stitch partners (0xff none) in an item; 0 = none
};
constexpr uint32_t kRegItemHead = 32;
inline uint32_t reg_item_width(int32_t max_n) { return max_n < 1 ? 1u : (uint32_t)max_n; }

// Largest component of the one-wave LDS tier (one 32-bit node word per
// lane of a wave).
constexpr int32_t kLds1MaxN = 2048;
// One-wave wide tier (big components whose planes and neighbour lists fit
// in LDS): at most 8 node words of 32 nodes per lane, so at most 16384
// nodes, and k <= 6 (beyond it the kernels it shares with the workgroup
// layout would need scratch memory); its offs words hold the first
// neighbour in 17 bits and the degree above them.
constexpr int32_t kWideMaxWords = 8;
constexpr int32_t kWideMaxK = 6;
constexpr int32_t kWideMaxN = 64 * 32 * kWideMaxWords;
constexpr uint32_t kWideBegBits = 17;

// One record per component (24 bytes), written by the search.
struct DevRecord {
  int32_t status;   // MPLD_FEASIBLE / MPLD_INFEASIBLE / MPLD_BUDGET_EXHAUSTED
  int32_t depth;    // rows in the partial solution at the stop (0 if infeasible)
  uint64_t nodes;   // search nodes
  uint64_t hash;    // trace fingerprint (trace.h; 0 when tracing is off)
};
static_assert(sizeof(DevRecord) == 24, "record is 24 bytes");

// A subtree task of an LDS-tier or big-tier component (the heavy-component
// split beyond the register tier): the subtree of root row `row` searched
// with its own node budget; its colors go to task colors + col_off.
struct LdsTask {
  int32_t item;        // launch-ordered descriptor index
  int32_t row;         // root row (color of node 0)
  int64_t budget;      // >= 1
  int64_t col_off;
};
static_assert(sizeof(LdsTask) == 24, "LDS task is 24 bytes");
// A resolved LDS-tier or big-tier component of the split: its record and
// where its colors come from.
struct LdsResolved {
  int32_t comp;        // record index
  int32_t out_off;     // first color entry
  int32_t n;
  int32_t pad;
  int64_t src_off;     // colors in the task color area, -1: none (all -1)
  DevRecord rec;
};
static_assert(sizeof(LdsResolved) == 48, "resolved entry is 48 bytes");

// Heavy-component engine (parallel subtree search).  A task is the subtree
// of the node reached from a component's root by taking `depth` rows
// (v | c << 8 each).
struct SplitTask {
  int32_t item;        // launch-ordered descriptor index of the component
  int32_t depth;       // depth of the subtree root (rows on the path)
  uint16_t rows[64];
};
static_assert(sizeof(SplitTask) == 136, "task is 136 bytes");
// Result of exploring one task with a node cap.
struct SplitResult {
  int32_t status;      // MPLD_FEASIBLE, MPLD_INFEASIBLE (subtree exhausted) or -1 (cap hit)
  int32_t nitems;      // split items written when the cap was hit
  uint64_t nodes;      // nodes explored (the subtree's own count when finished)
  uint32_t item_off;   // first of the task's items in the round's item pool
  uint32_t pad;
  uint64_t hash;       // traced engine, finished task: trace hash of its own nodes
};
static_assert(sizeof(SplitResult) == 32, "result is 32 bytes");
// One item of the split of a capped task, in depth-first order: `seg` nodes
// of the task's top levels are visited, then (kind 0) the subtree of the
// node reached by rows[0..levels-1] below the task root, or (kind 1) the
// task ends, or (kind 2) the last of the seg nodes was a solution.
struct SplitItem {
  uint32_t seg;
  uint32_t kind;
  uint16_t rows[4];
};
static_assert(sizeof(SplitItem) == 16, "item is 16 bytes");
constexpr int kSplitMaxLevels = 4;
// Output block of one task in a split round (all of a round's blocks in one
// buffer, read back with one copy): the result, then the solution (colors by
// local node, when the task found one).  A capped task's split items go to
// a pool shared by the round, at an offset taken with one atomic, so only
// the items that exist are read back.
constexpr uint32_t kSplitSolOffset = 32;
constexpr uint32_t kSplitBlockBytes = 96;
// Device-resident heavy-component engine.  Tasks of every round live in one
// array: round r runs the tasks [begin, end) and appends the subtasks of
// its capped tasks at `alloc`; a one-thread kernel between rounds moves the
// window on.  Capped tasks put their items in one pool at `pool`.
struct EngineHead {
  int32_t begin, end;   // tasks of the current round
  int32_t alloc;        // next free task slot (may pass the capacity)
  int32_t pool;         // next free item slot (may pass the capacity)
  int32_t pop;          // work counter of the current round
  int32_t rounds;       // rounds started
  int32_t overflow;     // an allocation did not fit (the host re-runs)
  int32_t pad[9];
};
static_assert(sizeof(EngineHead) == 64, "engine head is 64 bytes");
struct EngineTask {
  int32_t item;         // launch-ordered index of the component's register item
  int32_t depth;        // rows on the path from the root
  int32_t hc;           // heavy-component index
  int32_t skip;         // nonzero: a slot whose subtask could not be stored
  uint16_t rows[64];    // the path: v | c << 8 per depth
};
static_assert(sizeof(EngineTask) == 144, "engine task is 144 bytes");
// One item of a capped task's split (as SplitItem, with the subtask's task
// index instead of its rows).
struct EngineItem {
  uint32_t seg;
  int32_t child;        // >= 0: the subtask's task index; kEngineItemEnd: the
                        // task ends; kEngineItemSolution: the last seg node
                        // was a solution
  uint64_t hash;        // traced engine: trace hash of the seg nodes
};
static_assert(sizeof(EngineItem) == 16, "engine item is 16 bytes");
constexpr int32_t kEngineItemEnd = -1, kEngineItemSolution = -2;
constexpr int32_t kEngineSkipped = -3;   // task status: not run (skip slot) or not split (budget or space)

// A resolved heavy component written back by the device: its record and
// colors, scattered to their places by one small kernel.
struct HeavyWrite {
  int32_t comp;        // record index
  int32_t out_off;     // first color entry
  int32_t n;
  int32_t pad;
  DevRecord rec;
  int8_t colors[64];
};
static_assert(sizeof(HeavyWrite) == 104, "write-back entry is 104 bytes");

// Device bytes of the resumable register-tier search state of one
// component (serving): a 128-byte uniform head (counters, then up to eight
// 64-bit color planes), then 64 lanes x (u32 frame, u64 P snapshot, up to
// eight u64 plane snapshots, u32 stitch partner and its color).
constexpr uint64_t kRegStateBytes = 128 + 64 * 4 * (3 + 2 * 8 + 1);

}  // namespace mpld
