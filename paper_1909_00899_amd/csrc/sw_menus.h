// Compiled kernel menus (rows per lane) of libswscan.so.
#pragma once
#include "sw_internal.h"

namespace swk {

// Shared-query kernel menus: rows per lane for the 16-, 32- and 64-lane
// modes; menu k covers 64*seg64 query rows in every mode (0 = mode absent).
// Modes with more than 16 rows per lane are left out (0): they need more than
// 128 VGPRs with the end-cell copy, and the narrow modes they would give are
// slower than the 32-lane mode of the same menu.
constexpr SharedMenu kSharedMenus[] = {
    {4, 2, 1}, {8, 4, 2}, {12, 6, 3}, {16, 8, 4}, {0, 12, 6}, {0, 16, 8},
};
constexpr int kNumSharedMenus = sizeof(kSharedMenus) / sizeof(kSharedMenus[0]);

// Device-planned shared-query kernel: (rows per lane, lanes) compiled; the
// narrowest mode of each shared menu above.
struct DirectShape { int seg, lanes; };
constexpr DirectShape kDirectShapes[] = {
    {4, 16}, {8, 16}, {12, 16}, {16, 16}, {12, 32}, {16, 32},
};
constexpr int kNumDirectShapes = sizeof(kDirectShapes) / sizeof(kDirectShapes[0]);

// Per-pair kernel: rows per lane compiled.
constexpr int kPairSegs[] = {4, 6, 8, 10, 12, 16};
constexpr int kNumPairSegs = sizeof(kPairSegs) / sizeof(kPairSegs[0]);

// Device-planned per-pair kernel with eight-lane sub-groups (int16 lanes, byte
// profiles): rows per lane compiled, for queries of up to 64, 80, 104, 128
// and 152 residues (common short-read lengths fit with little padding; more
// rows per lane would spill registers).
constexpr int kPair8Segs[] = {8, 10, 13, 16, 19};
constexpr int kNumPair8Segs = sizeof(kPair8Segs) / sizeof(kPair8Segs[0]);

}  // namespace swk
