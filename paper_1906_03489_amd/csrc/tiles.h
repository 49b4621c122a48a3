// Tile configurations: elements per thread block ("slots") for each order.
// A slot is Q*Q threads in 3-D and Q threads in 2-D; LDS per slot is
// 3*Q*Q*(P+1) (3-D) scalars.  Several candidates per order are compiled and
// the autotuner picks among them; candidate 0 is the default.
#pragma once

namespace nk {

constexpr int kMaxTiles = 3;

// 3-D: elements per block, 0 = no candidate.
constexpr int kTileEPB3[11][kMaxTiles] = {
    {0, 0, 0},   // P = 0 (unused)
    {7, 28, 0},  // Q = 3:  63 / 252 threads
    {4, 16, 0},  // Q = 4:  64 / 256
    {5, 10, 0},  // Q = 5: 125 / 250
    {2, 7, 0},   // Q = 6:  72 / 252
    {1, 5, 0},   // Q = 7:  49 / 245
    {1, 2, 4},   // Q = 8:  64 / 128 / 256
    {1, 3, 0},   // Q = 9:  81 / 243
    {1, 2, 0},   // Q = 10: 100 / 200
    {1, 2, 0},   // Q = 11: 121 / 242
    {1, 0, 0},   // Q = 12: 144
};

// 2-D: elements per block (slot = Q threads).
constexpr int kTileEPB2[11][kMaxTiles] = {
    {0, 0, 0}, {21, 0, 0}, {16, 64, 0}, {12, 51, 0}, {10, 42, 0}, {9, 36, 0},
    {8, 32, 0}, {7, 28, 0}, {6, 25, 0},  {5, 23, 0},  {5, 21, 0},
};

// Elements per block of the single mixed-order launch (256 threads).
constexpr int kVarpThreads = 256;
constexpr int kVarpEPB[11] = {0, 28, 16, 10, 7, 5, 4, 3, 2, 2, 1};

constexpr bool op_has_tiles(int op) { return op <= 3; }

}  // namespace nk
