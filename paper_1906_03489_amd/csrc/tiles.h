// Tile configurations: elements per thread block ("slots") for each order.
// A slot is Q*Q threads in 3-D and Q threads in 2-D; LDS per slot is
// 3*Q*Q*(P+1) (3-D) scalars.  Several candidates per order are compiled and
// the autotuner picks among them; candidate 0 is the default.
#pragma once

namespace nk {

constexpr int kMaxTiles = 3;

// 3-D: elements per block, 0 = no candidate.  Slots hold slot_threads<Q>()
// threads: Q*Q rounded up to 16 or 64 for Q <= 8 (a slot never straddles a
// wavefront), Q*Q above.
constexpr int kTileEPB3[11][kMaxTiles] = {
    {0, 0, 0},   // P = 0 (unused)
    {4, 16, 0},  // Q = 3:  slot 16:  64 / 256 threads
    {4, 16, 0},  // Q = 4:  slot 16:  64 / 256
    {1, 4, 0},   // Q = 5:  slot 64:  64 / 256
    {1, 4, 0},   // Q = 6:  slot 64
    {1, 4, 0},   // Q = 7:  slot 64
    {1, 2, 4},   // Q = 8:  slot 64:  64 / 128 / 256
    {1, 3, 0},   // Q = 9:  slot 81:  81 / 243
    {1, 2, 0},   // Q = 10: slot 100: 100 / 200
    {1, 2, 0},   // Q = 11: slot 121: 121 / 242
    {1, 0, 0},   // Q = 12: slot 144
};

// 2-D: elements per block (slot = Q threads).
constexpr int kTileEPB2[11][kMaxTiles] = {
    {0, 0, 0}, {21, 0, 0}, {16, 64, 0}, {12, 51, 0}, {10, 42, 0}, {9, 36, 0},
    {8, 32, 0}, {7, 28, 0}, {6, 25, 0},  {5, 23, 0},  {5, 21, 0},
};

// Elements per block of the single mixed-order launch (256 threads).
constexpr int kVarpThreads = 256;
constexpr int kVarpEPB[11] = {0, 16, 16, 4, 4, 4, 4, 3, 2, 2, 1};

constexpr bool op_has_tiles(int op) { return op <= 3; }

// The 3-D Helmholtz operators (local and assembled) have each elements-per-
// block candidate in three forms: with the factors of the next point
// prefetched into a second register set, "lean" (one set: fewer registers,
// more waves per SIMD) and "deep" (kDeepPF sets: the loads of kDeepPF - 1
// points ahead in flight).  Which wins depends on the order and precision, so
// all are timed.
constexpr int kDeepPF = 4;
constexpr int kHelmForms = 3;

// One more Helmholtz candidate where a slot of Q*Q threads leaves lanes idle
// when rounded up to 64 (Q = 5, 6, 7: 25, 36, 49 of 64): slots of exactly
// Q*Q threads packed into blocks of up to 256 (block barriers between the
// stages).  Elements per block, 0 where there is no such candidate.
constexpr int packed_epb3(int P) {
  const int q2 = (P + 2) * (P + 2);
  return (q2 > 16 && q2 < 64) ? 256 / q2 : 0;
}
constexpr int epb3_count(int P) {
  int c = 0;
  for (int k = 0; k < kMaxTiles; ++k) c += kTileEPB3[P][k] > 0 ? 1 : 0;
  return c;
}
constexpr bool op_has_lean(int op) { return op == 2 || op == 3; }

// Every 3-D Helmholtz candidate above exists twice: with the I stage in
// even-odd point pairs (the first half of the list: fewer products) and
// point by point (the second half: fewer live registers).
constexpr bool helm_has_pt(int) { return true; }

}  // namespace nk
