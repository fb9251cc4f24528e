// Host-side construction of the dt-independent mesh context: DG-Q1 element
// and face integrals, block-ELL assembly of A_div, A_div Z, the element mass
// blocks, the Galerkin hierarchy of L = 2 Z^T A_div Z and the RAS tile
// inverses (paper Sections 3.1, 3.3.2, 4.2; Algorithm 2).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace dcg {

constexpr int kSlots = 5;        // self, x-1, x+1, y-1, y+1
constexpr int kTileCore = 4;     // 4 x 4 squares per RAS core
constexpr int kTileSlots = 32;   // core + face-neighbour layer
constexpr int kTileDofs = 128;   // 4 dofs per square
constexpr int kTileExt = 52;     // block squares + their outside neighbours
constexpr int kCoarsestN = 16;   // level 1 is 16 x 16 squares
constexpr int kCoarseDofs = 4 * kCoarsestN * kCoarsestN;

struct HostLevel {
  int n = 0;                       // squares per side on this level
  std::vector<double> L;           // [Ne][5][4][4]
  std::vector<int32_t> cols;       // [Ne][5], -1 = no neighbour
  // RAS data, levels k >= 2
  int tiles = 0;
  std::vector<int32_t> tile_elems; // [T][32], -1 = padded slot
  std::vector<int32_t> tile_ext;   // [T][52]: the 32 block squares, then the 20
                                   // squares at distance 1 outside the block
  std::vector<int32_t> tile_class; // [T] index into unique_inv
  std::vector<std::vector<double>> unique_inv;  // each [128][128] = (L_k)_i^{-1} (symmetric)
  std::vector<double> dw;          // [Ne] partition-of-unity weight 1 / #blocks containing e
  std::vector<int32_t> cover;      // [Ne][3] = tile * 32 + slot, -1 = none
  std::vector<int32_t> tile_dst;   // [T][32] = 3 e + k, k = rank of the tile in e's cover
};

struct HostContext {
  int n = 0, J = 0;
  double penalty = 10.0;
  std::vector<double> Adiv;        // [Ne][5][16][16]
  std::vector<double> AdivZ;       // [Ne][5][16][4]
  std::vector<double> M1;          // [Ne][4][4]
  std::vector<int32_t> cols;       // [Ne][5]
  std::vector<HostLevel> levels;   // levels[k - 1], k = 1..J
  std::vector<double> coarse_inv;  // [1024][1024]
};

// The 16 x 16 blocks of A* = (1/nu) M + dt A_div (eq. (pb_study)) of one
// square of each boundary class on the n x n grid: out[cls][slot][16][16],
// row-major, cls = cx + 3 cy with c = 0 at the low side (x = 0), 1 inside,
// 2 at the high side; rows and columns 4 c + j in the element-major order
// (c the stress component 11, 12, 21, 22, j the corner).  n >= 3.
void astar_class_blocks(int n, double penalty, double dt, double nu, std::vector<double>& out);

// J = log2(n / 16) + 1, or -1 if n is not 16 * 2^k (n <= 2048).
int num_levels(int n);

// Builds the full context; throws std::runtime_error on failure.  When
// ``with_tiles`` is false the RAS inverses and the coarsest inverse are
// skipped (used by the host-only assembly queries that do not need them).
void build_host_context(int n, double penalty, bool with_tiles, bool with_coarse,
                        HostContext& out);

}  // namespace dcg
