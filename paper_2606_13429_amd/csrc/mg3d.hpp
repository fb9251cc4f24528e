// Multigrid inner solve of the three-dimensional deflated CG (Section 4.2,
// the 3D case): the Multigrid iteration of Algorithm 3 with the W-cycle of
// Algorithm 4 on the Galerkin hierarchy of the SIPG Laplacian
// L = B_11 + B_22 + B_33 (Corollary 1: Z^T A* Z = (dt/3) L), smoothed by
// Restricted Additive Schwarz with one block per cube -- the cube and its
// face neighbours.  FP64 throughout.
//
// Levels k = 1 (coarsest, c^3 cubes, 2 <= c <= 4) .. J (finest, n^3 cubes),
// nested by 2 x 2 x 2 agglomeration; level vectors hold 8 values per cube,
// idx = 8 e + a (e = (ez n_k + ey) n_k + ex, corner a = ix + 2 iy + 4 iz).
//
// On the uniform grid a cube's operator rows depend only on which sides of
// the domain it touches, and its RAS update only on its distance (0, 1, 2
// or >= 3) from each side -- the update reads the local problems of its own
// and its neighbours' blocks, whose rows reach two cubes away -- so every
// level stores class tables instead of per-cube blocks:
//   op  [27][7][8][8]    row-major, op[cls][slot][a][b] = L_k(row a of the
//                        cube, column b of its slot neighbour); slots as in
//                        dcg3d.hpp (0 itself, 1/2 -x/+x, 3/4 -y/+y, 5/6 -z/+z);
//                        cls = cx + 3 cy + 9 cz, c_axis = 0 at the low side,
//                        2 at the high side, 1 inside
//   ras [343][8][200]    row-major: the RAS step's update of a cube,
//                        (S_k r)|_cube = ras[cls] r|_diamond, where the
//                        diamond is the 25 cubes within face-path distance
//                        2 (the cubes of every block that holds the cube),
//                        column 8 d + b for diamond cube d (kDiamond order),
//                        zero columns for cubes outside the domain;
//                        cls = px + 7 py + 49 pz with p = x (x < 3),
//                        6 - (n_k - 1 - x) (n_k - 1 - x < 3), else 3;
//                        levels with n_k < 6 take one class per cube,
//                        cls = e (at most 125)
// The coarsest level keeps the dense inverse of its operator, row-major.
// On the device, levels with more than kSplitMaxN cubes per side store both
// tables with the row index fastest (op [27][7 slots][8 columns][8 rows],
// ras [343][200 columns][8 rows], from op_rows_fastest / rows_fastest), so
// that the eight threads of a cube read one contiguous segment per column;
// smaller levels keep the row-major tables (one lane per row segment).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace dcg3 {

constexpr int kOpClasses = 27;
constexpr int kRasClasses = 343;
constexpr int kRasClassMinN = 6;   // smaller levels: one class per cube
constexpr int kDiamond = 25;
constexpr int kRasCols = 8 * kDiamond;
constexpr int kMaxCoarsest = 4;
constexpr int kSplitMaxN = 16;     // levels up to this size: one lane per term group

// Offsets (dx, dy, dz) of the diamond, |dx| + |dy| + |dz| <= 2, in the order
// z, then y, then x ascending.
void diamond_offsets(int off[kDiamond][3]);

struct Mg3Level {
  int n = 0;                 // cubes per side
  std::vector<double> op;    // [27][7][8][8]
  std::vector<double> ras;   // [343][8][200] (levels >= 2)
};

struct Mg3Hierarchy {
  std::vector<Mg3Level> lev;        // lev[k - 1] is level k
  std::vector<double> coarse_inv;   // [m_1][m_1], m_1 = 8 c^3
};

// A table of [classes][8 rows][cols] (row-major blocks) as
// [classes][cols][8 rows]; the operator table [27][7][8][8] as [27][7][8 b][8 a].
std::vector<double> rows_fastest(const std::vector<double>& t, int cols);
std::vector<double> op_rows_fastest(const std::vector<double>& op);

// Number of levels J for n cubes per side with the finest `levels` levels
// (0: down to the smallest coarsest size c >= 2); c = n / 2^(J-1) must lie
// in [2, 4].  Returns 0 when n admits no such hierarchy.
int mg3_num_levels(int n, int levels);

// Builds the hierarchy from the finest Laplacian blocks ld ([7][n^3][8][8],
// column-major per block, the layout of dcg3d.hpp): checks that every cube
// carries the blocks of its class bit for bit, forms each coarser level as
// P^T L P class by class, the RAS class tables of levels >= 2 and the
// coarsest inverse.  Throws std::runtime_error on failure.
Mg3Hierarchy build_mg3(int n, int J, const std::vector<double>& ld);

// ---- launchers (guard: the kernels do nothing while *guard == 0; NULL = run)
// r = f - L_k z (f = NULL: 0, z = NULL: 0), and with part != NULL the
// per-workgroup partial sums of r^2.
hipError_t launch_mg3_res(int nk, const double* op, const double* f, const double* z, double* r,
                          double* part, const int32_t* guard, hipStream_t st);
int mg3_res_blocks(int nk);
// True when level nk runs the small-level kernels (one lane per term group
// without LDS staging, row-major tables) rather than the brick kernels.
bool mg3_split(int nk);
// z = (zero ? 0 : z) + S_k r, ras the level's class table.
hipError_t launch_mg3_ras(int nk, const double* ras, const double* r, double* z, bool zero,
                          const int32_t* guard, hipStream_t st, hipEvent_t ev0 = nullptr,
                          hipEvent_t ev1 = nullptr);
// fc = P_k^T r (nf = fine cubes per side).
hipError_t launch_mg3_restrict(int nf, const double* r, double* fc, const int32_t* guard,
                               hipStream_t st);
// z += P_k zc, or z = P_k zc with assign.
hipError_t launch_mg3_prolong(int nf, const double* zc, double* z, bool assign,
                              const int32_t* guard, hipStream_t st);
// z = inv f (dense, m x m, row-major).
hipError_t launch_mg3_dense(int m, const double* inv, const double* f, double* z,
                            const int32_t* guard, hipStream_t st);

// Device state of one Multigrid iteration (Algorithm 3).
struct Mg3Scalars {
  double rel2;       // (relative tolerance)^2
  double thresh2;    // stop once ||s - L z||^2 <= thresh2 (set by the first test)
  double rr;         // the last ||s - L z||^2
  int32_t active;    // 1 while W-cycles remain to be applied
  int32_t first;     // 1 until the first test has read ||s||^2
  int32_t iters;     // W-cycles applied
  int32_t max_iters; // n_max of Algorithm 3
};
// Start of an inner solve: z = 0, scalars set for relative tolerance rel and
// at most max_iters cycles.
hipError_t launch_mg3_start(int64_t len, double* z, Mg3Scalars* sc, double rel2, int max_iters,
                            hipStream_t st);
// The stopping test of Algorithm 3 from the residual partials: clears
// active when ||s - L z||^2 <= thresh2 or max_iters cycles are done, else
// counts the cycle that follows.
hipError_t launch_mg3_test(int nparts, const double* part, Mg3Scalars* sc, hipStream_t st);
// y = a x.
hipError_t launch_mg3_scale(int64_t len, double a, const double* x, double* y, hipStream_t st);

}  // namespace dcg3
