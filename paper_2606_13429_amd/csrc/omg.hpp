// Multigrid on A* as the preconditioner of the flexible outer iteration:
// B(r) = one W-cycle (Algorithm 4) from zero on the Galerkin hierarchy of
// A* = (1/nu) M + dt A_div (eq. (pb_study)) with the RAS smoother of Section
// 4.2 applied to A*'s unknowns -- the outer multigrid the paper's
// conclusions leave to future work.  FP64 throughout.
//
// Levels k = 1 (coarsest, 8 x 8 squares) .. J (finest, n x n), nested by
// 2 x 2 agglomeration; a level's tensor space is four copies of the scalar
// DG-Q1 space, so the prolongation injects each stress component as the
// scalar hierarchy does.  Level vectors hold 16 values per square in the
// element-major order of the 2D solver, idx = 16 e + 4 c + j (c the stress
// component 11, 12, 21, 22, j = ix + 2 iy the corner).
//
// RAS blocks: one per square -- all four components on the square and its
// edge neighbours, clipped at the boundary; D = 1 / (blocks holding the dof).
// On the uniform grid a square's operator rows depend only on which sides it
// touches and its RAS update only on its distance 0, 1, 2 or >= 3 from each
// side, so every level stores class tables (row-major):
//   op  [9][5][16][16]   op[cls][slot][a][b] = A*_k(row a of the square,
//                        column b of its slot neighbour); slots 0 itself,
//                        1/2 x-1/x+1, 3/4 y-1/y+1; cls = cx + 3 cy, c = 0 at
//                        the low side, 2 at the high side, 1 inside
//   ras [49][16][208]    (S_k r) on a square = ras[cls] r on the 13 squares
//                        with |dx| + |dy| <= 2 (ordered by dy, then dx;
//                        column 16 d + b; zero for squares outside the
//                        domain); cls = px + 7 py with p = x (x < 3),
//                        6 - (n_k - 1 - x) (n_k - 1 - x < 3), else 3; levels
//                        below 6 squares per side take cls = e
// and the coarsest level the dense inverse of its operator, row-major.  The
// MFMA kernels read both tables in the operand order of v_mfma_f64_16x16x4f64
// (a 16-row table times 16 squares' gathered inputs, four columns a step):
//   opm  [9][20][64], rasm [49][52][64]: entry (cls, s, l) = row l % 16,
//                        column 4 s + l / 16 of the row-major table above
//                        (column 16 slot + b of op), so that one step's
//                        operand is one contiguous 512-byte load.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace dcg {

constexpr int kOmgDofs = 16;
constexpr int kOmgOpClasses = 9;
constexpr int kOmgRasClasses = 49;
constexpr int kOmgRasClassMinN = 6;
constexpr int kOmgDiamond = 13;
constexpr int kOmgRasCols = kOmgDofs * kOmgDiamond;
constexpr int kOmgCoarsest = 8;
constexpr int kOmgOpCols = 5 * kOmgDofs;   // self and the four edge neighbours
constexpr int kOmgRasSteps = kOmgRasCols / 4;
constexpr int kOmgOpSteps = kOmgOpCols / 4;

struct OmgLevel {
  int n = 0;
  std::vector<double> op;    // [9][5][16][16]
  std::vector<double> ras;   // [49][16][208] (levels >= 2)
};

struct OmgHierarchy {
  std::vector<OmgLevel> lev;        // lev[k - 1] is level k
  std::vector<double> coarse_inv;   // [16 c^2][16 c^2]
};

// Offsets (dx, dy) of the 2D diamond, |dx| + |dy| <= 2, by dy then dx.
void omg_diamond(int off[kOmgDiamond][2]);

// The operand order of a table of `classes` row-major 16 x cols class
// matrices (cols a multiple of 4): [classes][cols / 4][64].
std::vector<double> omg_operand_order(const std::vector<double>& tab, int classes, int cols);

// The operator table as 9 row-major 16 x 80 matrices (column 16 slot + b).
std::vector<double> omg_op_rows(const std::vector<double>& op);

// J = log2(n / 8) + 1 for n = 8 2^k >= 16, else 0.
int omg_num_levels(int n);

// Builds the hierarchy of A* for the n x n grid: the finest class table from
// the assembly, P^T A P class by class, the RAS update tables (block
// inverses by Cholesky) and the coarsest inverse.  Throws on failure.
OmgHierarchy build_omg(int n, double penalty, double dt, double nu);

// ---- launchers (FP64; level vectors as above)
// r = f - A*_k z (f may be NULL: r = -A*_k z); op and opm the level's
// operator table in both orders.
hipError_t launch_omg_res(int nk, const double* op, const double* opm, const double* f, const double* z,
                          double* r, hipStream_t st);
// z = (zero ? 0 : z) + S_k r; ras and rasm the level's RAS table in both orders.
hipError_t launch_omg_ras(int nk, const double* ras, const double* rasm, const double* r, double* z,
                          bool zero, hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// fc = P_k^T r (nf fine squares per side).
hipError_t launch_omg_restrict(int nf, const double* r, double* fc, hipStream_t st);
// z += P_k zc, or z = P_k zc with assign.
hipError_t launch_omg_prolong(int nf, const double* zc, double* z, bool assign, hipStream_t st);
// z = inv f (dense m x m, row-major).
hipError_t launch_omg_dense(int m, const double* inv, const double* f, double* z, hipStream_t st);

}  // namespace dcg
