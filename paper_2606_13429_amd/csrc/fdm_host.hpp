// Host set-up of the exact inner solve by fast diagonalisation on the uniform
// grid (the 2D path): one-dimensional DG-P1 matrices along an axis and their
// generalised eigen-decomposition K V = M V diag(lambda), V^T M V = I.
#pragma once
#include <vector>

namespace dcg {

struct FdmAxis {
  int N = 0;                 // 2 n dofs along the axis (dof 2 c + i, i = 0 left node)
  std::vector<double> V;     // [N][N] row-major, column j = eigenvector j
  std::vector<double> lam;   // [N]
};

// K: the 1D SIPG matrix on n cells of side 1/n (volume term, interior-node
// terms with penalty gamma, and the boundary-node term at the left end x = 0
// when left_bc, at the right end x = 1 when right_bc); M: the 1D DG-P1 mass
// matrix.  Both N x N row-major.
void sipg_axis(int n, double gamma, bool left_bc, std::vector<double>& K, std::vector<double>& M,
               bool right_bc = false);

// K V = M V Lambda, V^T M V = I, for the matrices of sipg_axis (M block
// diagonal with 2 x 2 blocks): Cholesky of M, Householder tridiagonalisation
// of R^{-T} K R^{-1} and the implicit QL iteration.
FdmAxis fdm_axis_factor(int n, double gamma, bool left_bc, bool right_bc = false);

// The same decomposition for given N x N row-major K (symmetric) and M
// (symmetric positive definite, block diagonal with 2 x 2 blocks).
FdmAxis fdm_factor(const std::vector<double>& K, const std::vector<double>& M, int N);

// K <- P^T K P, M <- P^T M P for the matrices of one axis on n cells (n
// even), with P the exact injection of DG-P1 on n / 2 cells (two fine cells
// per coarse cell) into DG-P1 on n cells: the one-dimensional factor of the
// Q1 injection of the 2 x 2-square agglomeration.
void galerkin_coarsen_axis(int n, std::vector<double>& K, std::vector<double>& M);

// Factors of the axis matrices of the level ``coarsenings`` steps below the
// finest grid of n squares per side in the Galerkin hierarchy L_{k-1} =
// P_k^T L_k P_k: since P_k = P (x) P, every level keeps the form
// M_k (x) K_k + K_k (x) M_k, so its exact inverse is again a fast
// diagonalisation.  Traction node at the left end (x = 0 and y = 0).
FdmAxis fdm_coarse_axis(int n, double gamma, int coarsenings);

}  // namespace dcg
