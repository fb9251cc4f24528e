// Host set-up of the exact inner solve by fast diagonalisation (2D path).
//
// On the uniform grid the SIPG Laplacian of Corollary 1 separates: with M the
// 1D DG-P1 mass matrix and K_x, K_y the 1D SIPG matrices of one axis (volume
// term, interior-node terms, and the traction boundary at x = 0 resp. y = 0),
//   L = M (x) K_x + K_y (x) M          on the tensor index (Iy, Ix),
// because every face integral factors into a 1D node term times the 1D mass
// along the face.  The generalised eigenvectors of each axis then diagonalise
// L exactly.  The eigen-decomposition is the Householder reduction to
// tridiagonal form followed by the implicit QL iteration with shifts
// (Bowdler, Martin, Reinsch and Wilkinson), written out here.
#include "fdm_host.hpp"

#include <cmath>
#include <stdexcept>

namespace dcg {

void sipg_axis(int n, double gamma, bool left_bc, std::vector<double>& K, std::vector<double>& M,
               bool right_bc) {
  const int N = 2 * n;
  const double h = 1.0 / n;
  K.assign((size_t)N * N, 0.0);
  M.assign((size_t)N * N, 0.0);
  auto at = [N](std::vector<double>& A, int i, int j) -> double& { return A[(size_t)i * N + j]; };
  const double d[2] = {-1.0 / h, 1.0 / h};   // derivatives of the two P1 functions of a cell
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        at(M, 2 * c + i, 2 * c + j) += h / 6.0 * (i == j ? 2.0 : 1.0);
        at(K, 2 * c + i, 2 * c + j) += h * d[i] * d[j];
      }
  // node term -{u'}[v] - {v'}[u] + gamma [u][v]: jump and mean derivative as
  // coefficient lists over the dofs
  struct Coef { int dof; double c; };
  auto node = [&](std::initializer_list<Coef> jump, std::initializer_list<Coef> mean) {
    for (const Coef& a : jump)
      for (const Coef& b : mean) {
        at(K, a.dof, b.dof) -= a.c * b.c;
        at(K, b.dof, a.dof) -= a.c * b.c;
      }
    for (const Coef& a : jump)
      for (const Coef& b : jump) at(K, a.dof, b.dof) += gamma * a.c * b.c;
  };
  for (int c = 0; c + 1 < n; ++c)   // interior node, jump u_left - u_right
    node({{2 * c + 1, 1.0}, {2 * c + 2, -1.0}},
         {{2 * c, 0.5 * d[0]}, {2 * c + 1, 0.5 * d[1]}, {2 * c + 2, 0.5 * d[0]}, {2 * c + 3, 0.5 * d[1]}});
  if (left_bc)                      // x = 0, outward normal -1: jump -u, single trace
    node({{0, -1.0}}, {{0, d[0]}, {1, d[1]}});
  if (right_bc)                     // x = 1, outward normal +1: jump u, single trace
    node({{N - 1, 1.0}}, {{N - 2, d[0]}, {N - 1, d[1]}});
}

namespace {

// A (symmetric, N x N row-major, overwritten) = Q T Q^T with T tridiagonal:
// diagonal d, subdiagonal e (e[i] = T[i+1][i]).
void householder_tridiag(std::vector<double>& A, int N, std::vector<double>& Q, std::vector<double>& d,
                         std::vector<double>& e) {
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * N + j]; };
  Q.assign((size_t)N * N, 0.0);
  for (int i = 0; i < N; ++i) Q[(size_t)i * N + i] = 1.0;
  std::vector<double> v(N), p(N), w(N);
  for (int k = 0; k + 2 < N; ++k) {
    double nx2 = 0.0;
    for (int i = k + 1; i < N; ++i) nx2 += a(i, k) * a(i, k);
    if (nx2 == 0.0) continue;
    const double x0 = a(k + 1, k);
    const double sub = x0 >= 0.0 ? -std::sqrt(nx2) : std::sqrt(nx2);   // the new T[k+1][k]
    double vv = 0.0;
    for (int i = k + 1; i < N; ++i) {
      v[i] = a(i, k) - (i == k + 1 ? sub : 0.0);
      vv += v[i] * v[i];
    }
    if (vv == 0.0) continue;
    const double beta = 2.0 / vv;           // H = I - beta v v^T maps the column to sub e_1
    double pv = 0.0;
    for (int i = k + 1; i < N; ++i) {
      double t = 0.0;
      for (int j = k + 1; j < N; ++j) t += a(i, j) * v[j];
      p[i] = beta * t;
      pv += p[i] * v[i];
    }
    const double half = 0.5 * beta * pv;
    for (int i = k + 1; i < N; ++i) w[i] = p[i] - half * v[i];
    for (int i = k + 1; i < N; ++i)         // trailing block <- H A H = A - v w^T - w v^T
      for (int j = k + 1; j < N; ++j) a(i, j) -= v[i] * w[j] + w[i] * v[j];
    a(k + 1, k) = a(k, k + 1) = sub;
    for (int i = k + 2; i < N; ++i) a(i, k) = a(k, i) = 0.0;
    for (int r = 0; r < N; ++r) {            // Q <- Q H
      double* q = &Q[(size_t)r * N];
      double t = 0.0;
      for (int j = k + 1; j < N; ++j) t += q[j] * v[j];
      t *= beta;
      for (int j = k + 1; j < N; ++j) q[j] -= t * v[j];
    }
  }
  d.resize(N);
  e.assign(N, 0.0);
  for (int i = 0; i < N; ++i) d[i] = a(i, i);
  for (int i = 0; i + 1 < N; ++i) e[i] = a(i + 1, i);
}

// Eigenvalues d and eigenvectors (columns of Z, which enters holding the
// tridiagonalising Q) of the symmetric tridiagonal matrix (d, e) by the
// implicit QL iteration: for each leading index l, shifted QL sweeps over the
// unreduced block [l, m] until e[l] is negligible; the plane rotations of each
// sweep are applied to the columns of Z.
void tridiag_ql(std::vector<double>& d, std::vector<double>& e, int N, std::vector<double>& Z) {
  e[N - 1] = 0.0;
  const double eps = 2.220446049250313e-16;
  for (int l = 0; l < N; ++l) {
    for (int sweep = 0;; ++sweep) {
      int m = l;
      while (m + 1 < N && std::fabs(e[m]) > eps * (std::fabs(d[m]) + std::fabs(d[m + 1]))) ++m;
      if (m == l) break;
      if (sweep == 100) throw std::runtime_error("tridiagonal QL iteration did not converge");
      // shift from the leading 2 x 2 block: the eigenvalue of it closer to d[l]
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, shift_acc = 0.0;
      bool split = false;
      for (int i = m - 1; i >= l; --i) {
        const double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {          // the block splits: restart with the smaller one
          d[i + 1] -= shift_acc;
          e[m] = 0.0;
          split = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - shift_acc;
        r = (d[i] - g) * s + 2.0 * c * b;
        shift_acc = s * r;
        d[i + 1] = g + shift_acc;
        g = c * r - b;
        for (int k = 0; k < N; ++k) {   // columns i, i+1 of Z
          double* zk = &Z[(size_t)k * N];
          const double zi1 = zk[i + 1];
          zk[i + 1] = s * zk[i] + c * zi1;
          zk[i] = c * zk[i] - s * zi1;
        }
      }
      if (split) continue;
      d[l] -= shift_acc;
      e[l] = g;
      e[m] = 0.0;
    }
  }
}

}  // namespace

FdmAxis fdm_factor(const std::vector<double>& K, const std::vector<double>& M, int N) {
  if (N % 2 || K.size() != size_t(N) * N || M.size() != size_t(N) * N)
    throw std::invalid_argument("fdm_factor: K and M must be N x N with N even");
  const int n = N / 2;
  // M = R^T R with R upper triangular 2 x 2 blocks; C = R^{-T} K R^{-1}
  std::vector<double> Ri((size_t)N * N, 0.0);
  for (int c = 0; c < n; ++c) {
    const double m00 = M[(size_t)(2 * c) * N + 2 * c], m01 = M[(size_t)(2 * c) * N + 2 * c + 1],
                 m11 = M[(size_t)(2 * c + 1) * N + 2 * c + 1];
    const double r00 = std::sqrt(m00), r01 = m01 / r00, r11 = std::sqrt(m11 - r01 * r01);
    Ri[(size_t)(2 * c) * N + 2 * c] = 1.0 / r00;
    Ri[(size_t)(2 * c) * N + 2 * c + 1] = -r01 / (r00 * r11);
    Ri[(size_t)(2 * c + 1) * N + 2 * c + 1] = 1.0 / r11;
  }
  // R^{-1} has only the 2 x 2 diagonal blocks: C[i][j] = sum over the blocks of i and j
  std::vector<double> C((size_t)N * N, 0.0);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      double t = 0.0;
      for (int a = 2 * (i / 2); a < 2 * (i / 2) + 2; ++a)
        for (int b = 2 * (j / 2); b < 2 * (j / 2) + 2; ++b)
          t += Ri[(size_t)a * N + i] * K[(size_t)a * N + b] * Ri[(size_t)b * N + j];
      C[(size_t)i * N + j] = t;
    }
  for (int i = 0; i < N; ++i)
    for (int j = i + 1; j < N; ++j) {
      const double v = 0.5 * (C[(size_t)i * N + j] + C[(size_t)j * N + i]);
      C[(size_t)i * N + j] = C[(size_t)j * N + i] = v;
    }
  std::vector<double> Q, d, e;
  householder_tridiag(C, N, Q, d, e);
  tridiag_ql(d, e, N, Q);
  FdmAxis out;
  out.N = N;
  out.lam = d;
  out.V.assign((size_t)N * N, 0.0);
  for (int i = 0; i < N; ++i)         // V = R^{-1} Q (R^{-1} block diagonal)
    for (int a = 2 * (i / 2); a < 2 * (i / 2) + 2; ++a) {
      const double ria = Ri[(size_t)i * N + a];
      if (ria == 0.0) continue;
      for (int j = 0; j < N; ++j) out.V[(size_t)i * N + j] += ria * Q[(size_t)a * N + j];
    }
  return out;
}

FdmAxis fdm_axis_factor(int n, double gamma, bool left_bc, bool right_bc) {
  std::vector<double> K, M;
  sipg_axis(n, gamma, left_bc, K, M, right_bc);
  return fdm_factor(K, M, 2 * n);
}

void galerkin_coarsen_axis(int n, std::vector<double>& K, std::vector<double>& M) {
  // P: coarse DG-P1 on n / 2 cells -> fine DG-P1 on n cells.  Fine cell
  // 2 c + s, node i sits at the local coordinate t = (s + i) / 2 of coarse
  // cell c, where the coarse left / right functions take 1 - t / t.
  if (n % 2) throw std::invalid_argument("galerkin_coarsen_axis: n must be even");
  const int N = 2 * n, Nc = n;
  std::vector<double> P((size_t)N * Nc, 0.0);
  for (int c = 0; c < n / 2; ++c)
    for (int s = 0; s < 2; ++s)
      for (int i = 0; i < 2; ++i) {
        const double t = 0.5 * (s + i);
        const int row = 2 * (2 * c + s) + i;
        P[(size_t)row * Nc + 2 * c] = 1.0 - t;
        P[(size_t)row * Nc + 2 * c + 1] = t;
      }
  auto ptap = [&](const std::vector<double>& A) {
    std::vector<double> AP((size_t)N * Nc, 0.0), C((size_t)Nc * Nc, 0.0);
    for (int i = 0; i < N; ++i)
      for (int k = 0; k < N; ++k) {
        const double a = A[(size_t)i * N + k];
        if (a == 0.0) continue;
        for (int j = 0; j < Nc; ++j) AP[(size_t)i * Nc + j] += a * P[(size_t)k * Nc + j];
      }
    for (int k = 0; k < N; ++k)
      for (int i = 0; i < Nc; ++i) {
        const double p = P[(size_t)k * Nc + i];
        if (p == 0.0) continue;
        for (int j = 0; j < Nc; ++j) C[(size_t)i * Nc + j] += p * AP[(size_t)k * Nc + j];
      }
    return C;
  };
  K = ptap(K);
  M = ptap(M);
}

FdmAxis fdm_coarse_axis(int n, double gamma, int coarsenings) {
  std::vector<double> K, M;
  sipg_axis(n, gamma, true, K, M);
  for (int l = 0; l < coarsenings; ++l) galerkin_coarsen_axis(n >> l, K, M);
  return fdm_factor(K, M, 2 * (n >> coarsenings));
}

}  // namespace dcg
