// Host construction of the three-dimensional multigrid hierarchy (Section
// 4.2, the 3D case; layouts in mg3d.hpp): class tables of the level
// operators, the Galerkin products P^T L P (Algorithm 2), the RAS update
// tables and the coarsest inverse.
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "dcg3d.hpp"
#include "mg3d.hpp"

namespace dcg3 {

namespace {

constexpr int kOff[kSlots][3] = {{0, 0, 0}, {-1, 0, 0}, {1, 0, 0}, {0, -1, 0},
                                 {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};

struct Cube {
  int x, y, z;
};

bool inside(const Cube& c, int n) {
  return c.x >= 0 && c.y >= 0 && c.z >= 0 && c.x < n && c.y < n && c.z < n;
}

Cube shift(const Cube& c, int slot) {
  return {c.x + kOff[slot][0], c.y + kOff[slot][1], c.z + kOff[slot][2]};
}

// The slot of the face neighbour d - c, 0 for d = c, -1 otherwise.
int slot_of(const Cube& c, const Cube& d) {
  for (int s = 0; s < kSlots; ++s)
    if (c.x + kOff[s][0] == d.x && c.y + kOff[s][1] == d.y && c.z + kOff[s][2] == d.z) return s;
  return -1;
}

int64_t index(const Cube& c, int n) { return ((int64_t)c.z * n + c.y) * n + c.x; }

int op_axis(int x, int n) { return x == 0 ? 0 : (x == n - 1 ? 2 : 1); }
int op_class(const Cube& c, int n) { return op_axis(c.x, n) + 3 * op_axis(c.y, n) + 9 * op_axis(c.z, n); }

int ras_axis(int x, int n) { return x < 3 ? x : (n - 1 - x < 3 ? 6 - (n - 1 - x) : 3); }

// Entry (i, J) of the injection of a coarse trilinear function into child q
// of its cube: the coarse basis function J evaluated at fine corner i.
double inject(int q, int i, int J) {
  double v = 1.0;
  for (int ax = 0; ax < 3; ++ax) {
    const double t = 0.5 * (((q >> ax) & 1) + ((i >> ax) & 1));
    v *= ((J >> ax) & 1) ? t : 1.0 - t;
  }
  return v;
}

const double* op_block(const std::vector<double>& op, int cls, int slot) {
  return op.data() + ((size_t)cls * kSlots + slot) * 64;
}

// Cholesky factorisation of the SPD m x m matrix a (row-major, lower part
// overwritten by the factor); throws if a pivot is not positive.
void cholesky(std::vector<double>& a, int m) {
  for (int j = 0; j < m; ++j) {
    double d = a[(size_t)j * m + j];
    for (int k = 0; k < j; ++k) d -= a[(size_t)j * m + k] * a[(size_t)j * m + k];
    if (!(d > 0.0)) throw std::runtime_error("multigrid local problem is not positive definite");
    d = std::sqrt(d);
    a[(size_t)j * m + j] = d;
    for (int i = j + 1; i < m; ++i) {
      double s = a[(size_t)i * m + j];
      for (int k = 0; k < j; ++k) s -= a[(size_t)i * m + k] * a[(size_t)j * m + k];
      a[(size_t)i * m + j] = s / d;
    }
  }
}

// Solves (G G^T) x = b in place with the factor of cholesky().
void cho_solve(const std::vector<double>& g, int m, double* b) {
  for (int i = 0; i < m; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= g[(size_t)i * m + k] * b[k];
    b[i] = s / g[(size_t)i * m + i];
  }
  for (int i = m - 1; i >= 0; --i) {
    double s = b[i];
    for (int k = i + 1; k < m; ++k) s -= g[(size_t)k * m + i] * b[k];
    b[i] = s / g[(size_t)i * m + i];
  }
}

// Class table of the finest level from the per-cube blocks, with the check
// that every cube of a class carries the same blocks bit for bit.
std::vector<double> finest_classes(int n, const std::vector<double>& ld) {
  const int64_t ne = (int64_t)n * n * n;
  std::vector<double> op((size_t)kOpClasses * kSlots * 64, 0.0);
  std::vector<char> seen(kOpClasses, 0);
  double blk[kSlots * 64];
  for (int z = 0; z < n; ++z)
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        const Cube c{x, y, z};
        const int64_t e = index(c, n);
        for (int s = 0; s < kSlots; ++s)
          for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b) blk[s * 64 + a * 8 + b] = ld[((size_t)s * ne + e) * 64 + b * 8 + a];
        const int cls = op_class(c, n);
        double* dst = op.data() + (size_t)cls * kSlots * 64;
        if (!seen[cls]) {
          std::memcpy(dst, blk, sizeof(blk));
          seen[cls] = 1;
        } else if (std::memcmp(dst, blk, sizeof(blk)) != 0) {
          throw std::runtime_error("Laplacian blocks differ inside a boundary class");
        }
      }
  return op;
}

// The blocks of coarse cube E of P^T L P: every pair (child c of E, face
// slot t of c) whose neighbour exists adds P_q^T L[c][t] P_q' to the block
// of the coarse slot that holds the neighbour's parent.
void galerkin_cube(const std::vector<double>& fop, int nf, const Cube& E, double out[kSlots * 64]) {
  std::memset(out, 0, sizeof(double) * kSlots * 64);
  for (int q = 0; q < 8; ++q) {
    const Cube c{2 * E.x + (q & 1), 2 * E.y + ((q >> 1) & 1), 2 * E.z + (q >> 2)};
    const int fcls = op_class(c, nf);
    for (int t = 0; t < kSlots; ++t) {
      const Cube d = shift(c, t);
      if (!inside(d, nf)) continue;
      const Cube D{d.x >> 1, d.y >> 1, d.z >> 1};
      const int s = slot_of(E, D);
      const int q2 = (d.x & 1) | ((d.y & 1) << 1) | ((d.z & 1) << 2);
      const double* L = op_block(fop, fcls, t);
      double T[8][8];   // L P_q2
      for (int i = 0; i < 8; ++i)
        for (int J = 0; J < 8; ++J) {
          double acc = 0.0;
          for (int j = 0; j < 8; ++j) acc += L[i * 8 + j] * inject(q2, j, J);
          T[i][J] = acc;
        }
      double* B = out + s * 64;
      for (int I = 0; I < 8; ++I)
        for (int J = 0; J < 8; ++J) {
          double acc = 0.0;
          for (int i = 0; i < 8; ++i) acc += inject(q, i, I) * T[i][J];
          B[I * 8 + J] += acc;
        }
    }
  }
}

std::vector<double> coarse_classes(const std::vector<double>& fop, int nc) {
  const int nf = 2 * nc;
  std::vector<double> op((size_t)kOpClasses * kSlots * 64, 0.0);
  std::vector<char> seen(kOpClasses, 0);
  double blk[kSlots * 64];
  const bool check_all = nc <= 8;   // small levels: every cube against its class
  for (int z = 0; z < nc; ++z)
    for (int y = 0; y < nc; ++y)
      for (int x = 0; x < nc; ++x) {
        const Cube E{x, y, z};
        const int cls = op_class(E, nc);
        if (seen[cls] && !check_all) continue;
        galerkin_cube(fop, nf, E, blk);
        double* dst = op.data() + (size_t)cls * kSlots * 64;
        if (!seen[cls]) {
          std::memcpy(dst, blk, sizeof(blk));
          seen[cls] = 1;
        } else if (std::memcmp(dst, blk, sizeof(blk)) != 0) {
          throw std::runtime_error("Galerkin blocks differ inside a boundary class");
        }
      }
  return op;
}

// The RAS update table of one level: for a representative cube of every
// class, the sum over the blocks holding it (its own and those of its face
// neighbours) of D (A_b^{-1} R_b r) restricted to the cube, as a map from r
// on the diamond.
std::vector<double> ras_classes(const std::vector<double>& op, int n) {
  int off[kDiamond][3];
  diamond_offsets(off);
  auto diamond_index = [&](int dx, int dy, int dz) {
    for (int d = 0; d < kDiamond; ++d)
      if (off[d][0] == dx && off[d][1] == dy && off[d][2] == dz) return d;
    throw std::runtime_error("cube outside the diamond");
  };
  std::vector<double> ras((size_t)kRasClasses * 8 * kRasCols, 0.0);
  // representatives: per axis the first coordinate of each distance class,
  // or on small levels every coordinate (one class per cube)
  const bool per_cube = n < kRasClassMinN;
  const int np = per_cube ? n : 7;
  std::vector<int> rep(np, -1);
  for (int p = 0; p < np; ++p)
    for (int x = 0; x < n; ++x)
      if ((per_cube ? x : ras_axis(x, n)) == p) {
        rep[p] = x;
        break;
      }
  std::vector<double> A, X;
  for (int pz = 0; pz < np; ++pz)
    for (int py = 0; py < np; ++py)
      for (int px = 0; px < np; ++px) {
        if (rep[px] < 0 || rep[py] < 0 || rep[pz] < 0) continue;
        const Cube c{rep[px], rep[py], rep[pz]};
        const int cls = px + np * py + np * np * pz;
        double* K = ras.data() + (size_t)cls * 8 * kRasCols;
        int count = 1;
        for (int s = 1; s < kSlots; ++s) count += inside(shift(c, s), n);
        const double w = 1.0 / count;
        for (int sb = 0; sb < kSlots; ++sb) {
          const Cube b = shift(c, sb);
          if (!inside(b, n)) continue;
          std::vector<Cube> cubes{b};
          for (int s = 1; s < kSlots; ++s)
            if (inside(shift(b, s), n)) cubes.push_back(shift(b, s));
          const int nb = (int)cubes.size(), m = 8 * nb;
          A.assign((size_t)m * m, 0.0);
          int ic = -1;
          for (int i = 0; i < nb; ++i) {
            if (cubes[i].x == c.x && cubes[i].y == c.y && cubes[i].z == c.z) ic = i;
            const int cls = op_class(cubes[i], n);
            for (int j = 0; j < nb; ++j) {
              const int s = slot_of(cubes[i], cubes[j]);
              if (s < 0) continue;
              const double* L = op_block(op, cls, s);
              for (int a = 0; a < 8; ++a)
                for (int bb = 0; bb < 8; ++bb) A[(size_t)(8 * i + a) * m + 8 * j + bb] = L[a * 8 + bb];
            }
          }
          cholesky(A, m);
          // columns of A_b^{-1} for the cube's dofs = its rows (A_b symmetric)
          X.assign((size_t)m, 0.0);
          for (int a = 0; a < 8; ++a) {
            std::fill(X.begin(), X.end(), 0.0);
            X[8 * ic + a] = 1.0;
            cho_solve(A, m, X.data());
            for (int j = 0; j < nb; ++j) {
              const int d = diamond_index(cubes[j].x - c.x, cubes[j].y - c.y, cubes[j].z - c.z);
              for (int bb = 0; bb < 8; ++bb) K[a * kRasCols + 8 * d + bb] += w * X[8 * j + bb];
            }
          }
        }
      }
  return ras;
}

std::vector<double> coarsest_inverse(const std::vector<double>& op, int n) {
  const int64_t ne = (int64_t)n * n * n;
  const int m = int(8 * ne);
  std::vector<double> A((size_t)m * m, 0.0);
  for (int z = 0; z < n; ++z)
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        const Cube c{x, y, z};
        const int cls = op_class(c, n);
        for (int s = 0; s < kSlots; ++s) {
          const Cube d = shift(c, s);
          if (!inside(d, n)) continue;
          const double* L = op_block(op, cls, s);
          for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b)
              A[(size_t)(8 * index(c, n) + a) * m + 8 * index(d, n) + b] = L[a * 8 + b];
        }
      }
  cholesky(A, m);
  std::vector<double> inv((size_t)m * m), col(m);
  for (int j = 0; j < m; ++j) {
    std::fill(col.begin(), col.end(), 0.0);
    col[j] = 1.0;
    cho_solve(A, m, col.data());
    for (int i = 0; i < m; ++i) inv[(size_t)i * m + j] = col[i];
  }
  return inv;
}

}  // namespace

void diamond_offsets(int off[kDiamond][3]) {
  int d = 0;
  for (int dz = -2; dz <= 2; ++dz)
    for (int dy = -2; dy <= 2; ++dy)
      for (int dx = -2; dx <= 2; ++dx)
        if (std::abs(dx) + std::abs(dy) + std::abs(dz) <= 2) {
          off[d][0] = dx;
          off[d][1] = dy;
          off[d][2] = dz;
          ++d;
        }
}

std::vector<double> rows_fastest(const std::vector<double>& t, int cols) {
  const size_t per = (size_t)8 * cols, nc = t.size() / per;
  std::vector<double> out(t.size());
  for (size_t c = 0; c < nc; ++c)
    for (int a = 0; a < 8; ++a)
      for (int j = 0; j < cols; ++j) out[c * per + (size_t)j * 8 + a] = t[c * per + (size_t)a * cols + j];
  return out;
}

std::vector<double> op_rows_fastest(const std::vector<double>& op) {
  std::vector<double> out(op.size());
  for (size_t blk = 0; blk < op.size() / 64; ++blk)
    for (int a = 0; a < 8; ++a)
      for (int b = 0; b < 8; ++b) out[blk * 64 + b * 8 + a] = op[blk * 64 + a * 8 + b];
  return out;
}

int mg3_num_levels(int n, int levels) {
  if (n < 2) return 0;
  if (levels <= 0) {
    int J = 1, c = n;
    while (c % 2 == 0 && c / 2 >= 2) {
      c /= 2;
      ++J;
    }
    return c <= kMaxCoarsest ? J : 0;
  }
  if (levels > 30 || n % (1 << (levels - 1))) return 0;
  const int c = n >> (levels - 1);
  return c >= 2 && c <= kMaxCoarsest ? levels : 0;
}

Mg3Hierarchy build_mg3(int n, int J, const std::vector<double>& ld) {
  Mg3Hierarchy H;
  H.lev.resize(J);
  H.lev[J - 1].n = n;
  H.lev[J - 1].op = finest_classes(n, ld);
  for (int k = J - 1; k >= 1; --k) {
    const int nc = H.lev[k].n / 2;
    H.lev[k - 1].n = nc;
    H.lev[k - 1].op = coarse_classes(H.lev[k].op, nc);
  }
  for (int k = 1; k < J; ++k) H.lev[k].ras = ras_classes(H.lev[k].op, H.lev[k].n);
  H.coarse_inv = coarsest_inverse(H.lev[0].op, H.lev[0].n);
  return H;
}

}  // namespace dcg3
