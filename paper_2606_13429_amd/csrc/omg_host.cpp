// Host construction of the hierarchy of A* for the outer multigrid
// preconditioner (layouts in omg.hpp): class tables of the level operators,
// the Galerkin products P^T A* P (Algorithm 2's rule), the RAS update tables
// of Section 4.2 and the coarsest inverse.
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <vector>

#include "host_setup.hpp"
#include "omg.hpp"

namespace dcg {

namespace {

constexpr int D = kOmgDofs;
constexpr int kOff[kSlots][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, -1}, {0, 1}};

struct Sq {
  int x, y;
};

bool inside(const Sq& c, int n) { return c.x >= 0 && c.y >= 0 && c.x < n && c.y < n; }
Sq shift(const Sq& c, int s) { return {c.x + kOff[s][0], c.y + kOff[s][1]}; }
int slot_of(const Sq& c, const Sq& d) {
  for (int s = 0; s < kSlots; ++s)
    if (c.x + kOff[s][0] == d.x && c.y + kOff[s][1] == d.y) return s;
  return -1;
}
int op_axis(int x, int n) { return x == 0 ? 0 : (x == n - 1 ? 2 : 1); }
int op_class(const Sq& c, int n) { return op_axis(c.x, n) + 3 * op_axis(c.y, n); }
int ras_axis(int x, int n) { return x < 3 ? x : (n - 1 - x < 3 ? 6 - (n - 1 - x) : 3); }

// The scalar injection of child q (q = qx + 2 qy) of a coarse square: the
// coarse corner function J evaluated at fine corner i.
double inject(int q, int i, int J) {
  double v = 1.0;
  for (int ax = 0; ax < 2; ++ax) {
    const double t = 0.5 * (((q >> ax) & 1) + ((i >> ax) & 1));
    v *= ((J >> ax) & 1) ? t : 1.0 - t;
  }
  return v;
}

const double* blk(const std::vector<double>& op, int cls, int slot) {
  return op.data() + ((size_t)cls * kSlots + slot) * D * D;
}

void cholesky(std::vector<double>& a, int m) {
  for (int j = 0; j < m; ++j) {
    double d = a[(size_t)j * m + j];
    for (int k = 0; k < j; ++k) d -= a[(size_t)j * m + k] * a[(size_t)j * m + k];
    if (!(d > 0.0)) throw std::runtime_error("outer multigrid: local problem not positive definite");
    d = std::sqrt(d);
    a[(size_t)j * m + j] = d;
    for (int i = j + 1; i < m; ++i) {
      double s = a[(size_t)i * m + j];
      for (int k = 0; k < j; ++k) s -= a[(size_t)i * m + k] * a[(size_t)j * m + k];
      a[(size_t)i * m + j] = s / d;
    }
  }
}

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

// Blocks of coarse square E of P^T A P, every component injected alike.
void galerkin_square(const std::vector<double>& fop, int nf, const Sq& E, double* out) {
  std::memset(out, 0, sizeof(double) * kSlots * D * D);
  for (int q = 0; q < 4; ++q) {
    const Sq c{2 * E.x + (q & 1), 2 * E.y + (q >> 1)};
    const int fcls = op_class(c, nf);
    for (int t = 0; t < kSlots; ++t) {
      const Sq d = shift(c, t);
      if (!inside(d, nf)) continue;
      const Sq P{d.x >> 1, d.y >> 1};
      const int s = slot_of(E, P);
      const int q2 = (d.x & 1) | ((d.y & 1) << 1);
      const double* A = blk(fop, fcls, t);
      double* B = out + s * D * D;
      for (int c1 = 0; c1 < 4; ++c1)
        for (int c2 = 0; c2 < 4; ++c2) {
          double T[4][4];   // A[c1][c2] P_q2
          for (int i = 0; i < 4; ++i)
            for (int J = 0; J < 4; ++J) {
              double acc = 0.0;
              for (int j = 0; j < 4; ++j) acc += A[(4 * c1 + i) * D + 4 * c2 + j] * inject(q2, j, J);
              T[i][J] = acc;
            }
          for (int I = 0; I < 4; ++I)
            for (int J = 0; J < 4; ++J) {
              double acc = 0.0;
              for (int i = 0; i < 4; ++i) acc += inject(q, i, I) * T[i][J];
              B[(4 * c1 + I) * D + 4 * c2 + J] += acc;
            }
        }
    }
  }
}

std::vector<double> coarse_classes(const std::vector<double>& fop, int nc) {
  std::vector<double> op((size_t)kOmgOpClasses * kSlots * D * D, 0.0);
  std::vector<char> seen(kOmgOpClasses, 0);
  std::vector<double> b(kSlots * D * D);
  for (int y = 0; y < nc; ++y)
    for (int x = 0; x < nc; ++x) {
      const Sq E{x, y};
      const int cls = op_class(E, nc);
      if (seen[cls] && nc > 16) continue;     // small levels: every square checked
      galerkin_square(fop, 2 * nc, E, b.data());
      double* dst = op.data() + (size_t)cls * kSlots * D * D;
      if (!seen[cls]) {
        std::memcpy(dst, b.data(), b.size() * sizeof(double));
        seen[cls] = 1;
      } else if (std::memcmp(dst, b.data(), b.size() * sizeof(double)) != 0) {
        throw std::runtime_error("outer multigrid: Galerkin blocks differ inside a boundary class");
      }
    }
  return op;
}

std::vector<double> ras_classes(const std::vector<double>& op, int n) {
  int off[kOmgDiamond][2];
  omg_diamond(off);
  auto dindex = [&](int dx, int dy) {
    for (int d = 0; d < kOmgDiamond; ++d)
      if (off[d][0] == dx && off[d][1] == dy) return d;
    throw std::runtime_error("square outside the diamond");
  };
  std::vector<double> ras((size_t)kOmgRasClasses * D * kOmgRasCols, 0.0);
  const bool per_square = n < kOmgRasClassMinN;
  const int np = per_square ? n : 7;
  std::vector<int> rep(np, -1);
  for (int p = 0; p < np; ++p)
    for (int x = 0; x < n; ++x)
      if ((per_square ? x : ras_axis(x, n)) == p) {
        rep[p] = x;
        break;
      }
  std::vector<double> A, X;
  for (int py = 0; py < np; ++py)
    for (int px = 0; px < np; ++px) {
      if (rep[px] < 0 || rep[py] < 0) continue;
      const Sq c{rep[px], rep[py]};
      double* K = ras.data() + (size_t)(px + np * py) * D * kOmgRasCols;
      int count = 1;
      for (int s = 1; s < kSlots; ++s) count += inside(shift(c, s), n);
      const double w = 1.0 / count;
      for (int sb = 0; sb < kSlots; ++sb) {
        const Sq b = shift(c, sb);
        if (!inside(b, n)) continue;
        std::vector<Sq> sq{b};
        for (int s = 1; s < kSlots; ++s)
          if (inside(shift(b, s), n)) sq.push_back(shift(b, s));
        const int nb = (int)sq.size(), m = D * nb;
        A.assign((size_t)m * m, 0.0);
        int ic = -1;
        for (int i = 0; i < nb; ++i) {
          if (sq[i].x == c.x && sq[i].y == c.y) ic = i;
          const int cls = op_class(sq[i], n);
          for (int j = 0; j < nb; ++j) {
            const int s = slot_of(sq[i], sq[j]);
            if (s < 0) continue;
            const double* L = blk(op, cls, s);
            for (int a = 0; a < D; ++a)
              for (int bb = 0; bb < D; ++bb) A[(size_t)(D * i + a) * m + D * j + bb] = L[a * D + bb];
          }
        }
        cholesky(A, m);
        X.assign(m, 0.0);
        for (int a = 0; a < D; ++a) {   // row a of A_b^{-1} on the square = column a (symmetric)
          std::fill(X.begin(), X.end(), 0.0);
          X[D * ic + a] = 1.0;
          cho_solve(A, m, X.data());
          for (int j = 0; j < nb; ++j) {
            const int d = dindex(sq[j].x - c.x, sq[j].y - c.y);
            for (int bb = 0; bb < D; ++bb) K[a * kOmgRasCols + D * d + bb] += w * X[D * j + bb];
          }
        }
      }
    }
  return ras;
}

std::vector<double> coarsest_inverse(const std::vector<double>& op, int n) {
  const int m = D * n * n;
  std::vector<double> A((size_t)m * m, 0.0);
  for (int y = 0; y < n; ++y)
    for (int x = 0; x < n; ++x) {
      const Sq c{x, y};
      const int cls = op_class(c, n);
      for (int s = 0; s < kSlots; ++s) {
        const Sq d = shift(c, s);
        if (!inside(d, n)) continue;
        const double* L = blk(op, cls, s);
        const int ec = y * n + x, ed = d.y * n + d.x;
        for (int a = 0; a < D; ++a)
          for (int b = 0; b < D; ++b) A[(size_t)(D * ec + a) * m + D * ed + b] = L[a * D + b];
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

void omg_diamond(int off[kOmgDiamond][2]) {
  int d = 0;
  for (int dy = -2; dy <= 2; ++dy)
    for (int dx = -2; dx <= 2; ++dx)
      if (std::abs(dx) + std::abs(dy) <= 2) {
        off[d][0] = dx;
        off[d][1] = dy;
        ++d;
      }
}

std::vector<double> omg_operand_order(const std::vector<double>& tab, int classes, int cols) {
  if (cols % 4 || tab.size() != (size_t)classes * D * cols)
    throw std::runtime_error("outer multigrid: table shape does not fit the operand order");
  const int steps = cols / 4;
  std::vector<double> out(tab.size());
  for (int c = 0; c < classes; ++c)
    for (int s = 0; s < steps; ++s)
      for (int l = 0; l < 64; ++l)
        out[((size_t)c * steps + s) * 64 + l] = tab[((size_t)c * D + l % 16) * cols + 4 * s + l / 16];
  return out;
}

std::vector<double> omg_op_rows(const std::vector<double>& op) {
  if (op.size() != (size_t)kOmgOpClasses * kSlots * D * D)
    throw std::runtime_error("outer multigrid: operator table of the wrong size");
  std::vector<double> out(op.size());
  for (int c = 0; c < kOmgOpClasses; ++c)
    for (int s = 0; s < kSlots; ++s)
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b)
          out[((size_t)c * D + a) * kOmgOpCols + D * s + b] = op[(((size_t)c * kSlots + s) * D + a) * D + b];
  return out;
}

int omg_num_levels(int n) {
  if (n < 2 * kOmgCoarsest || n % kOmgCoarsest) return 0;
  int r = n / kOmgCoarsest, J = 1;
  while (r > 1) {
    if (r & 1) return 0;
    r >>= 1;
    ++J;
  }
  return J;
}

OmgHierarchy build_omg(int n, double penalty, double dt, double nu) {
  const int J = omg_num_levels(n);
  if (J < 2) throw std::runtime_error("outer multigrid needs n = 8 * 2^k >= 16");
  OmgHierarchy H;
  H.lev.resize(J);
  H.lev[J - 1].n = n;
  astar_class_blocks(n, penalty, dt, nu, H.lev[J - 1].op);
  for (int k = J - 1; k >= 1; --k) {
    H.lev[k - 1].n = H.lev[k].n / 2;
    H.lev[k - 1].op = coarse_classes(H.lev[k].op, H.lev[k - 1].n);
  }
  for (int k = 1; k < J; ++k) H.lev[k].ras = ras_classes(H.lev[k].op, H.lev[k].n);
  H.coarse_inv = coarsest_inverse(H.lev[0].op, H.lev[0].n);
  return H;
}

}  // namespace dcg
