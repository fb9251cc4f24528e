// Host-side construction of the mesh context (see host_setup.hpp).
//
// Discretisation (paper Section 3.3.2 specialised to DG-Q1 on squares):
//   a^h_ij(s, t) = sum_K int d_i s d_j t
//                 - sum_F int ({d_i s} [[t]]_j + {d_j t} [[s]]_i)
//                 + sum_F gamma int [[s]]_i [[t]]_j,
// F ranging over interior faces and traction-boundary faces {x=0} u {y=0};
// [[v]]_i = sum over the sides of v n_i, {.} the mean of the traces (the
// single trace on a boundary face); gamma = penalty / h.  The flux term pairs
// the scalar average with one component of the vector jump, which makes
// sum_ij a_ij(s_ki, t_kj) the normal-jump SIPG form of (div s_k, div t_k).
// A_div = sum_{k,i,j} a_ij(sigma_ki, tau_kj) (eq. (component_form)); the
// unknown of square e is [sigma_11 sigma_12 sigma_21 sigma_22] x 4 corners.
#include "host_setup.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <thread>
#include <unordered_map>

namespace dcg {
namespace {

const double kGauss0 = (1.0 - 1.0 / std::sqrt(3.0)) / 2.0;
const double kGauss[2] = {kGauss0, 1.0 - kGauss0};
const double kGaussW[2] = {0.5, 0.5};
const double kInvSqrt2 = 0.70710678118654752440;

inline double lin(int i, double t) { return i ? t : 1.0 - t; }
inline double dlin(int i) { return i ? 1.0 : -1.0; }
inline double q1(int j, double xi, double eta) { return lin(j & 1, xi) * lin(j >> 1, eta); }
inline void q1_grad(int j, double xi, double eta, double h, double g[2]) {
  g[0] = dlin(j & 1) * lin(j >> 1, eta) / h;
  g[1] = lin(j & 1, xi) * dlin(j >> 1) / h;
}

// S[i][j][a][b]: volume part of a_ij(phi_b, phi_a) (test a, trial b).
struct Vol {
  double s[2][2][4][4];
};

Vol volume_forms(double h) {
  Vol v{};
  for (int qy = 0; qy < 2; ++qy)
    for (int qx = 0; qx < 2; ++qx) {
      double g[4][2];
      for (int a = 0; a < 4; ++a) q1_grad(a, kGauss[qx], kGauss[qy], h, g[a]);
      const double w = kGaussW[qx] * kGaussW[qy] * h * h;
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
          for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) v.s[i][j][a][b] += w * g[b][i] * g[a][j];
    }
  return v;
}

// One side of a face: the reference coordinate held fixed and the outward
// normal of that square.
struct Side {
  int fixed_axis;    // 0: xi = value, eta = g ; 1: eta = value, xi = g
  double value;
  double nrm[2];
};

// F[i][j][sa][sb][a][b]: face part of a_ij with the test function on side sa
// (corner a) and the trial function on side sb (corner b).
struct Face {
  int sides = 0;
  double f[2][2][2][2][4][4];
};

Face face_forms(const Side* sd, int ns, double h, double gamma) {
  Face F{};
  F.sides = ns;
  const double avg = ns == 2 ? 0.5 : 1.0;
  for (int q = 0; q < 2; ++q) {
    const double wq = kGaussW[q] * h;
    double val[2][4], grd[2][4][2];
    for (int s = 0; s < ns; ++s) {
      const double xi = sd[s].fixed_axis == 0 ? sd[s].value : kGauss[q];
      const double eta = sd[s].fixed_axis == 0 ? kGauss[q] : sd[s].value;
      for (int a = 0; a < 4; ++a) {
        val[s][a] = q1(a, xi, eta);
        q1_grad(a, xi, eta, h, grd[s][a]);
      }
    }
    for (int st = 0; st < ns; ++st)
      for (int ss = 0; ss < ns; ++ss)
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j)
            for (int a = 0; a < 4; ++a)
              for (int b = 0; b < 4; ++b) {
                const double jt = val[st][a] * sd[st].nrm[j];   // [[t]]_j
                const double js = val[ss][b] * sd[ss].nrm[i];   // [[s]]_i
                const double term = -avg * grd[ss][b][i] * jt - avg * grd[st][a][j] * js +
                                    gamma * js * jt;
                F.f[i][j][st][ss][a][b] += wq * term;
              }
  }
  return F;
}

// Adds the scalar forms (for every row k of the tensor) into a 16 x 16
// block: row 4 (2k + j) + a (test tau_kj, corner a), column 4 (2k + i) + b.
template <typename Src>
void add_tensor_block(double* blk, const Src& src) {
  for (int k = 0; k < 2; ++k)
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < 4; ++b)
            blk[(4 * (2 * k + j) + a) * 16 + 4 * (2 * k + i) + b] += src(i, j, a, b);
}

// Runs fn(i) for i in [0, count) on up to 16 threads (serially below
// ``serial_below`` items).  fn must not throw.
template <typename Fn>
void parallel_for(int64_t count, Fn fn, int64_t serial_below = 4096) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (count < serial_below) nt = 1;
  if (int64_t(nt) > count) nt = unsigned(std::max<int64_t>(1, count));
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([=, &fn]() {
      const int64_t lo = count * t / nt, hi = count * (t + 1) / nt;
      for (int64_t i = lo; i < hi; ++i) fn(i);
    });
  for (auto& x : th) x.join();
}

void set_cols(int n, std::vector<int32_t>& cols) {
  const int64_t ne = int64_t(n) * n;
  cols.assign(ne * kSlots, -1);
  for (int ey = 0; ey < n; ++ey)
    for (int ex = 0; ex < n; ++ex) {
      const int64_t e = int64_t(ey) * n + ex;
      int32_t* c = &cols[e * kSlots];
      c[0] = int32_t(e);
      if (ex > 0) c[1] = int32_t(e - 1);
      if (ex < n - 1) c[2] = int32_t(e + 1);
      if (ey > 0) c[3] = int32_t(e - n);
      if (ey < n - 1) c[4] = int32_t(e + n);
    }
}

// Dense SPD inverse through the Cholesky factor A = C C^T:
// W = C^{-1}, A^{-1} = W^T W.  Returns false if A is not positive definite.
bool spd_inverse(int n, const double* A, double* inv, int threads) {
  std::vector<double> C(size_t(n) * n, 0.0), W(size_t(n) * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = A[size_t(j) * n + j];
    for (int k = 0; k < j; ++k) d -= C[size_t(j) * n + k] * C[size_t(j) * n + k];
    if (!(d > 0.0)) return false;
    const double cjj = std::sqrt(d);
    C[size_t(j) * n + j] = cjj;
    for (int i = j + 1; i < n; ++i) {
      double s = A[size_t(i) * n + j];
      const double* ci = &C[size_t(i) * n];
      const double* cj = &C[size_t(j) * n];
      for (int k = 0; k < j; ++k) s -= ci[k] * cj[k];
      C[size_t(i) * n + j] = s / cjj;
    }
  }
  auto column = [&](int j) {           // column j of W = C^{-1}
    W[size_t(j) * n + j] = 1.0 / C[size_t(j) * n + j];
    for (int i = j + 1; i < n; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += C[size_t(i) * n + k] * W[size_t(k) * n + j];
      W[size_t(i) * n + j] = -s / C[size_t(i) * n + i];
    }
  };
  auto row = [&](int i) {              // row i of W^T W
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = std::max(i, j); k < n; ++k) s += W[size_t(k) * n + i] * W[size_t(k) * n + j];
      inv[size_t(i) * n + j] = s;
    }
  };
  if (threads <= 1) {
    for (int j = 0; j < n; ++j) column(j);
    for (int i = 0; i < n; ++i) row(i);
  } else {
    std::vector<std::thread> th;
    for (int t = 0; t < threads; ++t)
      th.emplace_back([&, t]() { for (int j = t; j < n; j += threads) column(j); });
    for (auto& x : th) x.join();
    th.clear();
    for (int t = 0; t < threads; ++t)
      th.emplace_back([&, t]() { for (int i = t; i < n; i += threads) row(i); });
    for (auto& x : th) x.join();
  }
  return true;
}

uint64_t fnv1a(const void* p, size_t bytes, uint64_t h = 1469598103934665603ull) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < bytes; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

// P_c[a][A]: coefficient of coarse corner A at fine corner a of child c
// (c = cx + 2 cy): the coarse bilinear function at ((cx + ax)/2, (cy + ay)/2).
void child_prolongation(double P[4][4][4]) {
  for (int c = 0; c < 4; ++c)
    for (int a = 0; a < 4; ++a) {
      const double xi = ((c & 1) + (a & 1)) * 0.5, eta = ((c >> 1) + (a >> 1)) * 0.5;
      for (int A = 0; A < 4; ++A) P[c][a][A] = lin(A & 1, xi) * lin(A >> 1, eta);
    }
}

void galerkin_coarsen(const HostLevel& f, HostLevel& c) {
  const int nf = f.n, nc = nf / 2;
  c.n = nc;
  set_cols(nc, c.cols);
  const int64_t nec = int64_t(nc) * nc;
  c.L.assign(nec * kSlots * 16, 0.0);
  double P[4][4][4];
  child_prolongation(P);
  parallel_for(nec, [&](int64_t E) {
    const int EX = int(E % nc), EY = int(E / nc);
    for (int ch = 0; ch < 4; ++ch) {
      const int ex = 2 * EX + (ch & 1), ey = 2 * EY + (ch >> 1);
      const int64_t e = int64_t(ey) * nf + ex;
      for (int s = 0; s < kSlots; ++s) {
        const int32_t e2 = f.cols[e * kSlots + s];
        if (e2 < 0) continue;
        const int ex2 = e2 % nf, ey2 = e2 / nf;
        const int EX2 = ex2 / 2, EY2 = ey2 / 2;
        const int ch2 = (ex2 & 1) + 2 * (ey2 & 1);
        int cs;
        if (EX2 == EX && EY2 == EY) cs = 0;
        else if (EX2 == EX - 1) cs = 1;
        else if (EX2 == EX + 1) cs = 2;
        else if (EY2 == EY - 1) cs = 3;
        else cs = 4;
        const double* Lf = &f.L[(e * kSlots + s) * 16];
        double* Lc = &c.L[(E * kSlots + cs) * 16];
        // Lc += P_ch^T Lf P_ch2
        double tmp[4][4];
        for (int a = 0; a < 4; ++a)
          for (int B = 0; B < 4; ++B) {
            double acc = 0.0;
            for (int b = 0; b < 4; ++b) acc += Lf[a * 4 + b] * P[ch2][b][B];
            tmp[a][B] = acc;
          }
        for (int A = 0; A < 4; ++A)
          for (int B = 0; B < 4; ++B) {
            double acc = 0.0;
            for (int a = 0; a < 4; ++a) acc += P[ch][a][A] * tmp[a][B];
            Lc[A * 4 + B] += acc;
          }
      }
    }
  });
}

void build_tiles(HostLevel& lv) {
  const int n = lv.n;
  if (n % kTileCore) throw std::runtime_error("level not divisible into 4 x 4 tiles");
  const int tpr = n / kTileCore;
  lv.tiles = tpr * tpr;
  const int64_t ne = int64_t(n) * n;
  lv.tile_elems.assign(int64_t(lv.tiles) * kTileSlots, -1);
  lv.tile_ext.assign(int64_t(lv.tiles) * kTileExt, -1);
  std::vector<int32_t> count(ne, 0);
  auto elem = [&](int ex, int ey) -> int32_t {
    return (ex < 0 || ey < 0 || ex >= n || ey >= n) ? -1 : int32_t(int64_t(ey) * n + ex);
  };
  for (int b = 0; b < tpr; ++b)
    for (int a = 0; a < tpr; ++a) {
      int32_t* te = &lv.tile_elems[(int64_t(b) * tpr + a) * kTileSlots];
      const int x0 = kTileCore * a, y0 = kTileCore * b;
      for (int ly = 0; ly < 4; ++ly)
        for (int lx = 0; lx < 4; ++lx) te[ly * 4 + lx] = elem(x0 + lx, y0 + ly);
      for (int l = 0; l < 4; ++l) {
        te[16 + l] = elem(x0 - 1, y0 + l);   // left layer
        te[20 + l] = elem(x0 + 4, y0 + l);   // right layer
        te[24 + l] = elem(x0 + l, y0 - 1);   // bottom layer
        te[28 + l] = elem(x0 + l, y0 + 4);   // top layer
      }
      for (int s = 0; s < kTileSlots; ++s)
        if (te[s] >= 0) ++count[te[s]];
      // extended pattern: block slots, then the ring at distance 1 outside it
      int32_t* tx = &lv.tile_ext[(int64_t(b) * tpr + a) * kTileExt];
      for (int s = 0; s < kTileSlots; ++s) tx[s] = te[s];
      for (int l = 0; l < 4; ++l) {
        tx[32 + l] = elem(x0 - 2, y0 + l);
        tx[36 + l] = elem(x0 + 5, y0 + l);
        tx[40 + l] = elem(x0 + l, y0 - 2);
        tx[44 + l] = elem(x0 + l, y0 + 5);
      }
      tx[48] = elem(x0 - 1, y0 - 1);
      tx[49] = elem(x0 + 4, y0 - 1);
      tx[50] = elem(x0 - 1, y0 + 4);
      tx[51] = elem(x0 + 4, y0 + 4);
    }
  // cover lists in increasing tile order (fixed summation order of the update)
  lv.cover.assign(ne * 3, -1);
  std::vector<int8_t> fill(ne, 0);
  for (int t = 0; t < lv.tiles; ++t)
    for (int s = 0; s < kTileSlots; ++s) {
      const int32_t e = lv.tile_elems[int64_t(t) * kTileSlots + s];
      if (e < 0) continue;
      if (fill[e] >= 3) throw std::runtime_error("square in more than 3 RAS blocks");
      lv.cover[e * 3 + fill[e]++] = t * kTileSlots + s;
    }
  lv.dw.resize(ne);
  for (int64_t e = 0; e < ne; ++e) lv.dw[e] = 1.0 / count[e];
  lv.tile_dst.assign(int64_t(lv.tiles) * kTileSlots, -1);
  for (int64_t e = 0; e < ne; ++e)
    for (int k = 0; k < 3; ++k) {
      const int32_t c = lv.cover[e * 3 + k];
      if (c >= 0) lv.tile_dst[c] = int32_t(e * 3 + k);
    }
  // local matrices (L_k)_i = R_i L_k R_i^T and weights D_i; identical local
  // problems (bit for bit) share one inverse computation
  lv.tile_class.assign(lv.tiles, -1);
  lv.unique_inv.clear();
  std::vector<std::vector<double>> uniq_mat;
  std::unordered_map<uint64_t, std::vector<int>> seen;
  std::vector<double> Aloc(kTileDofs * kTileDofs + kTileDofs);
  for (int t = 0; t < lv.tiles; ++t) {
    std::fill(Aloc.begin(), Aloc.end(), 0.0);
    const int32_t* te = &lv.tile_elems[int64_t(t) * kTileSlots];
    double* dvec = &Aloc[kTileDofs * kTileDofs];
    for (int p = 0; p < kTileSlots; ++p) {
      const int32_t ep = te[p];
      if (ep < 0) {
        for (int a = 0; a < 4; ++a) Aloc[(4 * p + a) * kTileDofs + 4 * p + a] = 1.0;
        continue;
      }
      for (int a = 0; a < 4; ++a) dvec[4 * p + a] = 1.0 / count[ep];
      for (int s = 0; s < kSlots; ++s) {
        const int32_t e2 = lv.cols[int64_t(ep) * kSlots + s];
        if (e2 < 0) continue;
        int q = -1;
        for (int qq = 0; qq < kTileSlots; ++qq)
          if (te[qq] == e2) { q = qq; break; }
        if (q < 0) continue;
        const double* Lb = &lv.L[(int64_t(ep) * kSlots + s) * 16];
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < 4; ++b) Aloc[(4 * p + a) * kTileDofs + 4 * q + b] = Lb[a * 4 + b];
      }
    }
    const uint64_t key = fnv1a(Aloc.data(), Aloc.size() * sizeof(double));
    int cls = -1;
    auto it = seen.find(key);
    if (it != seen.end())
      for (int u : it->second)
        if (std::memcmp(uniq_mat[u].data(), Aloc.data(), Aloc.size() * sizeof(double)) == 0) {
          cls = u;
          break;
        }
    if (cls < 0) {
      cls = int(uniq_mat.size());
      uniq_mat.push_back(Aloc);
      seen[key].push_back(cls);
    }
    lv.tile_class[t] = cls;
  }
  lv.unique_inv.resize(uniq_mat.size());
  std::vector<char> ok(uniq_mat.size(), 0);
  parallel_for(int64_t(uniq_mat.size()), [&](int64_t u) {
    std::vector<double> inv(kTileDofs * kTileDofs);
    if (!spd_inverse(kTileDofs, uniq_mat[u].data(), inv.data(), 1)) return;
    lv.unique_inv[u] = std::move(inv);
    ok[u] = 1;
  }, 2);
  for (char o : ok)
    if (!o) throw std::runtime_error("RAS local matrix not positive definite");
}

// The element and face integrals of one mesh size, and the five 16 x 16
// A_div blocks of square (ex, ey) (slot order self, x-1, x+1, y-1, y+1;
// added into blk, which the caller zeroes).
struct SquareForms {
  Vol vol;
  Face Fv, Fh, Fl, Fb;
  double mass[16];
};

SquareForms square_forms(int n, double penalty) {
  const double h = 1.0 / n, gamma = penalty / h;
  SquareForms F;
  F.vol = volume_forms(h);
  const Side vert[2] = {{0, 1.0, {1.0, 0.0}}, {0, 0.0, {-1.0, 0.0}}};    // left | right
  const Side horz[2] = {{1, 1.0, {0.0, 1.0}}, {1, 0.0, {0.0, -1.0}}};    // lower | upper
  const Side left[1] = {{0, 0.0, {-1.0, 0.0}}};
  const Side bottom[1] = {{1, 0.0, {0.0, -1.0}}};
  F.Fv = face_forms(vert, 2, h, gamma);
  F.Fh = face_forms(horz, 2, h, gamma);
  F.Fl = face_forms(left, 1, h, gamma);
  F.Fb = face_forms(bottom, 1, h, gamma);
  std::memset(F.mass, 0, sizeof F.mass);
  for (int qy = 0; qy < 2; ++qy)
    for (int qx = 0; qx < 2; ++qx)
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
          F.mass[a * 4 + b] += kGaussW[qx] * kGaussW[qy] * h * h * q1(a, kGauss[qx], kGauss[qy]) *
                               q1(b, kGauss[qx], kGauss[qy]);
  return F;
}

void square_adiv(const SquareForms& F, int n, int ex, int ey, double* blk) {
  double* self = blk;
  auto face = [](const Face& Fc, int st, int ss) {
    return [&Fc, st, ss](int i, int j, int a, int b) { return Fc.f[i][j][st][ss][a][b]; };
  };
  add_tensor_block(self, [&](int i, int j, int a, int b) { return F.vol.s[i][j][a][b]; });
  if (ex > 0) {                                   // face x = ex h, e is the right side
    add_tensor_block(self, face(F.Fv, 1, 1));
    add_tensor_block(blk + 1 * 256, face(F.Fv, 1, 0));
  } else {
    add_tensor_block(self, face(F.Fl, 0, 0));     // traction boundary x = 0
  }
  if (ex < n - 1) {                               // face x = (ex+1) h, e is the left side
    add_tensor_block(self, face(F.Fv, 0, 0));
    add_tensor_block(blk + 2 * 256, face(F.Fv, 0, 1));
  }
  if (ey > 0) {                                   // face y = ey h, e is the upper side
    add_tensor_block(self, face(F.Fh, 1, 1));
    add_tensor_block(blk + 3 * 256, face(F.Fh, 1, 0));
  } else {
    add_tensor_block(self, face(F.Fb, 0, 0));     // traction boundary y = 0
  }
  if (ey < n - 1) {                               // face y = (ey+1) h, e is the lower side
    add_tensor_block(self, face(F.Fh, 0, 0));
    add_tensor_block(blk + 4 * 256, face(F.Fh, 0, 1));
  }
}

}  // namespace

int num_levels(int n) {
  if (n < kCoarsestN || n > 2048 || n % kCoarsestN) return -1;
  int r = n / kCoarsestN, J = 1;
  while (r > 1) {
    if (r & 1) return -1;
    r >>= 1;
    ++J;
  }
  return J;
}

void astar_class_blocks(int n, double penalty, double dt, double nu, std::vector<double>& out) {
  if (n < 3) throw std::runtime_error("n must be >= 3");
  const SquareForms F = square_forms(n, penalty);
  // the dev-dev coefficients of Section 3.1 (d = 2), components 11, 12, 21, 22
  const double C[4][4] = {{0.5, 0, 0, -0.5}, {0, 1, 0, 0}, {0, 0, 1, 0}, {-0.5, 0, 0, 0.5}};
  out.assign(9 * kSlots * 256, 0.0);
  const int pos[3] = {0, 1, n - 1};
  std::vector<double> adiv(kSlots * 256);
  for (int cy = 0; cy < 3; ++cy)
    for (int cx = 0; cx < 3; ++cx) {
      std::fill(adiv.begin(), adiv.end(), 0.0);
      square_adiv(F, n, pos[cx], pos[cy], adiv.data());
      double* blk = &out[(cx + 3 * cy) * kSlots * 256];
      for (int s = 0; s < kSlots; ++s)
        for (int i = 0; i < 256; ++i) blk[s * 256 + i] = dt * adiv[s * 256 + i];
      for (int c = 0; c < 4; ++c)
        for (int c2 = 0; c2 < 4; ++c2)
          if (C[c][c2] != 0.0)
            for (int a = 0; a < 4; ++a)
              for (int b = 0; b < 4; ++b)
                blk[(4 * c + a) * 16 + 4 * c2 + b] += C[c][c2] * F.mass[a * 4 + b] / nu;
    }
}

void build_host_context(int n, double penalty, bool with_tiles, bool with_coarse,
                        HostContext& out) {
  const int J = num_levels(n);
  if (J < 0) throw std::runtime_error("n must be 16 * 2^k, 16 <= n <= 2048");
  if (!(penalty > 0.0)) throw std::runtime_error("penalty must be positive");
  out = HostContext();
  out.n = n;
  out.J = J;
  out.penalty = penalty;
  const int64_t ne = int64_t(n) * n;
  const SquareForms F = square_forms(n, penalty);
  const double* mass = F.mass;

  set_cols(n, out.cols);
  out.Adiv.assign(ne * kSlots * 256, 0.0);
  out.AdivZ.assign(ne * kSlots * 64, 0.0);
  out.M1.resize(ne * 16);
  parallel_for(ne, [&](int64_t e) {
    const int ex = int(e % n), ey = int(e / n);
    square_adiv(F, n, ex, ey, &out.Adiv[e * kSlots * 256]);
    for (int s = 0; s < kSlots; ++s) {              // A_div Z: Z puts q / sqrt(2) in 11, 22
      const double* A = &out.Adiv[(e * kSlots + s) * 256];
      double* AZ = &out.AdivZ[(e * kSlots + s) * 64];
      for (int r = 0; r < 16; ++r)
        for (int b = 0; b < 4; ++b) AZ[r * 4 + b] = (A[r * 16 + b] + A[r * 16 + 12 + b]) * kInvSqrt2;
    }
    std::memcpy(&out.M1[e * 16], mass, sizeof F.mass);
  });

  // finest Laplacian L_J = 2 Z^T A_div Z (Corollary 1 with dt factored out)
  out.levels.resize(J);
  HostLevel& fine = out.levels[J - 1];
  fine.n = n;
  fine.cols = out.cols;
  fine.L.assign(ne * kSlots * 16, 0.0);
  parallel_for(ne, [&](int64_t e) {
    for (int s = 0; s < kSlots; ++s) {
      const double* A = &out.Adiv[(e * kSlots + s) * 256];
      double* L = &fine.L[(e * kSlots + s) * 16];
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
          L[a * 4 + b] = A[a * 16 + b] + A[a * 16 + 12 + b] + A[(12 + a) * 16 + b] +
                         A[(12 + a) * 16 + 12 + b];
    }
  });
  for (int k = J; k > 1; --k) galerkin_coarsen(out.levels[k - 1], out.levels[k - 2]);
  if (with_tiles)
    for (int k = 2; k <= J; ++k) build_tiles(out.levels[k - 1]);
  if (with_coarse) {
    const HostLevel& c = out.levels[0];
    std::vector<double> dense(size_t(kCoarseDofs) * kCoarseDofs, 0.0);
    for (int64_t e = 0; e < int64_t(c.n) * c.n; ++e)
      for (int s = 0; s < kSlots; ++s) {
        const int32_t e2 = c.cols[e * kSlots + s];
        if (e2 < 0) continue;
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < 4; ++b)
            dense[size_t(4 * e + a) * kCoarseDofs + 4 * e2 + b] = c.L[(e * kSlots + s) * 16 + a * 4 + b];
      }
    out.coarse_inv.resize(dense.size());
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (!spd_inverse(kCoarseDofs, dense.data(), out.coarse_inv.data(), int(nt)))
      throw std::runtime_error("coarsest operator not positive definite");
  }
}

}  // namespace dcg
