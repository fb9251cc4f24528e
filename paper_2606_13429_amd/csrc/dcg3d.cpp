// Three-dimensional deflated CG on the device (the d = 3 case of Section 3.1):
// host assembly of the DG-Q1 element blocks, the resident device context, the
// outer iteration of Algorithm 2 and the extern "C" entry points dcg3d_*.
//
// Discretisation: the unit cube in n^3 cubes of side h = 1/n, discontinuous
// Q1 per stress component, 2x2x2 Gauss in elements and 2x2 Gauss on faces,
// penalty gamma = penalty / h, SIPG face terms (Section 3.3.2, the component
// reading of jumps and averages) on interior faces and on the outflow face
// {x = 1}, where the three-dimensional test of Section 4.2 imposes sigma n = 0.
//
// Solve: deflated CG with V of eq. (Vmatrix) for d = 3 (called Z), whose
// inner system Z^T A* Z = (dt/3)(B_11 + B_22 + B_33) (Corollary 1) is solved
// exactly by fast diagonalisation, by the Multigrid iteration of Algorithm 3
// (W-cycles with the RAS smoother of Section 4.2, mg3d_*.{cpp,hip}) or by
// block-Jacobi preconditioned CG, the iterative ones to the relative
// tolerance of eq. (fixed_tol) or eq. (tol); every vector operation runs in
// the kernels of dcg3d_kernels.hip and mg3d_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <memory>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/dcg.h"
#include "dcg3d.hpp"
#include "fdm_host.hpp"
#include "mg3d.hpp"

namespace {

using dcg3::kDof;
using dcg3::kNb;
using dcg3::kSlots;

struct Err3 : std::runtime_error {
  dcg_status status;
  Err3(dcg_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

void hipck(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  (void)hipGetLastError();
  throw Err3(e == hipErrorOutOfMemory ? DCG_ENOMEM : DCG_EDEVICE,
             std::string(what) + ": " + hipGetErrorString(e));
}
#define H3(expr) hipck((expr), #expr)

thread_local std::string g_last_error3;

// ---------------------------------------------------------------------------
// element and face blocks of the uniform hexahedral grid
// ---------------------------------------------------------------------------
struct CubeForms {
  double mass[kNb][kNb];
  double vol[3][3][kNb][kNb];                 // [i][j][test a][trial b]
  double face[3][2][2][3][3][kNb][kNb];       // [axis][test side][trial side][i][j][a][b]
  double out[3][3][kNb][kNb];                 // the x = 1 face of Gamma_out, one side
};

double bval(int i, double t) { return i ? t : 1.0 - t; }
double bder(int i) { return i ? 1.0 : -1.0; }

// Values and physical gradients of the 8 trilinear corner functions.
void basis(const double p[3], double h, double v[kNb], double g[kNb][3]) {
  for (int j = 0; j < kNb; ++j) {
    const int c[3] = {j & 1, (j >> 1) & 1, j >> 2};
    const double b0 = bval(c[0], p[0]), b1 = bval(c[1], p[1]), b2 = bval(c[2], p[2]);
    v[j] = b0 * b1 * b2;
    g[j][0] = bder(c[0]) * b1 * b2 / h;
    g[j][1] = b0 * bder(c[1]) * b2 / h;
    g[j][2] = b0 * b1 * bder(c[2]) / h;
  }
}

void build_forms(int n, double penalty, CubeForms& F) {
  std::memset(&F, 0, sizeof(F));
  const double h = 1.0 / n, gamma = penalty / h;
  const double gp[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  // volume: 2x2x2 Gauss, weight h^3 / 8 per point
  for (int qz = 0; qz < 2; ++qz)
    for (int qy = 0; qy < 2; ++qy)
      for (int qx = 0; qx < 2; ++qx) {
        const double p[3] = {gp[qx], gp[qy], gp[qz]};
        double v[kNb], g[kNb][3];
        basis(p, h, v, g);
        const double w = h * h * h / 8.0;
        for (int a = 0; a < kNb; ++a)
          for (int b = 0; b < kNb; ++b) {
            F.mass[a][b] += w * v[a] * v[b];
            for (int i = 0; i < 3; ++i)
              for (int j = 0; j < 3; ++j) F.vol[i][j][a][b] += w * g[b][i] * g[a][j];
          }
      }
  // faces: 2x2 Gauss, weight h^2 / 4 per point.  Side 0 is the element below
  // the face (its x_axis = 1 side, normal +e_axis), side 1 the element above
  // (x_axis = 0, normal -e_axis).  For test side t and trial side s:
  //   -{d_i sigma}[[tau]]_j - {d_j tau}[[sigma]]_i + gamma [[sigma]]_i [[tau]]_j
  for (int axis = 0; axis < 3; ++axis) {
    const int o0 = (axis + 1) % 3, o1 = (axis + 2) % 3;
    for (int q0 = 0; q0 < 2; ++q0)
      for (int q1 = 0; q1 < 2; ++q1) {
        double v[2][kNb], g[2][kNb][3], nrm[2][3] = {{0, 0, 0}, {0, 0, 0}};
        for (int side = 0; side < 2; ++side) {
          double p[3];
          p[axis] = side == 0 ? 1.0 : 0.0;
          p[o0] = gp[q0];
          p[o1] = gp[q1];
          basis(p, h, v[side], g[side]);
          nrm[side][axis] = side == 0 ? 1.0 : -1.0;
        }
        const double w = h * h / 4.0;
        for (int t = 0; t < 2; ++t)
          for (int s = 0; s < 2; ++s)
            for (int i = 0; i < 3; ++i)
              for (int j = 0; j < 3; ++j)
                for (int a = 0; a < kNb; ++a)
                  for (int b = 0; b < kNb; ++b)
                    F.face[axis][t][s][i][j][a][b] +=
                        w * (-0.5 * v[t][a] * nrm[t][j] * g[s][b][i] -
                             0.5 * g[t][a][j] * v[s][b] * nrm[s][i] +
                             gamma * v[t][a] * nrm[t][j] * v[s][b] * nrm[s][i]);
        if (axis == 0) {   // the outflow face x = 1: single trace, outward +e_x
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
              for (int a = 0; a < kNb; ++a)
                for (int b = 0; b < kNb; ++b)
                  F.out[i][j][a][b] +=
                      w * (-v[0][a] * nrm[0][j] * g[0][b][i] - g[0][a][j] * v[0][b] * nrm[0][i] +
                           gamma * v[0][a] * nrm[0][j] * v[0][b] * nrm[0][i]);
        }
      }
  }
}

// Inverse of an SPD 8 x 8 matrix by Gauss-Jordan elimination with partial
// pivoting; throws if it is singular.
void invert8(const double A[kNb][kNb], double X[kNb][kNb]) {
  double M[kNb][2 * kNb];
  for (int i = 0; i < kNb; ++i)
    for (int j = 0; j < kNb; ++j) {
      M[i][j] = A[i][j];
      M[i][kNb + j] = i == j ? 1.0 : 0.0;
    }
  for (int c = 0; c < kNb; ++c) {
    int piv = c;
    for (int i = c + 1; i < kNb; ++i)
      if (std::fabs(M[i][c]) > std::fabs(M[piv][c])) piv = i;
    if (!(std::fabs(M[piv][c]) > 0.0)) throw Err3(DCG_EINVAL, "singular diagonal block");
    if (piv != c)
      for (int j = 0; j < 2 * kNb; ++j) std::swap(M[c][j], M[piv][j]);
    const double d = M[c][c];
    for (int j = 0; j < 2 * kNb; ++j) M[c][j] /= d;
    for (int i = 0; i < kNb; ++i) {
      if (i == c) continue;
      const double f = M[i][c];
      for (int j = 0; j < 2 * kNb; ++j) M[i][j] -= f * M[c][j];
    }
  }
  for (int i = 0; i < kNb; ++i)
    for (int j = 0; j < kNb; ++j) X[i][j] = M[i][kNb + j];
}

// Host assembly of every block the device path uses (layouts in dcg3d.hpp).
void assemble3d(int n, double penalty, double dt, std::vector<double>& cd, std::vector<double>& ld,
                std::vector<double>& dinv, std::vector<double>& me) {
  const int64_t ne = (int64_t)n * n * n;
  auto forms = std::make_unique<CubeForms>();   // 60 KB: keep it off the stack
  CubeForms& F = *forms;
  build_forms(n, penalty, F);
  cd.assign((size_t)kSlots * ne * 576, 0.0);
  ld.assign((size_t)kSlots * ne * 64, 0.0);
  dinv.assign((size_t)ne * 64, 0.0);
  me.assign(64, 0.0);
  for (int a = 0; a < kNb; ++a)
    for (int b = 0; b < kNb; ++b) me[a * kNb + b] = F.mass[a][b];
  double self[3][3][kNb][kNb];
  for (int ez = 0; ez < n; ++ez)
    for (int ey = 0; ey < n; ++ey)
      for (int ex = 0; ex < n; ++ex) {
        const int64_t e = ((int64_t)ez * n + ey) * n + ex;
        const int c[3] = {ex, ey, ez};
        std::memcpy(self, F.vol, sizeof(self));
        auto add = [&](const double (&B)[3][3][kNb][kNb]) {
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
              for (int a = 0; a < kNb; ++a)
                for (int b = 0; b < kNb; ++b) self[i][j][a][b] += B[i][j][a][b];
        };
        auto put = [&](int slot, const double (&B)[3][3][kNb][kNb]) {
          double* blk = cd.data() + ((size_t)slot * ne + e) * 576;
          double* lb = ld.data() + ((size_t)slot * ne + e) * 64;
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
              for (int a = 0; a < kNb; ++a)
                for (int b = 0; b < kNb; ++b) {
                  // row 8 j + a (test component j), column 8 i + b (trial i)
                  blk[(8 * i + b) * 24 + 8 * j + a] = B[i][j][a][b];
                  if (i == j) lb[b * 8 + a] += B[i][j][a][b];
                }
        };
        for (int axis = 0; axis < 3; ++axis) {
          if (c[axis] + 1 < n) {           // element is the lower side of the +axis face
            add(F.face[axis][0][0]);
            put(2 + 2 * axis, F.face[axis][0][1]);
          }
          if (c[axis] > 0) {               // upper side of the -axis face
            add(F.face[axis][1][1]);
            put(1 + 2 * axis, F.face[axis][1][0]);
          }
        }
        if (ex == n - 1) add(F.out);
        put(0, self);
        // block-Jacobi: inverse of the diagonal block of (dt/3) L
        double dblk[kNb][kNb], inv[kNb][kNb];
        for (int a = 0; a < kNb; ++a)
          for (int b = 0; b < kNb; ++b)
            dblk[a][b] = dt / 3.0 * (self[0][0][a][b] + self[1][1][a][b] + self[2][2][a][b]);
        invert8(dblk, inv);
        for (int a = 0; a < kNb; ++a)
          for (int b = 0; b < kNb; ++b) dinv[(size_t)e * 64 + b * 8 + a] = inv[a][b];
      }
}

// ---------------------------------------------------------------------------
// exact inner solve by fast diagonalisation
// ---------------------------------------------------------------------------
// On the uniform grid the SIPG Laplacian is the Kronecker sum
//   L = M (x) M (x) K_x + M (x) K_y (x) M + K_z (x) M (x) M
// (tensor index (Iz, Iy, Ix), I = 2 e_axis + i_axis) of the 1D DG-P1 mass M and
// the 1D SIPG matrices K (volume term, interior-node terms and, for x only,
// the outflow node x = 1), because the face integrals of the 3D forms factor
// into 1D node terms times the 2D mass of the face.  With K_d V_d = M V_d
// Lambda_d, V_d^T M V_d = I (dcg::fdm_axis_factor),
//   L^{-1} = V diag(1 / (lx_i + ly_j + lz_k)) V^T,  V = V_z (x) V_y (x) V_x.
dcg::FdmAxis fdm3_axis(int n, double penalty, bool outflow) {
  return dcg::fdm_axis_factor(n, penalty * n, false, outflow);
}

template <typename T>
T* dev_alloc(size_t count) {
  void* p = nullptr;
  H3(hipMalloc(&p, count * sizeof(T)));
  return static_cast<T*>(p);
}

}  // namespace

struct dcg3d_ctx {
  int n = 0;
  int64_t ne = 0, nt = 0, ns = 0;     // elements, tensor length, scalar length
  double dt = 0, nu = 1, penalty = 0;
  dcg_options opt{};
  double* Cd = nullptr;
  double* Ld = nullptr;
  double* Dinv = nullptr;
  double* Me = nullptr;
  int inner_kind = DCG3D_INNER_FDM;
  double *fVx = nullptr, *fVxT = nullptr, *fVy = nullptr, *fVyT = nullptr, *flx = nullptr,
         *fly = nullptr;        // fast-diagonalisation factors (exact inner solve)
  // tensor workspace
  double *w = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *xh = nullptr, *pf = nullptr,
         *tz = nullptr;
  // scalar workspace
  double *s = nullptr, *yh = nullptr, *ir = nullptr, *iz = nullptr, *ip = nullptr, *iq = nullptr;
  double *part = nullptr, *part2 = nullptr, *dots = nullptr;
  dcg3::PcgScalars* sc = nullptr;
  dcg3::PcgScalars* sc_host = nullptr;
  double* dots_host = nullptr;
  std::string last_error;
  double t_setup_ms = 0;
  int64_t inner_total = 0, inner_solves = 0;
  // multigrid inner solve: level k at index k - 1
  int mg_J = 0, mg_m = 10;
  std::vector<int> mg_n;
  std::vector<double*> mg_op, mg_ras, mg_f, mg_z, mg_r;
  double* mg_cinv = nullptr;
  double* mg_part = nullptr;
  dcg3::Mg3Scalars* mg_sc = nullptr;
  dcg3::Mg3Scalars* mg_sc_host = nullptr;
  hipStream_t mg_cap = nullptr;
  hipGraphExec_t mg_graph = nullptr;
  int mg_recent[4] = {0, 0, 0, 0};
  int mg_nrecent = 0;
  // optional HIP-event timing of the dominant launches of the inner solves
  bool timing = false;
  std::vector<hipEvent_t> evs;
  size_t ev_used = 0;

  void time_mark() {
    if (ev_used == evs.size()) {
      hipEvent_t e;
      H3(hipEventCreate(&e));
      evs.push_back(e);
    }
    H3(hipEventRecord(evs[ev_used++], nullptr));
  }
  // A start / stop pair for a launch that records them itself.
  void event_pair(hipEvent_t& e0, hipEvent_t& e1) {
    while (evs.size() < ev_used + 2) {
      hipEvent_t e;
      H3(hipEventCreate(&e));
      evs.push_back(e);
    }
    e0 = evs[ev_used];
    e1 = evs[ev_used + 1];
    ev_used += 2;
  }

  ~dcg3d_ctx() {
    for (double* b : {Cd, Ld, Dinv, Me, w, r, p, q, xh, pf, tz, s, yh, ir, iz, ip, iq, part, part2, dots,
                      fVx, fVxT, fVy, fVyT, flx, fly})
      if (b) (void)hipFree(b);
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
    for (auto* v : {&mg_op, &mg_ras, &mg_f, &mg_z, &mg_r})
      for (double* b : *v)
        if (b) (void)hipFree(b);
    for (double* b : {mg_cinv, mg_part})
      if (b) (void)hipFree(b);
    if (mg_sc) (void)hipFree(mg_sc);
    if (mg_sc_host) (void)hipHostFree(mg_sc_host);
    if (mg_graph) (void)hipGraphExecDestroy(mg_graph);
    if (mg_cap) (void)hipStreamDestroy(mg_cap);
    if (sc) (void)hipFree(sc);
    if (sc_host) (void)hipHostFree(sc_host);
    if (dots_host) (void)hipHostFree(dots_host);
  }

  void setup() {
    ne = (int64_t)n * n * n;
    nt = ne * kDof;
    ns = ne * kNb;
    std::vector<double> cd, ld, dinv, me;
    assemble3d(n, penalty, dt, cd, ld, dinv, me);
    Cd = dev_alloc<double>(cd.size());
    Ld = dev_alloc<double>(ld.size());
    Dinv = dev_alloc<double>(dinv.size());
    Me = dev_alloc<double>(64);
    H3(hipMemcpy(Cd, cd.data(), cd.size() * sizeof(double), hipMemcpyHostToDevice));
    H3(hipMemcpy(Ld, ld.data(), ld.size() * sizeof(double), hipMemcpyHostToDevice));
    H3(hipMemcpy(Dinv, dinv.data(), dinv.size() * sizeof(double), hipMemcpyHostToDevice));
    H3(hipMemcpy(Me, me.data(), 64 * sizeof(double), hipMemcpyHostToDevice));
    if (inner_kind == DCG3D_INNER_FDM) {
      const int N = 2 * n;
      const dcg::FdmAxis fx = fdm3_axis(n, penalty, true), fy = fdm3_axis(n, penalty, false);
      std::vector<double> vxt((size_t)N * N), vyt((size_t)N * N);
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
          vxt[(size_t)j * N + i] = fx.V[(size_t)i * N + j];
          vyt[(size_t)j * N + i] = fy.V[(size_t)i * N + j];
        }
      for (double** b : {&fVx, &fVxT, &fVy, &fVyT}) *b = dev_alloc<double>((size_t)N * N);
      flx = dev_alloc<double>(N);
      fly = dev_alloc<double>(N);
      H3(hipMemcpy(fVx, fx.V.data(), (size_t)N * N * sizeof(double), hipMemcpyHostToDevice));
      H3(hipMemcpy(fVxT, vxt.data(), (size_t)N * N * sizeof(double), hipMemcpyHostToDevice));
      H3(hipMemcpy(fVy, fy.V.data(), (size_t)N * N * sizeof(double), hipMemcpyHostToDevice));
      H3(hipMemcpy(fVyT, vyt.data(), (size_t)N * N * sizeof(double), hipMemcpyHostToDevice));
      H3(hipMemcpy(flx, fx.lam.data(), N * sizeof(double), hipMemcpyHostToDevice));
      H3(hipMemcpy(fly, fy.lam.data(), N * sizeof(double), hipMemcpyHostToDevice));
    }
    if (inner_kind == DCG3D_INNER_MG) setup_mg(ld);
    for (double** b : {&w, &r, &p, &q, &xh, &pf, &tz}) *b = dev_alloc<double>(nt);
    for (double** b : {&s, &yh, &ir, &iz, &ip, &iq}) *b = dev_alloc<double>(ns);
    const int64_t np = 2 * ((ns + 255) / 256) + 1024;
    part = dev_alloc<double>(np);
    part2 = dev_alloc<double>(np);
    dots = dev_alloc<double>(8);
    H3(hipMalloc(&sc, sizeof(dcg3::PcgScalars)));
    H3(hipHostMalloc(&sc_host, sizeof(dcg3::PcgScalars), hipHostMallocDefault));
    H3(hipHostMalloc(&dots_host, 8 * sizeof(double), hipHostMallocDefault));
  }

  template <typename T>
  T* upload(const std::vector<T>& v) {
    T* d = dev_alloc<T>(v.size());
    H3(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return d;
  }

  // The Galerkin hierarchy of L, its class tables and level vectors.
  void setup_mg(const std::vector<double>& ld) {
    mg_J = dcg3::mg3_num_levels(n, opt.levels);
    if (mg_J < 1) throw Err3(DCG_EINVAL, "no multigrid hierarchy for this n and levels");
    mg_m = opt.smooth3d;
    const dcg3::Mg3Hierarchy H = dcg3::build_mg3(n, mg_J, ld);
    for (int k = 1; k <= mg_J; ++k) {
      const dcg3::Mg3Level& L = H.lev[k - 1];
      const int64_t len = 8 * (int64_t)L.n * L.n * L.n;
      mg_n.push_back(L.n);
      const bool split = dcg3::mg3_split(L.n);   // small levels: row-major tables
      mg_op.push_back(upload(split ? L.op : dcg3::op_rows_fastest(L.op)));
      mg_ras.push_back(k >= 2 ? upload(split ? L.ras : dcg3::rows_fastest(L.ras, dcg3::kRasCols)) : nullptr);
      mg_f.push_back(dev_alloc<double>(len));
      mg_z.push_back(dev_alloc<double>(len));
      mg_r.push_back(dev_alloc<double>(len));
    }
    mg_cinv = upload(H.coarse_inv);
    mg_part = dev_alloc<double>(dcg3::mg3_res_blocks(n));
    H3(hipMalloc(&mg_sc, sizeof(dcg3::Mg3Scalars)));
    H3(hipHostMalloc(&mg_sc_host, sizeof(dcg3::Mg3Scalars), hipHostMallocDefault));
    H3(hipStreamCreateWithFlags(&mg_cap, hipStreamNonBlocking));
  }

  // ---- the W-cycle (Algorithm 4) on level k, every launch guarded by g
  enum { kZero = 0, kWarm = 1, kResidualGiven = 2 };

  void mg_smooth(int k, int step, int mode, hipStream_t st, const int32_t* g, bool timed) {
    const int i = k - 1, nk = mg_n[i];
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) event_pair(e0, e1);
    if (step == 0 && mode == kZero) {          // z = S f
      H3(dcg3::launch_mg3_ras(nk, mg_ras[i], mg_f[i], mg_z[i], true, g, st, e0, e1));
      return;
    }
    if (!(step == 0 && mode == kResidualGiven))
      H3(dcg3::launch_mg3_res(nk, mg_op[i], mg_f[i], mg_z[i], mg_r[i], nullptr, g, st));
    H3(dcg3::launch_mg3_ras(nk, mg_ras[i], mg_r[i], mg_z[i], false, g, st, e0, e1));
  }

  void mg_cycle(int k, int mode, hipStream_t st, const int32_t* g) {
    const int i = k - 1;
    if (k == 1) {   // exact solve on the coarsest level
      H3(dcg3::launch_mg3_dense(8 * mg_n[0] * mg_n[0] * mg_n[0], mg_cinv, mg_f[0], mg_z[0], g, st));
      return;
    }
    const bool timed = timing && k == mg_J && st == nullptr;
    for (int s = 0; s < mg_m; ++s) mg_smooth(k, s, mode, st, g, timed);
    H3(dcg3::launch_mg3_res(mg_n[i], mg_op[i], mg_f[i], mg_z[i], mg_r[i], nullptr, g, st));
    H3(dcg3::launch_mg3_restrict(mg_n[i], mg_r[i], mg_f[i - 1], g, st));
    // coarse correction: gamma = 2 cycles from zero (the exact solve once)
    mg_cycle(k - 1, kZero, st, g);
    if (k - 1 > 1) mg_cycle(k - 1, kWarm, st, g);
    H3(dcg3::launch_mg3_prolong(mg_n[i], mg_z[i - 1], mg_z[i], false, g, st));
    for (int s = 0; s < mg_m; ++s) mg_smooth(k, s, kWarm, st, g, timed);
  }

  // One pass of Algorithm 3: the residual of the finest iterate, the
  // stopping test, and (while active) the W-cycle that starts from it.
  void mg_iteration(hipStream_t st) {
    const int J = mg_J, i = J - 1;
    const int32_t* g = &mg_sc->active;
    H3(dcg3::launch_mg3_res(mg_n[i], mg_op[i], mg_f[i], mg_z[i], mg_r[i], mg_part, g, st));
    H3(dcg3::launch_mg3_test(dcg3::mg3_res_blocks(mg_n[i]), mg_part, mg_sc, st));
    if (J == 1) {
      H3(dcg3::launch_mg3_dense(8 * mg_n[0] * mg_n[0] * mg_n[0], mg_cinv, mg_f[0], mg_z[0], g, st));
      return;
    }
    mg_cycle(J, kResidualGiven, st, g);
  }

  void mg_launch_iteration() {
    if (!opt.use_graph || timing) {
      mg_iteration(nullptr);
      return;
    }
    if (!mg_graph) {
      hipGraph_t gr = nullptr;
      H3(hipStreamBeginCapture(mg_cap, hipStreamCaptureModeThreadLocal));
      try {
        mg_iteration(mg_cap);
      } catch (...) {
        (void)hipStreamEndCapture(mg_cap, &gr);
        if (gr) (void)hipGraphDestroy(gr);
        throw;
      }
      H3(hipStreamEndCapture(mg_cap, &gr));
      const hipError_t e = hipGraphInstantiate(&mg_graph, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      H3(e);
    }
    H3(hipGraphLaunch(mg_graph, nullptr));
  }

  // yh = E^{-1} s, E = (dt/3) L, by Algorithm 3 on L to ||s - L z|| <= rel ||s||
  // (the same test as on E, yh = (3/dt) z).  Iterations are enqueued ahead of
  // the device-side test: as many as the fewest cycles of the last four
  // solves plus one, then one at a time.
  int inner_mg(const double* rhs, double* out, double rel) {
    const int i = mg_J - 1;
    const int64_t len = 8 * ne;
    copy(rhs, mg_f[i], len);
    H3(dcg3::launch_mg3_start(len, mg_z[i], mg_sc, rel * rel, opt.max_inner, nullptr));
    int pred = 0;
    if (mg_nrecent > 0) {
      pred = mg_recent[0];
      for (int j = 1; j < std::min(mg_nrecent, 4); ++j) pred = std::min(pred, mg_recent[j]);
    }
    int launched = 0;
    for (;;) {
      const int chunk = launched == 0 ? pred + 1 : 1;
      for (int c = 0; c < chunk; ++c) mg_launch_iteration();
      launched += chunk;
      H3(hipMemcpyAsync(mg_sc_host, mg_sc, sizeof(*mg_sc), hipMemcpyDeviceToHost, nullptr));
      H3(hipStreamSynchronize(nullptr));
      if (!mg_sc_host->active || launched > opt.max_inner + 1) break;
    }
    const int iters = mg_sc_host->iters;
    H3(dcg3::launch_mg3_scale(len, 3.0 / dt, mg_z[i], out, nullptr));
    mg_recent[mg_nrecent++ % 4] = iters;
    return iters;
  }

  // ---- building blocks on the legacy default stream
  double dot(const double* x, const double* y, int64_t len) {
    H3(dcg3::launch_dot(len, x, y, part, dots, nullptr));
    H3(hipMemcpyAsync(dots_host, dots, sizeof(double), hipMemcpyDeviceToHost, nullptr));
    H3(hipStreamSynchronize(nullptr));
    return dots_host[0];
  }
  void copy(const double* x, double* y, int64_t len) {
    H3(hipMemcpyAsync(y, x, len * sizeof(double), hipMemcpyDeviceToDevice, nullptr));
  }
  void astar(const double* x, double* y) {
    // the dominant kernel with the exact inner solve or none
    const bool timed = timing && (inner_kind == DCG3D_INNER_FDM || inner_kind == DCG3D_INNER_NONE);
    if (timed) time_mark();
    H3(dcg3::launch_astar3(n, Cd, Me, 1.0 / nu, dt, x, y, nullptr));
    if (timed) time_mark();
  }

  // yh = E^{-1} s to ||s - E yh|| <= rel ||s|| by block-Jacobi CG; returns the
  // number of steps.
  int inner(const double* rhs, double* out, double rel) {
    if (inner_kind == DCG3D_INNER_NONE) {    // no deflation: pi = 0, Algorithm 2 is CG on A*
      H3(dcg3::launch_fill(ns, 0.0, out, nullptr));
      inner_solves += 1;
      return 0;
    }
    if (inner_kind == DCG3D_INNER_FDM) {     // exact: E^{-1} = (3/dt) L^{-1}
      H3(dcg3::launch_fdm_solve(n, fVx, fVxT, fVy, fVyT, flx, fly, 3.0 / dt, rhs, out, ir, iz, nullptr));
      inner_solves += 1;
      return 0;
    }
    if (inner_kind == DCG3D_INNER_MG) {
      const int it = inner_mg(rhs, out, rel);
      inner_total += it;
      inner_solves += 1;
      return it;
    }
    H3(dcg3::launch_pcg_start(ne, Dinv, rhs, out, ir, iz, ip, part, sc, rel * rel, nullptr));
    H3(hipMemcpyAsync(sc_host, sc, sizeof(*sc), hipMemcpyDeviceToHost, nullptr));
    H3(hipStreamSynchronize(nullptr));
    const int nblk = int((ns + 255) / 256);
    int done = 0;
    while (sc_host->active && done < opt.max_inner) {
      const int chunk = std::min(8, opt.max_inner - done);
      for (int c = 0; c < chunk; ++c) {
        if (timing) time_mark();   // block-Jacobi CG: the Laplacian product dominates
        H3(dcg3::launch_lap3(n, Ld, dt / 3.0, ip, iq, part, nullptr));
        if (timing) time_mark();
        H3(dcg3::launch_pcg_step(ne, Dinv, out, ir, iz, ip, iq, part, part2, nblk, sc, nullptr));
      }
      done += chunk;
      H3(hipMemcpyAsync(sc_host, sc, sizeof(*sc), hipMemcpyDeviceToHost, nullptr));
      H3(hipStreamSynchronize(nullptr));
    }
    inner_total += sc_host->iters;
    inner_solves += 1;
    return sc_host->iters;
  }

  // Algorithm 2 with the CG outer iteration (d = 3).
  dcg_status solve(const double* f, double* x, double tol, dcg_stats* st) {
    const auto t0 = std::chrono::steady_clock::now();
    inner_total = inner_solves = 0;
    // inner tolerance: eq. (fixed_tol), or eq. (tol) inside the outer loop
    const double rel_in = opt.c_A > 0.0 ? opt.c_A * tol : opt.c_F * tol;
    const double fnorm = std::sqrt(dot(f, f, nt));
    dcg_stats out{};
    out.t_setup_ms = t_setup_ms;
    if (!std::isfinite(fnorm)) throw Err3(DCG_EINVAL, "right-hand side is not finite");
    if (fnorm == 0.0) {
      H3(dcg3::launch_fill(nt, 0.0, x, nullptr));
      H3(hipStreamSynchronize(nullptr));
      if (st) *st = out;
      return DCG_OK;
    }
    // prologue: pf = pi(f) = Z E^{-1} Z^T f, f_D = f - A* pf
    H3(dcg3::launch_zt3(ne, f, s, nullptr));
    inner(s, yh, rel_in);
    H3(dcg3::launch_fill(nt, 0.0, pf, nullptr));
    H3(dcg3::launch_zaxpy3(ne, 1.0, yh, pf, nullptr));
    astar(pf, w);
    copy(f, r, nt);
    H3(dcg3::launch_axpy(nt, -1.0, w, r, nullptr));
    H3(dcg3::launch_fill(nt, 0.0, xh, nullptr));
    copy(r, p, nt);
    double rho = dot(r, r, nt);
    int it = 0, pass = 0;
    dcg_status status = DCG_OK;
    double res = 0.0;
    while (true) {   // one pass of Algorithm 2; further passes are warm restarts from x
    while (it < opt.max_outer && std::sqrt(rho) > tol * fnorm) {
      // q = M_D p = w - dt A_div Z E^{-1} Z^T w, w = A* p
      astar(p, w);
      H3(dcg3::launch_zt3(ne, w, s, nullptr));
      inner(s, yh, opt.c_A > 0.0 ? opt.c_A * tol * fnorm / std::sqrt(rho) : rel_in);
      H3(dcg3::launch_adivz3(n, Cd, dt, w, yh, q, nullptr));
      const double pq = dot(p, q, nt);
      if (!(pq > 0.0) || !std::isfinite(pq)) {
        status = DCG_EBREAKDOWN;
        break;
      }
      const double alpha = rho / pq;
      H3(dcg3::launch_axpy(nt, alpha, p, xh, nullptr));
      H3(dcg3::launch_axpy(nt, -alpha, q, r, nullptr));
      const double rho_new = dot(r, r, nt);
      H3(dcg3::launch_xpby(nt, r, rho_new / rho, p, nullptr));
      rho = rho_new;
      ++it;
    }
    if (status == DCG_OK && std::sqrt(rho) > tol * fnorm) status = DCG_NOT_CONVERGED;
    // epilogue: x = (x_hat - pi(A* x_hat)) + pi(f)
    astar(xh, w);
    H3(dcg3::launch_zt3(ne, w, s, nullptr));
    inner(s, yh, rel_in);
    copy(xh, x, nt);
    H3(dcg3::launch_zaxpy3(ne, -1.0, yh, x, nullptr));
    H3(dcg3::launch_axpy(nt, 1.0, pf, x, nullptr));
    // true residual of the reconstructed x
    astar(x, w);
    copy(f, tz, nt);
    H3(dcg3::launch_axpy(nt, -1.0, w, tz, nullptr));
    res = std::sqrt(dot(tz, tz, nt));
    if (status != DCG_OK || res <= tol * fnorm || pass >= opt.restarts) break;
    // warm restart (not in the paper; the reading of the 2D solver): x_hat = x,
    // r = f_D - M_D x_hat with pi(f) and f_D of the first pass
    ++pass;
    copy(x, xh, nt);
    astar(pf, w);
    copy(f, r, nt);
    H3(dcg3::launch_axpy(nt, -1.0, w, r, nullptr));
    astar(xh, w);
    H3(dcg3::launch_zt3(ne, w, s, nullptr));
    inner(s, yh, rel_in);
    H3(dcg3::launch_adivz3(n, Cd, dt, w, yh, q, nullptr));
    H3(dcg3::launch_axpy(nt, -1.0, q, r, nullptr));
    copy(r, p, nt);
    rho = dot(r, r, nt);
    }
    if (opt.restarts > 0 && status == DCG_OK && res > tol * fnorm) status = DCG_NOT_CONVERGED;
    out.status = status;
    out.restarts = pass;
    out.outer_iters = it;
    out.total_wcycles = int32_t(inner_total);
    out.inner_solves = int32_t(inner_solves);
    out.inner_per_outer = it > 0 ? double(inner_total) / it : 0.0;
    out.rel_res_recurrence = std::sqrt(rho) / fnorm;
    out.rel_res_true = res / fnorm;
    out.t_solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (st) *st = out;
    return status;
  }

  void apply(int op, const double* in, double* outv, double tol) {
    switch (op) {
      case DCG3D_OP_ASTAR:
        astar(in, outv);
        break;
      case DCG3D_OP_ZT:
        H3(dcg3::launch_zt3(ne, in, outv, nullptr));
        break;
      case DCG3D_OP_Z:
        H3(dcg3::launch_fill(nt, 0.0, outv, nullptr));
        H3(dcg3::launch_zaxpy3(ne, 1.0, in, outv, nullptr));
        break;
      case DCG3D_OP_DEFLATED:
        astar(in, w);
        H3(dcg3::launch_zt3(ne, w, s, nullptr));
        inner(s, yh, tol);
        H3(dcg3::launch_adivz3(n, Cd, dt, w, yh, outv, nullptr));
        break;
      case DCG3D_OP_REDUCED:
        H3(dcg3::launch_lap3(n, Ld, dt / 3.0, in, outv, part, nullptr));
        break;
      case DCG3D_OP_INNER:
        inner(in, outv, tol);
        break;
      case DCG3D_OP_ADIVZ:
        H3(dcg3::launch_fill(nt, 0.0, tz, nullptr));
        H3(dcg3::launch_adivz3(n, Cd, -1.0, tz, in, outv, nullptr));
        break;
      default:
        throw Err3(DCG_EINVAL, "unknown operator");
    }
    H3(hipStreamSynchronize(nullptr));
  }

  // Level operators of the multigrid inner solve (dcg3d_mg_apply).
  void mg_apply(int op, int k, const double* in, const double* in2, double* outv) {
    if (inner_kind != DCG3D_INNER_MG) throw Err3(DCG_EINVAL, "the handle has no multigrid hierarchy");
    if (k < 1 || k > mg_J) throw Err3(DCG_EINVAL, "level out of range");
    const int i = k - 1, nk = mg_n[i];
    const int64_t len = 8 * (int64_t)nk * nk * nk;
    switch (op) {
      case DCG3D_MG_LAPLACE:    // out = -(0 - L z)
        H3(dcg3::launch_mg3_res(nk, mg_op[i], nullptr, in, mg_r[i], nullptr, nullptr, nullptr));
        H3(dcg3::launch_mg3_scale(len, -1.0, mg_r[i], outv, nullptr));
        break;
      case DCG3D_MG_RAS:
        if (k < 2) throw Err3(DCG_EINVAL, "the coarsest level has no smoother");
        if (!in2) {
          H3(dcg3::launch_mg3_ras(nk, mg_ras[i], in, outv, true, nullptr, nullptr));
        } else {
          copy(in2, outv, len);
          H3(dcg3::launch_mg3_res(nk, mg_op[i], in, in2, mg_r[i], nullptr, nullptr, nullptr));
          H3(dcg3::launch_mg3_ras(nk, mg_ras[i], mg_r[i], outv, false, nullptr, nullptr));
        }
        break;
      case DCG3D_MG_RESTRICT:
        if (k < 2) throw Err3(DCG_EINVAL, "restriction needs level >= 2");
        H3(dcg3::launch_mg3_restrict(nk, in, outv, nullptr, nullptr));
        break;
      case DCG3D_MG_PROLONG:
        if (k < 2) throw Err3(DCG_EINVAL, "prolongation needs level >= 2");
        H3(dcg3::launch_mg3_prolong(nk, in, outv, true, nullptr, nullptr));
        break;
      case DCG3D_MG_COARSE:
        if (k != 1) throw Err3(DCG_EINVAL, "the exact solve is on level 1");
        H3(dcg3::launch_mg3_dense(int(len), mg_cinv, in, outv, nullptr, nullptr));
        break;
      case DCG3D_MG_WCYCLE:
        copy(in, mg_f[i], len);
        if (in2) copy(in2, mg_z[i], len);
        mg_cycle(k, in2 ? kWarm : kZero, nullptr, nullptr);
        copy(mg_z[i], outv, len);
        break;
      default:
        throw Err3(DCG_EINVAL, "unknown multigrid operator");
    }
    H3(hipStreamSynchronize(nullptr));
  }
};

namespace {

dcg_status fail3(dcg3d_ctx* h, dcg_status s, const std::string& msg) {
  g_last_error3 = msg;
  if (h) h->last_error = msg;
  return s;
}

template <typename Fn>
dcg_status guarded3(dcg3d_ctx* h, Fn fn) {
  try {
    return fn();
  } catch (const Err3& e) {
    return fail3(h, e.status, e.what());
  } catch (const std::bad_alloc&) {
    return fail3(h, DCG_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail3(h, DCG_EINVAL, e.what());
  }
}

}  // namespace

extern "C" {

dcg_status dcg3d_setup(int32_t n, double penalty, double dt, double nu, int32_t inner,
                       const dcg_options* opt, dcg3d_handle* out) {
  if (!out) return fail3(nullptr, DCG_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 2 || n > DCG3D_MAX_N) return fail3(nullptr, DCG_EINVAL, "n must be in [2, 64]");
  if (inner != DCG3D_INNER_FDM && inner != DCG3D_INNER_PCG && inner != DCG3D_INNER_NONE &&
      inner != DCG3D_INNER_MG)
    return fail3(nullptr, DCG_EINVAL, "inner must be a dcg3d_inner");
  if (!(penalty > 0.0) || !std::isfinite(penalty)) return fail3(nullptr, DCG_EINVAL, "penalty must be positive");
  if (!(dt > 0.0) || !std::isfinite(dt) || !(nu > 0.0) || !std::isfinite(nu))
    return fail3(nullptr, DCG_EINVAL, "dt and nu must be positive");
  dcg_options o{};
  if (opt) {
    o = *opt;
  } else {
    dcg_mesh m{};
    dcg_defaults(&m, &o);
    o.prec = DCG_FP64;
    o.max_inner = DCG3D_DEFAULT_MAX_INNER;
  }
  if (o.prec != DCG_FP64) return fail3(nullptr, DCG_EINVAL, "the 3D solver computes in FP64 only");
  if (o.outer != DCG_OUTER_CG) return fail3(nullptr, DCG_EINVAL, "the 3D solver runs the CG outer iteration");
  if (!(o.c_A >= 0.0) || !std::isfinite(o.c_A)) return fail3(nullptr, DCG_EINVAL, "c_A must be >= 0");
  if (o.x0_given) return fail3(nullptr, DCG_EINVAL, "the 3D solver starts from x0 = 0");
  if (o.restarts < 0) return fail3(nullptr, DCG_EINVAL, "restarts must be >= 0");
  if (!(o.c_F > 0.0) || o.max_outer < 0 || o.max_inner < 1)
    return fail3(nullptr, DCG_EINVAL, "c_F must be > 0, max_outer >= 0, max_inner >= 1");
  if (inner == DCG3D_INNER_MG) {
    if (o.smooth3d < 1) return fail3(nullptr, DCG_EINVAL, "smooth3d must be >= 1");
    if (dcg3::mg3_num_levels(n, o.levels) < 1)
      return fail3(nullptr, DCG_EINVAL,
                   "multigrid needs n = c 2^(J-1) with a coarsest size c in [2, 4] (levels = J, 0 = all)");
  }
  auto* h = new (std::nothrow) dcg3d_ctx();
  if (!h) return fail3(nullptr, DCG_ENOMEM, "host allocation failed");
  h->n = n;
  h->inner_kind = inner;
  h->dt = dt;
  h->nu = nu;
  h->penalty = penalty;
  h->opt = o;
  const auto t0 = std::chrono::steady_clock::now();
  const dcg_status s = guarded3(h, [&] {
    h->setup();
    H3(hipDeviceSynchronize());
    return DCG_OK;
  });
  if (s != DCG_OK) {
    delete h;
    return s;
  }
  h->t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = h;
  return DCG_OK;
}

dcg_status dcg3d_solve(dcg3d_handle h, const double* b, double* x, double tol, dcg_stats* st) {
  if (!h || !b || !x) return fail3(h, DCG_EINVAL, "NULL argument");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail3(h, DCG_EINVAL, "tol must be positive");
  return guarded3(h, [&] { return h->solve(b, x, tol, st); });
}

dcg_status dcg3d_apply(dcg3d_handle h, dcg3d_op op, const double* in, double* out, double tol) {
  if (!h || !in || !out) return fail3(h, DCG_EINVAL, "NULL argument");
  if ((op == DCG3D_OP_DEFLATED || op == DCG3D_OP_INNER) && (!(tol > 0.0) || !std::isfinite(tol)))
    return fail3(h, DCG_EINVAL, "tol must be positive");
  return guarded3(h, [&] {
    h->apply(op, in, out, tol);
    return DCG_OK;
  });
}

dcg_status dcg3d_mg_apply(dcg3d_handle h, int32_t op, int32_t level, const double* in,
                          const double* in2, double* out) {
  if (!h || !in || !out) return fail3(h, DCG_EINVAL, "NULL argument");
  return guarded3(h, [&] {
    h->mg_apply(op, level, in, in2, out);
    return DCG_OK;
  });
}

dcg_status dcg3d_mg_levels(dcg3d_handle h, int32_t* levels, int32_t* coarsest) {
  if (!h || !levels || !coarsest) return fail3(h, DCG_EINVAL, "NULL argument");
  if (h->inner_kind != DCG3D_INNER_MG) return fail3(h, DCG_EINVAL, "the handle has no multigrid hierarchy");
  *levels = h->mg_J;
  *coarsest = h->mg_n[0];
  return DCG_OK;
}

dcg_status dcg3d_destroy(dcg3d_handle h) {
  delete h;
  return DCG_OK;
}

dcg_status dcg3d_host_blocks(int32_t n, double penalty, double dt, int32_t which, double* out) {
  if (!out) return fail3(nullptr, DCG_EINVAL, "out is NULL");
  if (n < 2 || n > DCG3D_MAX_HOST_BLOCKS_N) return fail3(nullptr, DCG_EINVAL, "n must be in [2, 16]");
  if (!(penalty > 0.0) || !(dt > 0.0)) return fail3(nullptr, DCG_EINVAL, "penalty and dt must be positive");
  if (which < 0 || which > 4) return fail3(nullptr, DCG_EINVAL, "which must be 0..4");
  return guarded3(nullptr, [&] {
    if (which == 4) {   // fast-diagonalisation factors: V_x, lambda_x, V_y, lambda_y
      const size_t N = 2 * (size_t)n;
      const dcg::FdmAxis fx = fdm3_axis(n, penalty, true), fy = fdm3_axis(n, penalty, false);
      double* o = out;
      for (const dcg::FdmAxis* f : {&fx, &fy}) {
        std::memcpy(o, f->V.data(), N * N * sizeof(double));
        std::memcpy(o + N * N, f->lam.data(), N * sizeof(double));
        o += N * N + N;
      }
      return DCG_OK;
    }
    std::vector<double> cd, ld, dinv, me;
    assemble3d(n, penalty, dt, cd, ld, dinv, me);
    const std::vector<double>* src[4] = {&cd, &ld, &dinv, &me};
    std::memcpy(out, src[which]->data(), src[which]->size() * sizeof(double));
    return DCG_OK;
  });
}

dcg_status dcg3d_host_mg(int32_t n, double penalty, int32_t levels, int32_t level, int32_t which,
                         double* out) {
  if (!out) return fail3(nullptr, DCG_EINVAL, "out is NULL");
  if (n < 2 || n > DCG3D_MAX_HOST_BLOCKS_N) return fail3(nullptr, DCG_EINVAL, "n must be in [2, 16]");
  if (!(penalty > 0.0)) return fail3(nullptr, DCG_EINVAL, "penalty must be positive");
  const int J = dcg3::mg3_num_levels(n, levels);
  if (J < 1) return fail3(nullptr, DCG_EINVAL, "no multigrid hierarchy for this n and levels");
  if (level < 1 || level > J) return fail3(nullptr, DCG_EINVAL, "level out of range");
  if (which < 0 || which > 2 || (which == 1 && level < 2) || (which == 2 && level != 1))
    return fail3(nullptr, DCG_EINVAL, "which must be 0, 1 (level >= 2) or 2 (level 1)");
  return guarded3(nullptr, [&] {
    std::vector<double> cd, ld, dinv, me;
    assemble3d(n, penalty, 1.0, cd, ld, dinv, me);
    const dcg3::Mg3Hierarchy H = dcg3::build_mg3(n, J, ld);
    const std::vector<double>& src =
        which == 0 ? H.lev[level - 1].op : (which == 1 ? H.lev[level - 1].ras : H.coarse_inv);
    std::memcpy(out, src.data(), src.size() * sizeof(double));
    return DCG_OK;
  });
}

dcg_status dcg3d_kernel_timing(dcg3d_handle h, int32_t enable) {
  if (!h) return fail3(nullptr, DCG_EINVAL, "NULL handle");
  return guarded3(h, [&] {
    H3(hipStreamSynchronize(nullptr));
    h->timing = enable != 0;
    h->ev_used = 0;
    return DCG_OK;
  });
}

dcg_status dcg3d_kernel_timing_read(dcg3d_handle h, double* total_ms, int64_t* launches) {
  if (!h || !total_ms || !launches) return fail3(h, DCG_EINVAL, "NULL argument");
  return guarded3(h, [&] {
    H3(hipStreamSynchronize(nullptr));
    double sum = 0.0;
    for (size_t i = 0; i + 1 < h->ev_used; i += 2) {
      float ms = 0.0f;
      H3(hipEventElapsedTime(&ms, h->evs[i], h->evs[i + 1]));
      sum += ms;
    }
    *total_ms = sum;
    *launches = int64_t(h->ev_used / 2);
    h->ev_used = 0;
    return DCG_OK;
  });
}

const char* dcg3d_last_error(dcg3d_handle h) { return h ? h->last_error.c_str() : g_last_error3.c_str(); }

}  // extern "C"
