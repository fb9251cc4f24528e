// Solver driver: the deflated-CG outer iteration (Algorithm 2), the inner
// Multigrid iteration (Algorithm 3) as FP64 iterative refinement around
// W-cycles (Algorithm 4) of the level real type, and the operator-level
// entry points.  All arithmetic runs in the kernels of kernels.hip; the host
// only enqueues launches and reads the device scalar block at the
// convergence tests.
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "fdm_host.hpp"
#include "wcycle.hpp"

namespace dcg {

void* Workspace::alloc(size_t b) {
  void* p = nullptr;
  DCG_HIP(hipMalloc(&p, b));
  allocations.push_back(p);
  bytes += b;
  return p;
}

void Workspace::release() {
  for (void* p : allocations) (void)hipFree(p);
  allocations.clear();
  if (sc_host) (void)hipHostFree(sc_host);
  sc_host = nullptr;
}

Workspace::~Workspace() { release(); }

void* FcgStore::alloc(size_t b) {
  void* p = nullptr;
  DCG_HIP(hipMalloc(&p, b));
  vecs.push_back(p);
  return p;
}

void FcgStore::release() {
  for (void* p : vecs) (void)hipFree(p);
  vecs.clear();
  for (void* p : {static_cast<void*>(dptr), static_cast<void*>(qptr), static_cast<void*>(dq),
                  static_cast<void*>(coef), static_cast<void*>(coef2), static_cast<void*>(part)})
    if (p) (void)hipFree(p);
  dptr = qptr = nullptr;
  dq = coef = coef2 = part = nullptr;
  d.clear();
  q.clear();
  R = 0;
}

void LevelBuffers::allocate(const MeshContext& m, bool fp32, bool batch, Workspace& ws) {
  batched = batch;
  const size_t rs = fp32 ? sizeof(float) : sizeof(double);
  const size_t cols = batch ? kBatch : 1;
  f.assign(m.J, nullptr);
  rr.assign(m.J, nullptr);
  for (int b = 0; b < 2; ++b) {
    z[b].assign(m.J, nullptr);
    Y[b].assign(m.J, nullptr);
  }
  for (int k = 1; k <= m.J; ++k) {
    const size_t ne = size_t(m.lv[k - 1].ne);
    f[k - 1] = ws.alloc(rs * 4 * ne * cols);
    if (!batch) rr[k - 1] = ws.alloc(rs * 4 * ne);
    for (int b = 0; b < 2; ++b) {
      z[b][k - 1] = ws.alloc(rs * 4 * ne * cols);
      if (k >= 2) {
        Y[b][k - 1] = ws.alloc(rs * 12 * ne * cols);
        DCG_HIP(hipMemset(Y[b][k - 1], 0, rs * 12 * ne * cols));
      }
    }
  }
}

}  // namespace dcg

dcg_ctx::~dcg_ctx() {
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(device);
  if (wgraph) (void)hipGraphExecDestroy(wgraph);
  for (hipEvent_t& e : kev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t& e : aev)
    if (e) (void)hipEventDestroy(e);
  omg.reset();
  if (capture_stream) (void)hipStreamDestroy(capture_stream);
  ws.release();
  (void)hipSetDevice(cur);
}

namespace dcg {
namespace {

constexpr double kTwo = 2.0;   // Z^T A* Z = (dt/2) L  =>  A* Z (2/dt) = 2 A_div Z
constexpr double kApplyTol = 1e-8;   // outer tolerance assumed by DCG_OP_INNER / DEFLATED

// Device buffers an inner solve works in: the handle's workspace, or the
// static scratch of dcg_apply_noalloc.
struct InnerWs {
  const LevelBuffers* lvb = nullptr;
  Scalars* sc = nullptr;
  double* part = nullptr;
  const CoarseFdm* cfdm = nullptr;   // coarsest solve of a shortened hierarchy
  bool graph = true;                 // the coarse correction may be a captured graph
};

InnerWs handle_ws(dcg_ctx* h) {
  InnerWs w;
  w.lvb = &h->ws.lvb;
  w.sc = h->ws.sc;
  w.part = h->ws.part;
  w.cfdm = h->lbase > 0 ? &h->cfdm : nullptr;
  return w;
}

template <typename T>
Cycle<T> make_cycle(dcg_ctx* h, const InnerWs& w) {
  Cycle<T> c(*h->mesh, *w.lvb, h->mp.pre, h->mp.post);
  c.base = h->lbase;
  c.group = h->opt.ras_group;
  c.cfdm = w.cfdm;
  if (h->ktime && h->kcycle++ % h->kstride == 0) {   // a sampled W-cycle
    c.timer.ev = h->kev;
    c.timer.max = dcg_ctx::kMaxTimed;
    c.timer.rec = &h->krec;
  }
  return c;
}

// Adds the elapsed times of the event pairs recorded since the last call
// (called after the stream has been synchronised).
void collect_kernel_times(dcg_ctx* h) {
  if (!h->ktime) return;
  for (int i = 0; i < h->krec; ++i) {
    float ms = 0.f;
    DCG_HIP(hipEventElapsedTime(&ms, h->kev[2 * i], h->kev[2 * i + 1]));
    h->ktime_ms += ms;
    ++h->klaunches;
  }
  h->krec = 0;
}

// Finest-level W-cycle from a zero initial guess; returns the finest state.
// The finest level's launches are issued directly (they are the long
// kernels, and the timed tile launches need real events); the coarse-grid
// correction below it -- two W-cycles of level J-1, about a hundred short
// launches -- is replayed as one captured HIP graph.
template <typename T>
LvState run_wcycle_finest(dcg_ctx* h, const InnerWs& w, hipStream_t st) {
  MeshContext& m = *h->mesh;
  const int J = m.J - h->lbase;   // levels of the cycle's own hierarchy
  const Cycle<T> cyc = make_cycle<T>(h, w);
  LvState s;
  if (J == 1 || !h->opt.use_graph || !w.graph) {
    cyc.wcycle(J, s, st);
    return s;
  }
  for (int i = 0; i < h->mp.pre; ++i) cyc.sweep_step(J, s, nullptr, st);
  cyc.restrict_step(J, s, st);
  if (!h->wgraph) {
    hipGraph_t g = nullptr;
    LvState c;
    DCG_HIP(hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal));
    try {
      cyc.coarse_correction(J, c, h->capture_stream);
    } catch (...) {
      (void)hipStreamEndCapture(h->capture_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    DCG_HIP(hipStreamEndCapture(h->capture_stream, &g));
    const hipError_t e = hipGraphInstantiate(&h->wgraph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    DCG_HIP(e);
    h->graph_state[0] = c.has_z;
    h->graph_state[1] = c.has_y;
    h->graph_state[2] = c.zb;
    h->graph_state[3] = c.yb;
  }
  DCG_HIP(hipGraphLaunch(h->wgraph, st));
  LvState c;
  c.has_z = h->graph_state[0];
  c.has_y = h->graph_state[1];
  c.zb = h->graph_state[2];
  c.yb = h->graph_state[3];
  cyc.post_smooth(J, s, c, st);
  return s;
}

// Resets the device scalar block and stores the operator parameters dt, 1/nu
// the kernels read from it.
void set_params(dcg_ctx* h, hipStream_t st) {
  Scalars init{};
  init.dt = h->dt;
  init.inv_nu = 1.0 / h->nu;
  *h->ws.sc_host = init;
  DCG_HIP(hipMemcpyAsync(h->ws.sc, h->ws.sc_host, sizeof(Scalars), hipMemcpyHostToDevice, st));
  DCG_HIP(hipStreamSynchronize(st));
}

void read_scalars(dcg_ctx* h, const Scalars* sc, hipStream_t st) {
  DCG_HIP(hipMemcpyAsync(h->ws.sc_host, sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
  DCG_HIP(hipStreamSynchronize(st));
}

void read_scalars(dcg_ctx* h, hipStream_t st) { read_scalars(h, h->ws.sc, st); }

// ------------------------------------------------------------ inner solve
// z ~= L^{-1} s (FP64) by the Multigrid iteration (Algorithm 3): W-cycles
// while ||s - L z|| / ||s|| > tol_c and fewer than max_inner cycles.  Each
// cycle is applied to the current FP64 residual and added in FP64, which for
// a linear cycle equals Wcycle(s, z) (iterative refinement form).  Returns
// the number of W-cycles.
//
// The test runs on the device (the reduction of ||s - L z||^2 sets the
// scalar block's inner_done), so the host enqueues cycles ahead of it: as
// many as the fewest the last inner solves took, then one at a time until
// the flag is read set.  A cycle enqueued after the test was met still runs
// its level kernels on scratch buffers, but its update of z, residual and
// count are no-ops, so z and the count are those of Algorithm 3.
template <typename T>
int inner_solve(dcg_ctx* h, const InnerWs& w, const double* s, double* z, double tol_c,
                hipStream_t st) {
  MeshContext& m = *h->mesh;
  const DeviceLevel& fine = m.lv[m.J - 1];
  const int64_t mlen = 4 * int64_t(fine.ne);
  T* fJ = static_cast<T*>(w.lvb->f[m.J - 1]);
  const int nb = refine_blocks(fine.ne);
  const int max_inner = h->opt.max_inner;
  const Scalars* guard = w.sc;
  DCG_HIP(launch_refine_residual<T>(true, fine.Lc64, fine.n, fine.ne, s, nullptr, fJ, w.part, st));
  DCG_HIP(launch_reduce(w.part, nb, kRedInnerS2, w.sc, st, Slots(), 1, tol_c * tol_c, max_inner));
  DCG_HIP(launch_fill<double>(mlen, 0.0, z, st));
  int ahead = max_inner;
  for (int c : h->inner_recent) ahead = std::min(ahead, c);
  ahead = std::max(ahead, 1);
  int enqueued = 0;
  while (true) {
    const int batch = std::min(ahead, max_inner - enqueued);
    for (int i = 0; i < batch; ++i, ++enqueued) {
      const LvState fs = run_wcycle_finest<T>(h, w, st);
      DCG_HIP(launch_refine_add<T>(fine.ne, false, fs.has_z, fs.has_y,
                                   static_cast<T*>(w.lvb->z[fs.zb][m.J - 1]),
                                   static_cast<T*>(w.lvb->Y[fs.yb][m.J - 1]), z, st, Slots(), 1,
                                   guard));
      DCG_HIP(launch_refine_residual<T>(false, fine.Lc64, fine.n, fine.ne, s, z, fJ, w.part, st,
                                        Slots(), 1, guard));
      DCG_HIP(launch_reduce(w.part, nb, kRedInnerR2, w.sc, st, Slots(), 1, 0.0, max_inner));
    }
    read_scalars(h, w.sc, st);
    collect_kernel_times(h);
    if (!std::isfinite(h->ws.sc_host->s2)) throw Error(DCG_EINVAL, "non-finite inner right-hand side");
    if (h->ws.sc_host->inner_done || enqueued >= max_inner) break;
    ahead = 1;
  }
  if (!std::isfinite(h->ws.sc_host->r2)) throw Error(DCG_EBREAKDOWN, "non-finite inner residual");
  const int cycles = h->ws.sc_host->inner_cycles;
  h->inner_recent[h->inner_next++ % dcg_ctx::kInnerRecent] = std::max(cycles, 1);
  return cycles;
}

int inner(dcg_ctx* h, const InnerWs& w, const double* s, double* z, double tol_c,
          hipStream_t st) {
  if (h->opt.inner == DCG_INNER_NONE) {   // no deflation: pi = 0 turns Algorithm 2 into CG on A*
    DCG_HIP(launch_fill<double>(4 * int64_t(h->mesh->ne), 0.0, z, st));
    return 0;
  }
  if (h->exact) {   // z = L^{-1} s exactly (fast diagonalisation); no W-cycles
    DCG_HIP(launch_fdm_solve2d(h->mesh->n, h->fV, h->fVT, h->flam, s, z, h->ft[0], h->ft[1], h->ft[2], st));
    return 0;
  }
  return h->fp32 ? inner_solve<float>(h, w, s, z, tol_c, st)
                 : inner_solve<double>(h, w, s, z, tol_c, st);
}

int inner(dcg_ctx* h, const double* s, double* z, double tol_c, hipStream_t st) {
  return inner(h, handle_ws(h), s, z, tol_c, st);
}

void check_ptr(const void* p, const char* what) {
  if (!p) throw Error(DCG_EINVAL, std::string(what) + " is NULL");
}

}  // namespace

void handle_init(dcg_ctx* h) {
  MeshContext& m = *h->mesh;
  Workspace& ws = h->ws;
  ws.ne = m.ne;
  const int64_t N = 16 * int64_t(m.ne), M = 4 * int64_t(m.ne);
  double** vecs[] = {&ws.xh, &ws.r, &ws.p[0], &ws.p[1], &ws.w, &ws.q};
  for (double** v : vecs) *v = static_cast<double*>(ws.alloc(sizeof(double) * N));
  double** svecs[] = {&ws.s, &ws.zref, &ws.zb, &ws.zt};
  for (double** v : svecs) *v = static_cast<double*>(ws.alloc(sizeof(double) * M));
  ws.part = static_cast<double*>(ws.alloc(sizeof(double) * 3 * kPartStride));
  ws.sc = static_cast<Scalars*>(ws.alloc(sizeof(Scalars)));
  DCG_HIP(hipHostMalloc(reinterpret_cast<void**>(&ws.sc_host), sizeof(Scalars), hipHostMallocDefault));
  std::memset(ws.sc_host, 0, sizeof(Scalars));
  DCG_HIP(hipMemcpy(ws.sc, ws.sc_host, sizeof(Scalars), hipMemcpyHostToDevice));
  ws.lvb.allocate(m, h->fp32, false, ws);
  LevelBuffers& nl = h->noalloc_lvb;
  nl.f.assign(m.J, nullptr);
  nl.rr.assign(m.J, nullptr);
  for (int b = 0; b < 2; ++b) {
    nl.z[b].assign(m.J, nullptr);
    nl.Y[b].assign(m.J, nullptr);
  }
  DCG_HIP(hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking));
  if (h->opt.inner == DCG_INNER_EXACT) {
    const FdmAxis f = fdm_axis_factor(m.n, h->mp.penalty * m.n, true);
    const int64_t NN = int64_t(f.N) * f.N;
    std::vector<double> vt(NN);
    for (int i = 0; i < f.N; ++i)
      for (int j = 0; j < f.N; ++j) vt[int64_t(j) * f.N + i] = f.V[int64_t(i) * f.N + j];
    h->fV = static_cast<double*>(ws.alloc(sizeof(double) * NN));
    h->fVT = static_cast<double*>(ws.alloc(sizeof(double) * NN));
    h->flam = static_cast<double*>(ws.alloc(sizeof(double) * f.N));
    for (double*& t : h->ft) t = static_cast<double*>(ws.alloc(sizeof(double) * M));
    DCG_HIP(hipMemcpy(h->fV, f.V.data(), sizeof(double) * NN, hipMemcpyHostToDevice));
    DCG_HIP(hipMemcpy(h->fVT, vt.data(), sizeof(double) * NN, hipMemcpyHostToDevice));
    DCG_HIP(hipMemcpy(h->flam, f.lam.data(), sizeof(double) * f.N, hipMemcpyHostToDevice));
    h->exact = true;
  }
  if (h->opt.inner == DCG_INNER_MG && h->opt.levels > 0 && h->opt.levels < m.J) {
    // shortened hierarchy: the coarsest level in use is stored level lbase + 1
    h->lbase = m.J - h->opt.levels;
    const FdmAxis f = fdm_coarse_axis(m.n, h->mp.penalty * m.n, h->opt.levels - 1);
    const int64_t NN = int64_t(f.N) * f.N;
    std::vector<double> vt(NN);
    for (int i = 0; i < f.N; ++i)
      for (int j = 0; j < f.N; ++j) vt[int64_t(j) * f.N + i] = f.V[int64_t(i) * f.N + j];
    double* V = static_cast<double*>(ws.alloc(sizeof(double) * NN));
    double* VT = static_cast<double*>(ws.alloc(sizeof(double) * NN));
    double* lam = static_cast<double*>(ws.alloc(sizeof(double) * f.N));
    for (double*& t : h->cfdm.t) t = static_cast<double*>(ws.alloc(sizeof(double) * NN));
    DCG_HIP(hipMemcpy(V, f.V.data(), sizeof(double) * NN, hipMemcpyHostToDevice));
    DCG_HIP(hipMemcpy(VT, vt.data(), sizeof(double) * NN, hipMemcpyHostToDevice));
    DCG_HIP(hipMemcpy(lam, f.lam.data(), sizeof(double) * f.N, hipMemcpyHostToDevice));
    h->cfdm.n = f.N / 2;
    h->cfdm.V = V;
    h->cfdm.VT = VT;
    h->cfdm.lam = lam;
  }
}

// ------------------------------------------------------------ stored directions
// (Re)sizes the slot tables of ``fs`` for R slots of vectors of length N.
void store_reserve(FcgStore& fs, int R, int64_t N) {
  if (fs.R == R) return;
  fs.release();
  fs.R = R;
  fs.d.assign(R, nullptr);
  fs.q.assign(R, nullptr);
  DCG_HIP(hipMalloc(&fs.dptr, sizeof(double*) * R));
  DCG_HIP(hipMalloc(&fs.qptr, sizeof(double*) * R));
  DCG_HIP(hipMalloc(&fs.dq, sizeof(double) * R));
  DCG_HIP(hipMalloc(&fs.coef, sizeof(double) * R));
  DCG_HIP(hipMalloc(&fs.coef2, sizeof(double) * R));
  DCG_HIP(hipMalloc(&fs.part, sizeof(double) * size_t(R) * fcg_coef_blocks(N)));
}

// Allocates the vectors of ``slot`` on first use (d, and q when ``with_q``)
// and publishes their addresses in the device pointer tables.
void store_slot(FcgStore& fs, int slot, int64_t N, bool with_q) {
  if (!fs.d[slot]) {
    fs.d[slot] = static_cast<double*>(fs.alloc(sizeof(double) * N));
    DCG_HIP(hipMemcpy(fs.dptr + slot, &fs.d[slot], sizeof(double*), hipMemcpyHostToDevice));
  }
  if (with_q && !fs.q[slot]) {
    fs.q[slot] = static_cast<double*>(fs.alloc(sizeof(double) * N));
    DCG_HIP(hipMemcpy(fs.qptr + slot, &fs.q[slot], sizeof(double*), hipMemcpyHostToDevice));
  }
}

// ------------------------------------------------------------ flexible CG
// Outer iterations of Algorithm 1 on the deflated system with the truncation
// of Remark 5: m_0 = 0, m_i = max{1, mod(i, m_max + 1)} (m_i = i for
// FCG(inf), m_max = 0).  Iteration i:
//   d_i = r_i - sum_{k = i - m_i}^{i - 1} (r_i, q_k) / (d_k, q_k) d_k
//   q_i = M_D d_i,  alpha = (d_i, r_i) / (d_i, q_i),  x += alpha d_i,  r -= alpha q_i.
// The directions live in a ring of m_max + 1 slots (FCG(inf): one slot per
// iteration, allocated as the iteration reaches it).
template <typename TolFn>
dcg_status outer_fcg(dcg_ctx* h, double lim, double& rho, int& it, int& cycles_total,
                     int& cycles_outer, int& inner_solves, TolFn tol_outer, hipStream_t st) {
  MeshContext& m = *h->mesh;
  Workspace& ws = h->ws;
  FcgStore& fs = ws.fcg;
  const int ne = m.ne;
  const int64_t N = 16 * int64_t(ne);
  const bool inf = h->opt.m_max == 0;
  const int R = inf ? h->opt.max_outer + 1 : h->opt.m_max + 1;
  store_reserve(fs, R, N);
  const int nbA = astar_blocks(ne);
  dcg_status status = DCG_OK;
  for (int i = 0;; ++i) {   // i: iteration of this pass (the window restarts with a pass)
    if (rho <= lim) break;
    if (it >= h->opt.max_outer) {
      status = DCG_NOT_CONVERGED;
      break;
    }
    const int mi = inf ? i : (i == 0 ? 0 : std::max(1, i % (h->opt.m_max + 1)));
    const int slot = i % R;
    store_slot(fs, slot, N, true);
    const int first = ((i - mi) % R + R) % R;
    // with the outer multigrid the direction is built from z_i = B r_i
    const double* base = ws.r;
    if (h->omg) {
      omg_apply(h, ws.r, h->omg->zp, st);
      base = h->omg->zp;
    }
    DCG_HIP(launch_fcg_coef(N, base, fs.qptr, fs.dq, first, mi, R, fs.part, fs.coef, st));
    int nbd = 0;
    DCG_HIP(launch_fcg_direction(N, base, ws.r, fs.dptr, first, mi, R, fs.coef, fs.d[slot], ws.part,
                                 &nbd, st));
    DCG_HIP(launch_reduce(ws.part, nbd, kRedDr, ws.sc, st));
    DCG_HIP(launch_astar(kAstarPlain, m.Cdiv, m.cols, m.M1, ne, fs.d[slot], nullptr, nullptr,
                         ws.sc, nullptr, ws.w, ws.s, nullptr, st));
    const int c = inner(h, ws.s, ws.zref, tol_outer(rho), st);
    cycles_total += c;
    cycles_outer += c;
    ++inner_solves;
    DCG_HIP(launch_deflate(false, m.AdivZ, m.cols, ne, kTwo, ws.zref, ws.w, fs.d[slot], fs.q[slot],
                           nullptr, ws.part, st));
    DCG_HIP(launch_reduce(ws.part, nbA, kRedFcgAlpha, ws.sc, st));   // alpha = (d, r) / (d, q)
    DCG_HIP(launch_copy<double>(1, &ws.sc->pq, fs.dq + slot, st));
    int nbu = 0;
    DCG_HIP(launch_cg_update(false, N, ws.sc, fs.d[slot], fs.q[slot], ws.xh, ws.r, ws.part, &nbu, st));
    DCG_HIP(launch_reduce(ws.part, nbu, kRedRho, ws.sc, st));
    ++it;
    read_scalars(h, st);
    if (ws.sc_host->breakdown) return DCG_EBREAKDOWN;
    rho = ws.sc_host->rho;
    if (!std::isfinite(rho)) return DCG_EBREAKDOWN;
  }
  return status;
}

// ------------------------------------------------------------ GMRES
// Unrestarted GMRES on the deflated system M_D x = f_D (Remark 6).  The
// Arnoldi basis v_0 = r / ||r||, v_{j+1} = (M_D v_j - sum_i h_ij v_i) / h_{j+1,j}
// lives on the device; each new vector is orthogonalised against the basis
// by two classical Gram-Schmidt passes (multi-dot, then one combined update,
// twice), which is as stable as modified Gram-Schmidt and needs two global
// reductions instead of j + 1.  The (j + 2) x (j + 1) Hessenberg column and
// its Givens rotations are handled on the host; the stopping test is the
// minimal residual |g_{j+1}| <= tol ||f||, and the inner tolerance of each
// product follows the current minimal residual.  x_hat = x_0 + V y at the end.
template <typename TolFn>
dcg_status outer_gmres(dcg_ctx* h, double lim, double& rho, int& it, int& cycles_total,
                       int& cycles_outer, int& inner_solves, TolFn tol_outer, hipStream_t st) {
  MeshContext& m = *h->mesh;
  Workspace& ws = h->ws;
  FcgStore& fs = ws.fcg;
  const int ne = m.ne;
  const int64_t N = 16 * int64_t(ne);
  const int R = h->opt.max_outer + 2;
  store_reserve(fs, R, N);
  double rnorm = std::sqrt(std::max(rho, 0.0));
  if (rho <= lim || it >= h->opt.max_outer)
    return rho <= lim ? DCG_OK : DCG_NOT_CONVERGED;
  const int it0 = it;   // the basis of this pass starts at slot 0
  store_slot(fs, 0, N, false);
  DCG_HIP(launch_scale(N, 1.0 / rnorm, ws.r, fs.d[0], st));
  std::vector<std::vector<double>> H;     // rotated Hessenberg columns
  std::vector<double> cs, sn, g{rnorm};
  std::vector<double> c1, c2;
  dcg_status status = DCG_OK;
  while (true) {
    if (rnorm * rnorm <= lim) break;
    if (it >= h->opt.max_outer) {
      status = DCG_NOT_CONVERGED;
      break;
    }
    const int j = it - it0;
    // q = M_D v_j
    DCG_HIP(launch_astar(kAstarPlain, m.Cdiv, m.cols, m.M1, ne, fs.d[j], nullptr, nullptr, ws.sc,
                         nullptr, ws.w, ws.s, nullptr, st));
    const int c = inner(h, ws.s, ws.zref, tol_outer(rnorm * rnorm), st);
    cycles_total += c;
    cycles_outer += c;
    ++inner_solves;
    DCG_HIP(launch_deflate(false, m.AdivZ, m.cols, ne, kTwo, ws.zref, ws.w, fs.d[j], ws.q, nullptr,
                           ws.part, st));
    // two Gram-Schmidt passes in place on q, then ||q||^2
    int nbd = 0;
    DCG_HIP(launch_fcg_coef(N, ws.q, fs.dptr, nullptr, 0, j + 1, R, fs.part, fs.coef, st));
    DCG_HIP(launch_fcg_direction(N, ws.q, nullptr, fs.dptr, 0, j + 1, R, fs.coef, ws.q, ws.part, &nbd, st));
    DCG_HIP(launch_fcg_coef(N, ws.q, fs.dptr, nullptr, 0, j + 1, R, fs.part, fs.coef2, st));
    DCG_HIP(launch_fcg_direction(N, ws.q, nullptr, fs.dptr, 0, j + 1, R, fs.coef2, ws.q, ws.part, &nbd, st));
    int nbu = 0;
    DCG_HIP(launch_axpy_dot(N, 0.0, ws.q, ws.q, ws.part, &nbu, st));
    DCG_HIP(launch_reduce(ws.part, nbu, kRedRho, ws.sc, st));
    read_scalars(h, st);
    c1.resize(j + 1);
    c2.resize(j + 1);
    DCG_HIP(hipMemcpy(c1.data(), fs.coef, sizeof(double) * (j + 1), hipMemcpyDeviceToHost));
    DCG_HIP(hipMemcpy(c2.data(), fs.coef2, sizeof(double) * (j + 1), hipMemcpyDeviceToHost));
    const double hn = std::sqrt(std::max(ws.sc_host->rho, 0.0));
    if (!std::isfinite(hn)) return DCG_EBREAKDOWN;
    std::vector<double> col(j + 2);
    for (int i = 0; i <= j; ++i) col[i] = -(c1[i] + c2[i]);
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {           // earlier rotations
      const double a = col[i], b = col[i + 1];
      col[i] = cs[i] * a + sn[i] * b;
      col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double den = std::hypot(col[j], col[j + 1]);
    if (!(den > 0.0)) return DCG_EBREAKDOWN;
    cs.push_back(col[j] / den);
    sn.push_back(col[j + 1] / den);
    col[j] = den;
    col[j + 1] = 0.0;
    g.push_back(-sn[j] * g[j]);
    g[j] = cs[j] * g[j];
    H.push_back(std::move(col));
    rnorm = std::fabs(g[j + 1]);
    ++it;
    if (hn > 0.0) {                          // hn = 0: invariant space, residual 0
      store_slot(fs, j + 1, N, false);
      DCG_HIP(launch_scale(N, 1.0 / hn, ws.q, fs.d[j + 1], st));
    }
  }
  rho = rnorm * rnorm;
  const int k = it - it0;
  if (k > 0) {                               // y = R^{-1} g, x_hat += V y
    std::vector<double> y(k);
    for (int r = k - 1; r >= 0; --r) {
      double acc = g[r];
      for (int cc = r + 1; cc < k; ++cc) acc -= H[cc][r] * y[cc];
      y[r] = acc / H[r][r];
    }
    DCG_HIP(hipMemcpy(fs.coef, y.data(), sizeof(double) * k, hipMemcpyHostToDevice));
    int nbd = 0;
    DCG_HIP(launch_fcg_direction(N, ws.xh, nullptr, fs.dptr, 0, k, R, fs.coef, ws.xh, ws.part, &nbd, st));
  }
  return status;
}

// ------------------------------------------------------------ solve
dcg_status solve(dcg_ctx* h, const double* b, double* x, double tol, dcg_stats* st,
                 hipStream_t stream) {
  check_ptr(b, "b");
  check_ptr(x, "x");
  if (!(tol >= 0.0) || !std::isfinite(tol)) throw Error(DCG_EINVAL, "tol must be finite and >= 0");
  const auto t0 = std::chrono::steady_clock::now();
  MeshContext& m = *h->mesh;
  Workspace& ws = h->ws;
  const int ne = m.ne;
  const int64_t N = 16 * int64_t(ne);
  const bool flex = h->opt.outer == DCG_OUTER_FCG1;
  // inner tolerances: eq. (fixed_tol) c_F tol, or eq. (tol) c_A tol ||b|| / ||r_i||
  // inside the outer loop with c_A tol for the prologue, start and epilogue solves
  const bool adaptive = h->opt.c_A > 0.0;
  const double tol_c = adaptive ? h->opt.c_A * tol : h->opt.c_F * tol;
  const int nbA = astar_blocks(ne);
  dcg_stats stats{};
  int cycles_total = 0, inner_solves = 0, cycles_outer = 0;
  set_params(h, stream);

  // prologue: pi(b) = Z E^{-1} Z^T b; f_D = b - A* pi(b) (eq. (defl_sys))
  DCG_HIP(launch_zt(ne, b, ws.s, stream));
  cycles_total += inner(h, ws.s, ws.zb, tol_c, stream);
  ++inner_solves;
  DCG_HIP(launch_deflate(true, m.AdivZ, m.cols, ne, kTwo, ws.zb, b, nullptr, ws.r, ws.p[0], ws.part,
                         stream));
  DCG_HIP(launch_reduce(ws.part, nbA, kRedB2Rho, ws.sc, stream));
  read_scalars(h, stream);
  const double b2 = ws.sc_host->b2;
  if (!std::isfinite(b2) || !std::isfinite(ws.sc_host->rho))
    throw Error(DCG_EINVAL, "b contains NaN or Inf");
  if (b2 == 0.0) {
    DCG_HIP(launch_fill<double>(N, 0.0, x, stream));
    DCG_HIP(hipStreamSynchronize(stream));
    stats.status = DCG_OK;
    stats.inner_solves = inner_solves;
    stats.t_setup_ms = h->t_setup_ms;
    stats.t_solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (st) *st = stats;
    return DCG_OK;
  }
  const double lim = tol * tol * b2;
  auto tol_outer = [&](double rho_i) {
    return adaptive ? h->opt.c_A * tol * std::sqrt(b2) / std::sqrt(rho_i) : tol_c;
  };
  int it = 0, pidx = 0, pass = 0;
  bool warm = h->opt.x0_given != 0;
  dcg_status status = DCG_OK;
  double rel_true = 0.0, rho = 0.0;
  while (true) {
    if (warm) {
      // x_hat_0 = x, r_0 = f_D - M_D x with M_D x = A* x - A* Z y_0,
      // y_0 = E^{-1} Z^T A* x (Algorithm 1 applied to the deflated system);
      // ws.r holds f_D
      DCG_HIP(launch_copy<double>(N, x, ws.xh, stream));
      DCG_HIP(launch_astar(kAstarPlain, m.Cdiv, m.cols, m.M1, ne, ws.xh, nullptr, nullptr,
                           ws.sc, nullptr, ws.w, ws.s, nullptr, stream));
      cycles_total += inner(h, ws.s, ws.zt, tol_c, stream);
      ++inner_solves;
      DCG_HIP(launch_deflate(false, m.AdivZ, m.cols, ne, kTwo, ws.zt, ws.w, ws.w, ws.q, nullptr,
                             ws.part, stream));
      int nbu = 0;
      DCG_HIP(launch_axpy_dot(N, -1.0, ws.q, ws.r, ws.part, &nbu, stream));
      DCG_HIP(launch_reduce(ws.part, nbu, kRedRho, ws.sc, stream));
      read_scalars(h, stream);
    } else {
      DCG_HIP(launch_fill<double>(N, 0.0, ws.xh, stream));
    }
    rho = ws.sc_host->rho;
    if (h->opt.outer == DCG_OUTER_FCG) {
      status = outer_fcg(h, lim, rho, it, cycles_total, cycles_outer, inner_solves, tol_outer,
                         stream);
    } else if (h->opt.outer == DCG_OUTER_GMRES) {
      status = outer_gmres(h, lim, rho, it, cycles_total, cycles_outer, inner_solves, tol_outer,
                           stream);
    } else {
      status = DCG_OK;
      for (int i = 0;; ++i) {   // i: iteration of this pass
        if (rho <= lim) break;
        if (it >= h->opt.max_outer) {
          status = DCG_NOT_CONVERGED;
          break;
        }
        // p_i = r_i + beta p_{i-1} fused into w = A* p_i, s = Z^T w
        const bool atimed = h->ktime;   // events recorded in the dispatch packet
        DCG_HIP(launch_astar(i == 0 ? kAstarFirst : kAstarDir, m.Cdiv, m.cols, m.M1, ne,
                             ws.r, ws.p[pidx], nullptr, ws.sc, ws.p[1 - pidx], ws.w, ws.s, nullptr,
                             stream, Slots(), 1, atimed ? h->aev[0] : nullptr,
                             atimed ? h->aev[1] : nullptr));
        pidx = 1 - pidx;
        const int c = inner(h, ws.s, ws.zref, tol_outer(rho), stream);
        cycles_total += c;
        cycles_outer += c;
        ++inner_solves;
        // q = w - A* Z y = M_D p  (y = (2/dt) z)
        DCG_HIP(launch_deflate(false, m.AdivZ, m.cols, ne, kTwo, ws.zref, ws.w, ws.p[pidx], ws.q,
                               nullptr, ws.part, stream));
        DCG_HIP(launch_reduce(ws.part, nbA, flex ? kRedFcgAlpha : kRedAlpha, ws.sc, stream));
        int nbu = 0;
        DCG_HIP(launch_cg_update(flex, N, ws.sc, ws.p[pidx], ws.q, ws.xh, ws.r, ws.part, &nbu,
                                 stream));
        DCG_HIP(launch_reduce(ws.part, nbu, flex ? kRedFcgBeta : kRedBeta, ws.sc, stream));
        ++it;
        read_scalars(h, stream);
        if (atimed) {   // both events have completed: read_scalars synchronised the stream
          float ms = 0.0f;
          DCG_HIP(hipEventElapsedTime(&ms, h->aev[0], h->aev[1]));
          h->atime_ms += ms;
          ++h->alaunches;
        }
        if (ws.sc_host->breakdown) {
          status = DCG_EBREAKDOWN;
          break;
        }
        rho = ws.sc_host->rho;
        if (!std::isfinite(rho)) {
          status = DCG_EBREAKDOWN;
          break;
        }
      }
    }
    stats.rel_res_recurrence = std::sqrt(std::max(rho, 0.0) / b2);

    // epilogue: x = (x_hat - pi(A* x_hat)) + pi(b)  (eq. (x_defl))
    DCG_HIP(launch_astar(kAstarPlain, m.Cdiv, m.cols, m.M1, ne, ws.xh, nullptr, nullptr,
                         ws.sc, nullptr, ws.w, ws.s, nullptr, stream));
    cycles_total += inner(h, ws.s, ws.zt, tol_c, stream);
    ++inner_solves;
    DCG_HIP(launch_reconstruct(ne, ws.xh, ws.zt, ws.zb, ws.sc, x, stream));
    DCG_HIP(launch_astar(kAstarResidual, m.Cdiv, m.cols, m.M1, ne, x, nullptr, b, ws.sc,
                         nullptr, ws.w, nullptr, ws.part, stream));
    DCG_HIP(launch_reduce(ws.part, nbA, kRedRes, ws.sc, stream));
    read_scalars(h, stream);
    rel_true = std::sqrt(ws.sc_host->res2 / b2);
    if (status != DCG_OK || rel_true <= tol || pass >= h->opt.restarts) break;
    // Algorithm 2 again from x_0 = x: restore r = f_D from the stored pi(b)
    ++pass;
    warm = true;
    DCG_HIP(launch_deflate(true, m.AdivZ, m.cols, ne, kTwo, ws.zb, b, nullptr, ws.r, ws.p[0],
                           ws.part, stream));
    DCG_HIP(launch_reduce(ws.part, nbA, kRedB2Rho, ws.sc, stream));
  }
  if (h->opt.restarts > 0 && status == DCG_OK && rel_true > tol) status = DCG_NOT_CONVERGED;
  stats.restarts = pass;
  stats.rel_res_true = rel_true;
  stats.status = status;
  stats.outer_iters = it;
  stats.total_wcycles = cycles_total;
  stats.inner_solves = inner_solves;
  stats.inner_per_outer = it > 0 ? double(cycles_outer) / it : 0.0;
  stats.t_setup_ms = h->t_setup_ms;
  stats.t_solve_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (st) *st = stats;
  if (status == DCG_EBREAKDOWN) throw Error(DCG_EBREAKDOWN, "outer iteration broke down ((p, q) <= 0 or non-finite)");
  return status;
}

void kernel_timing(dcg_ctx* h, int stride) {
  const bool enable = stride > 0;
  if (enable && !h->kev[0])
    for (hipEvent_t& e : h->kev) DCG_HIP(hipEventCreate(&e));
  if (enable && !h->aev[0])
    for (hipEvent_t& e : h->aev) DCG_HIP(hipEventCreate(&e));
  h->atime_ms = 0.0;
  h->alaunches = 0;
  if (h->wgraph) {
    DCG_HIP(hipGraphExecDestroy(h->wgraph));
    h->wgraph = nullptr;
  }
  h->ktime = enable;
  h->kstride = enable ? stride : 1;
  h->kcycle = 0;
  h->krec = 0;
  h->ktime_ms = 0.0;
  h->klaunches = 0;
}

// ------------------------------------------------------------ apply
namespace {

template <typename T>
void apply_level(dcg_ctx* h, dcg_op op, int k, const void* in, const void* in2, void* out,
                 hipStream_t st) {
  MeshContext& m = *h->mesh;
  if (k < 1 || k > m.J - h->lbase) throw Error(DCG_EINVAL, "level out of range");
  const DeviceLevel& d = m.lv[k - 1 + h->lbase];
  const int64_t mk = 4 * int64_t(d.ne);
  const T* x = static_cast<const T*>(in);
  T* y = static_cast<T*>(out);
  Cycle<T> cyc(m, h->ws.lvb, h->mp.pre, h->mp.post);
  cyc.base = h->lbase;
  cyc.group = h->opt.ras_group;
  if (h->lbase > 0) cyc.cfdm = &h->cfdm;
  switch (op) {
    case DCG_OP_LAPLACE:
      DCG_HIP(launch_lap<T>(false, level_L<T>(d), d.cols, d.ne, nullptr, x, y, st));
      break;
    case DCG_OP_RAS: {
      if (k < 2) throw Error(DCG_EINVAL, "RAS smoother exists on levels >= 2");
      check_ptr(in2, "in2 (z)");
      DCG_HIP(launch_copy<T>(mk, x, cyc.f(k), st));
      DCG_HIP(launch_copy<T>(mk, static_cast<const T*>(in2), cyc.z(k, 0), st));
      LvState s;
      s.has_z = true;
      cyc.sweep_step(k, s, nullptr, st);
      DCG_HIP(launch_resolve<T>(d.ne, s.has_z, cyc.z(k, s.zb), cyc.Y(k, s.yb), y, st));
      break;
    }
    case DCG_OP_RESTRICT:
      if (k < 2) throw Error(DCG_EINVAL, "restriction needs level >= 2");
      DCG_HIP(launch_restrict<T>(d.n / 2, x, y, st));
      break;
    case DCG_OP_PROLONG:
      if (k < 2) throw Error(DCG_EINVAL, "prolongation needs level >= 2");
      DCG_HIP(launch_fill<T>(mk, T(0), y, st));
      DCG_HIP(launch_prolong<T>(d.n / 2, x, y, st));
      break;
    case DCG_OP_COARSE:
      if (k != 1) throw Error(DCG_EINVAL, "coarse solve is on level 1");
      if (h->lbase > 0)
        DCG_HIP(launch_fdm_coarse<T>(h->cfdm.n, h->cfdm.V, h->cfdm.VT, h->cfdm.lam, x, y,
                                     h->cfdm.t[0], h->cfdm.t[1], h->cfdm.t[2], st));
      else
        DCG_HIP(launch_coarse<T>(m.coarse_inv, x, y, st));
      break;
    case DCG_OP_WCYCLE: {
      DCG_HIP(launch_copy<T>(mk, x, cyc.f(k), st));
      LvState s;
      if (in2) {
        DCG_HIP(launch_copy<T>(mk, static_cast<const T*>(in2), cyc.z(k, 0), st));
        s.has_z = true;
      }
      cyc.wcycle(k, s, st);
      if (s.has_y)
        DCG_HIP(launch_resolve<T>(d.ne, s.has_z, cyc.z(k, s.zb), cyc.Y(k, s.yb), y, st));
      else
        DCG_HIP(launch_copy<T>(mk, cyc.z(k, s.zb), y, st));
      break;
    }
    case DCG_OP_RAS_BATCH:
    case DCG_OP_WCYCLE_BATCH: {
      if (h->lbase > 0) throw Error(DCG_EINVAL, "the batched operators run the full hierarchy (levels = 0)");
      LevelBuffers& lb = h->ws.lvb_batch;
      if (lb.f.empty()) lb.allocate(m, h->fp32, true, h->ws);
      const Cycle<T> bc(m, lb, h->mp.pre, h->mp.post);
      const int64_t mb = mk * kBatch;
      const bool ras = op == DCG_OP_RAS_BATCH;
      if (ras && k < 2) throw Error(DCG_EINVAL, "RAS smoother exists on levels >= 2");
      if (ras) check_ptr(in2, "in2 (z)");
      if (h->mp.post < 1) throw Error(DCG_EINVAL, "the batched cycle needs post-smoothing (m2 >= 1)");
      DCG_HIP(launch_copy<T>(mb, x, bc.f(k), st));
      LvState s;
      if (in2) {
        DCG_HIP(launch_copy<T>(mb, static_cast<const T*>(in2), bc.z(k, 0), st));
        s.has_z = true;
      }
      if (ras)
        bc.sweep_step(k, s, nullptr, st);
      else
        bc.wcycle(k, s, st);
      if (s.has_y)
        DCG_HIP(launch_resolve_b<T>(d.ne, s.has_z, bc.z(k, s.zb), bc.Y(k, s.yb), y, st));
      else
        DCG_HIP(launch_copy<T>(mb, bc.z(k, s.zb), y, st));
      break;
    }
    default:
      throw Error(DCG_EINVAL, "unknown level operator");
  }
}

}  // namespace

dcg_status apply(dcg_ctx* h, dcg_op op, int level, const void* in, const void* in2, void* out,
                 hipStream_t st) {
  check_ptr(in, "in");
  check_ptr(out, "out");
  MeshContext& m = *h->mesh;
  const int ne = m.ne;
  const double* x = static_cast<const double*>(in);
  double* y = static_cast<double*>(out);
  if (op == DCG_OP_ASTAR || op == DCG_OP_DEFLATED) set_params(h, st);
  switch (op) {
    case DCG_OP_ASTAR:
      DCG_HIP(launch_astar(kAstarPlain, m.Cdiv, m.cols, m.M1, ne, x, nullptr,
                           nullptr, h->ws.sc, nullptr, y, nullptr, nullptr, st));
      break;
    case DCG_OP_ZT:
      DCG_HIP(launch_zt(ne, x, y, st));
      break;
    case DCG_OP_Z:
      DCG_HIP(launch_z(ne, x, 1.0, y, st));
      break;
    case DCG_OP_ADIVZ:
      DCG_HIP(launch_adivz(m.AdivZ, m.cols, ne, x, y, st));
      break;
    case DCG_OP_INNER: {
      inner(h, x, h->ws.zref, h->opt.c_F * kApplyTol, st);
      DCG_HIP(launch_scale(4 * int64_t(ne), 2.0 / h->dt, h->ws.zref, y, st));
      break;
    }
    case DCG_OP_DEFLATED: {
      DCG_HIP(launch_astar(kAstarPlain, m.Cdiv, m.cols, m.M1, ne, x, nullptr,
                           nullptr, h->ws.sc, nullptr, h->ws.w, h->ws.s, nullptr, st));
      inner(h, h->ws.s, h->ws.zref, h->opt.c_F * kApplyTol, st);
      DCG_HIP(launch_deflate(false, m.AdivZ, m.cols, ne, kTwo, h->ws.zref, h->ws.w, x, y, nullptr,
                             h->ws.part, st));
      break;
    }
    case DCG_OP_OMG_APPLY:
    case DCG_OP_OMG_LEVEL:
    case DCG_OP_OMG_RAS:
    case DCG_OP_OMG_RESTRICT:
    case DCG_OP_OMG_PROLONG:
    case DCG_OP_OMG_COARSE:
    case DCG_OP_OMG_WCYCLE:
      omg_apply_level(h, op, level, x, static_cast<const double*>(in2), y, st);
      break;
    default:
      if (h->fp32)
        apply_level<float>(h, op, level, in, in2, out, st);
      else
        apply_level<double>(h, op, level, in, in2, out, st);
  }
  DCG_HIP(hipStreamSynchronize(st));
  return DCG_OK;
}

}  // namespace dcg

namespace dcg {

// ------------------------------------------------------------ no-allocation apply
// dcg_apply_noalloc runs DCG_OP_INNER and DCG_OP_DEFLATED with every buffer
// its kernels write beside the caller's output -- scalars, partial sums, the
// inner iterate, the level vectors of the W-cycle, the coarsest-solve
// intermediates and, for DCG_OP_DEFLATED, A* p and Z^T A* p -- carved from
// one static device array instead of the handle's workspace.  Each device
// holds its own copy of the array (kNoallocBytes) until the process ends;
// its address on a device is read once with hipGetSymbolAddress, with that
// device current.  Calls that overlap on one device share the array and race.
constexpr size_t kNoallocBytes = size_t(48) << 20;

}  // namespace dcg

static __device__ __align__(256) unsigned char scratch[dcg::kNoallocBytes];

namespace dcg {
namespace {

std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch;   // device -> address of its scratch

unsigned char* scratch_address(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(device);
  if (it != g_scratch.end()) return it->second;
  void* ptr = nullptr;
  DCG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  unsigned char* p = static_cast<unsigned char*>(ptr);
  g_scratch[device] = p;
  return p;
}

// Bump allocation inside the scratch array (256-byte aligned pieces); with
// base == nullptr it only counts the bytes.
struct Carve {
  unsigned char* base;
  size_t used = 0;
  template <typename T>
  T* take(size_t count) {
    const size_t off = used;
    used += (sizeof(T) * count + 255) & ~size_t(255);
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
};

// Lays out the buffers of one call; returns the bytes it needs.
size_t noalloc_layout(dcg_ctx* h, bool deflated, unsigned char* base, InnerWs& w, double*& zref,
                      double*& wv, double*& sv, CoarseFdm& cf) {
  MeshContext& m = *h->mesh;
  const size_t rs = h->fp32 ? sizeof(float) : sizeof(double);
  Carve c{base};
  w.sc = c.take<Scalars>(1);
  w.part = c.take<double>(3 * size_t(kPartStride));
  zref = c.take<double>(4 * size_t(m.ne));
  wv = deflated ? c.take<double>(16 * size_t(m.ne)) : nullptr;
  sv = deflated ? c.take<double>(4 * size_t(m.ne)) : nullptr;
  LevelBuffers& lb = h->noalloc_lvb;
  for (int k = 1; k <= m.J; ++k) {
    const size_t ne = size_t(m.lv[k - 1].ne);
    lb.f[k - 1] = c.take<unsigned char>(rs * 4 * ne);
    lb.rr[k - 1] = c.take<unsigned char>(rs * 4 * ne);
    for (int b = 0; b < 2; ++b) {
      lb.z[b][k - 1] = c.take<unsigned char>(rs * 4 * ne);
      lb.Y[b][k - 1] = k >= 2 ? c.take<unsigned char>(rs * 12 * ne) : nullptr;
    }
  }
  w.lvb = &lb;
  w.cfdm = nullptr;
  w.graph = false;
  if (h->lbase > 0) {
    cf = h->cfdm;
    const size_t nn = size_t(2 * cf.n) * size_t(2 * cf.n);
    for (double*& t : cf.t) t = c.take<double>(nn);
    w.cfdm = &cf;
  }
  return c.used;
}

}  // namespace

size_t noalloc_capacity() { return kNoallocBytes; }

dcg_status apply_noalloc(dcg_ctx* h, dcg_op op, const double* in, double* out, hipStream_t st) {
  check_ptr(in, "in");
  check_ptr(out, "out");
  if (op != DCG_OP_INNER && op != DCG_OP_DEFLATED)
    throw Error(DCG_EINVAL, "dcg_apply_noalloc runs DCG_OP_INNER and DCG_OP_DEFLATED only");
  if (h->opt.inner != DCG_INNER_MG)
    throw Error(DCG_EINVAL, "dcg_apply_noalloc needs the multigrid inner solve (DCG_INNER_MG)");
  const bool deflated = op == DCG_OP_DEFLATED;
  InnerWs w;
  double *zref = nullptr, *wv = nullptr, *sv = nullptr;
  CoarseFdm cf;
  const size_t need = noalloc_layout(h, deflated, nullptr, w, zref, wv, sv, cf);
  if (need > kNoallocBytes)
    throw Error(DCG_EINVAL, "dcg_apply_noalloc: this mesh needs " + std::to_string(need) +
                                " bytes of scratch, the static array holds " +
                                std::to_string(kNoallocBytes) + " (n <= 256 fits)");
  noalloc_layout(h, deflated, scratch_address(h->device), w, zref, wv, sv, cf);
  MeshContext& m = *h->mesh;
  const int ne = m.ne;
  // the pending-output buffers of a level hold zeros in the cover slots no
  // block writes; the array keeps the previous call's values, so clear them
  for (int k = 2; k <= m.J; ++k)
    for (int b = 0; b < 2; ++b) {
      const int64_t len = 12 * int64_t(m.lv[k - 1].ne);
      if (h->fp32)
        DCG_HIP(launch_fill<float>(len, 0.f, static_cast<float*>(w.lvb->Y[b][k - 1]), st));
      else
        DCG_HIP(launch_fill<double>(len, 0.0, static_cast<double*>(w.lvb->Y[b][k - 1]), st));
    }
  if (deflated) {
    Scalars init{};
    init.dt = h->dt;
    init.inv_nu = 1.0 / h->nu;
    *h->ws.sc_host = init;
    DCG_HIP(hipMemcpyAsync(w.sc, h->ws.sc_host, sizeof(Scalars), hipMemcpyHostToDevice, st));
    DCG_HIP(launch_astar(kAstarPlain, m.Cdiv, m.cols, m.M1, ne, in, nullptr, nullptr, w.sc, nullptr,
                         wv, sv, nullptr, st));
    inner(h, w, sv, zref, h->opt.c_F * kApplyTol, st);
    DCG_HIP(launch_deflate(false, m.AdivZ, m.cols, ne, kTwo, zref, wv, in, out, nullptr, w.part, st));
  } else {
    inner(h, w, in, zref, h->opt.c_F * kApplyTol, st);
    DCG_HIP(launch_scale(4 * int64_t(ne), 2.0 / h->dt, zref, out, st));
  }
  DCG_HIP(hipStreamSynchronize(st));
  return DCG_OK;
}

}  // namespace dcg
