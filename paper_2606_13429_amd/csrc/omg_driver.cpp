// The outer multigrid preconditioner of a solver handle (omg.hpp): set-up of
// the A* hierarchy on the device, B(r) = Wcycle_J(r, 0) (Algorithm 4 on the
// hierarchy of A*, replayed as one captured HIP graph), and its level
// operators for dcg_apply.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "kernels.hpp"
#include "omg.hpp"
#include "runtime.hpp"

namespace dcg {

namespace {

constexpr int D = kOmgDofs;

template <typename T>
T* upload(Workspace& ws, const std::vector<T>& v) {
  T* d = static_cast<T*>(ws.alloc(v.size() * sizeof(T)));
  DCG_HIP(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return d;
}

enum { kZero = 0, kWarm = 1 };

int64_t level_len(const OuterMg& g, int k) { return (int64_t)D * g.n[k - 1] * g.n[k - 1]; }

void copy(const double* x, double* y, int64_t len, hipStream_t st) {
  if (x != y) DCG_HIP(hipMemcpyAsync(y, x, len * sizeof(double), hipMemcpyDeviceToDevice, st));
}

// The W-cycle on level k for f_k = g.f[k-1] into z_k = g.z[k-1].
void cycle(const OuterMg& g, int k, int mode, hipStream_t st) {
  const int i = k - 1, nk = g.n[i];
  if (k == 1) {
    DCG_HIP(launch_omg_dense(int(level_len(g, 1)), g.cinv, g.f[0], g.z[0], st));
    return;
  }
  for (int s = 0; s < g.m; ++s) {
    if (s == 0 && mode == kZero) {
      DCG_HIP(launch_omg_ras(nk, g.ras[i], g.rasm[i], g.f[i], g.z[i], true, st));
      continue;
    }
    DCG_HIP(launch_omg_res(nk, g.op[i], g.opm[i], g.f[i], g.z[i], g.r[i], st));
    DCG_HIP(launch_omg_ras(nk, g.ras[i], g.rasm[i], g.r[i], g.z[i], false, st));
  }
  DCG_HIP(launch_omg_res(nk, g.op[i], g.opm[i], g.f[i], g.z[i], g.r[i], st));
  DCG_HIP(launch_omg_restrict(nk, g.r[i], g.f[i - 1], st));
  cycle(g, k - 1, kZero, st);                 // gamma = 2 coarse cycles,
  if (k - 1 > 1) cycle(g, k - 1, kWarm, st);  // the exact solve once
  DCG_HIP(launch_omg_prolong(nk, g.z[i - 1], g.z[i], false, st));
  for (int s = 0; s < g.m; ++s) {
    DCG_HIP(launch_omg_res(nk, g.op[i], g.opm[i], g.f[i], g.z[i], g.r[i], st));
    DCG_HIP(launch_omg_ras(nk, g.ras[i], g.rasm[i], g.r[i], g.z[i], false, st));
  }
}

}  // namespace

OuterMg::~OuterMg() {
  if (graph) (void)hipGraphExecDestroy(graph);
}

void omg_setup(dcg_ctx* h) {
  Workspace& ws = h->ws;
  const OmgHierarchy H = build_omg(h->mesh->n, h->mp.penalty, h->dt, h->nu);
  auto g = std::make_unique<OuterMg>();
  g->J = int(H.lev.size());
  g->m = h->opt.outer_mg;
  for (int k = 1; k <= g->J; ++k) {
    const OmgLevel& L = H.lev[k - 1];
    const int64_t len = (int64_t)D * L.n * L.n;
    g->n.push_back(L.n);
    g->op.push_back(upload(ws, L.op));
    g->ras.push_back(k >= 2 ? upload(ws, L.ras) : nullptr);
    g->opm.push_back(upload(ws, omg_operand_order(omg_op_rows(L.op), kOmgOpClasses, kOmgOpCols)));
    g->rasm.push_back(k >= 2 ? upload(ws, omg_operand_order(L.ras, kOmgRasClasses, kOmgRasCols)) : nullptr);
    g->f.push_back(static_cast<double*>(ws.alloc(len * sizeof(double))));
    g->z.push_back(static_cast<double*>(ws.alloc(len * sizeof(double))));
    g->r.push_back(static_cast<double*>(ws.alloc(len * sizeof(double))));
  }
  g->cinv = upload(ws, H.coarse_inv);
  g->zp = static_cast<double*>(ws.alloc((int64_t)D * g->n[g->J - 1] * g->n[g->J - 1] * sizeof(double)));
  h->omg = std::move(g);
}

// z = B r on the finest level; replayed from a graph captured on first use.
void omg_apply(dcg_ctx* h, const double* r, double* z, hipStream_t st) {
  OuterMg& g = *h->omg;
  const int J = g.J;
  const int64_t len = level_len(g, J);
  if (!h->opt.use_graph) {
    copy(r, g.f[J - 1], len, st);
    cycle(g, J, kZero, st);
    copy(g.z[J - 1], z, len, st);
    return;
  }
  if (!g.graph || g.g_in != r || g.g_out != z) {
    if (g.graph) {
      DCG_HIP(hipGraphExecDestroy(g.graph));
      g.graph = nullptr;
    }
    hipGraph_t gr = nullptr;
    DCG_HIP(hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal));
    try {
      copy(r, g.f[J - 1], len, h->capture_stream);
      cycle(g, J, kZero, h->capture_stream);
      copy(g.z[J - 1], z, len, h->capture_stream);
    } catch (...) {
      (void)hipStreamEndCapture(h->capture_stream, &gr);
      if (gr) (void)hipGraphDestroy(gr);
      throw;
    }
    DCG_HIP(hipStreamEndCapture(h->capture_stream, &gr));
    const hipError_t e = hipGraphInstantiate(&g.graph, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    DCG_HIP(e);
    g.g_in = r;
    g.g_out = z;
  }
  DCG_HIP(hipGraphLaunch(g.graph, st));
}

void omg_apply_level(dcg_ctx* h, dcg_op op, int k, const double* in, const double* in2, double* out,
                     hipStream_t st) {
  if (!h->omg) throw Error(DCG_EINVAL, "the handle has no outer multigrid (opt.outer_mg = 0)");
  OuterMg& g = *h->omg;
  if (k < 1 || k > g.J) throw Error(DCG_EINVAL, "level out of range");
  const int i = k - 1, nk = g.n[i];
  const int64_t len = level_len(g, k);
  switch (op) {
    case DCG_OP_OMG_APPLY:
      if (k != g.J) throw Error(DCG_EINVAL, "DCG_OP_OMG_APPLY acts on the finest level");
      omg_apply(h, in, out, st);
      break;
    case DCG_OP_OMG_LEVEL:   // out = -(0 - A*_k in)
      DCG_HIP(launch_omg_res(nk, g.op[i], g.opm[i], nullptr, in, g.r[i], st));
      DCG_HIP(launch_scale(len, -1.0, g.r[i], out, st));
      break;
    case DCG_OP_OMG_RAS:
      if (k < 2) throw Error(DCG_EINVAL, "the coarsest level has no smoother");
      if (!in2) {
        DCG_HIP(launch_omg_ras(nk, g.ras[i], g.rasm[i], in, out, true, st));
      } else {
        copy(in2, out, len, st);
        DCG_HIP(launch_omg_res(nk, g.op[i], g.opm[i], in, in2, g.r[i], st));
        DCG_HIP(launch_omg_ras(nk, g.ras[i], g.rasm[i], g.r[i], out, false, st));
      }
      break;
    case DCG_OP_OMG_RESTRICT:
      if (k < 2) throw Error(DCG_EINVAL, "restriction needs level >= 2");
      DCG_HIP(launch_omg_restrict(nk, in, out, st));
      break;
    case DCG_OP_OMG_PROLONG:
      if (k < 2) throw Error(DCG_EINVAL, "prolongation needs level >= 2");
      DCG_HIP(launch_omg_prolong(nk, in, out, true, st));
      break;
    case DCG_OP_OMG_COARSE:
      if (k != 1) throw Error(DCG_EINVAL, "the exact solve is on level 1");
      DCG_HIP(launch_omg_dense(int(len), g.cinv, in, out, st));
      break;
    case DCG_OP_OMG_WCYCLE:
      copy(in, g.f[i], len, st);
      if (in2) copy(in2, g.z[i], len, st);
      cycle(g, k, in2 ? kWarm : kZero, st);
      copy(g.z[i], out, len, st);
      break;
    default:
      throw Error(DCG_EINVAL, "unknown outer multigrid operator");
  }
}

}  // namespace dcg
