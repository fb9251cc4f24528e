// extern "C" entry points of include/dcg.h: argument checks, handle
// management and conversion of library errors into dcg_status codes.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>

#include "fdm_host.hpp"
#include "omg.hpp"
#include "server.hpp"

namespace {

thread_local std::string g_last_error;

dcg_status fail(dcg_ctx* h, dcg_status s, const std::string& msg) {
  g_last_error = msg;
  if (h) h->last_error = msg;
  return s;
}

template <typename Fn>
dcg_status guarded(dcg_ctx* h, Fn fn) {
  try {
    return fn();
  } catch (const dcg::Error& e) {
    return fail(h, e.status, e.what());
  } catch (const std::bad_alloc&) {
    return fail(h, DCG_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(h, DCG_EINVAL, e.what());
  }
}

bool valid_mesh(const dcg_mesh& m, std::string& why) {
  if (dcg::num_levels(m.n) < 0) {
    why = "n must be 16 * 2^k with 16 <= n <= 2048";
    return false;
  }
  if (!(m.penalty > 0.0) || !std::isfinite(m.penalty)) {
    why = "penalty must be positive";
    return false;
  }
  if (m.pre < 0 || m.post < 0 || m.pre > 16 || m.post > 16) {
    why = "pre/post smoothing steps must be in [0, 16]";
    return false;
  }
  return true;
}

dcg_status check_options(const dcg_options& o) {
  if (o.prec != DCG_FP64 && o.prec != DCG_MIXED) return fail(nullptr, DCG_EINVAL, "bad precision");
  if (o.outer != DCG_OUTER_CG && o.outer != DCG_OUTER_FCG1 && o.outer != DCG_OUTER_FCG &&
      o.outer != DCG_OUTER_GMRES)
    return fail(nullptr, DCG_EINVAL, "bad outer variant");
  if (!(o.c_A >= 0.0) || !std::isfinite(o.c_A)) return fail(nullptr, DCG_EINVAL, "c_A must be >= 0");
  if (o.m_max < 0) return fail(nullptr, DCG_EINVAL, "m_max must be >= 0");
  if (o.inner != DCG_INNER_MG && o.inner != DCG_INNER_EXACT && o.inner != DCG_INNER_NONE)
    return fail(nullptr, DCG_EINVAL, "inner must be DCG_INNER_MG, DCG_INNER_EXACT or DCG_INNER_NONE");
  if (!(o.c_F > 0.0) || o.max_outer < 0 || o.max_inner < 1)
    return fail(nullptr, DCG_EINVAL, "c_F must be > 0, max_outer >= 0, max_inner >= 1");
  if (o.levels < 0) return fail(nullptr, DCG_EINVAL, "levels must be >= 0");
  if (o.restarts < 0) return fail(nullptr, DCG_EINVAL, "restarts must be >= 0");
  if (o.ras_group != 0 && o.ras_group != -1 && o.ras_group != 1 && o.ras_group != 2 &&
      o.ras_group != 4)
    return fail(nullptr, DCG_EINVAL, "ras_group must be 0, -1, 1, 2 or 4");
  if (o.outer_mg < 0) return fail(nullptr, DCG_EINVAL, "outer_mg must be >= 0");
  if (o.outer_mg > 0 && o.outer != DCG_OUTER_FCG)
    return fail(nullptr, DCG_EINVAL, "outer_mg needs the flexible outer iteration (DCG_OUTER_FCG)");
  return DCG_OK;
}

}  // namespace

extern "C" {

void dcg_defaults(dcg_mesh* mesh, dcg_options* opt) {
  if (mesh) {
    mesh->n = 512;
    mesh->penalty = 10.0;
    mesh->pre = 2;
    mesh->post = 2;
  }
  if (opt) {
    std::memset(opt, 0, sizeof *opt);
    opt->prec = DCG_MIXED;
    opt->outer = DCG_OUTER_CG;
    opt->c_F = 0.01;
    opt->max_outer = 50000;
    opt->max_inner = 100;
    opt->x0_given = 0;
    opt->use_graph = 1;
    opt->hbm_budget_bytes = 0;
    opt->max_pending = 4096;
    opt->c_A = 0.0;
    opt->m_max = 8;
    opt->smooth3d = 10;
  }
}

int32_t dcg_num_levels(int32_t n) { return dcg::num_levels(n); }

dcg_status dcg_setup(const dcg_mesh* mesh, double dt, double nu, const dcg_options* opt,
                     dcg_handle* out) {
  if (!mesh || !out) return fail(nullptr, DCG_EINVAL, "mesh and out must not be NULL");
  *out = nullptr;
  std::string why;
  if (!valid_mesh(*mesh, why)) return fail(nullptr, DCG_EINVAL, why);
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(nullptr, DCG_EINVAL, "dt must be positive");
  if (!(nu > 0.0) || !std::isfinite(nu)) return fail(nullptr, DCG_EINVAL, "nu must be positive");
  dcg_options o;
  dcg_defaults(nullptr, &o);
  if (opt) o = *opt;
  if (const dcg_status cs = check_options(o); cs != DCG_OK) return cs;
  if (o.inner == DCG_INNER_EXACT && mesh->n > 1024)
    return fail(nullptr, DCG_EINVAL, "DCG_INNER_EXACT needs n <= 1024");
  if (o.levels > dcg::num_levels(mesh->n))
    return fail(nullptr, DCG_EINVAL, "levels exceeds log2(n/16) + 1");
  if (o.levels > 0 && (mesh->n >> (o.levels - 1)) > 1024)
    return fail(nullptr, DCG_EINVAL, "levels leaves a coarsest level above 1024 x 1024 squares");
  dcg_ctx* h = nullptr;
  const dcg_status st = guarded(nullptr, [&]() {
    const auto t0 = std::chrono::steady_clock::now();
    h = new dcg_ctx();
    DCG_HIP(hipGetDevice(&h->device));
    h->mp = *mesh;
    h->opt = o;
    h->dt = dt;
    h->nu = nu;
    h->fp32 = o.prec == DCG_MIXED;
    h->mesh = dcg::get_context(mesh->n, mesh->penalty, h->fp32);
    dcg::handle_init(h);
    if (o.outer_mg > 0) dcg::omg_setup(h);
    h->t_setup_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return DCG_OK;
  });
  if (st != DCG_OK) {
    delete h;
    return st;
  }
  *out = h;
  return DCG_OK;
}

dcg_status dcg_solve(dcg_handle h, const double* b, double* x, double tol, dcg_stats* st,
                     void* hip_stream) {
  if (!h) return fail(nullptr, DCG_EINVAL, "NULL handle");
  return guarded(h, [&]() {
    return dcg::solve(h, b, x, tol, st, static_cast<hipStream_t>(hip_stream));
  });
}

dcg_status dcg_apply(dcg_handle h, dcg_op op, int32_t level, const void* in, const void* in2,
                     void* out, void* hip_stream) {
  if (!h) return fail(nullptr, DCG_EINVAL, "NULL handle");
  return guarded(h, [&]() {
    return dcg::apply(h, op, level, in, in2, out, static_cast<hipStream_t>(hip_stream));
  });
}

dcg_status dcg_apply_noalloc(dcg_handle h, dcg_op op, const double* in, double* out,
                             void* hip_stream) {
  if (!h) return fail(nullptr, DCG_EINVAL, "NULL handle");
  return guarded(h, [&]() {
    int cur = 0;
    DCG_HIP(hipGetDevice(&cur));
    if (cur != h->device) DCG_HIP(hipSetDevice(h->device));
    try {
      const dcg_status s = dcg::apply_noalloc(h, op, in, out, static_cast<hipStream_t>(hip_stream));
      if (cur != h->device) DCG_HIP(hipSetDevice(cur));
      return s;
    } catch (...) {
      if (cur != h->device) (void)hipSetDevice(cur);
      throw;
    }
  });
}

int64_t dcg_noalloc_bytes(void) { return int64_t(dcg::noalloc_capacity()); }

dcg_status dcg_host_outer_mg(int32_t n, double penalty, double dt, double nu, int32_t level,
                             int32_t which, double* dst, int64_t dst_len) {
  if (!dst) return fail(nullptr, DCG_EINVAL, "dst is NULL");
  const int J = dcg::omg_num_levels(n);
  if (J < 2 || n > 64) return fail(nullptr, DCG_EINVAL, "n must be 16 2^k <= 64");
  if (!(penalty > 0.0) || !(dt > 0.0) || !(nu > 0.0))
    return fail(nullptr, DCG_EINVAL, "penalty, dt and nu must be positive");
  if (level < 1 || level > J) return fail(nullptr, DCG_EINVAL, "level out of range");
  if (which < 0 || which > 4 || ((which == 1 || which == 4) && level < 2) || (which == 2 && level != 1))
    return fail(nullptr, DCG_EINVAL, "which must be 0, 1 (level >= 2), 2 (level 1), 3 or 4 (level >= 2)");
  return guarded(nullptr, [&]() -> dcg_status {
    const dcg::OmgHierarchy H = dcg::build_omg(n, penalty, dt, nu);
    const dcg::OmgLevel& L = H.lev[level - 1];
    std::vector<double> ordered;
    if (which == 3) ordered = dcg::omg_operand_order(dcg::omg_op_rows(L.op), dcg::kOmgOpClasses, dcg::kOmgOpCols);
    if (which == 4) ordered = dcg::omg_operand_order(L.ras, dcg::kOmgRasClasses, dcg::kOmgRasCols);
    const std::vector<double>& src =
        which == 0 ? L.op : (which == 1 ? L.ras : (which == 2 ? H.coarse_inv : ordered));
    if (dst_len < (int64_t)src.size()) return fail(nullptr, DCG_EINVAL, "dst too small");
    std::copy(src.begin(), src.end(), dst);
    return DCG_OK;
  });
}

dcg_status dcg_host_assemble(const dcg_mesh* mesh, int32_t which, int32_t level, double* dst,
                             int64_t dst_len, int32_t* cols, int64_t cols_len, int64_t* needed) {
  if (!mesh) return fail(nullptr, DCG_EINVAL, "mesh must not be NULL");
  std::string why;
  if (!valid_mesh(*mesh, why)) return fail(nullptr, DCG_EINVAL, why);
  if (which < 0 || which > 7) return fail(nullptr, DCG_EINVAL, "which must be in [0, 7]");
  if (which == 7) {   // fast-diagonalisation factors of the coarsest level of `level` levels
    if (level < 1 || level > dcg::num_levels(mesh->n))
      return fail(nullptr, DCG_EINVAL, "level out of range");
    if ((mesh->n >> (level - 1)) > 256) return fail(nullptr, DCG_EINVAL, "which = 7 needs a coarsest n <= 256");
    return guarded(nullptr, [&]() -> dcg_status {
      const dcg::FdmAxis f = dcg::fdm_coarse_axis(mesh->n, mesh->penalty * mesh->n, level - 1);
      const int64_t need = int64_t(f.N) * f.N + f.N;
      if (needed) *needed = need;
      if (dst) {
        if (dst_len < need) return fail(nullptr, DCG_EINVAL, "dst too small");
        std::copy(f.V.begin(), f.V.end(), dst);
        std::copy(f.lam.begin(), f.lam.end(), dst + int64_t(f.N) * f.N);
      }
      return DCG_OK;
    });
  }
  if (which == 6) {   // fast-diagonalisation factors of the exact inner solve: V then lambda
    if (mesh->n > 256) return fail(nullptr, DCG_EINVAL, "which = 6 needs n <= 256");
    return guarded(nullptr, [&]() -> dcg_status {
      const dcg::FdmAxis f = dcg::fdm_axis_factor(mesh->n, mesh->penalty * mesh->n, true);
      const int64_t need = int64_t(f.N) * f.N + f.N;
      if (needed) *needed = need;
      if (dst) {
        if (dst_len < need) return fail(nullptr, DCG_EINVAL, "dst too small");
        std::copy(f.V.begin(), f.V.end(), dst);
        std::copy(f.lam.begin(), f.lam.end(), dst + int64_t(f.N) * f.N);
      }
      return DCG_OK;
    });
  }
  return guarded(nullptr, [&]() -> dcg_status {
    const int J = dcg::num_levels(mesh->n);
    if ((which == 3 || which == 4) && (level < 1 || level > J))
      return fail(nullptr, DCG_EINVAL, "level out of range");
    if (which == 4 && level < 2) return fail(nullptr, DCG_EINVAL, "RAS tiles exist on levels >= 2");
    dcg::HostContext hc;
    dcg::build_host_context(mesh->n, mesh->penalty, which == 4, which == 5, hc);
    const int64_t ne = int64_t(mesh->n) * mesh->n;
    std::vector<double> tmp;
    const std::vector<double>* src = nullptr;
    const std::vector<int32_t>* csrc = nullptr;
    switch (which) {
      case 0: src = &hc.Adiv; csrc = &hc.cols; break;
      case 1: src = &hc.AdivZ; csrc = &hc.cols; break;
      case 2: src = &hc.M1; break;
      case 3: src = &hc.levels[level - 1].L; csrc = &hc.levels[level - 1].cols; break;
      case 4: {
        const dcg::HostLevel& hl = hc.levels[level - 1];
        const size_t per = size_t(dcg::kTileDofs) * dcg::kTileDofs;
        tmp.resize(per * hl.tiles);
        for (int t = 0; t < hl.tiles; ++t) {      // F[j][i] = (L_k)_t^{-1}[j][i] d_i
          const double* inv = hl.unique_inv[hl.tile_class[t]].data();
          for (int i = 0; i < dcg::kTileDofs; ++i) {
            const int32_t e = hl.tile_elems[int64_t(t) * dcg::kTileSlots + i / 4];
            const double di = e >= 0 ? hl.dw[e] : 0.0;
            for (int j = 0; j < dcg::kTileDofs; ++j)
              tmp[per * t + size_t(j) * dcg::kTileDofs + i] = inv[size_t(j) * dcg::kTileDofs + i] * di;
          }
        }
        src = &tmp;
        csrc = &hl.tile_elems;
        break;
      }
      case 5: src = &hc.coarse_inv; break;
    }
    (void)ne;
    if (needed) *needed = int64_t(src->size());
    if (!dst) return DCG_OK;
    if (dst_len < int64_t(src->size())) return fail(nullptr, DCG_EINVAL, "dst buffer too small");
    std::memcpy(dst, src->data(), src->size() * sizeof(double));
    if (cols && csrc) {
      if (cols_len < int64_t(csrc->size())) return fail(nullptr, DCG_EINVAL, "cols buffer too small");
      std::memcpy(cols, csrc->data(), csrc->size() * sizeof(int32_t));
    }
    return DCG_OK;
  });
}

dcg_status dcg_bdf2_rhs(dcg_handle h, const double* s1, const double* s2, const double* F,
                        double c, double* f, double* x0, void* hip_stream) {
  if (!h) return fail(nullptr, DCG_EINVAL, "NULL handle");
  if (!s1 || !s2 || !F || !f || !x0) return fail(h, DCG_EINVAL, "NULL vector");
  if (f == s1 || f == s2 || x0 == s1 || x0 == s2 || f == x0)
    return fail(h, DCG_EINVAL, "f and x0 must not alias the inputs or each other");
  if (!std::isfinite(c)) return fail(h, DCG_EINVAL, "c must be finite");
  return guarded(h, [&]() {
    const hipStream_t st = static_cast<hipStream_t>(hip_stream);
    DCG_HIP(dcg::launch_bdf2_rhs(h->mesh->ne, h->mesh->M1, 1.0 / h->nu, s1, s2, F, c, f, x0, st));
    DCG_HIP(hipStreamSynchronize(st));
    return DCG_OK;
  });
}

dcg_status dcg_kernel_timing(dcg_handle h, int32_t enable) {
  if (!h) return fail(nullptr, DCG_EINVAL, "NULL handle");
  if (enable < 0) return fail(h, DCG_EINVAL, "enable must be >= 0");
  return guarded(h, [&]() {
    dcg::kernel_timing(h, enable);
    return DCG_OK;
  });
}

dcg_status dcg_kernel_timing_read(dcg_handle h, double* total_ms, int64_t* launches) {
  if (!h) return fail(nullptr, DCG_EINVAL, "NULL handle");
  if (total_ms) *total_ms = h->ktime_ms;
  if (launches) *launches = h->klaunches;
  return DCG_OK;
}

dcg_status dcg_kernel_timing_read_astar(dcg_handle h, double* total_ms, int64_t* launches) {
  if (!h) return fail(nullptr, DCG_EINVAL, "NULL handle");
  if (total_ms) *total_ms = h->atime_ms;
  if (launches) *launches = h->alaunches;
  return DCG_OK;
}

dcg_status dcg_server_create(const dcg_options* opt, dcg_server* out) {
  if (!out) return fail(nullptr, DCG_EINVAL, "out must not be NULL");
  *out = nullptr;
  dcg_options o;
  dcg_defaults(nullptr, &o);
  if (opt) o = *opt;
  if (const dcg_status cs = check_options(o); cs != DCG_OK) return cs;
  if (o.outer_mg > 0) return fail(nullptr, DCG_EINVAL, "the server runs no outer multigrid (outer_mg = 0)");
  if (o.max_pending < 1) return fail(nullptr, DCG_EINVAL, "max_pending must be >= 1");
  if (o.outer == DCG_OUTER_FCG || o.outer == DCG_OUTER_GMRES)
    return fail(nullptr, DCG_EINVAL, "the server runs DCG_OUTER_CG or DCG_OUTER_FCG1");
  if (o.inner != DCG_INNER_MG) return fail(nullptr, DCG_EINVAL, "the server runs DCG_INNER_MG");
  if (o.levels != 0) return fail(nullptr, DCG_EINVAL, "the server runs the full hierarchy (levels = 0)");
  if (o.hbm_budget_bytes < 0) return fail(nullptr, DCG_EINVAL, "hbm_budget_bytes must be >= 0");
  return guarded(nullptr, [&]() {
    auto s = std::make_unique<dcg_srv>();
    s->server = std::make_unique<dcg::Server>(o);
    *out = s.release();
    return DCG_OK;
  });
}

dcg_status dcg_server_prepare(dcg_server s, const dcg_mesh* mesh) {
  if (!s || !mesh) return fail(nullptr, DCG_EINVAL, "server and mesh must not be NULL");
  std::string why;
  if (!valid_mesh(*mesh, why)) return fail(nullptr, DCG_EINVAL, why);
  return guarded(nullptr, [&]() {
    s->server->prepare(*mesh);
    return DCG_OK;
  });
}

dcg_status dcg_submit(dcg_server s, const dcg_mesh* mesh, double dt, double nu, const double* b,
                      double* x, double tol, uint64_t* ticket) {
  if (!s || !mesh || !ticket) return fail(nullptr, DCG_EINVAL, "server, mesh and ticket must not be NULL");
  std::string why;
  if (!valid_mesh(*mesh, why)) return fail(nullptr, DCG_EINVAL, why);
  if (mesh->post < 1) return fail(nullptr, DCG_EINVAL, "the server needs post >= 1");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(nullptr, DCG_EINVAL, "dt must be positive");
  if (!(nu > 0.0) || !std::isfinite(nu)) return fail(nullptr, DCG_EINVAL, "nu must be positive");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(nullptr, DCG_EINVAL, "tol must be finite and >= 0");
  if (!b || !x) return fail(nullptr, DCG_EINVAL, "b and x must not be NULL");
  return guarded(nullptr, [&]() { return s->server->submit(*mesh, dt, nu, b, x, tol, ticket); });
}

dcg_status dcg_poll(dcg_server s, uint64_t ticket, dcg_stats* st) {
  if (!s) return fail(nullptr, DCG_EINVAL, "NULL server");
  return guarded(nullptr, [&]() {
    std::string err;
    const dcg_status r = s->server->poll(ticket, st, &err);
    if (r < 0) g_last_error = err;
    return r;
  });
}

int64_t dcg_server_group_bytes(const dcg_mesh* mesh, dcg_precision prec) {
  std::string why;
  if (!mesh || !valid_mesh(*mesh, why) || (prec != DCG_FP64 && prec != DCG_MIXED)) return -1;
  return dcg::Server::group_bytes(mesh->n, prec == DCG_MIXED);
}

dcg_status dcg_server_counters(dcg_server s, int64_t* steps, int64_t* slot_steps) {
  if (!s) return fail(nullptr, DCG_EINVAL, "NULL server");
  s->server->counters(steps, slot_steps);
  return DCG_OK;
}

dcg_status dcg_server_destroy(dcg_server s) {
  if (!s) return fail(nullptr, DCG_EINVAL, "NULL server");
  return guarded(nullptr, [&]() {
    delete s;
    return DCG_OK;
  });
}

dcg_status dcg_destroy(dcg_handle h) {
  delete h;
  return DCG_OK;
}

const char* dcg_strerror(dcg_status s) {
  switch (s) {
    case DCG_OK: return "ok";
    case DCG_NOT_CONVERGED: return "not converged (max_outer reached)";
    case DCG_PENDING: return "pending";
    case DCG_EINVAL: return "invalid argument";
    case DCG_ENOMEM: return "out of memory";
    case DCG_EDEVICE: return "device error";
    case DCG_EAGAIN: return "queue full, try again";
    case DCG_ENOTFOUND: return "unknown ticket";
    case DCG_EBREAKDOWN: return "breakdown of the outer iteration";
  }
  return "unknown status";
}

const char* dcg_last_error(dcg_handle h) {
  return h ? h->last_error.c_str() : g_last_error.c_str();
}

void dcg_clear_cache(void) { dcg::clear_context_cache(); }

}  // extern "C"
