// Mesh contexts: host assembly (host_setup.cpp) converted to the device
// layouts of kernels.hpp and uploaded once per (device, n, penalty).
#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <thread>
#include <tuple>

#include "runtime.hpp"

namespace dcg {

void hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  const dcg_status s = (e == hipErrorOutOfMemory) ? DCG_ENOMEM : DCG_EDEVICE;
  throw Error(s, std::string(what) + ": " + hipGetErrorString(e));
}

void* MeshContext::alloc(size_t b) {
  void* p = nullptr;
  DCG_HIP(hipMalloc(&p, b));
  allocations.push_back(p);
  bytes += b;
  return p;
}

MeshContext::~MeshContext() {
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(device);
  for (void* p : allocations) (void)hipFree(p);
  (void)hipSetDevice(cur);
}

namespace {

template <typename Fn>
void threaded(int64_t count, Fn fn) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (count < 1024) nt = 1;
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([=, &fn]() {
      for (int64_t i = count * t / nt; i < count * (t + 1) / nt; ++i) fn(i);
    });
  for (auto& x : th) x.join();
}

// Uploads a [ne][slot][rows][cols] block array into the device layout
// double2 [slot][cols/2][ne][rows] in chunks of squares.
void upload_blocks_pairs(const std::vector<double>& host, int64_t ne, int rows, int ncol,
                         double2* dev) {
  const int kcs = ncol / 2;
  const int64_t chunk = 1 << 15;
  std::vector<double2> stage(size_t(chunk) * kSlots * kcs * rows);
  for (int64_t e0 = 0; e0 < ne; e0 += chunk) {
    const int64_t cnt = std::min(chunk, ne - e0);
    threaded(cnt, [&](int64_t de) {
      const int64_t e = e0 + de;
      for (int s = 0; s < kSlots; ++s)
        for (int kc = 0; kc < kcs; ++kc)
          for (int r = 0; r < rows; ++r) {
            const double* src = &host[((e * kSlots + s) * rows + r) * ncol + 2 * kc];
            stage[((size_t(s) * kcs + kc) * cnt + de) * rows + r] = make_double2(src[0], src[1]);
          }
    });
    for (int s = 0; s < kSlots; ++s)
      for (int kc = 0; kc < kcs; ++kc)
        DCG_HIP(hipMemcpy(dev + ((int64_t(s) * kcs + kc) * ne + e0) * rows,
                          &stage[(size_t(s) * kcs + kc) * cnt * rows], sizeof(double2) * cnt * rows,
                          hipMemcpyHostToDevice));
  }
}

// The div-div form acts on each row sigma_k = (sigma_k1, sigma_k2) of the
// stress separately and identically (Section 3.3.2), so every 16 x 16 block of
// A_div is diag(C, C) in the ordering (sigma_11, sigma_12 | sigma_21, sigma_22)
// x 4 corners, C 8 x 8.  Returns the C blocks [ne][slot][8][8] after checking
// that structure exactly.
std::vector<double> row_blocks(const std::vector<double>& A, int64_t ne) {
  std::vector<double> C(size_t(ne) * kSlots * 64);
  for (int64_t b = 0; b < ne * kSlots; ++b) {
    const double* a = &A[size_t(b) * 256];
    for (int r = 0; r < 16; ++r)
      for (int c = 0; c < 16; ++c) {
        const bool diag = (r < 8) == (c < 8);
        const double v = a[r * 16 + c];
        if (!diag ? v != 0.0 : v != a[(r % 8) * 16 + (c % 8)])
          throw Error(DCG_EDEVICE, "A_div block is not diag(C, C)");
      }
    for (int r = 0; r < 8; ++r)
      for (int c = 0; c < 8; ++c) C[size_t(b) * 64 + r * 8 + c] = a[r * 16 + c];
  }
  return C;
}

void upload_cols(const std::vector<int32_t>& host, int64_t ne, int32_t* dev) {
  std::vector<int32_t> t(size_t(ne) * kSlots);
  for (int64_t e = 0; e < ne; ++e)
    for (int s = 0; s < kSlots; ++s) t[size_t(s) * ne + e] = host[e * kSlots + s];
  DCG_HIP(hipMemcpy(dev, t.data(), t.size() * sizeof(int32_t), hipMemcpyHostToDevice));
}

template <typename T>
void upload_level_L(const HostLevel& hl, T* dev) {
  const int64_t ne = int64_t(hl.n) * hl.n;
  std::vector<T> t(size_t(ne) * kSlots * 16);
  for (int64_t e = 0; e < ne; ++e)
    for (int s = 0; s < kSlots; ++s)
      for (int k = 0; k < 16; ++k) t[(size_t(s) * ne + e) * 16 + k] = T(hl.L[(e * kSlots + s) * 16 + k]);
  DCG_HIP(hipMemcpy(dev, t.data(), t.size() * sizeof(T), hipMemcpyHostToDevice));
}

// Inverses of the distinct local problems in the packed symmetric layout of
// the sweep kernel: per class the 36 upper 16 x 16 blocks (P <= Q, row by
// row), each row-major.  Tiles address them through their class.
template <typename T>
void upload_factors(const HostLevel& hl, T* dev) {
  const int64_t per = 36 * 256;
  const int chunk = 512;
  const int classes = int(hl.unique_inv.size());
  std::vector<T> stage(size_t(chunk) * per);
  for (int t0 = 0; t0 < classes; t0 += chunk) {
    const int cnt = std::min(chunk, classes - t0);
    threaded(cnt, [&](int64_t dt) {
      const std::vector<double>& src = hl.unique_inv[t0 + dt];
      T* d = &stage[size_t(dt) * per];
      int b = 0;
      for (int P = 0; P < 8; ++P)
        for (int Q = P; Q < 8; ++Q, ++b)
          for (int ri = 0; ri < 16; ++ri)
            for (int ci = 0; ci < 16; ++ci)
              d[b * 256 + ri * 16 + ci] = T(src[size_t(16 * P + ri) * kTileDofs + 16 * Q + ci]);
    });
    DCG_HIP(hipMemcpy(dev + int64_t(t0) * per, stage.data(), sizeof(T) * cnt * per,
                      hipMemcpyHostToDevice));
  }
}

// The same inverses in the operand order of the grouped RAS step's MFMA
// products: per class [P 8][Q 8][lane 64][4], lane l of fragment (P, Q)
// holding row 16 P + l % 16, columns 16 Q + 4 (l / 16) .. + 3, so that each
// lane's operand of one 16 x 16 x 4 step is one contiguous vector and a
// fragment is one contiguous 1 KiB (FP32) run.
template <typename T>
void upload_fragments(const HostLevel& hl, T* dev) {
  const int64_t per = 64 * 64 * 4;
  const int classes = int(hl.unique_inv.size());
  std::vector<T> stage(size_t(classes) * per);
  threaded(classes, [&](int64_t c) {
    const std::vector<double>& src = hl.unique_inv[c];
    T* d = &stage[size_t(c) * per];
    for (int P = 0; P < 8; ++P)
      for (int Q = 0; Q < 8; ++Q)
        for (int l = 0; l < 64; ++l)
          for (int kk = 0; kk < 4; ++kk)
            d[((P * 8 + Q) * 64 + l) * 4 + kk] =
                T(src[size_t(16 * P + l % 16) * kTileDofs + 16 * Q + 4 * (l / 16) + kk]);
  });
  DCG_HIP(hipMemcpy(dev, stage.data(), sizeof(T) * stage.size(), hipMemcpyHostToDevice));
}

// The grouped RAS step derives the pending slot and the weight of a block
// square from the tile geometry instead of reading the tables: the blocks
// containing a square are its own tile and the neighbour tile on each side
// where the square lies on the core's edge (inside the domain), the pending
// slot is the writer's rank among them in increasing tile order (the order
// of the cover lists), and the weight is one over their number.  Checked
// here against the tables the host built, for every tile and block square.
void check_tile_geometry(const HostLevel& hl) {
  const int n = hl.n, tpr = n / 4;
  for (int t = 0; t < hl.tiles; ++t)
    for (int p = 0; p < kTileSlots; ++p) {
      const int32_t e = hl.tile_elems[int64_t(t) * kTileSlots + p];
      if (e < 0) continue;
      const int X = int(e % n), Y = int(e / n);
      const int TX = X >> 2, TY = Y >> 2, lx = X & 3, ly = Y & 3, T = TY * tpr + TX;
      const bool below = ly == 0 && TY > 0, left = lx == 0 && TX > 0;
      const bool right = lx == 3 && TX < tpr - 1, above = ly == 3 && TY < tpr - 1;
      const int count = 1 + below + left + right + above;
      const int rank = (below && T - tpr < t) + (left && T - 1 < t) + (T < t) +
                       (right && T + 1 < t) + (above && T + tpr < t);
      if (hl.tile_dst[int64_t(t) * kTileSlots + p] != 3 * e + rank || hl.dw[e] != 1.0 / count)
        throw Error(DCG_EINVAL, "RAS tile geometry differs from the cover lists");
    }
}

// Extra workgroups of the grouped RAS step with g x g tiles per group: for
// every group (row-major), the classes of its tiles in order of first
// appearance (tiles row by row within the group); the first is run by the
// group's own workgroup, every further one by an extra workgroup listed as
// (group, class).
std::vector<int32_t> group_extra(const HostLevel& hl, int g) {
  std::vector<int32_t> out;
  const int tpr = hl.n / kTileCore;
  if (tpr % g) return out;
  const int gpr = tpr / g;
  for (int G = 0; G < gpr * gpr; ++G) {
    std::vector<int32_t> seen;
    for (int i = 0; i < g * g; ++i) {
      const int t = (G / gpr * g + i / g) * tpr + G % gpr * g + i % g;
      const int32_t c = hl.tile_class[t];
      if (std::find(seen.begin(), seen.end(), c) != seen.end()) continue;
      if (!seen.empty()) {
        out.push_back(G);
        out.push_back(c);
      }
      seen.push_back(c);
    }
  }
  return out;
}

// The level operator's blocks per square class ([9][5][4][4], see
// square_class); every square of a class must carry bit-identical blocks,
// which the uniform grid guarantees and this checks.
std::vector<double> square_class_table(const HostLevel& hl) {
  const int n = hl.n;
  if (n < 3) throw Error(DCG_EINVAL, "level grid below 3 x 3 squares");
  std::vector<double> Lc(9 * kSlots * 16, 0.0);
  std::vector<char> seen(9, 0);
  for (int64_t e = 0; e < int64_t(n) * n; ++e) {
    const int c = square_class(int(e % n), int(e / n), n);
    const double* src = &hl.L[e * kSlots * 16];
    double* dst = &Lc[size_t(c) * kSlots * 16];
    if (!seen[c]) {
      std::memcpy(dst, src, sizeof(double) * kSlots * 16);
      seen[c] = 1;
    } else if (std::memcmp(dst, src, sizeof(double) * kSlots * 16) != 0) {
      throw Error(DCG_EINVAL, "level operator blocks differ within a square class");
    }
  }
  return Lc;
}

template <typename T>
T* upload_class_table(MeshContext* ctx, const std::vector<double>& Lc) {
  std::vector<T> t(Lc.begin(), Lc.end());
  T* dev = static_cast<T*>(ctx->alloc(sizeof(T) * t.size()));
  DCG_HIP(hipMemcpy(dev, t.data(), sizeof(T) * t.size(), hipMemcpyHostToDevice));
  return dev;
}

template <typename T>
void upload_weights(const HostLevel& hl, T* dev) {
  std::vector<T> t(hl.dw.size());
  for (size_t i = 0; i < t.size(); ++i) t[i] = T(hl.dw[i]);
  DCG_HIP(hipMemcpy(dev, t.data(), t.size() * sizeof(T), hipMemcpyHostToDevice));
}

struct Key {
  int device, n;
  double penalty;
  bool operator<(const Key& o) const {
    return std::tie(device, n, penalty) < std::tie(o.device, o.n, o.penalty);
  }
};
std::mutex g_cache_mu;
std::map<Key, std::shared_ptr<MeshContext>> g_cache;

std::shared_ptr<MeshContext> build_context(int device, int n, double penalty) {
  auto t0 = std::chrono::steady_clock::now();
  auto ctx = std::make_shared<MeshContext>();
  ctx->device = device;
  ctx->host = std::make_unique<HostContext>();
  HostContext& hc = *ctx->host;
  try {
    build_host_context(n, penalty, true, true, hc);
  } catch (const std::exception& ex) {
    throw Error(DCG_EINVAL, ex.what());
  }
  ctx->n = n;
  ctx->J = hc.J;
  ctx->ne = n * n;
  ctx->penalty = penalty;
  const int64_t ne = ctx->ne;
  ctx->Cdiv = static_cast<double2*>(ctx->alloc(sizeof(double) * ne * kSlots * 64));
  ctx->AdivZ = static_cast<double2*>(ctx->alloc(sizeof(double) * ne * kSlots * 64));
  ctx->M1 = static_cast<double*>(ctx->alloc(sizeof(double) * ne * 16));
  ctx->cols = static_cast<int32_t*>(ctx->alloc(sizeof(int32_t) * ne * kSlots));
  upload_blocks_pairs(row_blocks(hc.Adiv, ne), ne, 8, 8, ctx->Cdiv);
  upload_blocks_pairs(hc.AdivZ, ne, 16, 4, ctx->AdivZ);
  DCG_HIP(hipMemcpy(ctx->M1, hc.M1.data(), sizeof(double) * ne * 16, hipMemcpyHostToDevice));
  upload_cols(hc.cols, ne, ctx->cols);
  // the tensor blocks are not needed on the host any more
  std::vector<double>().swap(hc.Adiv);
  std::vector<double>().swap(hc.AdivZ);
  std::vector<double>().swap(hc.M1);
  ctx->lv.resize(hc.J);
  for (int k = 1; k <= hc.J; ++k) {
    const HostLevel& hl = hc.levels[k - 1];
    DeviceLevel& dl = ctx->lv[k - 1];
    dl.n = hl.n;
    dl.ne = hl.n * hl.n;
    dl.cols = static_cast<int32_t*>(ctx->alloc(sizeof(int32_t) * dl.ne * kSlots));
    upload_cols(hl.cols, dl.ne, dl.cols);
    // FP64 level operator: the refinement residual needs it at the finest
    // level and the FP64 form at every level
    dl.L64 = static_cast<double*>(ctx->alloc(sizeof(double) * dl.ne * kSlots * 16));
    upload_level_L<double>(hl, dl.L64);
    dl.Lc64 = upload_class_table<double>(ctx.get(), square_class_table(hl));
    if (k >= 2) {
      dl.tiles = hl.tiles;
      dl.tile_ext = static_cast<int32_t*>(ctx->alloc(sizeof(int32_t) * hl.tile_ext.size()));
      DCG_HIP(hipMemcpy(dl.tile_ext, hl.tile_ext.data(), sizeof(int32_t) * hl.tile_ext.size(),
                        hipMemcpyHostToDevice));
      dl.tile_dst = static_cast<int32_t*>(ctx->alloc(sizeof(int32_t) * hl.tile_dst.size()));
      DCG_HIP(hipMemcpy(dl.tile_dst, hl.tile_dst.data(), sizeof(int32_t) * hl.tile_dst.size(),
                        hipMemcpyHostToDevice));
      dl.classes = int(hl.unique_inv.size());
      for (int32_t c : hl.tile_class)
        if (c < 0 || c >= dl.classes) throw Error(DCG_EINVAL, "tile class out of range");
      check_tile_geometry(hl);
      for (int gi = 0; gi < 3; ++gi) {
        const std::vector<int32_t> ex = group_extra(hl, 1 << gi);
        dl.gx_extra_n[gi] = int(ex.size() / 2);
        if (ex.empty()) continue;
        dl.gx_extra[gi] = static_cast<int32_t*>(ctx->alloc(sizeof(int32_t) * ex.size()));
        DCG_HIP(hipMemcpy(dl.gx_extra[gi], ex.data(), sizeof(int32_t) * ex.size(),
                          hipMemcpyHostToDevice));
      }
      dl.fcls = static_cast<int32_t*>(ctx->alloc(sizeof(int32_t) * hl.tile_class.size()));
      DCG_HIP(hipMemcpy(dl.fcls, hl.tile_class.data(), sizeof(int32_t) * hl.tile_class.size(),
                        hipMemcpyHostToDevice));
    }
  }
  ctx->coarse_inv = static_cast<double*>(ctx->alloc(sizeof(double) * kCoarseDofs * kCoarseDofs));
  DCG_HIP(hipMemcpy(ctx->coarse_inv, hc.coarse_inv.data(),
                    sizeof(double) * kCoarseDofs * kCoarseDofs, hipMemcpyHostToDevice));
  ctx->t_build_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return ctx;
}

}  // namespace

void MeshContext::ensure_factors(bool fp32) {
  std::lock_guard<std::mutex> lk(mu);
  if (fp32 ? have_f32 : have_f64) return;
  if (!host) throw Error(DCG_EDEVICE, "mesh context lost its host data");
  int cur = 0;
  DCG_HIP(hipGetDevice(&cur));
  DCG_HIP(hipSetDevice(device));
  for (int k = 1; k <= J; ++k) {
    const HostLevel& hl = host->levels[k - 1];
    DeviceLevel& dl = lv[k - 1];
    if (fp32) {
      dl.L32 = static_cast<float*>(alloc(sizeof(float) * dl.ne * kSlots * 16));
      upload_level_L<float>(hl, dl.L32);
      dl.Lc32 = upload_class_table<float>(this, square_class_table(hl));
    }
    if (k >= 2) {
      const size_t cnt = size_t(dl.classes) * 36 * 256;
      const size_t fcnt = size_t(dl.classes) * 64 * 64 * 4;
      if (fp32) {
        dl.F32 = static_cast<float*>(alloc(sizeof(float) * cnt));
        upload_factors<float>(hl, dl.F32);
        dl.Fm32 = static_cast<float*>(alloc(sizeof(float) * fcnt));
        upload_fragments<float>(hl, dl.Fm32);
        dl.dw32 = static_cast<float*>(alloc(sizeof(float) * dl.ne));
        upload_weights<float>(hl, dl.dw32);
      } else {
        dl.F64 = static_cast<double*>(alloc(sizeof(double) * cnt));
        upload_factors<double>(hl, dl.F64);
        dl.Fm64 = static_cast<double*>(alloc(sizeof(double) * fcnt));
        upload_fragments<double>(hl, dl.Fm64);
        dl.dw64 = static_cast<double*>(alloc(sizeof(double) * dl.ne));
        upload_weights<double>(hl, dl.dw64);
      }
    }
  }
  (fp32 ? have_f32 : have_f64) = true;
  if (have_f32 && have_f64) host.reset();
  DCG_HIP(hipSetDevice(cur));
}

std::shared_ptr<MeshContext> get_context(int n, double penalty, bool fp32) {
  int device = 0;
  DCG_HIP(hipGetDevice(&device));
  std::shared_ptr<MeshContext> ctx;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find(Key{device, n, penalty});
    if (it != g_cache.end()) ctx = it->second;
  }
  if (!ctx) {
    auto built = build_context(device, n, penalty);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find(Key{device, n, penalty});
    if (it != g_cache.end()) {
      ctx = it->second;          // another thread won the race
    } else {
      g_cache[Key{device, n, penalty}] = built;
      ctx = built;
    }
  }
  ctx->ensure_factors(fp32);
  return ctx;
}

void release_context_if_unused(int n, double penalty) {
  int device = 0;
  DCG_HIP(hipGetDevice(&device));
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto it = g_cache.find(Key{device, n, penalty});
  if (it != g_cache.end() && it->second.use_count() == 1) g_cache.erase(it);
}

void clear_context_cache() {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_cache.clear();
}

}  // namespace dcg
