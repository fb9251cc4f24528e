// Serving engine: continuous batching of deflated-CG solves (Algorithm 2)
// that share a mesh.
//
// Requests with the same (n, penalty, m1, m2) form a group with kBatch
// request slots.  The group's dt-independent operators are the cached mesh
// context; dt and nu of each request live in its slot of the device scalar
// block, so requests of any dt share every matrix.  A server thread runs
// the groups in steps; one step advances every occupied slot by one unit:
//
//   * the outer-iteration work due for the slot (prologue deflation, the CG
//     update of Algorithm 2, the epilogue reconstruction), each as one
//     launch over the slots that need it (blockIdx.y = slot);
//   * one W-cycle (Algorithm 4) of the inner Multigrid iteration (Algorithm
//     3) for every slot that is inside an inner solve -- a single batched
//     cycle over all kBatch columns, the RAS tile solves as MFMA products;
//   * one copy of the kBatch scalar blocks to the host.
//
// The host then applies each slot's own tests -- inner convergence, outer
// convergence, max_outer, breakdown -- exactly as the single-request solver
// does, so a request performs the same iterations whatever shares its
// group.  A slot that finishes is refilled at the next step boundary.
//
// Two speculations save one step per inner solve and per outer iteration:
// a step that starts an inner solve also runs its first W-cycle (dropped if
// the inner right-hand side turns out to be zero), and the step that ends an
// outer iteration also starts the next one (dropped when the iteration has
// converged or reached max_outer).  Dropped work writes only buffers that
// the taken path overwrites before reading.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <tuple>
#include <unordered_map>

#include "server.hpp"
#include "wcycle.hpp"

namespace dcg {
namespace {

using Clock = std::chrono::steady_clock;
constexpr double kTwo = 2.0;   // A* Z (2/dt) z = 2 A_div Z z  (Z^T A* Z = (dt/2) L)

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

enum class Stage {
  kPro,       // prologue: s = Z^T b, inner solve for pi(b)
  kInner,     // inside an inner solve: one more W-cycle
  kPostPro,   // f_D = b - A* pi(b); then the first direction
  kPostIter,  // q = M_D p, CG update; then the next direction
  kEpi,       // A* x_hat, inner solve for pi(A* x_hat)
  kPostEpi    // x = (x_hat - pi(A* x_hat)) + pi(b), true residual
};
enum class Kind { kPro, kIter, kEpi };

struct Request {
  uint64_t ticket = 0;
  dcg_mesh mesh{};
  double dt = 0.0, nu = 1.0, tol = 0.0;
  const double* b = nullptr;
  double* x = nullptr;
  Clock::time_point t_submit, t_admit;
  dcg_status status = DCG_PENDING;
  dcg_stats stats{};
  std::string error;
};

struct Slot {
  Request* req = nullptr;
  bool in_step = false;   // part of the step in flight
  Stage stage = Stage::kPro;
  Kind kind = Kind::kPro;
  int cycles = 0;         // W-cycles of the current inner solve
  double inner_lim = 0.0;
  bool zero_inner = false;  // the inner result must be replaced by 0
  int it = 0, pidx = 0;
  int cycles_total = 0, cycles_outer = 0, inner_solves = 0;
  double b2 = 0.0, rho = 0.0, lim = 0.0;
  dcg_status final_status = DCG_OK;
};

struct GroupKey {
  int n, pre, post;
  double penalty;
  bool operator<(const GroupKey& o) const {
    return std::tie(n, pre, post, penalty) < std::tie(o.n, o.pre, o.post, o.penalty);
  }
};

// Launch lists of one step (indices into the pinned/device list block).
enum List : int {
  kLZt, kLDeflPro, kLDeflIter0, kLDeflIter1, kLAstarFirst, kLAstarDir0, kLAstarDir1,
  kLAstarPlain, kLInnerStart, kLInnerAll, kLAddFirst, kLAddMore, kLPostEpi, kNumLists
};

struct Group {
  GroupKey key{};
  std::shared_ptr<MeshContext> mesh;
  Workspace ws;
  int64_t N = 0, M = 0;   // tensor and scalar vector lengths
  double *b = nullptr, *xh = nullptr, *r = nullptr, *p[2] = {nullptr, nullptr};
  double *w = nullptr, *q = nullptr, *s = nullptr, *zref = nullptr, *zb = nullptr;
  Scalars* sc_init = nullptr;   // pinned, per-slot initial scalar blocks
  int32_t* lists_dev = nullptr;
  int32_t* lists_host = nullptr;   // pinned [kNumLists][kBatch]
  int counts[kNumLists] = {};
  hipStream_t stream = nullptr, capture = nullptr;
  hipEvent_t done = nullptr;
  hipGraphExec_t graph = nullptr;
  LvState graph_state;
  Slot slots[kBatch];
  int active = 0;
  bool inflight = false;
  bool any_cycle = false;
  Clock::time_point last_used;
  ~Group();
};

Group::~Group() {
  if (graph) (void)hipGraphExecDestroy(graph);
  if (done) (void)hipEventDestroy(done);
  if (stream) (void)hipStreamDestroy(stream);
  if (capture) (void)hipStreamDestroy(capture);
  if (sc_init) (void)hipHostFree(sc_init);
  if (lists_host) (void)hipHostFree(lists_host);
}

// Bytes of the per-group device workspace for mesh size n.
size_t workspace_bytes(int n, bool fp32) {
  const size_t ne = size_t(n) * n, N = 16 * ne, M = 4 * ne;
  size_t b = kBatch * (7 * N + 3 * M) * sizeof(double);
  b += kBatch * size_t(kSlotPart) * sizeof(double) + kBatch * sizeof(Scalars);
  b += kNumLists * kBatch * sizeof(int32_t);
  const size_t rs = fp32 ? 4 : 8;
  for (int nk = n; nk >= kCoarsestN; nk /= 2) {
    const size_t nek = size_t(nk) * nk;
    b += rs * kBatch * nek * (4 + 8 + (nk > kCoarsestN ? 24 : 0));
  }
  return b;
}

// Bytes of a mesh context (the allocations of the context upload).
size_t context_bytes(int n, bool fp32) {
  const size_t ne = size_t(n) * n;
  size_t b = ne * kSlots * (64 + 64) * sizeof(double) + ne * 16 * sizeof(double) +
             ne * kSlots * sizeof(int32_t);
  for (int nk = n; nk >= kCoarsestN; nk /= 2) {
    const size_t nek = size_t(nk) * nk;
    b += nek * kSlots * (sizeof(int32_t) + 16 * sizeof(double) + (fp32 ? 16 * sizeof(float) : 0));
    if (nk > kCoarsestN) {
      const size_t tiles = nek / 16;
      // distinct local problems: 9 on the uniform grid (3 x 3 tile positions)
      const size_t classes = std::min<size_t>(tiles, 16);
      b += tiles * (52 + 32 + 1) * sizeof(int32_t);
      b += (classes * 36 * 256 + nek) * (fp32 ? sizeof(float) : sizeof(double));
    }
  }
  return b + size_t(kCoarseDofs) * kCoarseDofs * sizeof(double);
}

}  // namespace

struct Server::Impl {
  dcg_options opt{};
  int device = 0;
  bool fp32 = true;
  size_t budget = 0;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> requests;   // unfinished + unpolled
  std::deque<Request*> queue;                                        // not yet admitted
  int unfinished = 0;
  // owned by the server thread
  std::map<GroupKey, std::unique_ptr<Group>> groups;
  std::atomic<int64_t> steps{0}, slot_steps{0};
  std::thread thread;

  void run();
  void step_all();
  void admit();
  bool make_room(size_t need);
  size_t used_bytes() const;
  Group* create_group(const GroupKey& key);
  void assign(Group& g, int i, Request* r);
  void enqueue_step(Group& g);
  void process(Group& g);
  void after_inner_start(Group& g, Slot& s, const Scalars& sc);
  void inner_done(Slot& s);
  void finish(Group& g, Slot& s, dcg_status st, const std::string& err = std::string());
  void fail_group(Group& g, const Error& e);
  void set_params(Group& g, int i);
};

namespace {

Slots slot_addr(const Group& g, int list) {
  Slots sl;
  sl.list = g.lists_dev + list * kBatch;
  sl.tstride = g.N;
  sl.sstride = g.M;
  sl.lstride = 4;
  sl.lsq = 4 * kBatch;
  return sl;
}

}  // namespace

size_t Server::Impl::used_bytes() const {
  size_t b = 0;
  std::map<int, size_t> ctx;
  for (const auto& kv : groups) {
    b += kv.second->ws.bytes;
    ctx[kv.first.n] = kv.second->mesh->bytes;
  }
  for (const auto& kv : ctx) b += kv.second;
  return b;
}

// Frees idle groups (oldest first) until ``need`` more bytes fit the budget.
bool Server::Impl::make_room(size_t need) {
  while (used_bytes() + need > budget) {
    auto victim = groups.end();
    for (auto it = groups.begin(); it != groups.end(); ++it)
      if (it->second->active == 0 && !it->second->inflight &&
          (victim == groups.end() || it->second->last_used < victim->second->last_used))
        victim = it;
    if (victim == groups.end()) return false;
    const int n = victim->first.n;
    const double pen = victim->first.penalty;
    groups.erase(victim);
    release_context_if_unused(n, pen);
  }
  return true;
}

Group* Server::Impl::create_group(const GroupKey& key) {
  auto g = std::make_unique<Group>();
  g->key = key;
  g->mesh = get_context(key.n, key.penalty, fp32);
  const MeshContext& m = *g->mesh;
  g->N = 16 * int64_t(m.ne);
  g->M = 4 * int64_t(m.ne);
  Workspace& ws = g->ws;
  ws.ne = m.ne;
  auto vec = [&](int64_t len) { return static_cast<double*>(ws.alloc(sizeof(double) * kBatch * len)); };
  g->b = vec(g->N);
  g->xh = vec(g->N);
  g->r = vec(g->N);
  g->p[0] = vec(g->N);
  g->p[1] = vec(g->N);
  g->w = vec(g->N);
  g->q = vec(g->N);
  g->s = vec(g->M);
  g->zref = vec(g->M);
  g->zb = vec(g->M);
  ws.part = static_cast<double*>(ws.alloc(sizeof(double) * kBatch * kSlotPart));
  ws.sc = static_cast<Scalars*>(ws.alloc(sizeof(Scalars) * kBatch));
  DCG_HIP(hipMemset(ws.sc, 0, sizeof(Scalars) * kBatch));
  g->lists_dev = static_cast<int32_t*>(ws.alloc(sizeof(int32_t) * kNumLists * kBatch));
  DCG_HIP(hipHostMalloc(reinterpret_cast<void**>(&ws.sc_host), sizeof(Scalars) * kBatch,
                        hipHostMallocDefault));
  DCG_HIP(hipHostMalloc(reinterpret_cast<void**>(&g->sc_init), sizeof(Scalars) * kBatch,
                        hipHostMallocDefault));
  DCG_HIP(hipHostMalloc(reinterpret_cast<void**>(&g->lists_host),
                        sizeof(int32_t) * kNumLists * kBatch, hipHostMallocDefault));
  ws.lvb.allocate(m, fp32, true, ws);
  DCG_HIP(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
  DCG_HIP(hipStreamCreateWithFlags(&g->capture, hipStreamNonBlocking));
  DCG_HIP(hipEventCreateWithFlags(&g->done, hipEventDisableTiming));
  g->last_used = Clock::now();
  Group* raw = g.get();
  groups[key] = std::move(g);
  return raw;
}

void Server::Impl::set_params(Group& g, int i) {
  const Request& r = *g.slots[i].req;
  Scalars init{};
  init.dt = r.dt;
  init.inv_nu = 1.0 / r.nu;
  g.sc_init[i] = init;
  DCG_HIP(hipMemcpyAsync(g.ws.sc + i, g.sc_init + i, sizeof(Scalars), hipMemcpyHostToDevice,
                         g.stream));
}

void Server::Impl::assign(Group& g, int i, Request* r) {
  Slot& s = g.slots[i];
  s = Slot();
  s.req = r;
  r->t_admit = Clock::now();
  set_params(g, i);
  DCG_HIP(hipMemcpyAsync(g.b + i * g.N, r->b, sizeof(double) * g.N, hipMemcpyDeviceToDevice,
                         g.stream));
  ++g.active;
  g.last_used = r->t_admit;
}

// Moves queued requests into free slots, in arrival order.  A request whose
// group cannot be created within the budget waits (idle groups are freed
// first); one that can never fit fails with DCG_ENOMEM.
void Server::Impl::admit() {
  std::vector<Request*> todo;
  {
    std::lock_guard<std::mutex> lk(mu);
    todo.assign(queue.begin(), queue.end());
  }
  std::vector<Request*> placed;
  std::vector<std::pair<Request*, Error>> failed;
  for (Request* r : todo) {
    const GroupKey key{r->mesh.n, r->mesh.pre, r->mesh.post, r->mesh.penalty};
    Group* g = nullptr;
    auto it = groups.find(key);
    if (it != groups.end()) {
      g = it->second.get();
    } else {
      bool have_ctx = false;
      for (const auto& kv : groups)
        if (kv.first.n == key.n && kv.first.penalty == key.penalty) have_ctx = true;
      const size_t need = workspace_bytes(key.n, fp32) + (have_ctx ? 0 : context_bytes(key.n, fp32));
      if (need > budget) {
        failed.emplace_back(r, Error(DCG_ENOMEM, "request needs " + std::to_string(need) +
                                                     " bytes of HBM, the budget is " +
                                                     std::to_string(budget)));
        continue;
      }
      if (!make_room(need)) continue;   // waits until a group drains
      try {
        g = create_group(key);
      } catch (const Error& e) {
        groups.erase(key);
        failed.emplace_back(r, e);
        continue;
      }
    }
    int free_slot = -1;
    for (int i = 0; i < kBatch; ++i)
      if (!g->slots[i].req) {
        free_slot = i;
        break;
      }
    if (free_slot < 0) continue;
    try {
      assign(*g, free_slot, r);
      placed.push_back(r);
    } catch (const Error& e) {
      g->slots[free_slot] = Slot();
      failed.emplace_back(r, e);
    }
  }
  if (placed.empty() && failed.empty()) return;
  std::lock_guard<std::mutex> lk(mu);
  for (Request* r : placed) queue.erase(std::find(queue.begin(), queue.end(), r));
  for (auto& f : failed) {
    queue.erase(std::find(queue.begin(), queue.end(), f.first));
    f.first->status = f.second.status;
    f.first->error = f.second.what();
    f.first->stats.status = f.second.status;
    --unfinished;
  }
}

void Server::Impl::enqueue_step(Group& g) {
  const MeshContext& m = *g.mesh;
  const int ne = m.ne;
  const bool flex = opt.outer == DCG_OUTER_FCG1;
  hipStream_t st = g.stream;
  int32_t* L = g.lists_host;
  std::fill(g.counts, g.counts + kNumLists, 0);
  auto add = [&](int list, int i) { L[list * kBatch + g.counts[list]++] = i; };
  for (int i = 0; i < kBatch; ++i) {
    Slot& s = g.slots[i];
    s.in_step = s.req != nullptr;
    if (!s.in_step) continue;
    if (s.zero_inner) {
      DCG_HIP(launch_fill<double>(g.M, 0.0, g.zref + i * g.M, st));
      s.zero_inner = false;
    }
    switch (s.stage) {
      case Stage::kPro:
        add(kLZt, i);
        add(kLInnerStart, i);
        break;
      case Stage::kInner:
        add(kLAddMore, i);
        add(kLInnerAll, i);
        break;
      case Stage::kPostPro:
        DCG_HIP(launch_copy<double>(g.M, g.zref + i * g.M, g.zb + i * g.M, st));
        DCG_HIP(launch_fill<double>(g.N, 0.0, g.xh + i * g.N, st));
        add(kLDeflPro, i);
        add(kLAstarFirst, i);
        add(kLInnerStart, i);
        break;
      case Stage::kPostIter:
        add(s.pidx ? kLDeflIter1 : kLDeflIter0, i);
        add(s.pidx ? kLAstarDir1 : kLAstarDir0, i);
        add(kLInnerStart, i);
        break;
      case Stage::kEpi:
        add(kLAstarPlain, i);
        add(kLInnerStart, i);
        break;
      case Stage::kPostEpi:
        add(kLPostEpi, i);
        break;
    }
  }
  for (int i = 0; i < g.counts[kLInnerStart]; ++i) {
    add(kLAddFirst, L[kLInnerStart * kBatch + i]);
    add(kLInnerAll, L[kLInnerStart * kBatch + i]);
  }
  DCG_HIP(hipMemcpyAsync(g.lists_dev, g.lists_host, sizeof(int32_t) * kNumLists * kBatch,
                         hipMemcpyHostToDevice, st));
  auto cnt = [&](int list) { return g.counts[list]; };
  auto sl = [&](int list) { return slot_addr(g, list); };
  const int nbA = astar_blocks(ne);

  // outer-iteration work
  if (cnt(kLDeflPro)) {
    DCG_HIP(launch_deflate(true, m.AdivZ, m.cols, ne, kTwo, g.zb, g.b, nullptr, g.r, g.p[0],
                           g.ws.part, st, sl(kLDeflPro), cnt(kLDeflPro)));
    DCG_HIP(launch_reduce(g.ws.part, nbA, kRedB2Rho, g.ws.sc, st, sl(kLDeflPro), cnt(kLDeflPro)));
  }
  for (int pi = 0; pi < 2; ++pi) {
    const int list = pi ? kLDeflIter1 : kLDeflIter0;
    if (!cnt(list)) continue;
    DCG_HIP(launch_deflate(false, m.AdivZ, m.cols, ne, kTwo, g.zref, g.w, g.p[pi], g.q, nullptr,
                           g.ws.part, st, sl(list), cnt(list)));
    DCG_HIP(launch_reduce(g.ws.part, nbA, flex ? kRedFcgAlpha : kRedAlpha, g.ws.sc, st, sl(list),
                          cnt(list)));
    int nbu = 0;
    DCG_HIP(launch_cg_update(flex, g.N, g.ws.sc, g.p[pi], g.q, g.xh, g.r, g.ws.part, &nbu, st,
                             sl(list), cnt(list)));
    DCG_HIP(launch_reduce(g.ws.part, nbu, flex ? kRedFcgBeta : kRedBeta, g.ws.sc, st, sl(list),
                          cnt(list)));
  }
  if (cnt(kLPostEpi)) {
    const int c = cnt(kLPostEpi);
    DCG_HIP(launch_reconstruct(ne, g.xh, g.zref, g.zb, g.ws.sc, g.q, st, sl(kLPostEpi), c));
    DCG_HIP(launch_astar(kAstarResidual, m.Cdiv, m.cols, m.M1, ne, g.q, nullptr, g.b, g.ws.sc,
                         nullptr, g.w, nullptr, g.ws.part, st, sl(kLPostEpi), c));
    DCG_HIP(launch_reduce(g.ws.part, nbA, kRedRes, g.ws.sc, st, sl(kLPostEpi), c));
    for (int k = 0; k < c; ++k) {
      const int i = L[kLPostEpi * kBatch + k];
      DCG_HIP(hipMemcpyAsync(g.slots[i].req->x, g.q + i * g.N, sizeof(double) * g.N,
                             hipMemcpyDeviceToDevice, st));
    }
  }
  // the next inner right-hand side s = Z^T (...)
  if (cnt(kLZt)) DCG_HIP(launch_zt(ne, g.b, g.s, st, sl(kLZt), cnt(kLZt)));
  if (cnt(kLAstarFirst))
    DCG_HIP(launch_astar(kAstarFirst, m.Cdiv, m.cols, m.M1, ne, g.r, g.p[0], nullptr, g.ws.sc,
                         g.p[1], g.w, g.s, nullptr, st, sl(kLAstarFirst), cnt(kLAstarFirst)));
  for (int pi = 0; pi < 2; ++pi) {
    const int list = pi ? kLAstarDir1 : kLAstarDir0;
    if (!cnt(list)) continue;
    DCG_HIP(launch_astar(kAstarDir, m.Cdiv, m.cols, m.M1, ne, g.r, g.p[pi], nullptr, g.ws.sc,
                         g.p[1 - pi], g.w, g.s, nullptr, st, sl(list), cnt(list)));
  }
  if (cnt(kLAstarPlain))
    DCG_HIP(launch_astar(kAstarPlain, m.Cdiv, m.cols, m.M1, ne, g.xh, nullptr, nullptr, g.ws.sc,
                         nullptr, g.w, g.s, nullptr, st, sl(kLAstarPlain), cnt(kLAstarPlain)));

  // inner Multigrid iteration: starts, one batched W-cycle, refinement
  const DeviceLevel& fine = m.lv[m.J - 1];
  const int nbR = refine_blocks(fine.ne);
  auto inner = [&](auto tag) {
    using T = decltype(tag);
    T* fJ = static_cast<T*>(g.ws.lvb.f[m.J - 1]);
    if (cnt(kLInnerStart)) {
      DCG_HIP(launch_refine_residual<T>(true, fine.Lc64, fine.n, fine.ne, g.s, nullptr, fJ,
                                        g.ws.part, st, sl(kLInnerStart), cnt(kLInnerStart)));
      DCG_HIP(launch_reduce(g.ws.part, nbR, kRedS2, g.ws.sc, st, sl(kLInnerStart),
                            cnt(kLInnerStart)));
    }
    g.any_cycle = cnt(kLInnerAll) > 0;
    if (!g.any_cycle) return;
    const Cycle<T> cyc(m, g.ws.lvb, g.key.pre, g.key.post);
    LvState fs;
    if (opt.use_graph) {
      if (!g.graph) {
        hipGraph_t gr = nullptr;
        LvState c;
        DCG_HIP(hipStreamBeginCapture(g.capture, hipStreamCaptureModeThreadLocal));
        try {
          cyc.wcycle(m.J, c, g.capture);
        } catch (...) {
          (void)hipStreamEndCapture(g.capture, &gr);
          if (gr) (void)hipGraphDestroy(gr);
          throw;
        }
        DCG_HIP(hipStreamEndCapture(g.capture, &gr));
        const hipError_t e = hipGraphInstantiate(&g.graph, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        DCG_HIP(e);
        g.graph_state = c;
      }
      DCG_HIP(hipGraphLaunch(g.graph, st));
      fs = g.graph_state;
    } else {
      cyc.wcycle(m.J, fs, st);
    }
    T* zJ = static_cast<T*>(g.ws.lvb.z[fs.zb][m.J - 1]);
    T* YJ = static_cast<T*>(g.ws.lvb.Y[fs.yb][m.J - 1]);
    if (cnt(kLAddFirst))
      DCG_HIP(launch_refine_add<T>(fine.ne, true, fs.has_z, fs.has_y, zJ, YJ, g.zref, st,
                                   sl(kLAddFirst), cnt(kLAddFirst)));
    if (cnt(kLAddMore))
      DCG_HIP(launch_refine_add<T>(fine.ne, false, fs.has_z, fs.has_y, zJ, YJ, g.zref, st,
                                   sl(kLAddMore), cnt(kLAddMore)));
    DCG_HIP(launch_refine_residual<T>(false, fine.Lc64, fine.n, fine.ne, g.s, g.zref, fJ,
                                      g.ws.part, st, sl(kLInnerAll), cnt(kLInnerAll)));
    DCG_HIP(launch_reduce(g.ws.part, nbR, kRedR2, g.ws.sc, st, sl(kLInnerAll), cnt(kLInnerAll)));
  };
  if (fp32)
    inner(float());
  else
    inner(double());

  DCG_HIP(hipMemcpyAsync(g.ws.sc_host, g.ws.sc, sizeof(Scalars) * kBatch, hipMemcpyDeviceToHost,
                         st));
  DCG_HIP(hipEventRecord(g.done, st));
  g.inflight = true;
  int occupied = 0;
  for (int i = 0; i < kBatch; ++i) occupied += g.slots[i].in_step;
  steps += 1;
  slot_steps += occupied;
}

void Server::Impl::inner_done(Slot& s) {
  s.stage = s.kind == Kind::kPro ? Stage::kPostPro
                                 : (s.kind == Kind::kIter ? Stage::kPostIter : Stage::kPostEpi);
}

// Host tests of the inner iteration after a step that started it (and ran
// its first W-cycle): the loop of the single-request inner solve, entered
// with r2 = s2.
void Server::Impl::after_inner_start(Group& g, Slot& s, const Scalars& sc) {
  ++s.inner_solves;
  const double s2 = sc.s2;
  if (!std::isfinite(s2)) {
    finish(g, s, DCG_EINVAL, "non-finite inner right-hand side");
    return;
  }
  // eq. (fixed_tol), or eq. (tol) with the outer residual of this iteration
  const double tol = s.req->tol;
  const double tol_c = opt.c_A <= 0.0 ? opt.c_F * tol
                       : (s.kind == Kind::kIter ? opt.c_A * tol * std::sqrt(s.b2) / std::sqrt(s.rho)
                                                : opt.c_A * tol);
  s.inner_lim = tol_c * tol_c * s2;
  s.cycles = 0;
  if (s2 > 0.0 && opt.max_inner > 0 && s2 > s.inner_lim) {
    s.cycles = 1;
    ++s.cycles_total;
    if (s.kind == Kind::kIter) ++s.cycles_outer;
    const double r2 = sc.r2;
    if (!std::isfinite(r2)) {
      finish(g, s, DCG_EBREAKDOWN, "non-finite inner residual");
      return;
    }
    if (s.cycles < opt.max_inner && r2 > s.inner_lim) {
      s.stage = Stage::kInner;
      return;
    }
  } else {
    s.zero_inner = true;   // no cycle counts: the inner result is 0
  }
  inner_done(s);
}

void Server::Impl::process(Group& g) {
  g.inflight = false;
  const Scalars* sc = g.ws.sc_host;
  for (int i = 0; i < kBatch; ++i) {
    Slot& s = g.slots[i];
    if (!s.req || !s.in_step) continue;
    s.in_step = false;
    const Scalars& c = sc[i];
    switch (s.stage) {
      case Stage::kPro:
        s.kind = Kind::kPro;
        after_inner_start(g, s, c);
        break;
      case Stage::kInner: {
        ++s.cycles;
        ++s.cycles_total;
        if (s.kind == Kind::kIter) ++s.cycles_outer;
        if (!std::isfinite(c.r2)) {
          finish(g, s, DCG_EBREAKDOWN, "non-finite inner residual");
          break;
        }
        if (!(s.cycles < opt.max_inner && c.r2 > s.inner_lim)) inner_done(s);
        break;
      }
      case Stage::kPostPro: {
        s.b2 = c.b2;
        s.rho = c.rho;
        if (!std::isfinite(s.b2) || !std::isfinite(s.rho)) {
          finish(g, s, DCG_EINVAL, "b contains NaN or Inf");
          break;
        }
        if (s.b2 == 0.0) {
          DCG_HIP(launch_fill<double>(g.N, 0.0, s.req->x, g.stream));
          DCG_HIP(hipStreamSynchronize(g.stream));
          s.req->stats.rel_res_recurrence = 0.0;
          s.req->stats.rel_res_true = 0.0;
          finish(g, s, DCG_OK);
          break;
        }
        s.lim = s.req->tol * s.req->tol * s.b2;
        if (s.rho <= s.lim) {
          s.stage = Stage::kEpi;
        } else if (s.it >= opt.max_outer) {
          s.final_status = DCG_NOT_CONVERGED;
          s.stage = Stage::kEpi;
        } else {
          s.pidx = 1;
          s.kind = Kind::kIter;
          after_inner_start(g, s, c);
        }
        break;
      }
      case Stage::kPostIter: {
        ++s.it;
        if (c.breakdown || !std::isfinite(c.rho)) {
          s.final_status = DCG_EBREAKDOWN;
          s.stage = Stage::kEpi;
          break;
        }
        s.rho = c.rho;
        if (s.rho <= s.lim) {
          s.stage = Stage::kEpi;
        } else if (s.it >= opt.max_outer) {
          s.final_status = DCG_NOT_CONVERGED;
          s.stage = Stage::kEpi;
        } else {
          s.pidx = 1 - s.pidx;
          s.kind = Kind::kIter;
          after_inner_start(g, s, c);
        }
        break;
      }
      case Stage::kEpi:
        s.kind = Kind::kEpi;
        after_inner_start(g, s, c);
        break;
      case Stage::kPostEpi: {
        dcg_stats& st = s.req->stats;
        st.rel_res_recurrence = std::sqrt(std::max(s.rho, 0.0) / s.b2);
        st.rel_res_true = std::sqrt(c.res2 / s.b2);
        finish(g, s, s.final_status,
               s.final_status == DCG_EBREAKDOWN
                   ? "outer iteration broke down ((p, q) <= 0 or non-finite)"
                   : std::string());
        break;
      }
    }
  }
}

void Server::Impl::finish(Group& g, Slot& s, dcg_status status, const std::string& err) {
  Request* r = s.req;
  const auto now = Clock::now();
  dcg_stats& st = r->stats;
  st.status = status;
  st.outer_iters = s.it;
  st.total_wcycles = s.cycles_total;
  st.inner_solves = s.inner_solves;
  st.inner_per_outer = s.it > 0 ? double(s.cycles_outer) / s.it : 0.0;
  st.t_setup_ms = 0.0;
  st.t_solve_ms = ms_between(r->t_admit, now);
  st.t_queue_ms = ms_between(r->t_submit, r->t_admit);
  s = Slot();
  --g.active;
  g.last_used = now;
  std::lock_guard<std::mutex> lk(mu);
  r->status = status;
  r->error = err;
  --unfinished;
}

void Server::Impl::fail_group(Group& g, const Error& e) {
  if (g.inflight) (void)hipStreamSynchronize(g.stream);
  g.inflight = false;
  for (Slot& s : g.slots)
    if (s.req) finish(g, s, e.status, e.what());
}

// Scheduler loop: admit, start a step on every idle group, then process
// every group whose step has completed (several groups' steps overlap on
// their streams, so the first to finish is handled first).
void Server::Impl::run() {
  (void)hipSetDevice(device);
  while (true) {
    {
      std::unique_lock<std::mutex> lk(mu);
      if (stop) break;
    }
    try {
      step_all();
    } catch (const std::exception& ex) {
      // anything but a library error (host allocation, ...): every running
      // request ends with it; the server keeps serving
      const Error e(dynamic_cast<const std::bad_alloc*>(&ex) ? DCG_ENOMEM : DCG_EDEVICE, ex.what());
      for (auto& kv : groups) fail_group(*kv.second, e);
    }
  }
  for (auto& kv : groups)
    if (kv.second->inflight) (void)hipStreamSynchronize(kv.second->stream);
  groups.clear();
}

// One pass of the scheduler loop.
void Server::Impl::step_all() {
  admit();
  for (auto& kv : groups) {
    Group& g = *kv.second;
    if (g.inflight || g.active == 0) continue;
    try {
      enqueue_step(g);
    } catch (const Error& e) {
      fail_group(g, e);
    }
  }
  bool any_inflight = false, progressed = false;
  for (auto& kv : groups) {
    Group& g = *kv.second;
    if (!g.inflight) continue;
    any_inflight = true;
    const hipError_t q = hipEventQuery(g.done);
    if (q == hipErrorNotReady) continue;
    progressed = true;
    try {
      DCG_HIP(q);
      process(g);
    } catch (const Error& e) {
      fail_group(g, e);
    }
  }
  if (!any_inflight) {
    std::unique_lock<std::mutex> lk(mu);
    cv.wait_for(lk, std::chrono::milliseconds(20), [&] { return stop || !queue.empty(); });
  } else if (!progressed) {
    std::this_thread::sleep_for(std::chrono::microseconds(5));
  }
}

Server::Server(const dcg_options& opt) : impl(new Impl()) {
  impl->opt = opt;
  impl->fp32 = opt.prec == DCG_MIXED;
  DCG_HIP(hipGetDevice(&impl->device));
  size_t free_b = 0, total_b = 0;
  DCG_HIP(hipMemGetInfo(&free_b, &total_b));
  impl->budget = opt.hbm_budget_bytes > 0 ? size_t(opt.hbm_budget_bytes) : total_b;
  impl->thread = std::thread([this]() { impl->run(); });
}

Server::~Server() {
  {
    std::lock_guard<std::mutex> lk(impl->mu);
    impl->stop = true;
  }
  impl->cv.notify_all();
  if (impl->thread.joinable()) impl->thread.join();
}

void Server::prepare(const dcg_mesh& mesh) {
  int cur = 0;
  DCG_HIP(hipGetDevice(&cur));
  DCG_HIP(hipSetDevice(impl->device));
  try {
    (void)get_context(mesh.n, mesh.penalty, impl->fp32);
  } catch (...) {
    (void)hipSetDevice(cur);
    throw;
  }
  DCG_HIP(hipSetDevice(cur));
}

dcg_status Server::submit(const dcg_mesh& mesh, double dt, double nu, const double* b, double* x,
                          double tol, uint64_t* ticket) {
  auto r = std::make_unique<Request>();
  r->mesh = mesh;
  r->dt = dt;
  r->nu = nu;
  r->tol = tol;
  r->b = b;
  r->x = x;
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(impl->mu);
    if (impl->unfinished >= impl->opt.max_pending)
      throw Error(DCG_EAGAIN, "server queue full (" + std::to_string(impl->unfinished) +
                                  " unfinished requests)");
    r->ticket = impl->next_ticket++;
    *ticket = r->ticket;
    impl->queue.push_back(r.get());
    ++impl->unfinished;
    impl->requests[r->ticket] = std::move(r);
  }
  impl->cv.notify_all();
  return DCG_OK;
}

dcg_status Server::poll(uint64_t ticket, dcg_stats* st, std::string* err) {
  std::lock_guard<std::mutex> lk(impl->mu);
  auto it = impl->requests.find(ticket);
  if (it == impl->requests.end()) throw Error(DCG_ENOTFOUND, "unknown ticket " + std::to_string(ticket));
  Request& r = *it->second;
  if (r.status == DCG_PENDING) return DCG_PENDING;
  if (st) *st = r.stats;
  const dcg_status s = r.status;
  if (err) *err = r.error;
  impl->requests.erase(it);
  return s;
}

int64_t Server::group_bytes(int n, bool fp32) {
  return int64_t(workspace_bytes(n, fp32) + context_bytes(n, fp32));
}

void Server::counters(int64_t* steps, int64_t* slot_steps) const {
  if (steps) *steps = impl->steps.load();
  if (slot_steps) *slot_steps = impl->slot_steps.load();
}

}  // namespace dcg
