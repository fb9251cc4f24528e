// Device-side mesh contexts, solver workspaces and handles.
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/dcg.h"
#include "host_setup.hpp"
#include "kernels.hpp"

namespace dcg {

// Error carrying a dcg_status; thrown inside the library, converted to a
// status at the C ABI.
struct Error : std::runtime_error {
  dcg_status status;
  Error(dcg_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

void hip_check(hipError_t e, const char* what);
#define DCG_HIP(expr) ::dcg::hip_check((expr), #expr)

// One multigrid level on the device.
struct DeviceLevel {
  int n = 0, ne = 0;
  int32_t* cols = nullptr;        // [5][ne]
  double* L64 = nullptr;          // [5][ne][4][4]
  float* L32 = nullptr;
  double* Lc64 = nullptr;         // class tables [9][5][4][4] of L64 / L32
  float* Lc32 = nullptr;
  int tiles = 0;                  // levels >= 2
  int32_t* tile_ext = nullptr;    // [tiles][52]
  int32_t* tile_dst = nullptr;    // [tiles][32]
  // packed symmetric inverses of the distinct local problems (bit-identical
  // local matrices and weights share one), [classes][36][16][16], and the
  // class of every tile
  float* F32 = nullptr;
  double* F64 = nullptr;
  // the same inverses in MFMA operand order, [classes][8][8][64][4]
  float* Fm32 = nullptr;
  double* Fm64 = nullptr;
  int32_t* fcls = nullptr;        // [tiles]
  int classes = 0;
  float* dw32 = nullptr;          // [ne] 1 / #blocks containing the square
  double* dw64 = nullptr;
  // grouped RAS step with g x g tiles per workgroup (g = 1, 2, 4 at index
  // 0, 1, 2): every class after the first of a group gets a workgroup of its
  // own, listed as (group, class) pairs [gx_extra_n[i]][2]
  int32_t* gx_extra[3] = {nullptr, nullptr, nullptr};
  int gx_extra_n[3] = {0, 0, 0};
};

// Dt-independent operators of one mesh on one device; shared by handles and
// by the serving engine (reference counted through shared_ptr).
struct MeshContext {
  int device = 0;
  int n = 0, J = 0, ne = 0;
  double penalty = 10.0;
  double2* Cdiv = nullptr;        // [5][4][ne][8]: A_div = diag(C, C) per block
  double2* AdivZ = nullptr;       // [5][2][ne][16]
  double* M1 = nullptr;           // [ne][16]
  int32_t* cols = nullptr;        // [5][ne]
  std::vector<DeviceLevel> lv;    // lv[k - 1]
  double* coarse_inv = nullptr;   // [1024][1024]
  size_t bytes = 0;
  double t_build_ms = 0.0;
  std::mutex mu;                  // guards lazy factor uploads
  std::unique_ptr<HostContext> host;   // kept until both factor precisions exist
  bool have_f32 = false, have_f64 = false;

  ~MeshContext();
  void ensure_factors(bool fp32);   // uploads L_k and tile inverses of that precision
  void* alloc(size_t bytes);
  std::vector<void*> allocations;
};

// Exact coarsest-level solve of a shortened hierarchy (coarsest level larger
// than the stored 16 x 16 one) by fast diagonalisation: the axis factors of
// that level's Galerkin operator (V, its transpose VT, both 2n x 2n
// row-major, eigenvalues lam) and three FP64 scratch vectors of 4 n^2.
struct CoarseFdm {
  int n = 0;                      // squares per side of the coarsest level
  const double* V = nullptr;
  const double* VT = nullptr;
  const double* lam = nullptr;
  double* t[3] = {nullptr, nullptr, nullptr};
};

// Returns the cached context of (current device, n, penalty), building and
// uploading it on first use.
std::shared_ptr<MeshContext> get_context(int n, double penalty, bool fp32);
void clear_context_cache();
// Drops the cached context of (current device, n, penalty) when nothing but
// the cache holds it.
void release_context_if_unused(int n, double penalty);

struct Workspace;

// Multigrid level buffers of one cycle instance (level real type, index
// k - 1; z and Y double-buffered).  batched: kBatch request-interleaved
// columns per vector.
struct LevelBuffers {
  bool batched = false;
  std::vector<void*> f, rr, z[2], Y[2];
  // Allocates every level of ``m`` through ws.alloc; the pending-output
  // buffers are zeroed once (cover slots no block uses are never written).
  void allocate(const MeshContext& m, bool fp32, bool batch, Workspace& ws);
};

// Stored directions of the flexible outer iteration (R slots of (d, q) with
// device pointer arrays and (d, q) values) or the Arnoldi basis of GMRES (d
// only); vectors are allocated on first use.
struct FcgStore {
  int R = 0;
  std::vector<double*> d, q;
  double** dptr = nullptr;
  double** qptr = nullptr;
  double* dq = nullptr;
  double* coef = nullptr;
  double* coef2 = nullptr;
  double* part = nullptr;
  std::vector<void*> vecs;
  void* alloc(size_t bytes);
  void release();
  ~FcgStore() { release(); }
};

// Device workspace of one solver handle (one request) or one serving batch.
struct Workspace {
  int ne = 0;
  size_t bytes = 0;
  std::vector<void*> allocations;
  double *xh = nullptr, *r = nullptr, *p[2] = {nullptr, nullptr}, *w = nullptr, *q = nullptr;
  double *s = nullptr, *zref = nullptr, *zb = nullptr, *zt = nullptr;
  double* part = nullptr;                 // [3][kPartStride]
  Scalars* sc = nullptr;                  // device
  Scalars* sc_host = nullptr;             // pinned host mirror
  LevelBuffers lvb;                       // W-cycle level buffers
  LevelBuffers lvb_batch;                 // batched level operators (allocated on first use)
  FcgStore fcg;                           // DCG_OUTER_FCG directions
  void* alloc(size_t bytes);
  void release();
  ~Workspace();
};

}  // namespace dcg

// Solver handle (the opaque dcg_handle of the C ABI).
namespace dcg {
// The outer multigrid preconditioner of a handle (omg.hpp, omg_driver.cpp):
// the A* hierarchy (level k at index k - 1; device arrays in the handle's
// workspace) and the graph of B(r) with the pointers it was captured for.
struct OuterMg {
  int J = 0, m = 2;
  std::vector<int> n;
  std::vector<double*> op, ras, f, z, r;
  std::vector<double*> opm, rasm;   // the tables in MFMA operand order
  double* cinv = nullptr;
  double* zp = nullptr;            // B r of the current outer iteration (16 n^2)
  hipGraphExec_t graph = nullptr;
  const double* g_in = nullptr;
  double* g_out = nullptr;
  ~OuterMg();
};
}  // namespace dcg

struct dcg_ctx {
  std::shared_ptr<dcg::MeshContext> mesh;
  dcg_mesh mp{};
  dcg_options opt{};
  double dt = 0.0, nu = 1.0;
  bool fp32 = true;
  dcg::Workspace ws;
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t wgraph = nullptr;        // coarse-grid correction of the finest level
  int graph_state[4] = {0, 0, 0, 0};      // level J-1 state the graph leaves behind
  std::string last_error;
  double t_setup_ms = 0.0;
  int device = 0;
  // live timing of the finest-level RAS tile kernel
  static constexpr int kMaxTimed = 256;   // event pairs between two reads of the stream
  bool ktime = false;
  hipEvent_t kev[2 * kMaxTimed] = {};
  int krec = 0;                 // event pairs recorded since they were last read
  int kstride = 1;              // time the finest steps of every kstride-th W-cycle
  int64_t kcycle = 0;           // W-cycles since timing was enabled
  double ktime_ms = 0.0;
  int64_t klaunches = 0;
  // and of the A* product with the direction update in the CG outer loop
  hipEvent_t aev[2] = {};
  double atime_ms = 0.0;
  int64_t alaunches = 0;
  // W-cycle counts of the last inner solves: the inner iteration enqueues as
  // many cycles as the fewest of them before reading its device-side test
  static constexpr int kInnerRecent = 4;
  int inner_recent[kInnerRecent] = {1, 1, 1, 1};
  int inner_next = 0;
  // exact inner solve (DCG_INNER_EXACT): fast-diagonalisation factors and
  // three scratch vectors, all in the workspace
  bool exact = false;
  double *fV = nullptr, *fVT = nullptr, *flam = nullptr, *ft[3] = {nullptr, nullptr, nullptr};
  // multigrid levels in use (opt.levels): the hierarchy of the inner solve
  // is stored levels lbase + 1 .. J, and with lbase > 0 its coarsest level is
  // solved by fast diagonalisation (cfdm, factors in the workspace)
  int lbase = 0;
  dcg::CoarseFdm cfdm;
  // level-buffer view of dcg_apply_noalloc (pointers into the static scratch
  // array; the tables are sized at setup so that the call allocates nothing)
  dcg::LevelBuffers noalloc_lvb;
  // outer multigrid preconditioner (opt.outer_mg > 0)
  std::unique_ptr<dcg::OuterMg> omg;
  ~dcg_ctx();
};

namespace dcg {
void handle_init(dcg_ctx* h);             // allocates the workspace
dcg_status solve(dcg_ctx* h, const double* b, double* x, double tol, dcg_stats* st,
                 hipStream_t stream);
void kernel_timing(dcg_ctx* h, int stride);   // 0 = off
dcg_status apply(dcg_ctx* h, dcg_op op, int level, const void* in, const void* in2, void* out,
                 hipStream_t stream);
// DCG_OP_INNER / DCG_OP_DEFLATED with every work buffer in the static scratch
// array (no device allocation); noalloc_capacity() is its size in bytes.
dcg_status apply_noalloc(dcg_ctx* h, dcg_op op, const double* in, double* out, hipStream_t stream);
size_t noalloc_capacity();
// The outer multigrid preconditioner: set-up (after handle_init), z = B r on
// the stream, and its level operators (DCG_OP_OMG_*).
void omg_setup(dcg_ctx* h);
void omg_apply(dcg_ctx* h, const double* r, double* z, hipStream_t st);
void omg_apply_level(dcg_ctx* h, dcg_op op, int k, const double* in, const double* in2, double* out,
                     hipStream_t st);
}  // namespace dcg
