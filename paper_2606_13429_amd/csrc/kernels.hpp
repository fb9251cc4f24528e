// Launchers of the gfx950 kernels of the deflated-CG hot path.  Every
// launcher enqueues on ``st`` and returns hipGetLastError() of the launch.
//
// Device layouts (Ne = squares of the level, all indices int32 except where
// a product can exceed 2^31):
//   tensor vectors   [16 e + 4 c + j]                 (FP64)
//   scalar vectors   [4 e + j]                        (FP64 or level real T)
//   A_div = diag(C, C) per block (one C for each stress row), stored as
//   C                double2 [slot][kc=4][Ne][row=8]   row r, columns 2kc, 2kc+1
//   A_div Z          double2 [slot][kc=2][Ne][row=16]
//   M_1              double  [Ne][16]
//   L_k              T       [slot][Ne][row=4][4]
//   cols             int32   [slot][Ne]               -1 = none
//   RAS factors      T       [class][36 blocks P <= Q][16][16]  packed upper blocks of the
//                                                     symmetric (L_k)_t^{-1}, row-major, one per
//                                                     distinct local problem (interior tiles of
//                                                     the uniform grid share one)
//   factor classes   int32   [tile]                   class of the tile's inverse
//   RAS weights      T       [Ne]                     1 / #blocks containing the square
//   pending slots    int32   [tile][32]               3 e + k for block square e
//   coarsest inverse double  [1024][1024]
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dcg {

// Device-resident scalars of one solve (read by the update kernels).
struct Scalars {
  double b2;        // ||b||^2
  double rho;       // (r, r)
  double pq;        // (p, q)
  double alpha, beta;
  double dr;        // (d, r) of the flexible variant
  double res2;      // ||b - A* x||^2 or the last plain dot
  double s2, r2;    // inner iteration: ||s||^2 and ||s - L z||^2
  double dt, inv_nu;  // operator parameters of this request (A* = (1/nu) M + dt A_div)
  double inner_lim2;  // inner iteration tested on the device: tol_c^2 ||s||^2
  double spare[4];
  int32_t breakdown;
  int32_t inner_done;    // the inner iteration has met its test or its cycle cap
  int32_t inner_cycles;  // W-cycles the inner iteration has counted
  int32_t pad;
};

enum ReduceOp : int {
  kRedB2Rho = 0,     // slots (b,b), (r,r)          -> b2, rho
  kRedAlpha = 1,     // slot (p,q)                  -> pq, alpha = rho / pq
  kRedBeta = 2,      // slot (r,r)                  -> beta = rho'/rho, rho = rho'
  kRedS2 = 3,        // slot ||r||^2 of the inner   -> s2 = r2 = sum
  kRedR2 = 4,        // slot ||r||^2 of the inner   -> r2
  kRedRes = 5,       // slot (v,v)                  -> res2
  kRedFcgAlpha = 6,  // slot (d,q)                  -> pq, alpha = dr / pq
  kRedFcgBeta = 7,   // slots (r,r),(r,q),(d,r)     -> rho, beta = -(r,q)/pq, dr
  kRedRho = 8,       // slot (r,r)                  -> rho (and dr = rho)
  kRedDr = 9,        // slot (d,r)                  -> dr
  // the inner iteration's test on the device (aux = tol_c^2, iaux = max cycles):
  kRedInnerS2 = 10,  // slot ||s||^2                -> s2 = r2, inner_lim2 = aux s2, cycles 0, done
  kRedInnerR2 = 11   // slot ||s - L z||^2          -> unless done: r2, ++cycles, done
};

constexpr int kPartStride = 1 << 16;   // max blocks of a reducing launch
constexpr int64_t kSlotPart = 3 * int64_t(kPartStride);   // partial sums per request

// Request addressing of the batched launches: blockIdx.y selects request
// list[y], whose vectors sit at base + request * stride and whose scalars and
// partial sums at sc + request, part + request * kSlotPart.  list == nullptr
// addresses one request (request 0) -- the single-solve path.  Finest-level
// vectors of the level type hold square e of the request at e * lsq +
// request * lstride: lsq = 4, lstride = 0 for one request, lsq = 4 kBatch,
// lstride = 4 for the request-interleaved layout of the batched cycle.
struct Slots {
  const int32_t* list = nullptr;
  int64_t tstride = 0;   // tensor vectors, 16 ne FP64
  int64_t sstride = 0;   // scalar FP64 vectors, 4 ne
  int64_t lstride = 0;   // finest-level vectors of the level type
  int64_t lsq = 4;
};

// Requests of one batched multigrid cycle: the N dimension of the MFMA tiles
// of the batched RAS step.  Batched level vectors are request-interleaved,
// [square][request][4] (pending outputs [3 square + k][request][4]).
constexpr int kBatch = 16;

enum AstarMode : int {
  kAstarPlain = 0,   // w = A* x
  kAstarDir = 1,     // u = x + beta p_old, p_new = u, w = A* u
  kAstarFirst = 2,   // u = x, p_new = u, w = A* u
  kAstarResidual = 3 // w = b - A* x, partial (w, w)
};

// Square class of a level operator on the uniform grid: the five blocks of
// L_k at square (ex, ey) depend only on whether the square touches the left
// or right (bottom or top) side of the domain, so 3 x 3 classes, 3 cy + cx
// with cx = 0 at ex = 0, 2 at ex = n - 1, 1 otherwise.  A class table
// Lc [class 9][slot 5][row 4][4] holds one copy per class; the host checks
// that every square of a class carries bit-identical blocks.
__host__ __device__ inline int square_class(int ex, int ey, int n) {
  const int cx = ex == 0 ? 0 : (ex == n - 1 ? 2 : 1);
  const int cy = ey == 0 ? 0 : (ey == n - 1 ? 2 : 1);
  return 3 * cy + cx;
}

// workgroups (= partial sums) of the reducing launches for ``ne`` squares
int astar_blocks(int ne);     // launch_astar and launch_deflate
int refine_blocks(int ne);    // launch_refine_residual

// (ev0, ev1: when non-null, recorded at the start and end of the dispatch)
hipError_t launch_astar(int mode, const double2* C, const int32_t* cols, const double* M1, int ne,
                        const double* x, const double* p_old, const double* b, const Scalars* sc,
                        double* p_new, double* w, double* s, double* part, hipStream_t st,
                        const Slots& sl = Slots(), int count = 1, hipEvent_t ev0 = nullptr,
                        hipEvent_t ev1 = nullptr);
// q = w - c * (A_div Z) z ; partial (p, q).  With ``prologue``: r = w - c AZ z
// written to q and to p_out, partials (w, w) and (q, q).
hipError_t launch_deflate(bool prologue, const double2* AZ, const int32_t* cols, int ne, double c,
                          const double* z, const double* w, const double* p, double* q,
                          double* p_out, double* part, hipStream_t st, const Slots& sl = Slots(),
                          int count = 1);
// q = AZ y (plain product, no partials)
hipError_t launch_adivz(const double2* AZ, const int32_t* cols, int ne, const double* y, double* out,
                        hipStream_t st);
// x += alpha p ; r -= alpha q ; partial (r, r)  [flexible: + (r,q), (p,r)]
hipError_t launch_cg_update(bool flexible, int64_t nvec, const Scalars* sc, const double* p,
                            const double* q, double* x, double* r, double* part, int* nblocks,
                            hipStream_t st, const Slots& sl = Slots(), int count = 1);
// r += a q ; partial (r, r)
hipError_t launch_axpy_dot(int64_t nvec, double a, const double* q, double* r, double* part,
                           int* nblocks, hipStream_t st);
hipError_t launch_reduce(const double* part, int nblocks, int op, Scalars* sc, hipStream_t st,
                         const Slots& sl = Slots(), int count = 1, double aux = 0.0, int iaux = 0);

hipError_t launch_zt(int ne, const double* w, double* s, hipStream_t st, const Slots& sl = Slots(),
                     int count = 1);
hipError_t launch_z(int ne, const double* y, double scale, double* v, hipStream_t st);
// x = (xh - Z (c zt)) + Z (c zb), c = 2 / dt of the request
hipError_t launch_reconstruct(int ne, const double* xh, const double* zt, const double* zb,
                              const Scalars* sc, double* x, hipStream_t st,
                              const Slots& sl = Slots(), int count = 1);
hipError_t launch_scale(int64_t n, double c, const double* in, double* out, hipStream_t st);
// f = (1/nu) M (4/3 s1 - 1/3 s2) + c F ; x0 = 2 s1 - s2
hipError_t launch_bdf2_rhs(int ne, const double* M1, double inv_nu, const double* s1,
                           const double* s2, const double* F, double c, double* f, double* x0,
                           hipStream_t st);

// Flexible CG with stored directions (Algorithm 1): the window of the m
// directions d_k, q_k = M_D d_k of slots (first + k) % R, k < m, is addressed
// through device pointer arrays dptr / qptr and the device array dq of
// (d_k, q_k).
//   launch_fcg_coef:      coef[k] = -(r, q_k) / dq_k, or -(r, q_k) when dq is
//                         nullptr (the Gram-Schmidt coefficients of GMRES) (partials in part, then a
//                         fixed-order reduction per k; ``part`` holds m x
//                         fcg_coef_blocks(n) doubles)
//   launch_fcg_direction: d = r + sum_k coef[k] d_k (k ascending), partial (d, rdot)
//                         with rdot = r when NULL (the preconditioned FCG builds d
//                         from z = B r and takes (d, r))
int fcg_coef_blocks(int64_t n);
hipError_t launch_fcg_coef(int64_t n, const double* r, const double* const* qptr, const double* dq,
                           int first, int m, int R, double* part, double* coef, hipStream_t st);
hipError_t launch_fcg_direction(int64_t n, const double* r, const double* rdot, const double* const* dptr, int first,
                                int m, int R, const double* coef, double* d, double* part,
                                int* nblocks, hipStream_t st);

// inner refinement (FP64 residual of the level-J Laplacian): Lc64 is the
// class table of L_J on the n x n grid (ne = n^2 squares)
// (guard: when non-null, the launch does nothing once guard->inner_done is set)
template <typename T>
hipError_t launch_refine_residual(bool first, const double* Lc64, int n, int ne, const double* s,
                                  const double* z, T* fJ, double* part, hipStream_t st,
                                  const Slots& sl = Slots(), int count = 1,
                                  const Scalars* guard = nullptr);

// multigrid level kernels
template <typename T>
hipError_t launch_lap(bool residual, const T* L, const int32_t* cols, int ne, const T* f, const T* z,
                      T* out, hipStream_t st);
template <typename T>
hipError_t launch_restrict(int nc, const T* r, T* rc, hipStream_t st);
template <typename T>
hipError_t launch_prolong(int nc, const T* ec, T* z, hipStream_t st);
template <typename T>
hipError_t launch_coarse(const double* inv, const T* f, T* z, hipStream_t st);
template <typename T>
hipError_t launch_fill(int64_t n, T v, T* x, hipStream_t st);
template <typename T>
hipError_t launch_copy(int64_t n, const T* x, T* y, hipStream_t st);

// ------------------------------------------------------------ fused W-cycle
// Arguments of one RAS step of level k (mg_kernels.hip).  z and Y of a level
// are double buffers; a step reads z_old (+ the pending tile outputs Y_old,
// + the prolongated coarse correction) and writes z_new (core squares of
// every tile) and its own tile outputs Y_new.
template <typename T>
struct SweepArgs {
  const T* F = nullptr;             // [classes][36][16][16] packed symmetric inverses
  const T* Fm = nullptr;            // the same, full, in MFMA operand order [classes][8][8][64][4]
  const int32_t* gextra = nullptr;  // grouped step: (group, class) of the extra workgroups
  int nextra = 0;
  const int32_t* fcls = nullptr;    // [tiles] class of the tile's inverse in F
  const T* dw = nullptr;            // [ne] partition-of-unity weight 1 / #blocks
  const int32_t* ext = nullptr;     // [tiles][52] block squares + outside neighbours
  int tiles = 0, n = 0, ne = 0;
  const T* L = nullptr;             // level operator [5][ne][4][4] (batched kernels)
  const T* Lc = nullptr;            // its class table [9][5][4][4]
  const int32_t* cols = nullptr;    // [5][ne]
  const int32_t* dst = nullptr;     // [tiles][32] pending slot 3 e + k of each block square
  const T* f = nullptr;
  const T* z_old = nullptr;
  const T* Y_old = nullptr;         // pending tile outputs [ne][3][4]
  T* z_new = nullptr;
  T* Y_new = nullptr;
  int has_z = 0, has_y = 0, write_z = 0;
  int prol = 0, nc = 0, c_has_y = 0;  // z += P (zc + pending Yc) of the coarser level
  const T* zc = nullptr;
  const T* Yc = nullptr;
};

template <typename T>
struct RestrictArgs {
  int n = 0, ne = 0;                // fine level
  const T* L = nullptr;
  const T* Lc = nullptr;            // class table of L
  const int32_t* cols = nullptr;
  const T* f = nullptr;
  const T* z_old = nullptr;
  const T* Y_old = nullptr;         // pending tile outputs [ne][3][4]
  T* z_new = nullptr;
  T* rc = nullptr;                  // coarse right-hand side P^T (f - L z)
  int has_z = 0, has_y = 0, write_z = 0;
};

template <typename T>
hipError_t launch_sweep(const SweepArgs<T>& a, int waves_per_tile, hipStream_t st);
// The same step with gx x gx tiles per workgroup and the tile solves as MFMA
// products of each class inverse with the group's residuals (n / 4 must be
// a multiple of gx; gx in {1, 2, 4}); a.gextra / a.nextra list the classes
// after the first of every group, each run by a workgroup of its own.
template <typename T>
hipError_t launch_sweep_g(const SweepArgs<T>& a, int gx, hipStream_t st, hipEvent_t ev0 = nullptr,
                          hipEvent_t ev1 = nullptr);
template <typename T>
hipError_t launch_restrict_res(const RestrictArgs<T>& a, hipStream_t st);
// out = (has_z ? z : 0) + pending Ye
template <typename T>
hipError_t launch_resolve(int ne, bool has_z, const T* z, const T* Ye, T* out, hipStream_t st);
// z64 = (first ? 0 : z64) + (double)((has_z ? z : 0) + (has_y ? pending Ye : 0))
// (z and Ye addressed through sl.lsq / sl.lstride)
template <typename T>
hipError_t launch_refine_add(int ne, bool first, bool has_z, bool has_y, const T* z, const T* Ye,
                             double* z64, hipStream_t st, const Slots& sl = Slots(), int count = 1,
                             const Scalars* guard = nullptr);

// ------------------------------------------------------------ batched cycle
// The same steps on kBatch request-interleaved columns (mg_batch.hip): the
// RAS step multiplies each tile inverse into the 128 x kBatch residual block
// with MFMA, the coarsest solve is a 1024 x 1024 by 1024 x kBatch FP64 MFMA
// product.  Column c of every output depends on column c of the inputs only.
template <typename T>
hipError_t launch_sweep_b(const SweepArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_restrict_res_b(const RestrictArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_coarse_b(const double* inv, const T* f, T* z, hipStream_t st);
template <typename T>
hipError_t launch_resolve_b(int ne, bool has_z, const T* z, const T* Ye, T* out, hipStream_t st);

// Exact inner solve on the uniform grid: z = L^{-1} s by fast
// diagonalisation, L = M (x) K + K (x) M on the tensor index (Iy, Ix) of the
// 2n x 2n grid of dofs, with K V = M V diag(lam), V^T M V = I (V, its
// transpose VT, both 2n x 2n row-major); s, z scalar vectors 4 e + j; t0..t2
// scratch of 4 n^2 doubles each.
hipError_t launch_fdm_solve2d(int n, const double* V, const double* VT, const double* lam,
                              const double* s, double* z, double* t0, double* t1, double* t2,
                              hipStream_t st);
// The same solve as the exact coarsest-level solve of a multigrid level of n
// squares per side with level vectors of type T (FP32 in the mixed form): f
// is widened to FP64, solved in FP64 and z rounded back to T.
template <typename T>
hipError_t launch_fdm_coarse(int n, const double* V, const double* VT, const double* lam,
                             const T* f, T* z, double* t0, double* t1, double* t2, hipStream_t st);

}  // namespace dcg
