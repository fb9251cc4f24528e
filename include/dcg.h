/*
 * dcg.h -- C ABI of the MI355X deflated-CG solver for the implicit time step
 * of the pseudo-stress Stokes problem.
 *
 * The operator (paper, Section 3, eq. (pb_study)) is A* = M + alpha A with
 *   M  the dev-dev mass form (mu^{-1} dev sigma, dev tau)  (Section 2.3),
 *   A  the div-div SIPG form sum_{k,i,j} a^h_ij(sigma_ki, tau_kj)
 *      (eq. (component_form), Section 3.3.2),
 *   alpha = dt (implicit Euler, Section 2.3), mu = nu.
 * discretised with discontinuous Q1 per stress component on the uniform grid
 * of n x n squares of the unit square, penalty gamma = penalty * n, SIPG face
 * terms on interior faces and on the traction boundary {x = 0} u {y = 0}.
 *
 * The solve is deflated CG (Section 4.1, Algorithm 2) with the deflation
 * basis V of eq. (Vmatrix) (called Z below), whose inner system
 * Z^T A* Z = (dt / 2) L is a scaled SIPG Laplacian (Corollary 1).  The inner
 * system is solved by the Multigrid iteration (Algorithm 3) of W-cycles
 * (Algorithm 4) with a Restricted Additive Schwarz smoother (Section 4.2) to
 * the fixed relative tolerance c_F * tol (eq. (fixed_tol)).
 *
 * Vector layout (every FP64 tensor vector passed through this ABI):
 *   length 16 n^2, element-major, idx = 16 e + 4 c + j with
 *   e = ey * n + ex (square (ex, ey) = [ex/n, (ex+1)/n] x [ey/n, (ey+1)/n]),
 *   c in {0: sigma_11, 1: sigma_12, 2: sigma_21, 3: sigma_22} (Section 3.1),
 *   j = ix + 2 iy the corner (ex + ix, ey + iy) / n of the square.
 * Scalar (Laplace / multigrid) vectors: length 4 n_k^2, idx = 4 e + j.
 *
 * Pointers: every vector argument is a DEVICE pointer on the current HIP
 * device unless stated otherwise; host buffers are marked "host".  The caller
 * owns all vectors; the library owns every matrix, hierarchy, workspace and
 * scratch buffer and frees them in dcg_destroy / dcg_server_destroy.  The
 * library never frees caller memory.  A stream argument is a hipStream_t
 * (NULL = the legacy default stream); the library enqueues its work there.
 *
 * Errors: negative status = error (nothing written to the output vector or
 * its contents are unspecified); dcg_last_error(h) / dcg_last_error(NULL)
 * give the message of the last failing call on that handle / thread.
 * Positive status DCG_NOT_CONVERGED: the output holds the reconstructed last
 * iterate and the stats are valid.
 */
#ifndef DCG_H
#define DCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DCG_OK = 0,
  DCG_NOT_CONVERGED = 1,  /* max_outer reached; x holds the last iterate      */
  DCG_PENDING = 2,        /* dcg_poll: request not finished yet               */
  DCG_EINVAL = -1,        /* bad argument, unsupported size, NaN/Inf input    */
  DCG_ENOMEM = -2,        /* device or host allocation failed / over budget   */
  DCG_EDEVICE = -3,       /* a HIP call or kernel launch failed               */
  DCG_EAGAIN = -4,        /* server queue full                                */
  DCG_ENOTFOUND = -5,     /* unknown ticket                                   */
  DCG_EBREAKDOWN = -6     /* (p, q) <= 0 or non-finite in the outer iteration */
} dcg_status;

typedef enum { DCG_FP64 = 0, DCG_MIXED = 1 } dcg_precision;
/* DCG_MIXED: multigrid levels (smoother, transfers, level SpMVs) in FP32 with
 * FP32 accumulation; outer CG, deflation, the inner refinement residual and
 * the coarsest Cholesky solve in FP64. */

typedef enum {
  DCG_OUTER_CG = 0,   /* Fletcher-Reeves beta = rho_new / rho (Tables 2-3)    */
  DCG_OUTER_FCG1 = 1, /* flexible CG with one stored direction, Algorithm 1
                         truncated to m_i = 1 (Remark 5, m_max = 1)           */
  DCG_OUTER_FCG = 2,  /* flexible CG, Algorithm 1 with the truncation of
                         Remark 5, m_0 = 0, m_i = max{1, mod(i, m_max + 1)};
                         m_max = 0 means FCG(inf), m_i = i (every direction
                         kept: 2 vectors of 16 n^2 doubles per iteration --
                         meant for small n).  dcg_solve only.                 */
  DCG_OUTER_GMRES = 3 /* unrestarted GMRES on the deflated system (Remark 6):
                         Arnoldi basis orthogonalised by two classical
                         Gram-Schmidt passes, stop on the minimal residual
                         ||r_i|| <= tol ||b||; keeps one vector of 16 n^2
                         doubles per iteration (small n).  dcg_solve only.    */
} dcg_outer;

typedef struct {
  int32_t n;        /* squares per side; 16 * 2^k for k >= 0, at most 2048   */
  double penalty;   /* alpha* of the SIPG penalty gamma = alpha* / h [10]     */
  int32_t pre;      /* m1 pre-smoothing RAS sweeps  [2]                       */
  int32_t post;     /* m2 post-smoothing RAS sweeps [2]                       */
} dcg_mesh;

typedef struct {
  dcg_precision prec;  /* [DCG_MIXED]                                         */
  dcg_outer outer;     /* [DCG_OUTER_CG]                                      */
  double c_F;          /* inner tolerance factor, tau^c = c_F * tol [0.01]    */
  int32_t max_outer;   /* [50000]                                             */
  int32_t max_inner;   /* W-cycles per inner solve, n_max of Alg. 3 [100]     */
  int32_t x0_given;    /* 0: x0 = 0; 1: x holds the initial guess on entry    */
  int32_t use_graph;   /* 1: replay each W-cycle as a captured HIP graph [1]  */
  int64_t hbm_budget_bytes; /* server admission budget, 0 = device total      */
  int32_t max_pending; /* server: unfinished requests before DCG_EAGAIN [4096] */
  double c_A;          /* > 0: adaptive inner tolerance of eq. (tol),
                          tau^c_i = c_A tol ||b|| / ||r_i|| for the inner solve
                          of outer iteration i and c_A tol for the prologue
                          and epilogue solves, instead of c_F tol [0 = off]   */
  int32_t m_max;       /* DCG_OUTER_FCG truncation, 0 = FCG(inf) [8]         */
  int32_t inner;       /* dcg_inner: the inner solver [DCG_INNER_MG]           */
  int32_t levels;      /* multigrid levels J of the inner W-cycle (Algorithm 4,
                          levels k = 1..J, Section 5 uses four).  0 = every
                          level down to 16 x 16 squares, J = log2(n/16) + 1;
                          1 <= levels < log2(n/16) + 1: the finest `levels`
                          levels of that hierarchy, whose coarsest level of
                          n / 2^(levels-1) squares per side (at most 1024) is
                          solved exactly by fast diagonalisation of its
                          Galerkin operator L_1 = M_1 (x) K_1 + K_1 (x) M_1
                          (the dense Cholesky solve up to rounding, without
                          forming the inverse).  dcg_solve / dcg_apply only;
                          the server and the _BATCH operators need 0.  [0]   */
  int32_t restarts;    /* dcg_solve: when the reconstructed x misses tol on its
                          true residual ||b - A* x|| / ||b|| (the recurrence
                          residual of inexact inner solves drifts from it),
                          run Algorithm 2 again from x_0 = x, at most this many
                          times (pi(b) and f_D are reused; counts and max_outer
                          cover every pass).  With restarts > 0 the status is
                          DCG_OK only if the true residual meets tol, else
                          DCG_NOT_CONVERGED; 0 keeps the paper's test on the
                          recurrence residual alone.  Ignored by the server. [0] */
  int32_t ras_group;   /* RAS step kernel of levels >= 2 (Section 4.2):
                          0 = automatic by level size; 1, 2 or 4 = one
                          workgroup per ras_group x ras_group tiles with the
                          tile solves as MFMA products of each class inverse
                          with the group's residuals; -1 = one tile per
                          wavefront group, scalar FMAs.  Same step either way
                          (up to rounding).  Not used by the server. [0]     */
  int32_t smooth3d;    /* 3D solver with DCG3D_INNER_MG: m pre- and m post-
                          smoothing RAS steps per level visit of the W-cycle
                          (the 3D runs of Section 4.2 use m = 10).  Ignored
                          elsewhere. [10]                                    */
  int32_t outer_mg;    /* DCG_OUTER_FCG, dcg_solve / dcg_apply only: > 0
                          preconditions the flexible outer iteration with B =
                          one W-cycle (Algorithm 4, outer_mg pre- and post-
                          smoothing RAS steps, gamma = 2) on the Galerkin
                          hierarchy of A* itself down to 8 x 8 squares, RAS
                          blocks of a square and its edge neighbours over all
                          four stress components, the coarsest level solved
                          by a dense FP64 inverse; the direction of Algorithm
                          1 is built from B r_i (the multigrid outer
                          preconditioner the paper's conclusions leave to
                          future work).  FP64, built per handle (A* depends
                          on dt).  0 = off. [0]                              */
} dcg_options;

/* Inner solver of dcg_solve.  DCG_INNER_MG is the paper's method: the
 * Multigrid iteration (Algorithm 3) of W-cycles with the RAS smoother to the
 * inner tolerance.  DCG_INNER_EXACT solves the inner system exactly (the
 * exact-inner deflated CG of Tables 1-2): on this uniform grid the SIPG
 * Laplacian of Corollary 1 is L = M (x) K + K (x) M on the (y, x) grid of
 * dofs with one-dimensional DG-P1 matrices M (mass) and K (SIPG, traction node
 * at the left end, identical along x and y), so L^{-1} = V' diag(1/(l_i + l_k))
 * V'^T with V' = V (x) V from the generalised eigenvectors K V = M V diag(l)
 * (fast diagonalisation: four dense 2n x 2n FP64 products per inner solve).
 * dcg_solve only, n <= 1024; stats count 0 W-cycles. */
typedef enum {
  DCG_INNER_MG = 0,
  DCG_INNER_EXACT = 1,
  DCG_INNER_NONE = 2   /* no deflation: every inner solve returns 0, so pi = 0,
                          f_D = f, M_D = A* and the reconstruction returns
                          x_hat -- plain CG on A* (the CG columns of Tables 1-2) */
} dcg_inner;

typedef struct {
  int32_t status;          /* dcg_status of the solve                         */
  int32_t outer_iters;     /* "Out" of Table 3                                */
  int32_t total_wcycles;   /* "Tot": every W-cycle of the solve               */
  int32_t inner_solves;    /* number of inner solves (prologue + epilogue too) */
  double inner_per_outer;  /* "Inn": W-cycles per outer iteration (mean)      */
  double rel_res_recurrence; /* ||r_i|| / ||b|| at exit                       */
  double rel_res_true;     /* ||b - A* x|| / ||b|| after reconstruction       */
  double t_setup_ms;       /* handle setup time (mesh context build/upload)   */
  double t_solve_ms;       /* wall time of dcg_solve; server: admission to done */
  double t_queue_ms;       /* server: submission to admission (0 for dcg_solve) */
  int32_t restarts;        /* warm restarts taken (dcg_options.restarts)       */
} dcg_stats;

typedef struct dcg_ctx* dcg_handle;
typedef struct dcg_srv* dcg_server;

/* Fills *mesh and *opt with the defaults shown in brackets above. */
void dcg_defaults(dcg_mesh* mesh, dcg_options* opt);

/* Builds (or reuses from the process-wide cache) the dt-independent mesh
 * context -- A_div, the element mass blocks, A_div Z, the Galerkin multigrid
 * hierarchy of L (Algorithm 2: Z_{k-1} = I Z_k I), the RAS tile inverses and
 * the coarsest inverse -- on the current device, and a solver handle for the
 * scalars dt > 0, nu > 0.  On the uniform grid the RAS local problems and the
 * level operators' blocks fall into 9 bit-identical classes per level
 * (interior, edges, corners); the context stores one tile inverse and one set
 * of operator blocks per class (setup checks the bit identity).  With
 * opt->levels > 0 the handle also holds the fast-diagonalisation factors of
 * its coarsest level.  opt may be NULL (defaults).  Returns DCG_EINVAL for
 * unsupported n / parameters, DCG_ENOMEM when device memory runs out. */
dcg_status dcg_setup(const dcg_mesh* mesh, double dt, double nu,
                     const dcg_options* opt, dcg_handle* out);

/* Solves A* x = b to ||r_i|| <= tol ||b|| (Section 4.1) by Algorithm 2 with
 * the outer variant of the handle's options: prologue f_D = b - A* pi(b),
 * outer iterations on the deflated system, epilogue
 * x = (x_hat - pi(A* x_hat)) + pi(b) (eq. (x_defl)).  b, x: device, length
 * 16 n^2, FP64, element-major; b is not modified.  Blocks until done.
 * st (host, may be NULL) receives the counts of Table 3 and the residuals. */
dcg_status dcg_solve(dcg_handle h, const double* b, double* x, double tol,
                     dcg_stats* st, void* hip_stream);

/* Operator-level entry points (for verification and composition).  All on
 * the handle's mesh context; vectors are device pointers.  "level" counts
 * the handle's multigrid levels 1 (coarsest: 16 x 16, or the coarsest level
 * of opt.levels) .. J (finest); level vectors are
 * FP32 in the DCG_MIXED form and FP64 in the DCG_FP64 form ("real" below).
 *
 *  op                 in           in2         out          computes
 *  DCG_OP_ASTAR       p  (f64,N)   -           w  (f64,N)   A* p  (eq. (pb_study))
 *  DCG_OP_ZT          w  (f64,N)   -           s  (f64,m)   Z^T w  (eq. (Vmatrix))
 *  DCG_OP_Z           y  (f64,m)   -           v  (f64,N)   Z y
 *  DCG_OP_ADIVZ       y  (f64,m)   -           v  (f64,N)   A_div Z y
 *  DCG_OP_DEFLATED    p  (f64,N)   -           q  (f64,N)   M_D p = A*(p - pi(A* p))
 *  DCG_OP_INNER       s  (f64,m)   -           y  (f64,m)   (Z^T A* Z)^{-1} s by Alg. 3
 *  DCG_OP_LAPLACE     z  (real,m_k) -          v  (real,m_k) L_k z (L_J = 2 Z^T A_div Z)
 *  DCG_OP_RAS         f  (real,m_k) z (real)   z' (real,m_k) z + S_k (f - L_k z)
 *  DCG_OP_RESTRICT    r  (real,m_k) -          rc (real,m_{k-1}) P_k^T r
 *  DCG_OP_PROLONG     e  (real,m_{k-1}) -      v  (real,m_k) P_k e
 *  DCG_OP_COARSE      f  (real,m_1) -          z  (real,m_1) L_1^{-1} f (FP64 inverse, or
 *                                                            FP64 fast diagonalisation)
 *  DCG_OP_WCYCLE      f  (real,m_k) z0 (real or NULL = 0)  z (real,m_k)  Wcycle_k(f, z0)
 *  DCG_OP_RAS_BATCH   f  (real,16 m_k) z (real)  z' (real,16 m_k)  DCG_OP_RAS of 16 vectors
 *  DCG_OP_WCYCLE_BATCH f (real,16 m_k) z0 (or NULL) z (real,16 m_k) DCG_OP_WCYCLE of 16 vectors
 *
 * The _BATCH operators run the kernels of the serving engine: 16 level
 * vectors interleaved as idx = (16 e + c) 4 + j (vector c = 0..15), the RAS
 * tile solves as MFMA products with the 16 residuals; they need post >= 1.
 *
 * Level operators act on L_k = (2/dt) Z_k (the dt-free Laplacian hierarchy);
 * the hierarchy of Algorithm 2 is Z_k = (dt/2) L_k.  m = 4 n^2, m_k = 4 n_k^2.
 * Returns DCG_EINVAL for a bad op/level or NULL pointer. */
typedef enum {
  DCG_OP_ASTAR = 0, DCG_OP_ZT = 1, DCG_OP_Z = 2, DCG_OP_ADIVZ = 3,
  DCG_OP_DEFLATED = 4, DCG_OP_INNER = 5, DCG_OP_LAPLACE = 6, DCG_OP_RAS = 7,
  DCG_OP_RESTRICT = 8, DCG_OP_PROLONG = 9, DCG_OP_COARSE = 10, DCG_OP_WCYCLE = 11,
  DCG_OP_RAS_BATCH = 12, DCG_OP_WCYCLE_BATCH = 13,
  /* the outer multigrid preconditioner (opt.outer_mg > 0), FP64 tensor level
   * vectors of 16 n_k^2 values in the element-major layout, levels k = 1
   * (8 x 8 squares) .. J = log2(n/8) + 1:
   *  DCG_OP_OMG_APPLY    r (J)       -          z (J)       B r, one W-cycle from zero
   *  DCG_OP_OMG_LEVEL    z (k)       -          v (k)       A*_k z (A*_J = A*)
   *  DCG_OP_OMG_RAS      f (k)       z or NULL  z' (k)      z + S_k (f - A*_k z), k >= 2
   *  DCG_OP_OMG_RESTRICT r (k)       -          rc (k - 1)  P_k^T r, k >= 2
   *  DCG_OP_OMG_PROLONG  e (k - 1)   -          v (k)       P_k e, k >= 2
   *  DCG_OP_OMG_COARSE   f (1)       -          z (1)       (A*_1)^{-1} f
   *  DCG_OP_OMG_WCYCLE   f (k)       z0 or NULL z (k)       Wcycle_k(f, z0) */
  DCG_OP_OMG_APPLY = 14, DCG_OP_OMG_LEVEL = 15, DCG_OP_OMG_RAS = 16, DCG_OP_OMG_RESTRICT = 17,
  DCG_OP_OMG_PROLONG = 18, DCG_OP_OMG_COARSE = 19, DCG_OP_OMG_WCYCLE = 20
} dcg_op;

dcg_status dcg_apply(dcg_handle h, dcg_op op, int32_t level, const void* in,
                     const void* in2, void* out, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): dcg_apply's
 * DCG_OP_INNER and DCG_OP_DEFLATED (same operands, same kernels, same result)
 * with every buffer the kernels write besides `out` -- the scalar block,
 * partial sums, the inner iterate, the W-cycle's level vectors and, for
 * DCG_OP_DEFLATED, A* p and Z^T A* p -- in one static device array of
 * dcg_noalloc_bytes() bytes (48 MiB: every mesh up to n = 256 in either
 * precision) instead of the handle's workspace.  The call allocates nothing;
 * each device it runs on holds its own copy of the array until the process
 * ends.  The handle must use the multigrid inner solve (DCG_INNER_MG).
 * Returns DCG_EINVAL for another op or inner solver, and for a mesh whose
 * buffers exceed the array (the message gives both sizes).  The handle's
 * device is made current for the call.  The array is shared by every call
 * on a device and keeps the previous call's contents: calls that overlap on
 * one device (other threads, other streams) race and must be serialised by
 * the caller.  Blocks until done, like dcg_apply. */
dcg_status dcg_apply_noalloc(dcg_handle h, dcg_op op, const double* in, double* out,
                             void* hip_stream);
int64_t dcg_noalloc_bytes(void);

/* Number of multigrid levels J of a mesh (log2(n/16) + 1), or -1. */
int32_t dcg_num_levels(int32_t n);

/* Host-only assembly, no device needed: writes one assembled matrix of the
 * mesh context into the host buffer ``dst`` as a dense row-major FP64 block
 * array in the block-ELL layout used on the device, and the int32 column
 * (neighbour element) indices into ``cols`` (host, may be NULL):
 *   which = 0: A_div,    blocks 16 x 16, dst [n^2][5][16][16]
 *   which = 1: A_div Z,  blocks 16 x 4,  dst [n^2][5][16][4]
 *   which = 2: M_1,      element mass 4 x 4, dst [n^2][4][4] (cols unused)
 *   which = 3: L_level,  blocks 4 x 4,   dst [n_k^2][5][4][4]
 *   which = 4: RAS tile inverses of level, D_i-weighted, dst [T_k][128][128]
 *              (F[j][i] = (L_k)_i^{-1}[j][i] d_i), cols [T_k][32] = squares
 *   which = 5: coarsest inverse L_1^{-1}, dst [1024][1024]
 *   which = 6: exact inner solve factors (n <= 256): the axis eigenvectors
 *              V [2n][2n] row-major, then the eigenvalues lam [2n]
 *   which = 7: the same factors of the coarsest level of the hierarchy with
 *              ``level`` levels (opt.levels; 1 <= level <= J), whose axis
 *              has N = 2 n / 2^(level-1) dofs (N <= 512): V [N][N], lam [N]
 * Slots are (self, x-1, x+1, y-1, y+1); a missing neighbour has a zero
 * block and column index -1.  ``dst_len`` is the buffer length in doubles;
 * *needed (may be NULL) receives the required length.  Returns DCG_EINVAL
 * when the buffer is too small or the arguments are invalid. */
dcg_status dcg_host_assemble(const dcg_mesh* mesh, int32_t which, int32_t level,
                             double* dst, int64_t dst_len, int32_t* cols,
                             int64_t cols_len, int64_t* needed);

/* Host only (no device call): the class tables of the outer multigrid
 * preconditioner (opt.outer_mg) for n = 16 2^k <= 64, penalty, dt, nu, on
 * level `level` (1 = 8 x 8 squares .. J = log2(n/8) + 1), into the HOST
 * buffer dst of dst_len doubles.  On the uniform grid a square's rows of A*_k
 * depend only on the domain sides it touches and its RAS update only on its
 * distance 0, 1, 2 or >= 3 from each side.  which = 0: the operator table
 * [9][5][16][16], entry (cls, slot, a, b) = A*_k(row a of a square of class
 * cls = cx + 3 cy -- c_axis 0 at the low side, 2 at the high side, 1 inside --
 * column b of its slot neighbour: 0 itself, 1/2 x-1/x+1, 3/4 y-1/y+1), rows
 * and columns 4 c + j (element-major); 1 (level >= 2): the RAS update table
 * [49][16][208], (S_k r) on a square of class px + 7 py (p = x for x < 3,
 * 6 - (n_k - 1 - x) for n_k - 1 - x < 3, else 3) equals table[cls] times r on
 * the 13 squares (dx, dy) with |dx| + |dy| <= 2 (by dy, then dx; column
 * 16 d + b); 2 (level 1): the inverse of A*_1, [1024][1024] row-major;
 * 3 and 4 (level >= 2 for 4): the tables 0 and 1 in the operand order of the
 * MFMA kernels, [9][20][64] and [49][52][64], entry (cls, s, l) = row l % 16,
 * column 4 s + l / 16 of the class's matrix (for table 0 the 16 x 80 matrix
 * with column 16 slot + b).
 * DCG_EINVAL for bad arguments or a short buffer. */
dcg_status dcg_host_outer_mg(int32_t n, double penalty, double dt, double nu, int32_t level,
                             int32_t which, double* dst, int64_t dst_len);

/* BDF2 time stepping (Section 2.3, implicit multistep family; BDF2 reading):
 * for M d(sigma)/dt + A sigma = F the step n solves (M + alpha A) sigma^n = f
 * with alpha = 2 dt_step / 3 and
 *   f  = M (4/3 s1 - 1/3 s2) + c F,   c = 2 dt_step / 3,
 * s1 = sigma^{n-1}, s2 = sigma^{n-2}; the warm start is x0 = 2 s1 - s2.
 * This entry point computes f and x0 (device FP64 tensor vectors, element-
 * major; f and x0 must not alias the inputs) with the handle's mass M =
 * (1/nu) C (x) M_1; the solve itself is dcg_solve on a handle created with
 * dt = alpha and x0_given = 1. */
dcg_status dcg_bdf2_rhs(dcg_handle h, const double* s1, const double* s2, const double* F,
                        double c, double* f, double* x0, void* hip_stream);

/* Live timing of the dominant kernel of the solve, the RAS step of the
 * finest level (Section 4.2, (A_J)_i^{-1} applied to every block).
 * enable = k > 0: the finest-level launches of every k-th W-cycle enqueued by
 * dcg_solve on this handle (k = 1: every launch; the inner iteration
 * enqueues a few cycles beyond its test, which run the same kernels) carry a
 * pair of HIP events on the solve's stream: recorded in the dispatch packet
 * of the grouped RAS kernel (the kernel's own start and end), around the
 * launch for the per-tile kernel.  Those launches are issued outside the
 * captured graph; the elapsed times are accumulated at the solver's syncs.
 * enable = 0 switches the timing off.  Enabling or disabling discards the
 * captured graph.  _read returns the accumulated milliseconds and launch
 * count since the last enable. */
dcg_status dcg_kernel_timing(dcg_handle h, int32_t enable);
dcg_status dcg_kernel_timing_read(dcg_handle h, double* total_ms, int64_t* launches);
/* The same for the A* product with the fused direction update of the CG outer
 * loop (eq. (pb_study), Section 3.1; events in its dispatch packet): summed
 * duration and count of its launches since dcg_kernel_timing enabled the
 * timing (CG and FCG(1) outer variants). */
dcg_status dcg_kernel_timing_read_astar(dcg_handle h, double* total_ms, int64_t* launches);

/* ---------------------------------------------------------------- serving
 * A server solves many requests A*_i x_i = b_i concurrently on the current
 * device by continuous batching.  Requests that share (n, penalty, pre,
 * post) share one resident mesh context and are advanced together, up to 16
 * at a time: one launch per step of the outer iteration covers every
 * request at that step (dt and nu are per-request scalars; A* = (1/nu) C (x)
 * M_1 + dt A_div is never assembled per request), and the inner W-cycles of
 * all of them run as one batched cycle whose RAS tile solves (Section 4.2)
 * are matrix products of each tile inverse with the 16 requests' residuals
 * (MFMA).  Each request keeps its own convergence tests, so it performs the
 * iterations of Algorithm 2 / 3 it would perform alone, and its result does
 * not depend on the other requests of the batch (bitwise).
 *
 * opt: precision, outer variant, c_F, max_outer, max_inner, use_graph for
 * every request; hbm_budget_bytes bounds the device memory of the resident
 * mesh contexts plus the batch workspaces (a request whose group does not
 * fit waits until idle groups can be released; one that cannot fit even on
 * an idle server fails with DCG_ENOMEM); max_pending bounds the unfinished
 * requests (DCG_EAGAIN beyond).  x0_given is ignored: solves start at 0.
 * The server runs one host thread and its own HIP streams on the device
 * current at creation.  Requires post >= 1. */
dcg_status dcg_server_create(const dcg_options* opt, dcg_server* out);

/* Builds the mesh context of ``mesh`` ahead of traffic (as the first
 * request of that mesh would); optional. */
dcg_status dcg_server_prepare(dcg_server s, const dcg_mesh* mesh);

/* Queues one solve; returns at once with *ticket.  b, x: device, length
 * 16 n^2, FP64, element-major; b must hold its values when this is called
 * and both must stay allocated until dcg_poll returns a terminal status (b
 * is copied at admission, x is written at completion).  tol as dcg_solve.
 * DCG_EAGAIN: max_pending requests are unfinished.  DCG_EINVAL: bad
 * arguments (checked here, not at admission). */
dcg_status dcg_submit(dcg_server s, const dcg_mesh* mesh, double dt, double nu,
                      const double* b, double* x, double tol, uint64_t* ticket);

/* DCG_PENDING while the request is queued or running.  Otherwise returns
 * its terminal status (as dcg_solve would), fills *st (may be NULL; also
 * for errors) and forgets the ticket; dcg_last_error(NULL) then gives the
 * message of a failed request.  DCG_ENOTFOUND: unknown or already
 * reported ticket. */
dcg_status dcg_poll(dcg_server s, uint64_t ticket, dcg_stats* st);

/* Device bytes a server group of ``mesh`` occupies in precision ``prec``:
 * its mesh context plus the workspace of 16 request slots (the quantity the
 * admission test charges against hbm_budget_bytes); -1 for a bad mesh. */
int64_t dcg_server_group_bytes(const dcg_mesh* mesh, dcg_precision prec);

/* Steps run so far and the occupied request slots summed over them
 * (slot_steps / steps = mean batch occupancy). */
dcg_status dcg_server_counters(dcg_server s, int64_t* steps, int64_t* slot_steps);

/* Stops the server thread (unfinished requests are abandoned: their x is
 * unspecified) and frees every buffer it owns. */
dcg_status dcg_server_destroy(dcg_server s);

dcg_status dcg_destroy(dcg_handle h);
const char* dcg_strerror(dcg_status s);
const char* dcg_last_error(dcg_handle h);

/* Releases every cached mesh context (all devices).  Handles keep their own
 * reference; call after destroying them to return the memory. */
void dcg_clear_cache(void);

/* ---------------------------------------------------------------------------
 * Three-dimensional solver: the d = 3 block structure of Section 3.1.
 *
 * Unknowns: the nine components sigma_ki (Section 3.1, d = 3), discontinuous
 * Q1 on the grid of n x n x n cubes of the unit cube; M = mu^{-1} C_9 (x) M_1
 * with the printed 9 x 9 coefficient matrix, A = blockdiag(C_3, C_3, C_3),
 * C_3 = [B_ij] from the SIPG forms a^h_ij, i, j in {1, 2, 3}
 * (Section 3.3.2), penalty gamma = penalty * n, SIPG face terms on interior
 * faces and on the outflow face {x = 1} (where the 3D test of Section 4.2
 * imposes sigma n = 0).  Deflation basis Z = V of eq. (Vmatrix) for d = 3,
 * so Z^T A* Z = (dt/3)(B_11 + B_22 + B_33) (Corollary 1).
 *
 * Solve: Algorithm 2 with the CG outer iteration.  The inner system
 * E = Z^T A* Z = (dt/3) L is solved either exactly (DCG3D_INNER_FDM, the
 * setting of Table 5, left): on this uniform grid L is the Kronecker sum of
 * one-dimensional DG matrices, L = M (x) M (x) K_x + M (x) K_y (x) M +
 * K_z (x) M (x) M, so L^{-1} = V diag(1/(lx + ly + lz)) V^T with the
 * generalised eigenvectors of each axis (fast diagonalisation, six axis
 * passes); or by block-Jacobi preconditioned CG to the relative residual
 * c_F * tol (eq. (fixed_tol)), at most max_inner steps (DCG3D_INNER_PCG).
 * Everything runs in FP64 on the device; dcg_stats.total_wcycles counts inner
 * CG steps (0 for the exact solve).
 *
 * Layout (device pointers, FP64): tensor vectors 72 n^3 values, element-major,
 * idx = 72 e + 8 c + a with e = (ez n + ey) n + ex, c = 3 k + i for
 * sigma_{k+1,i+1}, a = ix + 2 iy + 4 iz the corner (ex + ix, ey + iy, ez + iz)/n;
 * scalar (inner) vectors 8 n^3 values, idx = 8 e + a.  All work is enqueued
 * on the legacy default stream and the calls return after it has finished.
 * The caller owns the vectors, the handle owns its operators (about
 * 33 KB per element) and workspaces.  Errors as above; dcg3d_last_error. */
#define DCG3D_MAX_N 64
#define DCG3D_DEFAULT_MAX_INNER 20000

typedef struct dcg3d_ctx* dcg3d_handle;

typedef enum {
  DCG3D_INNER_FDM = 0,    /* exact inner solve by fast diagonalisation (default)  */
  DCG3D_INNER_PCG = 1,    /* block-Jacobi CG to c_F * tol                           */
  DCG3D_INNER_NONE = 2,   /* no deflation: plain CG on A* (the CG column of Table 5)  */
  DCG3D_INNER_MG = 3      /* the Multigrid iteration of Algorithm 3 with W-cycles and
                             the RAS smoother (Section 4.2, the 3D case; see below)   */
} dcg3d_inner;

typedef enum {
  DCG3D_OP_ASTAR = 0,     /* out = A* in            (tensor -> tensor), eq. (pb_study)        */
  DCG3D_OP_ZT = 1,        /* out = Z^T in           (tensor -> scalar), eq. (Vmatrix)         */
  DCG3D_OP_Z = 2,         /* out = Z in             (scalar -> tensor)                        */
  DCG3D_OP_DEFLATED = 3,  /* out = M_D in = A*(in - Z E^{-1} Z^T A* in), inner to tol, Alg. 2 */
  DCG3D_OP_REDUCED = 4,   /* out = E in, E = Z^T A* Z (scalar), Corollary 1                   */
  DCG3D_OP_INNER = 5,     /* out = E^{-1} in by the inner solver (PCG: to relative residual tol) */
  DCG3D_OP_ADIVZ = 6      /* out = A_div Z in       (scalar -> tensor), Corollary 1 (proof)   */
} dcg3d_op;

/* Assembles the operators on the host and uploads them (2 <= n <= 64,
 * penalty > 0, dt > 0, nu = mu > 0, inner a dcg3d_inner).  opt may be NULL (defaults of
 * dcg_defaults with prec = DCG_FP64 and max_inner = DCG3D_DEFAULT_MAX_INNER);
 * the 3D solver takes prec = DCG_FP64, outer = DCG_OUTER_CG and x0_given = 0
 * and rejects other values with DCG_EINVAL.  The iterative inner solves stop
 * at the relative residual c_F tol (eq. (fixed_tol)), or with c_A > 0 at
 * c_A tol ||b|| / ||r_i|| inside the outer loop and c_A tol for the prologue
 * and epilogue (eq. (tol)); max_inner is their n_max.  opt->restarts = R > 0
 * reruns Algorithm 2 from the reconstructed x while its true residual misses
 * tol, at most R times (pi(b) and f_D of the first pass; the status is then
 * DCG_OK only if the true residual meets tol), as in dcg_solve.
 *
 * DCG3D_INNER_MG: the Galerkin hierarchy of L = B_11 + B_22 + B_33 (levels
 * k = 1..J by 2 x 2 x 2 agglomeration, trilinear injection P_k, L_{k-1} =
 * P_k^T L_k P_k; opt->levels = J, 0 = down to the smallest coarsest size
 * c = n / 2^(J-1) >= 2, which must lie in [2, 4], else DCG_EINVAL), a RAS
 * smoother with one block per cube -- the cube and its face neighbours, the
 * local problems solved exactly, D = 1 / (blocks holding the dof) -- with
 * opt->smooth3d steps before and after each coarse correction, gamma = 2,
 * and the exact solve on level 1 by a dense inverse.  The multigrid runs on
 * L and returns (3/dt) z (E = (dt/3) L, the same relative residual); every
 * step runs on the device, the stopping test too (each pass of Algorithm 3
 * is one captured HIP graph when opt->use_graph, enqueued ahead of the
 * test's result); total_wcycles counts W-cycles. */
dcg_status dcg3d_setup(int32_t n, double penalty, double dt, double nu, int32_t inner,
                       const dcg_options* opt, dcg3d_handle* out);
/* Solves A* x = b to ||r|| <= tol ||b|| (the recurrence residual of the
 * deflated system, Section 4.1); st (may be NULL) receives the counts and the
 * true residual of the reconstructed x. */
dcg_status dcg3d_solve(dcg3d_handle h, const double* b, double* x, double tol, dcg_stats* st);
/* One operator of the path (tol is used by DCG3D_OP_DEFLATED and
 * DCG3D_OP_INNER only). */
dcg_status dcg3d_apply(dcg3d_handle h, dcg3d_op op, const double* in, double* out, double tol);
dcg_status dcg3d_destroy(dcg3d_handle h);
const char* dcg3d_last_error(dcg3d_handle h);

/* Level operators of the DCG3D_INNER_MG hierarchy (for verification; the
 * Laplacian hierarchy L_k, not scaled by dt).  Level vectors: device, FP64,
 * 8 n_k^3 values, idx = 8 e + a as above, n_k = n / 2^(J-k).
 *
 *  op                  in            in2              out         computes
 *  DCG3D_MG_LAPLACE    z (level k)   -                v (k)       L_k z
 *  DCG3D_MG_RAS        f (k)         z (k) or NULL=0  z' (k)      z + S_k (f - L_k z), k >= 2
 *  DCG3D_MG_RESTRICT   r (k)         -                rc (k - 1)  P_k^T r, k >= 2
 *  DCG3D_MG_PROLONG    e (k - 1)     -                v (k)       P_k e, k >= 2
 *  DCG3D_MG_COARSE     f (1)         -                z (1)       L_1^{-1} f (dense FP64 inverse)
 *  DCG3D_MG_WCYCLE     f (k)         z0 (k) or NULL=0 z (k)       Wcycle_k(f, z0), Algorithm 4
 *
 * Blocks until done; DCG_EINVAL for another inner solver, a bad op or
 * level, or a NULL in / out. */
typedef enum {
  DCG3D_MG_LAPLACE = 0, DCG3D_MG_RAS = 1, DCG3D_MG_RESTRICT = 2, DCG3D_MG_PROLONG = 3,
  DCG3D_MG_COARSE = 4, DCG3D_MG_WCYCLE = 5
} dcg3d_mg_op;
dcg_status dcg3d_mg_apply(dcg3d_handle h, int32_t op, int32_t level, const double* in,
                          const double* in2, double* out);
/* The hierarchy of a DCG3D_INNER_MG handle: J and the coarsest size c. */
dcg_status dcg3d_mg_levels(dcg3d_handle h, int32_t* levels, int32_t* coarsest);
/* Measurement: while enabled, every launch of the dominant kernel of the 3D
 * solve -- the A* product with the exact inner solve, the inner Laplacian
 * product with block-Jacobi CG -- is bracketed by HIP events on
 * the legacy default stream; _read returns their summed duration and count
 * since the last enable / read and restarts the count. */
dcg_status dcg3d_kernel_timing(dcg3d_handle h, int32_t enable);
dcg_status dcg3d_kernel_timing_read(dcg3d_handle h, double* total_ms, int64_t* launches);

/* Host only (no device call, 2 <= n <= 16): copies the blocks the 3D path
 * assembles into the HOST buffer out, for checks of the assembly without a
 * GPU.  which = 0: the blocks C_3 of A_div, [7][n^3][24][24] (face slot 0 the
 * element, 1 / 2 its -x / +x neighbour, 3 / 4 -y / +y, 5 / 6 -z / +z), entry
 * (row 8 j + a, column 8 i + b) = a^h_ij(phi_b on the neighbour, phi_a on the
 * element) at index (slot n^3 + e) 576 + (8 i + b) 24 + 8 j + a, zero where the
 * neighbour does not exist; 1: B_11 + B_22 + B_33 in the same slots,
 * [7][n^3][8][8], entry (a, b) at (slot n^3 + e) 64 + 8 b + a; 2: the inverses
 * of the diagonal blocks of (dt/3)(B_11 + B_22 + B_33), [n^3][8][8], entry
 * (a, b) at 64 e + 8 b + a; 3: the element mass matrix of M_1, [8][8];
 * 4: the fast-diagonalisation factors of the exact inner solve, V_x [2n][2n]
 * row-major (column i = eigenvector i), lambda_x [2n], then V_y, lambda_y. */
#define DCG3D_MAX_HOST_BLOCKS_N 16
dcg_status dcg3d_host_blocks(int32_t n, double penalty, double dt, int32_t which, double* out);

/* Host only (no device call, 2 <= n <= 16): the class tables the multigrid
 * inner solve uploads, for level `level` of the hierarchy with `levels`
 * levels (as opt->levels), into the HOST buffer out.  On the uniform grid a
 * cube's operator rows depend only on the domain sides it touches and its
 * RAS update only on its distance 0, 1, 2 or >= 3 from each side.  which = 0:
 * the operator table [27][7][8][8], entry (cls, slot, a, b) = L_k(row a of a
 * cube of class cls = cx + 3 cy + 9 cz -- c_axis 0 at the low side, 2 at the
 * high side, 1 inside -- column b of its slot neighbour), row-major, zero
 * for classes and neighbours absent on the level; 1 (k >= 2): the RAS
 * update table [343][8][200], (S_k r) on a cube of class px + 7 py + 49 pz
 * (p = x for x < 3, 6 - (n_k - 1 - x) for n_k - 1 - x < 3, else 3; on
 * levels with n_k < 6 the class is the cube index e) equals
 * table[cls] times r on the 25 cubes (dx, dy, dz) with |dx|+|dy|+|dz| <= 2
 * (ordered by dz, then dy, then dx ascending; column 8 d + b), zero rows for
 * absent classes; 2 (k = 1): the inverse of L_1, [8 c^3][8 c^3] row-major.
 * DCG_EINVAL for a bad n, levels, level or which. */
dcg_status dcg3d_host_mg(int32_t n, double penalty, int32_t levels, int32_t level, int32_t which,
                         double* out);

#ifdef __cplusplus
}
#endif
#endif /* DCG_H */
