// Three-dimensional deflated CG (the d = 3 form of Section 3.1): device data
// layout and kernel launchers.
//
// Mesh: n^3 cubes of the unit cube, element e = (ez n + ey) n + ex, DG-Q1 per
// stress component, corner a = ix + 2 iy + 4 iz.  Tensor vectors hold 72
// values per element, idx = 72 e + 8 c + a with c = 3 k + i for sigma_{k+1,i+1};
// scalar vectors 8 per element, idx = 8 e + a.
//
// Face slots of an element: 0 itself, 1 / 2 the -x / +x neighbour, 3 / 4 -y /
// +y, 5 / 6 -z / +z.
//
//   Cd [7][ne][24][24]  the 3 x 3 block C_3 = [B_ij] of A_div (Section 3.1)
//                       coupling element e (test) to its slot-s neighbour
//                       (trial), column-major: entry (row r = 8 j + a,
//                       column 8 i + b) at ((s ne + e) 24 + 8 i + b) 24 + r;
//                       row block j = test component, column block i = trial
//                       component within a row k of the tensor
//   Ld [7][ne][8][8]    B_11 + B_22 + B_33 (the SIPG Laplacian of
//                       Corollary 1), column-major per block
//   Dinv[ne][8][8]      inverse of the diagonal block of (dt/3) Ld,
//                       column-major (block-Jacobi preconditioner)
//   Me [8][8]           element mass matrix of M_1 (uniform mesh)
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dcg3 {

constexpr int kNb = 8;        // Q1 basis functions per cube
constexpr int kComp = 9;      // stress components
constexpr int kDof = 72;      // values per element of a tensor vector
constexpr int kSlots = 7;     // the element and its 6 face neighbours

// Scalars of the inner PCG iteration, kept on the device between launches.
struct PcgScalars {
  double rho;       // (r, z)
  double rr;        // (r, r)
  double pq;        // (p, E p)
  double alpha, beta;
  double thresh2;   // stop once (r, r) <= thresh2
  int32_t active;   // 0 once converged: the update kernels then change nothing
  int32_t iters;    // PCG steps taken
};

// Workgroup count of the partial-sum kernels for vectors of length len.
int partial_blocks(int64_t len);

// y = A* x = inv_nu (C_9 (x) M_1) x + dt A_div x, tensor vectors.
hipError_t launch_astar3(int n, const double* Cd, const double* Me, double inv_nu, double dt,
                         const double* x, double* y, hipStream_t st);
// q = w - dt A_div Z yh (Z = V of eq. (Vmatrix), d = 3); yh a scalar vector.
hipError_t launch_adivz3(int n, const double* Cd, double dt, const double* w, const double* yh,
                         double* q, hipStream_t st);
// s = Z^T w.
hipError_t launch_zt3(int64_t ne, const double* w, double* s, hipStream_t st);
// x += a Z y.
hipError_t launch_zaxpy3(int64_t ne, double a, const double* y, double* x, hipStream_t st);
// q = scale Ld p (scalar vectors) and per-workgroup partials of (p, q).
hipError_t launch_lap3(int n, const double* Ld, double scale, const double* p, double* q,
                       double* part, hipStream_t st);
// PCG set-up: r = s, x = 0, z = Dinv r, p = z, rho = (r, z), rr = (r, r),
// thresh2 = rel2 * rr, active = rr > thresh2 (two launches plus the final sums).
hipError_t launch_pcg_start(int64_t ne, const double* Dinv, const double* s, double* x, double* r,
                            double* z, double* p, double* part, PcgScalars* sc, double rel2,
                            hipStream_t st);
// One PCG step after q = E p and its partials: alpha, x += alpha p,
// r -= alpha q, z = Dinv r, rho, rr, beta, p = z + beta p.
hipError_t launch_pcg_step(int64_t ne, const double* Dinv, double* x, double* r, double* z,
                           double* p, const double* q, double* part, double* part2, int nblk_q,
                           PcgScalars* sc, hipStream_t st);
// Exact inner solve out = scale V diag(1 / (lx_i + ly_j + ly_k)) V^T in by fast
// diagonalisation (V = Vy (x) Vy (x) Vx on the tensor index (Iz, Iy, Ix);
// the y and z axes share one factor), in six axis passes through the
// scalar buffers t1, t2; Vd row-major [j][i] = (V_d)_{j i}, VdT its
// transpose.  Needs 2 n <= 256.
hipError_t launch_fdm_solve(int n, const double* Vx, const double* VxT, const double* Vy,
                            const double* VyT, const double* lx, const double* ly, double scale,
                            const double* in, double* out, double* t1, double* t2, hipStream_t st);
// out[0] = sum_i x_i y_i (fixed summation order).
hipError_t launch_dot(int64_t len, const double* x, const double* y, double* part, double* out,
                      hipStream_t st);
// y += a x; y = x + b y.
hipError_t launch_axpy(int64_t len, double a, const double* x, double* y, hipStream_t st);
hipError_t launch_xpby(int64_t len, const double* x, double b, double* y, hipStream_t st);
hipError_t launch_fill(int64_t len, double v, double* x, hipStream_t st);

}  // namespace dcg3
