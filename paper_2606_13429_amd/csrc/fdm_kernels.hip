// Device side of the exact inner solve by fast diagonalisation (2D path):
// z = L^{-1} s = V' diag(1 / (lam_y + lam_x)) V'^T s with V' = V (x) V on the
// tensor index (Iy, Ix), applied as four dense N x N products (N = 2 n):
//   T1 = S V,  T2 = (V^T T1) ./ (lam_i + lam_k),  T3 = V T2,  Z = T3 V^T,
// with S, Z the scalar vectors rearranged from the element-major layout
// 4 e + j (e = ey n + ex, j = ix + 2 iy) to the row-major tensor (Iy, Ix),
// Ix = 2 ex + ix.  The products are FP64 register-blocked GEMMs staged
// through LDS (each thread forms a 1 x 1, 2 x 2 or 4 x 4 block of C).  The
// same solve serves as the exact coarsest-level solve of a shortened
// multigrid hierarchy, whose level vectors may be FP32.
#include <cstdint>

#include "kernels.hpp"

namespace dcg {
namespace {

template <int TILE, int KK>
struct GemmCfg {
  static constexpr int kT = TILE;                   // C tile per workgroup
  static constexpr int kK = KK;                     // k step
  static constexpr int kR = TILE / 16;              // outputs per thread along each axis
};
constexpr int kGThreads = 256;

// C = A B (N x N row-major); with la: C[i][k] *= 1 / (la[i] + lb[k]).  A
// 16 x 16 grid of threads, each forming a kR x kR block of the TILE x TILE tile.
template <int TILE, int KK>
__global__ __launch_bounds__(kGThreads) void k_gemm(int N, const double* __restrict__ A,
                                                    const double* __restrict__ B, double* __restrict__ C,
                                                    const double* __restrict__ la,
                                                    const double* __restrict__ lb) {
  using G = GemmCfg<TILE, KK>;
  __shared__ double As[G::kK][G::kT + 2];   // A tile transposed: As[k][row]
  __shared__ double Bs[G::kK][G::kT + 2];
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  const int row0 = blockIdx.y * G::kT, col0 = blockIdx.x * G::kT;
  double acc[G::kR][G::kR] = {};
  for (int k0 = 0; k0 < N; k0 += G::kK) {
    for (int t = tid; t < G::kT * G::kK; t += kGThreads) {
      const int r = t / G::kK, kk = t % G::kK;      // A: row r, column k0 + kk
      const int gr = row0 + r, gk = k0 + kk;
      As[kk][r] = (gr < N && gk < N) ? A[(int64_t)gr * N + gk] : 0.0;
      const int kb = t / G::kT, c = t % G::kT;      // B: row k0 + kb, column c
      const int gkb = k0 + kb, gc = col0 + c;
      Bs[kb][c] = (gkb < N && gc < N) ? B[(int64_t)gkb * N + gc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < G::kK; ++kk) {
      double a[G::kR], b[G::kR];
#pragma unroll
      for (int q = 0; q < G::kR; ++q) {
        a[q] = As[kk][ty * G::kR + q];
        b[q] = Bs[kk][tx * G::kR + q];
      }
#pragma unroll
      for (int i = 0; i < G::kR; ++i)
#pragma unroll
        for (int j = 0; j < G::kR; ++j) acc[i][j] += a[i] * b[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < G::kR; ++i) {
    const int gr = row0 + ty * G::kR + i;
    if (gr >= N) continue;
#pragma unroll
    for (int j = 0; j < G::kR; ++j) {
      const int gc = col0 + tx * G::kR + j;
      if (gc >= N) continue;
      double v = acc[i][j];
      if (la) v *= 1.0 / (la[gr] + lb[gc]);
      C[(int64_t)gr * N + gc] = v;
    }
  }
}

// to_tensor: T[(2 ey + iy) N + 2 ex + ix] = s[4 e + j]; otherwise the inverse.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(kGThreads) void k_fdm_permute(int n, int to_tensor,
                                                           const Tin* __restrict__ in,
                                                           Tout* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)kGThreads + threadIdx.x;
  const int64_t total = 4 * (int64_t)n * n;
  if (i >= total) return;
  const int N = 2 * n;
  const int64_t e = i >> 2;
  const int j = int(i & 3);
  const int ex = int(e % n), ey = int(e / n);
  const int64_t t = (int64_t)(2 * ey + (j >> 1)) * N + 2 * ex + (j & 1);
  if (to_tensor) out[t] = Tout(in[i]);
  else out[i] = Tout(in[t]);
}

hipError_t gemm(int N, const double* A, const double* B, double* C, const double* la,
                const double* lb, hipStream_t st) {
  // 32 x 32 tiles (2 x 2 per thread) keep at least about 4 workgroups per CU up
  // to N = 1024; 64 x 64 (4 x 4 per thread) above.  Small products (coarse
  // levels, N <= 256) are latency-bound: 16 x 16 tiles with 64-deep k steps
  // give more workgroups and fewer LDS round trips.
  if (N <= 256) {
    const dim3 grid((N + 15) / 16, (N + 15) / 16);
    k_gemm<16, 64><<<grid, kGThreads, 0, st>>>(N, A, B, C, la, lb);
  } else if (N <= 1024) {
    const dim3 grid((N + 31) / 32, (N + 31) / 32);
    k_gemm<32, 16><<<grid, kGThreads, 0, st>>>(N, A, B, C, la, lb);
  } else {
    const dim3 grid((N + 63) / 64, (N + 63) / 64);
    k_gemm<64, 16><<<grid, kGThreads, 0, st>>>(N, A, B, C, la, lb);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t fdm_solve(int n, const double* V, const double* VT, const double* lam, const T* s, T* z,
                     double* t0, double* t1, double* t2, hipStream_t st) {
  const int N = 2 * n;
  const int64_t total = 4 * (int64_t)n * n;
  const int pb = int((total + kGThreads - 1) / kGThreads);
  k_fdm_permute<T, double><<<pb, kGThreads, 0, st>>>(n, 1, s, t0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = gemm(N, t0, V, t1, nullptr, nullptr, st)) != hipSuccess) return e;   // x: S V
  if ((e = gemm(N, VT, t1, t2, lam, lam, st)) != hipSuccess) return e;          // y: V^T T1, scaled
  if ((e = gemm(N, V, t2, t0, nullptr, nullptr, st)) != hipSuccess) return e;   // y: V T2
  if ((e = gemm(N, t0, VT, t1, nullptr, nullptr, st)) != hipSuccess) return e;  // x: T3 V^T
  k_fdm_permute<double, T><<<pb, kGThreads, 0, st>>>(n, 0, t1, z);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fdm_solve2d(int n, const double* V, const double* VT, const double* lam,
                              const double* s, double* z, double* t0, double* t1, double* t2,
                              hipStream_t st) {
  return fdm_solve<double>(n, V, VT, lam, s, z, t0, t1, t2, st);
}

template <typename T>
hipError_t launch_fdm_coarse(int n, const double* V, const double* VT, const double* lam,
                             const T* f, T* z, double* t0, double* t1, double* t2, hipStream_t st) {
  return fdm_solve<T>(n, V, VT, lam, f, z, t0, t1, t2, st);
}

template hipError_t launch_fdm_coarse<float>(int, const double*, const double*, const double*,
                                             const float*, float*, double*, double*, double*,
                                             hipStream_t);
template hipError_t launch_fdm_coarse<double>(int, const double*, const double*, const double*,
                                              const double*, double*, double*, double*, double*,
                                              hipStream_t);

}  // namespace dcg
