// Device side of the exact inner solve by fast diagonalisation (2D path):
// z = L^{-1} s = V' diag(1 / (lam_y + lam_x)) V'^T s with V' = V (x) V on the
// tensor index (Iy, Ix), applied as four dense N x N products (N = 2 n):
//   T1 = S V,  T2 = (V^T T1) ./ (lam_i + lam_k),  T3 = V T2,  Z = T3 V^T,
// with S, Z the scalar vectors rearranged from the element-major layout
// 4 e + j (e = ey n + ex, j = ix + 2 iy) to the row-major tensor (Iy, Ix),
// Ix = 2 ex + ix.  The products are FP64 register-blocked GEMMs staged
// through LDS (each thread forms a 2 x 2 or 4 x 4 block of C).  The
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
  // to N = 1024; 64 x 64 (4 x 4 per thread) above
  if (N <= 1024) {
    const dim3 grid((N + 31) / 32, (N + 31) / 32);
    k_gemm<32, 16><<<grid, kGThreads, 0, st>>>(N, A, B, C, la, lb);
  } else {
    const dim3 grid((N + 63) / 64, (N + 63) / 64);
    k_gemm<64, 16><<<grid, kGThreads, 0, st>>>(N, A, B, C, la, lb);
  }
  return hipGetLastError();
}

// Small grids (N = 2 n in {32, 64, 128, 256}: coarse levels) in two passes
// with the layout change folded into the loads and stores, one workgroup per
// row:
//   pass 1: T2[i][k] = (sum_a sum_c V[a][i] S[a][c] V[c][k]) / (lam_i + lam_k),
//           row i of U = V^T S, then of U V;
//   pass 2: Z[a][c] = sum_i sum_k V[a][i] T2[i][k] V[c][k],
//           row a of W = V T2, then of W V^T.
// Thread t forms a partial sum for column t % N over the contraction range
// [p N / P, (p + 1) N / P), p = t / N, P = 256 / N; the P partials of a
// column are added in LDS in ascending p (fixed order).
constexpr int kFThreads = 256;

__device__ __forceinline__ int64_t tensor_to_elem(int n, int a, int c) {
  return 4 * ((int64_t)(a >> 1) * n + (c >> 1)) + (c & 1) + 2 * (a & 1);
}

// sum over p of part[p N + c] for the threads t < N (column c = t)
__device__ __forceinline__ double column_total(const double* part, int N, int P, int c) {
  double t = 0.0;
  for (int p = 0; p < P; ++p) t += part[p * N + c];
  return t;
}

template <typename T>
__global__ __launch_bounds__(kFThreads) void k_fdm_pass1(int n, const double* __restrict__ V,
                                                         const double* __restrict__ VT,
                                                         const double* __restrict__ lam,
                                                         const T* __restrict__ s, double* __restrict__ T2) {
  __shared__ double lhs[kFThreads];
  __shared__ double mid[kFThreads];
  __shared__ double part[kFThreads];
  const int N = 2 * n, P = kFThreads / N, len = N / P;
  const int tid = threadIdx.x, c = tid % N, q0 = (tid / N) * len;
  const int i = blockIdx.x;
  if (tid < N) lhs[tid] = VT[(int64_t)i * N + tid];     // row i of V^T
  __syncthreads();
  // rows a, a + 1 (a even) of column c sit at sc[0] and sc[2] of the square
  // row a / 2; consecutive square rows are 4 n apart
  const T* sc = s + tensor_to_elem(n, q0, c);
  const int64_t step = 4 * (int64_t)n;
  double u = 0.0;
#pragma unroll 8
  for (int a = q0; a < q0 + len; a += 2, sc += step)
    u += lhs[a] * double(sc[0]) + lhs[a + 1] * double(sc[2]);
  part[tid] = u;
  __syncthreads();
  if (tid < N) mid[tid] = column_total(part, N, P, tid);   // U[i][c]
  __syncthreads();
  double t = 0.0;
#pragma unroll 16
  for (int q = q0; q < q0 + len; ++q) t += mid[q] * V[(int64_t)q * N + c];
  part[tid] = t;
  __syncthreads();
  if (tid < N) T2[(int64_t)i * N + tid] = column_total(part, N, P, tid) * (1.0 / (lam[i] + lam[tid]));
}

template <typename T>
__global__ __launch_bounds__(kFThreads) void k_fdm_pass2(int n, const double* __restrict__ V,
                                                         const double* __restrict__ VT,
                                                         const double* __restrict__ T2, T* __restrict__ z) {
  __shared__ double lhs[kFThreads];
  __shared__ double mid[kFThreads];
  __shared__ double part[kFThreads];
  const int N = 2 * n, P = kFThreads / N, len = N / P;
  const int tid = threadIdx.x, c = tid % N, q0 = (tid / N) * len;
  const int a = blockIdx.x;
  if (tid < N) lhs[tid] = V[(int64_t)a * N + tid];      // row a of V
  __syncthreads();
  double w = 0.0;
#pragma unroll 16
  for (int i = q0; i < q0 + len; ++i) w += lhs[i] * T2[(int64_t)i * N + c];
  part[tid] = w;
  __syncthreads();
  if (tid < N) mid[tid] = column_total(part, N, P, tid);   // W[a][c]
  __syncthreads();
  double v = 0.0;
#pragma unroll 16
  for (int k = q0; k < q0 + len; ++k) v += mid[k] * VT[(int64_t)k * N + c];
  part[tid] = v;
  __syncthreads();
  if (tid < N) z[tensor_to_elem(n, a, tid)] = T(column_total(part, N, P, tid));
}

template <typename T>
hipError_t fdm_solve(int n, const double* V, const double* VT, const double* lam, const T* s, T* z,
                     double* t0, double* t1, double* t2, hipStream_t st) {
  const int N = 2 * n;
  if (N >= 32 && N <= kFThreads && kFThreads % N == 0) {
    k_fdm_pass1<T><<<N, kFThreads, 0, st>>>(n, V, VT, lam, s, t0);
    k_fdm_pass2<T><<<N, kFThreads, 0, st>>>(n, V, VT, t0, z);
    return hipGetLastError();
  }
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
