// Kernels of the three-dimensional multigrid inner solve (Section 4.2, the 3D
// case; layouts in mg3d.hpp).  Level vectors hold 8 FP64 values per cube.
// One thread per (cube, row): 32 cubes per 256-thread workgroup, the eight
// threads of a cube read its neighbours' values together.  The class tables
// (operator 27 x 7 blocks, RAS updates 343 x 8 x 200) are shared by every
// cube of a class and stay in the caches.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "dcg3d.hpp"
#include "mg3d.hpp"

namespace dcg3 {

namespace {

constexpr int kThreads = 256;
constexpr int kCubesPerBlock = kThreads / 8;

__device__ __forceinline__ int op_axis(int x, int n) { return x == 0 ? 0 : (x == n - 1 ? 2 : 1); }
__device__ __forceinline__ int ras_axis(int x, int n) {
  return x < 3 ? x : (n - 1 - x < 3 ? 6 - (n - 1 - x) : 3);
}

__device__ __forceinline__ bool stopped(const int32_t* guard) { return guard && *guard == 0; }

// Sum over the workgroup in a fixed order; valid in thread 0.
__device__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

__global__ __launch_bounds__(kThreads) void k_mg3_res(int n, const double* __restrict__ op,
                                                      const double* __restrict__ f,
                                                      const double* __restrict__ z,
                                                      double* __restrict__ r,
                                                      double* __restrict__ part,
                                                      const int32_t* __restrict__ guard) {
  if (stopped(guard)) return;
  __shared__ double sh[kThreads];
  const int64_t ne = (int64_t)n * n * n;
  const int64_t e = (int64_t)blockIdx.x * kCubesPerBlock + threadIdx.x / 8;
  const int a = threadIdx.x & 7;
  double v = 0.0;
  if (e < ne) {
    const int x = int(e % n), y = int((e / n) % n), zz = int(e / ((int64_t)n * n));
    const int cls = op_axis(x, n) + 3 * op_axis(y, n) + 9 * op_axis(zz, n);
    const int c[3] = {x, y, zz};
    double acc = f ? f[8 * e + a] : 0.0;
    if (z) {
#pragma unroll
      for (int s = 0; s < kSlots; ++s) {
        const int ax = s == 0 ? 0 : (s - 1) >> 1;
        const int dir = s == 0 ? 0 : ((s & 1) ? -1 : 1);
        const int q = c[ax] + dir;
        if (q < 0 || q >= n) continue;
        int64_t nb = e;
        if (s) nb += dir * (ax == 0 ? 1 : (ax == 1 ? (int64_t)n : (int64_t)n * n));
        const double* row = op + ((cls * kSlots + s) * 8 + a) * 8;
        const double* zn = z + 8 * nb;
#pragma unroll
        for (int b = 0; b < 8; ++b) acc -= row[b] * zn[b];
      }
    }
    r[8 * e + a] = acc;
    v = acc * acc;
  }
  if (part) {
    const double s = block_sum(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
  }
}

struct DiamondTable {
  int8_t d[kDiamond][3];
};

__global__ __launch_bounds__(kThreads) void k_mg3_ras(int n, const double* __restrict__ ras,
                                                      const double* __restrict__ r,
                                                      double* __restrict__ z, int zero,
                                                      DiamondTable dt,
                                                      const int32_t* __restrict__ guard) {
  if (stopped(guard)) return;
  const int64_t ne = (int64_t)n * n * n;
  const int64_t e = (int64_t)blockIdx.x * kCubesPerBlock + threadIdx.x / 8;
  const int a = threadIdx.x & 7;
  if (e >= ne) return;
  const int x = int(e % n), y = int((e / n) % n), zz = int(e / ((int64_t)n * n));
  const int cls = n < kRasClassMinN ? int(e) : ras_axis(x, n) + 7 * ras_axis(y, n) + 49 * ras_axis(zz, n);
  const double* K = ras + ((int64_t)cls * 8 + a) * kRasCols;
  double acc = zero ? 0.0 : z[8 * e + a];
#pragma unroll 5
  for (int d = 0; d < kDiamond; ++d) {
    const int qx = x + dt.d[d][0], qy = y + dt.d[d][1], qz = zz + dt.d[d][2];
    if (qx < 0 || qy < 0 || qz < 0 || qx >= n || qy >= n || qz >= n) continue;
    const double* rn = r + 8 * (((int64_t)qz * n + qy) * n + qx);
    const double* k = K + 8 * d;
#pragma unroll
    for (int b = 0; b < 8; ++b) acc += k[b] * rn[b];
  }
  z[8 * e + a] = acc;
}

__device__ __forceinline__ double inject(int q, int i, int J) {
  double v = 1.0;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const double t = 0.5 * (((q >> ax) & 1) + ((i >> ax) & 1));
    v *= ((J >> ax) & 1) ? t : 1.0 - t;
  }
  return v;
}

__global__ __launch_bounds__(kThreads) void k_mg3_restrict(int nf, const double* __restrict__ r,
                                                           double* __restrict__ fc,
                                                           const int32_t* __restrict__ guard) {
  if (stopped(guard)) return;
  const int nc = nf / 2;
  const int64_t nec = (int64_t)nc * nc * nc;
  const int64_t E = (int64_t)blockIdx.x * kCubesPerBlock + threadIdx.x / 8;
  const int J = threadIdx.x & 7;
  if (E >= nec) return;
  const int X = int(E % nc), Y = int((E / nc) % nc), Z = int(E / ((int64_t)nc * nc));
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int64_t c = ((int64_t)(2 * Z + (q >> 2)) * nf + 2 * Y + ((q >> 1) & 1)) * nf + 2 * X + (q & 1);
    const double* rc = r + 8 * c;
#pragma unroll
    for (int i = 0; i < 8; ++i) acc += inject(q, i, J) * rc[i];
  }
  fc[8 * E + J] = acc;
}

__global__ __launch_bounds__(kThreads) void k_mg3_prolong(int nf, const double* __restrict__ zc,
                                                          double* __restrict__ z, int assign,
                                                          const int32_t* __restrict__ guard) {
  if (stopped(guard)) return;
  const int nc = nf / 2;
  const int64_t ne = (int64_t)nf * nf * nf;
  const int64_t e = (int64_t)blockIdx.x * kCubesPerBlock + threadIdx.x / 8;
  const int i = threadIdx.x & 7;
  if (e >= ne) return;
  const int x = int(e % nf), y = int((e / nf) % nf), zz = int(e / ((int64_t)nf * nf));
  const int q = (x & 1) | ((y & 1) << 1) | ((zz & 1) << 2);
  const double* zE = zc + 8 * (((int64_t)(zz >> 1) * nc + (y >> 1)) * nc + (x >> 1));
  double acc = 0.0;
#pragma unroll
  for (int J = 0; J < 8; ++J) acc += inject(q, i, J) * zE[J];
  z[8 * e + i] = assign ? acc : z[8 * e + i] + acc;
}

__global__ __launch_bounds__(kThreads) void k_mg3_dense(int m, const double* __restrict__ inv,
                                                        const double* __restrict__ f,
                                                        double* __restrict__ z,
                                                        const int32_t* __restrict__ guard) {
  if (stopped(guard)) return;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= m) return;
  const double* row = inv + (int64_t)i * m;
  double acc = 0.0;
  for (int j = 0; j < m; ++j) acc += row[j] * f[j];
  z[i] = acc;
}

__global__ __launch_bounds__(kThreads) void k_mg3_start(int64_t len, double* __restrict__ z,
                                                        Mg3Scalars* sc, double rel2, int max_iters) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * kThreads)
    z[i] = 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->rel2 = rel2;
    sc->thresh2 = 0.0;
    sc->rr = 0.0;
    sc->active = 1;
    sc->first = 1;
    sc->iters = 0;
    sc->max_iters = max_iters;
  }
}

__global__ __launch_bounds__(kThreads) void k_mg3_test(int nparts, const double* __restrict__ part,
                                                       Mg3Scalars* sc) {
  if (sc->active == 0) return;
  __shared__ double sh[kThreads];
  double v = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kThreads) v += part[i];
  const double rr = block_sum(v, sh);
  if (threadIdx.x == 0) {
    if (sc->first) {
      sc->thresh2 = sc->rel2 * rr;
      sc->first = 0;
    }
    sc->rr = rr;
    if (!(rr > sc->thresh2) || sc->iters >= sc->max_iters)
      sc->active = 0;
    else
      sc->iters += 1;
  }
}

__global__ __launch_bounds__(kThreads) void k_mg3_scale(int64_t len, double a,
                                                        const double* __restrict__ x,
                                                        double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < len) y[i] = a * x[i];
}

unsigned cube_blocks(int64_t cubes) { return unsigned((cubes + kCubesPerBlock - 1) / kCubesPerBlock); }

DiamondTable make_diamond() {
  int off[kDiamond][3];
  diamond_offsets(off);
  DiamondTable t;
  for (int d = 0; d < kDiamond; ++d)
    for (int c = 0; c < 3; ++c) t.d[d][c] = int8_t(off[d][c]);
  return t;
}

}  // namespace

int mg3_res_blocks(int nk) { return int(cube_blocks((int64_t)nk * nk * nk)); }

hipError_t launch_mg3_res(int nk, const double* op, const double* f, const double* z, double* r,
                          double* part, const int32_t* guard, hipStream_t st) {
  hipLaunchKernelGGL(k_mg3_res, dim3(mg3_res_blocks(nk)), dim3(kThreads), 0, st, nk, op, f, z, r,
                     part, guard);
  return hipGetLastError();
}

hipError_t launch_mg3_ras(int nk, const double* ras, const double* r, double* z, bool zero,
                          const int32_t* guard, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  static const DiamondTable dt = make_diamond();
  hipExtLaunchKernelGGL(k_mg3_ras, dim3(cube_blocks((int64_t)nk * nk * nk)), dim3(kThreads), 0, st,
                        ev0, ev1, 0, nk, ras, r, z, int(zero), dt, guard);
  return hipGetLastError();
}

hipError_t launch_mg3_restrict(int nf, const double* r, double* fc, const int32_t* guard,
                               hipStream_t st) {
  const int nc = nf / 2;
  hipLaunchKernelGGL(k_mg3_restrict, dim3(cube_blocks((int64_t)nc * nc * nc)), dim3(kThreads), 0, st,
                     nf, r, fc, guard);
  return hipGetLastError();
}

hipError_t launch_mg3_prolong(int nf, const double* zc, double* z, bool assign,
                              const int32_t* guard, hipStream_t st) {
  hipLaunchKernelGGL(k_mg3_prolong, dim3(cube_blocks((int64_t)nf * nf * nf)), dim3(kThreads), 0, st,
                     nf, zc, z, int(assign), guard);
  return hipGetLastError();
}

hipError_t launch_mg3_dense(int m, const double* inv, const double* f, double* z,
                            const int32_t* guard, hipStream_t st) {
  hipLaunchKernelGGL(k_mg3_dense, dim3((m + kThreads - 1) / kThreads), dim3(kThreads), 0, st, m, inv,
                     f, z, guard);
  return hipGetLastError();
}

hipError_t launch_mg3_start(int64_t len, double* z, Mg3Scalars* sc, double rel2, int max_iters,
                            hipStream_t st) {
  const int64_t want = (len + kThreads - 1) / kThreads;
  const unsigned blocks = unsigned(want < 1 ? 1 : (want > 1024 ? 1024 : want));
  hipLaunchKernelGGL(k_mg3_start, dim3(blocks), dim3(kThreads), 0, st, len, z, sc, rel2, max_iters);
  return hipGetLastError();
}

hipError_t launch_mg3_test(int nparts, const double* part, Mg3Scalars* sc, hipStream_t st) {
  hipLaunchKernelGGL(k_mg3_test, dim3(1), dim3(kThreads), 0, st, nparts, part, sc);
  return hipGetLastError();
}

hipError_t launch_mg3_scale(int64_t len, double a, const double* x, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_mg3_scale, dim3(unsigned((len + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                     st, len, a, x, y);
  return hipGetLastError();
}

}  // namespace dcg3
