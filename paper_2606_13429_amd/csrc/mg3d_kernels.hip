// Kernels of the three-dimensional multigrid inner solve (Section 4.2, the 3D
// case; layouts in mg3d.hpp).  Level vectors hold 8 FP64 values per cube.
// The residual and the RAS step run on bricks staged in LDS on large levels
// and split every output over a few lanes on small ones; the transfers run
// one thread per (cube, row).  The class tables (operator
// 27 x 7 blocks, RAS updates 343 x 8 x 200) are shared by every cube of a
// class and stay in the caches.
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

// ---- residual and RAS step on large levels (n_k > kSplitMaxN): bricks of
// 4 x 4 x 4 cubes per 512-thread workgroup.  The workgroup stages the input
// vector on the brick and a halo (zeros outside the domain) in LDS,
// component-major with a padded stride; thread t computes row t & 7 of cube
// t >> 3 of the brick.  These levels store the class tables with the row
// index fastest (mg3d.hpp), so the eight threads of a cube read one
// contiguous 64-byte segment per column and the cubes of one class in a
// wavefront share it.
constexpr int kBrick = 4;
constexpr int kBrickThreads = 512;

template <int H>
struct Box {
  static constexpr int X = kBrick + 2 * H;
  static constexpr int N = X * X * X;
  static constexpr int S = N + 1;   // component stride (padding spreads the banks)
};

__host__ __device__ constexpr int bricks_along(int n) { return (n + kBrick - 1) / kBrick; }

// lds[b S + c] = v on box cube c, component b (0 outside the domain or v = NULL).
template <int H>
__device__ __forceinline__ void stage_box(int n, int x0, int y0, int z0, const double* __restrict__ v,
                                          double* lds) {
  using B = Box<H>;
  for (int i = threadIdx.x; i < B::N * 8; i += kBrickThreads) {
    const int c = i >> 3, b = i & 7;
    const int x = x0 - H + c % B::X, y = y0 - H + (c / B::X) % B::X, z = z0 - H + c / (B::X * B::X);
    double val = 0.0;
    if (v && x >= 0 && y >= 0 && z >= 0 && x < n && y < n && z < n)
      val = v[8 * (((int64_t)z * n + y) * n + x) + b];
    lds[b * B::S + c] = val;
  }
}

struct Lane {
  int row;        // the thread's row of its cube
  int x, y, z;    // the cube
  int lx, ly, lz; // its place in the brick
  int x0, y0, z0; // the brick's origin
  bool valid;     // inside the domain
  int64_t e;
};

__device__ __forceinline__ Lane lane_cube(int n) {
  const int nb = bricks_along(n);
  const int b = blockIdx.x;
  Lane L;
  L.row = threadIdx.x & 7;
  const int c = threadIdx.x >> 3;
  L.lx = c & 3;
  L.ly = (c >> 2) & 3;
  L.lz = c >> 4;
  L.x0 = (b % nb) * kBrick;
  L.y0 = ((b / nb) % nb) * kBrick;
  L.z0 = (b / (nb * nb)) * kBrick;
  L.x = L.x0 + L.lx;
  L.y = L.y0 + L.ly;
  L.z = L.z0 + L.lz;
  L.valid = L.x < n && L.y < n && L.z < n;
  L.e = ((int64_t)L.z * n + L.y) * n + L.x;
  return L;
}

__global__ __launch_bounds__(kBrickThreads) void k_mg3_res(int n, const double* __restrict__ opT,
                                                           const double* __restrict__ f,
                                                           const double* __restrict__ z,
                                                           double* __restrict__ r,
                                                           double* __restrict__ part,
                                                           const int32_t* __restrict__ guard) {
  if (stopped(guard)) return;
  using B = Box<1>;
  __shared__ double zs[8 * B::S];
  __shared__ double sh[kBrickThreads / 64];
  const Lane L = lane_cube(n);
  stage_box<1>(n, L.x0, L.y0, L.z0, z, zs);
  __syncthreads();
  constexpr int off[kSlots] = {0, -1, 1, -B::X, B::X, -B::X * B::X, B::X * B::X};
  const int cls = op_axis(L.x, n) + 3 * op_axis(L.y, n) + 9 * op_axis(L.z, n);
  // opT[cls][slot][b][row]
  const double* col = opT + (int64_t)cls * kSlots * 64 + L.row;
  const int o = ((L.lz + 1) * B::X + L.ly + 1) * B::X + L.lx + 1;
  double acc = (L.valid && f) ? f[8 * L.e + L.row] : 0.0;
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    const double* cs = col + 64 * s;
    const double* zn = zs + o + off[s];
#pragma unroll
    for (int b = 0; b < 8; ++b) acc -= cs[8 * b] * zn[b * B::S];
  }
  if (L.valid) r[8 * L.e + L.row] = acc;
  if (part) {   // the workgroup's sum of r^2, fixed order: lanes, then wavefronts
    double v = L.valid ? acc * acc : 0.0;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sum = 0.0;
      for (int w = 0; w < kBrickThreads / 64; ++w) sum += sh[w];
      part[blockIdx.x] = sum;
    }
  }
}

// The diamond (|dx| + |dy| + |dz| <= 2) as cube offsets, in the order of
// diamond_offsets().
struct DiamondOff {
  int d[kDiamond][3];
  constexpr DiamondOff() : d() {
    int k = 0;
    for (int dz = -2; dz <= 2; ++dz)
      for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) {
          const int a = (dx < 0 ? -dx : dx) + (dy < 0 ? -dy : dy) + (dz < 0 ? -dz : dz);
          if (a <= 2) {
            d[k][0] = dx;
            d[k][1] = dy;
            d[k][2] = dz;
            ++k;
          }
        }
  }
};

// The diamond as offsets in the halo-2 box, in the same order.
struct DiamondBox {
  int o[kDiamond];
  constexpr DiamondBox() : o() {
    const DiamondOff D;
    for (int d = 0; d < kDiamond; ++d) o[d] = (D.d[d][2] * Box<2>::X + D.d[d][1]) * Box<2>::X + D.d[d][0];
  }
};

__global__ __launch_bounds__(kBrickThreads) void k_mg3_ras(int n, const double* __restrict__ rasT,
                                                           const double* __restrict__ r,
                                                           double* __restrict__ z, int zero,
                                                           const int32_t* __restrict__ guard) {
  if (stopped(guard)) return;
  using B = Box<2>;
  __shared__ double rs[8 * B::S];
  const Lane L = lane_cube(n);
  stage_box<2>(n, L.x0, L.y0, L.z0, r, rs);
  __syncthreads();
  constexpr DiamondBox D;
  const int cls = ras_axis(L.x, n) + 7 * ras_axis(L.y, n) + 49 * ras_axis(L.z, n);
  // rasT[cls][column 200][row]
  const double* col = rasT + (int64_t)cls * 8 * kRasCols + L.row;
  const int o = ((L.lz + 2) * B::X + L.ly + 2) * B::X + L.lx + 2;
  double acc = (L.valid && !zero) ? z[8 * L.e + L.row] : 0.0;
  // five diamond cubes per loop trip keep the code small with their table
  // loads in flight together
#pragma unroll 5
  for (int d = 0; d < kDiamond; ++d) {
    const double* cd = col + 64 * d;
    const double* rd = rs + o + D.o[d];
#pragma unroll
    for (int b = 0; b < 8; ++b) acc += cd[8 * b] * rd[b * B::S];
  }
  if (L.valid) z[8 * L.e + L.row] = acc;
}

// ---- residual and RAS step on small levels (n_k <= kSplitMaxN): one lane
// per (cube, row, term group), so that every lane issues a single round of
// loads -- the table row segment and the neighbour's values, 64 bytes each
// -- and the groups are summed by a fixed shuffle tree.  These levels use
// the row-major tables.
// RAS: 32 lanes per output (lane d < 25 takes diamond cube d), 8 outputs per
// 256-thread workgroup.
__global__ __launch_bounds__(kThreads) void k_mg3_ras_split(int n, const double* __restrict__ ras,
                                                            const double* __restrict__ r,
                                                            double* __restrict__ z, int zero,
                                                            const int32_t* __restrict__ guard) {
  if (stopped(guard)) return;
  constexpr DiamondOff D;
  const int64_t ne = (int64_t)n * n * n;
  const int64_t out = (int64_t)blockIdx.x * (kThreads / 32) + (threadIdx.x >> 5);
  const int d = threadIdx.x & 31;
  const int64_t e = out >> 3;
  const int row = int(out & 7);
  double acc = 0.0;
  if (e < ne && d < kDiamond) {
    const int x = int(e % n), y = int((e / n) % n), zz = int(e / ((int64_t)n * n));
    const int qx = x + D.d[d][0], qy = y + D.d[d][1], qz = zz + D.d[d][2];
    if (qx >= 0 && qy >= 0 && qz >= 0 && qx < n && qy < n && qz < n) {
      const int cls = n < kRasClassMinN ? int(e) : ras_axis(x, n) + 7 * ras_axis(y, n) + 49 * ras_axis(zz, n);
      const double* K = ras + ((int64_t)cls * 8 + row) * kRasCols + 8 * d;
      const double* rn = r + 8 * (((int64_t)qz * n + qy) * n + qx);
#pragma unroll
      for (int b = 0; b < 8; ++b) acc += K[b] * rn[b];
    }
  }
#pragma unroll
  for (int m = 16; m > 0; m >>= 1) acc += __shfl_xor(acc, m, 32);
  if (d == 0 && e < ne) z[8 * e + row] = (zero ? 0.0 : z[8 * e + row]) + acc;
}

// Residual: 8 lanes per output (lane s < 7 takes face slot s), 32 outputs per
// 256-thread workgroup; with part, the workgroup's sum of r^2.
__global__ __launch_bounds__(kThreads) void k_mg3_res_split(int n, const double* __restrict__ op,
                                                            const double* __restrict__ f,
                                                            const double* __restrict__ z,
                                                            double* __restrict__ r,
                                                            double* __restrict__ part,
                                                            const int32_t* __restrict__ guard) {
  if (stopped(guard)) return;
  __shared__ double sh[kThreads / 64];
  const int64_t ne = (int64_t)n * n * n;
  const int64_t out = (int64_t)blockIdx.x * (kThreads / 8) + (threadIdx.x >> 3);
  const int s = threadIdx.x & 7;
  const int64_t e = out >> 3;
  const int row = int(out & 7);
  double acc = 0.0;
  if (e < ne && s < kSlots && z) {
    const int c[3] = {int(e % n), int((e / n) % n), int(e / ((int64_t)n * n))};
    const int ax = s == 0 ? 0 : (s - 1) >> 1;
    const int dir = s == 0 ? 0 : ((s & 1) ? -1 : 1);
    const int q = c[ax] + dir;
    if (q >= 0 && q < n) {
      const int cls = op_axis(c[0], n) + 3 * op_axis(c[1], n) + 9 * op_axis(c[2], n);
      const int64_t nb = e + dir * (ax == 0 ? 1 : (ax == 1 ? (int64_t)n : (int64_t)n * n));
      const double* row_p = op + ((cls * kSlots + s) * 8 + row) * 8;
      const double* zn = z + 8 * nb;
#pragma unroll
      for (int b = 0; b < 8; ++b) acc -= row_p[b] * zn[b];
    }
  }
#pragma unroll
  for (int m = 4; m > 0; m >>= 1) acc += __shfl_xor(acc, m, 8);
  double v = 0.0;
  if (s == 0 && e < ne) {
    acc += f ? f[8 * e + row] : 0.0;
    r[8 * e + row] = acc;
    v = acc * acc;
  }
  if (part) {   // the workgroup's sum of r^2, fixed order: lanes, then wavefronts
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sum = 0.0;
      for (int w = 0; w < kThreads / 64; ++w) sum += sh[w];
      part[blockIdx.x] = sum;
    }
  }
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

unsigned brick_blocks(int n) { return unsigned(bricks_along(n) * bricks_along(n) * bricks_along(n)); }

}  // namespace

bool mg3_split(int nk) { return nk <= kSplitMaxN; }

int mg3_res_blocks(int nk) {
  return mg3_split(nk) ? int((8 * (int64_t)nk * nk * nk + kThreads / 8 - 1) / (kThreads / 8))
                       : int(brick_blocks(nk));
}

hipError_t launch_mg3_res(int nk, const double* op, const double* f, const double* z, double* r,
                          double* part, const int32_t* guard, hipStream_t st) {
  if (mg3_split(nk))
    hipLaunchKernelGGL(k_mg3_res_split, dim3(mg3_res_blocks(nk)), dim3(kThreads), 0, st, nk, op, f, z,
                       r, part, guard);
  else
    hipLaunchKernelGGL(k_mg3_res, dim3(mg3_res_blocks(nk)), dim3(kBrickThreads), 0, st, nk, op, f, z, r,
                       part, guard);
  return hipGetLastError();
}

hipError_t launch_mg3_ras(int nk, const double* ras, const double* r, double* z, bool zero,
                          const int32_t* guard, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (mg3_split(nk)) {
    const int64_t outs = 8 * (int64_t)nk * nk * nk;
    hipExtLaunchKernelGGL(k_mg3_ras_split, dim3(unsigned((outs + kThreads / 32 - 1) / (kThreads / 32))),
                          dim3(kThreads), 0, st, ev0, ev1, 0, nk, ras, r, z, int(zero), guard);
  } else {
    hipExtLaunchKernelGGL(k_mg3_ras, dim3(brick_blocks(nk)), dim3(kBrickThreads), 0, st, ev0, ev1, 0, nk,
                          ras, r, z, int(zero), guard);
  }
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
