// Kernels of the outer multigrid preconditioner (W-cycle on A*, layouts in
// omg.hpp).  Level vectors hold 16 FP64 values per square.
//
// The RAS step and the residual split every output (square, row) over a few
// lanes on levels of at most kOmgSplitMaxN squares per side (one lane per
// diamond square resp. face slot, one round of 128-byte loads each, a fixed
// shuffle sum), where a launch has few workgroups and its time is one
// thread's chain of loads.  Larger levels stage the input on 8 x 8 bricks in
// LDS: up to kOmgBrick1MaxN squares per side every wavefront computes one row
// of the brick's 64 squares with the table rows read per lane; above, every
// wavefront computes four rows with the table rows read at wave-uniform
// addresses through scalar loads (the fastest form measured at each size).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "host_setup.hpp"
#include "omg.hpp"

namespace dcg {

namespace {

constexpr int D = kOmgDofs;
constexpr int kThreads = 256;
constexpr int kOmgSplitMaxN = 64;
constexpr int kOmgBrick1MaxN = 256;

__device__ __forceinline__ int op_axis(int x, int n) { return x == 0 ? 0 : (x == n - 1 ? 2 : 1); }
__device__ __forceinline__ int ras_axis(int x, int n) {
  return x < 3 ? x : (n - 1 - x < 3 ? 6 - (n - 1 - x) : 3);
}
__device__ __forceinline__ int ras_class(int x, int y, int n) {
  return n < kOmgRasClassMinN ? y * n + x : ras_axis(x, n) + 7 * ras_axis(y, n);
}

// The 2D diamond (|dx| + |dy| <= 2), by dy then dx (omg_diamond).
struct Diamond2 {
  int d[kOmgDiamond][2];
  constexpr Diamond2() : d() {
    int k = 0;
    for (int dy = -2; dy <= 2; ++dy)
      for (int dx = -2; dx <= 2; ++dx)
        if ((dx < 0 ? -dx : dx) + (dy < 0 ? -dy : dy) <= 2) {
          d[k][0] = dx;
          d[k][1] = dy;
          ++k;
        }
  }
};

constexpr int kSlotOff[kSlots][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, -1}, {0, 1}};

// ---- small levels
// RAS: 16 lanes per output (lane d < 13 takes diamond square d), 16 outputs
// per workgroup.
__global__ __launch_bounds__(kThreads) void k_omg_ras_split(int n, const double* __restrict__ ras,
                                                            const double* __restrict__ r,
                                                            double* __restrict__ z, int zero) {
  constexpr Diamond2 DM;
  const int64_t ne = (int64_t)n * n;
  const int64_t out = (int64_t)blockIdx.x * (kThreads / 16) + (threadIdx.x >> 4);
  const int d = threadIdx.x & 15;
  const int64_t e = out / D;
  const int row = int(out % D);
  double acc = 0.0;
  if (e < ne && d < kOmgDiamond) {
    const int x = int(e % n), y = int(e / n);
    const int qx = x + DM.d[d][0], qy = y + DM.d[d][1];
    if (qx >= 0 && qy >= 0 && qx < n && qy < n) {
      const double* K = ras + ((int64_t)ras_class(x, y, n) * D + row) * kOmgRasCols + D * d;
      const double* rn = r + D * ((int64_t)qy * n + qx);
#pragma unroll
      for (int b = 0; b < D; ++b) acc += K[b] * rn[b];
    }
  }
#pragma unroll
  for (int m = 8; m > 0; m >>= 1) acc += __shfl_xor(acc, m, 16);
  if (d == 0 && e < ne) z[D * e + row] = (zero ? 0.0 : z[D * e + row]) + acc;
}

// Residual: 8 lanes per output (lane s < 5 takes face slot s), 32 outputs per
// workgroup.
__global__ __launch_bounds__(kThreads) void k_omg_res_split(int n, const double* __restrict__ op,
                                                            const double* __restrict__ f,
                                                            const double* __restrict__ z,
                                                            double* __restrict__ r) {
  const int64_t ne = (int64_t)n * n;
  const int64_t out = (int64_t)blockIdx.x * (kThreads / 8) + (threadIdx.x >> 3);
  const int s = threadIdx.x & 7;
  const int64_t e = out / D;
  const int row = int(out % D);
  double acc = 0.0;
  if (e < ne && s < kSlots) {
    const int x = int(e % n), y = int(e / n);
    const int qx = x + kSlotOff[s][0], qy = y + kSlotOff[s][1];
    if (qx >= 0 && qy >= 0 && qx < n && qy < n) {
      const int cls = op_axis(x, n) + 3 * op_axis(y, n);
      const double* A = op + ((cls * kSlots + s) * D + row) * D;
      const double* zn = z + D * ((int64_t)qy * n + qx);
#pragma unroll
      for (int b = 0; b < D; ++b) acc -= A[b] * zn[b];
    }
  }
#pragma unroll
  for (int m = 4; m > 0; m >>= 1) acc += __shfl_xor(acc, m, 8);
  if (s == 0 && e < ne) r[D * e + row] = (f ? f[D * e + row] : 0.0) + acc;
}

// ---- large levels (kOmgSplitMaxN < n_k <= kOmgBrick1MaxN): bricks of 8 x 8
// squares per 1024-thread workgroup, 16 wavefronts (one per row), the
// table rows read per lane
constexpr int kBrick = 8;
constexpr int kBrickThreads = 64 * D;

template <int H>
struct Box2 {
  static constexpr int X = kBrick + 2 * H;
  static constexpr int N = X * X;
  static constexpr int S = N + 1;   // component stride (padding spreads the banks)
};

template <int H>
__device__ __forceinline__ void stage_box(int n, int x0, int y0, const double* __restrict__ v,
                                          double* lds) {
  using B = Box2<H>;
  for (int i = threadIdx.x; i < B::N * D; i += blockDim.x) {
    const int c = i / D, b = i % D;
    const int x = x0 - H + c % B::X, y = y0 - H + c / B::X;
    double val = 0.0;
    if (x >= 0 && y >= 0 && x < n && y < n) val = v[D * ((int64_t)y * n + x) + b];
    lds[b * B::S + c] = val;
  }
}

using ConstPtr = const __attribute__((address_space(4))) double*;
__device__ __forceinline__ ConstPtr as_const(const double* p) { return (ConstPtr)p; }

struct BrickLane {
  int row, lx, ly, x, y, x0, y0;
  bool valid;
  int64_t e;
};

__device__ __forceinline__ BrickLane brick_lane(int n) {
  const int nb = (n + kBrick - 1) / kBrick;
  BrickLane L;
  L.x0 = (blockIdx.x % nb) * kBrick;
  L.y0 = (blockIdx.x / nb) * kBrick;
  L.row = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = threadIdx.x & 63;
  L.lx = c & 7;
  L.ly = c >> 3;
  L.x = L.x0 + L.lx;
  L.y = L.y0 + L.ly;
  L.valid = L.x < n && L.y < n;
  L.e = (int64_t)L.y * n + L.x;
  return L;
}

template <typename P>
__device__ __forceinline__ double ras_row(P K, const double* rs, int o, double acc) {
  using B = Box2<2>;
  constexpr Diamond2 DM;
#pragma unroll
  for (int d = 0; d < kOmgDiamond; ++d) {
    const int od = DM.d[d][1] * B::X + DM.d[d][0];
#pragma unroll
    for (int b = 0; b < D; ++b) acc += K[D * d + b] * rs[b * B::S + o + od];
  }
  return acc;
}

__global__ __launch_bounds__(kBrickThreads) void k_omg_ras(int n, const double* __restrict__ ras,
                                                           const double* __restrict__ r,
                                                           double* __restrict__ z, int zero) {
  using B = Box2<2>;
  __shared__ double rs[D * B::S];
  const BrickLane L = brick_lane(n);
  stage_box<2>(n, L.x0, L.y0, r, rs);
  __syncthreads();
  const int cls = ras_class(L.valid ? L.x : L.x0, L.valid ? L.y : L.y0, n);
  const int first = __builtin_amdgcn_readfirstlane(cls);
  const bool uniform = __all(!L.valid || cls == first);
  const int o = (L.ly + 2) * B::X + L.lx + 2;
  double acc = (L.valid && !zero) ? z[D * L.e + L.row] : 0.0;
  if (uniform)
    acc = ras_row(as_const(ras + ((int64_t)first * D + L.row) * kOmgRasCols), rs, o, acc);
  else
    acc = ras_row(ras + ((int64_t)cls * D + L.row) * kOmgRasCols, rs, o, acc);
  if (L.valid) z[D * L.e + L.row] = acc;
}

template <typename P>
__device__ __forceinline__ double res_row(P A, const double* zs, int o, double acc) {
  using B = Box2<1>;
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    const int os = kSlotOff[s][1] * B::X + kSlotOff[s][0];
#pragma unroll
    for (int b = 0; b < D; ++b) acc -= A[s * D * D + b] * zs[b * B::S + o + os];
  }
  return acc;
}

__global__ __launch_bounds__(kBrickThreads) void k_omg_res(int n, const double* __restrict__ op,
                                                           const double* __restrict__ f,
                                                           const double* __restrict__ z,
                                                           double* __restrict__ r) {
  using B = Box2<1>;
  __shared__ double zs[D * B::S];
  const BrickLane L = brick_lane(n);
  stage_box<1>(n, L.x0, L.y0, z, zs);
  __syncthreads();
  const int cls = L.valid ? op_axis(L.x, n) + 3 * op_axis(L.y, n) : 4;
  const int first = __builtin_amdgcn_readfirstlane(cls);
  const bool uniform = __all(!L.valid || cls == first);
  const int o = (L.ly + 1) * B::X + L.lx + 1;
  double acc = (L.valid && f) ? f[D * L.e + L.row] : 0.0;
  if (uniform)
    acc = res_row(as_const(op + ((int64_t)first * kSlots * D + L.row) * D), zs, o, acc);
  else
    acc = res_row(op + ((int64_t)cls * kSlots * D + L.row) * D, zs, o, acc);
  if (L.valid) r[D * L.e + L.row] = acc;
}

// ---- the largest levels (n_k > kOmgBrick1MaxN): bricks of 8 x 8 squares per
// 256-thread workgroup, wavefront w computing rows 4w .. 4w + 3 of the
// brick's 64 squares (one square per lane), so that every value staged in
// LDS serves four rows.
// The table rows come through scalar loads at wave-uniform addresses: a
// wavefront whose squares share one class reads its four rows once; a
// boundary wavefront takes its few distinct classes one after the other,
// every lane computing with each and keeping the result of its own.
constexpr int kRowsPerWave = 4;
constexpr int kBrick4Threads = 64 * D / kRowsPerWave;

// acc[j] += sum over the diamond of K(row j, 16 d + b) r_d[b] (K =
// kRowsPerWave consecutive rows of a class, row-major [row][208], at a
// wave-uniform address).
__device__ __forceinline__ void ras_rows4(ConstPtr K, const double* rs, int o, double acc[kRowsPerWave]) {
  using B = Box2<2>;
  constexpr Diamond2 DM;
  // one diamond square per trip keeps the registers of the four rows free
  // of spills
#pragma unroll 1
  for (int d = 0; d < kOmgDiamond; ++d) {
    const int od = DM.d[d][1] * B::X + DM.d[d][0];
#pragma unroll
    for (int b = 0; b < D; ++b) {
      const double rv = rs[b * B::S + o + od];
#pragma unroll
      for (int j = 0; j < kRowsPerWave; ++j) acc[j] += K[j * kOmgRasCols + D * d + b] * rv;
    }
  }
}

__global__ __launch_bounds__(kBrick4Threads) void k_omg_ras4(int n, const double* __restrict__ ras,
                                                           const double* __restrict__ r,
                                                           double* __restrict__ z, int zero) {
  using B = Box2<2>;
  __shared__ double rs[D * B::S];
  const BrickLane L = brick_lane(n);
  stage_box<2>(n, L.x0, L.y0, r, rs);
  __syncthreads();
  const int row0 = __builtin_amdgcn_readfirstlane((threadIdx.x >> 6) * kRowsPerWave);
  const int cls = L.valid ? ras_class(L.x, L.y, n) : -1;
  const int o = (L.ly + 2) * B::X + L.lx + 2;
  double acc[kRowsPerWave];
#pragma unroll
  for (int j = 0; j < kRowsPerWave; ++j) acc[j] = (L.valid && !zero) ? z[D * L.e + row0 + j] : 0.0;
  uint64_t pending = __ballot(L.valid);
  while (pending) {   // the wavefront's distinct classes, one per trip (one trip inside)
    const int c = __builtin_amdgcn_readfirstlane(__shfl(cls, __builtin_ctzll(pending), 64));
    double t[kRowsPerWave];
#pragma unroll
    for (int j = 0; j < kRowsPerWave; ++j) t[j] = acc[j];
    ras_rows4((ConstPtr)ras + ((int64_t)c * D + row0) * kOmgRasCols, rs, o, t);
    const bool mine = cls == c;
    if (mine) {
#pragma unroll
      for (int j = 0; j < kRowsPerWave; ++j) acc[j] = t[j];
    }
    pending &= ~__ballot(mine);
  }
  if (L.valid) {
#pragma unroll
    for (int j = 0; j < kRowsPerWave; ++j) z[D * L.e + row0 + j] = acc[j];
  }
}

// acc[j] -= sum over the 5 slots of A(row j, neighbour column b) z_nb[b]
// (A = kRowsPerWave consecutive rows of a class's blocks, [slot][row][16]).
__device__ __forceinline__ void res_rows4(ConstPtr A, const double* zs, int o, double acc[kRowsPerWave]) {
  using B = Box2<1>;
#pragma unroll 1
  for (int s = 0; s < kSlots; ++s) {
    const int os = kSlotOff[s][1] * B::X + kSlotOff[s][0];
#pragma unroll
    for (int b = 0; b < D; ++b) {
      const double zv = zs[b * B::S + o + os];
#pragma unroll
      for (int j = 0; j < kRowsPerWave; ++j) acc[j] -= A[s * D * D + j * D + b] * zv;
    }
  }
}

__global__ __launch_bounds__(kBrick4Threads) void k_omg_res4(int n, const double* __restrict__ op,
                                                           const double* __restrict__ f,
                                                           const double* __restrict__ z,
                                                           double* __restrict__ r) {
  using B = Box2<1>;
  __shared__ double zs[D * B::S];
  const BrickLane L = brick_lane(n);
  stage_box<1>(n, L.x0, L.y0, z, zs);
  __syncthreads();
  const int row0 = __builtin_amdgcn_readfirstlane((threadIdx.x >> 6) * kRowsPerWave);
  const int cls = L.valid ? op_axis(L.x, n) + 3 * op_axis(L.y, n) : -1;
  const int o = (L.ly + 1) * B::X + L.lx + 1;
  double acc[kRowsPerWave];
#pragma unroll
  for (int j = 0; j < kRowsPerWave; ++j) acc[j] = (L.valid && f) ? f[D * L.e + row0 + j] : 0.0;
  uint64_t pending = __ballot(L.valid);
  while (pending) {
    const int c = __builtin_amdgcn_readfirstlane(__shfl(cls, __builtin_ctzll(pending), 64));
    double t[kRowsPerWave];
#pragma unroll
    for (int j = 0; j < kRowsPerWave; ++j) t[j] = acc[j];
    res_rows4((ConstPtr)op + ((int64_t)c * kSlots * D + row0) * D, zs, o, t);
    const bool mine = cls == c;
    if (mine) {
#pragma unroll
      for (int j = 0; j < kRowsPerWave; ++j) acc[j] = t[j];
    }
    pending &= ~__ballot(mine);
  }
  if (L.valid) {
#pragma unroll
    for (int j = 0; j < kRowsPerWave; ++j) r[D * L.e + row0 + j] = acc[j];
  }
}

// ---- transfers: one thread per (square, dof); every component injected alike
__device__ __forceinline__ double inject(int q, int i, int J) {
  double v = 1.0;
#pragma unroll
  for (int ax = 0; ax < 2; ++ax) {
    const double t = 0.5 * (((q >> ax) & 1) + ((i >> ax) & 1));
    v *= ((J >> ax) & 1) ? t : 1.0 - t;
  }
  return v;
}

__global__ __launch_bounds__(kThreads) void k_omg_restrict(int nf, const double* __restrict__ r,
                                                           double* __restrict__ fc) {
  const int nc = nf / 2;
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= (int64_t)D * nc * nc) return;
  const int64_t E = t / D;
  const int dof = int(t % D), c = dof >> 2, J = dof & 3;
  const int X = int(E % nc), Y = int(E / nc);
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double* rc = r + D * ((int64_t)(2 * Y + (q >> 1)) * nf + 2 * X + (q & 1)) + 4 * c;
#pragma unroll
    for (int i = 0; i < 4; ++i) acc += inject(q, i, J) * rc[i];
  }
  fc[t] = acc;
}

__global__ __launch_bounds__(kThreads) void k_omg_prolong(int nf, const double* __restrict__ zc,
                                                          double* __restrict__ z, int assign) {
  const int nc = nf / 2;
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= (int64_t)D * nf * nf) return;
  const int64_t e = t / D;
  const int dof = int(t % D), c = dof >> 2, i = dof & 3;
  const int x = int(e % nf), y = int(e / nf);
  const int q = (x & 1) | ((y & 1) << 1);
  const double* zE = zc + D * ((int64_t)(y >> 1) * nc + (x >> 1)) + 4 * c;
  double acc = 0.0;
#pragma unroll
  for (int J = 0; J < 4; ++J) acc += inject(q, i, J) * zE[J];
  z[t] = assign ? acc : z[t] + acc;
}

// z = inv f: one wavefront per row, lanes over the columns, a fixed shuffle sum.
__global__ __launch_bounds__(kThreads) void k_omg_dense(int m, const double* __restrict__ inv,
                                                        const double* __restrict__ f,
                                                        double* __restrict__ z) {
  const int row = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  double acc = 0.0;
  if (row < m) {
    const double* a = inv + (int64_t)row * m;
    for (int j = lane; j < m; j += 64) acc += a[j] * f[j];
  }
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) acc += __shfl_xor(acc, s, 64);
  if (row < m && lane == 0) z[row] = acc;
}

unsigned blocks_for(int64_t threads) { return unsigned((threads + kThreads - 1) / kThreads); }

}  // namespace

hipError_t launch_omg_res(int nk, const double* op, const double* f, const double* z, double* r,
                          hipStream_t st) {
  if (nk <= kOmgSplitMaxN)
    hipLaunchKernelGGL(k_omg_res_split, dim3(blocks_for(8 * (int64_t)D * nk * nk)), dim3(kThreads), 0, st,
                       nk, op, f, z, r);
  else if (nk <= kOmgBrick1MaxN)
    hipLaunchKernelGGL(k_omg_res, dim3(unsigned(((nk + kBrick - 1) / kBrick) * ((nk + kBrick - 1) / kBrick))),
                       dim3(kBrickThreads), 0, st, nk, op, f, z, r);
  else
    hipLaunchKernelGGL(k_omg_res4, dim3(unsigned(((nk + kBrick - 1) / kBrick) * ((nk + kBrick - 1) / kBrick))),
                       dim3(kBrick4Threads), 0, st, nk, op, f, z, r);
  return hipGetLastError();
}

hipError_t launch_omg_ras(int nk, const double* ras, const double* r, double* z, bool zero,
                          hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (nk <= kOmgSplitMaxN)
    hipExtLaunchKernelGGL(k_omg_ras_split, dim3(blocks_for(16 * (int64_t)D * nk * nk)), dim3(kThreads), 0,
                          st, ev0, ev1, 0, nk, ras, r, z, int(zero));
  else if (nk <= kOmgBrick1MaxN)
    hipExtLaunchKernelGGL(k_omg_ras, dim3(unsigned(((nk + kBrick - 1) / kBrick) * ((nk + kBrick - 1) / kBrick))),
                          dim3(kBrickThreads), 0, st, ev0, ev1, 0, nk, ras, r, z, int(zero));
  else
    hipExtLaunchKernelGGL(k_omg_ras4, dim3(unsigned(((nk + kBrick - 1) / kBrick) * ((nk + kBrick - 1) / kBrick))),
                          dim3(kBrick4Threads), 0, st, ev0, ev1, 0, nk, ras, r, z, int(zero));
  return hipGetLastError();
}

hipError_t launch_omg_restrict(int nf, const double* r, double* fc, hipStream_t st) {
  const int nc = nf / 2;
  hipLaunchKernelGGL(k_omg_restrict, dim3(blocks_for((int64_t)D * nc * nc)), dim3(kThreads), 0, st, nf, r,
                     fc);
  return hipGetLastError();
}

hipError_t launch_omg_prolong(int nf, const double* zc, double* z, bool assign, hipStream_t st) {
  hipLaunchKernelGGL(k_omg_prolong, dim3(blocks_for((int64_t)D * nf * nf)), dim3(kThreads), 0, st, nf, zc,
                     z, int(assign));
  return hipGetLastError();
}

hipError_t launch_omg_dense(int m, const double* inv, const double* f, double* z, hipStream_t st) {
  hipLaunchKernelGGL(k_omg_dense, dim3(unsigned((m + kThreads / 64 - 1) / (kThreads / 64))), dim3(kThreads),
                     0, st, m, inv, f, z);
  return hipGetLastError();
}

}  // namespace dcg
