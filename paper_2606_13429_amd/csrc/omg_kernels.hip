// Kernels of the outer multigrid preconditioner (W-cycle on A*, layouts in
// omg.hpp).  Level vectors hold 16 FP64 values per square.
//
// The RAS step and the residual split every output (square, row) over a few
// lanes on levels of at most kOmgSplitMaxN squares per side (one lane per
// diamond square resp. face slot, one round of 128-byte loads each, a fixed
// shuffle sum), where a launch has few workgroups and its time is one
// thread's chain of loads.  Larger levels stage the input of an 8 x 8 brick
// in LDS and run the step as FP64 MFMA products of the class tables with the
// brick's gathered inputs (measured against vector-FMA bricks with the table
// rows read per lane or through scalar loads: 2-5x faster from 128 squares
// per side up, 1.3x at 64; slower than the split kernels below 64, where
// every brick is a boundary brick whose several classes cost one trip each).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "host_setup.hpp"
#include "omg.hpp"

namespace dcg {

namespace {

constexpr int D = kOmgDofs;
constexpr int kThreads = 256;
constexpr int kOmgSplitMaxN = 32;

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

// ---- large levels: 8 x 8 bricks with their input staged in LDS
constexpr int kBrick = 8;

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

// ---- MFMA form: on an 8 x 8 brick the step is a class table (16 rows) times
// the gathered inputs of the brick's squares, 16 squares per wavefront as the
// columns of v_mfma_f64_16x16x4f64, four table columns a step.  Lane l
// supplies row l % 16, column 4 s + l / 16 of the table (the operand-order
// tables make one step's operand one contiguous 512-byte run) and, for square
// l % 16 of its wavefront, input value 4 s + l / 16 of that square's window
// from LDS; it receives rows 4 v + l / 16 (v = 0..3) of square l % 16.
// Interior bricks (every square of the interior class) stage the one class
// table in LDS next to the input and run the products from LDS with two
// accumulators; boundary bricks, dispatched first, take the distinct classes
// of each wavefront one after the other with the table read from global
// memory, keeping for each square the product with its own class.
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kMfmaThreads = 256;   // 4 wavefronts x 16 squares = one brick
constexpr int kRasInterior = 3 + 7 * 3;
constexpr int kOpInterior = 1 + 3 * 1;

struct MfmaLane {
  int x0, y0, x, y, q, o1, o2;   // brick, square, output row group, LDS offsets (halo 1 / 2)
  bool interior;
  int64_t e;
};

// Workgroup -> brick: the ring of boundary bricks first, then the interior.
__device__ __forceinline__ MfmaLane mfma_lane(int n) {
  const int nb = n / kBrick, ring = nb > 1 ? 4 * (nb - 1) : 1;
  const int b = blockIdx.x;
  int bx, by;
  if (b < ring) {
    if (b < nb) {
      bx = b;
      by = 0;
    } else if (b < 2 * nb) {
      bx = b - nb;
      by = nb - 1;
    } else {
      const int t = b - 2 * nb;
      bx = t < nb - 2 ? 0 : nb - 1;
      by = 1 + (t < nb - 2 ? t : t - (nb - 2));
    }
  } else {
    const int t = b - ring;
    bx = 1 + t % (nb - 2);
    by = 1 + t / (nb - 2);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = lane & 15, lx = j & 7, ly = 2 * w + (j >> 3);
  MfmaLane L;
  L.x0 = bx * kBrick;
  L.y0 = by * kBrick;
  L.interior = b >= ring;
  L.x = L.x0 + lx;
  L.y = L.y0 + ly;
  L.q = lane >> 4;
  L.o1 = (ly + 1) * Box2<1>::X + lx + 1;
  L.o2 = (ly + 2) * Box2<2>::X + lx + 2;
  L.e = (int64_t)L.y * n + L.x;
  return L;
}

__device__ __forceinline__ v4d mfma64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Copies one class table (steps x 64 doubles, operand order) into LDS.
template <int STEPS>
__device__ __forceinline__ void stage_table(const double* __restrict__ src, double* kt) {
  for (int i = threadIdx.x; i < STEPS * 64; i += kMfmaThreads) kt[i] = src[i];
}

// RAS products over the 13-square diamond: Kv(s) is the lane's table operand
// of step s, the input of step s the LDS plane 4 (s % 4) + q at the square's
// offset plus the diamond offset of s / 4.
template <typename KV>
__device__ __forceinline__ v4d ras_chain(KV Kv, const double* rs, const MfmaLane& L, v4d t) {
  using B = Box2<2>;
  constexpr Diamond2 DM;
  v4d t1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int d = 0; d < kOmgDiamond; ++d) {
    const int od = DM.d[d][1] * B::X + DM.d[d][0];
    t = mfma64(Kv(4 * d), rs[(0 + L.q) * B::S + L.o2 + od], t);
    t1 = mfma64(Kv(4 * d + 1), rs[(4 + L.q) * B::S + L.o2 + od], t1);
    t = mfma64(Kv(4 * d + 2), rs[(8 + L.q) * B::S + L.o2 + od], t);
    t1 = mfma64(Kv(4 * d + 3), rs[(12 + L.q) * B::S + L.o2 + od], t1);
  }
  return t + t1;
}

template <typename KV>
__device__ __forceinline__ v4d res_chain(KV Kv, const double* zs, const MfmaLane& L) {
  using B = Box2<1>;
  v4d t = {0.0, 0.0, 0.0, 0.0}, t1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int sl = 0; sl < kSlots; ++sl) {
    const int os = kSlotOff[sl][1] * B::X + kSlotOff[sl][0];
    t = mfma64(Kv(4 * sl), zs[(0 + L.q) * B::S + L.o1 + os], t);
    t1 = mfma64(Kv(4 * sl + 1), zs[(4 + L.q) * B::S + L.o1 + os], t1);
    t = mfma64(Kv(4 * sl + 2), zs[(8 + L.q) * B::S + L.o1 + os], t);
    t1 = mfma64(Kv(4 * sl + 3), zs[(12 + L.q) * B::S + L.o1 + os], t1);
  }
  return t + t1;
}

// Boundary bricks: the lanes of a wavefront take squares of as few classes as
// possible -- square slot i of the brick (wavefront i / 16, lane i % 16) gets
// the square of rank i in the order (class, position) -- so that an edge brick
// needs at most two class trips per wavefront.  cls_of(x, y) is the class.
template <typename CF>
__device__ __forceinline__ void sort_squares(MfmaLane& L, int n, CF cls_of, int* scls, int* sperm) {
  if (threadIdx.x < kBrick * kBrick)
    scls[threadIdx.x] = cls_of(L.x0 + (threadIdx.x & 7), L.y0 + (threadIdx.x >> 3));
  __syncthreads();
  if (threadIdx.x < kBrick * kBrick) {
    const int me = threadIdx.x, c = scls[me];
    int rank = 0;
    for (int i = 0; i < kBrick * kBrick; ++i) {
      const int ci = scls[i];
      rank += (ci < c) || (ci == c && i < me);
    }
    sperm[rank] = me;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, sq = sperm[16 * (threadIdx.x >> 6) + (lane & 15)];
  const int lx = sq & 7, ly = sq >> 3;
  L.x = L.x0 + lx;
  L.y = L.y0 + ly;
  L.o1 = (ly + 1) * Box2<1>::X + lx + 1;
  L.o2 = (ly + 2) * Box2<2>::X + lx + 2;
  L.e = (int64_t)L.y * n + L.x;
}

// three workgroups fit a compute unit's LDS; registers are kept to match
__global__ __launch_bounds__(kMfmaThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_omg_ras_m(int n, const double* __restrict__ rasm,
                                                            const double* __restrict__ r,
                                                            double* __restrict__ z, int zero) {
  using B = Box2<2>;
  __shared__ double rs[D * B::S];
  __shared__ double kt[kOmgRasSteps * 64];
  __shared__ int scls[kBrick * kBrick], sperm[kBrick * kBrick];
  MfmaLane L = mfma_lane(n);
  const int lane = threadIdx.x & 63;
  if (L.interior) stage_table<kOmgRasSteps>(rasm + (int64_t)kRasInterior * kOmgRasSteps * 64, kt);
  stage_box<2>(n, L.x0, L.y0, r, rs);
  if (!L.interior) sort_squares(L, n, [n](int x, int y) { return ras_class(x, y, n); }, scls, sperm);
  v4d acc;
#pragma unroll
  for (int v = 0; v < 4; ++v) acc[v] = zero ? 0.0 : z[D * L.e + 4 * v + L.q];
  __syncthreads();
  if (L.interior) {
    acc = ras_chain([&](int st) { return kt[lane + 64 * st]; }, rs, L, acc);
  } else {
    const int cls = ras_class(L.x, L.y, n);
    uint64_t pending = __ballot(true);
    while (pending) {   // the wavefront's distinct classes, one per trip
      const int c = __builtin_amdgcn_readfirstlane(__shfl(cls, __builtin_ctzll(pending), 64));
      const double* K = rasm + (int64_t)c * kOmgRasSteps * 64 + lane;
      double a[kOmgRasSteps];   // the trip's operands requested ahead of the products
#pragma unroll
      for (int st = 0; st < kOmgRasSteps; ++st) a[st] = K[64 * st];
      const v4d t = ras_chain([&](int st) { return a[st]; }, rs, L, acc);
      const bool mine = cls == c;
      if (mine) acc = t;
      pending &= ~__ballot(mine);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) z[D * L.e + 4 * v + L.q] = acc[v];
}

__global__ __launch_bounds__(kMfmaThreads) void k_omg_res_m(int n, const double* __restrict__ opm,
                                                            const double* __restrict__ f,
                                                            const double* __restrict__ z,
                                                            double* __restrict__ r) {
  using B = Box2<1>;
  __shared__ double zs[D * B::S];
  __shared__ double kt[kOmgOpSteps * 64];
  __shared__ int scls[kBrick * kBrick], sperm[kBrick * kBrick];
  MfmaLane L = mfma_lane(n);
  const int lane = threadIdx.x & 63;
  if (L.interior) stage_table<kOmgOpSteps>(opm + (int64_t)kOpInterior * kOmgOpSteps * 64, kt);
  stage_box<1>(n, L.x0, L.y0, z, zs);
  if (!L.interior)
    sort_squares(L, n, [n](int x, int y) { return op_axis(x, n) + 3 * op_axis(y, n); }, scls, sperm);
  double fv[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) fv[v] = f ? f[D * L.e + 4 * v + L.q] : 0.0;
  __syncthreads();
  v4d acc;
  if (L.interior) {
    acc = res_chain([&](int st) { return kt[lane + 64 * st]; }, zs, L);
  } else {
    const int cls = op_axis(L.x, n) + 3 * op_axis(L.y, n);
    acc = v4d{0.0, 0.0, 0.0, 0.0};
    uint64_t pending = __ballot(true);
    while (pending) {
      const int c = __builtin_amdgcn_readfirstlane(__shfl(cls, __builtin_ctzll(pending), 64));
      const double* K = opm + (int64_t)c * kOmgOpSteps * 64 + lane;
      double a[kOmgOpSteps];
#pragma unroll
      for (int st = 0; st < kOmgOpSteps; ++st) a[st] = K[64 * st];
      const v4d t = res_chain([&](int st) { return a[st]; }, zs, L);
      const bool mine = cls == c;
      if (mine) acc = t;
      pending &= ~__ballot(mine);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) r[D * L.e + 4 * v + L.q] = fv[v] - acc[v];
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
unsigned bricks(int nk) { return unsigned((nk / kBrick) * (nk / kBrick)); }

}  // namespace

hipError_t launch_omg_res(int nk, const double* op, const double* opm, const double* f, const double* z,
                          double* r, hipStream_t st) {
  if (nk <= kOmgSplitMaxN) {
    hipLaunchKernelGGL(k_omg_res_split, dim3(blocks_for(8 * (int64_t)D * nk * nk)), dim3(kThreads), 0, st,
                       nk, op, f, z, r);
  } else {
    if (nk % kBrick) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_omg_res_m, dim3(bricks(nk)), dim3(kMfmaThreads), 0, st, nk, opm, f, z, r);
  }
  return hipGetLastError();
}

hipError_t launch_omg_ras(int nk, const double* ras, const double* rasm, const double* r, double* z,
                          bool zero, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (nk <= kOmgSplitMaxN) {
    hipExtLaunchKernelGGL(k_omg_ras_split, dim3(blocks_for(16 * (int64_t)D * nk * nk)), dim3(kThreads), 0,
                          st, ev0, ev1, 0, nk, ras, r, z, int(zero));
  } else {
    if (nk % kBrick) return hipErrorInvalidValue;
    hipExtLaunchKernelGGL(k_omg_ras_m, dim3(bricks(nk)), dim3(kMfmaThreads), 0, st, ev0, ev1, 0, nk, rasm,
                          r, z, int(zero));
  }
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
