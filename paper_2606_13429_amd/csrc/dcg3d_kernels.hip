// Kernels of the three-dimensional deflated CG (the d = 3 block structure of
// Section 3.1; deflation as in Algorithm 2 with V of eq. (Vmatrix)).
//
// The A* product and the deflation correction are HBM-bound FP64 streams of
// the 24 x 24 blocks C_3 (32 KB per element): one thread per (element, row of
// C_3) computes that row for the three tensor rows k, so every block entry is
// read once and used three times; the neighbour values of 8 elements are
// staged in LDS.  The inner Laplace system (dt/3) L (Corollary 1, d = 3) is
// solved by block-Jacobi preconditioned CG whose scalars stay on the device;
// every reduction is a fixed-order two-stage sum, so results are
// reproducible bit for bit.
#include <cmath>

#include "dcg3d.hpp"

namespace dcg3 {
namespace {

constexpr int kThreads = 256;
constexpr int kEpw = 8;                    // elements per workgroup (A* and A_div Z)
constexpr int kAThreads = kEpw * 24;       // one thread per row of C_3
constexpr int kMaxPartials = 1024;

__device__ __forceinline__ int nbr3(int n, int e, int s) {
  const int ex = e % n, ey = (e / n) % n, ez = e / (n * n);
  switch (s) {
    case 0: return e;
    case 1: return ex > 0 ? e - 1 : -1;
    case 2: return ex + 1 < n ? e + 1 : -1;
    case 3: return ey > 0 ? e - n : -1;
    case 4: return ey + 1 < n ? e + n : -1;
    case 5: return ez > 0 ? e - n * n : -1;
    default: return ez + 1 < n ? e + n * n : -1;
  }
}

// Sum over the workgroup (kThreads threads, all participating); valid in
// thread 0.  Fixed order: butterfly within each wavefront, then the 4
// wavefront sums in order.
__device__ double block_sum(double v, double* lds) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  return ((lds[0] + lds[1]) + lds[2]) + lds[3];
}

// Sum of part[0 .. cnt) by one workgroup, fixed order.
__device__ double final_sum(const double* __restrict__ part, int cnt, double* lds) {
  double v = 0.0;
  for (int i = threadIdx.x; i < cnt; i += kThreads) v += part[i];
  return block_sum(v, lds);
}

__global__ __launch_bounds__(kAThreads) void k_astar3(int n, const double* __restrict__ Cd,
                                                      const double* __restrict__ Me, double inv_nu,
                                                      double dt, const double* __restrict__ x,
                                                      double* __restrict__ y) {
  const int ne = n * n * n;
  __shared__ double xs[kEpw][kSlots][kDof];
  __shared__ double me[kNb * kNb];
  const int tid = threadIdx.x;
  const int e0 = blockIdx.x * kEpw;
  if (tid < kNb * kNb) me[tid] = Me[tid];
  for (int idx = tid; idx < kEpw * kSlots * kDof; idx += kAThreads) {
    const int el = idx / (kSlots * kDof), rem = idx % (kSlots * kDof);
    const int s = rem / kDof, v = rem % kDof;
    const int e = e0 + el;
    const int nb = e < ne ? nbr3(n, e, s) : -1;
    xs[el][s][v] = nb >= 0 ? x[(int64_t)nb * kDof + v] : 0.0;
  }
  __syncthreads();
  const int el = tid / 24, r = tid % 24;
  const int e = e0 + el;
  if (e >= ne) return;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int s = 0; s < kSlots; ++s) {
    if (nbr3(n, e, s) < 0) continue;
    const double* c = Cd + ((int64_t)s * ne + e) * 576 + r;
    const double* xv = xs[el][s];
#pragma unroll 8
    for (int col = 0; col < 24; ++col) {
      const double cv = __builtin_nontemporal_load(c + col * 24);   // streamed once per launch
      acc[0] += cv * xv[col];
      acc[1] += cv * xv[24 + col];
      acc[2] += cv * xv[48 + col];
    }
  }
  // (C_9 (x) M_1) x on the element: off-diagonal components carry weight 1,
  // the diagonal ones 2/3 on themselves and -1/3 on the other two.
  const int j = r >> 3, a = r & 7;
  const double* xe = xs[el][0];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double m = 0.0;
    if (k != j) {
      const double* xc = xe + 8 * (3 * k + j);
#pragma unroll
      for (int b = 0; b < kNb; ++b) m += me[a * kNb + b] * xc[b];
    } else {
      const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
#pragma unroll
      for (int b = 0; b < kNb; ++b) {
        const double dv = (2.0 / 3.0) * xe[32 * k + b] - (1.0 / 3.0) * (xe[32 * k1 + b] + xe[32 * k2 + b]);
        m += me[a * kNb + b] * dv;
      }
    }
    y[(int64_t)e * kDof + 8 * (3 * k + j) + a] = inv_nu * m + dt * acc[k];
  }
}

__global__ __launch_bounds__(kAThreads) void k_adivz3(int n, const double* __restrict__ Cd, double dt,
                                                      double inv_sqrt3, const double* __restrict__ w,
                                                      const double* __restrict__ yh,
                                                      double* __restrict__ q) {
  const int ne = n * n * n;
  __shared__ double ys[kEpw][kSlots][kNb];
  const int tid = threadIdx.x;
  const int e0 = blockIdx.x * kEpw;
  for (int idx = tid; idx < kEpw * kSlots * kNb; idx += kAThreads) {
    const int el = idx / (kSlots * kNb), rem = idx % (kSlots * kNb);
    const int s = rem / kNb, b = rem % kNb;
    const int e = e0 + el;
    const int nb = e < ne ? nbr3(n, e, s) : -1;
    ys[el][s][b] = nb >= 0 ? yh[(int64_t)nb * kNb + b] * inv_sqrt3 : 0.0;
  }
  __syncthreads();
  const int el = tid / 24, r = tid % 24;
  const int e = e0 + el;
  if (e >= ne) return;
  // (A_div Z yh) at tensor row k, test component j: column block i = k of C_3
  double acc[3] = {0.0, 0.0, 0.0};
  for (int s = 0; s < kSlots; ++s) {
    if (nbr3(n, e, s) < 0) continue;
    const double* c = Cd + ((int64_t)s * ne + e) * 576 + r;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int b = 0; b < kNb; ++b) acc[k] += __builtin_nontemporal_load(c + (8 * k + b) * 24) * ys[el][s][b];
  }
  const int j = r >> 3, a = r & 7;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int64_t i = (int64_t)e * kDof + 8 * (3 * k + j) + a;
    q[i] = w[i] - dt * acc[k];
  }
}

__global__ __launch_bounds__(kThreads) void k_zt3(int64_t ne, double inv_sqrt3,
                                                  const double* __restrict__ w, double* __restrict__ s) {
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (i >= ne * kNb) return;
  const int64_t e = i >> 3;
  const int a = int(i & 7);
  const double* we = w + e * kDof + a;
  s[i] = ((we[0] + we[32]) + we[64]) * inv_sqrt3;
}

__global__ __launch_bounds__(kThreads) void k_zaxpy3(int64_t ne, double c, const double* __restrict__ y,
                                                     double* __restrict__ x) {
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (i >= ne * kNb) return;
  const int64_t e = i >> 3;
  const int a = int(i & 7);
  const double v = c * y[i];
  double* xe = x + e * kDof + a;
  xe[0] += v;
  xe[32] += v;
  xe[64] += v;
}

__global__ __launch_bounds__(kThreads) void k_lap3(int n, const double* __restrict__ Ld, double scale,
                                                   const double* __restrict__ p, double* __restrict__ q,
                                                   double* __restrict__ part) {
  __shared__ double lds[4];
  const int ne = n * n * n;
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  double pq = 0.0;
  if (i < (int64_t)ne * kNb) {
    const int e = int(i >> 3), a = int(i & 7);
    double acc = 0.0;
    for (int s = 0; s < kSlots; ++s) {
      const int nb = nbr3(n, e, s);
      if (nb < 0) continue;
      const double* l = Ld + ((int64_t)s * ne + e) * 64 + a;
      const double* pn = p + (int64_t)nb * kNb;
#pragma unroll
      for (int b = 0; b < kNb; ++b) acc += l[8 * b] * pn[b];
    }
    const double v = scale * acc;
    q[i] = v;
    pq = p[i] * v;
  }
  pq = block_sum(pq, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = pq;
}

// z = Dinv r on the element of thread i (r of the element in LDS rl).
__device__ __forceinline__ double bj_apply(const double* __restrict__ Dinv, int64_t e, int a,
                                           const double* rl) {
  const double* d = Dinv + e * 64 + a;
  double z = 0.0;
#pragma unroll
  for (int b = 0; b < kNb; ++b) z += d[8 * b] * rl[b];
  return z;
}

__global__ __launch_bounds__(kThreads) void k_pcg_init(int64_t ne, const double* __restrict__ Dinv,
                                                       const double* __restrict__ s, double* __restrict__ x,
                                                       double* __restrict__ r, double* __restrict__ z,
                                                       double* __restrict__ p, double* __restrict__ part) {
  __shared__ double rl[kThreads];
  __shared__ double lds[4];
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  const bool live = i < ne * kNb;
  const double rv = live ? s[i] : 0.0;
  rl[threadIdx.x] = rv;
  __syncthreads();
  double rz = 0.0, rr = 0.0;
  if (live) {
    const double zv = bj_apply(Dinv, i >> 3, int(i & 7), rl + (threadIdx.x & ~7));
    x[i] = 0.0;
    r[i] = rv;
    z[i] = zv;
    p[i] = zv;
    rz = rv * zv;
    rr = rv * rv;
  }
  rz = block_sum(rz, lds);
  rr = block_sum(rr, lds);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = rz;
    part[gridDim.x + blockIdx.x] = rr;
  }
}

__global__ __launch_bounds__(kThreads) void k_pcg_init_final(const double* __restrict__ part, int cnt,
                                                             double rel2, PcgScalars* sc) {
  __shared__ double lds[4];
  const double rz = final_sum(part, cnt, lds);
  const double rr = final_sum(part + cnt, cnt, lds);
  if (threadIdx.x == 0) {
    sc->rho = rz;
    sc->rr = rr;
    sc->pq = 0.0;
    sc->alpha = sc->beta = 0.0;
    sc->thresh2 = rel2 * rr;
    sc->active = (rr > sc->thresh2 && rr > 0.0) ? 1 : 0;
    sc->iters = 0;
  }
}

__global__ __launch_bounds__(kThreads) void k_pcg_alpha(const double* __restrict__ part, int cnt,
                                                        PcgScalars* sc) {
  __shared__ double lds[4];
  const double pq = final_sum(part, cnt, lds);
  if (threadIdx.x == 0) {
    sc->pq = pq;
    if (sc->active && pq > 0.0 && std::isfinite(pq)) {
      sc->alpha = sc->rho / pq;
    } else {
      sc->alpha = 0.0;
      sc->active = 0;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_pcg_update(int64_t ne, const double* __restrict__ Dinv,
                                                         double* __restrict__ x, double* __restrict__ r,
                                                         double* __restrict__ z, const double* __restrict__ p,
                                                         const double* __restrict__ q,
                                                         double* __restrict__ part,
                                                         const PcgScalars* sc) {
  __shared__ double rl[kThreads];
  __shared__ double lds[4];
  const double alpha = sc->alpha;
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  const bool live = i < ne * kNb;
  double rv = 0.0;
  if (live) {
    x[i] += alpha * p[i];
    rv = r[i] - alpha * q[i];
    r[i] = rv;
  }
  rl[threadIdx.x] = rv;
  __syncthreads();
  double rz = 0.0, rr = 0.0;
  if (live) {
    const double zv = bj_apply(Dinv, i >> 3, int(i & 7), rl + (threadIdx.x & ~7));
    z[i] = zv;
    rz = rv * zv;
    rr = rv * rv;
  }
  rz = block_sum(rz, lds);
  rr = block_sum(rr, lds);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = rz;
    part[gridDim.x + blockIdx.x] = rr;
  }
}

__global__ __launch_bounds__(kThreads) void k_pcg_beta(const double* __restrict__ part, int cnt,
                                                       PcgScalars* sc) {
  __shared__ double lds[4];
  const double rz = final_sum(part, cnt, lds);
  const double rr = final_sum(part + cnt, cnt, lds);
  if (threadIdx.x == 0) {
    if (sc->active) {
      sc->beta = rz / sc->rho;
      sc->rho = rz;
      sc->rr = rr;
      sc->iters += 1;
      if (!(rr > sc->thresh2)) sc->active = 0;
    } else {
      sc->beta = 0.0;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_pcg_dir(int64_t len, const double* __restrict__ z,
                                                      double* __restrict__ p, const PcgScalars* sc) {
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (i < len) p[i] = z[i] + sc->beta * p[i];
}

__global__ __launch_bounds__(kThreads) void k_dot_partial(int64_t len, const double* __restrict__ x,
                                                          const double* __restrict__ y,
                                                          double* __restrict__ part) {
  __shared__ double lds[4];
  double v = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * kThreads)
    v += x[i] * y[i];
  v = block_sum(v, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ __launch_bounds__(kThreads) void k_dot_final(const double* __restrict__ part, int cnt,
                                                        double* __restrict__ out) {
  __shared__ double lds[4];
  const double v = final_sum(part, cnt, lds);
  if (threadIdx.x == 0) out[0] = v;
}

__global__ __launch_bounds__(kThreads) void k_axpy(int64_t len, double a, const double* __restrict__ x,
                                                   double* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (i < len) y[i] += a * x[i];
}

__global__ __launch_bounds__(kThreads) void k_xpby(int64_t len, const double* __restrict__ x, double b,
                                                   double* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (i < len) y[i] = x[i] + b * y[i];
}

__global__ __launch_bounds__(kThreads) void k_fill(int64_t len, double v, double* __restrict__ x) {
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (i < len) x[i] = v;
}

// Position of tensor index (Ix, Iy, Iz), I = 2 e_axis + i_axis, in the
// element-major scalar layout 8 e + a or in the tensor layout (Iz N + Iy) N + Ix.
template <bool ELEM>
__device__ __forceinline__ int64_t fdm_pos(int n, int Ix, int Iy, int Iz) {
  const int N = 2 * n;
  if (ELEM) {
    const int64_t e = ((int64_t)(Iz >> 1) * n + (Iy >> 1)) * n + (Ix >> 1);
    return 8 * e + (Ix & 1) + 2 * (Iy & 1) + 4 * (Iz & 1);
  }
  return ((int64_t)Iz * N + Iy) * N + Ix;
}

// One pass of the fast diagonalisation: out_i = sum_j A[j N + i] in_j along
// one axis of the (2n)^3 tensor, optionally scaled by
// scale / (lx[Ix] + ly[Iy] + ly[Iz]).  One workgroup takes 256 / N lines of N
// values, staged in LDS; thread (line, i) forms output i of its line.
template <bool IN_ELEM, bool OUT_ELEM>
__global__ __launch_bounds__(kThreads) void k_fdm_axis(int n, int axis, const double* __restrict__ A,
                                                       const double* __restrict__ in,
                                                       double* __restrict__ out,
                                                       const double* __restrict__ lx,
                                                       const double* __restrict__ ly, double scale) {
  __shared__ double line[kThreads];
  const int N = 2 * n;
  const int lpw = kThreads / N;
  const int ll = threadIdx.x / N, i = threadIdx.x % N;
  const int64_t g = (int64_t)blockIdx.x * lpw + ll;
  const bool live = ll < lpw && g < (int64_t)N * N;
  int I[3] = {0, 0, 0};
  if (live) {
    const int o1 = int(g % N), o2 = int(g / N);
    const int a1 = axis == 0 ? 1 : 0, a2 = axis == 2 ? 1 : 2;
    I[a1] = o1;
    I[a2] = o2;
    I[axis] = i;
    line[threadIdx.x] = in[fdm_pos<IN_ELEM>(n, I[0], I[1], I[2])];
  }
  __syncthreads();
  if (!live) return;
  const double* lv = line + ll * N;
  double acc = 0.0;
  for (int j = 0; j < N; ++j) acc += A[j * N + i] * lv[j];
  if (lx) acc *= scale / (lx[I[0]] + ly[I[1]] + ly[I[2]]);
  out[fdm_pos<OUT_ELEM>(n, I[0], I[1], I[2])] = acc;
}

int blocks_for(int64_t len) { return int((len + kThreads - 1) / kThreads); }

const double kInvSqrt3 = 1.0 / std::sqrt(3.0);

}  // namespace

int partial_blocks(int64_t len) {
  const int64_t b = (len + kThreads - 1) / kThreads;
  return int(b < kMaxPartials ? (b > 0 ? b : 1) : kMaxPartials);
}

hipError_t launch_astar3(int n, const double* Cd, const double* Me, double inv_nu, double dt,
                         const double* x, double* y, hipStream_t st) {
  const int ne = n * n * n;
  k_astar3<<<(ne + kEpw - 1) / kEpw, kAThreads, 0, st>>>(n, Cd, Me, inv_nu, dt, x, y);
  return hipGetLastError();
}

hipError_t launch_adivz3(int n, const double* Cd, double dt, const double* w, const double* yh,
                         double* q, hipStream_t st) {
  const int ne = n * n * n;
  k_adivz3<<<(ne + kEpw - 1) / kEpw, kAThreads, 0, st>>>(n, Cd, dt, kInvSqrt3, w, yh, q);
  return hipGetLastError();
}

hipError_t launch_zt3(int64_t ne, const double* w, double* s, hipStream_t st) {
  k_zt3<<<blocks_for(ne * kNb), kThreads, 0, st>>>(ne, kInvSqrt3, w, s);
  return hipGetLastError();
}

hipError_t launch_zaxpy3(int64_t ne, double a, const double* y, double* x, hipStream_t st) {
  k_zaxpy3<<<blocks_for(ne * kNb), kThreads, 0, st>>>(ne, a * kInvSqrt3, y, x);
  return hipGetLastError();
}

hipError_t launch_lap3(int n, const double* Ld, double scale, const double* p, double* q,
                       double* part, hipStream_t st) {
  const int64_t ne = (int64_t)n * n * n;
  k_lap3<<<blocks_for(ne * kNb), kThreads, 0, st>>>(n, Ld, scale, p, q, part);
  return hipGetLastError();
}

hipError_t launch_pcg_start(int64_t ne, const double* Dinv, const double* s, double* x, double* r,
                            double* z, double* p, double* part, PcgScalars* sc, double rel2,
                            hipStream_t st) {
  const int g = blocks_for(ne * kNb);
  k_pcg_init<<<g, kThreads, 0, st>>>(ne, Dinv, s, x, r, z, p, part);
  k_pcg_init_final<<<1, kThreads, 0, st>>>(part, g, rel2, sc);
  return hipGetLastError();
}

hipError_t launch_pcg_step(int64_t ne, const double* Dinv, double* x, double* r, double* z,
                           double* p, const double* q, double* part, double* part2, int nblk_q,
                           PcgScalars* sc, hipStream_t st) {
  const int g = blocks_for(ne * kNb);
  k_pcg_alpha<<<1, kThreads, 0, st>>>(part, nblk_q, sc);
  k_pcg_update<<<g, kThreads, 0, st>>>(ne, Dinv, x, r, z, p, q, part2, sc);
  k_pcg_beta<<<1, kThreads, 0, st>>>(part2, g, sc);
  k_pcg_dir<<<g, kThreads, 0, st>>>(ne * kNb, z, p, sc);
  return hipGetLastError();
}

hipError_t launch_fdm_solve(int n, const double* Vx, const double* VxT, const double* Vy,
                            const double* VyT, const double* lx, const double* ly, double scale,
                            const double* in, double* out, double* t1, double* t2, hipStream_t st) {
  const int N = 2 * n;
  if (N > kThreads) return hipErrorInvalidValue;
  const int lpw = kThreads / N;
  const int grid = int(((int64_t)N * N + lpw - 1) / lpw);
  k_fdm_axis<true, false><<<grid, kThreads, 0, st>>>(n, 0, Vx, in, t1, nullptr, nullptr, 0.0);
  k_fdm_axis<false, false><<<grid, kThreads, 0, st>>>(n, 1, Vy, t1, t2, nullptr, nullptr, 0.0);
  k_fdm_axis<false, false><<<grid, kThreads, 0, st>>>(n, 2, Vy, t2, t1, lx, ly, scale);
  k_fdm_axis<false, false><<<grid, kThreads, 0, st>>>(n, 2, VyT, t1, t2, nullptr, nullptr, 0.0);
  k_fdm_axis<false, false><<<grid, kThreads, 0, st>>>(n, 1, VyT, t2, t1, nullptr, nullptr, 0.0);
  k_fdm_axis<false, true><<<grid, kThreads, 0, st>>>(n, 0, VxT, t1, out, nullptr, nullptr, 0.0);
  return hipGetLastError();
}

hipError_t launch_dot(int64_t len, const double* x, const double* y, double* part, double* out,
                      hipStream_t st) {
  const int g = partial_blocks(len);
  k_dot_partial<<<g, kThreads, 0, st>>>(len, x, y, part);
  k_dot_final<<<1, kThreads, 0, st>>>(part, g, out);
  return hipGetLastError();
}

hipError_t launch_axpy(int64_t len, double a, const double* x, double* y, hipStream_t st) {
  k_axpy<<<blocks_for(len), kThreads, 0, st>>>(len, a, x, y);
  return hipGetLastError();
}

hipError_t launch_xpby(int64_t len, const double* x, double b, double* y, hipStream_t st) {
  k_xpby<<<blocks_for(len), kThreads, 0, st>>>(len, x, b, y);
  return hipGetLastError();
}

hipError_t launch_fill(int64_t len, double v, double* x, hipStream_t st) {
  k_fill<<<blocks_for(len), kThreads, 0, st>>>(len, v, x);
  return hipGetLastError();
}

}  // namespace dcg3
