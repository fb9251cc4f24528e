// gfx950 kernels of the deflated-CG hot path (paper Section 4, Algorithms 2-4).
//
// Everything here is bandwidth bound (well under 1 flop per byte), so the
// kernels are organised around coalesced 16-byte loads of the stored
// operators: a wavefront of 64 lanes reads 1 KiB per load instruction, the
// operator layouts (kernels.hpp) put consecutive lanes on consecutive
// 16-byte words, and vector operands come from L2 / LDS.  Dot products are
// two-stage and deterministic: a fixed-order wave64 shuffle tree and an LDS
// tree per workgroup, per-workgroup partials, and one fixed-order final
// pass (no floating-point atomics anywhere).
#include <hip/hip_ext.h>

#include "kernels.hpp"
#include "mg_common.hpp"

#include <cmath>

namespace dcg {
namespace {

constexpr int kThreads = 256;
constexpr double kInvSqrt2 = 0.70710678118654752440;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Workgroup sum of v (all 256 threads participate); result valid in thread 0.
__device__ inline double block_sum(double v, double* lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = (lds[0] + lds[1]) + (lds[2] + lds[3]);
  return s;
}

using mg::ld4;   // 4-vector loads shared with the multigrid kernels

// A 16-byte load with the non-temporal hint, for operator blocks that a
// launch streams once.
typedef double stream2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ stream2 load_stream(const double2* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const stream2*>(p));
}

inline int grid_for(int64_t items, int per_block, int cap) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  return int(g < cap ? g : cap);
}

// ============================================================ outer kernels
// w = (1/nu) M u + dt A_div u, s = Z^T w.  Thread (square e, row r); one
// workgroup = 16 squares.  M = C (x) M_1 with C the dev-dev coefficient
// matrix (Section 3.1): rows 11/22 see (u11 - u22)/2, rows 12/21 see u.
__device__ inline int slot_id(const Slots& sl) { return sl.list ? sl.list[blockIdx.y] : 0; }

template <int MODE>
__global__ __launch_bounds__(kThreads) void k_astar(
    const double2* __restrict__ C, const int32_t* __restrict__ cols, const double* __restrict__ M1,
    int ne, const double* __restrict__ x, const double* __restrict__ p_old,
    const double* __restrict__ b, const Scalars* __restrict__ sc, double* __restrict__ p_new,
    double* __restrict__ w, double* __restrict__ s, double* __restrict__ part, Slots sl) {
  __shared__ double lds[4];
  const int slot = slot_id(sl);
  x += slot * sl.tstride;
  if (p_old) p_old += slot * sl.tstride;
  if (b) b += slot * sl.tstride;
  if (p_new) p_new += slot * sl.tstride;
  if (w) w += slot * sl.tstride;
  if (s) s += slot * sl.sstride;
  sc += slot;
  if (part) part += slot * kSlotPart;
  const double dt = sc->dt, inv_nu = sc->inv_nu;
  const int r = threadIdx.x & 15;
  const double beta = MODE == kAstarDir ? sc->beta : 0.0;
  const int groups = (ne + 15) >> 4;
  double dot = 0.0;
  for (int g = blockIdx.x; g < groups; g += gridDim.x) {
    const int e = (g << 4) + (threadIdx.x >> 4);
    const bool valid = e < ne;
    double acc = 0.0, wv = 0.0;
    // Lane r of a square loads value r of each vector it needs; the 16 lanes of
    // the square exchange values by shuffles (the neighbour of a slot is the
    // same for all 16, so the branches and shuffles are uniform within the
    // group).  u0 = the direction at the own square.
    double u0 = 0.0;
    if (valid) {
      u0 = x[16 * (int64_t)e + r];
      if (MODE == kAstarDir) u0 += beta * p_old[16 * (int64_t)e + r];
    }
    // A_div part, row r of diag(C, C): row r % 8 of C applied to the 8 values
    // of stress row r / 8 of each neighbour
    const int o = (r >> 3) * 8;
#pragma unroll
    for (int slot = 0; slot < 5; ++slot) {
      const int c = valid ? cols[slot * ne + e] : -1;
      double ur = u0;
      if (slot != 0 && c >= 0) {
        ur = x[16 * (int64_t)c + r];
        if (MODE == kAstarDir) ur += beta * p_old[16 * (int64_t)c + r];
      }
      double u[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) u[m] = __shfl(ur, o + m, 16);
      if (c >= 0) {
        // the blocks are streamed once per launch: non-temporal loads keep
        // them from displacing the vectors in the caches (181 -> 168 us at
        // n = 512)
        const double2* Cb = C + ((int64_t)slot * 4 * ne + e) * 8 + (r & 7);
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
          const stream2 a = load_stream(Cb + (int64_t)kc * ne * 8);
          acc += a.x * u[2 * kc] + a.y * u[2 * kc + 1];
        }
      }
    }
    // mass part (1/nu)(C_dev (x) M_1) u of the own square: row (cc, j) needs
    // the corners of sigma_11 and sigma_22 (cc = 0, 3) or of sigma_cc (cc = 1, 2)
    const int cc = r >> 2, j = r & 3;
    double s11[4], s22[4], sc4[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      s11[m] = __shfl(u0, m, 16);
      s22[m] = __shfl(u0, 12 + m, 16);
      sc4[m] = __shfl(u0, 4 * cc + m, 16);
    }
    if (valid) {
      double m1[4];
      ld4(M1 + 16 * (int64_t)e + 4 * j, m1);
      double mu;
      if (cc == 0 || cc == 3) {
        mu = 0.5 * (m1[0] * (s11[0] - s22[0]) + m1[1] * (s11[1] - s22[1]) +
                    m1[2] * (s11[2] - s22[2]) + m1[3] * (s11[3] - s22[3]));
        if (cc == 3) mu = -mu;
      } else {
        mu = m1[0] * sc4[0] + m1[1] * sc4[1] + m1[2] * sc4[2] + m1[3] * sc4[3];
      }
      wv = inv_nu * mu + dt * acc;
      if (MODE == kAstarResidual) {
        wv = b[16 * (int64_t)e + r] - wv;
        dot += wv * wv;
      }
      if (w) w[16 * (int64_t)e + r] = wv;
      if (MODE == kAstarDir || MODE == kAstarFirst) p_new[16 * (int64_t)e + r] = u0;
    }
    // s = Z^T w: lanes r = j and r = 12 + j of the same square
    const double w22 = __shfl_down(wv, 12, 16);
    if (s && valid && r < 4) s[4 * (int64_t)e + r] = (wv + w22) * kInvSqrt2;
  }
  if (MODE == kAstarResidual) {
    const double t = block_sum(dot, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
  }
}

// q = w - c (A_div Z) z, partial (p, q); prologue: r = w - c AZ z -> q, p_out,
// partials (w, w), (r, r).
template <bool PROLOGUE>
__global__ __launch_bounds__(kThreads) void k_deflate(
    const double2* __restrict__ AZ, const int32_t* __restrict__ cols, int ne, double c,
    const double* __restrict__ z, const double* __restrict__ w, const double* __restrict__ p,
    double* __restrict__ q, double* __restrict__ p_out, double* __restrict__ part, Slots sl) {
  __shared__ double lds[4];
  const int slot = slot_id(sl);
  z += slot * sl.sstride;
  w += slot * sl.tstride;
  if (p) p += slot * sl.tstride;
  q += slot * sl.tstride;
  if (p_out) p_out += slot * sl.tstride;
  part += slot * kSlotPart;
  const int r = threadIdx.x & 15;
  const int groups = (ne + 15) >> 4;
  double d0 = 0.0, d1 = 0.0;
  for (int g = blockIdx.x; g < groups; g += gridDim.x) {
    const int e = (g << 4) + (threadIdx.x >> 4);
    if (e >= ne) continue;
    double acc = 0.0;
#pragma unroll
    for (int slot = 0; slot < 5; ++slot) {
      const int col = cols[slot * ne + e];
      if (col < 0) continue;
      const double2* zc = reinterpret_cast<const double2*>(z + 4 * (int64_t)col);
      const double2* Ab = AZ + ((int64_t)slot * 2 * ne + e) * 16 + r;
      const stream2 a0 = load_stream(Ab), a1 = load_stream(Ab + (int64_t)ne * 16);
      const double2 z0 = zc[0], z1 = zc[1];
      acc += a0.x * z0.x + a0.y * z0.y + a1.x * z1.x + a1.y * z1.y;
    }
    const int64_t i = 16 * (int64_t)e + r;
    const double wv = w[i];
    const double qv = wv - c * acc;
    q[i] = qv;
    if (PROLOGUE) {
      p_out[i] = qv;
      d0 += wv * wv;
      d1 += qv * qv;
    } else {
      d0 += p[i] * qv;
    }
  }
  const double t0 = block_sum(d0, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = t0;
  if (PROLOGUE) {
    const double t1 = block_sum(d1, lds);
    if (threadIdx.x == 0) part[kPartStride + blockIdx.x] = t1;
  }
}

__global__ __launch_bounds__(kThreads) void k_adivz(const double2* __restrict__ AZ,
                                                    const int32_t* __restrict__ cols, int ne,
                                                    const double* __restrict__ y,
                                                    double* __restrict__ out) {
  const int e = blockIdx.x * 16 + (threadIdx.x >> 4);
  const int r = threadIdx.x & 15;
  if (e >= ne) return;
  double acc = 0.0;
  for (int slot = 0; slot < 5; ++slot) {
    const int col = cols[slot * ne + e];
    if (col < 0) continue;
    const double2* zc = reinterpret_cast<const double2*>(y + 4 * (int64_t)col);
    const double2* Ab = AZ + ((int64_t)slot * 2 * ne + e) * 16 + r;
    const double2 a0 = Ab[0], a1 = Ab[(int64_t)ne * 16];
    acc += a0.x * zc[0].x + a0.y * zc[0].y + a1.x * zc[1].x + a1.y * zc[1].y;
  }
  out[16 * (int64_t)e + r] = acc;
}

// x += alpha p; r -= alpha q; partial (r, r) [flexible: (r,q), (p,r)]
template <bool FLEX>
__global__ __launch_bounds__(kThreads) void k_cg_update(int64_t n, const Scalars* __restrict__ sc,
                                                        const double* __restrict__ p,
                                                        const double* __restrict__ q,
                                                        double* __restrict__ x,
                                                        double* __restrict__ r,
                                                        double* __restrict__ part, Slots sl) {
  __shared__ double lds[4];
  const int slot = slot_id(sl);
  p += slot * sl.tstride;
  q += slot * sl.tstride;
  x += slot * sl.tstride;
  r += slot * sl.tstride;
  sc += slot;
  part += slot * kSlotPart;
  const double alpha = sc->alpha;
  double rr = 0.0, rq = 0.0, pr = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const double pi = p[i], qi = q[i];
    x[i] = x[i] + alpha * pi;
    const double ri = r[i] - alpha * qi;
    r[i] = ri;
    rr += ri * ri;
    if (FLEX) {
      rq += ri * qi;
      pr += pi * ri;
    }
  }
  const double t0 = block_sum(rr, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = t0;
  if (FLEX) {
    const double t1 = block_sum(rq, lds);
    if (threadIdx.x == 0) part[kPartStride + blockIdx.x] = t1;
    const double t2 = block_sum(pr, lds);
    if (threadIdx.x == 0) part[2 * kPartStride + blockIdx.x] = t2;
  }
}

__global__ __launch_bounds__(kThreads) void k_axpy_dot(int64_t n, double a,
                                                       const double* __restrict__ q,
                                                       double* __restrict__ r,
                                                       double* __restrict__ part) {
  __shared__ double lds[4];
  double rr = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const double ri = r[i] + a * q[i];
    r[i] = ri;
    rr += ri * ri;
  }
  const double t = block_sum(rr, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kThreads) void k_reduce(const double* __restrict__ part, int nb,
                                                     int op, Scalars* __restrict__ sc, Slots sl,
                                                     double aux, int iaux) {
  __shared__ double sm[kThreads];
  const int slot = slot_id(sl);
  part += slot * kSlotPart;
  sc += slot;
  if (op == kRedInnerR2 && sc->inner_done) return;   // the partials were not recomputed
  const int nslot = op == kRedB2Rho ? 2 : (op == kRedFcgBeta ? 3 : 1);
  double sums[3] = {0.0, 0.0, 0.0};
  for (int slot = 0; slot < nslot; ++slot) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += kThreads) v += part[slot * kPartStride + i];
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
      if (threadIdx.x < h) sm[threadIdx.x] += sm[threadIdx.x + h];
      __syncthreads();
    }
    sums[slot] = sm[0];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  switch (op) {
    case kRedB2Rho:
      sc->b2 = sums[0];
      sc->rho = sums[1];
      sc->dr = sums[1];
      break;
    case kRedAlpha:
    case kRedFcgAlpha: {
      const double pq = sums[0];
      sc->pq = pq;
      if (!(pq > 0.0) || !isfinite(pq)) {
        sc->breakdown = 1;
        sc->alpha = 0.0;
      } else {
        sc->alpha = (op == kRedAlpha ? sc->rho : sc->dr) / pq;
      }
      break;
    }
    case kRedBeta:
      sc->beta = sc->rho > 0.0 ? sums[0] / sc->rho : 0.0;
      sc->rho = sums[0];
      sc->dr = sums[0];
      break;
    case kRedFcgBeta: {
      const double beta = sc->pq > 0.0 ? -sums[1] / sc->pq : 0.0;
      sc->rho = sums[0];
      sc->beta = beta;
      sc->dr = sums[0] + beta * sums[2];
      break;
    }
    case kRedS2:
      sc->s2 = sums[0];
      sc->r2 = sums[0];
      break;
    case kRedInnerS2:
      sc->s2 = sums[0];
      sc->r2 = sums[0];
      sc->inner_lim2 = aux * sums[0];
      sc->inner_cycles = 0;
      sc->inner_done = !(sums[0] > aux * sums[0]) || iaux <= 0;
      break;
    case kRedInnerR2:
      sc->r2 = sums[0];
      sc->inner_cycles += 1;
      sc->inner_done = !(sums[0] > sc->inner_lim2) || sc->inner_cycles >= iaux;
      break;
    case kRedR2:
      sc->r2 = sums[0];
      break;
    case kRedRes:
      sc->res2 = sums[0];
      break;
    case kRedRho:
      sc->rho = sums[0];
      sc->dr = sums[0];
      break;
    case kRedDr:
      sc->dr = sums[0];
      break;
  }
}

// Partial (r, q_k) for the k-th window direction (blockIdx.y = k).
__global__ __launch_bounds__(kThreads) void k_fcg_dot(int64_t n, const double* __restrict__ r,
                                                      const double* const* __restrict__ qptr,
                                                      int first, int R, double* __restrict__ part) {
  __shared__ double lds[4];
  const int k = blockIdx.y;
  const double* q = qptr[(first + k) % R];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    acc += r[i] * q[i];
  const double t = block_sum(acc, lds);
  if (threadIdx.x == 0) part[(int64_t)k * gridDim.x + blockIdx.x] = t;
}

// coef[k] = -(sum of the k-th partials, in block order) / dq_k (dq == nullptr: -sum).
__global__ __launch_bounds__(kThreads) void k_fcg_coef(const double* __restrict__ part, int nb,
                                                       const double* __restrict__ dq, int first,
                                                       int R, double* __restrict__ coef) {
  __shared__ double lds[4];
  const int k = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += kThreads) acc += part[(int64_t)k * nb + b];
  const double t = block_sum(acc, lds);
  if (threadIdx.x == 0) coef[k] = dq ? -t / dq[(first + k) % R] : -t;
}

// d may alias r (in-place Gram-Schmidt update): element i is read before it is
// written by the same thread.
__global__ __launch_bounds__(kThreads) void k_fcg_direction(
    int64_t n, const double* r, const double* rdot, const double* const* __restrict__ dptr, int first,
    int m, int R, const double* __restrict__ coef, double* d, double* __restrict__ part) {
  __shared__ double lds[4];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const double ri = r[i];
    double di = ri;
    for (int k = 0; k < m; ++k) di += coef[k] * dptr[(first + k) % R][i];
    d[i] = di;
    acc += di * (rdot ? rdot[i] : ri);
  }
  const double t = block_sum(acc, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kThreads) void k_zt(int ne, const double* __restrict__ w,
                                                 double* __restrict__ s, Slots sl) {
  const int slot = slot_id(sl);
  w += slot * sl.tstride;
  s += slot * sl.sstride;
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (i >= 4 * (int64_t)ne) return;
  const int64_t e = i >> 2, j = i & 3;
  s[i] = (w[16 * e + j] + w[16 * e + 12 + j]) * kInvSqrt2;
}

__global__ __launch_bounds__(kThreads) void k_z(int ne, const double* __restrict__ y, double c,
                                                double* __restrict__ v) {
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (i >= 16 * (int64_t)ne) return;
  const int64_t e = i >> 4, cc = (i >> 2) & 3, j = i & 3;
  v[i] = (cc == 0 || cc == 3) ? (c * y[4 * e + j]) * kInvSqrt2 : 0.0;
}

// x = (xh - Z (c zt)) + Z (c zb)  (eq. (x_defl) with pi(b) reused)
__global__ __launch_bounds__(kThreads) void k_reconstruct(int ne, const double* __restrict__ xh,
                                                          const double* __restrict__ zt,
                                                          const double* __restrict__ zb,
                                                          const Scalars* __restrict__ sc,
                                                          double* __restrict__ x, Slots sl) {
  const int slot = slot_id(sl);
  xh += slot * sl.tstride;
  zt += slot * sl.sstride;
  zb += slot * sl.sstride;
  x += slot * sl.tstride;
  const double c = 2.0 / sc[slot].dt;
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (i >= 16 * (int64_t)ne) return;
  const int64_t e = i >> 4, cc = (i >> 2) & 3, j = i & 3;
  double v = xh[i];
  if (cc == 0 || cc == 3) {
    v = v - (c * zt[4 * e + j]) * kInvSqrt2;
    v = v + (c * zb[4 * e + j]) * kInvSqrt2;
  }
  x[i] = v;
}

// BDF2 right-hand side and warm start: f = (1/nu) (C (x) M_1)(4/3 s1 - 1/3 s2)
// + c F, x0 = 2 s1 - s2; thread (square, row).
__global__ __launch_bounds__(kThreads) void k_bdf2_rhs(int ne, const double* __restrict__ M1,
                                                       double inv_nu, const double* __restrict__ s1,
                                                       const double* __restrict__ s2,
                                                       const double* __restrict__ F, double c,
                                                       double* __restrict__ f,
                                                       double* __restrict__ x0) {
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (i >= 16 * (int64_t)ne) return;
  const int64_t e = i >> 4;
  const int r = int(i & 15), cc = r >> 2, j = r & 3;
  double u[16];
#pragma unroll
  for (int k = 0; k < 16; ++k)
    u[k] = 4.0 / 3.0 * s1[16 * e + k] - 1.0 / 3.0 * s2[16 * e + k];
  double m[4];
  ld4(M1 + 16 * e + 4 * j, m);
  double mu;
  if (cc == 0 || cc == 3) {
    mu = 0.5 * (m[0] * (u[0] - u[12]) + m[1] * (u[1] - u[13]) + m[2] * (u[2] - u[14]) +
                m[3] * (u[3] - u[15]));
    if (cc == 3) mu = -mu;
  } else {
    const int o = 4 * cc;
    mu = m[0] * u[o] + m[1] * u[o + 1] + m[2] * u[o + 2] + m[3] * u[o + 3];
  }
  f[i] = inv_nu * mu + c * F[i];
  x0[i] = 2.0 * s1[i] - s2[i];
}

__global__ __launch_bounds__(kThreads) void k_scale(int64_t n, double c,
                                                    const double* __restrict__ in,
                                                    double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (i < n) out[i] = c * in[i];
}

// ============================================================ inner refinement
// r = s - L64 z (first: r = s) in FP64, fJ = (T) r, partial ||r||^2.
// Thread (square e, row a): one workgroup = 64 squares.
template <typename T, bool FIRST>
__global__ __launch_bounds__(kThreads) void k_refine_residual(
    const double* __restrict__ Lc, int n, int ne, const double* __restrict__ s,
    const double* __restrict__ z, T* __restrict__ fJ, double* __restrict__ part, Slots sl,
    const Scalars* __restrict__ guard) {
  __shared__ double lds[4];
  if (guard && guard->inner_done) return;
  const int slot = slot_id(sl);
  s += slot * sl.sstride;
  if (z) z += slot * sl.sstride;
  fJ += slot * sl.lstride;
  part += slot * kSlotPart;
  const int a = threadIdx.x & 3;
  const int groups = (ne + 63) >> 6;
  double nrm = 0.0;
  for (int g = blockIdx.x; g < groups; g += gridDim.x) {
    const int e = (g << 6) + (threadIdx.x >> 2);
    if (e >= ne) continue;
    double acc = 0.0;
    if (!FIRST) {                // blocks of the square's class, neighbours from (ex, ey)
      const int ex = e % n, ey = e / n;
      const double* Le = Lc + square_class(ex, ey, n) * 80 + 4 * a;
#pragma unroll
      for (int sn = 0; sn < 5; ++sn) {
        const int dx = sn == 1 ? -1 : (sn == 2 ? 1 : 0), dy = sn == 3 ? -1 : (sn == 4 ? 1 : 0);
        if (ex + dx < 0 || ex + dx >= n || ey + dy < 0 || ey + dy >= n) continue;
        double l[4], zc[4];
        ld4(Le + 16 * sn, l);
        ld4(z + 4 * ((int64_t)e + dx + (int64_t)dy * n), zc);
        acc += l[0] * zc[0] + l[1] * zc[1] + l[2] * zc[2] + l[3] * zc[3];
      }
    }
    const int64_t i = 4 * (int64_t)e + a;
    const double rv = s[i] - acc;
    fJ[e * sl.lsq + a] = static_cast<T>(rv);
    nrm += rv * rv;
  }
  const double t = block_sum(nrm, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}


// ============================================================ multigrid levels
// out = L z (RES = false) or out = f - L z (RES = true); thread (square, row).
template <typename T, bool RES>
__global__ __launch_bounds__(kThreads) void k_lap(const T* __restrict__ L,
                                                  const int32_t* __restrict__ cols, int ne,
                                                  const T* __restrict__ f, const T* __restrict__ z,
                                                  T* __restrict__ out) {
  const int e = blockIdx.x * 64 + (threadIdx.x >> 2);
  const int a = threadIdx.x & 3;
  if (e >= ne) return;
  T acc = T(0);
#pragma unroll
  for (int slot = 0; slot < 5; ++slot) {
    const int col = cols[slot * ne + e];
    if (col < 0) continue;
    T l[4], zc[4];
    ld4(L + (((int64_t)slot * ne + e) * 4 + a) * 4, l);
    ld4(z + 4 * (int64_t)col, zc);
    acc += l[0] * zc[0] + l[1] * zc[1] + l[2] * zc[2] + l[3] * zc[3];
  }
  const int64_t i = 4 * (int64_t)e + a;
  out[i] = RES ? f[i] - acc : acc;
}

// Coefficient of coarse corner A at fine corner a of child ch: the coarse
// bilinear function at ((ch_x + a_x)/2, (ch_y + a_y)/2); values in
// {0, 1/4, 1/2, 1}, exact in any precision.
template <typename T>
__device__ inline T pcoef(int ch, int a, int A) {
  const int px = (ch & 1) + (a & 1), py = (ch >> 1) + (a >> 1);   // position in halves
  const int wx = (A & 1) ? px : 2 - px, wy = (A >> 1) ? py : 2 - py;
  return T(wx * wy) * T(0.25);
}

// rc = P^T r; thread per coarse dof (E, A)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_restrict(int nc, const T* __restrict__ r,
                                                       T* __restrict__ rc) {
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  const int64_t nec = (int64_t)nc * nc;
  if (i >= 4 * nec) return;
  const int64_t E = i >> 2;
  const int A = int(i & 3);
  const int EX = int(E % nc), EY = int(E / nc);
  const int nf = 2 * nc;
  T acc = T(0);
#pragma unroll
  for (int ch = 0; ch < 4; ++ch) {
    const int64_t e = (int64_t)(2 * EY + (ch >> 1)) * nf + 2 * EX + (ch & 1);
    T v[4];
    ld4(r + 4 * e, v);
#pragma unroll
    for (int a = 0; a < 4; ++a) acc += pcoef<T>(ch, a, A) * v[a];
  }
  rc[i] = acc;
}

// z += P ec; thread per fine dof (e, a)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_prolong(int nc, const T* __restrict__ ec,
                                                      T* __restrict__ z) {
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  const int nf = 2 * nc;
  if (i >= 4 * (int64_t)nf * nf) return;
  const int64_t e = i >> 2;
  const int a = int(i & 3);
  const int ex = int(e % nf), ey = int(e / nf);
  const int ch = (ex & 1) + 2 * (ey & 1);
  const int64_t E = (int64_t)(ey >> 1) * nc + (ex >> 1);
  T v[4];
  ld4(ec + 4 * E, v);
  T acc = T(0);
#pragma unroll
  for (int A = 0; A < 4; ++A) acc += pcoef<T>(ch, a, A) * v[A];
  z[i] = z[i] + acc;
}

// z = L_1^{-1} f with the FP64 inverse; one wavefront per row.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_coarse(const double* __restrict__ inv,
                                                     const T* __restrict__ f, T* __restrict__ z) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= 1024) return;
  const double* ir = inv + (int64_t)row * 1024;
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int j = lane + 64 * m;
    acc += ir[j] * static_cast<double>(f[j]);
  }
  acc = wave_sum(acc);
  if (lane == 0) z[row] = static_cast<T>(acc);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_fill(int64_t n, T v, T* __restrict__ x) {
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (i < n) x[i] = v;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_copy(int64_t n, const T* __restrict__ x,
                                                   T* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (i < n) y[i] = x[i];
}

}  // namespace

// ============================================================ launchers
hipError_t launch_astar(int mode, const double2* C, const int32_t* cols, const double* M1, int ne,
                        const double* x, const double* p_old, const double* b, const Scalars* sc,
                        double* p_new, double* w, double* s, double* part, hipStream_t st,
                        const Slots& sl, int count, hipEvent_t ev0, hipEvent_t ev1) {
  const dim3 grid(grid_for(ne, 16, kPartStride), count);
  // timed launches record their events in the dispatch packet itself
  switch (mode) {
    case kAstarPlain:
      hipExtLaunchKernelGGL(k_astar<kAstarPlain>, grid, dim3(kThreads), 0, st, ev0, ev1, 0, C, cols,
                            M1, ne, x, p_old, b, sc, p_new, w, s, part, sl);
      break;
    case kAstarDir:
      hipExtLaunchKernelGGL(k_astar<kAstarDir>, grid, dim3(kThreads), 0, st, ev0, ev1, 0, C, cols,
                            M1, ne, x, p_old, b, sc, p_new, w, s, part, sl);
      break;
    case kAstarFirst:
      hipExtLaunchKernelGGL(k_astar<kAstarFirst>, grid, dim3(kThreads), 0, st, ev0, ev1, 0, C, cols,
                            M1, ne, x, p_old, b, sc, p_new, w, s, part, sl);
      break;
    case kAstarResidual:
      hipExtLaunchKernelGGL(k_astar<kAstarResidual>, grid, dim3(kThreads), 0, st, ev0, ev1, 0, C,
                            cols, M1, ne, x, p_old, b, sc, p_new, w, s, part, sl);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int astar_blocks(int ne) { return grid_for(ne, 16, kPartStride); }

hipError_t launch_deflate(bool prologue, const double2* AZ, const int32_t* cols, int ne, double c,
                          const double* z, const double* w, const double* p, double* q,
                          double* p_out, double* part, hipStream_t st, const Slots& sl, int count) {
  const dim3 grid(grid_for(ne, 16, kPartStride), count);
  if (prologue)
    k_deflate<true><<<grid, kThreads, 0, st>>>(AZ, cols, ne, c, z, w, p, q, p_out, part, sl);
  else
    k_deflate<false><<<grid, kThreads, 0, st>>>(AZ, cols, ne, c, z, w, p, q, p_out, part, sl);
  return hipGetLastError();
}

hipError_t launch_adivz(const double2* AZ, const int32_t* cols, int ne, const double* y, double* out,
                        hipStream_t st) {
  k_adivz<<<grid_for(ne, 16, 1 << 30), kThreads, 0, st>>>(AZ, cols, ne, y, out);
  return hipGetLastError();
}

hipError_t launch_cg_update(bool flexible, int64_t nvec, const Scalars* sc, const double* p,
                            const double* q, double* x, double* r, double* part, int* nblocks,
                            hipStream_t st, const Slots& sl, int count) {
  const int gx = grid_for(nvec, kThreads * 4, 8192);
  *nblocks = gx;
  const dim3 grid(gx, count);
  if (flexible)
    k_cg_update<true><<<grid, kThreads, 0, st>>>(nvec, sc, p, q, x, r, part, sl);
  else
    k_cg_update<false><<<grid, kThreads, 0, st>>>(nvec, sc, p, q, x, r, part, sl);
  return hipGetLastError();
}

int fcg_coef_blocks(int64_t n) { return grid_for(n, kThreads * 8, 128); }

hipError_t launch_fcg_coef(int64_t n, const double* r, const double* const* qptr, const double* dq,
                           int first, int m, int R, double* part, double* coef, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  const int nb = fcg_coef_blocks(n);
  k_fcg_dot<<<dim3(nb, m), kThreads, 0, st>>>(n, r, qptr, first, R, part);
  k_fcg_coef<<<m, kThreads, 0, st>>>(part, nb, dq, first, R, coef);
  return hipGetLastError();
}

hipError_t launch_fcg_direction(int64_t n, const double* r, const double* rdot, const double* const* dptr, int first,
                                int m, int R, const double* coef, double* d, double* part,
                                int* nblocks, hipStream_t st) {
  const int grid = grid_for(n, kThreads * 4, 8192);
  *nblocks = grid;
  k_fcg_direction<<<grid, kThreads, 0, st>>>(n, r, rdot, dptr, first, m, R, coef, d, part);
  return hipGetLastError();
}

hipError_t launch_axpy_dot(int64_t nvec, double a, const double* q, double* r, double* part,
                           int* nblocks, hipStream_t st) {
  const int grid = grid_for(nvec, kThreads * 4, 8192);
  *nblocks = grid;
  k_axpy_dot<<<grid, kThreads, 0, st>>>(nvec, a, q, r, part);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* part, int nblocks, int op, Scalars* sc, hipStream_t st,
                         const Slots& sl, int count, double aux, int iaux) {
  k_reduce<<<dim3(1, count), kThreads, 0, st>>>(part, nblocks, op, sc, sl, aux, iaux);
  return hipGetLastError();
}

hipError_t launch_zt(int ne, const double* w, double* s, hipStream_t st, const Slots& sl, int count) {
  k_zt<<<dim3(grid_for(4 * (int64_t)ne, kThreads, 1 << 30), count), kThreads, 0, st>>>(ne, w, s, sl);
  return hipGetLastError();
}

hipError_t launch_z(int ne, const double* y, double scale, double* v, hipStream_t st) {
  k_z<<<grid_for(16 * (int64_t)ne, kThreads, 1 << 30), kThreads, 0, st>>>(ne, y, scale, v);
  return hipGetLastError();
}

hipError_t launch_reconstruct(int ne, const double* xh, const double* zt, const double* zb,
                              const Scalars* sc, double* x, hipStream_t st, const Slots& sl,
                              int count) {
  k_reconstruct<<<dim3(grid_for(16 * (int64_t)ne, kThreads, 1 << 30), count), kThreads, 0, st>>>(
      ne, xh, zt, zb, sc, x, sl);
  return hipGetLastError();
}

hipError_t launch_bdf2_rhs(int ne, const double* M1, double inv_nu, const double* s1,
                           const double* s2, const double* F, double c, double* f, double* x0,
                           hipStream_t st) {
  k_bdf2_rhs<<<grid_for(16 * (int64_t)ne, kThreads, 1 << 30), kThreads, 0, st>>>(ne, M1, inv_nu, s1, s2,
                                                                                F, c, f, x0);
  return hipGetLastError();
}

hipError_t launch_scale(int64_t n, double c, const double* in, double* out, hipStream_t st) {
  k_scale<<<grid_for(n, kThreads, 1 << 30), kThreads, 0, st>>>(n, c, in, out);
  return hipGetLastError();
}

int refine_blocks(int ne) { return grid_for(ne, 64, kPartStride); }

template <typename T>
hipError_t launch_refine_residual(bool first, const double* Lc64, int n, int ne, const double* s,
                                  const double* z, T* fJ, double* part, hipStream_t st,
                                  const Slots& sl, int count, const Scalars* guard) {
  if (!Lc64 || n < 3 || int64_t(n) * n != ne) return hipErrorInvalidValue;
  const dim3 grid(refine_blocks(ne), count);
  if (first)
    k_refine_residual<T, true><<<grid, kThreads, 0, st>>>(Lc64, n, ne, s, z, fJ, part, sl, guard);
  else
    k_refine_residual<T, false><<<grid, kThreads, 0, st>>>(Lc64, n, ne, s, z, fJ, part, sl, guard);
  return hipGetLastError();
}


template <typename T>
hipError_t launch_lap(bool residual, const T* L, const int32_t* cols, int ne, const T* f, const T* z,
                      T* out, hipStream_t st) {
  const int grid = grid_for(ne, 64, 1 << 30);
  if (residual)
    k_lap<T, true><<<grid, kThreads, 0, st>>>(L, cols, ne, f, z, out);
  else
    k_lap<T, false><<<grid, kThreads, 0, st>>>(L, cols, ne, f, z, out);
  return hipGetLastError();
}



template <typename T>
hipError_t launch_restrict(int nc, const T* r, T* rc, hipStream_t st) {
  k_restrict<T><<<grid_for(4 * (int64_t)nc * nc, kThreads, 1 << 30), kThreads, 0, st>>>(nc, r, rc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong(int nc, const T* ec, T* z, hipStream_t st) {
  k_prolong<T><<<grid_for(16 * (int64_t)nc * nc, kThreads, 1 << 30), kThreads, 0, st>>>(nc, ec, z);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse(const double* inv, const T* f, T* z, hipStream_t st) {
  k_coarse<T><<<256, kThreads, 0, st>>>(inv, f, z);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(int64_t n, T v, T* x, hipStream_t st) {
  k_fill<T><<<grid_for(n, kThreads, 1 << 30), kThreads, 0, st>>>(n, v, x);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(int64_t n, const T* x, T* y, hipStream_t st) {
  k_copy<T><<<grid_for(n, kThreads, 1 << 30), kThreads, 0, st>>>(n, x, y);
  return hipGetLastError();
}

#define DCG_INSTANTIATE(T)                                                                      \
  template hipError_t launch_refine_residual<T>(bool, const double*, int, int, const double*,  \
                                                const double*, T*, double*, hipStream_t,       \
                                                const Slots&, int, const Scalars*);            \
  template hipError_t launch_lap<T>(bool, const T*, const int32_t*, int, const T*, const T*, T*, \
                                    hipStream_t);                                              \
  template hipError_t launch_restrict<T>(int, const T*, T*, hipStream_t);                      \
  template hipError_t launch_prolong<T>(int, const T*, T*, hipStream_t);                       \
  template hipError_t launch_coarse<T>(const double*, const T*, T*, hipStream_t);              \
  template hipError_t launch_fill<T>(int64_t, T, T*, hipStream_t);                             \
  template hipError_t launch_copy<T>(int64_t, const T*, T*, hipStream_t);

DCG_INSTANTIATE(float)
DCG_INSTANTIATE(double)

}  // namespace dcg
