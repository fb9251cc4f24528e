// Fused multigrid kernels of the W-cycle (paper Algorithm 4 with the RAS
// smoother of Section 4.2).
//
// A RAS step z <- z + S_k (f - L_k z), S_k = sum_i R_i^T D_i (L_k)_i^{-1} R_i,
// is one launch of k_sweep.  The update sum_i R_i^T y_i of a step is left
// "pending": the tile outputs y_i stay in a buffer Y and the next kernel that
// needs z (the next step, the restriction, the prolongation of the parent
// level or the refinement update) adds them on the fly from the cover lists
// (the at most 3 blocks containing a square, in increasing block order).
// z and Y are double-buffered so that a launch reads the previous step's
// values while writing its own.  One W-cycle level visit with m1 = m2 = 2 is
// then five launches: two pre-smoothing steps, the fused residual +
// restriction, and two post-smoothing steps (the first one adding the
// prolongated coarse correction).
//
// k_sweep, per tile t (a group of WPT wavefronts):
//   1. z_new on the 52 squares within distance 1 of the tile (the 32 block
//      squares and their 20 outside neighbours): z_old + pending Y
//      [+ P (z_coarse + pending Y_coarse)], in LDS; the tile writes z_new of
//      its 16 core squares (every square is the core of exactly one tile);
//   2. r = f - L_k z_new on the 128 block dofs, in LDS;
//   3. Y_new[t] = D_t (L_k)_t^{-1} r: the factor rows are streamed with
//      16-byte loads, each lane owning 4 (FP32) or 2 (FP64) output columns,
//      the WPT wavefronts splitting the 128 rows and reducing in LDS.
#include <type_traits>

#include "kernels.hpp"
#include "mg_common.hpp"

namespace dcg {
namespace {
using namespace mg;

constexpr int kThreads = 256;

// z of square e after the pending update (and the pending prolongation).
// Pending tile outputs are stored per square: Ye[e][k][4] holds the output
// of the k-th block containing e (blocks in increasing order, unused slots
// stay zero), so the update is z + Ye[e][0] + Ye[e][1] + Ye[e][2].
template <typename T>
__device__ inline void add_pending(const T* Ye, int e, T z[4]) {
  T y0[4], y1[4], y2[4];
  ld4(Ye + 12 * (int64_t)e, y0);
  ld4(Ye + 12 * (int64_t)e + 4, y1);
  ld4(Ye + 12 * (int64_t)e + 8, y2);
#pragma unroll
  for (int j = 0; j < 4; ++j) z[j] = ((z[j] + y0[j]) + y1[j]) + y2[j];
}

// Row j of block s of the level operator at square e, from its class table.
template <typename T, typename Args>
__device__ __forceinline__ const T* op_row(const Args& a, int s, int e, int j) {
  return a.Lc + (square_class(e % a.n, e / a.n, a.n) * 5 + s) * 16 + 4 * j;
}

template <typename T>
__device__ inline void current_z(const SweepArgs<T>& a, int e, T z[4]) {
  if (a.has_z) {
    ld4(a.z_old + 4 * (int64_t)e, z);
  } else {
    z[0] = z[1] = z[2] = z[3] = T(0);
  }
  if (a.has_y) add_pending(a.Y_old, e, z);
  if (a.prol) {
    const int ex = e % a.n, ey = e / a.n;
    const int E = (ey >> 1) * a.nc + (ex >> 1);
    const int ch = (ex & 1) + 2 * (ey & 1);
    T ec[4];
    ld4(a.zc + 4 * (int64_t)E, ec);
    if (a.c_has_y) add_pending(a.Yc, E, ec);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      z[j] += pcoef<T>(ch, j, 0) * ec[0] + pcoef<T>(ch, j, 1) * ec[1] +
              pcoef<T>(ch, j, 2) * ec[2] + pcoef<T>(ch, j, 3) * ec[3];
  }
}

// Packed symmetric tile inverse: (L_k)_t^{-1} is stored as its 36 upper
// 16 x 16 blocks (P <= Q, row by row), block b = (blk_p(b), blk_q(b)).  Lane
// l of a wavefront holds row l / 4, columns 4 (l % 4) .. + 3 of a block (the
// 4 consecutive values at offset 4 l), so a block is one 16-byte load per
// lane (FP32) or two (FP64).  A block contributes B r_Q to u_P and, off the
// diagonal, B^T r_P to u_Q; both partial sums stay in registers until one
// reduction per tile.
__host__ __device__ constexpr int blk_p(int b) {
  int p = 0;
  while (b >= 8 - p) { b -= 8 - p; ++p; }
  return p;
}
__host__ __device__ constexpr int blk_q(int b) {
  int p = 0;
  while (b >= 8 - p) { b -= 8 - p; ++p; }
  return p + b;
}

template <typename T, int B>
__device__ __forceinline__ void blk_fma(const T v[4], const T* r, int ri, int cg, T (&rowp)[8],
                                        T (&colp)[8][4]) {
  constexpr int P = blk_p(B), Q = blk_q(B);
  const T* rq = r + 16 * Q + 4 * cg;
  rowp[P] += v[0] * rq[0] + v[1] * rq[1] + v[2] * rq[2] + v[3] * rq[3];
  if constexpr (P != Q) {
    const T rp = r[16 * P + ri];
    colp[Q][0] += v[0] * rp;
    colp[Q][1] += v[1] * rp;
    colp[Q][2] += v[2] * rp;
    colp[Q][3] += v[3] * rp;
  }
}

// Blocks B0 .. B0 + NB - 1 of one wavefront; the first NP come prefetched.
template <typename T, int B0, int NB, int NP, int K = 0>
__device__ __forceinline__ void wave_blocks(const T* Ft, const T (&pf)[NP][4], const T* r, int lane,
                                            T (&rowp)[8], T (&colp)[8][4]) {
  if constexpr (K < NB) {
    const int ri = lane >> 2, cg = lane & 3;
    if constexpr (K < NP) {
      blk_fma<T, B0 + K>(pf[K], r, ri, cg, rowp, colp);
    } else {
      T v[4];
      ld4(Ft + (B0 + K) * 256 + 4 * lane, v);
      blk_fma<T, B0 + K>(v, r, ri, cg, rowp, colp);
    }
    wave_blocks<T, B0, NB, NP, K + 1>(Ft, pf, r, lane, rowp, colp);
  }
}

template <typename T, int WPT>
__global__ __launch_bounds__(kThreads) void k_sweep(SweepArgs<T> a) {
  constexpr int TPB = 4 / WPT;          // tiles per workgroup
  constexpr int G = 64 * WPT;           // threads per tile
  constexpr int ROWS = 128 / WPT;       // factor rows per wavefront
  constexpr int RPT = (128 + G - 1) / G;  // residual rows per thread
  constexpr int NBW = 36 / WPT;         // packed blocks per wavefront
  constexpr int NP = NBW < 8 ? NBW : 8; // blocks prefetched before the residual
  __shared__ T zn[TPB][52][4];
  __shared__ T rl[TPB][128];
  __shared__ T rp[4][8][16];            // row-part sums per wavefront
  __shared__ T cp[4][8][16][4];         // column-part sums per wavefront
  const int tl = threadIdx.x / G;       // tile within the workgroup
  const int g = threadIdx.x % G;        // thread within the tile group
  const int wave = g >> 6, lane = threadIdx.x & 63;
  const int t = xcd_band_index(blockIdx.x, gridDim.x) * TPB + tl;
  const bool live = t < a.tiles;
  const bool need_z = a.has_z || a.has_y || a.prol;

  // Every global load of the step is issued up front (one memory round
  // trip): the first factor blocks, the operator rows of this thread's
  // residual rows, and the iterate of the squares this thread resolves.
  const T* Ft = a.F + (int64_t)(live ? a.fcls[t] : 0) * (36 * 256);
  T pf[NP][4];
  if (live) {
#pragma unroll
    for (int k = 0; k < NP; ++k) ld4(Ft + (wave * NBW + k) * 256 + 4 * lane, pf[k]);
  }
  // The operator rows are hoisted too on the latency-bound small levels; on
  // the streaming levels (one wavefront per tile) they are loaded at use to
  // keep the register count, and with it the occupancy, where it is.
  constexpr bool HOIST = WPT > 1;
  constexpr int RH = HOIST ? RPT : 1;
  T lrow[RH][5][4];
  T fval[RPT];
  int nb[RPT][5];                       // extended slot of each neighbour, -1 = none
  int esq[RPT];
  if (live) {
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int i = g + u * G;
      fval[u] = T(0);
      esq[u] = -1;
      for (int s = 0; s < 5; ++s) nb[u][s] = -1;
      if (i < 128) {
        const int p = i >> 2, j = i & 3;
        const int e = ext_square(t, p, a.n);
        esq[u] = e;
        if (e >= 0) {
          fval[u] = a.f[4 * (int64_t)e + j];
          const int ex = e % a.n, ey = e / a.n;
#pragma unroll
          for (int s = 0; s < 5; ++s) {
            const int dx = s == 1 ? -1 : (s == 2 ? 1 : 0), dy = s == 3 ? -1 : (s == 4 ? 1 : 0);
            const bool in = ex + dx >= 0 && ex + dx < a.n && ey + dy >= 0 && ey + dy < a.n;
            if (in && need_z) {
              nb[u][s] = nbr_slot(p, s);
              if constexpr (HOIST) ld4(op_row<T>(a, s, e, j), lrow[u][s]);
            }
          }
        }
      }
    }
  }
  if (live && need_z) {
    for (int q = g; q < 52; q += G) {
      const int e = ext_square(t, q, a.n);
      T z[4] = {T(0), T(0), T(0), T(0)};
      if (e >= 0) current_z(a, e, z);
      zn[tl][q][0] = z[0]; zn[tl][q][1] = z[1]; zn[tl][q][2] = z[2]; zn[tl][q][3] = z[3];
    }
  }
  __syncthreads();
  if (live && a.write_z && g < 16) {
    const int e = ext_square(t, g, a.n);
    const T v[4] = {zn[tl][g][0], zn[tl][g][1], zn[tl][g][2], zn[tl][g][3]};
    st4(a.z_new + 4 * (int64_t)e, v);
  }
  if (live) {
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int i = g + u * G;
      if (i >= 128) continue;
      T acc = T(0);
#pragma unroll
      for (int s = 0; s < 5; ++s) {
        const int q = nb[u][s];
        if (q < 0) continue;
        T l[4];
        if constexpr (HOIST) {
          l[0] = lrow[u][s][0]; l[1] = lrow[u][s][1]; l[2] = lrow[u][s][2]; l[3] = lrow[u][s][3];
        } else {
          ld4(op_row<T>(a, s, esq[u], i & 3), l);
        }
        acc += l[0] * zn[tl][q][0] + l[1] * zn[tl][q][1] + l[2] * zn[tl][q][2] + l[3] * zn[tl][q][3];
      }
      rl[tl][i] = fval[u] - acc;
    }
  }
  __syncthreads();

  // u = (L_k)_t^{-1} r from the packed blocks, then Y_t = D_t u
  T rowp[8], colp[8][4];
#pragma unroll
  for (int P = 0; P < 8; ++P) {
    rowp[P] = T(0);
    colp[P][0] = colp[P][1] = colp[P][2] = colp[P][3] = T(0);
  }
  if (live) {
    const T* r = rl[tl];
    if constexpr (WPT == 1) {
      wave_blocks<T, 0, NBW, NP>(Ft, pf, r, lane, rowp, colp);
    } else if constexpr (WPT == 2) {
      if (wave == 0) wave_blocks<T, 0, NBW, NP>(Ft, pf, r, lane, rowp, colp);
      else wave_blocks<T, NBW, NBW, NP>(Ft, pf, r, lane, rowp, colp);
    } else {
      if (wave == 0) wave_blocks<T, 0, NBW, NP>(Ft, pf, r, lane, rowp, colp);
      else if (wave == 1) wave_blocks<T, NBW, NBW, NP>(Ft, pf, r, lane, rowp, colp);
      else if (wave == 2) wave_blocks<T, 2 * NBW, NBW, NP>(Ft, pf, r, lane, rowp, colp);
      else wave_blocks<T, 3 * NBW, NBW, NP>(Ft, pf, r, lane, rowp, colp);
    }
  }
  // row parts: the 4 lanes of a row; column parts: the 4 rows of a 16-lane
  // group, then across the 4 groups and the wavefronts in LDS
#pragma unroll
  for (int P = 0; P < 8; ++P) {
    rowp[P] += __shfl_xor(rowp[P], 1, 64);
    rowp[P] += __shfl_xor(rowp[P], 2, 64);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      colp[P][k] += __shfl_xor(colp[P][k], 4, 64);
      colp[P][k] += __shfl_xor(colp[P][k], 8, 64);
    }
  }
  const int w = threadIdx.x >> 6;
  if ((lane & 3) == 0) {
#pragma unroll
    for (int P = 0; P < 8; ++P) rp[w][P][lane >> 2] = rowp[P];
  }
  if ((lane & 12) == 0) {
    const int cg = lane & 3, m = lane >> 4;
#pragma unroll
    for (int Q = 0; Q < 8; ++Q)
#pragma unroll
      for (int k = 0; k < 4; ++k) cp[w][Q][4 * cg + k][m] = colp[Q][k];
  }
  __syncthreads();
  if (live) {
    for (int o = g; o < 128; o += G) {        // every output of the tile
      const int P = o >> 4, i = o & 15;
      T u = T(0);
      for (int ww = tl * WPT; ww < (tl + 1) * WPT; ++ww)
        u += rp[ww][P][i] + ((cp[ww][P][i][0] + cp[ww][P][i][1]) + (cp[ww][P][i][2] + cp[ww][P][i][3]));
      const int p = o >> 2;
      const int e = ext_square(t, p, a.n);
      if (e >= 0) a.Y_new[4 * (int64_t)a.dst[(int64_t)t * 32 + p] + (o & 3)] = a.dw[e] * u;
    }
  }
}

// Pending update + residual + restriction: z_new = z_old + pending Y (written
// for every square), r = f - L z_new, rc = P^T r.  One workgroup = 16
// coarse squares x (4 children x 4 dofs).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_restrict_res(RestrictArgs<T> a) {
  __shared__ T rl[kThreads];
  const int E = xcd_band_index(blockIdx.x, gridDim.x) * 16 + (threadIdx.x >> 4);
  const int ch = (threadIdx.x >> 2) & 3, j = threadIdx.x & 3;
  const int nc = a.n >> 1;
  const bool live = E < nc * nc;
  T rv = T(0);
  if (live) {
    const int EX = E % nc, EY = E / nc;
    const int ex = 2 * EX + (ch & 1), ey = 2 * EY + (ch >> 1);
    const int e = ey * a.n + ex;
    T acc = T(0);
#pragma unroll
    for (int s = 0; s < 5; ++s) {
      const int dx = s == 1 ? -1 : (s == 2 ? 1 : 0), dy = s == 3 ? -1 : (s == 4 ? 1 : 0);
      if (ex + dx < 0 || ex + dx >= a.n || ey + dy < 0 || ey + dy >= a.n) continue;
      const int c = e + dy * a.n + dx;
      T z[4] = {T(0), T(0), T(0), T(0)};
      if (a.has_z) ld4(a.z_old + 4 * (int64_t)c, z);
      if (a.has_y) add_pending(a.Y_old, c, z);
      if (s == 0 && a.write_z) a.z_new[4 * (int64_t)e + j] = z[j];
      T l[4];
      ld4(op_row<T>(a, s, e, j), l);
      acc += l[0] * z[0] + l[1] * z[1] + l[2] * z[2] + l[3] * z[3];
    }
    rv = a.f[4 * (int64_t)e + j] - acc;
  }
  rl[threadIdx.x] = rv;
  __syncthreads();
  const int k = threadIdx.x & 15;
  if (live && k < 4) {
    const int base = threadIdx.x & ~15;
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) acc += pcoef<T>(c, jj, k) * rl[base + 4 * c + jj];
    a.rc[4 * (int64_t)E + k] = acc;
  }
}

// out = z (or 0) + pending Y: resolves a level's pending update.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_resolve(int ne, int has_z, const T* __restrict__ z,
                                                      const T* __restrict__ Ye, T* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (i >= 4 * (int64_t)ne) return;
  const int64_t e = i >> 2;
  const int j = int(i & 3);
  const T v = has_z ? z[i] : T(0);
  out[i] = ((v + Ye[12 * e + j]) + Ye[12 * e + 4 + j]) + Ye[12 * e + 8 + j];
}

// z64 (+)= (double)(z (or 0) + pending Y): the finest-level W-cycle result
// resolved in the level type and added to the FP64 inner iterate.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_refine_add(int ne, int first, int has_z, int has_y,
                                                         const T* __restrict__ z,
                                                         const T* __restrict__ Ye,
                                                         double* __restrict__ z64, Slots sl) {
  const int slot = sl.list ? sl.list[blockIdx.y] : 0;
  z += slot * sl.lstride;
  Ye += slot * sl.lstride;
  z64 += slot * sl.sstride;
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (i >= 4 * (int64_t)ne) return;
  const int64_t e = i >> 2;
  const int j = int(i & 3);
  const int64_t q = sl.lsq;
  T v = has_z ? z[e * q + j] : T(0);
  if (has_y) v = ((v + Ye[3 * e * q + j]) + Ye[(3 * e + 1) * q + j]) + Ye[(3 * e + 2) * q + j];
  const double d = static_cast<double>(v);
  z64[i] = first ? d : z64[i] + d;
}

}  // namespace

template <typename T>
hipError_t launch_sweep(const SweepArgs<T>& a, int wpt, hipStream_t st) {
  const int tpb = 4 / wpt;
  const int grid = (a.tiles + tpb - 1) / tpb;
  switch (wpt) {
    case 1: k_sweep<T, 1><<<grid, kThreads, 0, st>>>(a); break;
    case 2: k_sweep<T, 2><<<grid, kThreads, 0, st>>>(a); break;
    case 4: k_sweep<T, 4><<<grid, kThreads, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict_res(const RestrictArgs<T>& a, hipStream_t st) {
  const int nc = a.n / 2;
  const int grid = (nc * nc + 15) / 16;
  k_restrict_res<T><<<grid, kThreads, 0, st>>>(a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_resolve(int ne, bool has_z, const T* z, const T* Ye, T* out, hipStream_t st) {
  const int64_t n = 4 * (int64_t)ne;
  k_resolve<T><<<int((n + kThreads - 1) / kThreads), kThreads, 0, st>>>(ne, has_z, z, Ye, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_refine_add(int ne, bool first, bool has_z, bool has_y, const T* z, const T* Ye,
                             double* z64, hipStream_t st, const Slots& sl, int count) {
  const int64_t n = 4 * (int64_t)ne;
  k_refine_add<T><<<dim3(int((n + kThreads - 1) / kThreads), count), kThreads, 0, st>>>(
      ne, first, has_z, has_y, z, Ye, z64, sl);
  return hipGetLastError();
}

#define DCG_MG_INSTANTIATE(T)                                                                 \
  template hipError_t launch_sweep<T>(const SweepArgs<T>&, int, hipStream_t);                 \
  template hipError_t launch_restrict_res<T>(const RestrictArgs<T>&, hipStream_t);            \
  template hipError_t launch_resolve<T>(int, bool, const T*, const T*, T*, hipStream_t);      \
  template hipError_t launch_refine_add<T>(int, bool, bool, bool, const T*, const T*, double*, \
                                           hipStream_t, const Slots&, int);

DCG_MG_INSTANTIATE(float)
DCG_MG_INSTANTIATE(double)

}  // namespace dcg
