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
#include <hip/hip_ext.h>

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

// One RAS step for a GX x GX group of tiles per workgroup (4 GX x 4 GX core
// squares), the tile solves as MFMA products.  On the uniform grid every
// tile of a group has one of a few local problems (its class: interior,
// edge, corner), so the group's residuals form a 128 x GX^2 matrix U whose
// columns of one class are multiplied by that class's inverse in one
// 16 x 16 x 4 MFMA product (columns of other classes enter as zeros, which
// adds nothing); a boundary group runs one masked product per class present.
// Compared with one tile per wavefront (k_sweep), the class inverse is read
// once per group instead of once per tile, z is loaded once per frame square
// instead of once per neighbouring tile, and the residual is formed once per
// square instead of once per block containing it.
//
// The step is bound by memory latency, so every load that does not depend
// on another is issued first (the iterate, pending outputs and, in the
// first post-smoothing step (PROL), the coarse correction of the frame; f;
// the operator's class table; the tile classes), and the class inverse,
// which needs the first tile's class, as soon as the frame registers are
// free.  The pending slot and weight of an output follow from the tile
// geometry (checked against the host's cover lists when the context is
// built), so the outputs need no table.
//   1. z_new on the frame of squares within distance 2 of the group core
//      (z_old + pending Y [+ P (z_coarse + pending Y_coarse)]), in LDS; the
//      core squares are written to z_new;
//   2. r = f - L_k z_new on the block squares (core + 1), in LDS, one
//      thread per square, the operator rows from the class table in LDS;
//   3. per class: wavefront w computes row blocks w and 7 - w of
//      (L_k)_c^{-1} U_c, 8 column blocks x 4 k-steps, the operand fragments
//      read in MFMA order (one 16 / 32 byte vector per lane and fragment);
//   4. Y_t = D_t u_t written to the pending slot of each block square.
template <typename T, bool PROL>
__device__ __forceinline__ void load_frame(const SweepArgs<T>& a, int e, bool ok, T (&v)[PROL ? 8 : 4][4]) {
  // v[0] z_old, v[1..3] pending Y, v[4] coarse z, v[5..7] coarse pending Y
#pragma unroll
  for (int i = 0; i < (PROL ? 8 : 4); ++i) v[i][0] = v[i][1] = v[i][2] = v[i][3] = T(0);
  if (!ok) return;
  if (a.has_z) ld4(a.z_old + 4 * (int64_t)e, v[0]);
  if (a.has_y) {
    ld4(a.Y_old + 12 * (int64_t)e, v[1]);
    ld4(a.Y_old + 12 * (int64_t)e + 4, v[2]);
    ld4(a.Y_old + 12 * (int64_t)e + 8, v[3]);
  }
  if constexpr (PROL) {
    const int ex = e % a.n, ey = e / a.n;
    const int E = (ey >> 1) * a.nc + (ex >> 1);
    ld4(a.zc + 4 * (int64_t)E, v[4]);
    if (a.c_has_y) {
      ld4(a.Yc + 12 * (int64_t)E, v[5]);
      ld4(a.Yc + 12 * (int64_t)E + 4, v[6]);
      ld4(a.Yc + 12 * (int64_t)E + 8, v[7]);
    }
  }
}

// z_new of square e from its loaded values (the order of current_z)
template <typename T, bool PROL>
__device__ __forceinline__ void combine_frame(const SweepArgs<T>& a, int e,
                                              const T (&v)[PROL ? 8 : 4][4], T z[4]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) z[j] = v[0][j];
  if (a.has_y) {
#pragma unroll
    for (int j = 0; j < 4; ++j) z[j] = ((z[j] + v[1][j]) + v[2][j]) + v[3][j];
  }
  if constexpr (PROL) {
    T ec[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) ec[j] = v[4][j];
    if (a.c_has_y) {
#pragma unroll
      for (int j = 0; j < 4; ++j) ec[j] = ((ec[j] + v[5][j]) + v[6][j]) + v[7][j];
    }
    const int ch = (e % a.n & 1) + 2 * (e / a.n & 1);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      z[j] += pcoef<T>(ch, j, 0) * ec[0] + pcoef<T>(ch, j, 1) * ec[1] +
              pcoef<T>(ch, j, 2) * ec[2] + pcoef<T>(ch, j, 3) * ec[3];
  }
}

template <typename T, int GX, bool PROL>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : 2)))
void k_sweep_g(SweepArgs<T> a) {
  using V = typename Mfma<T>::v4;
  constexpr int C = 4 * GX;        // core squares per side
  constexpr int FS = C + 4;        // z frame: core +- 2
  constexpr int RS = C + 2;        // residual frame: core +- 1
  constexpr int NT = GX * GX;      // tiles = MFMA columns in use
  constexpr int NZ = (FS * FS + kThreads - 1) / kThreads;   // frame squares per thread
  constexpr int NR = (RS * RS + kThreads - 1) / kThreads;   // residual squares per thread
  constexpr int NV = PROL ? 8 : 4; // loaded 4-vectors per frame square
  constexpr int NLC = 9 * 5 * 16;  // class table of the level operator
  constexpr int NLU = (NLC / 4 + kThreads - 1) / kThreads;
  // class-inverse fragments requested ahead of the MFMA loop
  constexpr int PD = 4;
  static_assert(NT <= 16, "at most 16 tiles per group");
  __shared__ __align__(16) T zf[FS * FS][4];
  __shared__ __align__(16) T rf[RS * RS][4];
  __shared__ __align__(16) T lc[NLC];
  __shared__ int tcls[NT];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tpr = a.n >> 2, gpr = tpr / GX, G0 = gpr * gpr;
  // workgroups 0 .. G0 - 1 run the class of each group's first tile, the
  // extra ones a further class of the group in the extra list
  const bool extra = (int)blockIdx.x >= G0;
  const int g = extra ? a.gextra[2 * (blockIdx.x - G0)] : xcd_band_index(blockIdx.x, G0);
  const int X0 = C * (g % gpr), Y0 = C * (g / gpr);
  const int t00 = GX * (g / gpr) * tpr + GX * (g % gpr);
  const bool need_z = a.has_z || a.has_y || PROL;
  const int r = lane & 15, k = lane >> 4;
  const int Pw[2] = {wave, 7 - wave};

  // ---- every load that needs no other one, in one batch: the tile
  // classes, the operator's class table, f, and the frame values
  const int c0 = extra ? a.gextra[2 * (blockIdx.x - G0) + 1] : a.fcls[t00];
  const int tc = tid < NT ? a.fcls[t00 + (tid / GX) * tpr + tid % GX] : 0;
  T lcv[NLU][4];
#pragma unroll
  for (int u = 0; u < NLU; ++u)
    if (tid + u * kThreads < NLC / 4) ld4(a.Lc + 4 * (tid + u * kThreads), lcv[u]);
  T fr[NR][4];
#pragma unroll
  for (int u = 0; u < NR; ++u) {
    const int q = tid + u * kThreads;
    const int rx = q % RS, ry = q / RS;
    const int X = X0 + rx - 1, Y = Y0 + ry - 1;
    fr[u][0] = fr[u][1] = fr[u][2] = fr[u][3] = T(0);
    const bool corner = (rx == 0 || rx == RS - 1) && (ry == 0 || ry == RS - 1);
    if (q < RS * RS && !corner && X >= 0 && Y >= 0 && X < a.n && Y < a.n)
      ld4(a.f + 4 * ((int64_t)Y * a.n + X), fr[u]);
  }
  T fv[NZ][NV][4];
  if (need_z) {
#pragma unroll
    for (int u = 0; u < NZ; ++u) {
      const int q = tid + u * kThreads;
      const int fx = q % FS, fy = q / FS;
      const int X = X0 + fx - 2, Y = Y0 + fy - 2;
      const bool ox = fx < 2 || fx >= FS - 2, oy = fy < 2 || fy >= FS - 2;
      // the four 2 x 2 frame corners hold no neighbour of a block square,
      // except their inner squares (the diagonal corners of the layer)
      const bool unused = ox && oy && !((fx == 1 || fx == FS - 2) && (fy == 1 || fy == FS - 2));
      const bool ok = q < FS * FS && !unused && X >= 0 && Y >= 0 && X < a.n && Y < a.n;
      load_frame<T, PROL>(a, ok ? Y * a.n + X : 0, ok, fv[u]);
    }
  }

  // ---- LDS: tile classes, class table, z_new on the frame
  if (tid < NT) tcls[tid] = tc;
#pragma unroll
  for (int u = 0; u < NLU; ++u)
    if (tid + u * kThreads < NLC / 4) st4(&lc[4 * (tid + u * kThreads)], lcv[u]);
  if (need_z) {
#pragma unroll
    for (int u = 0; u < NZ; ++u) {
      const int q = tid + u * kThreads;
      if (q >= FS * FS) continue;
      const int fx = q % FS, fy = q / FS;
      const int X = X0 + fx - 2, Y = Y0 + fy - 2;
      T z[4];
      combine_frame<T, PROL>(a, Y * a.n + X, fv[u], z);
      st4(&zf[q][0], z);
      const bool core = fx >= 2 && fx < FS - 2 && fy >= 2 && fy < FS - 2;
      if (a.write_z && !extra && core) st4(a.z_new + 4 * ((int64_t)Y * a.n + X), z);
    }
  }

  // ---- the class inverse of this workgroup's class, requested now that the frame
  // registers are free; it arrives while the residual is formed
  auto load_q = [&](const T* F, int Q, T (&dst)[2][4]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) ld4(F + ((Pw[h] * 8 + Q) * 64 + lane) * 4, dst[h]);
  };
  T av[PD][2][4];
  {
    const T* F0 = a.Fm + (int64_t)c0 * (64 * 256);
#pragma unroll
    for (int Q = 0; Q < PD; ++Q) load_q(F0, Q, av[Q]);
  }
  __syncthreads();

  // ---- residual on the block squares
#pragma unroll
  for (int u = 0; u < NR; ++u) {
    const int q = tid + u * kThreads;
    if (q >= RS * RS) continue;
    const int rx = q % RS, ry = q / RS;
    const int X = X0 + rx - 1, Y = Y0 + ry - 1;
    const bool corner = (rx == 0 || rx == RS - 1) && (ry == 0 || ry == RS - 1);
    T res[4] = {fr[u][0], fr[u][1], fr[u][2], fr[u][3]};
    if (need_z && !corner && X >= 0 && Y >= 0 && X < a.n && Y < a.n) {
      const T* lr = lc + square_class(X, Y, a.n) * 80;
      T acc[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int s = 0; s < 5; ++s) {
        const int dx = s == 1 ? -1 : (s == 2 ? 1 : 0), dy = s == 3 ? -1 : (s == 4 ? 1 : 0);
        if (X + dx < 0 || X + dx >= a.n || Y + dy < 0 || Y + dy >= a.n) continue;
        T zq[4];
        ld4(zf[(ry + 1 + dy) * FS + rx + 1 + dx], zq);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const T* l = lr + 16 * s + 4 * j;
          acc[j] += l[0] * zq[0] + l[1] * zq[1] + l[2] * zq[2] + l[3] * zq[3];
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) res[j] -= acc[j];
    }
    st4(&rf[q][0], res);
  }
  __syncthreads();

  // ---- MFMA product of the class inverse with the residual columns of the
  // tiles of this class (other columns enter as zeros); the B operand of
  // lane (r, k) is tile r's residual at block slot 4 Q + k
  const int rtx = 4 * (r % GX) + 1, rty = 4 * (r / GX) + 1;   // tile r in the residual frame
  const bool col = r < NT && tcls[r < NT ? r : 0] == c0;
  const T* Fc = a.Fm + (int64_t)c0 * (64 * 256);
  V acc0 = {T(0), T(0), T(0), T(0)}, acc1 = {T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int Q = 0; Q < 8; ++Q) {
    T bq[4] = {T(0), T(0), T(0), T(0)};
    if (col) {
      int px, py;
      slot_pos(4 * Q + k, px, py);
      ld4(&rf[(rty + py) * RS + rtx + px][0], bq);
    }
    T aq[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) aq[h][kk] = av[Q % PD][h][kk];
    if (Q + PD < 8) load_q(Fc, Q + PD, av[Q % PD]);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      acc0 = Mfma<T>::mac(aq[0][kk], bq[kk], acc0);
      acc1 = Mfma<T>::mac(aq[1][kk], bq[kk], acc1);
    }
  }

  // ---- outputs: FP32 lanes hold rows 4 k + v of row block P (block slot
  // 4 P + k, corner v), FP64 lanes rows 4 v + k (slot 4 P + v, corner k)
  if (!col) return;
  const int t = t00 + (r / GX) * tpr + r % GX;
  constexpr int NO = sizeof(T) == 4 ? 1 : 4;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const V& acc = h == 0 ? acc0 : acc1;
#pragma unroll
    for (int v = 0; v < NO; ++v) {
      const int p = NO == 1 ? 4 * Pw[h] + k : 4 * Pw[h] + v;
      int px, py;
      slot_pos(p, px, py);
      const int X = X0 + rtx - 1 + px, Y = Y0 + rty - 1 + py;
      if (X < 0 || Y < 0 || X >= a.n || Y >= a.n) continue;
      // blocks containing (X, Y): its core tile T and the neighbour tile on
      // each side where the square lies on T's core edge; the pending slot
      // is this tile's rank among them in increasing order
      const int TX = X >> 2, TY = Y >> 2, lx = X & 3, ly = Y & 3, Tc = TY * tpr + TX;
      const bool below = ly == 0 && TY > 0, left = lx == 0 && TX > 0;
      const bool right = lx == 3 && TX < tpr - 1, above = ly == 3 && TY < tpr - 1;
      const int count = 1 + below + left + right + above;
      const int rank = (below && Tc - tpr < t) + (left && Tc - 1 < t) + (Tc < t) +
                       (right && Tc + 1 < t) + (above && Tc + tpr < t);
      const T w = count == 1 ? T(1) : (count == 2 ? T(0.5) : T(1.0 / 3.0));
      const int64_t slot = 3 * ((int64_t)Y * a.n + X) + rank;
      if constexpr (NO == 1) {
        const T y[4] = {w * acc[0], w * acc[1], w * acc[2], w * acc[3]};
        st4(a.Y_new + 4 * slot, y);
      } else {
        a.Y_new[4 * slot + k] = w * acc[v];
      }
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
                                                         double* __restrict__ z64, Slots sl,
                                                         const Scalars* __restrict__ guard) {
  if (guard && guard->inner_done) return;
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
hipError_t launch_sweep_g(const SweepArgs<T>& a, int gx, hipStream_t st, hipEvent_t ev0,
                          hipEvent_t ev1) {
  const int tpr = a.n / 4;
  if (gx <= 0 || tpr % gx || a.tiles != tpr * tpr) return hipErrorInvalidValue;
  int grid = (tpr / gx) * (tpr / gx);
  if (!a.Fm || (a.nextra > 0 && !a.gextra)) return hipErrorInvalidValue;
  grid += a.nextra;
  // timed launches record their events in the dispatch packet itself
#define DCG_SWEEP_G(G, P)                                                                        \
  hipExtLaunchKernelGGL(k_sweep_g<T, G, P>, dim3(grid), dim3(kThreads), 0, st, ev0, ev1, 0, a)
  switch (gx * 2 + (a.prol ? 1 : 0)) {
    case 2: DCG_SWEEP_G(1, false); break;
    case 3: DCG_SWEEP_G(1, true); break;
    case 4: DCG_SWEEP_G(2, false); break;
    case 5: DCG_SWEEP_G(2, true); break;
    case 8: DCG_SWEEP_G(4, false); break;
    case 9: DCG_SWEEP_G(4, true); break;
    default: return hipErrorInvalidValue;
  }
#undef DCG_SWEEP_G
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
                             double* z64, hipStream_t st, const Slots& sl, int count,
                             const Scalars* guard) {
  const int64_t n = 4 * (int64_t)ne;
  k_refine_add<T><<<dim3(int((n + kThreads - 1) / kThreads), count), kThreads, 0, st>>>(
      ne, first, has_z, has_y, z, Ye, z64, sl, guard);
  return hipGetLastError();
}

#define DCG_MG_INSTANTIATE(T)                                                                 \
  template hipError_t launch_sweep<T>(const SweepArgs<T>&, int, hipStream_t);                 \
  template hipError_t launch_sweep_g<T>(const SweepArgs<T>&, int, hipStream_t, hipEvent_t,    \
                                        hipEvent_t);                                           \
  template hipError_t launch_restrict_res<T>(const RestrictArgs<T>&, hipStream_t);            \
  template hipError_t launch_resolve<T>(int, bool, const T*, const T*, T*, hipStream_t);      \
  template hipError_t launch_refine_add<T>(int, bool, bool, bool, const T*, const T*, double*, \
                                           hipStream_t, const Slots&, int, const Scalars*);

DCG_MG_INSTANTIATE(float)
DCG_MG_INSTANTIATE(double)

}  // namespace dcg
