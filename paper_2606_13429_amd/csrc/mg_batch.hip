// Batched W-cycle kernels: the multigrid steps of mg_kernels.hip (Algorithm 4
// with the RAS smoother of Section 4.2) applied to kBatch requests that share
// one mesh.  Level vectors are request-interleaved, [square][request][4], so
// that a square's values of all requests are one contiguous 256 B (FP32) or
// 512 B (FP64) run.
//
// The RAS step is where batching changes the arithmetic shape: for one
// request the tile solve u = (L_k)_t^{-1} r is a 128 x 128 matrix-vector
// product bound by the factor stream; for kBatch requests it is a
// 128 x 128 by 128 x kBatch product, done with v_mfma_*_16x16x4 (FP32 or
// FP64 by the level type) so that the factor bytes are paid once for all
// requests.  Column c of every MFMA output reads column c of the operand
// only, so a request's result does not depend on which other requests share
// the batch.
#include <type_traits>

#include "kernels.hpp"
#include "mg_common.hpp"

namespace dcg {
namespace {
using namespace mg;

constexpr int kThreads = 256;
constexpr int B = kBatch;
constexpr int kCoarse = 1024;   // dofs of the 16 x 16 coarsest level

__device__ __forceinline__ int64_t at(int64_t e, int c) { return (e * B + c) * 4; }

// z += pending tile outputs of square e, request c (blocks in increasing
// order; unused cover slots hold zeros).
template <typename T>
__device__ __forceinline__ void add_pending_b(const T* Ye, int64_t e, int c, T z[4]) {
  T y0[4], y1[4], y2[4];
  ld4(Ye + at(3 * e, c), y0);
  ld4(Ye + at(3 * e + 1, c), y1);
  ld4(Ye + at(3 * e + 2, c), y2);
#pragma unroll
  for (int j = 0; j < 4; ++j) z[j] = ((z[j] + y0[j]) + y1[j]) + y2[j];
}

template <typename T>
__device__ __forceinline__ void current_z_b(const SweepArgs<T>& a, int e, int c, T z[4]) {
  if (a.has_z) {
    ld4(a.z_old + at(e, c), z);
  } else {
    z[0] = z[1] = z[2] = z[3] = T(0);
  }
  if (a.has_y) add_pending_b(a.Y_old, e, c, z);
  if (a.prol) {
    const int ex = e % a.n, ey = e / a.n;
    const int E = (ey >> 1) * a.nc + (ex >> 1);
    const int ch = (ex & 1) + 2 * (ey & 1);
    T ec[4];
    ld4(a.zc + at(E, c), ec);
    if (a.c_has_y) add_pending_b(a.Yc, E, c, ec);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      z[j] += pcoef<T>(ch, j, 0) * ec[0] + pcoef<T>(ch, j, 1) * ec[1] +
              pcoef<T>(ch, j, 2) * ec[2] + pcoef<T>(ch, j, 3) * ec[3];
  }
}

// One RAS step of level k for kBatch requests, one tile per workgroup:
//   1. the tile's factor operands are requested first (they are the bytes
//      the step streams from HBM);
//   2. z on the 52 squares near the tile: z_old + pending Y [+ P e_coarse],
//      kept in LDS; the core squares are written to z_new;
//   3. U = f - L_k z on the 32 block squares (128 x kBatch), in LDS, each
//      operator row loaded once for four requests;
//   4. wavefront w computes the row blocks P = w and P = 7 - w of
//      (L_k)_t^{-1} U: 8 column blocks Q x 4 MFMA k-steps each.  Blocks
//      with P <= Q are read as stored (row r, columns 4k..4k+3 as one
//      vector load), the others as the transpose of the stored (Q, P);
//   5. Y_t = D_t U written to the pending slot of each block square.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_sweep_b(SweepArgs<T> a) {
  using V = typename Mfma<T>::v4;
  __shared__ __align__(16) T zn[52][B][4];
  __shared__ __align__(16) T ul[32][B][4];
  const int t = xcd_band_index(blockIdx.x, gridDim.x);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, k = lane >> 4;
  const int Pw[2] = {wave, 7 - wave};
  const bool need_z = a.has_z || a.has_y || a.prol;

  // MFMA A operands: lane (r, k) of k-step kk holds row 16 P + r, column
  // 16 Q + 4 k + kk of the tile inverse; column blocks are loaded two ahead
  // of their use (the first two before the gather and residual phases)
  const T* Ft = a.F + (int64_t)a.fcls[t] * (36 * 256);   // grid = tiles
  auto load_q = [&](int Q, T (&dst)[2][4]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int P = Pw[h];
      if (P <= Q) {
        ld4(Ft + blk_index(P, Q) * 256 + r * 16 + 4 * k, dst[h]);
      } else {
        const T* bt = Ft + blk_index(Q, P) * 256 + 64 * k + r;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) dst[h][kk] = bt[16 * kk];
      }
    }
  };
  T av[3][2][4];
  load_q(0, av[0]);
  load_q(1, av[1]);

  for (int it = tid; it < 52 * B; it += kThreads) {
    const int q = it / B, c = it % B;
    const int e = ext_square(t, q, a.n);
    T z[4] = {T(0), T(0), T(0), T(0)};
    if (e >= 0 && need_z) current_z_b(a, e, c, z);
    st4(&zn[q][c][0], z);
  }
  __syncthreads();
  if (a.write_z) {   // the 16 core squares x kBatch requests, one per thread
    const int q = tid / B, c = tid % B;
    const int e = ext_square(t, q, a.n);
    T z[4];
    ld4(&zn[q][c][0], z);
    st4(a.z_new + at(e, c), z);
  }
  // U = f - L_k z: thread (block square p, row j, requests 4 g .. 4 g + 3), so
  // that each operator row is loaded once and applied to four requests' z
  // from LDS
#pragma unroll
  for (int k2 = 0; k2 < 32 * 16 / kThreads; ++k2) {
    const int it = tid + k2 * kThreads;
    const int p = it >> 4, j = (it >> 2) & 3, g = it & 3;
    const int e = ext_square(t, p, a.n);
    T u[4] = {T(0), T(0), T(0), T(0)};
    if (e >= 0) {
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) u[cc] = a.f[at(e, 4 * g + cc) + j];
      if (need_z) {
        const int ex = e % a.n, ey = e / a.n;
        T acc[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int s = 0; s < 5; ++s) {
          const int dx = s == 1 ? -1 : (s == 2 ? 1 : 0), dy = s == 3 ? -1 : (s == 4 ? 1 : 0);
          if (ex + dx < 0 || ex + dx >= a.n || ey + dy < 0 || ey + dy >= a.n) continue;
          T l[4];
          ld4(a.L + (((int64_t)s * a.ne + e) * 4 + j) * 4, l);
          const int q = nbr_slot(p, s);
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) {
            T zq[4];
            ld4(&zn[q][4 * g + cc][0], zq);
            acc[cc] += l[0] * zq[0] + l[1] * zq[1] + l[2] * zq[2] + l[3] * zq[3];
          }
        }
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) u[cc] -= acc[cc];
      }
    }
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) ul[p][4 * g + cc][j] = u[cc];
  }
  __syncthreads();

  // MFMA B operand of column block Q: lane (k, c = r) holds U[16 Q + 4 k + kk][c]
  V acc0 = {T(0), T(0), T(0), T(0)}, acc1 = {T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int Q = 0; Q < 8; ++Q) {
    if (Q + 2 < 8) load_q(Q + 2, av[(Q + 2) % 3]);
    T bq[4];
    ld4(&ul[4 * Q + k][r][0], bq);
    const T (&aq)[2][4] = av[Q % 3];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      acc0 = Mfma<T>::mac(aq[0][kk], bq[kk], acc0);
      acc1 = Mfma<T>::mac(aq[1][kk], bq[kk], acc1);
    }
  }

#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const V& acc = h == 0 ? acc0 : acc1;
    const int P = Pw[h];
    if constexpr (std::is_same<T, float>::value) {
      // rows 4 k + v: square 4 P + k, corner v, request r
      const int p = 4 * P + k;
      const int e = ext_square(t, p, a.n);
      if (e >= 0) {
        const T w = a.dw[e];
        const T y[4] = {w * acc[0], w * acc[1], w * acc[2], w * acc[3]};
        st4(a.Y_new + at(a.dst[t * 32 + p], r), y);
      }
    } else {
      // rows 4 v + k: square 4 P + v, corner k, request r
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = 4 * P + v;
        const int e = ext_square(t, p, a.n);
        if (e >= 0) a.Y_new[at(a.dst[t * 32 + p], r) + k] = a.dw[e] * acc[v];
      }
    }
  }
}

// Pending update + residual + restriction for kBatch requests: one
// wavefront per coarse square, lane = (child, request); the four children's
// restricted contributions are summed across lanes.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_restrict_res_b(RestrictArgs<T> a) {
  const int nc = a.n >> 1;
  const int E = xcd_band_index(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  if (E >= nc * nc) return;   // whole wavefronts
  const int ch = (threadIdx.x >> 4) & 3, c = threadIdx.x & 15;
  const int EX = E % nc, EY = E / nc;
  const int ex = 2 * EX + (ch & 1), ey = 2 * EY + (ch >> 1);
  const int e = ey * a.n + ex;
  T acc[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    const int dx = s == 1 ? -1 : (s == 2 ? 1 : 0), dy = s == 3 ? -1 : (s == 4 ? 1 : 0);
    if (ex + dx < 0 || ex + dx >= a.n || ey + dy < 0 || ey + dy >= a.n) continue;
    const int cn = e + dy * a.n + dx;
    T z[4] = {T(0), T(0), T(0), T(0)};
    if (a.has_z) ld4(a.z_old + at(cn, c), z);
    if (a.has_y) add_pending_b(a.Y_old, cn, c, z);
    if (s == 0 && a.write_z) st4(a.z_new + at(e, c), z);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      T l[4];
      ld4(a.L + (((int64_t)s * a.ne + e) * 4 + j) * 4, l);
      acc[j] += l[0] * z[0] + l[1] * z[1] + l[2] * z[2] + l[3] * z[3];
    }
  }
  T rv[4];
  ld4(a.f + at(e, c), rv);
#pragma unroll
  for (int j = 0; j < 4; ++j) rv[j] -= acc[j];
  T ck[4];
#pragma unroll
  for (int K = 0; K < 4; ++K) {
    ck[K] = pcoef<T>(ch, 0, K) * rv[0] + pcoef<T>(ch, 1, K) * rv[1] + pcoef<T>(ch, 2, K) * rv[2] +
            pcoef<T>(ch, 3, K) * rv[3];
    ck[K] += __shfl_xor(ck[K], 16, 64);
    ck[K] += __shfl_xor(ck[K], 32, 64);
  }
  if (ch == 0) st4(a.rc + at(E, c), ck);
}

// Exact coarsest solve for kBatch requests, z = L_1^{-1} f in FP64: the
// 1024 x 1024 inverse times the 1024 x kBatch right-hand sides with FP64
// MFMA.  Workgroup R owns rows 16 R .. 16 R + 15; wavefront w the quarter
// 256 w .. 256 w + 255 of the contraction, summed in LDS in wavefront order.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_coarse_b(const double* __restrict__ inv,
                                                       const T* __restrict__ f, T* __restrict__ z) {
  using V = Mfma<double>::v4;
  __shared__ double red[4][4][64];
  const int R = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, k = lane >> 4;
  const double* ir = inv + (int64_t)(16 * R + r) * kCoarse + 4 * k;
  V acc = {0.0, 0.0, 0.0, 0.0};
  for (int g = 16 * wave; g < 16 * wave + 16; ++g) {   // contraction dofs 16 g .. 16 g + 15
    double av[4];
    ld4(ir + 16 * g, av);
    T bv[4];
    ld4(f + at(4 * g + k, r), bv);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) acc = Mfma<double>::mac(av[kk], static_cast<double>(bv[kk]), acc);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) red[wave][v][lane] = acc[v];
  __syncthreads();
  if (wave == 0) {
    // rows 4 v + k of the block: square 4 R + v, corner k, request r
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double s = ((red[0][v][lane] + red[1][v][lane]) + red[2][v][lane]) + red[3][v][lane];
      z[at(4 * R + v, r) + k] = static_cast<T>(s);
    }
  }
}

// out = (has_z ? z : 0) + pending Ye for kBatch requests.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_resolve_b(int ne, int has_z, const T* __restrict__ z,
                                                        const T* __restrict__ Ye,
                                                        T* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (i >= 4 * (int64_t)B * ne) return;
  const int64_t e = i / (4 * B);
  const int c = int((i >> 2) % B), j = int(i & 3);
  const T v = has_z ? z[i] : T(0);
  out[i] = ((v + Ye[at(3 * e, c) + j]) + Ye[at(3 * e + 1, c) + j]) + Ye[at(3 * e + 2, c) + j];
}

}  // namespace

template <typename T>
hipError_t launch_resolve_b(int ne, bool has_z, const T* z, const T* Ye, T* out, hipStream_t st) {
  const int64_t n = 4 * (int64_t)B * ne;
  k_resolve_b<T><<<int((n + kThreads - 1) / kThreads), kThreads, 0, st>>>(ne, has_z, z, Ye, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep_b(const SweepArgs<T>& a, hipStream_t st) {
  if (a.tiles <= 0 || a.n < 8 || (a.n & 3)) return hipErrorInvalidValue;
  k_sweep_b<T><<<a.tiles, kThreads, 0, st>>>(a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict_res_b(const RestrictArgs<T>& a, hipStream_t st) {
  const int nc = a.n / 2;
  k_restrict_res_b<T><<<(nc * nc + 3) / 4, kThreads, 0, st>>>(a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse_b(const double* inv, const T* f, T* z, hipStream_t st) {
  k_coarse_b<T><<<kCoarse / 16, kThreads, 0, st>>>(inv, f, z);
  return hipGetLastError();
}

#define DCG_MGB_INSTANTIATE(T)                                                              \
  template hipError_t launch_sweep_b<T>(const SweepArgs<T>&, hipStream_t);                  \
  template hipError_t launch_restrict_res_b<T>(const RestrictArgs<T>&, hipStream_t);        \
  template hipError_t launch_coarse_b<T>(const double*, const T*, T*, hipStream_t);       \
  template hipError_t launch_resolve_b<T>(int, bool, const T*, const T*, T*, hipStream_t);

DCG_MGB_INSTANTIATE(float)
DCG_MGB_INSTANTIATE(double)

}  // namespace dcg
