// Device helpers shared by the multigrid kernels of the single-request
// (mg_kernels.hip) and batched (mg_batch.hip) W-cycles: vector loads, the
// Q1 prolongation coefficients and the geometry of the RAS blocks (Section
// 4.2: a 4 x 4 core of squares plus the layer of squares across its faces).
//
// Block slots p < 32 of a tile: 0..15 the core (x = p % 4, y = p / 4), then
// the layer x = -1, x = 4, y = -1, y = 4 (4 squares each).  Extended slots
// 32..51 add the squares at distance 1 outside the block: x = -2, x = 5,
// y = -2, y = 5 (4 each) and the 4 diagonal corners.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dcg {
namespace mg {

__device__ __forceinline__ void ld4(const float* p, float v[4]) {
  const float4 t = *reinterpret_cast<const float4*>(p);
  v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
}
__device__ __forceinline__ void ld4(const double* p, double v[4]) {
  const double2 a = reinterpret_cast<const double2*>(p)[0];
  const double2 b = reinterpret_cast<const double2*>(p)[1];
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void st4(float* p, const float v[4]) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void st4(double* p, const double v[4]) {
  reinterpret_cast<double2*>(p)[0] = make_double2(v[0], v[1]);
  reinterpret_cast<double2*>(p)[1] = make_double2(v[2], v[3]);
}

// 16 x 16 x 4 MFMA of the level type.  Operand lanes: A holds (row l % 16,
// k l / 16), B holds (k l / 16, column l % 16).  The accumulator of lane l
// holds column l % 16 and rows 4 (l / 16) + v (FP32) or 4 v + l / 16 (FP64),
// v = 0..3.
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mac(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mac(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// Coefficient of coarse corner A at fine corner a of child ch (exact).
template <typename T>
__device__ __forceinline__ T pcoef(int ch, int a, int A) {
  const int px = (ch & 1) + (a & 1), py = (ch >> 1) + (a >> 1);
  const int wx = (A & 1) ? px : 2 - px, wy = (A >> 1) ? py : 2 - py;
  return T(wx * wy) * T(0.25);
}

// Position (relative to the tile origin) of block slot p < 32.
__device__ __forceinline__ void slot_pos(int p, int& px, int& py) {
  if (p < 16) { px = p & 3; py = p >> 2; }
  else if (p < 20) { px = -1; py = p - 16; }
  else if (p < 24) { px = 4; py = p - 20; }
  else if (p < 28) { px = p - 24; py = -1; }
  else { px = p - 28; py = 4; }
}

// Extended slot (0..51) of the position, -1 outside the pattern.
__device__ __forceinline__ int pos_slot(int px, int py) {
  const bool cx = px >= 0 && px < 4, cy = py >= 0 && py < 4;
  if (cx && cy) return py * 4 + px;
  if (cy) {
    if (px == -1) return 16 + py;
    if (px == 4) return 20 + py;
    if (px == -2) return 32 + py;
    if (px == 5) return 36 + py;
    return -1;
  }
  if (cx) {
    if (py == -1) return 24 + px;
    if (py == 4) return 28 + px;
    if (py == -2) return 40 + px;
    if (py == 5) return 44 + px;
    return -1;
  }
  if (px == -1 && py == -1) return 48;
  if (px == 4 && py == -1) return 49;
  if (px == -1 && py == 4) return 50;
  if (px == 4 && py == 4) return 51;
  return -1;
}

__device__ __forceinline__ int nbr_slot(int p, int s) {
  int px, py;
  slot_pos(p, px, py);
  const int dx = s == 1 ? -1 : (s == 2 ? 1 : 0);
  const int dy = s == 3 ? -1 : (s == 4 ? 1 : 0);
  return pos_slot(px + dx, py + dy);
}

// Position (relative to the tile origin) of extended slot q < 52.
__device__ __forceinline__ void ext_pos(int q, int& px, int& py) {
  if (q < 32) { slot_pos(q, px, py); return; }
  if (q < 36) { px = -2; py = q - 32; }
  else if (q < 40) { px = 5; py = q - 36; }
  else if (q < 44) { px = q - 40; py = -2; }
  else if (q < 48) { px = q - 44; py = 5; }
  else { px = (q & 1) ? 4 : -1; py = (q < 50) ? -1 : 4; }
}

// Square of extended slot q of tile t on an n x n grid (-1 outside).
__device__ __forceinline__ int ext_square(int t, int q, int n) {
  const int tpr = n >> 2;
  int px, py;
  ext_pos(q, px, py);
  const int x = 4 * (t % tpr) + px, y = 4 * (t / tpr) + py;
  return (x < 0 || y < 0 || x >= n || y >= n) ? -1 : y * n + x;
}

// Workgroups are dispatched to the 8 XCDs (each with its own L2) round-robin
// by workgroup id.  Tiles that share squares (the layer and the outside
// neighbours of a block) should be handled by the same XCD, so workgroup b
// takes logical index (b mod 8) * (G / 8) + b / 8: XCD x processes the
// contiguous range x G / 8 .. (x + 1) G / 8 - 1 (a band of tile rows).  Only
// grids of at most kXcdBandMaxGrid workgroups are remapped: the largest
// grids stream their factors from HBM, where the eight separate fronts of
// the band order measured slower (4 % at n = 512) while the cache-resident
// levels gain 5-20 %.  Grids not divisible by 8 keep the identity.
#ifndef DCG_XCD_BAND_MAX_GRID
#define DCG_XCD_BAND_MAX_GRID 2048
#endif
constexpr int kXcdBandMaxGrid = DCG_XCD_BAND_MAX_GRID;
__device__ __forceinline__ int xcd_band_index(int b, int G) {
  return ((G & 7) || G > kXcdBandMaxGrid) ? b : (b & 7) * (G >> 3) + (b >> 3);
}

// Index of block (P, Q), P <= Q, in the packed upper-triangular order
// (row by row) of the symmetric tile inverses.
__host__ __device__ constexpr int blk_index(int P, int Q) { return P * (15 - P) / 2 + Q; }

}  // namespace mg
}  // namespace dcg
