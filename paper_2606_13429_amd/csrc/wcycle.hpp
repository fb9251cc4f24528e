// Host driver of the W-cycle (Algorithm 4) over the fused level kernels,
// shared by the single-request solver and the batched serving engine.
//
// The iterate of a level between launches is z = (has_z ? z[zb] : 0) +
// (has_y ? pending tile outputs Y[yb] : 0) (see mg_kernels.hip).  The host
// replays the same deterministic state sequence for every cycle, so a
// captured graph of a cycle stays valid across replays.
#pragma once
#include "runtime.hpp"

namespace dcg {

struct LvState {
  bool has_z = false, has_y = false;
  int zb = 0, yb = 0;
};

// Records an event pair around every finest-level RAS step (live kernel
// timing); ev == nullptr disables it.
struct SweepTimer {
  hipEvent_t* ev = nullptr;
  int max = 0;
  int* rec = nullptr;
};

inline int waves_per_tile(int tiles) { return tiles >= 4096 ? 1 : (tiles >= 1024 ? 2 : 4); }

// Tiles per side of a workgroup of the grouped (MFMA) RAS step, 0 for the
// per-tile kernel.  ``choice`` is dcg_options.ras_group: 0 picks by level
// size, -1 forces the per-tile kernel, 1 / 2 / 4 that group side.  Measured
// on MI355X (FP32, per step): 4 x 4 groups take 17.7 / 10.0 / 7.5 us at
// n = 512 / 256 / 128, 2 x 2 groups 36 / 14 / 8.3 us, single tiles
// 106 / 32 / 11 us, the per-tile kernel 60 / 18 / 9.2 us.
#ifndef DCG_GROUP_MIN_TILES
#define DCG_GROUP_MIN_TILES 1024
#endif
inline int ras_group_side(int tiles, int choice) {
  if (choice < 0) return 0;
  if (choice > 0) return choice;
  return tiles >= DCG_GROUP_MIN_TILES ? 4 : 0;
}

template <typename T>
const T* level_L(const DeviceLevel& d);
template <>
inline const float* level_L<float>(const DeviceLevel& d) { return d.L32; }
template <>
inline const double* level_L<double>(const DeviceLevel& d) { return d.L64; }
template <typename T>
const T* level_Lc(const DeviceLevel& d);
template <>
inline const float* level_Lc<float>(const DeviceLevel& d) { return d.Lc32; }
template <>
inline const double* level_Lc<double>(const DeviceLevel& d) { return d.Lc64; }
template <typename T>
const T* level_dw(const DeviceLevel& d);
template <>
inline const float* level_dw<float>(const DeviceLevel& d) { return d.dw32; }
template <>
inline const double* level_dw<double>(const DeviceLevel& d) { return d.dw64; }
template <typename T>
const T* level_Fm(const DeviceLevel& d);
template <>
inline const float* level_Fm<float>(const DeviceLevel& d) { return d.Fm32; }
template <>
inline const double* level_Fm<double>(const DeviceLevel& d) { return d.Fm64; }
template <typename T>
const T* level_F(const DeviceLevel& d);
template <>
inline const float* level_F<float>(const DeviceLevel& d) { return d.F32; }
template <>
inline const double* level_F<double>(const DeviceLevel& d) { return d.F64; }

// Levels are numbered 1 (coarsest) .. J of the cycle's own hierarchy, which
// is the stored one shifted by ``base``: cycle level k is stored level
// k + base.  With base > 0 the coarsest level is solved by fast
// diagonalisation (``cfdm``); with base = 0 by the stored dense inverse.
template <typename T>
struct Cycle {
  const MeshContext& m;
  const LevelBuffers& b;
  int pre = 2, post = 2;
  SweepTimer timer;
  int base = 0;
  const CoarseFdm* cfdm = nullptr;
  int group = 0;                  // dcg_options.ras_group

  Cycle(const MeshContext& mesh, const LevelBuffers& bufs, int m1, int m2)
      : m(mesh), b(bufs), pre(m1), post(m2) {}

  const DeviceLevel& lev(int k) const { return m.lv[k - 1 + base]; }
  T* f(int k) const { return static_cast<T*>(b.f[k - 1 + base]); }
  T* rr(int k) const { return static_cast<T*>(b.rr[k - 1 + base]); }
  T* z(int k, int i) const { return static_cast<T*>(b.z[i][k - 1 + base]); }
  T* Y(int k, int i) const { return static_cast<T*>(b.Y[i][k - 1 + base]); }

  // One RAS step z <- z + S_k (f - L_k z) of level k; ``coarse`` (optional)
  // is the state of level k-1 whose prolongation P e is added first.
  void sweep_step(int k, LvState& s, const LvState* coarse, hipStream_t st) const {
    const DeviceLevel& d = lev(k);
    SweepArgs<T> a;
    a.F = level_F<T>(d);
    a.Fm = level_Fm<T>(d);
    a.fcls = d.fcls;
    a.dw = level_dw<T>(d);
    a.ext = d.tile_ext;
    a.tiles = d.tiles;
    a.n = d.n;
    a.ne = d.ne;
    a.L = level_L<T>(d);
    a.Lc = level_Lc<T>(d);
    a.cols = d.cols;
    a.dst = d.tile_dst;
    a.f = f(k);
    a.has_z = s.has_z;
    a.has_y = s.has_y;
    a.z_old = z(k, s.zb);
    a.Y_old = Y(k, s.yb);
    if (coarse) {
      a.prol = 1;
      a.nc = d.n / 2;
      a.zc = z(k - 1, coarse->zb);
      a.c_has_y = coarse->has_y;
      if (coarse->has_y) a.Yc = Y(k - 1, coarse->yb);
    }
    const bool changes = s.has_y || coarse != nullptr;
    const int zb_new = changes ? 1 - s.zb : s.zb;
    a.write_z = changes;
    a.z_new = z(k, zb_new);
    a.Y_new = Y(k, 1 - s.yb);
    const bool timed = timer.ev && k + base == m.J && *timer.rec < timer.max;
    const int gx = ras_group_side(d.tiles, group);
    if (b.batched || gx <= 0) {
      if (timed) DCG_HIP(hipEventRecord(timer.ev[2 * *timer.rec], st));
      if (b.batched)
        DCG_HIP(launch_sweep_b<T>(a, st));
      else
        DCG_HIP(launch_sweep<T>(a, waves_per_tile(d.tiles), st));
      if (timed) DCG_HIP(hipEventRecord(timer.ev[2 * (*timer.rec)++ + 1], st));
    } else {
      const int gi = gx == 1 ? 0 : (gx == 2 ? 1 : 2);
      a.gextra = d.gx_extra[gi];
      a.nextra = d.gx_extra_n[gi];
      // the grouped step records its timing events in the dispatch packet
      hipEvent_t e0 = timed ? timer.ev[2 * *timer.rec] : nullptr;
      hipEvent_t e1 = timed ? timer.ev[2 * *timer.rec + 1] : nullptr;
      DCG_HIP(launch_sweep_g<T>(a, gx, st, e0, e1));
      if (timed) ++*timer.rec;
    }
    s.has_z = s.has_z || changes;
    s.zb = zb_new;
    s.has_y = true;
    s.yb = 1 - s.yb;
  }

  // Resolves the pending update and restricts the residual:
  // f_{k-1} = P_k^T (f_k - L_k z).
  void restrict_step(int k, LvState& s, hipStream_t st) const {
    const DeviceLevel& d = lev(k);
    RestrictArgs<T> a;
    a.n = d.n;
    a.ne = d.ne;
    a.L = level_L<T>(d);
    a.Lc = level_Lc<T>(d);
    a.cols = d.cols;
    a.f = f(k);
    a.has_z = s.has_z;
    a.has_y = s.has_y;
    a.z_old = z(k, s.zb);
    a.Y_old = Y(k, s.yb);
    a.write_z = s.has_y;
    a.z_new = z(k, 1 - s.zb);
    a.rc = f(k - 1);
    if (b.batched)
      DCG_HIP(launch_restrict_res_b<T>(a, st));
    else
      DCG_HIP(launch_restrict_res<T>(a, st));
    if (s.has_y) {
      s.zb = 1 - s.zb;
      s.has_z = true;
    }
    s.has_y = false;
  }

  // Post-smoothing of level k after the coarse correction ``c`` of level
  // k-1: the first RAS step adds P e; without post-smoothing the coarse
  // iterate is resolved and prolongated on its own (single-request only).
  void post_smooth(int k, LvState& s, const LvState& c, hipStream_t st) const {
    if (post > 0) {
      sweep_step(k, s, &c, st);
      for (int i = 1; i < post; ++i) sweep_step(k, s, nullptr, st);
      return;
    }
    if (b.batched) throw Error(DCG_EINVAL, "the batched cycle needs post-smoothing (m2 >= 1)");
    const DeviceLevel& d = lev(k);
    const int64_t mc = 4 * int64_t(lev(k - 1).ne);
    T* e = rr(k - 1);
    if (c.has_y)
      DCG_HIP(launch_resolve<T>(lev(k - 1).ne, c.has_z, z(k - 1, c.zb), Y(k - 1, c.yb), e, st));
    else
      DCG_HIP(launch_copy<T>(mc, z(k - 1, c.zb), e, st));
    if (!s.has_z) DCG_HIP(launch_fill<T>(4 * int64_t(d.ne), T(0), z(k, s.zb), st));
    DCG_HIP(launch_prolong<T>(d.n / 2, e, z(k, s.zb), st));
    s.has_z = true;
  }

  // Level k W-cycle (Algorithm 4) on f_k from the iterate described by ``s``.
  void wcycle(int k, LvState& s, hipStream_t st) const {
    if (k == 1) {   // exact coarsest solve; the initial guess is irrelevant
      if (cfdm) {
        if (b.batched) throw Error(DCG_EINVAL, "the batched cycle runs the full hierarchy");
        DCG_HIP(launch_fdm_coarse<T>(cfdm->n, cfdm->V, cfdm->VT, cfdm->lam, f(1), z(1, 0),
                                     cfdm->t[0], cfdm->t[1], cfdm->t[2], st));
      } else if (b.batched)
        DCG_HIP(launch_coarse_b<T>(m.coarse_inv, f(1), z(1, 0), st));
      else
        DCG_HIP(launch_coarse<T>(m.coarse_inv, f(1), z(1, 0), st));
      s = LvState();
      s.has_z = true;
      return;
    }
    for (int i = 0; i < pre; ++i) sweep_step(k, s, nullptr, st);
    restrict_step(k, s, st);
    LvState c;                                     // coarse iterate starts at 0
    coarse_correction(k, c, st);
    post_smooth(k, s, c, st);
  }

  // The two coarse W-cycles of level k-1 (Algorithm 4: e_bar from 0, then e
  // from e_bar).  On level 1 both calls return the same exact solve, so the
  // second is skipped.
  void coarse_correction(int k, LvState& c, hipStream_t st) const {
    wcycle(k - 1, c, st);
    if (k - 1 >= 2) wcycle(k - 1, c, st);
  }
};

}  // namespace dcg
