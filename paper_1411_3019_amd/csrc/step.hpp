// step.hpp -- the step kernel of the RATTLE + Langevin hot path (gfx950) and
// the finish kernel that shares its force arithmetic.
//
// Per-particle kernels run one thread per particle over "tiles": 256
// consecutive slots of one job.  A launch covers the tiles of many jobs
// (tile -> job table), so one launch advances every resident system.
//
// Step kernel (one launch per time step), for particle i of a job at step s:
//   input  x^s (buffer parity xin), p^{s-1/2} (or p^s at a start), neighbour list
//   force  F_i(x^s) from the list (and, for bead models, bonds, bends, wall)
//   f^s    = b [F - gamma p^{s-1/2} + 1/2 sqrt(m) k (xi^s + xi^{s-1})]   (Algorithm S1)
//   p^s    = q - (n.q / n.n) n,   q = p^{s-1/2} + dt/2 f^s,  n = n(x^s)  (Algorithm 1, 2nd loop)
//   x^{s+1}, p^{s+1/2} from the scalar-Newton position stage          (Algorithm 1, 1st loop)
// so that one kernel does the force stage and momentum stage of step s-1 -> s
// and the position stage of s -> s+1.  The state between launches is
// (x^s, p^{s-1/2}) plus the normals xi^{s-1} of the previous draw (the noise
// cache; regenerating them from the Philox counter gives the same values).
// No force array is stored.
//
// Only templates and inline functions live here: each step translation unit
// instantiates the kernels it launches.
#pragma once

#include "device.hpp"

namespace mdk {

// An error at step s stops the job from step s + 1 on (only that launch can
// record one, so every recording lane stores the same step).  Each failing
// particle offers (particle index << 2 | code) and the smallest is kept: the
// report names the same particle whatever the order of the workgroups.
__device__ __forceinline__ void record_error(JobBook& K, int code, uint32_t id, long long s) {
  atomicMin(&K.err_key, ((unsigned long long)id << 2) | (unsigned long long)code);
  K.err_step = s;
  atomicMin(&K.stop_at, s + 1);
}

// An FP32-class particle whose force terms left the exact-sum range.
__device__ __forceinline__ void record_breach(JobBook& K) { atomicAdd(&K.sum_breaches, 1); }

__device__ __forceinline__ double nn3(double x, double y, double z) { return x * x + y * y + z * z; }
__device__ __forceinline__ double dot3(double ax, double ay, double az, double bx, double by, double bz) {
  return ax * bx + ay * by + az * bz;
}

// Noise amplitude sqrt(m) k of Algorithm S1 for one particle.
__device__ __forceinline__ double noise_amp(const JobDev& J, double m) {
  return J.uniform_mass ? J.noise_km : sqrt(m) * J.noise_k;
}

// Random part of the combined force of Algorithm S1 for one particle,
// regenerated from the counter: 1/2 sqrt(m) k (xi^s + xi^{s-1}) (at a start:
// sqrt(m) k xi^s, the previous draw being taken equal to this one).  Used by
// the finish kernel; the step kernel takes xi^{s-1} from the noise cache,
// which holds exactly these values.
template <bool kF64>
__device__ __forceinline__ void langevin_kick(const JobDev& J, uint32_t id, double m, long long s, bool start,
                                              double& rx, double& ry, double& rz) {
  rx = ry = rz = 0.0;
  if (!(J.gamma > 0.0) || (J.mode == kModeStartGiven && start)) return;
  double a0, a1, a2;
  langevin_normals<kF64>(J.seed, id, s, a0, a1, a2);
  const double k = noise_amp(J, m);
  if (start) {
    rx = k * a0;
    ry = k * a1;
    rz = k * a2;
  } else {
    double r0, r1, r2;
    langevin_normals<kF64>(J.seed, id, s - 1, r0, r1, r2);
    const double hk = 0.5 * k;
    rx = hk * (a0 + r0);
    ry = hk * (a1 + r1);
    rz = hk * (a2 + r2);
  }
}

// Combined force f^s = b [F - gamma p + random part] (Algorithm S1); at a
// start with a force handed in by the caller, that force.
__device__ __forceinline__ void combined_force(const JobDev& J, const DevBufs& B, uint32_t id, bool start, double Fx,
                                               double Fy, double Fz, double px, double py, double pz, double rx,
                                               double ry, double rz, double& fx, double& fy, double& fz) {
  if (J.mode == kModeStartGiven && start) {
    const int64_t o = J.off + id;
    fx = B.FC[3 * o];
    fy = B.FC[3 * o + 1];
    fz = B.FC[3 * o + 2];
    return;
  }
  if (J.gamma > 0.0) {
    fx = J.b * (Fx - J.gamma * px + rx);
    fy = J.b * (Fy - J.gamma * py + ry);
    fz = J.b * (Fz - J.gamma * pz + rz);
  } else {
    fx = Fx;
    fy = Fy;
    fz = Fz;
  }
}

// Bead-model forces on slot i (particle index id): typed pairs, then bonds,
// bends and the wall; returns the particle's energy share (kEnergy).
template <bool kEnergy, bool kF64, class Pos>
__device__ __forceinline__ double model_forces(const JobDev& J, const ModelDev& M, const DevBufs& B,
                                               const double* __restrict__ X, int64_t first, int64_t i, uint32_t id,
                                               int cnt, const Rows3& q, double xi, double yi, double zi, Pos pos,
                                               double& Fx, double& Fy, double& Fz, bool& exact,
                                               const double* tab = nullptr) {
  const int ti = B.TYPE[J.scur][i];
  if (J.periodic[0] | J.periodic[1] | J.periodic[2])
    pair_forces_model<true, kF64>(J, M, B, i, cnt, q, ti, xi, yi, zi, pos, Fx, Fy, Fz, exact, tab);
  else
    pair_forces_model<false, kF64>(J, M, B, i, cnt, q, ti, xi, yi, zi, pos, Fx, Fy, Fz, exact, tab);
  double u = kEnergy ? pair_energy_model(J, M, B, X, first, i, ti, xi, yi, zi) : 0.0;
  double xs[15];
  int tid[5];
  // the step kernel finds the molecule's beads in its window; the finish
  // kernel (kEnergy) through the inverse permutation
  const uint2 bw = kEnergy ? make_uint2(0xFFFFFFFFu, 0xFFFFFFFFu) : B.BW[i];
  molecule_window(J, M, B, X, id, xi, yi, zi, ti, bw, pos, xs, tid);
  u += bonded_forces(J, M, B, X, id, tid, xs, Fx, Fy, Fz, tab);
  return u;
}

// Halo slots of a tile staged in LDS by the step kernel (window entries
// 256 .. 256 + kHaloLds - 1); a tile with a longer halo reads the rest of its
// window through the halo list in global memory.
#ifndef MDK_HALO_LDS
#define MDK_HALO_LDS 640
#endif
constexpr int kHaloLdsDefault = MDK_HALO_LDS;
template <int kH>
constexpr size_t window_lds_bytes() {
  return sizeof(double) * 3 * (kTile + kH);
}

// One workgroup per tile.  The tile's window (own positions, then its halo)
// is staged in LDS while the noise is drawn; after one barrier each
// wavefront works on its own 64 slots and leaves as soon as they are done.
// jobs, models: the job and bead-model records (B.jobs, B.models) as
// separate no-alias arguments: nothing the kernel stores can change them, so
// the compiler reads them with scalar loads wherever they are used.
template <bool kF64, bool kModel, bool kAll, bool kStream, int kH>
__device__ __forceinline__ void step_body(const DevBufs& B, const JobDev* __restrict__ jobs,
                                          const ModelDev* __restrict__ models, const int* __restrict__ tile_job,
                                          const int64_t* __restrict__ tile_first, const int* __restrict__ ntiles_ptr,
                                          int t, double* win, double* mtab) {
  // the grid may be larger than the tile list (it is sized once per graph);
  // surplus workgroups leave at once
  const int ntiles = uniform_int(*ntiles_ptr);
  if ((int)blockIdx.x >= ntiles) return;
  const int b = xcd_remap((int)blockIdx.x, ntiles);
  const int job = uniform_int(tile_job[b]);
  const int64_t first = uniform_i64(tile_first[b]);
  const JobDev& J = jobs[job];
  JobBook& K = B.book[job];
  if (t >= J.remaining) return;
  const long long s = J.step0 + t;
  // a tile whose accumulated displacement passed skin/2 during step s-1 (or an
  // error) set stop_at <= s: the lists are no longer valid for forces at x^s
  // (stop_at only decreases, and never below s + 1 during this launch, so
  // every wavefront of the workgroup takes the same branch)
  if (s >= (long long)uniform_i64(K.stop_at)) return;
  // bead model: the type-pair tables of this tile's job in LDS
  if (kModel) {
    const ModelDev& M = models[job];
    const int q = (int)threadIdx.x;
    constexpr int kP = kMaxTypes * kMaxTypes;
    if (q < kP) {
      mtab[q] = M.rc2[q];
      mtab[kP + q] = M.sig2[q];
      mtab[2 * kP + q] = M.eps24[q];
      mtab[3 * kP + q] = M.r0[q];
    }
  }
  const bool start = (J.mode != kModeSteady) && (t == 0);
  const int xin = J.xcur ^ (t & 1);
  const double* __restrict__ X = B.X[xin];
  double* __restrict__ Xo = B.X[xin ^ 1];
  double* __restrict__ P = B.P[J.pcur];
  const int lane = (int)threadIdx.x;
  const int64_t i = first + lane;
  const bool valid = i < J.off + J.n;
  const int64_t gt = first / kTile;
  const bool pairs = J.pair_kind != kPairNone;
  const int nh = pairs ? uniform_int((int)B.HCNT[gt]) : 0;
  const int nst = min(nh, min(kH, B.hcap));
  const uint32_t* __restrict__ hl = B.HALO + gt * (int64_t)B.hcap;
  double xi = 0.0, yi = 0.0, zi = 0.0;
  uint32_t id = 0u;
  int cnt = 0;
  if (valid) {
    xi = X[3 * i];
    yi = X[3 * i + 1];
    zi = X[3 * i + 2];
    id = B.ID[J.scur][i];
    if (pairs) cnt = (int)B.NCNT[i];
  }
  // the window: own positions, then the staged part of the halo
  win[3 * lane] = xi;
  win[3 * lane + 1] = yi;
  win[3 * lane + 2] = zi;
  constexpr int kPer = (kH + kTile - 1) / kTile;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int h = lane + q * kTile;
    if (h < nst) {
      const int64_t j = hl[h];
      const double a0 = X[3 * j], a1 = X[3 * j + 1], a2 = X[3 * j + 2];
      win[3 * (kTile + h)] = a0;
      win[3 * (kTile + h) + 1] = a1;
      win[3 * (kTile + h) + 2] = a2;
    }
  }
  const Rows3 rows = load_rows3(B, i, cnt);
  const double m = valid ? (J.uniform_mass ? J.mass : B.MASS[J.scur][i]) : 1.0;
  // Langevin noise of this step while the loads are in flight: xi^s is drawn
  // and cached, xi^{s-1} comes from the cache
  double rx = 0.0, ry = 0.0, rz = 0.0;
  if (valid && J.gamma > 0.0) {
    double a0, a1, a2, r0 = 0.0, r1 = 0.0, r2 = 0.0;
    if (kF64) {
      double* zc = B.NZD[J.pcur] + 3 * i;
      if (!start) {
        r0 = zc[0];
        r1 = zc[1];
        r2 = zc[2];
      }
      normals3(J.seed, id, s, a0, a1, a2);
      zc[0] = a0;
      zc[1] = a1;
      zc[2] = a2;
    } else {
      float* zc = B.NZF[J.pcur] + 3 * i;
      if (!start) {
        r0 = (double)zc[0];
        r1 = (double)zc[1];
        r2 = (double)zc[2];
      }
      float z0, z1, z2;
      normals3_f32(J.seed, id, s, z0, z1, z2);
      zc[0] = z0;
      zc[1] = z1;
      zc[2] = z2;
      a0 = (double)z0;
      a1 = (double)z1;
      a2 = (double)z2;
    }
    const double k = noise_amp(J, m);
    if (!start) {
      const double hk = 0.5 * k;
      rx = hk * (a0 + r0);
      ry = hk * (a1 + r1);
      rz = hk * (a2 + r2);
    } else if (J.mode == kModeStart) {
      rx = k * a0;
      ry = k * a1;
      rz = k * a2;
    }
  }
  __syncthreads();
  double disp2 = 0.0;
  int iters = 0;
  if (valid) {
    double Fx = 0.0, Fy = 0.0, Fz = 0.0;
    bool exact = true;
    if (pairs) {
      auto lds_pos = [&](uint32_t e, double& ax, double& ay, double& az) {
        const double* w = win + 3 * e;
        ax = w[0];
        ay = w[1];
        az = w[2];
      };
      // a halo longer than the staged part: the rest through the halo list
      auto mixed_pos = [&](uint32_t e, double& ax, double& ay, double& az) {
        if (e < (uint32_t)(kTile + kH)) {
          const double* w = win + 3 * e;
          ax = w[0];
          ay = w[1];
          az = w[2];
        } else {
          const int64_t j = hl[min((int64_t)(e - kTile), (int64_t)B.hcap - 1)];
          ax = X[3 * j];
          ay = X[3 * j + 1];
          az = X[3 * j + 2];
        }
      };
      if (kModel) {
        const ModelDev& M = models[job];
        if (nh <= kH)
          model_forces<false, kF64>(J, M, B, X, first, i, id, cnt, rows, xi, yi, zi, lds_pos, Fx, Fy, Fz, exact,
                                    mtab);
        else
          model_forces<false, kF64>(J, M, B, X, first, i, id, cnt, rows, xi, yi, zi, mixed_pos, Fx, Fy, Fz, exact,
                                    mtab);
      } else {
        if (nh <= kH)
          pair_forces<kF64>(J, B, i, cnt, rows, xi, yi, zi, lds_pos, Fx, Fy, Fz, exact);
        else
          pair_forces<kF64>(J, B, i, cnt, rows, xi, yi, zi, mixed_pos, Fx, Fy, Fz, exact);
      }
      if (!exact) record_breach(K);
    }
    // the particle's own momentum and flag are loaded after the force loop,
    // which keeps them out of the loop's live registers
    double px = P[3 * i], py = P[3 * i + 1], pz = P[3 * i + 2];
    const bool cons = B.FLG[J.scur][i] != 0;
    double fx, fy, fz;
    combined_force(J, B, id, start, Fx, Fy, Fz, px, py, pz, rx, ry, rz, fx, fy, fz);
    double nx = 0.0, ny = 0.0, nz = 0.0, g0 = 0.0, inv_nn = 0.0;
    if (cons) {
      g0 = surf_eval<kAll>(J, xi, yi, zi, nx, ny, nz);
      inv_nn = rcp64(nn3(nx, ny, nz));
    }
    // momentum stage of step s-1 -> s: tangent projection (closed form of the linear Newton)
    if (!start) {
      px += J.half_dt * fx;
      py += J.half_dt * fy;
      pz += J.half_dt * fz;
      if (cons) {
        const double a = dot3(nx, ny, nz, px, py, pz) * inv_nn;
        px -= a * nx;
        py -= a * ny;
        pz -= a * nz;
      }
    }
    // position stage of step s -> s+1
    px += J.half_dt * fx;
    py += J.half_dt * fy;
    pz += J.half_dt * fz;
    const MassTerms mt = mass_terms(J, m);
    double x1, y1, z1;
    if (cons) {
      iters = rattle_position<kAll>(J, mt, xi, yi, zi, g0, nx, ny, nz, inv_nn, px, py, pz, x1, y1, z1);
      if (iters < 0) {
        record_error(K, kErrNewton, id, s);
        iters = -iters;
      }
    } else {
      x1 = xi + mt.dtm * px;
      y1 = yi + mt.dtm * py;
      z1 = zi + mt.dtm * pz;
    }
    if (kStream) {
      // streaming stores: the new state is not read again in this launch, so
      // it should not displace the neighbour positions the other workgroups
      // are staging from L2.  Used when the step's data exceed the Infinity
      // Cache; when they fit, ordinary stores leave the new state there for
      // the next step.  A template parameter, not a runtime flag: with both
      // forms in one kernel the compiler merges part of them into ordinary
      // stores.
      __builtin_nontemporal_store(x1, Xo + 3 * i);
      __builtin_nontemporal_store(y1, Xo + 3 * i + 1);
      __builtin_nontemporal_store(z1, Xo + 3 * i + 2);
      __builtin_nontemporal_store(px, P + 3 * i);
      __builtin_nontemporal_store(py, P + 3 * i + 1);
      __builtin_nontemporal_store(pz, P + 3 * i + 2);
    } else {
      Xo[3 * i] = x1;
      Xo[3 * i + 1] = y1;
      Xo[3 * i + 2] = z1;
      P[3 * i] = px;
      P[3 * i + 1] = py;
      P[3 * i + 2] = pz;
    }
    const double dx = x1 - xi, dy = y1 - yi, dz = z1 - zi;
    disp2 = dx * dx + dy * dy + dz * dz;
    if (!(disp2 <= 1e300) || !(fabs(px) + fabs(py) + fabs(pz) <= 1e300)) {
      record_error(K, kErrNaN, id, s);
      disp2 = 0.0;
    }
  }
  // per-group bound on the displacement since the last build: sum over steps of
  // the group's largest displacement; only this wavefront touches its entry
  double m2 = disp2;
  int im = iters;
  for (int o = 32; o > 0; o >>= 1) {
    m2 = fmax(m2, __shfl_xor(m2, o, 64));
    im = max(im, __shfl_xor(im, o, 64));
  }
  if (lane % kGroup == 0) {
    const int64_t g = i / kGroup;
    const double a = B.TACC[g] + sqrt(m2);
    B.TACC[g] = a;
    if (a > J.half_skin) atomicMin(&K.stop_at, s + 1);
    if (im > K.newton_max) atomicMax(&K.newton_max, im);
  }
}

// Step kernels, one per force class.  kAll: jobs on any surface (else the
// quadrics and the plane only); kWaves: occupancy target in wavefronts per
// SIMD (register budget); kH: halo entries staged in LDS.  The instances the
// engine launches are chosen at run time (md_tune).
#define MDK_STEP_KERNEL(NAME, F64, MODEL)                                                                          \
  template <bool kAll, bool kStream, int kWaves, int kH>                                                           \
  __global__ void __launch_bounds__(kTile) __attribute__((amdgpu_waves_per_eu(kWaves, 8)))                         \
  NAME(DevBufs B, const JobDev* __restrict__ jobs, const ModelDev* __restrict__ models,                           \
       const int* __restrict__ tile_job, const int64_t* __restrict__ tile_first,                                   \
       const int* __restrict__ ntiles_ptr, int t) {                                                                \
    __shared__ double win[3 * (kTile + kH)];                                                                       \
    __shared__ double mtab[MODEL ? kModelTab : 1];                                                                 \
    step_body<F64, MODEL, kAll, kStream, kH>(B, jobs, models, tile_job, tile_first, ntiles_ptr, t, win, mtab);     \
  }

MDK_STEP_KERNEL(k_step_f64, true, false)
MDK_STEP_KERNEL(k_step_f32, false, false)
MDK_STEP_KERNEL(k_step_model, true, true)
MDK_STEP_KERNEL(k_step_model_f32, false, true)
#undef MDK_STEP_KERNEL

// Finish: state at the current step m (x^m, p^m, f^m) and per-particle
// diagnostics, written by particle index.  Forces from the same list and the
// same arithmetic as the step kernel, neighbour positions read through the
// window's slots in global memory.
template <bool kF64>
__global__ void __launch_bounds__(kTile) k_finish(DevBufs B, const int* __restrict__ tile_job,
                                                  const int64_t* __restrict__ tile_first) {
  const int job = uniform_int(tile_job[blockIdx.x]);
  const int64_t first = uniform_i64(tile_first[blockIdx.x]);
  const JobDev& J = B.jobs[job];
  const int64_t C = B.C;
  const int64_t i = first + threadIdx.x;
  if (i >= J.off + J.n) return;
  const double* __restrict__ X = B.X[J.xcur];
  const double* __restrict__ P = B.P[J.pcur];
  const double xi = X[3 * i], yi = X[3 * i + 1], zi = X[3 * i + 2];
  double px = P[3 * i], py = P[3 * i + 1], pz = P[3 * i + 2];
  const uint32_t id = B.ID[J.scur][i];
  const bool cons = B.FLG[J.scur][i] != 0;
  const double m = J.uniform_mass ? J.mass : B.MASS[J.scur][i];
  const bool start = J.mode != kModeSteady;
  const long long s = J.step0;
  double Fx = 0.0, Fy = 0.0, Fz = 0.0, Ui = 0.0;
  if (J.pair_kind != kPairNone) {
    const int cnt = (int)B.NCNT[i];
    const Rows3 rows = load_rows3(B, i, cnt);
    auto gpos = [&](uint32_t e, double& ax, double& ay, double& az) {
      const int64_t j = window_slot(B, first, e);
      ax = X[3 * j];
      ay = X[3 * j + 1];
      az = X[3 * j + 2];
    };
    bool exact = true;
    if (J.model) {
      Ui = model_forces<true, kF64>(J, B.models[job], B, X, first, i, id, cnt, rows, xi, yi, zi, gpos, Fx, Fy, Fz,
                                    exact);
    } else {
      pair_forces<kF64>(J, B, i, cnt, rows, xi, yi, zi, gpos, Fx, Fy, Fz, exact);
      Ui = pair_energy(J, B, X, first, i, xi, yi, zi);
    }
  }
  double rx, ry, rz, fx, fy, fz;
  langevin_kick<kF64>(J, id, m, s, start, rx, ry, rz);
  combined_force(J, B, id, start, Fx, Fy, Fz, px, py, pz, rx, ry, rz, fx, fy, fz);
  double nx = 0.0, ny = 0.0, nz = 0.0, g = 0.0, inv_nn = 0.0;
  if (cons) {
    g = surf_eval(J, xi, yi, zi, nx, ny, nz);
    inv_nn = rcp64(nn3(nx, ny, nz));
  }
  if (!start) {
    px += J.half_dt * fx;
    py += J.half_dt * fy;
    pz += J.half_dt * fz;
    if (cons) {
      const double a = dot3(nx, ny, nz, px, py, pz) * inv_nn;
      px -= a * nx;
      py -= a * ny;
      pz -= a * nz;
    }
  }
  const int64_t o = J.off + id;
  B.OX[3 * o] = xi;
  B.OX[3 * o + 1] = yi;
  B.OX[3 * o + 2] = zi;
  B.OP[3 * o] = px;
  B.OP[3 * o + 1] = py;
  B.OP[3 * o + 2] = pz;
  B.OF[3 * o] = fx;
  B.OF[3 * o + 1] = fy;
  B.OF[3 * o + 2] = fz;
  B.OD[o] = 0.5 * (px * px + py * py + pz * pz) / m;
  B.OD[C + o] = Ui;
  double gd = 0.0, nv = 0.0;
  if (cons) {
    const double nl = sqrt(nn3(nx, ny, nz));
    gd = fabs(g) / nl;
    nv = fabs(dot3(nx, ny, nz, px, py, pz)) / (nl * m);
  }
  B.OD[2 * C + o] = gd;
  B.OD[3 * C + o] = nv;
}

}  // namespace mdk
