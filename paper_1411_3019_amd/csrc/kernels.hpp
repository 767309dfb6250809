// kernels.hpp -- HIP kernels of the RATTLE + Langevin hot path (gfx950).
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
// (x^s, p^{s-1/2}); no force array is stored and the previous random force is
// regenerated from the Philox counter.
#pragma once

#include "device.hpp"

namespace mdk {

// An error at step s stops the job from step s + 1 on.
__device__ __forceinline__ void record_error(JobBook& K, int code, uint32_t id, long long s) {
  if (atomicCAS(&K.err_code, 0, code) == 0) K.err_id = (int)id;
  atomicMin(&K.stop_at, s + 1);
}

// Bead-model forces on slot i (particle index id): typed pairs, then bonds,
// bends and the wall; returns the particle's energy share (kEnergy).
template <bool kEnergy, bool kF64>
__device__ __forceinline__ double model_forces(const JobDev& J, const ModelDev& M, const DevBufs& B,
                                               const double* __restrict__ X, int64_t i, uint32_t id, double xi,
                                               double yi, double zi, double& Fx, double& Fy, double& Fz,
                                               const double* tab = nullptr) {
  const int ti = B.TYPE[J.scur][i];
  if (J.periodic[0] | J.periodic[1] | J.periodic[2])
    pair_forces_model<true, kF64>(J, M, B, X, i, ti, xi, yi, zi, Fx, Fy, Fz, tab);
  else
    pair_forces_model<false, kF64>(J, M, B, X, i, ti, xi, yi, zi, Fx, Fy, Fz, tab);
  double u = kEnergy ? pair_energy_model(J, M, B, X, i, ti, xi, yi, zi) : 0.0;
  double xs[15];
  int tid[5];
  molecule_window(J, M, B, X, id, xi, yi, zi, ti, xs, tid);
  u += bonded_forces(J, M, B, X, id, tid, xs, Fx, Fy, Fz, tab);
  return u;
}

// Random part of the combined force of Algorithm S1 for one particle:
// 1/2 sqrt(m) k (xi^s + xi^{s-1}) (at a start: sqrt(m) k xi^s, the previous
// draw being taken equal to this one).  Independent of the pair forces, so it
// is computed while the neighbour gathers are in flight.
template <bool kF64>
__device__ __forceinline__ void langevin_kick(const JobDev& J, uint32_t id, double m, long long s, bool start,
                                              double& rx, double& ry, double& rz) {
  rx = ry = rz = 0.0;
  if (!(J.gamma > 0.0) || (J.mode == kModeStartGiven && start)) return;
  double a0, a1, a2;
  langevin_normals<kF64>(J.seed, id, s, a0, a1, a2);
  const double k = sqrt(m) * J.noise_k;
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

// One workgroup per tile; each wavefront works on its own 64 slots of the
// tile and shares no barrier with the others, so it leaves as soon as its own
// particles are done.  (Workgroups of one wavefront would be capped by the
// per-CU workgroup limit well below the register-bound occupancy.)
template <bool kF64, bool kModel, bool kStream>
__device__ __forceinline__ void step_body(const DevBufs& B, const int* __restrict__ tile_job,
                                          const int64_t* __restrict__ tile_first, const int* __restrict__ ntiles_ptr,
                                          int t) {
  // the grid may be larger than the tile list (it is sized once per graph);
  // surplus workgroups leave at once
  const int ntiles = uniform_int(*ntiles_ptr);
  if ((int)blockIdx.x >= ntiles) return;
  const int b = xcd_remap((int)blockIdx.x, ntiles);
  const int job = uniform_int(tile_job[b]);
  const int64_t first = uniform_i64(tile_first[b]) + (int64_t)uniform_int((int)threadIdx.x / kGroup) * kGroup;
  const JobDev& J = B.jobs[job];
  JobBook& K = B.book[job];
  // bead model: the type-pair tables of this tile's job in LDS, so that the
  // typed lookups of the force loop and the bonds are LDS reads instead of
  // vector-memory loads
  // (every wavefront of the workgroup reaches this barrier: the job is the
  // tile's, and the per-wavefront exits come after it)
  __shared__ double mtab[kModel ? kModelTab : 1];
  if (kModel) {
    const ModelDev& M = B.models[job];
    const int q = (int)threadIdx.x;
    constexpr int kP = kMaxTypes * kMaxTypes;
    if (q < kP) {
      mtab[q] = M.rc2[q];
      mtab[kP + q] = M.sig2[q];
      mtab[2 * kP + q] = M.eps24[q];
      mtab[3 * kP + q] = M.r0[q];
    }
    __syncthreads();
  }
  if (t >= J.remaining || first >= J.off + J.n) return;
  const long long s = J.step0 + t;
  // a tile whose accumulated displacement passed skin/2 during step s-1 (or an
  // error) set stop_at <= s: the lists are no longer valid for forces at x^s
  if (s >= K.stop_at) return;
  const bool start = (J.mode != kModeSteady) && (t == 0);
  const int xin = J.xcur ^ (t & 1);
  const double* __restrict__ X = B.X[xin];
  double* __restrict__ Xo = B.X[xin ^ 1];
  double* __restrict__ P = B.P[J.pcur];
  const int64_t C = B.C;
  const int64_t i = first + (threadIdx.x % kGroup);
  double disp2 = 0.0;
  int iters = 0;
  if (i < J.off + J.n) {
    const double xi = X[3 * i], yi = X[3 * i + 1], zi = X[3 * i + 2];
    const uint32_t id = B.ID[J.scur][i];
    const double m = J.uniform_mass ? J.mass : B.MASS[J.scur][i];
    // noise first: pure arithmetic that overlaps the latency of the list and
    // neighbour loads issued next
    double rx, ry, rz;
    langevin_kick<kF64>(J, id, m, s, start, rx, ry, rz);
    double Fx = 0.0, Fy = 0.0, Fz = 0.0;
    if (J.pair_kind != kPairNone) {
      if (kModel)
        model_forces<false, kF64>(J, B.models[job], B, X, i, id, xi, yi, zi, Fx, Fy, Fz, mtab);
      else
        pair_forces<kF64>(J, B, X, i, xi, yi, zi, Fx, Fy, Fz);
    }
    // the particle's own momentum and flag are loaded after the force loop,
    // which keeps them out of the loop's live registers
    double px = P[3 * i], py = P[3 * i + 1], pz = P[3 * i + 2];
    const bool cons = B.FLG[J.scur][i] != 0;
    double fx, fy, fz;
    combined_force(J, B, id, start, Fx, Fy, Fz, px, py, pz, rx, ry, rz, fx, fy, fz);
    double nx = 0.0, ny = 0.0, nz = 0.0, g0 = 0.0;
    if (cons) g0 = surf_eval(J, xi, yi, zi, nx, ny, nz);
    // momentum stage of step s-1 -> s: tangent projection (closed form of the linear Newton)
    if (!start) {
      px += J.half_dt * fx;
      py += J.half_dt * fy;
      pz += J.half_dt * fz;
      if (cons) {
        const double a = (nx * px + ny * py + nz * pz) / (nx * nx + ny * ny + nz * nz);
        px -= a * nx;
        py -= a * ny;
        pz -= a * nz;
      }
    }
    // position stage of step s -> s+1
    px += J.half_dt * fx;
    py += J.half_dt * fy;
    pz += J.half_dt * fz;
    double x1, y1, z1;
    if (cons) {
      iters = rattle_position(J, m, xi, yi, zi, g0, nx, ny, nz, px, py, pz, x1, y1, z1);
      if (iters < 0) {
        record_error(K, kErrNewton, id, s);
        iters = -iters;
      }
    } else {
      const double dtm = J.dt / m;
      x1 = xi + dtm * px;
      y1 = yi + dtm * py;
      z1 = zi + dtm * pz;
    }
    if (kStream) {
      // streaming stores: the new state is not read again in this launch, so
      // it should not displace the neighbour positions the other waves are
      // gathering from L2 (2M torus: step kernel 119 -> 107 us).  Used when the
      // step's data exceed the Infinity Cache; when they fit, ordinary stores
      // leave the new state there for the next step (1M particles: 5 % faster).
      // A template parameter, not a runtime flag: with both forms in one
      // kernel the compiler merges part of them into ordinary stores.
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
  if (threadIdx.x % kGroup == 0) {
    const int64_t g = first / kGroup;
    const double a = B.TACC[g] + sqrt(m2);
    B.TACC[g] = a;
    if (a > J.half_skin) atomicMin(&K.stop_at, s + 1);
    if (im > K.newton_max) atomicMax(&K.newton_max, im);
  }
}

#ifndef MDK_STEP32_WAVES
#define MDK_STEP32_WAVES 5
#endif

// FP32 pair forces (and FP32 Box-Muller): occupancy target MDK_STEP32_WAVES
// wavefronts per SIMD.
template <bool kStream>
__global__ void __launch_bounds__(kTile) __attribute__((amdgpu_waves_per_eu(MDK_STEP32_WAVES, 8)))
k_step_f32(DevBufs B, const int* __restrict__ tile_job, const int64_t* __restrict__ tile_first,
           const int* __restrict__ ntiles_ptr, int t) {
  step_body<false, false, kStream>(B, tile_job, tile_first, ntiles_ptr, t);
}

// FP64 pair forces and FP64 Box-Muller.
template <bool kStream>
__global__ void __launch_bounds__(kTile) k_step_f64(DevBufs B, const int* __restrict__ tile_job,
                                                    const int64_t* __restrict__ tile_first,
                                                    const int* __restrict__ ntiles_ptr, int t) {
  step_body<true, false, kStream>(B, tile_job, tile_first, ntiles_ptr, t);
}

#ifndef MDK_STEPMODEL_WAVES
#define MDK_STEPMODEL_WAVES 5
#endif

// Bead-model jobs: typed pairs, bonds, bends and the wall (FP64 force class);
// occupancy target MDK_STEPMODEL_WAVES wavefronts per SIMD (5 fits without
// spilling).
template <bool kStream>
__global__ void __launch_bounds__(kTile) __attribute__((amdgpu_waves_per_eu(MDK_STEPMODEL_WAVES, 8)))
k_step_model(DevBufs B, const int* __restrict__ tile_job, const int64_t* __restrict__ tile_first,
             const int* __restrict__ ntiles_ptr, int t) {
  step_body<true, true, kStream>(B, tile_job, tile_first, ntiles_ptr, t);
}

// The same with FP32 pair terms (and the FP32 Box-Muller transform).
template <bool kStream>
__global__ void __launch_bounds__(kTile) __attribute__((amdgpu_waves_per_eu(MDK_STEPMODEL_WAVES, 8)))
k_step_model_f32(DevBufs B, const int* __restrict__ tile_job, const int64_t* __restrict__ tile_first,
                 const int* __restrict__ ntiles_ptr, int t) {
  step_body<false, true, kStream>(B, tile_job, tile_first, ntiles_ptr, t);
}

// Finish: state at the current step m (x^m, p^m, f^m) and per-particle
// diagnostics, written by particle index.
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
    if (J.model) {
      Ui = model_forces<true, kF64>(J, B.models[job], B, X, i, id, xi, yi, zi, Fx, Fy, Fz);
    } else {
      pair_forces<kF64>(J, B, X, i, xi, yi, zi, Fx, Fy, Fz);
      Ui = pair_energy(J, B, X, i, xi, yi, zi);
    }
  }
  double rx, ry, rz, fx, fy, fz;
  langevin_kick<kF64>(J, id, m, s, start, rx, ry, rz);
  combined_force(J, B, id, start, Fx, Fy, Fz, px, py, pz, rx, ry, rz, fx, fy, fz);
  double nx = 0.0, ny = 0.0, nz = 0.0, g = 0.0;
  if (cons) g = surf_eval(J, xi, yi, zi, nx, ny, nz);
  if (!start) {
    px += J.half_dt * fx;
    py += J.half_dt * fy;
    pz += J.half_dt * fz;
    if (cons) {
      const double a = (nx * px + ny * py + nz * pz) / (nx * nx + ny * ny + nz * nz);
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
    const double nn = sqrt(nx * nx + ny * ny + nz * nz);
    gd = fabs(g) / nn;
    nv = fabs(nx * px + ny * py + nz * pz) / (nn * m);
  }
  B.OD[2 * C + o] = gd;
  B.OD[3 * C + o] = nv;
}

// ---------------------------------------------------------------------------
// Neighbour-list build: occupied-cell bitmap -> compact cell index by popcount
// prefix -> counting sort of particles into raster cell order -> lists.
// ---------------------------------------------------------------------------

// Cell coordinate along dimension k: wrapped into the grid when periodic (in
// FP64, exact for the integers involved; no 64-bit integer division), clamped
// to the edge cells otherwise.  The final clamp also keeps a wrap rounded far
// from the box, or a NaN, inside the grid.
__device__ __forceinline__ int cell_coord(const JobDev& J, int k, double v) {
  double c = floor((v - J.glo[k]) * J.inv_cs[k]);
  const double nc = (double)J.nc[k];
  if (J.periodic[k]) c -= nc * floor(c / nc);
  return (int)fmin(fmax(c, 0.0), nc - 1.0);
}

__device__ __forceinline__ uint32_t raster_of(const JobDev& J, int cx, int cy, int cz) {
  return ((uint32_t)cx * (uint32_t)J.nc[1] + (uint32_t)cy) * (uint32_t)J.nc[2] + (uint32_t)cz;
}

// Zero [base + start, base + start + len) for each range.
struct Range {
  int64_t start;
  int64_t len;
};

__global__ void k_zero_ranges(uint32_t* __restrict__ base, const Range* __restrict__ ranges, int nranges) {
  const Range r = ranges[blockIdx.y];
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < r.len; k += (int64_t)gridDim.x * blockDim.x)
    base[r.start + k] = 0u;
}

// Wavefront-level combining of atomics on equal addresses.  After a build the
// particles are stored in cell order, so neighbouring lanes usually share a
// bitmap word / cell counter.  Lanes are grouped into runs of equal keys; the
// runs of a wavefront issue their atomics in one instruction (runs with equal
// keys that are not adjacent simply issue separate atomics).
constexpr uint32_t kNoKey = 0xFFFFFFFFu;

__device__ __forceinline__ unsigned long long lanemask_le(int lane) {
  return lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
}

// First lane of the run of equal keys that contains this lane.
__device__ __forceinline__ int run_start(uint32_t key, int lane, unsigned long long* heads_out) {
  const uint32_t prev = __shfl_up(key, 1, 64);
  const bool head = lane == 0 || prev != key;
  const unsigned long long heads = __ballot(head);
  *heads_out = heads;
  return 63 - __clzll((long long)(heads & lanemask_le(lane)));
}

__global__ void __launch_bounds__(kTile) k_mark(DevBufs B, const int* __restrict__ tile_job,
                                                const int64_t* __restrict__ tile_first) {
  const int job = uniform_int(tile_job[blockIdx.x]);
  const JobDev& J = B.jobs[job];
  const int64_t i = uniform_i64(tile_first[blockIdx.x]) + threadIdx.x;
  const bool valid = i < J.off + J.n;
  uint32_t key = kNoKey, bits = 0u;
  if (valid) {
    const double* X = B.X[J.xcur];
    const double px = X[3 * i], py = X[3 * i + 1], pz = X[3 * i + 2];
    const int cx = cell_coord(J, 0, px), cy = cell_coord(J, 1, py), cz = cell_coord(J, 2, pz);
    const uint32_t r = raster_of(J, cx, cy, cz);
    B.RASTER[i] = r;
    key = r >> 5;
    bits = 1u << (r & 31);
  }
  const int lane = threadIdx.x & 63;
  unsigned long long heads;
  const int start = run_start(key, lane, &heads);
  // OR over the run, accumulated towards its last lane
  uint32_t v = bits;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, 64);
    if (lane - o >= start) v |= t;
  }
  const bool tail = lane == 63 || ((heads >> (lane + 1)) & 1ull);
  if (tail && key != kNoKey) atomicOr(&B.BM[J.bm_off + key], v);
  // a list build starts the job's bookkeeping afresh (stored last, so that no
  // read of the job record has to wait behind it)
  if (i == J.off) B.book[job] = fresh_book();
}

__global__ void __launch_bounds__(kTile) k_count(DevBufs B, const int* __restrict__ tile_job,
                                                 const int64_t* __restrict__ tile_first) {
  const int job = uniform_int(tile_job[blockIdx.x]);
  const JobDev& J = B.jobs[job];
  const int64_t i = uniform_i64(tile_first[blockIdx.x]) + threadIdx.x;
  const bool valid = i < J.off + J.n;
  uint32_t key = kNoKey;
  if (valid) {
    const uint32_t r = B.RASTER[i];
    const int64_t w = J.bm_off + (r >> 5);
    key = B.WOFF[w] + __popc(B.BM[w] & ((1u << (r & 31)) - 1u));
    B.CID[i] = key;
  }
  const int lane = threadIdx.x & 63;
  unsigned long long heads;
  const int start = run_start(key, lane, &heads);
  uint32_t base = 0u;
  if (start == lane && key != kNoKey) {
    const unsigned long long later = heads & ~lanemask_le(lane);
    const int next = later ? __ffsll((long long)later) - 1 : 64;
    base = atomicAdd(&B.CCNT[J.off + key], (uint32_t)(next - lane));
  }
  base = __shfl(base, start, 64);
  if (valid) B.RANK[i] = base + (uint32_t)(lane - start);
}

// Destination of every slot in the new (cell) order: SRC[new slot] = old slot,
// and the inverse permutation by particle index.
__global__ void __launch_bounds__(kTile) k_perm(DevBufs B, const int* __restrict__ tile_job,
                                                const int64_t* __restrict__ tile_first) {
  const int job = uniform_int(tile_job[blockIdx.x]);
  const JobDev& J = B.jobs[job];
  const int64_t i = uniform_i64(tile_first[blockIdx.x]) + threadIdx.x;
  const int64_t off = J.off;
  if (i >= off + J.n) return;
  // the independent loads first, together
  const uint32_t cid = B.CID[i], rank = B.RANK[i], id = B.ID[J.scur][i];
  const int64_t d = off + B.CSTART[off + cid] + rank;
  B.SRC[d] = (uint32_t)(i - off);
  B.INV[off + id] = (uint32_t)(d - off);
}

// Gather the state into the new order: consecutive threads write consecutive
// slots (whole cache lines), the reads follow the permutation.
__global__ void __launch_bounds__(kTile) k_gather(DevBufs B, const int* __restrict__ tile_job,
                                                  const int64_t* __restrict__ tile_first) {
  const int job = uniform_int(tile_job[blockIdx.x]);
  const JobDev& J = B.jobs[job];
  const int64_t d = uniform_i64(tile_first[blockIdx.x]) + threadIdx.x;
  if (d >= J.off + J.n) return;
  const int64_t i = J.off + B.SRC[d];
  const double* __restrict__ Xs = B.X[J.xcur];
  double* __restrict__ Xd = B.X[J.xcur ^ 1];
  const double* __restrict__ Ps = B.P[J.pcur];
  double* __restrict__ Pd = B.P[J.pcur ^ 1];
  // every load before the first store: source and destination are different
  // buffers, and this way the loads are in flight together instead of each
  // waiting for the store before it
  double x[3], p[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    x[k] = Xs[3 * i + k];
    p[k] = Ps[3 * i + k];
  }
  const int sc = J.scur;
  const bool per_mass = !J.uniform_mass, model = J.model != 0;
  const uint32_t id = B.ID[sc][i];
  const uint8_t flag = B.FLG[sc][i];
  const double mass = per_mass ? B.MASS[sc][i] : 0.0;
  const uint8_t type = model ? B.TYPE[sc][i] : (uint8_t)0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    Xd[3 * d + k] = x[k];
    Pd[3 * d + k] = p[k];
  }
  B.ID[sc ^ 1][d] = id;
  B.FLG[sc ^ 1][d] = flag;
  if (per_mass) B.MASS[sc ^ 1][d] = mass;
  uint32_t w = id;
  if (model) {
    // bead model: the type rides in the top two bits of the record's index
    B.TYPE[sc ^ 1][d] = type;
    w |= (uint32_t)type << kTypeShift;
  }
  B.PK[d] = make_float4((float)x[0], (float)x[1], (float)x[2], __uint_as_float(w));
}

// Occupied cells with raster index below r, for the compact cell index.
__device__ __forceinline__ uint32_t cells_before(const DevBufs& B, const JobDev& J, uint32_t r) {
  const int64_t w = J.bm_off + (r >> 5);
  return B.WOFF[w] + __popc(B.BM[w] & ((1u << (r & 31)) - 1u));
}

// Cell coordinate c + d along dimension k for a stencil offset d in {-1,0,1}:
// wrapped when periodic (offsets that would repeat a cell when the periodic
// count is below 3 are dropped), dropped outside a non-periodic grid.
__device__ __forceinline__ bool stencil_coord(const JobDev& J, int k, int c, int d, int& out) {
  const int nc = J.nc[k];
  if (J.periodic[k]) {
    if (nc < 3 && (d < 0 || d >= nc)) return false;
    out = (c + d + nc) % nc;
    return true;
  }
  out = c + d;
  return out >= 0 && out < nc;
}

// Slot ranges (relative to the job) of one stencil column: cells (x, y, z-1..z+1),
// split in two runs when z wraps.
struct ColumnRange {
  uint32_t b0, e0, b1, e1;
};

__device__ __forceinline__ ColumnRange column_range(const DevBufs& B, const JobDev& J, int cx, int cy, int col,
                                                    int za0, int zb0, int za1, int zb1) {
  ColumnRange r{0u, 0u, 0u, 0u};
  int ax, ay;
  if (!stencil_coord(J, 0, cx, col / 3 - 1, ax) || !stencil_coord(J, 1, cy, col % 3 - 1, ay)) return r;
  const int64_t base = J.off;
  const uint32_t c0 = ((uint32_t)ax * (uint32_t)J.nc[1] + (uint32_t)ay) * (uint32_t)J.nc[2];
  r.b0 = B.CSTART[base + cells_before(B, J, c0 + (uint32_t)za0)];
  r.e0 = B.CSTART[base + cells_before(B, J, c0 + (uint32_t)zb0 + 1u)];
  if (zb1 >= za1) {
    r.b1 = B.CSTART[base + cells_before(B, J, c0 + (uint32_t)za1)];
    r.e1 = B.CSTART[base + cells_before(B, J, c0 + (uint32_t)zb1 + 1u)];
  }
  return r;
}

// Insert particle index q into this lane's list, kept sorted by particle index
// in LDS ([kmax][kNlistBlock], thread-minor so lanes hit distinct banks).  cnt counts every
// candidate accepted, stored or not (cnt > kmax signals overflow).
__device__ __forceinline__ void list_insert(uint32_t* kid, int lane, int kmax, int& cnt, uint32_t q) {
  if (cnt < kmax) {
    int k = cnt;
    while (k > 0 && kid[(k - 1) * kNlistBlock + lane] > q) {
      kid[k * kNlistBlock + lane] = kid[(k - 1) * kNlistBlock + lane];
      --k;
    }
    kid[k * kNlistBlock + lane] = q;
  }
  ++cnt;
}

// Append slot q to this lane's list in LDS (lists of the FP32 class stay in
// the order the stencil walk finds them, which is slot order).
__device__ __forceinline__ void list_append(uint32_t* kid, int lane, int kmax, int& cnt, uint32_t q) {
  if (cnt < kmax) kid[cnt * kNlistBlock + lane] = q;
  ++cnt;
}

// z cells of the stencil around cz: [za0, zb0] and, when z wraps, [za1, zb1].
__device__ __forceinline__ void z_runs(const JobDev& J, int cz, int& za0, int& zb0, int& za1, int& zb1) {
  const int ncz = J.nc[2];
  za1 = 0, zb1 = -1;
  if (J.periodic[2] && ncz >= 3) {
    if (cz == 0) {
      za0 = 0, zb0 = 1, za1 = ncz - 1, zb1 = ncz - 1;
    } else if (cz == ncz - 1) {
      za0 = 0, zb0 = 0, za1 = cz - 1, zb1 = cz;
    } else {
      za0 = cz - 1, zb0 = cz + 1;
    }
  } else if (J.periodic[2]) {
    za0 = 0, zb0 = ncz - 1;
  } else {
    za0 = cz > 0 ? cz - 1 : 0;
    zb0 = cz + 1 < ncz ? cz + 1 : ncz - 1;
  }
}

// One lane walks its own 27-cell stencil: 9 contiguous z-runs of slots, the next
// column's lookups in flight while the current one is scanned.  Candidates are
// read from the packed FP32 records (one 16-byte load each), kListBatch at a
// time; the last batch of a run is padded with repeats of its last record.
// The FP32 distance test uses the list radius widened by a bound on the FP32
// rounding of both positions and of the separation (times eight), so it accepts
// every pair closer than the list radius; the few extra pairs it may accept lie
// beyond the cut-off and add nothing to the forces.
#ifndef MDK_LIST_BATCH
#define MDK_LIST_BATCH 4
#endif
constexpr int kListBatch = MDK_LIST_BATCH;

__device__ __forceinline__ void min_image_f(const JobDev& J, float& dx, float& dy, float& dz) {
  if (J.periodic[0]) dx -= (float)J.box_len[0] * rintf(dx * (float)J.inv_box_len[0]);
  if (J.periodic[1]) dy -= (float)J.box_len[1] * rintf(dy * (float)J.inv_box_len[1]);
  if (J.periodic[2]) dz -= (float)J.box_len[2] * rintf(dz * (float)J.inv_box_len[2]);
}

// kModel: bead model (FP64 class): each candidate is tested against the list
// radius of its type pair, rc_ab + skin, and pairs inside a molecule are left out.
template <bool kSorted, bool kModel>
__device__ __forceinline__ void nlist_lane(const DevBufs& B, const JobDev& J, int64_t i, double xi, double yi,
                                           double zi, int cx, int cy, int cz, uint32_t* kid, int lane, int kmax,
                                           int& cnt, uint32_t myid, const ModelDev* M, int ti) {
  int za0, zb0, za1, zb1;
  z_runs(J, cz, za0, zb0, za1, zb1);
  const int64_t base = J.off;
  const bool anyper = J.periodic[0] | J.periodic[1] | J.periodic[2];
  const float4* __restrict__ PK = B.PK;
  double lper = 0.0;
  for (int k = 0; k < 3; ++k)
    if (J.periodic[k]) lper = fmax(lper, J.box_len[k]);
  const double rl = sqrt(J.rlist2);
  const double delta = 0x1p-21 * (2.0 * fmax(fabs(xi), fmax(fabs(yi), fabs(zi))) + 3.0 * rl + lper);
  const float thr = (float)((rl + delta) * (rl + delta) * (1.0 + 0x1p-20));
  const float xf = (float)xi, yf = (float)yi, zf = (float)zi;
  // bead model: list radius per partner type (rounding bound as above, which
  // covers the shorter radii too); candidates with particle index in
  // [mstart, mstart + bpm) share this molecule
  float tthr[kMaxTypes];
  if (kModel) {
    const double skin = 2.0 * J.half_skin;
#pragma unroll
    for (int b = 0; b < kMaxTypes; ++b) {
      const double r = sqrt(M->rc2[ti * kMaxTypes + b]) + skin;
      tthr[b] = (float)((r + delta) * (r + delta) * (1.0 + 0x1p-20));
    }
  }
  const uint32_t bpm = (uint32_t)J.bpm, mstart = bpm != 0u ? (myid / bpm) * bpm : 0u;  // bpm = 0: no molecules
  auto scan = [&](uint32_t b, uint32_t e) {
    const int64_t end = base + e;
    if (b >= e) return;
    // software-pipelined: the next batch's records are loaded while this one is
    // tested (past the end the loads repeat the last record and are not used)
    float4 nxt[kListBatch];
#pragma unroll
    for (int u = 0; u < kListBatch; ++u) nxt[u] = PK[base + b + u < end ? base + b + u : end - 1];
    for (int64_t j = base + b; j < end; j += kListBatch) {
      float4 r[kListBatch];
#pragma unroll
      for (int u = 0; u < kListBatch; ++u) {
        r[u] = nxt[u];
        const int64_t jn = j + kListBatch + u;
        nxt[u] = PK[jn < end ? jn : end - 1];
      }
#pragma unroll
      for (int u = 0; u < kListBatch; ++u) {
        float dx = xf - r[u].x, dy = yf - r[u].y, dz = zf - r[u].z;
        if (anyper) min_image_f(J, dx, dy, dz);
        const float d2 = dx * dx + dy * dy + dz * dz;
        const uint32_t w = __float_as_uint(r[u].w);
        uint32_t q;
        bool take;
        if (kModel) {
          const uint32_t tj = w >> kTypeShift;
          q = w & kIdMask;
          const float t = tj == 0u ? tthr[0] : (tj == 1u ? tthr[1] : (tj == 2u ? tthr[2] : tthr[3]));
          take = d2 < t && q - mstart >= bpm;
        } else {
          q = w;
          take = d2 < thr && w - mstart >= bpm;
        }
        if (j + u < end && j + u != i && take) {
          if (kSorted)
            list_insert(kid, lane, kmax, cnt, q);
          else  // job-local slot (bead model: partner type in the top bits)
            list_append(kid, lane, kmax, cnt, (uint32_t)(j + u - base) | (kModel ? w & ~kIdMask : 0u));
        }
      }
    }
  };
  ColumnRange cur = column_range(B, J, cx, cy, 0, za0, zb0, za1, zb1);
  for (int col = 0; col < 9; ++col) {
    ColumnRange nxt{0u, 0u, 0u, 0u};
    if (col + 1 < 9) nxt = column_range(B, J, cx, cy, col + 1, za0, zb0, za1, zb1);
    scan(cur.b0, cur.e0);
    scan(cur.b1, cur.e1);
    cur = nxt;
  }
}

// One uint4 row of a list (entries k .. k+3 of slot i).  Streaming (as the
// step's state stores, when the data exceed the Infinity Cache): the lists
// are read in the next step, not in this launch, and would otherwise
// displace the candidate records the build is reading from L2.
template <bool kStream>
__device__ __forceinline__ void store_row(uint32_t* NL, int64_t C, int k, int64_t i, const uint32_t* v) {
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  const v4u row = {v[0], v[1], v[2], v[3]};
  v4u* dst = reinterpret_cast<v4u*>(NL) + (int64_t)(k >> 2) * C + i;
  if (kStream)
    __builtin_nontemporal_store(row, dst);
  else
    *dst = row;
}

// Neighbour-list build, one lane per slot of the freshly sorted (raster cell)
// order, one workgroup per tile.  Each lane walks its own stencil and
// stages its list in LDS.  FP64 class: kept sorted by particle index and mapped
// back to slots through the inverse permutation of the sort, so that the FP64
// force sums run in particle-index order.  FP32 class: slots in the order the
// walk finds them (ascending), since its force sums do not depend on the order;
// neighbouring lanes then read neighbouring memory in the force loop.
// kWithModel: the instance launched when a bead-model job is among those built
// (the plain instance keeps the model path out of its register budget).
template <bool kWithModel, bool kStream>
__global__ void __launch_bounds__(kNlistBlock) k_nlist(DevBufs B, const int* __restrict__ tile_job,
                                                       const int64_t* __restrict__ tile_first) {
  extern __shared__ uint32_t kid[];  // lists [kmax][kNlistBlock]
  const int kmax = B.kmax;
  const int tile = (int)blockIdx.x / kNlistPerTile;
  const int job = uniform_int(tile_job[tile]);
  const JobDev& J = B.jobs[job];
  const int lane = threadIdx.x;
  const int64_t i = uniform_i64(tile_first[tile]) + ((int)blockIdx.x % kNlistPerTile) * kNlistBlock + lane;
  const int64_t base = J.off;
  int cnt = 0;
  if (i < J.off + J.n && J.pair_kind == kPairNone) {
    B.NCNT[i] = 0u;  // no pair potential: empty lists (the build only sorts)
  } else if (i < J.off + J.n) {
    const double* __restrict__ X = B.X[J.xcur ^ 1];  // the sorted copies written by k_gather
    const double xi = X[3 * i], yi = X[3 * i + 1], zi = X[3 * i + 2];
    const int cx = cell_coord(J, 0, xi), cy = cell_coord(J, 1, yi), cz = cell_coord(J, 2, zi);
    const int64_t C = B.C;
    int stored;
    if (J.force_fp64) {
      // FP64 class: sorted by particle index, mapped back to slots through the
      // inverse permutation, four lookups in flight at a time
      if (kWithModel && J.model)
        nlist_lane<true, kWithModel>(B, J, i, xi, yi, zi, cx, cy, cz, kid, lane, kmax, cnt, B.ID[J.scur ^ 1][i],
                               B.models + job, B.TYPE[J.scur ^ 1][i]);
      else
        nlist_lane<true, false>(B, J, i, xi, yi, zi, cx, cy, cz, kid, lane, kmax, cnt, 0u, nullptr, 0);
      stored = cnt < kmax ? cnt : kmax;
      // bead model: the partner's type rides in the top two bits of the entry
      const uint8_t* __restrict__ T = B.TYPE[J.scur ^ 1];
      const bool typed = kWithModel && J.model;
      for (int k = 0; k < stored; k += 4) {
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint32_t q = k + u < stored ? kid[(k + u) * kNlistBlock + lane] : 0u;  // 0: a valid index
          const uint32_t sl = (uint32_t)base + B.INV[base + q];
          v[u] = k + u < stored ? sl : 0u;
          if (typed && k + u < stored) v[u] |= (uint32_t)T[sl] << kTypeShift;
        }
        store_row<kStream>(B.NL, C, k, i, v);
      }
    } else {
      // FP32 class: slot order, as found
      if (kWithModel && J.model)
        nlist_lane<false, kWithModel>(B, J, i, xi, yi, zi, cx, cy, cz, kid, lane, kmax, cnt, B.ID[J.scur ^ 1][i],
                                      B.models + job, B.TYPE[J.scur ^ 1][i]);
      else
        nlist_lane<false, false>(B, J, i, xi, yi, zi, cx, cy, cz, kid, lane, kmax, cnt, 0u, nullptr, 0);
      stored = cnt < kmax ? cnt : kmax;
      for (int k = 0; k < stored; k += 4) {
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          // job-local slot, with the bead model's partner type in the top bits
          const uint32_t q = kid[(k + u) * kNlistBlock + lane];
          const uint32_t sl = kWithModel && J.model ? ((uint32_t)base + (q & kIdMask)) | (q & ~kIdMask)
                                                    : (uint32_t)base + q;
          v[u] = k + u < stored ? sl : 0u;
        }
        store_row<kStream>(B.NL, C, k, i, v);
      }
    }
    B.NCNT[i] = (uint32_t)stored;
  }
  // list statistics of these 64 slots (no atomics); an overflow stops the job
  // before its first step on these lists
  uint32_t mx = (uint32_t)cnt, sm = (uint32_t)(cnt < kmax ? cnt : kmax);
  for (int o = 32; o > 0; o >>= 1) {
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
    sm += (uint32_t)__shfl_xor((int)sm, o, 64);
  }
  const int64_t g0 = i - (lane % kGroup);
  if (lane % kGroup == 0 && g0 < J.off + J.n) {
    B.NLSTAT[2 * (g0 / kGroup)] = mx;
    B.NLSTAT[2 * (g0 / kGroup) + 1] = sm;
    if ((int)mx > kmax) atomicMin(&B.book[job].stop_at, (long long)J.step0);
  }
}

// Diagnostics of one job from the finish kernel's per-particle values (Section
// 3.1: K and U summed, constraint residuals maximised), in two passes with a
// fixed reduction tree, so the result depends only on n, not on scheduling.
// Pass 1: workgroup b reduces its contiguous chunk into part[4 b .. 4 b + 3];
// pass 2: one workgroup reduces the partials into out[0..3] = K, U, gdist_max,
// nv_max.
constexpr int kDiagThreads = 256;
constexpr int kDiagBlocks = 256;

__device__ __forceinline__ void diag_tree(double* sk, double* su, double* sg, double* sv, int tid) {
  for (int w = kDiagThreads / 2; w > 0; w >>= 1) {
    __syncthreads();
    if (tid < w) {
      sk[tid] += sk[tid + w];
      su[tid] += su[tid + w];
      sg[tid] = fmax(sg[tid], sg[tid + w]);
      sv[tid] = fmax(sv[tid], sv[tid + w]);
    }
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kDiagThreads) k_diag_partial(const double* __restrict__ OD, int64_t C, int64_t off,
                                                               int64_t n, double* __restrict__ part) {
  __shared__ double sk[kDiagThreads], su[kDiagThreads], sg[kDiagThreads], sv[kDiagThreads];
  const int tid = threadIdx.x;
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * chunk, b1 = min(b0 + chunk, n);
  double k = 0.0, u = 0.0, g = 0.0, v = 0.0;
  for (int64_t i = b0 + tid; i < b1; i += kDiagThreads) {
    k += OD[off + i];
    u += OD[C + off + i];
    g = fmax(g, OD[2 * C + off + i]);
    v = fmax(v, OD[3 * C + off + i]);
  }
  sk[tid] = k, su[tid] = u, sg[tid] = g, sv[tid] = v;
  diag_tree(sk, su, sg, sv, tid);
  if (tid == 0) {
    double* o = part + 4 * blockIdx.x;
    o[0] = sk[0], o[1] = su[0], o[2] = sg[0], o[3] = sv[0];
  }
}

__global__ void __launch_bounds__(kDiagThreads) k_diag_final(const double* __restrict__ part, int nb,
                                                             double* __restrict__ out) {
  __shared__ double sk[kDiagThreads], su[kDiagThreads], sg[kDiagThreads], sv[kDiagThreads];
  const int tid = threadIdx.x;
  double k = 0.0, u = 0.0, g = 0.0, v = 0.0;
  for (int b = tid; b < nb; b += kDiagThreads) {
    k += part[4 * b];
    u += part[4 * b + 1];
    g = fmax(g, part[4 * b + 2]);
    v = fmax(v, part[4 * b + 3]);
  }
  sk[tid] = k, su[tid] = u, sg[tid] = g, sv[tid] = v;
  diag_tree(sk, su, sg, sv, tid);
  if (tid == 0) out[0] = sk[0], out[1] = su[0], out[2] = sg[0], out[3] = sv[0];
}

// Per-job reductions read by the host after a chunk of steps: the largest
// per-tile displacement bound and, after list builds, the list statistics.
// One workgroup per job record.
constexpr int kStatsThreads = 1024;
__global__ void __launch_bounds__(kStatsThreads) k_job_stats(DevBufs B, int with_lists) {
  __shared__ double ra[kStatsThreads / 64], rs[kStatsThreads / 64];
  __shared__ uint32_t rm[kStatsThreads / 64];
  const int job = blockIdx.x;
  const JobDev& J = B.jobs[job];
  if (J.n <= 0) return;
  double a = 0.0, sm = 0.0;
  uint32_t mx = 0u;
  const int64_t g0 = J.off / kGroup, g1 = (J.off + J.n + kGroup - 1) / kGroup;
  // four independent loads in flight per thread (one workgroup serves a job)
  constexpr int64_t kStride = kStatsThreads;
  int64_t g = g0 + threadIdx.x;
  for (; g + 3 * kStride < g1; g += 4 * kStride) {
    const double t0 = B.TACC[g], t1 = B.TACC[g + kStride], t2 = B.TACC[g + 2 * kStride], t3 = B.TACC[g + 3 * kStride];
    a = fmax(fmax(a, fmax(t0, t1)), fmax(t2, t3));
  }
  for (; g < g1; g += kStride) a = fmax(a, B.TACC[g]);
  if (with_lists) {
    // list-length sums are integers: exact in FP64 in any order
    const uint2* __restrict__ st = reinterpret_cast<const uint2*>(B.NLSTAT);
    g = g0 + threadIdx.x;
    for (; g + 3 * kStride < g1; g += 4 * kStride) {
      const uint2 q0 = st[g], q1 = st[g + kStride], q2 = st[g + 2 * kStride], q3 = st[g + 3 * kStride];
      mx = max(mx, max(max(q0.x, q1.x), max(q2.x, q3.x)));
      sm += (double)q0.y + (double)q1.y + (double)q2.y + (double)q3.y;
    }
    for (; g < g1; g += kStride) {
      const uint2 q = st[g];
      mx = max(mx, q.x);
      sm += (double)q.y;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    a = fmax(a, __shfl_xor(a, o, 64));
    sm += __shfl_xor(sm, o, 64);
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) ra[w] = a, rs[w] = sm, rm[w] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < kStatsThreads / 64; ++q) a = fmax(a, ra[q]), sm += rs[q], mx = max(mx, rm[q]);
    JobBook& K = B.book[job];
    K.a_now = a;
    if (with_lists) {
      K.nl_max = (int)mx;
      K.nl_sum = sm;
    }
  }
}

// Dynamic LDS of k_nlist for a list capacity kmax.
constexpr size_t nlist_lds_bytes(int kmax) { return (size_t)kmax * kNlistBlock * sizeof(uint32_t); }

// ---------------------------------------------------------------------------
// Segmented exclusive scan, three passes, staged in LDS.
// A chunk is a piece of one segment; chunks of a segment are consecutive in
// the chunk list.  Pass A scans each chunk in LDS and writes its total; pass B
// scans the totals within each segment (one workgroup); pass C adds them.
// ---------------------------------------------------------------------------
struct Chunk {
  int64_t start;   // element index of the chunk's first element
  int len;         // elements in the chunk (<= kScanChunk)
  int seg_first;   // index (in the chunk list) of the segment's first chunk
};

constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kScanChunk = kScanThreads * kScanPer;

template <bool kPopc>
__global__ void __launch_bounds__(kScanThreads) k_scan_a(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                         const Chunk* __restrict__ chunks, uint32_t* __restrict__ sums) {
  __shared__ uint32_t tot[kScanThreads];
  const Chunk ch = chunks[blockIdx.x];
  uint32_t v[kScanPer];
  uint32_t run = 0;
#pragma unroll
  for (int e = 0; e < kScanPer; ++e) {
    const int idx = threadIdx.x * kScanPer + e;
    uint32_t a = idx < ch.len ? in[ch.start + idx] : 0u;
    if (kPopc) a = __popc(a);
    v[e] = run;
    run += a;
  }
  tot[threadIdx.x] = run;
  __syncthreads();
  // Hillis-Steele inclusive scan of the per-thread totals
  for (int o = 1; o < kScanThreads; o <<= 1) {
    const uint32_t add = threadIdx.x >= o ? tot[threadIdx.x - o] : 0u;
    __syncthreads();
    tot[threadIdx.x] += add;
    __syncthreads();
  }
  const uint32_t base = threadIdx.x > 0 ? tot[threadIdx.x - 1] : 0u;
#pragma unroll
  for (int e = 0; e < kScanPer; ++e) {
    const int idx = threadIdx.x * kScanPer + e;
    if (idx < ch.len) out[ch.start + idx] = base + v[e];
  }
  if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = tot[kScanThreads - 1];
}

constexpr int kScanB = 1024;

// Segmented exclusive scan of the chunk totals in one workgroup, 1024 at a
// time, carrying the running total of the segment that crosses a tile edge.
__global__ void __launch_bounds__(kScanB) k_scan_b(uint32_t* __restrict__ sums, const Chunk* __restrict__ chunks,
                                                   int nchunks) {
  __shared__ uint32_t sv[kScanB];
  __shared__ int sf[kScanB];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0u;
  __syncthreads();
  for (int base = 0; base < nchunks; base += kScanB) {
    const int c = base + threadIdx.x;
    const bool in = c < nchunks;
    const uint32_t v = in ? sums[c] : 0u;
    const int head = in ? (chunks[c].seg_first == c) : 1;
    sv[threadIdx.x] = v;
    sf[threadIdx.x] = head;
    __syncthreads();
    for (int o = 1; o < kScanB; o <<= 1) {
      uint32_t av = 0u;
      int af = 0;
      const bool take = threadIdx.x >= o;
      if (take) {
        av = sv[threadIdx.x - o];
        af = sf[threadIdx.x - o];
      }
      __syncthreads();
      if (take && !sf[threadIdx.x]) sv[threadIdx.x] += av;
      if (take) sf[threadIdx.x] |= af;
      __syncthreads();
    }
    uint32_t incl = sv[threadIdx.x];
    if (!sf[threadIdx.x]) incl += carry;  // no segment start between the tile edge and here
    if (in) sums[c] = incl - v;
    __syncthreads();
    if (threadIdx.x == kScanB - 1) carry = incl;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_c(uint32_t* __restrict__ out, const Chunk* __restrict__ chunks,
                                                         const uint32_t* __restrict__ sums) {
  const Chunk ch = chunks[blockIdx.x];
  const uint32_t add = sums[blockIdx.x];
  if (add == 0u) return;
  for (int idx = threadIdx.x; idx < ch.len; idx += kScanThreads) out[ch.start + idx] += add;
}

}  // namespace mdk
