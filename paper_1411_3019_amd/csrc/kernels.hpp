// kernels.hpp -- HIP kernels of the RATTLE + Langevin hot path (gfx950).
//
// Per-particle kernels run one thread per particle over "tiles": 256
// consecutive slots of one job.  A launch covers the tiles of many jobs
// (tile -> job table), so one launch advances every resident system.
//
// Step kernel (one launch per time step), for particle i of a job at step s:
//   input  x^s (buffer parity xin), p^{s-1/2} (or p^s at a start), neighbour list
//   force  F_i(x^s) from the list (sorted by particle index)
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

// Maximum of a non-negative double over the workgroup, then atomically into
// *dst (the bit patterns of non-negative doubles order like the values).
__device__ __forceinline__ void block_max_to(double v, unsigned long long* dst, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
    atomicMax(dst, (unsigned long long)__double_as_longlong(m));
  }
}

__device__ __forceinline__ int block_max_int(int v, int* red) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  int m = red[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = max(m, red[w]);
  return m;
}

__device__ __forceinline__ void record_error(JobBook& K, int code, uint32_t id) {
  if (atomicCAS(&K.err_code, 0, code) == 0) K.err_id = (int)id;
  atomicOr(&K.flags, (int)kFlagError);
}

// Combined force f^s of Algorithm S1 for one particle (FP64 arithmetic; the
// normals come from the FP64 or the FP32 Box-Muller transform with kF64).
template <bool kF64>
__device__ __forceinline__ void combined_force(const JobDev& J, const DevBufs& B, int64_t i, uint32_t id,
                                               double m, long long s, double Fx, double Fy, double Fz,
                                               double px, double py, double pz, bool start, double& fx,
                                               double& fy, double& fz) {
  if (J.mode == kModeStartGiven && start) {
    const int64_t o = J.off + id;
    fx = B.FC[o];
    fy = B.FC[B.C + o];
    fz = B.FC[2 * B.C + o];
    return;
  }
  if (J.gamma > 0.0) {
    double a0, a1, a2;
    langevin_normals<kF64>(J.seed, id, s, a0, a1, a2);
    const double k = sqrt(m) * J.noise_k;
    if (start) {
      // no earlier draw exists: the previous draw is taken equal to this one
      fx = J.b * (Fx - J.gamma * px + k * a0);
      fy = J.b * (Fy - J.gamma * py + k * a1);
      fz = J.b * (Fz - J.gamma * pz + k * a2);
    } else {
      double r0, r1, r2;
      langevin_normals<kF64>(J.seed, id, s - 1, r0, r1, r2);
      const double hk = 0.5 * k;
      fx = J.b * (Fx - J.gamma * px + hk * (a0 + r0));
      fy = J.b * (Fy - J.gamma * py + hk * (a1 + r1));
      fz = J.b * (Fz - J.gamma * pz + hk * (a2 + r2));
    }
  } else {
    fx = Fx;
    fy = Fy;
    fz = Fz;
  }
}

template <bool kF64>
__global__ void __launch_bounds__(kTile) k_step(DevBufs B, const int* __restrict__ tile_job,
                                                const int64_t* __restrict__ tile_first,
                                                const int* __restrict__ ntiles_ptr, int t) {
  __shared__ double red[kTile / 64];
  __shared__ int redi[kTile / 64];
  // the grid may be larger than the tile list (it is sized once per graph);
  // surplus workgroups leave at once
  const int ntiles = *ntiles_ptr;
  if ((int)blockIdx.x >= ntiles) return;
  const int b = xcd_remap((int)blockIdx.x, ntiles);
  const int job = tile_job[b];
  const int64_t first = tile_first[b];
  const JobDev& J = B.jobs[job];
  JobBook& K = B.book[job];
  if (K.flags != 0 || t >= J.remaining) return;
  const long long s = J.step0 + t;
  const bool start = (J.mode != kModeSteady) && (t == 0);
  // list validity: accumulated displacement since the last build, through step s-1
  const double A = K.acc[(s + 1) & 1] + __longlong_as_double((long long)K.dmax[(s + 2) % 3]);
  if (A > J.half_skin) {
    if (threadIdx.x == 0) {
      K.stale_step = s;
      atomicOr(&K.flags, (int)kFlagStale);
    }
    return;
  }
  if (first == J.off && threadIdx.x == 0) {
    K.acc[s & 1] = A;
    K.dmax[(s + 1) % 3] = 0ull;
  }
  const int xin = J.xcur ^ (t & 1);
  const double* __restrict__ X = B.X[xin];
  double* __restrict__ Xo = B.X[xin ^ 1];
  double* __restrict__ P = B.P[J.pcur];
  const int64_t C = B.C;
  const int64_t i = first + threadIdx.x;
  double disp = 0.0;
  int iters = 0;
  if (i < J.off + J.n) {
    const double xi = X[i], yi = X[C + i], zi = X[2 * C + i];
    double Fx = 0.0, Fy = 0.0, Fz = 0.0;
    if (J.pair_kind != kPairNone) pair_forces<kF64>(J, B, X, i, xi, yi, zi, Fx, Fy, Fz);
    // the particle's own momentum and tags are loaded after the force loop,
    // which keeps them out of the loop's live registers
    double px = P[i], py = P[C + i], pz = P[2 * C + i];
    const uint32_t id = B.ID[J.scur][i];
    const bool cons = B.FLG[J.scur][i] != 0;
    const double m = J.uniform_mass ? J.mass : B.MASS[J.scur][i];
    double fx, fy, fz;
    combined_force<kF64>(J, B, i, id, m, s, Fx, Fy, Fz, px, py, pz, start, fx, fy, fz);
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
        record_error(K, kErrNewton, id);
        iters = -iters;
      }
    } else {
      const double dtm = J.dt / m;
      x1 = xi + dtm * px;
      y1 = yi + dtm * py;
      z1 = zi + dtm * pz;
    }
    Xo[i] = x1;
    Xo[C + i] = y1;
    Xo[2 * C + i] = z1;
    P[i] = px;
    P[C + i] = py;
    P[2 * C + i] = pz;
    const double dx = x1 - xi, dy = y1 - yi, dz = z1 - zi;
    disp = sqrt(dx * dx + dy * dy + dz * dz);
    if (!(disp <= 1e300) || !(fabs(px) + fabs(py) + fabs(pz) <= 1e300)) {
      record_error(K, kErrNaN, id);
      disp = 0.0;
    }
  }
  block_max_to(disp, &K.dmax[s % 3], red);
  const int im = block_max_int(iters, redi);
  if (threadIdx.x == 0 && im > 0) atomicMax(&K.newton_max, im);
}

// Finish: state at the current step m (x^m, p^m, f^m) and per-particle
// diagnostics, written by particle index.
template <bool kF64>
__global__ void __launch_bounds__(kTile) k_finish(DevBufs B, const int* __restrict__ tile_job,
                                                  const int64_t* __restrict__ tile_first) {
  const int job = tile_job[blockIdx.x];
  const int64_t first = tile_first[blockIdx.x];
  const JobDev& J = B.jobs[job];
  const int64_t C = B.C;
  const int64_t i = first + threadIdx.x;
  if (i >= J.off + J.n) return;
  const double* __restrict__ X = B.X[J.xcur];
  const double* __restrict__ P = B.P[J.pcur];
  const double xi = X[i], yi = X[C + i], zi = X[2 * C + i];
  double px = P[i], py = P[C + i], pz = P[2 * C + i];
  const uint32_t id = B.ID[J.scur][i];
  const bool cons = B.FLG[J.scur][i] != 0;
  const double m = J.uniform_mass ? J.mass : B.MASS[J.scur][i];
  const bool start = J.mode != kModeSteady;
  const long long s = J.step0;
  double Fx = 0.0, Fy = 0.0, Fz = 0.0, Ui = 0.0;
  if (J.pair_kind != kPairNone) {
    pair_forces<kF64>(J, B, X, i, xi, yi, zi, Fx, Fy, Fz);
    Ui = pair_energy(J, B, X, i, xi, yi, zi);
  }
  double fx, fy, fz;
  combined_force<kF64>(J, B, i, id, m, s, Fx, Fy, Fz, px, py, pz, start, fx, fy, fz);
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
  B.OX[o] = xi;
  B.OX[C + o] = yi;
  B.OX[2 * C + o] = zi;
  B.OP[o] = px;
  B.OP[C + o] = py;
  B.OP[2 * C + o] = pz;
  B.OF[o] = fx;
  B.OF[C + o] = fy;
  B.OF[2 * C + o] = fz;
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

__device__ __forceinline__ int cell_coord(const JobDev& J, int k, double v) {
  long long c = (long long)floor((v - J.glo[k]) * J.inv_cs[k]);
  const long long nc = J.nc[k];
  if (J.periodic[k]) {
    c %= nc;
    if (c < 0) c += nc;
  } else {
    c = c < 0 ? 0 : (c >= nc ? nc - 1 : c);
  }
  return (int)c;
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

// Wavefront-level combining of atomics on equal addresses: after a build the
// particles are stored in cell order, so neighbouring lanes usually hit the
// same bitmap word / cell counter.  One lane per distinct key issues the atomic.
constexpr uint32_t kNoKey = 0xFFFFFFFFu;

__global__ void __launch_bounds__(kTile) k_mark(DevBufs B, const int* __restrict__ tile_job,
                                                const int64_t* __restrict__ tile_first) {
  const int job = tile_job[blockIdx.x];
  const JobDev& J = B.jobs[job];
  const int64_t i = tile_first[blockIdx.x] + threadIdx.x;
  const bool valid = i < J.off + J.n;
  uint32_t key = kNoKey, bits = 0u;
  if (valid) {
    const double* X = B.X[J.xcur];
    const int64_t C = B.C;
    const int cx = cell_coord(J, 0, X[i]), cy = cell_coord(J, 1, X[C + i]), cz = cell_coord(J, 2, X[2 * C + i]);
    const uint32_t r = raster_of(J, cx, cy, cz);
    B.RASTER[i] = r;
    key = r >> 5;
    bits = 1u << (r & 31);
  }
  const int lane = threadIdx.x & 63;
  for (;;) {
    const unsigned long long act = __ballot(key != kNoKey);
    if (act == 0ull) break;
    const int leader = __ffsll((long long)act) - 1;
    const uint32_t k0 = __shfl(key, leader, 64);
    const bool mine = key == k0;
    uint32_t v = mine ? bits : 0u;
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    if (lane == leader) atomicOr(&B.BM[J.bm_off + k0], v);
    if (mine) key = kNoKey;
  }
}

__global__ void __launch_bounds__(kTile) k_count(DevBufs B, const int* __restrict__ tile_job,
                                                 const int64_t* __restrict__ tile_first) {
  const int job = tile_job[blockIdx.x];
  const JobDev& J = B.jobs[job];
  const int64_t i = tile_first[blockIdx.x] + threadIdx.x;
  const bool valid = i < J.off + J.n;
  uint32_t key = kNoKey;
  if (valid) {
    const uint32_t r = B.RASTER[i];
    const int64_t w = J.bm_off + (r >> 5);
    key = B.WOFF[w] + __popc(B.BM[w] & ((1u << (r & 31)) - 1u));
    B.CID[i] = key;
  }
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t rank = 0u;
  for (;;) {
    const unsigned long long act = __ballot(key != kNoKey);
    if (act == 0ull) break;
    const int leader = __ffsll((long long)act) - 1;
    const uint32_t k0 = __shfl(key, leader, 64);
    const unsigned long long m = __ballot(key == k0);
    uint32_t base = 0u;
    if (lane == leader) base = atomicAdd(&B.CCNT[J.off + k0], (uint32_t)__popcll(m));
    base = __shfl(base, leader, 64);
    if (key == k0) {
      rank = base + (uint32_t)__popcll(m & below);
      key = kNoKey;
    }
  }
  if (valid) B.RANK[i] = rank;
}

__global__ void __launch_bounds__(kTile) k_scatter(DevBufs B, const int* __restrict__ tile_job,
                                                   const int64_t* __restrict__ tile_first) {
  const int job = tile_job[blockIdx.x];
  const JobDev& J = B.jobs[job];
  const int64_t i = tile_first[blockIdx.x] + threadIdx.x;
  if (i >= J.off + J.n) return;
  const int64_t C = B.C;
  const int64_t d = J.off + B.CSTART[J.off + B.CID[i]] + B.RANK[i];
  const double* Xs = B.X[J.xcur];
  double* Xd = B.X[J.xcur ^ 1];
  const double* Ps = B.P[J.pcur];
  double* Pd = B.P[J.pcur ^ 1];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    Xd[k * C + d] = Xs[k * C + i];
    Pd[k * C + d] = Ps[k * C + i];
  }
  B.ID[J.scur ^ 1][d] = B.ID[J.scur][i];
  B.FLG[J.scur ^ 1][d] = B.FLG[J.scur][i];
  if (!J.uniform_mass) B.MASS[J.scur ^ 1][d] = B.MASS[J.scur][i];
}

// Offsets of the stencil along one dimension, without repeats when the
// periodic cell count is below 3.
__device__ __forceinline__ int stencil(const JobDev& J, int k, int c, int* out) {
  const int nc = J.nc[k];
  if (J.periodic[k]) {
    if (nc >= 3) {
      out[0] = (c + nc - 1) % nc;
      out[1] = c;
      out[2] = (c + 1) % nc;
      return 3;
    }
    out[0] = 0;
    if (nc == 2) out[1] = 1;
    return nc;
  }
  int m = 0;
  if (c > 0) out[m++] = c - 1;
  out[m++] = c;
  if (c + 1 < nc) out[m++] = c + 1;
  return m;
}

// Occupied cells with raster index below r, for the compact cell index.
__device__ __forceinline__ uint32_t cells_before(const DevBufs& B, const JobDev& J, uint32_t r) {
  const int64_t w = J.bm_off + (r >> 5);
  return B.WOFF[w] + __popc(B.BM[w] & ((1u << (r & 31)) - 1u));
}

// One wavefront per workgroup; each lane builds the list of one slot of the
// freshly sorted order.  Slots are in raster cell order (x-major, z fastest),
// so for each of the 9 (dx, dy) columns of the 27-cell stencil the cells
// z-1..z+1 are one contiguous slot range, found from two popcount lookups.
// Accepted neighbours are kept sorted by particle index in LDS
// ([kmax][64], lane-minor so lanes hit distinct banks).
__global__ void __launch_bounds__(kNlistBlock) k_nlist(DevBufs B, const int* __restrict__ tile_job,
                                                       const int64_t* __restrict__ tile_first) {
  extern __shared__ uint32_t lds[];
  const int kmax = B.kmax;
  uint32_t* kid = lds;
  uint32_t* kslot = lds + kmax * kNlistBlock;
  const int job = tile_job[blockIdx.x >> 2];
  const JobDev& J = B.jobs[job];
  const int64_t i = tile_first[blockIdx.x >> 2] + (blockIdx.x & 3) * kNlistBlock + threadIdx.x;
  if (i >= J.off + J.n) return;
  const int lane = threadIdx.x;
  const int64_t C = B.C;
  const int xs = J.xcur ^ 1, ss = J.scur ^ 1;  // the sorted copies written by k_scatter
  const double* __restrict__ X = B.X[xs];
  const uint32_t* __restrict__ ID = B.ID[ss];
  const double xi = X[i], yi = X[C + i], zi = X[2 * C + i];
  const int cx = cell_coord(J, 0, xi), cy = cell_coord(J, 1, yi), cz = cell_coord(J, 2, zi);
  int sx[3], sy[3];
  const int nx = stencil(J, 0, cx, sx), ny = stencil(J, 1, cy, sy);
  // z runs: [za0, zb0] and possibly a wrapped [za1, zb1]
  const int ncz = J.nc[2];
  int za[2], zb[2], nrun;
  if (J.periodic[2] && ncz >= 3) {
    if (cz == 0) {
      za[0] = 0, zb[0] = 1, za[1] = ncz - 1, zb[1] = ncz - 1, nrun = 2;
    } else if (cz == ncz - 1) {
      za[0] = 0, zb[0] = 0, za[1] = cz - 1, zb[1] = cz, nrun = 2;
    } else {
      za[0] = cz - 1, zb[0] = cz + 1, nrun = 1;
    }
  } else if (J.periodic[2]) {
    za[0] = 0, zb[0] = ncz - 1, nrun = 1;
  } else {
    za[0] = cz > 0 ? cz - 1 : 0;
    zb[0] = cz + 1 < ncz ? cz + 1 : ncz - 1;
    nrun = 1;
  }
  const bool anyper = J.periodic[0] | J.periodic[1] | J.periodic[2];
  const int64_t base = J.off;
  int cnt = 0;
  for (int a = 0; a < nx; ++a)
    for (int bb = 0; bb < ny; ++bb)
      for (int q = 0; q < nrun; ++q) {
        const uint32_t r0 = raster_of(J, sx[a], sy[bb], za[q]);
        const uint32_t r1 = raster_of(J, sx[a], sy[bb], zb[q]) + 1u;
        const int64_t beg = base + B.CSTART[base + cells_before(B, J, r0)];
        const int64_t end = base + B.CSTART[base + cells_before(B, J, r1)];
        for (int64_t j = beg; j < end; ++j) {
          if (j == i) continue;
          double dx = xi - X[j], dy = yi - X[C + j], dz = zi - X[2 * C + j];
          if (anyper) min_image(J, dx, dy, dz);
          if (dx * dx + dy * dy + dz * dz >= J.rlist2) continue;
          const uint32_t qid = ID[j];
          if (cnt < kmax) {
            int k = cnt;
            while (k > 0 && kid[(k - 1) * kNlistBlock + lane] > qid) {
              kid[k * kNlistBlock + lane] = kid[(k - 1) * kNlistBlock + lane];
              kslot[k * kNlistBlock + lane] = kslot[(k - 1) * kNlistBlock + lane];
              --k;
            }
            kid[k * kNlistBlock + lane] = qid;
            kslot[k * kNlistBlock + lane] = (uint32_t)j;
          }
          ++cnt;
        }
      }
  const int stored = cnt < kmax ? cnt : kmax;
  for (int k = 0; k < stored; ++k) B.NL[(int64_t)k * C + i] = kslot[k * kNlistBlock + lane];
  B.NCNT[i] = (uint32_t)stored;
  atomicMax(&B.book[job].nl_max, cnt);
  atomicAdd(&B.book[job].nl_sum, (unsigned long long)stored);
}

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
