// device.hpp -- per-particle device math for the RATTLE + Langevin step.
//
// Everything here is FP64 except the optional FP32 pair-force path.  The
// constants of the Philox4x32-10 generator are those published by Salmon et
// al. (SC'11).  The RATTLE position stage is the scalar form of the Newton
// iteration of Algorithm 1: because the first three rows of its Jacobian are
// -I, J^{-1} r reduces to one scalar update of lambda per iteration, which is
// the analytic solve the paper reports as fastest (SI Section S2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace mdk {

constexpr int kGroup = 64;          // slots per wavefront; per displacement accumulator and list statistic
constexpr int kTile = 256;          // particles per workgroup in per-particle kernels
constexpr int kNlistBlock = kTile;  // threads per workgroup in the list build
constexpr int kNlistPerTile = kTile / kNlistBlock;

enum : int { kSurfNone = 0, kSurfPlane = 1, kSurfSphere = 2, kSurfEllipsoid = 3, kSurfTorus = 4,
             kSurfCylinder = 5, kSurfHeight = 6, kSurfBridge = 7 };
enum : int { kPairNone = 0, kPairLJ = 1, kPairLJSmooth = 2 };
enum : int { kModeSteady = 0, kModeStart = 1, kModeStartGiven = 2 };
enum : int { kErrNewton = 1, kErrNaN = 2 };

// Per-job constants, written by the host before each launch set.
struct JobDev {
  double dt, half_dt, gamma, b;     // b = 1 / (1 + dt gamma / 2)        (Algorithm S1)
  double noise_k;                   // sqrt(2 kT gamma / dt); times sqrt(m) per particle
  double mass, inv_mass;            // used when uniform_mass
  double eps, sig2, rc2, rlist2;    // pair parameters; rlist = rc + skin
  double phic, dphic;               // phi(rc) and phi'(rc)              (Eq. S1)
  double half_skin;
  double newton_tol;
  double surf[8];
  double box_len[3], inv_box_len[3];
  double glo[3], inv_cs[3];
  int nc[3];
  int periodic[3];
  int surf_kind, pair_kind, force_fp64, uniform_mass;
  int newton_cap, mode, xcur, pcur;
  int scur, newton_frozen;
  int model, bpm;                   // bead model of the job (record in DevBufs::models); beads per molecule
  uint64_t seed;
  int64_t off, n, bm_off;
  int64_t step0, remaining;
};

// Per-job bookkeeping written by the device.  Touched by atomics only on
// rare events (a list going stale, an error, a new Newton maximum), so that
// workgroups never contend for these words in the common case.
constexpr long long kNever = 0x7FFFFFFFFFFFFFFFLL;
struct JobBook {
  long long stop_at;                // first step that must not run: stale list, list overflow or error (kNever if none)
  int err_code;
  int err_id;
  int newton_max;
  int nl_max;                       // largest neighbour count of the last list build (above kmax: overflow)
  double nl_sum;                    // sum of the stored neighbour counts of the last list build
  double a_now;                     // largest per-tile displacement bound since the last list build
};
__host__ __device__ constexpr JobBook fresh_book() { return JobBook{kNever, 0, 0, 0, 0, 0.0, 0.0}; }

// Bead model of one job (SI, Virus capsid self-assembly), tables by type pair
// a * kMaxTypes + b (symmetric).
constexpr int kMaxTypes = 4;
// Bead-model jobs carry the bead type in the top two bits of the candidate
// record's particle index (such jobs hold fewer than 2^30 particles).
constexpr int kTypeShift = 30;
constexpr uint32_t kIdMask = (1u << kTypeShift) - 1u;

struct ModelDev {
  double sig2[kMaxTypes * kMaxTypes];
  double eps4[kMaxTypes * kMaxTypes];
  double eps24[kMaxTypes * kMaxTypes];
  double rc2[kMaxTypes * kMaxTypes];
  double phic[kMaxTypes * kMaxTypes];   // phi(rc_ab), the energy shift
  double r0[kMaxTypes * kMaxTypes];
  double kb, ka, theta0;
  double wall_eps, wall_sig, wall_radius, wall_cut;  // wall_cut = 2^(1/6) wall_sig
  int ntypes, bpm;
};

// Device buffers, passed by value to every kernel.
struct DevBufs {
  double* X[2];        // positions, AoS [C][3]; parity flips every step
  double* P[2];        // momenta, AoS [C][3]; parity flips at rebuilds
  uint32_t* ID[2];     // particle index within its job; parity flips at rebuilds
  uint8_t* FLG[2];     // 1 = constrained
  double* MASS[2];     // per-particle mass (jobs with non-uniform mass)
  double* FC;          // combined force handed in by the caller, AoS [C][3], by job offset + id
  double* OX;          // outputs of the finish kernel (AoS [C][3]), by job offset + id
  double* OP;
  double* OF;
  double* OD;          // [4][C]: kinetic energy, potential energy share, |g|/|n|, |n.v|/|n|
  uint32_t* NL;        // neighbour slots: entry k of slot i at ((k/4) C + i) 4 + k%4, i.e. rows of uint4
                       // [kmax/4][C] (kmax is a multiple of 4), four entries per load
  uint32_t* NCNT;      // neighbour count per slot
  uint32_t* BM;        // occupied-cell bitmap words (per job segment)
  uint32_t* WOFF;      // exclusive popcount prefix per bitmap word (job-local)
  uint32_t* CCNT;      // particles per occupied cell, at job offset + compact cell
  uint32_t* CSTART;    // exclusive prefix of CCNT (job-local)
  uint32_t* RASTER;    // raster cell index per slot
  uint32_t* CID;       // compact cell index per slot
  uint32_t* RANK;      // rank within the cell per slot
  uint32_t* INV;       // slot of each particle index after the last sort, by job offset + index
  uint32_t* SRC;       // old slot (job-relative) of each new slot during a sort
  float4* PK;          // list-build candidates in the sorted order: FP32 position, particle index bits
  uint8_t* TYPE[2];    // bead type (jobs with a bead model); parity as ID
  const ModelDev* models;  // per job
  double* TACC;        // per group of 64 slots: accumulated max displacement since the last build
  uint32_t* NLSTAT;    // per group of 64 slots, from the last list build: (max count, sum of stored counts)
  JobDev* jobs;
  JobBook* book;
  int64_t C;           // slot capacity (SoA stride)
  int kmax;
  int pad2;
};

// ---------------------------------------------------------------------------
// Philox4x32-10 and Box-Muller normals.
// Counter (id, step lo, step hi, 0), key (seed lo, seed hi);
// u = (w + 1/2) 2^-32; z0, z1 from (w0, w1), z2 from (w2, w3).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32->64 multiply (v_mad_u64_u32) gives both halves
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ __forceinline__ void normals3(uint64_t seed, uint32_t id, long long step, double& z0, double& z1,
                                         double& z2) {
  uint32_t c0 = id, c1 = (uint32_t)(unsigned long long)step, c2 = (uint32_t)((unsigned long long)step >> 32),
           c3 = 0u;
  philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double inv32 = 2.3283064365386963e-10;  // 2^-32
  const double u0 = ((double)c0 + 0.5) * inv32;
  const double u1 = ((double)c1 + 0.5) * inv32;
  const double u2 = ((double)c2 + 0.5) * inv32;
  const double u3 = ((double)c3 + 0.5) * inv32;
  const double r0 = sqrt(-2.0 * log(u0));
  const double r1 = sqrt(-2.0 * log(u2));
  double s1, co1;
  sincospi(2.0 * u1, &s1, &co1);
  z0 = r0 * co1;
  z1 = r0 * s1;
  z2 = r1 * cospi(2.0 * u3);
}

// The same normals with the Box-Muller transform in FP32 on the hardware
// transcendental units (v_log_f32; v_sin_f32 / v_cos_f32 take their argument in
// revolutions, so sin(2 pi u) is one instruction).  Used with FP32 pair forces;
// the normals differ from the FP64 transform by ~1e-6 relative.
__device__ __forceinline__ void normals3_fast(uint64_t seed, uint32_t id, long long step, double& z0, double& z1,
                                              double& z2) {
  uint32_t c0 = id, c1 = (uint32_t)(unsigned long long)step, c2 = (uint32_t)((unsigned long long)step >> 32),
           c3 = 0u;
  philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double inv32 = 2.3283064365386963e-10;  // 2^-32
  const float u0 = (float)(((double)c0 + 0.5) * inv32);
  const float u1 = (float)(((double)c1 + 0.5) * inv32);
  const float u2 = (float)(((double)c2 + 0.5) * inv32);
  const float u3 = (float)(((double)c3 + 0.5) * inv32);
  const float r0 = sqrtf(-2.0f * __logf(u0));
  const float r1 = sqrtf(-2.0f * __logf(u2));
  z0 = (double)(r0 * __builtin_amdgcn_cosf(u1));
  z1 = (double)(r0 * __builtin_amdgcn_sinf(u1));
  z2 = (double)(r1 * __builtin_amdgcn_cosf(u3));
}

template <bool kF64>
__device__ __forceinline__ void langevin_normals(uint64_t seed, uint32_t id, long long step, double& z0, double& z1,
                                                 double& z2) {
  if (kF64)
    normals3(seed, id, step, z0, z1, z2);
  else
    normals3_fast(seed, id, step, z0, z1, z2);
}

// ---------------------------------------------------------------------------
// Surfaces: g(x) and n = dg/dx (un-normalised, Eq. 4).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double surf_eval(const JobDev& J, double x, double y, double z, double& nx, double& ny,
                                            double& nz) {
  const double* q = J.surf;
  switch (J.surf_kind) {
    case kSurfPlane:
      nx = q[3];
      ny = q[4];
      nz = q[5];
      return q[3] * (x - q[0]) + q[4] * (y - q[1]) + q[5] * (z - q[2]);
    case kSurfSphere: {
      const double d0 = x - q[0], d1 = y - q[1], d2 = z - q[2];
      nx = 2.0 * d0;
      ny = 2.0 * d1;
      nz = 2.0 * d2;
      return d0 * d0 + d1 * d1 + d2 * d2 - q[3] * q[3];
    }
    case kSurfEllipsoid: {
      // q[3..5] hold 1/a^2, 1/b^2, 1/c^2 on the device
      const double d0 = x - q[0], d1 = y - q[1], d2 = z - q[2];
      nx = 2.0 * d0 * q[3];
      ny = 2.0 * d1 * q[4];
      nz = 2.0 * d2 * q[5];
      return d0 * d0 * q[3] + d1 * d1 * q[4] + d2 * d2 * q[5] - 1.0;
    }
    case kSurfTorus: {
      const double d0 = x - q[0], d1 = y - q[1], d2 = z - q[2];
      const double rho = sqrt(d0 * d0 + d1 * d1);
      const double e = rho - q[3];
      const double s = 2.0 * (1.0 - q[3] / rho);
      nx = s * d0;
      ny = s * d1;
      nz = 2.0 * d2;
      return e * e + d2 * d2 - q[4] * q[4];
    }
    case kSurfCylinder: {
      const double d0 = x - q[0], d1 = y - q[1], d2 = z - q[2];
      nx = 2.0 * q[3] * d0;
      ny = 2.0 * q[4] * d1;
      nz = 2.0 * q[5] * d2;
      return q[3] * d0 * d0 + q[4] * d1 * d1 + q[5] * d2 * d2 - q[6] * q[6];
    }
    case kSurfHeight: {
      // q[2], q[3] hold 2/Lx, 2/Ly on the device (sinpi/cospi arguments)
      double sx, cx, sy, cy;
      sincospi(q[2] * x, &sx, &cx);
      sincospi(q[3] * y, &sy, &cy);
      const double kx = M_PI * q[2], ky = M_PI * q[3];
      nx = -q[1] * kx * cx * sy;
      ny = -q[1] * ky * sx * cy;
      nz = 1.0;
      return z - q[0] - q[1] * sx * sy;
    }
    case kSurfBridge: {
      // piecewise (SI S3.1): q[3..7] hold Lb/2, Rb, R, Rb + R, R/Rb on the device;
      // the piece is chosen by the evaluation point
      const double u = x - q[0], dy = y - q[1], dz = z - q[2];
      const double r2 = dy * dy + dz * dz;
      if (fabs(u) <= q[3]) {  // bridge cylinder, scaled by -R/Rb
        nx = 0.0;
        ny = -2.0 * q[7] * dy;
        nz = -2.0 * q[7] * dz;
        return q[7] * (q[4] * q[4] - r2);
      }
      const double r = sqrt(r2);
      const double ue = u > 0.0 ? u - q[3] : u + q[3];  // from the connector's end of the bridge
      if (r < q[6]) {  // connector: distance to the circle of radius R about r = Rb + R
        const double f = 2.0 * (1.0 - q[6] / r);
        nx = 2.0 * ue;
        ny = f * dy;
        nz = f * dz;
        const double e = r - q[6];
        return ue * ue + e * e - q[5] * q[5];
      }
      const double a = u > 0.0 ? 2.0 * q[5] : -2.0 * q[5];  // plane x = x0 +- (Lb/2 + R)
      nx = a;
      ny = nz = 0.0;
      return a * (ue - (u > 0.0 ? q[5] : -q[5]));
    }
    default:
      nx = ny = nz = 0.0;
      return 0.0;
  }
}

__device__ __forceinline__ double maxabs3(double a, double b, double c) {
  return fmax(fabs(a), fmax(fabs(b), fabs(c)));
}

// ---------------------------------------------------------------------------
// RATTLE position stage (Algorithm 1, first loop) for one particle.
// Input: x^m, the half-kicked momentum pt = p^m + dt/2 f^m, n^m = n(x^m) and
// g(x^m).  Output: x^{m+1} = x~ - c lambda n^m and p^{m+1/2} = pt - dt/2 lambda n^m
// with x~ = x^m + dt/m pt and c = dt^2/(2m).
// Newton iterates (identical to Algorithm 1's 4x4 iteration):
//   first:  lambda = [g(x^m) + n^m.(x~ - x^m)] / (c n^m.n^m)
//   then:   lambda += g(x') / (c n(x').n^m),  x' = x~ - c lambda n^m
// Stop: eta > 0: max(|g(x')|, |r_x|_inf) < eta (residual before the update);
//       eta = 0: position update within 16 ulp of max(1, |x'|_inf).
// Returns the iteration count, or -count when the cap was hit.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int rattle_position(const JobDev& J, double m, double x0, double y0, double z0,
                                               double g0, double nx, double ny, double nz, double& px,
                                               double& py, double& pz, double& x1, double& y1, double& z1) {
  const double dtm = J.dt / m;
  const double c = J.dt * dtm * 0.5;
  const double xt = x0 + dtm * px, yt = y0 + dtm * py, zt = z0 + dtm * pz;
  const double eps16 = 16.0 * 2.220446049250313e-16;
  // iteration 1: linearisation at x^m (the start x' = x^m, lambda = 0 of Algorithm 1)
  const double rx = xt - x0, ry = yt - y0, rz = zt - z0;
  const double nn = nx * nx + ny * ny + nz * nz;
  double lam = (g0 + nx * rx + ny * ry + nz * rz) / (c * nn);
  double xc = xt - c * lam * nx, yc = yt - c * lam * ny, zc = zt - c * lam * nz;
  bool done;
  if (J.newton_tol > 0.0) {
    done = fmax(fabs(g0), maxabs3(rx, ry, rz)) < J.newton_tol;
  } else {
    const double upd = maxabs3(xc - x0, yc - y0, zc - z0);
    done = upd <= eps16 * fmax(1.0, maxabs3(xc, yc, zc));
  }
  int it = 1;
  while (!done && it < J.newton_cap) {
    ++it;
    double mx, my, mz;
    const double g = surf_eval(J, xc, yc, zc, mx, my, mz);
    // full Newton: dg/dx at the iterate; frozen normal: at x^m (SI, Performance)
    const double dl = g / (c * (J.newton_frozen ? nn : mx * nx + my * ny + mz * nz));
    lam += dl;
    const double xn = xt - c * lam * nx, yn = yt - c * lam * ny, zn = zt - c * lam * nz;
    if (J.newton_tol > 0.0) {
      done = fabs(g) < J.newton_tol;
    } else {
      done = maxabs3(xn - xc, yn - yc, zn - zc) <= eps16 * fmax(1.0, maxabs3(xn, yn, zn));
    }
    xc = xn;
    yc = yn;
    zc = zn;
  }
  x1 = xc;
  y1 = yc;
  z1 = zc;
  const double hl = J.half_dt * lam;
  px -= hl * nx;
  py -= hl * ny;
  pz -= hl * nz;
  return done ? it : -it;
}

// Minimum image along periodic dimensions.
__device__ __forceinline__ void min_image(const JobDev& J, double& dx, double& dy, double& dz) {
  if (J.periodic[0]) dx -= J.box_len[0] * rint(dx * J.inv_box_len[0]);
  if (J.periodic[1]) dy -= J.box_len[1] * rint(dy * J.inv_box_len[1]);
  if (J.periodic[2]) dz -= J.box_len[2] * rint(dz * J.inv_box_len[2]);
}

// Force coefficient c of one pair, F_i += c (x_i - x_j), for r^2 < rc^2
// (Eq. S1: -dV/dr / r); zero beyond the cut-off.
template <typename real, bool kSmooth>
__device__ __forceinline__ real pair_coef(const JobDev& J, double r2, real eps24, real sig2, real dphic) {
  if (!(r2 < J.rc2)) return (real)0;
  const real r2r = (real)r2;
  // FP32: the hardware reciprocal (1 ulp); FP64: a correctly rounded division
  const real inv = sizeof(real) == 8 ? (real)(1.0 / (double)r2r) : (real)__builtin_amdgcn_rcpf((float)r2r);
  const real s2 = sig2 * inv;
  const real s6 = s2 * s2 * s2;
  real coef = eps24 * inv * s6 * ((real)2 * s6 - (real)1);
  if (kSmooth) {
    const real rinv = sizeof(real) == 8 ? (real)(1.0 / sqrt((double)r2r)) : (real)rsqrtf((float)r2r);
    coef += dphic * rinv;
  }
  return coef;
}

// Rounds t to a multiple of 2^-32 (for |t| < 2^19).  Sums of such values are
// exact in FP64 while their magnitude stays below 2^21, so they do not depend
// on the order of the terms.
__device__ __forceinline__ double on_grid(double t) {
  constexpr double kM = 0x1.8p20;  // 1.5 * 2^20: t + kM has an ulp of 2^-32
  return (t + kM) - kM;
}

// The product c x rounded onto the same grid with a single rounding: the fused
// multiply-add rounds c x + kM to a multiple of 2^-32, and removing kM is
// exact.  One instruction fewer per component than rounding the product first,
// and without its double rounding.
__device__ __forceinline__ double grid_product(double c, double x) {
  constexpr double kM = 0x1.8p20;
  return __builtin_fma(c, x, kM) - kM;
}

// Pair forces on slot i from its neighbour list.  FP64 class: FP64 terms
// summed in list order, the list being sorted by particle index.  FP32 class:
// separations and the cut-off test in FP64, the force coefficient in FP32, its
// product with the separation rounded onto the 2^-32 grid and summed in FP64,
// which makes the sum exact and independent of the list order (the lists of
// this class are in slot order).  The loop issues
// the gathers of kForceBatch neighbours before using them.  Specialised on the
// potential's form and on periodicity so the loop carries no dead work.
constexpr int kForceBatch = 4;  // neighbour gathers in flight per force-loop iteration: one uint4 list row

template <bool kF64, bool kSmooth, bool kPer>
__device__ __forceinline__ void pair_forces_impl(const JobDev& J, const DevBufs& B, const double* __restrict__ X,
                                                 int64_t i, double xi, double yi, double zi, double& Fx,
                                                 double& Fy, double& Fz) {
  using real = typename std::conditional<kF64, double, float>::type;
  const int64_t C = B.C;
  const int cnt = (int)B.NCNT[i];
  const uint4* __restrict__ nl = reinterpret_cast<const uint4*>(B.NL) + i;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  const real eps24 = (real)(24.0 * J.eps);
  const real sig2 = (real)J.sig2;
  const real dphic = (real)J.dphic;
  auto add = [&](double dx, double dy, double dz) {
    if (kPer) min_image(J, dx, dy, dz);
    const double r2 = dx * dx + dy * dy + dz * dz;
    const real c = pair_coef<real, kSmooth>(J, r2, eps24, sig2, dphic);
    if (kF64) {
      fx += c * dx;
      fy += c * dy;
      fz += c * dz;
    } else {
      const double c64 = (double)c;
      fx += grid_product(c64, dx);
      fy += grid_product(c64, dy);
      fz += grid_product(c64, dz);
    }
  };
  static_assert(kForceBatch == 4, "one uint4 row of the list per batch");
  int k = 0;
  for (; k + kForceBatch <= cnt; k += kForceBatch) {
    const uint4 q = nl[(int64_t)(k >> 2) * C];
    const int64_t j[kForceBatch] = {(int64_t)q.x, (int64_t)q.y, (int64_t)q.z, (int64_t)q.w};
    double ax[kForceBatch], ay[kForceBatch], az[kForceBatch];
#pragma unroll
    for (int u = 0; u < kForceBatch; ++u) {
      ax[u] = X[3 * j[u]];
      ay[u] = X[3 * j[u] + 1];
      az[u] = X[3 * j[u] + 2];
    }
#pragma unroll
    for (int u = 0; u < kForceBatch; ++u) add(xi - ax[u], yi - ay[u], zi - az[u]);
  }
  if (k < cnt) {
    const uint4 q = nl[(int64_t)(k >> 2) * C];
    const uint32_t jt[3] = {q.x, q.y, q.z};
#pragma unroll
    for (int u = 0; u < 3; ++u)
      if (k + u < cnt) {
        const int64_t j = jt[u];
        add(xi - X[3 * j], yi - X[3 * j + 1], zi - X[3 * j + 2]);
      }
  }
  Fx = fx;
  Fy = fy;
  Fz = fz;
}

template <bool kF64>
__device__ __forceinline__ void pair_forces(const JobDev& J, const DevBufs& B, const double* __restrict__ X,
                                            int64_t i, double xi, double yi, double zi, double& Fx, double& Fy,
                                            double& Fz) {
  const bool smooth = J.pair_kind == kPairLJSmooth;
  const bool per = J.periodic[0] | J.periodic[1] | J.periodic[2];
  if (smooth) {
    if (per)
      pair_forces_impl<kF64, true, true>(J, B, X, i, xi, yi, zi, Fx, Fy, Fz);
    else
      pair_forces_impl<kF64, true, false>(J, B, X, i, xi, yi, zi, Fx, Fy, Fz);
  } else {
    if (per)
      pair_forces_impl<kF64, false, true>(J, B, X, i, xi, yi, zi, Fx, Fy, Fz);
    else
      pair_forces_impl<kF64, false, false>(J, B, X, i, xi, yi, zi, Fx, Fy, Fz);
  }
}

// Energy share U_i = 1/2 sum_j V_ij (Eq. S1), FP64, for diagnostics; for the
// FP32 class the terms go on the exact-sum grid like the forces.
__device__ __forceinline__ double pair_energy(const JobDev& J, const DevBufs& B, const double* __restrict__ X,
                                              int64_t i, double xi, double yi, double zi) {
  const int64_t C = B.C;
  const int cnt = (int)B.NCNT[i];
  const bool smooth = J.pair_kind == kPairLJSmooth;
  const bool anyper = J.periodic[0] | J.periodic[1] | J.periodic[2];
  const double rc = sqrt(J.rc2);
  double u = 0.0;
  for (int k = 0; k < cnt; ++k) {
    const int64_t j = B.NL[(((int64_t)(k >> 2) * C + i) << 2) + (k & 3)];
    double dx = xi - X[3 * j], dy = yi - X[3 * j + 1], dz = zi - X[3 * j + 2];
    if (anyper) min_image(J, dx, dy, dz);
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (!(r2 < J.rc2)) continue;
    const double s2 = J.sig2 / r2;
    const double s6 = s2 * s2 * s2;
    double v = 4.0 * J.eps * s6 * (s6 - 1.0) - J.phic;
    if (smooth) v -= (sqrt(r2) - rc) * J.dphic;
    // FP32 class: lists in slot order, terms on the exact-sum grid
    u += J.force_fp64 ? 0.5 * v : on_grid(0.5 * v);
  }
  return u;
}

// ---------------------------------------------------------------------------
// Bead model (SI, Virus capsid self-assembly).  Pair terms in either force
// class (FP64: summed in particle-index order; FP32: FP32 coefficients times FP64
// separations on the exact-sum grid); bonded terms always FP64.
// ---------------------------------------------------------------------------

// Pair forces on slot i (type ti) from its list, typed truncated-shifted LJ;
// pairs inside a molecule are not in the list.  tab: the job's rc^2, sigma^2,
// 24 eps and bond rest-length tables staged in LDS by the caller (kModelTab
// doubles), or nullptr to read them from the model record.
constexpr int kModelTab = 4 * kMaxTypes * kMaxTypes;

template <bool kPer, bool kF64>
__device__ __forceinline__ void pair_forces_model(const JobDev& J, const ModelDev& M, const DevBufs& B,
                                                  const double* __restrict__ X, int64_t i, int ti, double xi,
                                                  double yi, double zi, double& Fx, double& Fy, double& Fz,
                                                  const double* tab) {
  const int64_t C = B.C;
  const int cnt = (int)B.NCNT[i];
  const uint4* __restrict__ nl = reinterpret_cast<const uint4*>(B.NL) + i;
  const double* row_rc2 = (tab ? tab : M.rc2) + ti * kMaxTypes;
  const double* row_sig2 = (tab ? tab + kMaxTypes * kMaxTypes : M.sig2) + ti * kMaxTypes;
  const double* row_eps24 = (tab ? tab + 2 * kMaxTypes * kMaxTypes : M.eps24) + ti * kMaxTypes;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  // entry: slot in the low bits, partner type in the top two; the partner's
  // position and the pair's table entries are loaded side by side
  auto add = [&](uint32_t e, double ax, double ay, double az) {
    const uint32_t tj = e >> kTypeShift;
    double dx = xi - ax, dy = yi - ay, dz = zi - az;
    if (kPer) min_image(J, dx, dy, dz);
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (!(r2 < row_rc2[tj])) return;
    if (kF64) {
      const double inv = 1.0 / r2;
      const double s2 = row_sig2[tj] * inv;
      const double s6 = s2 * s2 * s2;
      const double c = row_eps24[tj] * inv * s6 * (2.0 * s6 - 1.0);
      fx += c * dx;
      fy += c * dy;
      fz += c * dz;
    } else {
      const float inv = __builtin_amdgcn_rcpf((float)r2);
      const float s2 = (float)row_sig2[tj] * inv;
      const float s6 = s2 * s2 * s2;
      const float c = (float)row_eps24[tj] * inv * s6 * (2.0f * s6 - 1.0f);
      const double c64 = (double)c;
      fx += grid_product(c64, dx);
      fy += grid_product(c64, dy);
      fz += grid_product(c64, dz);
    }
  };
  int k = 0;
  for (; k + 4 <= cnt; k += 4) {
    const uint4 q = nl[(int64_t)(k >> 2) * C];
    const uint32_t e[4] = {q.x, q.y, q.z, q.w};
    double ax[4], ay[4], az[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t j = e[u] & kIdMask;
      ax[u] = X[3 * j];
      ay[u] = X[3 * j + 1];
      az[u] = X[3 * j + 2];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) add(e[u], ax[u], ay[u], az[u]);
  }
  if (k < cnt) {
    const uint4 q = nl[(int64_t)(k >> 2) * C];
    const uint32_t e[3] = {q.x, q.y, q.z};
#pragma unroll
    for (int u = 0; u < 3; ++u)
      if (k + u < cnt) {
        const int64_t j = e[u] & kIdMask;
        add(e[u], X[3 * j], X[3 * j + 1], X[3 * j + 2]);
      }
  }
  Fx = fx;
  Fy = fy;
  Fz = fz;
}

// Energy share of slot i from the typed pairs (half of each pair).
__device__ __forceinline__ double pair_energy_model(const JobDev& J, const ModelDev& M, const DevBufs& B,
                                                    const double* __restrict__ X, int64_t i, int ti, double xi,
                                                    double yi, double zi) {
  const int64_t C = B.C;
  const int cnt = (int)B.NCNT[i];
  const bool anyper = J.periodic[0] | J.periodic[1] | J.periodic[2];
  double u = 0.0;
  for (int k = 0; k < cnt; ++k) {
    const uint32_t e = B.NL[(((int64_t)(k >> 2) * C + i) << 2) + (k & 3)];
    const int64_t j = e & kIdMask;
    const int p = ti * kMaxTypes + (int)(e >> kTypeShift);
    double dx = xi - X[3 * j], dy = yi - X[3 * j + 1], dz = zi - X[3 * j + 2];
    if (anyper) min_image(J, dx, dy, dz);
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (!(r2 < M.rc2[p])) continue;
    const double s2 = M.sig2[p] / r2;
    const double s6 = s2 * s2 * s2;
    const double v = 0.5 * (M.eps4[p] * s6 * (s6 - 1.0) - M.phic[p]);
    u += J.force_fp64 ? v : on_grid(v);  // FP32 class: slot-ordered lists, exact-sum grid
  }
  return u;
}

// Position of the particle with job-local index id (through the inverse
// permutation of the last sort).
__device__ __forceinline__ void pos_of(const JobDev& J, const DevBufs& B, const double* __restrict__ X,
                                       int64_t id, double* out) {
  const int64_t s = J.off + B.INV[J.off + id];
  out[0] = X[3 * s];
  out[1] = X[3 * s + 1];
  out[2] = X[3 * s + 2];
}

// Bonds to the previous and next bead, bends centred at the previous, this and
// the next bead, and the wall, added to F in that order; returns the energy
// share of this bead (half of each bond, a third of each bend, its wall term).
// The bend force is 2 ka (theta - theta0)/sin(theta) times the gradient of
// cos(theta); where sin(theta) vanishes that ratio takes its limit (-1 at
// theta = theta0 = pi).
__device__ __forceinline__ double bonded_forces(const JobDev& J, const ModelDev& M, const DevBufs& B,
                                                const double* __restrict__ X, int64_t id, const int* tid,
                                                const double* xs, double& Fx, double& Fy, double& Fz,
                                                const double* tab) {
  const double* r0_tab = tab ? tab + 3 * kMaxTypes * kMaxTypes : M.r0;
  // xs: positions of beads id-2 .. id+2 (3 doubles each; those outside the
  // molecule unused); tid: their types
  double u = 0.0;
  const int64_t bpm = M.bpm;
  const int64_t m0 = bpm > 0 ? (id / bpm) * bpm : id, m1 = bpm > 0 ? min(m0 + bpm, (int64_t)J.n) : id + 1;
  const double* xi = xs + 6;
  auto bond = [&](int q) {  // partner slot q in xs (1 or 3)
    double d[3] = {xi[0] - xs[3 * q], xi[1] - xs[3 * q + 1], xi[2] - xs[3 * q + 2]};
    if (J.periodic[0] | J.periodic[1] | J.periodic[2]) min_image(J, d[0], d[1], d[2]);
    const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double r0 = r0_tab[tid[2] * kMaxTypes + tid[q]];
    const double c = -2.0 * M.kb * (r - r0) / r;
    Fx += c * d[0];
    Fy += c * d[1];
    Fz += c * d[2];
    u += 0.5 * (M.kb * (r - r0) * (r - r0));
  };
  if (bpm > 1) {
    if (id - 1 >= m0) bond(1);
    if (id + 1 < m1) bond(3);
    for (int cb = 1; cb <= 3; ++cb) {  // bend centred at bead id - 2 + cb
      const int64_t b = id - 2 + cb;
      if (b - 1 < m0 || b + 1 >= m1) continue;
      const double* xa = xs + 3 * (cb - 1);
      const double* xb = xs + 3 * cb;
      const double* xc = xs + 3 * (cb + 1);
      double uu_[3] = {xa[0] - xb[0], xa[1] - xb[1], xa[2] - xb[2]};
      double vv_[3] = {xc[0] - xb[0], xc[1] - xb[1], xc[2] - xb[2]};
      if (J.periodic[0] | J.periodic[1] | J.periodic[2]) {
        min_image(J, uu_[0], uu_[1], uu_[2]);
        min_image(J, vv_[0], vv_[1], vv_[2]);
      }
      const double uu = uu_[0] * uu_[0] + uu_[1] * uu_[1] + uu_[2] * uu_[2];
      const double vv = vv_[0] * vv_[0] + vv_[1] * vv_[1] + vv_[2] * vv_[2];
      const double nu = sqrt(uu), nv = sqrt(vv);
      const double inn = 1.0 / (nu * nv);
      double cs = (uu_[0] * vv_[0] + uu_[1] * vv_[1] + uu_[2] * vv_[2]) * inn;
      cs = fmin(1.0, fmax(-1.0, cs));
      const double th = acos(cs), sn = sqrt(1.0 - cs * cs);
      const double dth = th - M.theta0;
      double ratio;
      if (sn > 1e-12)
        ratio = dth / sn;
      else
        ratio = fabs(dth) < 1e-6 ? (th > 1.5 ? -1.0 : 1.0) : dth / 1e-12;
      const double k2 = 2.0 * M.ka * ratio;
      const double cu = cs / uu, cv = cs / vv;
      // this bead is the first end (cb = 3), the middle (cb = 2) or the second end (cb = 1)
      double g[3];
      for (int k = 0; k < 3; ++k) {
        const double ga = vv_[k] * inn - cu * uu_[k];
        const double gc = uu_[k] * inn - cv * vv_[k];
        g[k] = cb == 3 ? ga : (cb == 1 ? gc : -(ga + gc));
      }
      Fx += k2 * g[0];
      Fy += k2 * g[1];
      Fz += k2 * g[2];
      u += (M.ka * dth * dth) / 3.0;
    }
  }
  if (M.wall_eps > 0.0) {
    double d[3] = {xi[0] - J.surf[0], xi[1] - J.surf[1], xi[2] - J.surf[2]};
    const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double s = r - M.wall_radius;
    double f[3] = {0.0, 0.0, 0.0};
    if (s < M.wall_cut && r > 0.0) {
      const double sr = M.wall_sig / s;
      const double s6 = sr * sr * sr * sr * sr * sr, s12 = s6 * s6;
      const double dphi = -24.0 * M.wall_eps * (2.0 * s12 - s6) / s;
      for (int k = 0; k < 3; ++k) f[k] = -dphi * d[k] / r;
      u += 4.0 * M.wall_eps * (s12 - s6) + M.wall_eps;
    }
    Fx += f[0];
    Fy += f[1];
    Fz += f[2];
  }
  return u;
}

// Gather the positions and types of beads id-2 .. id+2 of id's molecule.
__device__ __forceinline__ void molecule_window(const JobDev& J, const ModelDev& M, const DevBufs& B,
                                                const double* __restrict__ X, int64_t id, double xi, double yi,
                                                double zi, int ti, double* xs, int* tid) {
  const int64_t bpm = M.bpm;
  const int64_t m0 = bpm > 0 ? (id / bpm) * bpm : id, m1 = bpm > 0 ? min(m0 + bpm, (int64_t)J.n) : id + 1;
  const uint8_t* __restrict__ T = B.TYPE[J.scur];
  for (int q = 0; q < 5; ++q) {
    const int64_t g = id - 2 + q;
    tid[q] = 0;
    xs[3 * q] = xs[3 * q + 1] = xs[3 * q + 2] = 0.0;
    if (q == 2) {
      xs[6] = xi, xs[7] = yi, xs[8] = zi;
      tid[2] = ti;
    } else if (g >= m0 && g < m1) {
      pos_of(J, B, X, g, xs + 3 * q);
      tid[q] = T[J.off + B.INV[J.off + g]];
    }
  }
}

// Workgroup-uniform values read from memory are moved to scalar registers, so
// that everything addressed through them (the job record in particular) is
// loaded with scalar loads instead of occupying vector registers.
__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// XCD-aware workgroup order: the dispatcher deals workgroups round-robin over
// the 8 XCDs; remap so that each XCD walks one contiguous range of tiles
// (neighbouring tiles share neighbour data in that XCD's L2).
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int xcd = b & 7;
  const int local = b >> 3;
  const int per = G >> 3;
  const int rem = G & 7;
  return xcd * per + (xcd < rem ? xcd : rem) + local;
}

}  // namespace mdk
