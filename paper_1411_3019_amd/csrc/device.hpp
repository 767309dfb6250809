// device.hpp -- per-particle device math for the RATTLE + Langevin step.
//
// Positions, momenta, the RATTLE solves and the tangent projection are FP64;
// pair forces are FP64 or FP32 (force class).  The constants of the
// Philox4x32-10 generator are those published by Salmon et al. (SC'11).  The
// RATTLE position stage is the scalar form of the Newton iteration of
// Algorithm 1: because the first three rows of its Jacobian are -I, J^{-1} r
// reduces to one scalar update of lambda per iteration, which is the analytic
// solve the paper reports as fastest (SI Section S2).
//
// Neighbour lists index a per-tile "window": the tile's own 256 slots
// (entries 0..255, slot = tile start + entry) followed by the tile's halo, the
// sorted list of other slots any of its particles has as a neighbour (entry
// 256 + h is halo[h]).  The step kernel stages the window's positions in LDS
// once per step, so the force loop reads neighbours from LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace mdk {

constexpr int kGroup = 64;          // slots per wavefront; per displacement accumulator and list statistic
constexpr int kTile = 256;          // particles per workgroup in per-particle kernels; one list window
constexpr int kNlistBlock = kTile;  // threads per workgroup in the list build
constexpr int kRow = 8;             // list entries per 16-byte row (16-bit entries)

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
  double noise_km;                  // noise_k sqrt(mass) (uniform mass)
  double dtm, cpos, inv_cpos;       // dt/m, c = dt^2/(2m), 1/c (uniform mass)
  double eps, sig2, rc2, rlist2;    // pair parameters; rlist = rc + skin
  double phic, dphic;               // phi(rc) and phi'(rc)              (Eq. S1)
  double half_skin;
  double newton_tol;
  double grid_bias;                 // 1.5 2^20: FP32-class terms are rounded onto the 2^-32 grid of [2^20, 2^21)
  float grid_cmax;                  // FP32-class sums are exact while every pair coefficient is below this
  int pad0;
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
  long long err_step;               // step whose launch found the error (-1 if none)
  unsigned long long err_key;       // smallest (particle index << 2 | error code) among the particles that
                                    // failed at err_step (kNoError if none): the same report in any schedule
  int newton_max;
  int nl_max;                       // largest neighbour count of the last list build (above kmax: overflow)
  double nl_sum;                    // sum of the stored neighbour counts of the last list build
  double a_now;                     // largest per-tile displacement bound since the last list build
  int halo_max;                     // largest tile halo of the last build (above the capacity: overflow)
  int build_fail;                   // the last build could not stage a tile's candidates (see k_nlist)
  int sum_breaches;                 // particles whose FP32-class force terms left the exact-sum range
};
constexpr unsigned long long kNoError = ~0ull;
__host__ __device__ constexpr JobBook fresh_book() {
  return JobBook{kNever, -1, kNoError, 0, 0, 0.0, 0.0, 0, 0, 0};
}

// Bead model of one job (SI, Virus capsid self-assembly), tables by type pair
// a * kMaxTypes + b (symmetric).
constexpr int kMaxTypes = 4;
// Bead-model list entries carry the partner's type in their top two bits.
constexpr int kEntryTypeShift = 14;
constexpr uint32_t kEntryMask = (1u << kEntryTypeShift) - 1u;
constexpr int kTypeShift = 30;      // type bits of a 32-bit index (candidate records of the list build)
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
  double* NZD[2];      // normals of the last step's Langevin draw, FP64 class, AoS [C][3]; parity as P
  float* NZF[2];       // the same for the FP32 class (FP32 normals), AoS [C][3]
  double* FC;          // combined force handed in by the caller, AoS [C][3], by job offset + id
  double* OX;          // outputs of the finish kernel (AoS [C][3]), by job offset + id
  double* OP;
  double* OF;
  double* OD;          // [4][C]: kinetic energy, potential energy share, |g|/|n|, |n.v|/|n|
  uint16_t* NL;        // window entries: entry k of slot i at ((k/8) C + i) 8 + k%8, i.e. rows of
                       // 8 entries [kmax/8][C] (kmax a multiple of 8), one 16-byte load per row
  uint32_t* NCNT;      // neighbour count per slot
  uint32_t* HALO;      // per tile (slot / 256): hcap slots (absolute), sorted; the window's entries 256..
  uint32_t* HCNT;      // per tile: halo length
  uint32_t* BM;        // occupied-cell bitmap words (per job segment)
  uint32_t* WOFF;      // exclusive popcount prefix per bitmap word (job-local)
  uint32_t* CCNT;      // particles per occupied cell, at job offset + compact cell
  uint32_t* CSTART;    // exclusive prefix of CCNT (job-local)
  uint32_t* RASTER;    // raster cell index per slot
  uint32_t* CID;       // compact cell index per slot
  uint32_t* RANK;      // rank within the cell per slot
  uint32_t* INV;       // slot of each particle index after the last sort, by job offset + index (bead-model jobs only)
  uint2* BW;           // bead-model jobs: window entries of beads id-2, id-1 (x) and id+1, id+2 (y) of slot i's
                       // molecule, 16 bits each with the type in the top two; 0xFFFF: outside the window or molecule
  uint32_t* KKEY;      // list build, wide instance, when the window records do not fit LDS: [tile][256 + hcap], else null
  float4* PK;          // list-build candidates in the sorted order: FP32 position, particle index
                       // (bead model: type in the top two bits)
  uint8_t* TYPE[2];    // bead type (jobs with a bead model); parity as ID
  const ModelDev* models;  // per job
  double* TACC;        // per group of 64 slots: accumulated max displacement since the last build
  uint32_t* NLSTAT;    // per group of 64 slots, from the last list build: (max count, sum of stored counts)
  JobDev* jobs;
  JobBook* book;
  int64_t C;           // slot capacity (SoA stride)
  int kmax;
  int hcap;            // halo capacity per tile
  int no_bw;           // 1: the list build leaves BW empty (bonded partners through the inverse permutation)
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
__device__ __forceinline__ void normals3_f32(uint64_t seed, uint32_t id, long long step, float& z0, float& z1,
                                             float& z2) {
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
  z0 = r0 * __builtin_amdgcn_cosf(u1);
  z1 = r0 * __builtin_amdgcn_sinf(u1);
  z2 = r1 * __builtin_amdgcn_cosf(u3);
}

__device__ __forceinline__ void normals3_fast(uint64_t seed, uint32_t id, long long step, double& z0, double& z1,
                                              double& z2) {
  float a, b, c;
  normals3_f32(seed, id, step, a, b, c);
  z0 = (double)a;
  z1 = (double)b;
  z2 = (double)c;
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
// FP64 reciprocal and reciprocal square root: the hardware estimates refined
// by two Newton steps each (about one ulp; the step kernel and the finish
// kernel use the same routines, so they agree bit for bit).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rcp64(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = __builtin_fma(-d, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-d, r, 1.0);
  return __builtin_fma(r, e, r);
}

__device__ __forceinline__ double rsqrt64(double a) {
  double y = __builtin_amdgcn_rsq(a);
  double h = a * y;
  double r = __builtin_fma(-h, y, 1.0);
  y = __builtin_fma(0.5 * y, r, y);
  h = a * y;
  r = __builtin_fma(-h, y, 1.0);
  return __builtin_fma(0.5 * y, r, y);
}

// ---------------------------------------------------------------------------
// Surfaces: g(x) and n = dg/dx (un-normalised, Eq. 4).  kAll: every kind; the
// step kernels of jobs on the quadric surfaces (and the plane) are built
// without the height field and the bridge, whose transcendentals and pieces
// would otherwise set their register budget.
// ---------------------------------------------------------------------------
constexpr bool heavy_surface(int kind) { return kind == kSurfHeight || kind == kSurfBridge; }

template <bool kAll = true>
__device__ __forceinline__ double surf_eval(const JobDev& J, double x, double y, double z, double& nx, double& ny,
                                            double& nz) {
  const double* q = J.surf;
  if (!kAll && heavy_surface(J.surf_kind)) {
    nx = ny = nz = 0.0;
    return 0.0;
  }
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
      // rho and 1/rho from one reciprocal square root
      const double d0 = x - q[0], d1 = y - q[1], d2 = z - q[2];
      const double rho2 = d0 * d0 + d1 * d1;
      const double ir = rsqrt64(rho2);
      const double e = rho2 * ir - q[3];
      const double s = 2.0 - 2.0 * q[3] * ir;
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
      const double ir = rsqrt64(r2);
      const double r = r2 > 0.0 ? r2 * ir : 0.0;
      const double ue = u > 0.0 ? u - q[3] : u + q[3];  // from the connector's end of the bridge
      if (r < q[6]) {  // connector: distance to the circle of radius R about r = Rb + R
        const double f = 2.0 - 2.0 * q[6] * ir;
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

// Mass-dependent constants of one particle: dt/m, c = dt^2/(2m) and 1/c.
struct MassTerms {
  double dtm, c, ic;
};
__device__ __forceinline__ MassTerms mass_terms(const JobDev& J, double m) {
  if (J.uniform_mass) return MassTerms{J.dtm, J.cpos, J.inv_cpos};
  const double im = rcp64(m);
  const double dtm = J.dt * im;
  return MassTerms{dtm, 0.5 * J.dt * dtm, 2.0 * m / (J.dt * J.dt)};
}

// ---------------------------------------------------------------------------
// RATTLE position stage (Algorithm 1, first loop) for one particle.
// Input: x^m, the half-kicked momentum pt = p^m + dt/2 f^m, n^m = n(x^m),
// g(x^m) and 1/(n^m.n^m).  Output: x^{m+1} = x~ - c lambda n^m and
// p^{m+1/2} = pt - dt/2 lambda n^m with x~ = x^m + dt/m pt and c = dt^2/(2m).
// Newton iterates (identical to Algorithm 1's 4x4 iteration):
//   first:  lambda = [g(x^m) + n^m.(x~ - x^m)] / (c n^m.n^m)
//   then:   lambda += g(x') / (c n(x').n^m),  x' = x~ - c lambda n^m
// Stop: eta > 0: max(|g(x')|, |r_x|_inf) < eta (residual before the update);
//       eta = 0: position update within 16 ulp of max(1, |x'|_inf).
// Returns the iteration count, or -count when the cap was hit.
// ---------------------------------------------------------------------------
template <bool kAll = true>
__device__ __forceinline__ int rattle_position(const JobDev& J, const MassTerms& mt, double x0, double y0, double z0,
                                               double g0, double nx, double ny, double nz, double inv_nn,
                                               double& px, double& py, double& pz, double& x1, double& y1,
                                               double& z1) {
  const double dtm = mt.dtm, c = mt.c;
  const double xt = x0 + dtm * px, yt = y0 + dtm * py, zt = z0 + dtm * pz;
  const double eps16 = 16.0 * 2.220446049250313e-16;
  // iteration 1: linearisation at x^m (the start x' = x^m, lambda = 0 of Algorithm 1)
  const double rx = xt - x0, ry = yt - y0, rz = zt - z0;
  double lam = (g0 + nx * rx + ny * ry + nz * rz) * (mt.ic * inv_nn);
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
    const double g = surf_eval<kAll>(J, xc, yc, zc, mx, my, mz);
    // full Newton: dg/dx at the iterate; frozen normal: at x^m (SI, Performance)
    const double dl = g * mt.ic * (J.newton_frozen ? inv_nn : rcp64(mx * nx + my * ny + mz * nz));
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

// ---------------------------------------------------------------------------
// Pair terms (Eq. S1).  The force on i from j is c (x_i - x_j) with
// c = -V'(r)/r for r < rc, 0 beyond.
//
// FP64 class: c in FP64, the terms summed in list order (lists of this class
// are sorted by particle index).
// FP32 class: c in FP32 from the FP64 r^2; each term c dx rounded once onto
// the grid of multiples of 2^-32 (a fused multiply-add with 1.5 2^20, whose
// result then lies in [2^20, 2^21) with an ulp of 2^-32 while |c dx| < 2^19).
// The bit pattern of such a double is an affine function of its value, so the
// terms are summed exactly as 64-bit integers of their bit patterns: the sum
// does not depend on the order of the terms, which lets these lists stay in
// any order.  Each particle checks that its largest coefficient kept every term
// inside that range; a particle that fails (a pair closer than about half a
// sigma) is summed again in FP64 and reported (JobBook::sum_breaches).
// ---------------------------------------------------------------------------
// Exact sum of FP32-class terms (see above).
struct GridSum {
  uint64_t x, y, z;
  int cmax;  // largest coefficient as integer bits (positive floats order as integers)
  __device__ __forceinline__ void clear() {
    x = y = z = 0;
    cmax = 0;
  }
  __device__ __forceinline__ void add(float c, double dx, double dy, double dz, double bias) {
    const double c64 = (double)c;
    x += (uint64_t)__double_as_longlong(__builtin_fma(c64, dx, bias));
    y += (uint64_t)__double_as_longlong(__builtin_fma(c64, dy, bias));
    z += (uint64_t)__double_as_longlong(__builtin_fma(c64, dz, bias));
    cmax = max(cmax, __float_as_int(c));
  }
  // F from n terms; false when a term may have left [2^20, 2^21)
  __device__ __forceinline__ bool get(int n, float guard, double& Fx, double& Fy, double& Fz) const {
    const uint64_t base = (uint64_t)n * (uint64_t)__double_as_longlong(0x1.8p20);
    Fx = (double)(int64_t)(x - base) * 0x1p-32;
    Fy = (double)(int64_t)(y - base) * 0x1p-32;
    Fz = (double)(int64_t)(z - base) * 0x1p-32;
    return cmax < __float_as_int(guard);
  }
};

// Slot (absolute) of window entry e of the tile starting at slot first.
__device__ __forceinline__ int64_t window_slot(const DevBufs& B, int64_t first, uint32_t e) {
  if (e < (uint32_t)kTile) return first + e;
  const int64_t h = min((int64_t)(e - kTile), (int64_t)B.hcap - 1);
  return (int64_t)B.HALO[(first / kTile) * (int64_t)B.hcap + h];
}

// One 16-byte row (8 entries) of slot i's list.
__device__ __forceinline__ uint4 list_row(const DevBufs& B, int64_t i, int r) {
  return reinterpret_cast<const uint4*>(B.NL)[(int64_t)r * B.C + i];
}

__device__ __forceinline__ uint32_t row_entry(const uint4& q, int u) {
  const uint32_t w = u < 2 ? q.x : (u < 4 ? q.y : (u < 6 ? q.z : q.w));
  return (w >> ((u & 1) * 16)) & 0xFFFFu;
}

// The same for an index u known only at run time.
__device__ __forceinline__ uint32_t row_entry_dyn(uint4 q, int u) { return row_entry(q, u); }

// The first two rows of a list (16 entries), loaded ahead of the force loop.
struct Rows3 {
  uint4 r0, r1;
};
__device__ __forceinline__ Rows3 load_rows3(const DevBufs& B, int64_t i, int cnt) {
  Rows3 q;
  q.r0 = q.r1 = make_uint4(0u, 0u, 0u, 0u);
  if (cnt > 0) q.r0 = list_row(B, i, 0);
  if (cnt > kRow) q.r1 = list_row(B, i, 1);
  return q;
}

// Calls f(entry) for the cnt entries of slot i's list, in list order: one
// row of eight entries at a time, the next row loading while one is processed
// (the first two come in q).
template <class F>
__device__ __forceinline__ void for_entries(const DevBufs& B, int64_t i, int cnt, const Rows3& q, F f) {
  uint4 cur = q.r0, nxt = q.r1;
  for (int k0 = 0; k0 < cnt; k0 += kRow) {
    const uint4 r = cur;
    cur = nxt;
    if (k0 + 2 * kRow < cnt) nxt = list_row(B, i, k0 / kRow + 2);
#pragma unroll
    for (int u = 0; u < kRow; ++u)
      if (k0 + u < cnt) f(row_entry(r, u));
  }
}

// Pair forces of slot i (list of cnt window entries, first rows q) from
// positions fetched by pos(e, ax, ay, az).  Plain or smoothed LJ, minimum
// image where periodic (uniform flags: one copy of the loop).  exact: false
// when an FP32-class term left the exact range (the forces are then the FP64
// sum of the same terms in list order).
template <bool kF64, class Pos>
__device__ __forceinline__ void pair_forces(const JobDev& J, const DevBufs& B, int64_t i, int cnt, const Rows3& q,
                                            double xi, double yi, double zi, Pos pos, double& Fx, double& Fy,
                                            double& Fz, bool& exact) {
  const double rc2 = J.rc2;
  const bool smooth = J.pair_kind == kPairLJSmooth;
  const bool per = J.periodic[0] | J.periodic[1] | J.periodic[2];
  exact = true;
  auto sep = [&](uint32_t e, double& dx, double& dy, double& dz) {
    double ax, ay, az;
    pos(e, ax, ay, az);
    dx = xi - ax;
    dy = yi - ay;
    dz = zi - az;
    if (per) min_image(J, dx, dy, dz);
    return dx * dx + dy * dy + dz * dz;
  };
  if (kF64) {
    const double eps24 = 24.0 * J.eps, sig2 = J.sig2, dphic = J.dphic;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for_entries(B, i, cnt, q, [&](uint32_t e) {
      double dx, dy, dz;
      const double r2 = sep(e, dx, dy, dz);
      if (r2 < rc2) {
        const double inv = 1.0 / r2;
        const double s2 = sig2 * inv;
        const double s6 = s2 * s2 * s2;
        double c = eps24 * inv * s6 * (2.0 * s6 - 1.0);
        if (smooth) c += dphic / sqrt(r2);
        fx += c * dx;
        fy += c * dy;
        fz += c * dz;
      }
    });
    Fx = fx;
    Fy = fy;
    Fz = fz;
  } else {
    const float eps24 = (float)(24.0 * J.eps), sig2 = (float)J.sig2, dphic = (float)J.dphic;
    const double bias = J.grid_bias;
    auto coef_t = [&](double r2, auto smooth_tag) {
      const float r2f = (float)r2;
      const float inv = __builtin_amdgcn_rcpf(r2f);
      const float s2 = sig2 * inv;
      const float s6 = s2 * s2 * s2;
      float c = eps24 * inv * s6 * (2.0f * s6 - 1.0f);
      if constexpr (decltype(smooth_tag)::value) c += dphic * __builtin_amdgcn_rsqf(r2f);
      return c;
    };
    auto coef = [&](double r2) { return smooth ? coef_t(r2, std::true_type{}) : coef_t(r2, std::false_type{}); };
    GridSum s;
    s.clear();
    int nadd = 0;  // terms added
    // the smoothed potential's extra term only where it is used (one copy of
    // the loop per form)
    auto run = [&](auto smooth_tag) {
      for_entries(B, i, cnt, q, [&](uint32_t e) {
        double dx, dy, dz;
        const double r2 = sep(e, dx, dy, dz);
        float c = coef_t(r2, smooth_tag);
        c = r2 < rc2 ? c : 0.0f;
        s.add(c, dx, dy, dz, bias);
      });
    };
    if (smooth)
      run(std::true_type{});
    else
      run(std::false_type{});
    nadd = cnt;
    exact = s.get(nadd, J.grid_cmax, Fx, Fy, Fz);
    if (!exact) {
      // (rare: a plain loop, kept out of the unrolled code)
      double fx = 0.0, fy = 0.0, fz = 0.0;
#pragma nounroll
      for (int k = 0; k < cnt; ++k) {
        double dx, dy, dz;
        const double r2 = sep(row_entry_dyn(list_row(B, i, k / kRow), k % kRow), dx, dy, dz);
        if (r2 < rc2) {
          const double c = (double)coef(r2);
          fx += c * dx;
          fy += c * dy;
          fz += c * dz;
        }
      }
      Fx = fx;
      Fy = fy;
      Fz = fz;
    }
  }
}

// Energy share U_i = 1/2 sum_j V_ij (Eq. S1), FP64, for diagnostics; for the
// FP32 class the terms go on the 2^-32 grid (summed in FP64: exact while the
// partial sums stay below 2^21).
__device__ __forceinline__ double pair_energy(const JobDev& J, const DevBufs& B, const double* __restrict__ X,
                                              int64_t first, int64_t i, double xi, double yi, double zi) {
  const int cnt = (int)B.NCNT[i];
  const bool smooth = J.pair_kind == kPairLJSmooth;
  const bool anyper = J.periodic[0] | J.periodic[1] | J.periodic[2];
  const double rc = sqrt(J.rc2);
  double u = 0.0;
  for (int k = 0; k < cnt; ++k) {
    const int64_t j = window_slot(B, first, row_entry(list_row(B, i, k / kRow), k % kRow));
    double dx = xi - X[3 * j], dy = yi - X[3 * j + 1], dz = zi - X[3 * j + 2];
    if (anyper) min_image(J, dx, dy, dz);
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (!(r2 < J.rc2)) continue;
    const double s2 = J.sig2 / r2;
    const double s6 = s2 * s2 * s2;
    double v = 4.0 * J.eps * s6 * (s6 - 1.0) - J.phic;
    if (smooth) v -= (sqrt(r2) - rc) * J.dphic;
    u += J.force_fp64 ? 0.5 * v : (__builtin_fma(0.5, v, 0x1.8p20) - 0x1.8p20);
  }
  return u;
}

// ---------------------------------------------------------------------------
// Bead model (SI, Virus capsid self-assembly).  Pair terms in either force
// class; bonded terms always FP64.  List entries carry the partner's type in
// their top two bits; pairs inside a molecule are not in the list.  tab: the
// job's rc^2, sigma^2, 24 eps and bond rest-length tables (kModelTab doubles,
// staged in LDS by the step kernel), or nullptr to read the model record.
// ---------------------------------------------------------------------------
constexpr int kModelTab = 4 * kMaxTypes * kMaxTypes;

template <bool kPer, bool kF64, class Pos>
__device__ __forceinline__ void pair_forces_model(const JobDev& J, const ModelDev& M, const DevBufs& B, int64_t i,
                                                  int cnt, const Rows3& q, int ti, double xi, double yi, double zi,
                                                  Pos pos, double& Fx, double& Fy, double& Fz, bool& exact,
                                                  const double* tab) {
  const double* row_rc2 = (tab ? tab : M.rc2) + ti * kMaxTypes;
  const double* row_sig2 = (tab ? tab + kMaxTypes * kMaxTypes : M.sig2) + ti * kMaxTypes;
  const double* row_eps24 = (tab ? tab + 2 * kMaxTypes * kMaxTypes : M.eps24) + ti * kMaxTypes;
  exact = true;
  auto sep = [&](uint32_t e, double& dx, double& dy, double& dz) {
    double ax, ay, az;
    pos(e & kEntryMask, ax, ay, az);
    dx = xi - ax;
    dy = yi - ay;
    dz = zi - az;
    if (kPer) min_image(J, dx, dy, dz);
    return dx * dx + dy * dy + dz * dz;
  };
  auto coef_f = [&](uint32_t tj, double r2) -> float {
    const float inv = __builtin_amdgcn_rcpf((float)r2);
    const float s2 = (float)row_sig2[tj] * inv;
    const float s6 = s2 * s2 * s2;
    return (float)row_eps24[tj] * inv * s6 * (2.0f * s6 - 1.0f);
  };
  if (kF64) {
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for_entries(B, i, cnt, q, [&](uint32_t e) {
      const uint32_t tj = e >> kEntryTypeShift;
      double dx, dy, dz;
      const double r2 = sep(e, dx, dy, dz);
      if (r2 < row_rc2[tj]) {
        const double inv = 1.0 / r2;
        const double s2 = row_sig2[tj] * inv;
        const double s6 = s2 * s2 * s2;
        const double c = row_eps24[tj] * inv * s6 * (2.0 * s6 - 1.0);
        fx += c * dx;
        fy += c * dy;
        fz += c * dz;
      }
    });
    Fx = fx;
    Fy = fy;
    Fz = fz;
  } else {
    const double bias = J.grid_bias;
    GridSum s;
    s.clear();
    for_entries(B, i, cnt, q, [&](uint32_t e) {
      const uint32_t tj = e >> kEntryTypeShift;
      double dx, dy, dz;
      const double r2 = sep(e, dx, dy, dz);
      float c = coef_f(tj, r2);
      c = r2 < row_rc2[tj] ? c : 0.0f;
      s.add(c, dx, dy, dz, bias);
    });
    exact = s.get(cnt, J.grid_cmax, Fx, Fy, Fz);
    if (!exact) {
      double fx = 0.0, fy = 0.0, fz = 0.0;
#pragma nounroll
      for (int k = 0; k < cnt; ++k) {
        const uint32_t e = row_entry_dyn(list_row(B, i, k / kRow), k % kRow);
        const uint32_t tj = e >> kEntryTypeShift;
        double dx, dy, dz;
        const double r2 = sep(e, dx, dy, dz);
        if (r2 < row_rc2[tj]) {
          const double c = (double)coef_f(tj, r2);
          fx += c * dx;
          fy += c * dy;
          fz += c * dz;
        }
      }
      Fx = fx;
      Fy = fy;
      Fz = fz;
    }
  }
}

// Energy share of slot i from the typed pairs (half of each pair).
__device__ __forceinline__ double pair_energy_model(const JobDev& J, const ModelDev& M, const DevBufs& B,
                                                    const double* __restrict__ X, int64_t first, int64_t i, int ti,
                                                    double xi, double yi, double zi) {
  const int cnt = (int)B.NCNT[i];
  const bool anyper = J.periodic[0] | J.periodic[1] | J.periodic[2];
  double u = 0.0;
  for (int k = 0; k < cnt; ++k) {
    const uint32_t e = row_entry(list_row(B, i, k / kRow), k % kRow);
    const int64_t j = window_slot(B, first, e & kEntryMask);
    const int p = ti * kMaxTypes + (int)(e >> kEntryTypeShift);
    double dx = xi - X[3 * j], dy = yi - X[3 * j + 1], dz = zi - X[3 * j + 2];
    if (anyper) min_image(J, dx, dy, dz);
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (!(r2 < M.rc2[p])) continue;
    const double s2 = M.sig2[p] / r2;
    const double s6 = s2 * s2 * s2;
    const double v = 0.5 * (M.eps4[p] * s6 * (s6 - 1.0) - M.phic[p]);
    u += J.force_fp64 ? v : (__builtin_fma(1.0, v, 0x1.8p20) - 0x1.8p20);
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

// Gather the positions and types of beads id-2 .. id+2 of id's molecule:
// from the tile's window through the entries bw (pos), else (an entry 0xFFFF
// for a bead of the molecule) through the inverse permutation.
template <class Pos>
__device__ __forceinline__ void molecule_window(const JobDev& J, const ModelDev& M, const DevBufs& B,
                                                const double* __restrict__ X, int64_t id, double xi, double yi,
                                                double zi, int ti, uint2 bw, Pos pos, double* xs, int* tid) {
  const int64_t bpm = M.bpm;
  const int64_t m0 = bpm > 0 ? (id / bpm) * bpm : id, m1 = bpm > 0 ? min(m0 + bpm, (int64_t)J.n) : id + 1;
  const uint8_t* __restrict__ T = B.TYPE[J.scur];
  const uint32_t ent[5] = {bw.x & 0xFFFFu, bw.x >> 16, 0u, bw.y & 0xFFFFu, bw.y >> 16};
  for (int q = 0; q < 5; ++q) {
    const int64_t g = id - 2 + q;
    tid[q] = 0;
    xs[3 * q] = xs[3 * q + 1] = xs[3 * q + 2] = 0.0;
    if (q == 2) {
      xs[6] = xi, xs[7] = yi, xs[8] = zi;
      tid[2] = ti;
    } else if (g >= m0 && g < m1) {
      if (ent[q] != 0xFFFFu) {
        pos(ent[q] & kEntryMask, xs[3 * q], xs[3 * q + 1], xs[3 * q + 2]);
        tid[q] = (int)(ent[q] >> kEntryTypeShift);
      } else {
        pos_of(J, B, X, g, xs + 3 * q);
        tid[q] = T[J.off + B.INV[J.off + g]];
      }
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
