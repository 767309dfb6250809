/*
 * oracle.c -- FP64 CPU oracle (TEST INFRASTRUCTURE; see mdo.h).
 *
 * Plain, slow and written to be checked against the paper by eye:
 *   - Algorithm 1 is executed as printed: each Newton iteration forms the
 *     residual r and the Jacobian J of the bordered 4x4 system and solves
 *     J d = r with Gaussian elimination (partial pivoting); no closed-form
 *     shortcut is used here.
 *   - Algorithm S1 is executed in its order: position stage for all
 *     particles, then new pair forces, noise and the force combination, then
 *     the momentum stage for all particles.
 *   - Pair forces follow the definition F_i = -sum_{j != i} dV_ij/dx_i, with
 *     the terms added in increasing j.  The linked-cell search only skips pairs
 *     beyond the cut-off, whose terms are exactly zero; candidates are sorted
 *     by j so the additions happen in the same order as the all-pairs loop.
 *
 * Readings of the paper taken here (each one also listed in the design notes):
 *   - The garbled residuals in the text of Section 2.2 are read from
 *     Algorithm 1, whose Jacobian is the exact derivative of its residual.
 *   - The half-step momentum handed to the force stage is evaluated with the
 *     final multiplier lambda, so that x^{m+1} = x^m + (dt/m) p^{m+1/2} holds.
 *   - eta = 0 selects "iterate to round-off": stop once the Newton update of
 *     the position (momentum) is within 16 ulp of its scale.
 *   - The linear term of the smoothed potential carries the sign that makes
 *     the force vanish at r_c, which is the property the paper states.
 *   - Algorithm S1 writes the previous draw as f_r^n; it is read as the draw
 *     of the previous step.  At the first step the previous draw is taken to
 *     be the current one and p^{m+1/2} is replaced by p^m.
 *   - Noise: Philox4x32-10, counter (id, step lo, step hi, 0), key
 *     (seed lo, seed hi); u = (w + 1/2) 2^-32; Box-Muller on (w0,w1) and
 *     (w2,w3); the third normal is the cosine branch of the second pair.
 */
#include "mdo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).                        */
/* ------------------------------------------------------------------------ */

static void philox_round(uint32_t c[4], const uint32_t k[2]) {
  const uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
  const uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
  const uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
  const uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
  const uint32_t n0 = hi1 ^ c[1] ^ k[0];
  const uint32_t n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

int mdo_threads(void) { return omp_get_max_threads(); }

void mdo_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
}

void mdo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k[0] += 0x9E3779B9u;
      k[1] += 0xBB67AE85u;
    }
    philox_round(c, k);
  }
  memcpy(out, c, sizeof(c));
}

void mdo_normals(uint64_t seed, uint32_t id, int64_t step, double z[3]) {
  const uint64_t s = (uint64_t)step;
  const uint32_t ctr[4] = {id, (uint32_t)s, (uint32_t)(s >> 32), 0u};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  mdo_philox4x32_10(ctr, key, w);
  const double two32 = 4294967296.0;
  double u[4];
  for (int k = 0; k < 4; ++k) u[k] = ((double)w[k] + 0.5) / two32;
  const double r0 = sqrt(-2.0 * log(u[0]));
  const double r1 = sqrt(-2.0 * log(u[2]));
  z[0] = r0 * cos(2.0 * M_PI * u[1]);
  z[1] = r0 * sin(2.0 * M_PI * u[1]);
  z[2] = r1 * cos(2.0 * M_PI * u[3]);
}

/* ------------------------------------------------------------------------ */
/* Surfaces g(x) and n = dg/dx (Eq. 1 and 4; SI Section S3.1).              */
/* ------------------------------------------------------------------------ */

double mdo_surface_g(const mdo_params* P, const double x[3], double grad[3]) {
  const double* q = P->surf;
  const double alpha = (P->gscale != 0.0) ? P->gscale : 1.0;
  double g = 0.0;
  switch (P->surface) {
    case MDO_SURF_PLANE: {
      g = q[3] * (x[0] - q[0]) + q[4] * (x[1] - q[1]) + q[5] * (x[2] - q[2]);
      grad[0] = q[3];
      grad[1] = q[4];
      grad[2] = q[5];
      break;
    }
    case MDO_SURF_SPHERE: {
      const double d0 = x[0] - q[0], d1 = x[1] - q[1], d2 = x[2] - q[2];
      g = d0 * d0 + d1 * d1 + d2 * d2 - q[3] * q[3];
      grad[0] = 2.0 * d0;
      grad[1] = 2.0 * d1;
      grad[2] = 2.0 * d2;
      break;
    }
    case MDO_SURF_ELLIPSOID: {
      const double d0 = x[0] - q[0], d1 = x[1] - q[1], d2 = x[2] - q[2];
      const double a2 = q[3] * q[3], b2 = q[4] * q[4], c2 = q[5] * q[5];
      g = d0 * d0 / a2 + d1 * d1 / b2 + d2 * d2 / c2 - 1.0;
      grad[0] = 2.0 * d0 / a2;
      grad[1] = 2.0 * d1 / b2;
      grad[2] = 2.0 * d2 / c2;
      break;
    }
    case MDO_SURF_TORUS: {
      /* The connector of SI Section S3.1 with its axis along z: the distance
       * to a circle of radius Rt in the (rho, z) half-plane. */
      const double d0 = x[0] - q[0], d1 = x[1] - q[1], d2 = x[2] - q[2];
      const double rho = sqrt(d0 * d0 + d1 * d1);
      const double e = rho - q[3];
      g = e * e + d2 * d2 - q[4] * q[4];
      const double s = 2.0 * (1.0 - q[3] / rho);
      grad[0] = s * d0;
      grad[1] = s * d1;
      grad[2] = 2.0 * d2;
      break;
    }
    case MDO_SURF_CYLINDER: {
      const double d0 = x[0] - q[0], d1 = x[1] - q[1], d2 = x[2] - q[2];
      g = q[3] * d0 * d0 + q[4] * d1 * d1 + q[5] * d2 * d2 - q[6] * q[6];
      grad[0] = 2.0 * q[3] * d0;
      grad[1] = 2.0 * q[4] * d1;
      grad[2] = 2.0 * q[5] * d2;
      break;
    }
    case MDO_SURF_HEIGHT: {
      const double kx = 2.0 * M_PI / q[2], ky = 2.0 * M_PI / q[3];
      const double sx = sin(kx * x[0]), cx = cos(kx * x[0]);
      const double sy = sin(ky * x[1]), cy = cos(ky * x[1]);
      g = x[2] - q[0] - q[1] * sx * sy;
      grad[0] = -q[1] * kx * cx * sy;
      grad[1] = -q[1] * ky * sx * cy;
      grad[2] = 1.0;
      break;
    }
    case MDO_SURF_BRIDGE: {
      /* SI Section S3.1: the bridge between two blocks is a cylinder along x
       * (a = 0, b = c = 1, radius Rb), joined at each end by a connector
       * (distance to a circle of radius R in the (x, r) plane, centred at
       * x = x0 +- Lb/2, r = R0 + R with R0 = Rb) to a plane perpendicular to x.
       * The piece is chosen by position: |x - x0| <= Lb/2 the cylinder, else
       * r < Rb + R the connector, else the plane.  RATTLE is unchanged under
       * g -> alpha g, so each piece is multiplied by the constant that makes
       * n continuous where the pieces meet on the surface (|n| = 2R there):
       * the cylinder by -R/Rb, the plane's coefficient a = +-2R. */
      const double u = x[0] - q[0], dy = x[1] - q[1], dz = x[2] - q[2];
      const double half = 0.5 * q[3], Rb = q[4], R = q[5], rc = Rb + R;
      const double r = sqrt(dy * dy + dz * dz);
      if (fabs(u) <= half) {
        const double s = -R / Rb;
        g = s * (dy * dy + dz * dz - Rb * Rb);
        grad[0] = 0.0;
        grad[1] = 2.0 * s * dy;
        grad[2] = 2.0 * s * dz;
      } else if (r < rc) {
        const double x0 = u > 0.0 ? half : -half;
        const double e = r - rc;
        g = (u - x0) * (u - x0) + e * e - R * R;
        const double f = 2.0 * (1.0 - rc / r);
        grad[0] = 2.0 * (u - x0);
        grad[1] = f * dy;
        grad[2] = f * dz;
      } else {
        const double a = u > 0.0 ? 2.0 * R : -2.0 * R;
        const double xp = u > 0.0 ? half + R : -(half + R);
        g = a * (u - xp);
        grad[0] = a;
        grad[1] = 0.0;
        grad[2] = 0.0;
      }
      break;
    }
    default:
      grad[0] = grad[1] = grad[2] = 0.0;
      return 0.0;
  }
  grad[0] *= alpha;
  grad[1] *= alpha;
  grad[2] *= alpha;
  return alpha * g;
}

/* ------------------------------------------------------------------------ */
/* Pair potential, Eq. S1.                                                   */
/* ------------------------------------------------------------------------ */

/* phi(r) = 4 eps [(sigma/r)^12 - (sigma/r)^6] and its derivative. */
static double lj_phi(double eps, double sigma, double r, double* dphi) {
  const double sr = sigma / r;
  const double s6 = sr * sr * sr * sr * sr * sr;
  const double s12 = s6 * s6;
  *dphi = -24.0 * eps * (2.0 * s12 - s6) / r;
  return 4.0 * eps * (s12 - s6);
}

/* Energy V(r) and the scalar c such that the force on i from j is c*(x_i-x_j). */
static double pair_term(const mdo_params* P, double r2, double* coef) {
  const double r = sqrt(r2);
  double dphi, dphic;
  const double phi = lj_phi(P->eps, P->sigma, r, &dphi);
  const double phic = lj_phi(P->eps, P->sigma, P->rc, &dphic);
  if (P->pair == MDO_PAIR_LJ) {
    *coef = -dphi / r;
    return phi - phic;
  }
  /* linearly smoothed: V* = phi - phi(rc) - (r - rc) phi'(rc) */
  *coef = (-dphi + dphic) / r;
  return phi - phic - (r - P->rc) * dphic;
}

static void min_image(const mdo_params* P, double d[3]) {
  for (int k = 0; k < 3; ++k) {
    if (P->periodic[k]) {
      const double L = P->box_hi[k] - P->box_lo[k];
      d[k] -= L * nearbyint(d[k] / L);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Bead model (SI, Virus capsid self-assembly).                              */
/* ------------------------------------------------------------------------ */

static int type_of(const mdo_params* P, int64_t i) { return P->types ? P->types[i] : 0; }

static double model_sigma(const mdo_model* M, int a, int b) { return 0.5 * (M->sigma[a] + M->sigma[b]); }

static double model_rc(const mdo_model* M, int a, int b) {
  return M->rc[a][b] > 0.0 ? M->rc[a][b] : pow(2.0, 1.0 / 6.0) * model_sigma(M, a, b);
}

static double model_r0(const mdo_model* M, int a, int b) {
  return M->r0[a][b] > 0.0 ? M->r0[a][b] : pow(2.0, 1.0 / 6.0) * (M->sigma[a] + M->sigma[b]) / 4.0;
}

/* Truncated-shifted LJ of the type pair (a, b): energy and c with force c*d. */
static double model_pair(const mdo_model* M, int a, int b, double r2, double* coef) {
  const double r = sqrt(r2), s = model_sigma(M, a, b), rc = model_rc(M, a, b);
  double dphi, dphic;
  const double phi = lj_phi(M->eps[a][b], s, r, &dphi);
  const double phic = lj_phi(M->eps[a][b], s, rc, &dphic);
  *coef = -dphi / r;
  return phi - phic;
}

static int same_molecule(const mdo_model* M, int64_t i, int64_t j) { return M->bpm > 0 && i / M->bpm == j / M->bpm; }

/* Bond between i and j: force on i and energy kb (r - r0)^2. */
static double bond_term(const mdo_params* P, const double* x, int64_t i, int64_t j, double f[3]) {
  const mdo_model* M = &P->model;
  double d[3] = {x[3 * i] - x[3 * j], x[3 * i + 1] - x[3 * j + 1], x[3 * i + 2] - x[3 * j + 2]};
  min_image(P, d);
  const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  const double r0 = model_r0(M, type_of(P, i), type_of(P, j));
  const double c = -2.0 * M->kb * (r - r0) / r;
  for (int k = 0; k < 3; ++k) f[k] = c * d[k];
  return M->kb * (r - r0) * (r - r0);
}

/* Bend at b between bonds b->a and b->c: force on particle `on` (one of a, b,
 * c) and energy ka (theta - theta0)^2, theta = angle between x_a - x_b and
 * x_c - x_b.  dV/dx = 2 ka (theta - theta0) dtheta/dcos dcos/dx with dtheta/dcos
 * = -1/sin(theta); where sin(theta) vanishes, (theta - theta0)/sin(theta) takes
 * its limit (-1 at theta = theta0 = pi, the straight molecule). */
static double bend_term(const mdo_params* P, const double* x, int64_t a, int64_t b, int64_t c, int64_t on,
                        double f[3]) {
  const mdo_model* M = &P->model;
  double u[3] = {x[3 * a] - x[3 * b], x[3 * a + 1] - x[3 * b + 1], x[3 * a + 2] - x[3 * b + 2]};
  double v[3] = {x[3 * c] - x[3 * b], x[3 * c + 1] - x[3 * b + 1], x[3 * c + 2] - x[3 * b + 2]};
  min_image(P, u);
  min_image(P, v);
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2], vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const double nu = sqrt(uu), nv = sqrt(vv);
  double cs = (u[0] * v[0] + u[1] * v[1] + u[2] * v[2]) / (nu * nv);
  if (cs > 1.0) cs = 1.0;
  if (cs < -1.0) cs = -1.0;
  const double th = acos(cs), sn = sqrt(1.0 - cs * cs);
  const double dth = th - M->theta0;
  double ratio;
  if (sn > 1e-12) ratio = dth / sn;
  else ratio = (fabs(dth) < 1e-6) ? (th > 1.5 ? -1.0 : 1.0) : dth / 1e-12;
  /* F = -dV/dx = 2 ka ratio dcos/dx */
  const double k2 = 2.0 * M->ka * ratio;
  double ga[3], gc[3];
  for (int k = 0; k < 3; ++k) {
    ga[k] = v[k] / (nu * nv) - cs * u[k] / uu;
    gc[k] = u[k] / (nu * nv) - cs * v[k] / vv;
  }
  for (int k = 0; k < 3; ++k) {
    const double g = on == a ? ga[k] : (on == c ? gc[k] : -(ga[k] + gc[k]));
    f[k] = k2 * g;
  }
  return M->ka * dth * dth;
}

/* Wall about the surface centre: force on i and energy. */
static double wall_term(const mdo_params* P, const double* x, int64_t i, double f[3]) {
  const mdo_model* M = &P->model;
  f[0] = f[1] = f[2] = 0.0;
  if (!(M->wall_eps > 0.0)) return 0.0;
  double d[3] = {x[3 * i] - P->surf[0], x[3 * i + 1] - P->surf[1], x[3 * i + 2] - P->surf[2]};
  const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  const double s = r - M->wall_radius;
  if (!(s < pow(2.0, 1.0 / 6.0) * M->wall_sigma) || !(r > 0.0)) return 0.0;
  double dphi;
  const double phi = lj_phi(M->wall_eps, M->wall_sigma, s, &dphi);
  for (int k = 0; k < 3; ++k) f[k] = -dphi * d[k] / r;
  return phi + M->wall_eps;
}

/* Bonded and wall forces on i, in a fixed order: bonds to i-1 and i+1, bends
 * centred at i-1, i and i+1, the wall.  Returns i's energy share (half of each
 * bond, a third of each bend, all of its wall term). */
static double bonded_i(const mdo_params* P, int64_t n, const double* x, int64_t i, double Fi[3]) {
  const mdo_model* M = &P->model;
  double u = 0.0, f[3];
  if (M->bpm > 1) {
    const int64_t m0 = (i / M->bpm) * M->bpm, m1 = m0 + M->bpm < n ? m0 + M->bpm : n;
    if (i - 1 >= m0) {
      u += 0.5 * bond_term(P, x, i, i - 1, f);
      for (int k = 0; k < 3; ++k) Fi[k] += f[k];
    }
    if (i + 1 < m1) {
      u += 0.5 * bond_term(P, x, i, i + 1, f);
      for (int k = 0; k < 3; ++k) Fi[k] += f[k];
    }
    for (int64_t b = i - 1; b <= i + 1; ++b) {
      if (b - 1 < m0 || b + 1 >= m1) continue;
      u += bend_term(P, x, b - 1, b, b + 1, i, f) / 3.0;
      for (int k = 0; k < 3; ++k) Fi[k] += f[k];
    }
  }
  u += wall_term(P, x, i, f);
  for (int k = 0; k < 3; ++k) Fi[k] += f[k];
  return u;
}

/* Interaction of i with the candidates js[0..nj) (ascending, may include i). */
static void accumulate_i(const mdo_params* P, int64_t i, const double* x, const int64_t* js,
                         int64_t nj, double Fi[3], double* Ui) {
  const double rc2 = P->rc * P->rc;
  const int model = P->model.ntypes > 0;
  const int ti = model ? type_of(P, i) : 0;
  double f0 = 0.0, f1 = 0.0, f2 = 0.0, u = 0.0;
  for (int64_t t = 0; t < nj; ++t) {
    const int64_t j = js[t];
    if (j == i) continue;
    if (model && same_molecule(&P->model, i, j)) continue;
    double d[3] = {x[3 * i] - x[3 * j], x[3 * i + 1] - x[3 * j + 1], x[3 * i + 2] - x[3 * j + 2]};
    min_image(P, d);
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double c, v;
    if (model) {
      const int tj = type_of(P, j);
      const double rcij = model_rc(&P->model, ti, tj);
      if (r2 >= rcij * rcij) continue;
      v = model_pair(&P->model, ti, tj, r2, &c);
    } else {
      if (r2 >= rc2) continue;
      v = pair_term(P, r2, &c);
    }
    f0 += c * d[0];
    f1 += c * d[1];
    f2 += c * d[2];
    u += 0.5 * v;
  }
  Fi[0] = f0;
  Fi[1] = f1;
  Fi[2] = f2;
  *Ui = u;
}

static int cmp_i64(const void* a, const void* b) {
  const int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

typedef struct {
  int nc[3];
  double lo[3], cs[3];
  int64_t ncell;
  int64_t* head;
  int64_t* next;
} cells_t;

static int64_t cell_coord(const cells_t* C, const mdo_params* P, int k, double v) {
  int64_t c = (int64_t)floor((v - C->lo[k]) / C->cs[k]);
  if (P->periodic[k]) {
    c %= C->nc[k];
    if (c < 0) c += C->nc[k];
  } else {
    if (c < 0) c = 0;
    if (c >= C->nc[k]) c = C->nc[k] - 1;
  }
  return c;
}

/* Linked cells of side >= rc.  Returns 0 if the all-pairs loop must be used. */
static int cells_build(const mdo_params* P, int64_t n, const double* x, cells_t* C) {
  memset(C, 0, sizeof(*C));
  for (int k = 0; k < 3; ++k) {
    double lo, hi;
    if (P->periodic[k]) {
      lo = P->box_lo[k];
      hi = P->box_hi[k];
    } else {
      lo = hi = x[k];
      for (int64_t i = 1; i < n; ++i) {
        if (x[3 * i + k] < lo) lo = x[3 * i + k];
        if (x[3 * i + k] > hi) hi = x[3 * i + k];
      }
    }
    const double ext = hi - lo;
    int nc = (int)floor(ext / P->rc);
    if (P->periodic[k] && nc < 3) return 0;
    if (nc < 1) nc = 1;
    C->nc[k] = nc;
    C->lo[k] = lo;
    C->cs[k] = (ext > 0.0) ? ext / nc : 1.0;
  }
  C->ncell = (int64_t)C->nc[0] * C->nc[1] * C->nc[2];
  if (C->ncell > 400000000LL) return 0;
  C->head = (int64_t*)malloc(sizeof(int64_t) * (size_t)C->ncell);
  C->next = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!C->head || !C->next) {
    free(C->head);
    free(C->next);
    return 0;
  }
  for (int64_t c = 0; c < C->ncell; ++c) C->head[c] = -1;
  for (int64_t i = n - 1; i >= 0; --i) {
    const int64_t cx = cell_coord(C, P, 0, x[3 * i]);
    const int64_t cy = cell_coord(C, P, 1, x[3 * i + 1]);
    const int64_t cz = cell_coord(C, P, 2, x[3 * i + 2]);
    const int64_t c = (cx * C->nc[1] + cy) * C->nc[2] + cz;
    C->next[i] = C->head[c];
    C->head[c] = i;
  }
  return 1;
}

int mdo_forces(const mdo_params* P, int64_t n, const double* x, double* F, double* upart,
               double* U) {
  if (n < 0 || !x || !F) return MDO_EINVAL;
  double* ui = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  if (!ui) return MDO_ENOMEM;
  if (P->pair == MDO_PAIR_NONE || n == 0) {
    for (int64_t i = 0; i < 3 * n; ++i) F[i] = 0.0;
    for (int64_t i = 0; i < n; ++i) ui[i] = 0.0;
  } else {
    cells_t C;
    const int have_cells = P->use_cells ? cells_build(P, n, x, &C) : 0;
    int failed = 0;
#pragma omp parallel
    {
      int64_t cap = have_cells ? 256 : n;
      int64_t* js = (int64_t*)malloc(sizeof(int64_t) * (size_t)(cap > 0 ? cap : 1));
      if (!js) {
#pragma omp atomic write
        failed = 1;
      }
      if (!have_cells && js)
        for (int64_t j = 0; j < n; ++j) js[j] = j;
#pragma omp for schedule(static)
      for (int64_t i = 0; i < n; ++i) {
        if (!js) continue;
        int64_t nj = n;
        if (have_cells) {
          nj = 0;
          const int64_t c0[3] = {cell_coord(&C, P, 0, x[3 * i]), cell_coord(&C, P, 1, x[3 * i + 1]),
                                 cell_coord(&C, P, 2, x[3 * i + 2])};
          for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
              for (int dz = -1; dz <= 1; ++dz) {
                int64_t cc[3] = {c0[0] + dx, c0[1] + dy, c0[2] + dz};
                int skip = 0;
                for (int k = 0; k < 3; ++k) {
                  if (P->periodic[k]) {
                    cc[k] = (cc[k] + C.nc[k]) % C.nc[k];
                  } else if (cc[k] < 0 || cc[k] >= C.nc[k]) {
                    skip = 1;
                  }
                }
                if (skip) continue;
                const int64_t c = (cc[0] * C.nc[1] + cc[1]) * C.nc[2] + cc[2];
                for (int64_t j = C.head[c]; j >= 0; j = C.next[j]) {
                  if (nj == cap) {
                    cap *= 2;
                    int64_t* grown = (int64_t*)realloc(js, sizeof(int64_t) * (size_t)cap);
                    if (!grown) abort();
                    js = grown;
                  }
                  js[nj++] = j;
                }
              }
          qsort(js, (size_t)nj, sizeof(int64_t), cmp_i64);
        }
        accumulate_i(P, i, x, js, nj, &F[3 * i], &ui[i]);
        if (P->model.ntypes > 0) ui[i] += bonded_i(P, n, x, i, &F[3 * i]);
      }
      free(js);
    }
    if (have_cells) {
      free(C.head);
      free(C.next);
    }
    if (failed) {
      free(ui);
      return MDO_ENOMEM;
    }
  }
  double utot = 0.0;
  for (int64_t i = 0; i < n; ++i) utot += ui[i];
  if (upart)
    for (int64_t i = 0; i < n; ++i) upart[i] = ui[i];
  if (U) *U = utot;
  free(ui);
  return MDO_OK;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1: the two Newton stages for one particle.                     */
/* ------------------------------------------------------------------------ */

/* Solve A d = r for a 4x4 system by Gaussian elimination with partial pivoting. */
static int solve4(double A[4][4], double r[4], double d[4]) {
  double M[4][5];
  for (int i = 0; i < 4; ++i) {
    for (int j = 0; j < 4; ++j) M[i][j] = A[i][j];
    M[i][4] = r[i];
  }
  for (int col = 0; col < 4; ++col) {
    int piv = col;
    for (int i = col + 1; i < 4; ++i)
      if (fabs(M[i][col]) > fabs(M[piv][col])) piv = i;
    if (M[piv][col] == 0.0) return -1;
    if (piv != col)
      for (int j = 0; j < 5; ++j) {
        const double t = M[col][j];
        M[col][j] = M[piv][j];
        M[piv][j] = t;
      }
    for (int i = col + 1; i < 4; ++i) {
      const double fac = M[i][col] / M[col][col];
      for (int j = col; j < 5; ++j) M[i][j] -= fac * M[col][j];
    }
  }
  for (int i = 3; i >= 0; --i) {
    double s = M[i][4];
    for (int j = i + 1; j < 4; ++j) s -= M[i][j] * d[j];
    d[i] = s / M[i][i];
  }
  return 0;
}

static double maxabs3(const double v[3]) {
  double m = fabs(v[0]);
  if (fabs(v[1]) > m) m = fabs(v[1]);
  if (fabs(v[2]) > m) m = fabs(v[2]);
  return m;
}

static int iter_cap(const mdo_params* P) { return P->max_iter > 0 ? P->max_iter : 32; }

int mdo_position_stage(const mdo_params* P, const double xm[3], const double pm[3],
                       const double fm[3], double m, double xn[3], double ph[3], double* lambda,
                       int* iters) {
  const double dt = P->dt;
  double nm[3];
  (void)mdo_surface_g(P, xm, nm);
  double lam = 0.0;
  xn[0] = xm[0];
  xn[1] = xm[1];
  xn[2] = xm[2];
  const int cap = iter_cap(P);
  int it = 0, done = 0;
  while (!done && it < cap) {
    ++it;
    for (int k = 0; k < 3; ++k) ph[k] = pm[k] + 0.5 * dt * (fm[k] - lam * nm[k]);
    double nn[3];
    double r[4];
    for (int k = 0; k < 3; ++k) r[k] = xm[k] - xn[k] + (dt / m) * ph[k];
    r[3] = mdo_surface_g(P, xn, nn);
    const double c = dt * dt / (2.0 * m);
    /* full Newton: dg/dx at the iterate; frozen normal: at x^m (SI, Performance) */
    const double* jr = P->frozen ? nm : nn;
    double J[4][4] = {{-1.0, 0.0, 0.0, -c * nm[0]},
                      {0.0, -1.0, 0.0, -c * nm[1]},
                      {0.0, 0.0, -1.0, -c * nm[2]},
                      {jr[0], jr[1], jr[2], 0.0}};
    double d[4];
    if (solve4(J, r, d) != 0) return MDO_ENEWTON;
    for (int k = 0; k < 3; ++k) xn[k] -= d[k];
    lam -= d[3];
    if (P->eta > 0.0) {
      double rn = fabs(r[3]);
      for (int k = 0; k < 3; ++k)
        if (fabs(r[k]) > rn) rn = fabs(r[k]);
      done = rn < P->eta;
    } else {
      const double scale = fmax(1.0, maxabs3(xn));
      done = maxabs3(d) <= 16.0 * DBL_EPSILON * scale;
    }
  }
  for (int k = 0; k < 3; ++k) ph[k] = pm[k] + 0.5 * dt * (fm[k] - lam * nm[k]);
  if (lambda) *lambda = lam;
  if (iters) *iters = it;
  return done ? MDO_OK : MDO_ENEWTON;
}

int mdo_momentum_stage(const mdo_params* P, const double xn[3], const double ph[3],
                       const double fn[3], double m, double pn[3], double* mu, int* iters) {
  const double dt = P->dt;
  double nn[3];
  (void)mdo_surface_g(P, xn, nn);
  double u = 0.0;
  for (int k = 0; k < 3; ++k) pn[k] = ph[k] + 0.5 * dt * fn[k];
  const int cap = iter_cap(P);
  int it = 0, done = 0;
  while (!done && it < cap) {
    ++it;
    double pdot[3], r[4];
    for (int k = 0; k < 3; ++k) pdot[k] = fn[k] - u * nn[k];
    for (int k = 0; k < 3; ++k) r[k] = ph[k] - pn[k] + 0.5 * dt * pdot[k];
    r[3] = (nn[0] * pn[0] + nn[1] * pn[1] + nn[2] * pn[2]) / m;
    double J[4][4] = {{-1.0, 0.0, 0.0, -0.5 * dt * nn[0]},
                      {0.0, -1.0, 0.0, -0.5 * dt * nn[1]},
                      {0.0, 0.0, -1.0, -0.5 * dt * nn[2]},
                      {nn[0] / m, nn[1] / m, nn[2] / m, 0.0}};
    double d[4];
    if (solve4(J, r, d) != 0) return MDO_ENEWTON;
    for (int k = 0; k < 3; ++k) pn[k] -= d[k];
    u -= d[3];
    if (P->eta > 0.0) {
      double rn = fabs(r[3]);
      for (int k = 0; k < 3; ++k)
        if (fabs(r[k]) > rn) rn = fabs(r[k]);
      done = rn < P->eta;
    } else {
      const double scale = fmax(1.0, maxabs3(pn));
      done = maxabs3(d) <= 16.0 * DBL_EPSILON * scale;
    }
  }
  if (mu) *mu = u;
  if (iters) *iters = it;
  return done ? MDO_OK : MDO_ENEWTON;
}

/* ------------------------------------------------------------------------ */
/* Algorithm S1: the full step.                                              */
/* ------------------------------------------------------------------------ */

static int is_constrained(const mdo_params* P, const uint8_t* cons, int64_t i) {
  if (P->surface == MDO_SURF_NONE) return 0;
  return cons ? (cons[i] != 0) : 1;
}

static double mass_of(const double* mass, int64_t i) { return mass ? mass[i] : 1.0; }

/* Random force f_r = sqrt(2 m kT / (tau dt)) (r_x, r_y, r_z) of Algorithm S1. */
static void random_force(const mdo_params* P, double m, int64_t i, int64_t step, double fr[3]) {
  double z[3];
  mdo_normals(P->seed, (uint32_t)i, step, z);
  const double s = sqrt(2.0 * m * P->kT * P->gamma / P->dt);
  fr[0] = s * z[0];
  fr[1] = s * z[1];
  fr[2] = s * z[2];
}

int mdo_init_force(const mdo_params* P, int64_t n, const double* x, const double* p,
                   const double* mass, const uint8_t* cons, int64_t step0, double* f) {
  (void)cons;
  double* F = (double*)malloc(sizeof(double) * (size_t)(3 * n + 1));
  if (!F) return MDO_ENOMEM;
  int rc = mdo_forces(P, n, x, F, NULL, NULL);
  if (rc != MDO_OK) {
    free(F);
    return rc;
  }
  if (P->gamma > 0.0) {
    const double b = 1.0 / (1.0 + 0.5 * P->dt * P->gamma);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      const double m = mass_of(mass, i);
      double fr[3];
      random_force(P, m, i, step0, fr);
      for (int k = 0; k < 3; ++k)
        f[3 * i + k] = b * (F[3 * i + k] - P->gamma * p[3 * i + k] + fr[k]);
    }
  } else {
    for (int64_t i = 0; i < 3 * n; ++i) f[i] = F[i];
  }
  free(F);
  return MDO_OK;
}

int mdo_run(const mdo_params* P, int64_t n, double* x, double* p, double* f,
            const double* mass, const uint8_t* cons, int64_t* step, int64_t nsteps,
            int* max_iter_seen) {
  if (n < 0 || nsteps < 0 || !step) return MDO_EINVAL;
  const size_t bytes = sizeof(double) * (size_t)(3 * n + 1);
  double* x1 = (double*)malloc(bytes);
  double* ph = (double*)malloc(bytes);
  double* F = (double*)malloc(bytes);
  if (!x1 || !ph || !F) {
    free(x1);
    free(ph);
    free(F);
    return MDO_ENOMEM;
  }
  const double b = (P->gamma > 0.0) ? 1.0 / (1.0 + 0.5 * P->dt * P->gamma) : 1.0;
  int status = MDO_OK;
  int maxit = 0;
  for (int64_t s = 0; s < nsteps && status == MDO_OK; ++s) {
    const int64_t k = *step;
    int bad = 0, smax = 0;
    /* Position stage, all particles. */
#pragma omp parallel for schedule(static) reduction(max : smax) reduction(| : bad)
    for (int64_t i = 0; i < n; ++i) {
      const double m = mass_of(mass, i);
      if (is_constrained(P, cons, i)) {
        int it = 0;
        if (mdo_position_stage(P, &x[3 * i], &p[3 * i], &f[3 * i], m, &x1[3 * i], &ph[3 * i],
                               NULL, &it) != MDO_OK)
          bad |= 1;
        if (it > smax) smax = it;
      } else {
        for (int q = 0; q < 3; ++q) {
          ph[3 * i + q] = p[3 * i + q] + 0.5 * P->dt * f[3 * i + q];
          x1[3 * i + q] = x[3 * i + q] + (P->dt / m) * ph[3 * i + q];
        }
      }
    }
    if (bad) {
      status = MDO_ENEWTON;
      break;
    }
    /* Force stage. */
    status = mdo_forces(P, n, x1, F, NULL, NULL);
    if (status != MDO_OK) break;
    /* Force combination and momentum stage. */
#pragma omp parallel for schedule(static) reduction(max : smax) reduction(| : bad)
    for (int64_t i = 0; i < n; ++i) {
      const double m = mass_of(mass, i);
      double fn[3];
      if (P->gamma > 0.0) {
        double fr_new[3], fr_old[3];
        random_force(P, m, i, k + 1, fr_new);
        random_force(P, m, i, k, fr_old);
        for (int q = 0; q < 3; ++q)
          fn[q] = b * (F[3 * i + q] - P->gamma * ph[3 * i + q] + 0.5 * (fr_new[q] + fr_old[q]));
      } else {
        for (int q = 0; q < 3; ++q) fn[q] = F[3 * i + q];
      }
      if (is_constrained(P, cons, i)) {
        int it = 0;
        if (mdo_momentum_stage(P, &x1[3 * i], &ph[3 * i], fn, m, &p[3 * i], NULL, &it) != MDO_OK)
          bad |= 1;
        if (it > smax) smax = it;
      } else {
        for (int q = 0; q < 3; ++q) p[3 * i + q] = ph[3 * i + q] + 0.5 * P->dt * fn[q];
      }
      for (int q = 0; q < 3; ++q) f[3 * i + q] = fn[q];
    }
    if (bad) {
      status = MDO_ENEWTON;
      break;
    }
    memcpy(x, x1, sizeof(double) * (size_t)(3 * n));
    if (smax > maxit) maxit = smax;
    *step = k + 1;
  }
  if (max_iter_seen) *max_iter_seen = maxit;
  free(x1);
  free(ph);
  free(F);
  return status;
}

int mdo_diag(const mdo_params* P, int64_t n, const double* x, const double* p,
             const double* mass, const uint8_t* cons, double out[6]) {
  double* F = (double*)malloc(sizeof(double) * (size_t)(3 * n + 1));
  if (!F) return MDO_ENOMEM;
  double U = 0.0;
  int rc = mdo_forces(P, n, x, F, NULL, &U);
  free(F);
  if (rc != MDO_OK) return rc;
  double K = 0.0, ndof = 0.0, gmax = 0.0, nvmax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double m = mass_of(mass, i);
    const double* pi = &p[3 * i];
    K += (pi[0] * pi[0] + pi[1] * pi[1] + pi[2] * pi[2]) / (2.0 * m);
    if (is_constrained(P, cons, i)) {
      ndof += 2.0;
      double gr[3];
      const double g = mdo_surface_g(P, &x[3 * i], gr);
      const double gn = sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
      const double dist = fabs(g) / gn;
      const double nv = fabs(gr[0] * pi[0] + gr[1] * pi[1] + gr[2] * pi[2]) / (gn * m);
      if (dist > gmax) gmax = dist;
      if (nv > nvmax) nvmax = nv;
    } else {
      ndof += 3.0;
    }
  }
  out[0] = K;
  out[1] = U;
  out[2] = ndof;
  out[3] = ndof > 0.0 ? 2.0 * K / ndof : 0.0;
  out[4] = gmax;
  out[5] = nvmax;
  return MDO_OK;
}
