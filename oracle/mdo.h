/*
 * mdo.h -- FP64 CPU oracle for molecular dynamics of particles held on an
 * implicit surface g(x) = 0 by RATTLE, under the Gronbech-Jensen/Farago
 * Langevin step (Paquay & Kusters, "A method for molecular dynamics on
 * curved surfaces", arXiv:1411.3019).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the reference that the GPU path
 * is checked against.  It shares no code, header, table or helper with the
 * GPU library; only tests, the smoke check and the benchmark's CPU-baseline
 * leg may load it.  Nothing in the product path may call it.
 *
 * What it computes, with the passage each part follows:
 *   - Hamiltonian with one Lagrange multiplier per particle and the
 *     constrained equations of motion: Eq. 1-4 (Section 2.1).
 *   - Position stage (Newton on the 4x4 bordered system for x^{m+1} and
 *     lambda) and momentum stage (Newton for p^{m+1} and mu): Algorithm 1
 *     (Section 2.2), taken literally, with a general 4x4 solve per iteration.
 *   - Langevin force combination: Algorithm S1 (SI, Section S1.2).
 *   - Truncated-shifted and linearly smoothed Lennard-Jones: Eq. S1.
 *   - Surfaces: sphere (Section 2.1), plane / cylinder / connector (torus)
 *     from the constraint functions of SI Section S3.1; ellipsoid and height
 *     field are written out in the same form.
 *   - Temperature with 2 degrees of freedom per constrained particle and 3
 *     per free one (Section 3.1).
 *   - Normal deviates: Philox4x32-10 (Salmon et al., SC'11) with the
 *     Box-Muller transform; the paper only asks for standard normals.
 *
 * Arrays are AoS: x[3*i + k].  All floating point is double.  Every entry
 * point returns 0 on success and a negative code on error.
 */
#ifndef MDO_H
#define MDO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MDO_SURF_NONE = 0,      /* no constraint                                   */
  MDO_SURF_PLANE = 1,     /* prm: x0 y0 z0 a b c       g = a(x-x0)+b(y-y0)+c(z-z0)       */
  MDO_SURF_SPHERE = 2,    /* prm: cx cy cz R           g = |x-c|^2 - R^2                 */
  MDO_SURF_ELLIPSOID = 3, /* prm: cx cy cz a b c       g = sum (x_k-c_k)^2/a_k^2 - 1     */
  MDO_SURF_TORUS = 4,     /* prm: cx cy cz Rt r        g = (rho-Rt)^2 + (z-cz)^2 - r^2   */
  MDO_SURF_CYLINDER = 5,  /* prm: x0 y0 z0 a b c R     g = a(x-x0)^2+b(y-y0)^2+c(z-z0)^2-R^2 */
  MDO_SURF_HEIGHT = 6,    /* prm: z0 A Lx Ly           g = z - z0 - A sin(2pi x/Lx) sin(2pi y/Ly) */
  MDO_SURF_BRIDGE = 7     /* prm: x0 y0 z0 Lb Rb R     piecewise (SI S3.1): a cylinder of radius Rb
                           * along x over |x-x0| <= Lb/2, connectors (R0 = Rb, tube radius R) at
                           * each end, and the planes x = x0 +- (Lb/2 + R) beyond them; each
                           * piece is scaled so that n is continuous across the joins */
};

enum {
  MDO_PAIR_NONE = 0,
  MDO_PAIR_LJ = 1,        /* truncated and shifted, Eq. S1 first form  */
  MDO_PAIR_LJ_SMOOTH = 2  /* linearly smoothed, Eq. S1 second form     */
};

enum {
  MDO_OK = 0,
  MDO_EINVAL = -1,
  MDO_ENEWTON = -4,       /* Newton iteration cap reached */
  MDO_ENOMEM = -6
};

/* Bead model of the capsid example (SI, Virus capsid self-assembly): bead
 * types with additive size mixing, truncated-shifted LJ per type pair (only
 * between beads of different molecules), linear molecules of bpm consecutive
 * particle indices with harmonic bonds V = kb (r - r0)^2 between neighbours and
 * bends V = ka (theta - theta0)^2 on consecutive triples (theta: the angle at
 * the middle bead between its two bonds, pi when straight), and a repulsive LJ
 * wall about the surface centre, 4 ew [(sw/d)^12 - (sw/d)^6 + 1/4] for
 * d = r - Rw < 2^(1/6) sw.  ntypes = 0 disables the model. */
#define MDO_MAX_TYPES 4
typedef struct {
  int ntypes;
  int bpm;              /* beads per molecule; 0: no molecules            */
  double sigma[MDO_MAX_TYPES];
  double eps[MDO_MAX_TYPES][MDO_MAX_TYPES];  /* LJ well depth per type pair */
  double rc[MDO_MAX_TYPES][MDO_MAX_TYPES];  /* 0: 2^(1/6) sigma_ij (purely repulsive) */
  double kb;
  double r0[MDO_MAX_TYPES][MDO_MAX_TYPES];  /* 0: 2^(1/6) (sigma_i + sigma_j) / 4 */
  double ka, theta0;
  double wall_eps, wall_sigma, wall_radius; /* wall_eps 0: no wall        */
} mdo_model;

typedef struct {
  double dt;            /* time step                                            */
  double kT;            /* thermal energy                                       */
  double gamma;         /* 1/tau of Algorithm S1; 0 means no thermostat (NVE)   */
  double eps, sigma, rc;/* Lennard-Jones parameters and cut-off                 */
  int pair;             /* MDO_PAIR_*                                           */
  int surface;          /* MDO_SURF_*                                           */
  double surf[8];       /* surface parameters, layout per kind above            */
  double gscale;        /* g is multiplied by this (0 is read as 1)             */
  double box_lo[3], box_hi[3];
  int periodic[3];      /* minimum image along dimensions flagged 1             */
  uint64_t seed;        /* Philox key                                           */
  double eta;           /* Newton tolerance on ||r||_inf; 0: iterate to round-off */
  int max_iter;         /* Newton iteration cap (0 is read as 32)               */
  int use_cells;        /* 1: linked-cell search; 0: all pairs                  */
  int frozen;           /* 1: the constraint row of the position-stage Jacobian
                           keeps n(x^m) instead of n at the iterate (the
                           frozen-normal variant of SI, Performance)          */
  mdo_model model;      /* bead model (model.ntypes > 0); rc must then be the
                           largest pair cut-off (cell size)                   */
  const uint8_t* types; /* bead type per particle (NULL: all type 0)          */
} mdo_params;

/* Philox4x32-10 block function: out = Philox(ctr, key). */
void mdo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* OpenMP threads the oracle's loops use (for reporting its timing), and a setter. */
int mdo_threads(void);
void mdo_set_threads(int n);

/* Three standard normals for particle id at step `step` (counter
 * (id, step lo, step hi, 0), key (seed lo, seed hi)), by Box-Muller. */
void mdo_normals(uint64_t seed, uint32_t id, int64_t step, double z[3]);

/* g(x) and its gradient n = dg/dx (not normalised, Eq. 4). */
double mdo_surface_g(const mdo_params* P, const double x[3], double grad[3]);

/* Pair forces F_i = -sum_j dV_ij/dx_i and total potential energy U.
 * upart (optional) receives U_i = 1/2 sum_j V_ij. */
int mdo_forces(const mdo_params* P, int64_t n, const double* x, double* F,
               double* upart, double* U);

/* Combined force at the first step (no previous draw or half-step momentum
 * exists): f = b [F(x) - p/tau + f_r^{step0}]; f = F(x) when gamma = 0. */
int mdo_init_force(const mdo_params* P, int64_t n, const double* x, const double* p,
                   const double* mass, const uint8_t* cons, int64_t step0, double* f);

/* Algorithm 1 position stage for one particle. */
int mdo_position_stage(const mdo_params* P, const double xm[3], const double pm[3],
                       const double fm[3], double m, double xn[3], double ph[3],
                       double* lambda, int* iters);

/* Algorithm 1 momentum stage for one particle. */
int mdo_momentum_stage(const mdo_params* P, const double xn[3], const double ph[3],
                       const double fn[3], double m, double pn[3], double* mu, int* iters);

/* Advance nsteps full steps (Algorithm S1 wrapped around Algorithm 1).
 * State in/out: x, p (full step), f (combined force), *step.
 * mass may be NULL (all 1); cons may be NULL (all constrained when a surface
 * is set).  *max_iter_seen (optional) receives the largest Newton count. */
int mdo_run(const mdo_params* P, int64_t n, double* x, double* p, double* f,
            const double* mass, const uint8_t* cons, int64_t* step, int64_t nsteps,
            int* max_iter_seen);

/* Diagnostics: out[0]=K, out[1]=U, out[2]=N_dof, out[3]=kT=2K/N_dof,
 * out[4]=max |g|/|grad g|, out[5]=max |n_hat . p/m|. */
int mdo_diag(const mdo_params* P, int64_t n, const double* x, const double* p,
             const double* mass, const uint8_t* cons, double out[6]);

#ifdef __cplusplus
}
#endif
#endif
