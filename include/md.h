/*
 * md.h -- C ABI of the MI355X (gfx950) library for molecular dynamics of
 * particles held on an implicit surface g(x) = 0 by a per-particle RATTLE
 * constraint under the Gronbech-Jensen/Farago Langevin step.
 *
 * Method: Paquay & Kusters, "A method for molecular dynamics on curved
 * surfaces" (arXiv:1411.3019).
 *   - state and equations of motion: Eq. 1-4 (Section 2.1): particles with
 *     position x_i, momentum p_i, mass m_i; constraint g(x_i) = 0 with the
 *     un-normalised normal n = dg/dx; pair potential V_ij;
 *   - one time step: Algorithm 1 (Section 2.2) inside Algorithm S1 (SI,
 *     Section S1.2); both RATTLE stages are solved per particle (the
 *     Jacobian solve in closed form, as Section 2.2 and SI Section S2 say is
 *     possible and fastest);
 *   - pair potentials: Eq. S1 (truncated-shifted and linearly smoothed LJ);
 *   - only some particles may be constrained (Section 1);
 *   - temperature kT = 2K/N_dof with 2 dof per constrained particle
 *     (Section 3.1).
 *
 * Conventions for every entry point:
 *   - returns 0 (MD_OK) or a negative MD_E* code; never aborts or throws
 *     across the ABI; md_strerror() names the code;
 *   - host arrays are owned by the caller, read or written during the call
 *     only, and are AoS: x[3*i + k] for particle i, component k;
 *   - a context or pool owns all device memory it allocates and releases it
 *     in md_destroy / md_pool_destroy;
 *   - one context or pool per host thread; calls on one object must not
 *     overlap;
 *   - all GPU work is ordered on the stream given at creation (a hipStream_t;
 *     NULL makes the library create its own stream of default priority);
 *     calls that return host data synchronise that stream.
 *
 * Results do not depend on the neighbour-list rebuild schedule or on which
 * other jobs share a pool: pair forces are summed over neighbours in the
 * order of their particle index, and every per-particle quantity depends on
 * the particle's own job only.
 */
#ifndef MD_H
#define MD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------------- */
#define MD_OK 0
#define MD_EINVAL -1    /* invalid argument or parameter                         */
#define MD_ESTATE -2    /* call out of order (e.g. md_step before particles)     */
#define MD_EOFFSURF -3  /* input particle off the surface or with normal momentum */
#define MD_ENEWTON -4   /* RATTLE Newton iteration hit its cap                    */
#define MD_ENAN -5      /* non-finite position or momentum                        */
#define MD_ENOMEM -6    /* device or host allocation failed                       */
#define MD_EAGAIN -7    /* pool: no room for the job right now                    */
#define MD_EHIP -8      /* HIP runtime error                                      */
#define MD_ENOTFOUND -9 /* pool: unknown job id                                   */

/* ---- surfaces g(x) and their parameter layout (prm[]) -----------------------
 * The normal is n = dg/dx, used un-normalised as in Eq. 4.
 *   MD_SURF_NONE       no constraint (every particle moves freely)
 *   MD_SURF_PLANE      x0 y0 z0 a b c     g = a(x-x0) + b(y-y0) + c(z-z0)      (SI S3.1)
 *   MD_SURF_SPHERE     cx cy cz R         g = |x-c|^2 - R^2                    (Section 2.1)
 *   MD_SURF_ELLIPSOID  cx cy cz a b c     g = sum_k (x_k-c_k)^2/a_k^2 - 1
 *   MD_SURF_TORUS      cx cy cz Rt r      g = (rho - Rt)^2 + (z-cz)^2 - r^2,
 *                                         rho = |(x-cx, y-cy)|; the connector of
 *                                         SI S3.1 with its axis along z
 *   MD_SURF_CYLINDER   x0 y0 z0 a b c R   g = a(x-x0)^2 + b(y-y0)^2 + c(z-z0)^2 - R^2,
 *                                         one of a, b, c zero            (SI S3.1)
 *   MD_SURF_HEIGHT     z0 A Lx Ly         g = z - z0 - A sin(2 pi x/Lx) sin(2 pi y/Ly);
 *                                         needs a box periodic in x and y
 *   MD_SURF_BRIDGE     x0 y0 z0 Lb Rb R   piecewise (SI S3.1, the thylakoid bridge): with
 *                                         u = x-x0, r = |(y-y0, z-z0)|, h = Lb/2:
 *                                         |u| <= h:        cylinder (R/Rb)(Rb^2 - r^2);
 *                                         else r < Rb+R:   connector (|u|-h)^2 + (r-Rb-R)^2 - R^2;
 *                                         else:            plane 2R(|u| - h - R).
 *                                         The piece is chosen by the position g is
 *                                         evaluated at; the factors make n continuous
 *                                         where pieces meet (|n| = 2R there).  Lb >= 0,
 *                                         Rb, R > 0; along periodic y or z the box side
 *                                         must be at least 2(Rb + R).  */
#define MD_SURF_NONE 0
#define MD_SURF_PLANE 1
#define MD_SURF_SPHERE 2
#define MD_SURF_ELLIPSOID 3
#define MD_SURF_TORUS 4
#define MD_SURF_CYLINDER 5
#define MD_SURF_HEIGHT 6
#define MD_SURF_BRIDGE 7
#define MD_SURF_MAXPRM 8

/* ---- pair potentials (Eq. S1) ---------------------------------------------- */
#define MD_PAIR_NONE 0
#define MD_PAIR_LJ 1        /* phi(r) - phi(rc) for r < rc; WCA is rc = 2^(1/6) sigma */
#define MD_PAIR_LJ_SMOOTH 2 /* phi(r) - phi(rc) - (r - rc) phi'(rc) for r < rc       */

/* ---- parameters --------------------------------------------------------------
 * gamma is the rate 1/tau of Algorithm S1 (friction m gamma, noise
 * sqrt(2 m kT gamma / dt)); gamma = 0 gives plain constant-energy dynamics.
 * force_fp64 = 1 computes pair forces in FP64, summed in particle-index order;
 * 0 computes each pair coefficient in FP32 from the FP64 separation and sums
 * the terms exactly (each rounded once to a 2^-32 grid, summed without
 * rounding), so the result does not depend on the order of the terms while
 * every term stays below 2^19 (md_diag.exact_sum_breaches counts the
 * exceptions).  Positions, momenta, the RATTLE solves and the tangent
 * projection are always FP64.
 * newton_tol is the paper's eta on ||r||_inf (Section 2.2); 0 iterates to
 * round-off (stop when the Newton update is within 16 ulp of the position).
 * skin: neighbour-list skin (0 selects 0.3 sigma); lists are rebuilt before
 * any particle has moved more than skin/2.
 * box: for a periodic dimension, [box_lo, box_hi) is the period; for a
 * non-periodic one a non-empty [box_lo, box_hi) bounds the cell grid, else the
 * grid is sized from the surface (or, with no surface, from the particles).  */
typedef struct md_params {
  double dt;
  double kT;
  double gamma;
  double eps;
  double sigma;
  double rc;
  int pair_kind;
  int force_fp64;
  double skin;
  double box_lo[3];
  double box_hi[3];
  int periodic[3];
  uint64_t seed;          /* Philox key of the Langevin noise                   */
  double newton_tol;
  int newton_max_iter;    /* 0 selects 32                                       */
  int newton_frozen;      /* 1: position-stage Newton keeps the normal of x^m in
                             its Jacobian (the frozen-normal variant, SI,
                             Performance); 0: full Newton (default)            */
  int device;             /* HIP device ordinal                                 */
  void* stream;           /* hipStream_t or NULL                                */
} md_params;

/* ---- bead model ----------------------------------------------------------------
 * The bead model of the capsid example (SI, Virus capsid self-assembly), for a
 * system (md_set_model) or a pool job (md_job_desc.model):
 *  - bead types 0..ntypes-1 with sizes sigma[a]; sigma_ab = (sigma_a + sigma_b)/2
 *    (additive mixing);
 *  - truncated-shifted LJ per type pair, V = phi(r) - phi(rc_ab) for r < rc_ab,
 *    phi = 4 eps_ab [(sigma_ab/r)^12 - (sigma_ab/r)^6]; rc_ab = 0 selects
 *    2^(1/6) sigma_ab (purely repulsive); only between beads of different
 *    molecules;
 *  - molecules: particles kB .. kB+B-1 (B = beads_per_molecule, particle
 *    indices as passed to md_set_particles) form a linear molecule, with bonds
 *    V = kb (r - r0_ab)^2 between consecutive beads (r0_ab = 0 selects
 *    2^(1/6)(sigma_a + sigma_b)/4) and bends V = ka (theta - theta0)^2 on
 *    consecutive triples, theta the angle at the middle bead between its two
 *    bonds (pi when straight);
 *  - a repulsive wall about the surface centre c, for d = |x - c| - wall_radius
 *    below 2^(1/6) wall_sigma: V = 4 wall_eps [(s/d)^12 - (s/d)^6 + 1/4],
 *    s = wall_sigma; wall_eps = 0: no wall.
 * Requires pair_kind MD_PAIR_LJ; force_fp64 selects the pair terms' class as
 * for plain systems (bonds, bends and the wall are always FP64).  params.rc is
 * not used (the cell grid and lists use the largest rc_ab).  Tables are
 * symmetric: entry [a][b] is used for a <= b. */
#define MD_MAX_TYPES 4
typedef struct md_model {
  int ntypes;                              /* 1 .. MD_MAX_TYPES                     */
  int beads_per_molecule;                  /* 0: no molecules (no bonds, bends or exclusions) */
  double sigma[MD_MAX_TYPES];
  double eps[MD_MAX_TYPES][MD_MAX_TYPES];
  double rc[MD_MAX_TYPES][MD_MAX_TYPES];
  double kb;
  double r0[MD_MAX_TYPES][MD_MAX_TYPES];
  double ka;
  double theta0;
  double wall_eps;
  double wall_sigma;
  double wall_radius;
} md_model;

/* Diagnostics of the current state (computed by md_get_state / md_pool_fetch).
 * K = sum p^2/2m, U = sum_{i<j} V_ij, kT = 2K/N_dof (Section 3.1),
 * gdist_max = max |g|/|n| over constrained particles, nv_max = max |n.p|/(|n| m).
 * After a device error (MD_ENEWTON, MD_ENAN) the state is the one after the
 * failing step (undefined for the failing particle): step = error_step + 1. */
typedef struct md_diag {
  double K;
  double U;
  double ndof;
  double kT;
  double gdist_max;
  double nv_max;
  int64_t step;
  int64_t rebuilds;       /* neighbour-list builds so far                       */
  int newton_iter_max;    /* largest Newton iteration count seen                */
  int nlist_max;          /* largest neighbour count at the last build          */
  int error_index;        /* smallest particle index among those that failed at
                             error_step (the same in any schedule), or -1      */
  int exact_sum_breaches; /* FP32 class: particle-steps whose pair terms left the
                             exact-sum range (a pair closer than about sigma/2);
                             those forces were summed in FP64 in list order, so
                             they may depend on the order of the terms         */
  int64_t error_step;     /* step whose launch found the device error, or -1   */
} md_diag;

/* Counters and GPU times of the work done so far.  step_kernel_ms and
 * rebuild_ms are measured with HIP events recorded on the library's stream
 * around every chunk of step launches and every neighbour-list build. */
typedef struct md_stats {
  int64_t steps;          /* particle-system steps advanced (summed over jobs)  */
  int64_t particle_steps; /* particles x steps advanced                         */
  int64_t step_launches;  /* step-kernel launches                                */
  int64_t chunks;         /* chunk (graph) launches                              */
  int64_t builds;         /* neighbour-list build passes                         */
  double step_kernel_ms;  /* GPU time of the step chunks                         */
  double rebuild_ms;      /* GPU time of the list builds                         */
  double nl_mean;         /* mean neighbours per particle at the last build      */
  int step_variant;       /* FP32-class step-kernel instance in use (md_tune)    */
  int step_waves;         /* its occupancy target, wavefronts per SIMD           */
  int step_halo_lds;      /* its halo entries staged in LDS per 256-slot tile    */
  int list_capacity;      /* neighbour-list capacity, entries per particle       */
  double skin;            /* neighbour-list skin in use (a context; 0 for a pool) */
  double reserved;
} md_stats;

/* ---- one system ------------------------------------------------------------ */
typedef struct md_ctx md_ctx;

/* Create a context on params->device.  *out receives the handle. */
int md_create(const md_params* params, md_ctx** out);

/* Set the constraint g(x) = 0 (kind and prm as listed above, nprm values).
 * Must precede md_set_particles. */
int md_set_surface(md_ctx* ctx, int kind, const double* prm, int nprm);

/* Bead model for the next md_set_particles (see md_model): copies *model and
 * types[0..n) (the bead type of each particle, by particle index); n must equal
 * the particle count given to md_set_particles, and below 2^30.  model = NULL
 * removes the model.  MD_EINVAL for a type outside 0..ntypes-1, a non-positive
 * size or well depth, or negative stiffnesses. */
int md_set_model(md_ctx* ctx, const md_model* model, const uint8_t* types, int64_t n);

/* Set the particles: n positions x and momenta p (host, AoS, n*3 doubles).
 * mass: n masses or NULL (all 1).  constrained: n flags or NULL (all
 * constrained when a surface is set).  fcomb: the combined force f^m of
 * Algorithm S1 carried from an earlier run (n*3, e.g. from md_get_state) or
 * NULL; with NULL the first step uses f^0 = b [F(x^0) - gamma p^0 + f_r^0].
 * step0: the step index m of this state (the noise counter), so that
 * get_state -> set_particles resumes a run exactly.
 * Constrained particles must satisfy |g|/(|n| max(1,|x|_inf)) <= 1e-9 and
 * |n.p|/(|n| max(1,|p|_inf)) <= 1e-9, else MD_EOFFSURF (nothing is projected
 * silently). */
int md_set_particles(md_ctx* ctx, int64_t n, const double* x, const double* p,
                     const double* mass, const uint8_t* constrained, const double* fcomb,
                     int64_t step0);

/* Advance nsteps time steps (Algorithm S1 around Algorithm 1).  Returns after
 * the work is done; MD_ENEWTON / MD_ENAN report a failure, and md_get_state's
 * diagnostics then name the failing step (error_step) and particle.
 * MD_ENOMEM when the neighbour lists need more entries than the list build can
 * hold (its rows live in LDS: a cut-off far beyond the particle spacing), or
 * when device memory for larger lists or halos cannot be allocated. */
int md_step(md_ctx* ctx, int64_t nsteps);

/* md_set_particles with device pointers (e.g. PyTorch tensors on the same
 * device): the arrays have the host variant's layouts, are read on the
 * context's stream (params.stream) before the call returns, and are not
 * retained; the caller owns them.  Same checks and errors as md_set_particles;
 * MD_EHIP if a copy fails. */
int md_set_particles_dev(md_ctx* ctx, int64_t n, const double* x, const double* p, const double* mass,
                         const uint8_t* constrained, const double* fcomb, int64_t step0);

/* Copy the state at the current step m: positions x^m, momenta p^m (tangent),
 * optionally the combined force f^m (fcomb, n*3), the step index and
 * diagnostics.  Any pointer may be NULL. */
int md_get_state(md_ctx* ctx, double* x, double* p, double* fcomb, int64_t* step, md_diag* diag);

/* md_get_state into device pointers (x, p, fcomb: n*3 doubles each, caller
 * owned, any may be NULL): filled by device-to-device copies on the context's
 * stream, complete when the call returns; step and diag are host pointers. */
int md_get_state_dev(md_ctx* ctx, double* x, double* p, double* fcomb, int64_t* step, md_diag* diag);

/* md_get_state_dev for callers that cannot allocate memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): same
 * arguments, results and bits as md_get_state_dev, but the call allocates and
 * frees no device or pinned host memory.  The diagnostics reduction works in a
 * static device array of 8224 bytes (the partials of at most 256 blocks and
 * the four sums; every job size fits), one per device, held until the
 * process ends; calls on one device share it, so calls that overlap on one
 * device (several contexts on different streams) race.  MD_ENOMEM if the
 * call would need larger neighbour-list capacity than the context holds (a
 * list build is due and the lists outgrew it); md_get_state_dev grows it. */
int md_get_state_dev_noalloc(md_ctx* ctx, double* x, double* p, double* fcomb, int64_t* step, md_diag* diag);

/* Counters and event-timed GPU work of this context (see md_stats). */
int md_get_stats(md_ctx* ctx, md_stats* stats);

/* Autotune the live system: first the FP32-class step-kernel instance (the
 * compiled variants differ in occupancy target and in how many halo entries
 * a tile stages in LDS; FP64-class and bead-model jobs have one instance),
 * then the neighbour-list skin (skins[0..nskins), or a built-in set
 * {0.2, 0.3, 0.4, 0.5, 0.6, 0.8} sigma when skins is NULL).  Each trial
 * runs one step (which takes the list build a new choice may force) and then
 * trial_steps steps scored by GPU time per step (HIP events, so graph capture
 * does not count): an instance by its step kernels alone, twice (all
 * instances in turn, then in reverse order; the faster trial counts), a skin
 * by step kernels and list builds together.  The fastest instance and skin
 * stay in effect and md_get_stats reports them.  The system really advances
 * (2 * instances + skins) * (trial_steps + 1) steps: results
 * depend on neither choice, so the trajectory is the one md_step would have
 * produced.  best_skin and best_us_per_step (GPU microseconds per step) may be
 * NULL.  Candidate skins whose cell grid does not fit the context's memory are
 * skipped. */
int md_tune(md_ctx* ctx, int trial_steps, const double* skins, int nskins, double* best_skin,
            double* best_us_per_step);

/* Release every resource of the context. */
void md_destroy(md_ctx* ctx);

/* Human-readable name of a status code. */
const char* md_strerror(int code);

/* ---- many independent systems resident at once (batched / serving) --------
 * A pool keeps many jobs' state on the device and advances all of them with
 * one set of launches per step; jobs of any size and surface share the
 * launches.  Each job's result equals the result of running it alone. */
typedef struct md_pool md_pool;

typedef struct md_job_desc {
  md_params params;       /* device and stream are ignored (the pool's are used) */
  int surface_kind;
  double surface_prm[MD_SURF_MAXPRM];
  int64_t n;
  const double* x;        /* host, n*3 */
  const double* p;        /* host, n*3 */
  const double* mass;     /* host, n or NULL */
  const uint8_t* constrained; /* host, n or NULL */
  int64_t step0;
  int64_t nsteps;         /* steps to run before the job is done */
  const md_model* model;  /* bead model (see md_model) or NULL; params.rc is then not used */
  const uint8_t* types;   /* host, n bead types when model is set */
} md_job_desc;

/* Device bytes one job of n particles needs (for admission by HBM budget). */
size_t md_job_footprint(int64_t n, int surface_kind, const double* surface_prm,
                        const md_params* params);

/* Create a pool that may use up to hbm_budget_bytes of device memory for job
 * state and up to max_jobs resident jobs. */
int md_pool_create(size_t hbm_budget_bytes, int max_jobs, int device, void* stream,
                   md_pool** out);

/* Admit a job: copies its state to the device.  MD_EAGAIN when the budget or
 * the job slots are exhausted (retry after releasing finished jobs). */
int md_pool_admit(md_pool* pool, const md_job_desc* job, int* job_id);

/* Advance every resident, unfinished job by up to steps_chunk steps. */
int md_pool_run(md_pool* pool, int steps_chunk);

/* Enqueue one chunk of up to steps_chunk steps (at most 32) for every
 * resident, unfinished job and return without waiting for it, so that the
 * caller can admit jobs (md_pool_admit) while the chunk runs: their uploads go
 * to slots the chunk does not touch and follow it on the stream.  The chunk is
 * completed (waited for, its steps counted) by the next md_pool_launch,
 * md_pool_run, md_pool_poll, md_pool_fetch, md_pool_release or
 * md_pool_destroy; md_pool_get_stats and md_pool_usage report completed
 * chunks only. */
int md_pool_launch(md_pool* pool, int steps_chunk);

/* List jobs that have finished (or failed) and have not been fetched yet:
 * up to cap ids into done_ids, count into *ndone. */
int md_pool_poll(md_pool* pool, int* done_ids, int cap, int* ndone);

/* Copy a job's state (x, p: n*3; diag optional).  Returns the job's own status
 * (MD_OK, or the device error that stopped it). */
int md_pool_fetch(md_pool* pool, int job_id, double* x, double* p, md_diag* diag);

/* md_pool_fetch for n jobs at once (job_ids[0..n)): x[q], p[q] receive job
 * job_ids[q]'s state (host, n_q*3 each; either array or entry may be NULL),
 * diag[q] its diagnostics and status[q] its own status (MD_ENOTFOUND for an
 * unknown id); diag and status may be NULL.  The jobs' finish work runs as
 * one launch per force class over all their tiles, their diagnostics as one
 * pair of reductions (the same pieces and trees as md_pool_fetch, so the same
 * bits), and their results come back in one copy, waited for once. */
int md_pool_fetch_many(md_pool* pool, const int* job_ids, int n, double* const* x, double* const* p, md_diag* diag,
                       int* status);

/* Free a job's slots and memory. */
int md_pool_release(md_pool* pool, int job_id);

/* Number of resident jobs and of particles they hold. */
int md_pool_usage(md_pool* pool, int* jobs, int64_t* particles, size_t* bytes);

/* Counters and event-timed GPU work of this pool (see md_stats). */
int md_pool_get_stats(md_pool* pool, md_stats* stats);

void md_pool_destroy(md_pool* pool);

#ifdef __cplusplus
}
#endif
#endif
