/*
 * fempic.h - C ABI of the MI355X (gfx950) higher-order charge-conserving
 * electromagnetic finite-element particle-in-cell hot path.
 *
 * Method: Crawford, Ramachandran, O'Connor, Luginsland, Shanker, "Higher Order
 * Charge Conserving Electromagnetic Finite Element Particle in Cell Method"
 * (arXiv 2111.12411).  Section references below are to that paper.
 *
 * Conventions for every function:
 *   - returns FEMPIC_OK (0) or a negative fempic status;
 *   - no C++ exception crosses the boundary; the message of the last failure on
 *     the calling thread is returned by fempic_last_error();
 *   - every pointer argument is a HOST pointer; input arrays are copied before
 *     the call returns and are never retained;
 *   - output arrays are caller-owned with explicit lengths (FEMPIC_EINVAL if a
 *     length is too short); out-parameters are written only on FEMPIC_OK;
 *   - handles are opaque, owned by the caller, released by the matching
 *     *_destroy; destroying NULL is a no-op;
 *   - device-side failures (crossing cap, solver failure, HIP errors) are sticky
 *     for a run and are reported by the next call that synchronises it.
 * Units are SI.  Fields are E in V/m and B in T; the W1 coefficients e_i have
 * units V and the W2 coefficients b_l units Wb.
 */
#ifndef FEMPIC_H
#define FEMPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define FEMPIC_OK 0
#define FEMPIC_EINVAL (-1)   /* bad argument */
#define FEMPIC_ENOMEM (-2)   /* host or device allocation failed / over budget */
#define FEMPIC_EMESH (-3)    /* degenerate or non-manifold mesh */
#define FEMPIC_EOUTSIDE (-4) /* a particle lies outside the mesh */
#define FEMPIC_ECROSS (-5)   /* more than 64 tet crossings in one step */
#define FEMPIC_ESOLVE (-6)   /* linear solver did not reach its tolerance */
#define FEMPIC_EDEVICE (-7)  /* HIP runtime error */
#define FEMPIC_EAGAIN (-8)   /* poll: result not ready */
#define FEMPIC_EBUSY (-9)    /* server: no capacity / run busy */

#define FEMPIC_FP64 0  /* every step of the path in FP64 */
#define FEMPIC_MIXED 1 /* FP32 gather/push and FP32 inner solve; FP64 positions,
                          tracking, deposit, residuals and refinement */

#define FEMPIC_PUSH_AB4 0   /* fourth-order Adams-Bashforth push, quartic path (Sec. III-B) */
#define FEMPIC_PUSH_BORIS 1 /* Boris leapfrog, straight path (the push is de-linked from
                               the current mapping, Sec. III-B); velocities are v^{n-1/2} */

#define FEMPIC_FIELD_PEC 0    /* walls are perfect conductors: n x E = 0 (Sec. II, Dirichlet
                                 condition), the wall W1 DoFs are not unknowns */
#define FEMPIC_FIELD_ABSORB 1 /* first-order absorbing walls: the impedance condition of
                                 Sec. II with Psi_I = 0 and the free-space admittance
                                 Y = 1/eta0; every W1 DoF is an unknown and the surface
                                 impedance matrix of Sec. III-A,
                                 [*I]_ij = Y int_walls (n x W1_i) . (n x W1_j) dS,
                                 enters Ampere's law: *eps de/dt + *I e = K^T *nu b - dg/dt */

#define FEMPIC_REFLECT 0 /* particles reflect specularly at PEC walls */
#define FEMPIC_ABSORB 1  /* a particle that reaches a wall deposits its current up to
                            the wall and leaves the run there */

typedef struct fempic_mesh_s *fempic_mesh;
typedef struct fempic_run_s *fempic_run;
typedef struct fempic_server_s *fempic_server;

/* Text of the last failure on this thread ("" if none). */
const char *fempic_last_error(void);

/* ------------------------------------------------------------------ mesh
 * Tetrahedral complex {nodes, edges, faces, tets} (Sec. III-A).  Every boundary
 * face is a PEC wall: n x E = 0 (Sec. II, Dirichlet condition).  `order` is the
 * basis order k of the Appendix (1 = classic Whitney, 2 = second order).
 * Field DoFs (Sec. III-A, Appendix): E in the order-k edge (W1) space,
 * B in the order-k face (W2) space; charge is measured with the order-k nodal
 * (W0) functions.
 *
 * fempic_mesh_create: xyz is [n_vert][3] doubles; tet4 is [n_tet][4] vertex ids
 *   (any order; they are sorted internally).  EMESH if a tet has zero volume, a
 *   face is shared by more than two tets, or an id is out of range.
 * fempic_mesh_create_cube: the N^3 Kuhn-split cube [0,L]^3, 6 N^3 tets
 *   (tet 6h+p of hex h = i + N(j + N l) follows axis permutation p in
 *   lexicographic order).  1 <= N <= 126 (fewer than 2^21 vertices); EINVAL
 *   otherwise, before anything of that size is allocated.
 * fempic_mesh_destroy may be called while runs made on the mesh still exist:
 *   each run keeps what it needs of the mesh until it is destroyed.
 *
 * DoF numbering used by every exported vector (natural order):
 *   edges / faces are sorted vertex tuples numbered lexicographically;
 *   W1 k=1: edge id.  k=2: 2*edge + {0: (3 l_lo - 1) W, 1: (3 l_hi - 1) W},
 *           2*E + 2*face + {0: 3 l_c W_ab, 1: 3 l_b W_ac};
 *   W2 k=1: face id.  k=2: 3*face + x -> (4 l_x - 1) W_abc (x = a,b,c),
 *           3*F + 3*tet + f -> 4 l_d W_f (local faces f = 0,1,2);
 *   W0 k=1: vertex id.  k=2: vertex id, then n_vert + edge (2 l_a l_b).
 */
int32_t fempic_mesh_create(const double *xyz, int64_t n_vert, const int64_t *tet4, int64_t n_tet,
                           int32_t order, fempic_mesh *out);
int32_t fempic_mesh_create_cube(int32_t N, double L, int32_t order, fempic_mesh *out);
int32_t fempic_mesh_destroy(fempic_mesh mesh);

typedef struct {
    int64_t n_vert, n_edge, n_face, n_tet;
    int64_t n1, n1_int; /* W1 DoFs: all / off the walls (the unknowns with PEC walls;
                           with absorbing walls all n1 are)                  */
    int64_t n2;         /* W2 DoFs                                           */
    int64_t n0, n0_int; /* W0 DoFs: all / interior (Gauss-law check rows)    */
    int32_t order, n1_loc, n2_loc, n0_loc;
    /* Explicit (leapfrog) time-step limit bound 2/sqrt(max_T lmax(M1_T^-1 S_T)),
       S_T the element curl-curl matrix; the implicit scheme has no such limit. */
    double dt_cfl;
} fempic_mesh_info_t;
int32_t fempic_mesh_info(fempic_mesh mesh, fempic_mesh_info_t *out);

/* ------------------------------------------------------------------- run
 * A run owns the device state of one simulation on the current HIP device:
 * e, b, accumulated current moments, particles, operators, workspace.
 * The field update is Newmark-beta (Sec. III-B, eq. (maxnmb)) with parameters
 * gamma, beta: 1/2, 1/4 (the paper's choice: the trapezoidal rule, two-level
 * form) or any other unconditionally stable pair, 2 beta >= gamma >= 1/2, such
 * as backward difference (1.5, 1) or Galerkin (1.5, 0.8) of Sec. IV-D, in the
 * three-level form, which starts from a field history at rest (the fields
 * before the first step equal those at load or fields_set); EINVAL otherwise.
 * Both keep Gauss's law: the current enters with the time stencil of the
 * mass term.  `hip_stream` may be NULL (the run
 * creates its own default-priority stream).  pcg_rtol is the relative residual
 * the field solve must reach (ESOLVE otherwise); the residual is evaluated in
 * double-double, against a right-hand side formed in double-double, and the
 * solve is refined on to a relative residual of 1e-17 when pcg_rtol is larger,
 * so that the solve adds no drift to the Gauss residual over long runs.
 * pcg_maxit caps the iterations of each (inner) PCG solve.
 * spill_slots is reserved and ignored: the buffer of path segments outside the
 * particle's home tet grows on demand (a step that overflows it is redone after
 * the buffer doubles; ENOMEM if that keeps failing).  A path that crosses more
 * than 64 faces in one step fails the step with ECROSS.
 */
typedef struct {
    int32_t precision;   /* FEMPIC_FP64 or FEMPIC_MIXED */
    double dt;           /* time step [s] */
    double gamma, beta;  /* Newmark-beta: 0.5, 0.25, or 2 beta >= gamma >= 0.5 */
    double pcg_rtol;     /* e.g. 1e-14 */
    int32_t pcg_maxit;   /* e.g. 5000 */
    int32_t particle_bc; /* FEMPIC_REFLECT or FEMPIC_ABSORB (other values: EINVAL).
                            Both conserve charge on the interior nodes: the
                            interior W0 functions vanish on the walls */
    int32_t spill_slots; /* reserved, ignored */
    int32_t gauss_every; /* 0: off; k > 0: fempic_step evaluates the Gauss-law
                            residuals (fempic_gauss_residual) after every step
                            whose count is a multiple of k, into
                            fempic_stats_t.gauss (one device wait each) */
    int32_t pusher;      /* FEMPIC_PUSH_AB4 (0) or FEMPIC_PUSH_BORIS; with Boris the
                            loaded velocity is taken as v^{-1/2}, the step moves
                            along the straight path r^n + s dt v^{n+1/2} and deposits
                            its exact path integral, and fempic_history_get is EINVAL */
    int32_t field_bc;    /* FEMPIC_FIELD_PEC (0) or FEMPIC_FIELD_ABSORB; absorbing walls
                            need gamma, beta = 1/2, 1/4 (EINVAL otherwise) and are
                            stepped by the trapezoidal rule like the rest:
                            (A + dt/2 *I)(e^{n+1} - e^n) = dt K^T *nu (b^n - dt/2 K e^n)
                            - dt *I e^n - (g^{n+1} - g^n).  Gauss's law on the interior
                            nodes is unchanged (*I G = 0 there) */
} fempic_params;

int32_t fempic_run_create(fempic_mesh mesh, const fempic_params *params, void *hip_stream, fempic_run *out);
int32_t fempic_run_destroy(fempic_run run);

/* Load n particles of one species (charge q [C], mass m [kg], macro weight w):
 * pos, vel are [n][3].  Locates every particle (EOUTSIDE if one is outside),
 * and starts the 4th-order Adams-Bashforth history from the current fields:
 * a^{-j} = a^0, v^{-j} = v^0 - j dt a^0 (j = 1..3).  Records the nodal charge
 * rho~^0 as the reference of the Gauss-law check.  Replaces earlier particles.
 * EINVAL for a non-finite position or velocity (nothing reaches the device). */
int32_t fempic_particles_load(fempic_run run, const double *pos, const double *vel, int64_t n, double q, double m,
                              double w);

/* Append n particles of the loaded species (pos, vel [n][3], ids after the
 * existing ones), between steps: a beam source (Table III injects a few
 * particles every step).  Each is located (EOUTSIDE if outside the mesh) and
 * started like a loaded particle.  Their charge enters the run here rather than
 * through a current, so it joins the Gauss check's reference rho~^0, as the
 * charge present at load does; injected on a wall, where the interior W0
 * functions vanish, it adds nothing there.  The buffers grow by half again when
 * they are full; the next step sorts the particles again.  EINVAL before a
 * load, for a non-finite position or velocity, or for a NULL array with n > 0. */
int32_t fempic_particles_inject(fempic_run run, const double *pos, const double *vel, int64_t n);

/* Advance n_steps PIC steps (Sec. III, PIC cycle; Sec. III-B) on the run's
 * stream.  Per step: particles in tet order (a sort after load; each step then
 * orders them for the next from its own exit queue and spill records); gather
 * E, B at r^n; AB4 push along the quartic path; track across tets (PEC walls
 * reflect); deposit g^{n+1} - g^n with the exact path integral of the W1 basis;
 * solve A (e^{n+1} - e^n) = dt K^T *nu (b^n - dt/2 K e^n) - (g^{n+1} - g^n),
 * A = *eps + dt^2/4 K^T *nu K, by PCG (Jacobi, or 2x2 block Jacobi at order 2;
 * FP32 PCG inside FP64 refinement in mixed precision);
 * b^{n+1} = b^n - dt/2 K (e^n + e^{n+1}) (gamma, beta = 1/2, 1/4; other pairs take
 * the three-level form with A = *eps + (beta/gamma)^2 dt^2 K^T *nu K and the
 * previous step's fields and current).  The call waits on the device once per
 * particle phase (queue and spill counts, error flags) and every 8 PCG
 * iterations; the last step's final field updates may still be queued when it
 * returns (fempic_sync waits for them). */
int32_t fempic_step(fempic_run run, int32_t n_steps);

/* Wait for the run's queued work; reports sticky device failures. */
int32_t fempic_sync(fempic_run run);

/* Gauss's law check (Sec. II, Gauss laws; Sec. IV-D): on the interior nodal DoFs
 * (the running sums e and g are kept with compensated summation, and the
 * products below are evaluated in double-double, so the residuals measure the
 * scheme, not the rounding of FP64 running sums),
 *   out[0] = R_G = |G^T *eps e + (rho~^n - rho~^0)| / |rho~^n - rho~^0|,
 *   out[1] = R_C = |G^T g - (rho~^n - rho~^0)| / ...  (deposit only),
 *   out[2] = R_S = |G^T (*eps e + g)| / ...          (solve only),
 * with rho~_j = q w sum_p W0_j(r_p), g the accumulated current moments and G
 * the gradient matrix (grad W0_j = sum_i G_ij W1_i; its entries are thirds at
 * order 2, so the check multiplies by 3 G, whose entries are integers, and
 * divides the products by 3).  Synchronises. */
int32_t fempic_gauss_residual(fempic_run run, double out[3]);

/* fempic_gauss_residual without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same values, bit for bit, as
 * fempic_gauss_residual.  Its intermediates (per-tet partial charges, the
 * nodal vectors, reduction partials) live in a static device array of the
 * library, 96 MiB on every device it runs on, held until the process ends.
 * Nothing is allocated: no hipMalloc, no installed allocator, no library
 * routine that allocates.  EINVAL when the run's mesh needs more scratch than
 * that (8 n_tet n0_loc + 24 n0_int + 16 n1_int bytes, n1 in place of n1_int
 * with absorbing walls, and 64 KiB: up to about the
 * 40^3 cube at order 2).  Every call on a device shares that device's array, so
 * calls that overlap on one device (runs on different streams or threads) race
 * and must be serialised by the caller.  Synchronises the run's stream. */
int32_t fempic_gauss_residual_noalloc(fempic_run run, double out[3]);

/* Copy fields out / in (natural numbering; e has n1 entries, b has n2).
 * fields_set zeroes e on PEC walls (absorbing walls keep it); EINVAL for a
 * non-finite coefficient. */
int32_t fempic_fields_get(fempic_run run, double *e, int64_t ne, double *b, int64_t nb);
int32_t fempic_fields_set(fempic_run run, const double *e, int64_t ne, const double *b, int64_t nb);

/* Current moments deposited by the last step, g^{n+1} - g^n (natural numbering,
 * n1 entries; zero on the walls). */
int32_t fempic_deposit_get(fempic_run run, double *dg, int64_t n);

/* The matrix of the implicit field update (Sec. III-A, eq. (maxwell_semi), in
 * the Newmark-beta form of Sec. III-B: A = *eps + (beta/gamma)^2 dt^2 K^T *nu K,
 * plus dt/2 *I with absorbing walls) applied to W1 coefficients: y = A x over
 * the unknown W1 DoFs.
 * x and y have n >= n1 entries in the natural numbering (as fields_get's e);
 * entries of x on PEC walls are ignored and those of y are set to 0.
 * form: FEMPIC_OP_ASSEMBLED, the assembled FP64 matrix (the one the solve's
 * residuals use), or FEMPIC_OP_ITERATION, the form its PCG iterations apply:
 * in the iterations' precision (FP32 for the inner solve of mixed precision)
 * and, with PEC walls, tet by tet from the geometry instead of the assembled
 * matrix (unless FEMPIC_MATFREE=0 was set when the run was made).  Host
 * buffers; synchronous.  EINVAL for a short buffer, a non-finite x or an
 * unknown form. */
#define FEMPIC_OP_ASSEMBLED 0
#define FEMPIC_OP_ITERATION 1
int32_t fempic_field_matvec(fempic_run run, const double *x, double *y, int64_t n, int32_t form);

/* Nodal charge measured with the order-k W0 functions (Sec. III-A: charge on
 * the primal nodes; Sec. IV-D, the Gauss check): rho[j] = q w sum_p W0_j(r_p)
 * at the current positions, and rho0 the reference taken at load (natural W0
 * numbering, n >= n0 entries each; 0 on W0 DoFs on the walls, which the check
 * leaves out).  Either pointer may be NULL.  Synchronises; EINVAL before a load. */
int32_t fempic_rho_get(fempic_run run, double *rho, double *rho0, int64_t n);

/* Impressed magnetic flux density (Sec. III-C, eq. (conB); Tables I and II): an
 * external B (magnets, lenses) that pushes the particles but does not enter
 * Ampere's law.
 * fempic_impressed_points writes the points at which the caller samples B:
 * n1d^3 per tet (a collapsed Gauss-Legendre rule, 1 <= n1d <= 8), tet-major,
 * xyz [n_tet * n1d^3][3]; n >= n_tet * n1d^3 points, else EINVAL.
 * fempic_impressed_set takes B at those points (B [n_tet * n1d^3][3], tesla,
 * same n1d), forms the moments f_l = <W2_l, B / mu0> and projects: with
 * constrained = 0, *nu b = f; with constrained = 1, b is the *nu-orthogonal
 * projection onto the faces whose discrete divergence vanishes (the solution of
 * the saddle-point system of eq. (conB); computed as b = K a over the curl of
 * every edge function, which spans those faces on a simply connected mesh, so
 * div b is zero to rounding).  The run keeps b as its impressed field from then
 * on (also through checkpoints): the gather uses b_self + b.  b_out (NULL, or
 * >= n2 entries) receives b in natural face numbering.  EINVAL on bad sizes or a
 * non-finite B; ESOLVE if a projection solve does not converge. */
int32_t fempic_impressed_points(fempic_mesh mesh, int32_t n1d, double *xyz, int64_t n);
int32_t fempic_impressed_set(fempic_run run, const double *B, int64_t n, int32_t n1d, int32_t constrained,
                             double *b_out, int64_t nb);

/* Particle state in load order: pos, vel [n][3]; tet [n] (any may be NULL);
 * n >= the number loaded.  A particle absorbed at a wall has tet -1 and NaN
 * position and velocity.  The run holds each position as the barycentric
 * coordinates of the particle in its tet (taken over exactly from tet to tet
 * and from step to step, which keeps the deposit's charge continuity free of
 * the rounding of the tets' barycentric maps); pos is computed from them,
 * x_0 + sum_m l_m (x_m - x_0) over the tet's vertices x_m. */
int32_t fempic_particles_get(fempic_run run, double *pos, double *vel, int64_t *tet, int64_t n);

/* Full AB4 history in load order: vh, ah are [n][3][3] = v^{n-1..n-3}, a^{n-1..n-3}
 * (NaN for absorbed particles). */
int32_t fempic_history_get(fempic_run run, double *vh, double *ah, int64_t n);

/* ------------------------------------------------------------- checkpoint
 * fempic_run_save writes the run's state to the file at `path` (created or
 * replaced): the particles (positions as barycentric coordinates in their
 * tets), with their AB4 velocity and acceleration histories
 * in the run's storage precision and in the order the next step takes them;
 * e, b, the accumulated current moments and the reference charge of the
 * Gauss-law check; the three-level scheme's previous fields and current; the
 * species and the step counter.  Synchronises; the run
 * itself is unchanged.
 * fempic_run_load reads such a file into a run created on the same mesh (same
 * sizes and order) with the same precision, dt, gamma and beta, replacing its particles and
 * fields and clearing a sticky failure.  The steps a run takes after the load
 * equal, bit for bit, those the saved run takes after the save.
 * EINVAL: null path; a file that cannot be opened, read or written; a file of
 * another mesh, precision or dt; a damaged file (checksum, particle ids, tets
 * outside the mesh, non-finite positions, velocities, histories or fields).  The
 * format is this library's own, in native byte order. */
int32_t fempic_run_save(fempic_run run, const char *path);
int32_t fempic_run_load(fempic_run run, const char *path);

/* Step log: after every step of fempic_step, append one JSON object on a line
 * of its own to the file at `path` and flush it: {"step", "n_particles",
 * "particle_ms", "particle_kernel_ms", "continue_kernel_ms", "field_ms",
 * "pcg_iters", "pcg_relres", "crossings", "reflections", "absorbed", "spills"} of that step
 * (fields as in fempic_stats_t, for the one step), plus "gauss": [R_G, R_C, R_S]
 * on the steps params.gauss_every evaluates them.  Non-finite values are
 * written as null.  NULL or "" stops logging.  EINVAL if the file cannot be
 * opened; a failed write fails the step with EINVAL. */
int32_t fempic_run_set_log(fempic_run run, const char *path);

/* -------------------------------------------------------------- allocator
 * Routes the device buffers that runs and servers make from now on through
 * the caller's allocator (a framework's caching allocator, say):
 * alloc(bytes, ctx) returns memory of the current HIP device, at least `bytes`
 * long and 256-byte aligned, or NULL (the call that needed it fails with
 * ENOMEM); release(ptr, ctx) takes it back.  The library synchronises the
 * device before each release, so no queued work uses the memory when the
 * caller gets it back.  A buffer keeps the allocator that made it, so the two
 * functions and ctx must stay valid while any of their buffers exists.  They
 * may be called on any thread the library runs on (a server steps its runs on
 * threads of its own).  Both NULL restores hipMalloc/hipFree; one NULL is
 * EINVAL.  Process-wide; pinned host staging memory is not affected. */
typedef void *(*fempic_alloc_fn)(size_t bytes, void *ctx);
typedef void (*fempic_free_fn)(void *ptr, void *ctx);
int32_t fempic_set_allocator(fempic_alloc_fn alloc, fempic_free_fn release, void *ctx);

/* Per-run statistics of the last fempic_step call. */
typedef struct {
    int64_t steps;            /* steps taken by this run */
    int64_t n_particles;      /* particles in the run now */
    int64_t n_loaded;         /* particles loaded (n_particles + those absorbed since) */
    int64_t absorbed;         /* last step: particles absorbed at a wall */
    int64_t absorbed_total;   /* since load */
    double particle_ms;       /* last call: device time of ordering + particle + deposit reduction, ms */
    double particle_kernel_ms;/* last call: device time of the particle kernel (gather, push, first segment), ms;
                                 steps whose particle phase replayed a graph do not count (phase_replays) */
    double continue_kernel_ms;/* last call: device time of the kernel that tracks paths leaving their tet, ms
                                 (the same steps only) */
    double field_ms;          /* last call: device time of the field update, ms */
    int32_t pcg_iters;        /* last step's PCG iterations (inner iterations in mixed mode) */
    double pcg_relres;        /* last step's final FP64 relative residual */
    int64_t crossings;        /* last step: face crossings (all particles) */
    int64_t reflections;      /* last step: wall reflections */
    int64_t spills;           /* last step: segments outside the particle's tet */
    double gauss[3];          /* R_G, R_C, R_S at step gauss_step (params.gauss_every) */
    int64_t gauss_step;       /* step count of that evaluation; 0: none yet */
    int64_t a_rows, a_nnz;    /* system matrix A of the field solve: rows (interior W1 DoFs), nonzeros */
    int64_t device_bytes;     /* device memory the run holds now */
    int64_t device_peak_bytes;/* and the most it has held */
    int64_t phase_replays;    /* last call: steps whose particle phase replayed a captured HIP graph (runs
                                 of a server, or FEMPIC_PHASE_GRAPHS=1 in the environment) */
    int32_t field_op;         /* the operator the PCG iterations apply: 0 the assembled matrix, 1 tet by
                                 tet, 2 tet by tet with the two DoFs of each edge and face taken together */
    int64_t a_inc;            /* (tet, local position) incidences of A's rows: the products that the
                                 tet-by-tet operator sums */
} fempic_stats_t;
int32_t fempic_stats(fempic_run run, fempic_stats_t *out);

/* Device bytes a run needs: operators, fields, solver vectors, particle state
 * (two buffers), sort, exit queue and the initial buffer of segments outside
 * their home tet (1.5 n records).  A run whose crossings need a larger buffer
 * grows it during a step.  Operator sizes are bounded per row by what Kuhn
 * cubes reach (order 1: 17 nonzeros per row of A, order 2: 46); a mesh of much
 * higher vertex valence can need more.
 * fempic_footprint: for a mesh of n_tet tets whose entity counts are those of a
 *   Kuhn cube with 6 N^3 = n_tet (exact for such cubes).  EINVAL for order not
 *   1|2, n_tet < 1, n_particles < 0 or an unknown precision.
 * fempic_footprint_mesh: the same from the counts of a built mesh.
 * Both assume PEC walls; with absorbing walls (params.field_bc) the wall W1
 * DoFs are unknowns too and the run holds their solver vectors and the surface
 * impedance matrix as well (the server budgets that). */
int32_t fempic_footprint(int32_t order, int64_t n_tet, int64_t n_particles, int32_t precision, size_t *bytes);
int32_t fempic_footprint_mesh(fempic_mesh mesh, int64_t n_particles, int32_t precision, size_t *bytes);

/* ----------------------------------------------------------- serving
 * Continuous batching of independent runs on one GPU.  A server owns a worker
 * thread.  Jobs are admitted in arrival order when their device footprint
 * (fempic_footprint of the cube) fits the HBM budget and a slot is free; a run
 * may not hold more device memory than it was admitted with (a step that would
 * need more, to grow its buffer of segments outside their home tet, fails the
 * job with ENOMEM).  Steps of resident runs interleave on
 * separate streams, and a finished run frees its memory for the next job.
 * fempic_submit copies the job's inputs and returns a ticket at once
 * (ENOMEM if the job could never fit the budget).  fempic_poll returns EAGAIN
 * until the job is done, then fills *out; result arrays stay owned by the server
 * until fempic_result_release.
 */
typedef struct {
    size_t hbm_budget; /* bytes of device memory the server may use */
    int32_t max_slots; /* runs resident at once */
} fempic_server_params;

typedef struct {
    int32_t N;          /* Kuhn cube N^3 */
    double L;
    int32_t order;
    fempic_params params;
    const double *pos, *vel; /* [n][3] */
    int64_t n;
    double q, m, w;
    int32_t n_steps;
} fempic_job;

typedef struct {
    int32_t status;       /* job status (FEMPIC_OK or the failure) */
    int64_t n1, n2, n;    /* lengths of e, b and particles */
    const double *e, *b;  /* final fields (natural numbering) */
    const double *pos, *vel;
    double gauss[3];      /* R_G, R_C, R_S at the end */
    double queue_ms;      /* submit -> admission */
    double run_ms;        /* admission -> done */
    const double *step_done_ms; /* [n_steps] completion time of each step, ms since admission */
    int32_t n_steps;
    const char *message;  /* why the job failed ("" when it did not); owned like the arrays */
} fempic_job_result;

int32_t fempic_server_create(const fempic_server_params *params, fempic_server *out);
int32_t fempic_server_destroy(fempic_server server);
int32_t fempic_submit(fempic_server server, const fempic_job *job, int64_t *ticket);
int32_t fempic_poll(fempic_server server, int64_t ticket, fempic_job_result *out);
int32_t fempic_result_release(fempic_server server, int64_t ticket);

#ifdef __cplusplus
}
#endif
#endif /* FEMPIC_H */
