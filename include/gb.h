/*
 * gb.h -- C ABI of the MI355X library for the ALE nodal DG Galerkin-Boltzmann
 * hot path (arXiv 2607.00199, "A High-Order ALE DG Method for the Boltzmann
 * Equation in Nearly Incompressible Flows").
 *
 * What the library computes
 *   The semi-discrete ALE form of the Galerkin-Boltzmann moment system
 *   (Section 2, eq. ale_bns; Section 3, eq. semi_discrete_form) on a moving
 *   mesh of straight-sided simplices (triangles: 6 fields, tetrahedra: 10
 *   fields), advanced by the four-stage semi-analytic Runge-Kutta method
 *   (Section 4) with the geometric factors rebuilt from the vertex positions
 *   at every stage (Section 5).  Every step of that path runs in HIP kernels
 *   on one gfx950 GPU.
 *
 * Conventions shared by all calls
 *   - Every call returns gb_status; GB_OK is 0.  On any other status,
 *     gb_last_error() returns a thread-local message.  No C++ exception
 *     crosses this interface.
 *   - Host arrays are plain C arrays owned by the caller; the library copies
 *     what it needs and never keeps a host pointer.
 *   - Field layout of every state array is [K][NF][Np] (element, field,
 *     node), FP64 on the host.  Field order: rho, m_x, m_y, S_xy, S_xx/sqrt2,
 *     S_yy/sqrt2 in 2D (the q1..q6 of Section 2, with rho u = c m_x); in 3D
 *     rho, m_x, m_y, m_z, S_xy, S_xz, S_yz, S_xx/sqrt2, S_yy/sqrt2, S_zz/sqrt2.
 *   - Node order inside an element is the lattice order of the Warp & Blend
 *     nodes (Section 3): s-rows outer, r inner (3D: t, s, r).
 *   - Faces: triangle (v0,v1), (v1,v2), (v2,v0); tetrahedron (v0,v1,v2),
 *     (v0,v1,v3), (v1,v2,v3), (v0,v2,v3).
 *   - Handles are single-threaded: one context drives one HIP stream.
 *   - Kernel faults inside the hot path (an element with J <= 0, a
 *     non-positive density or a NaN) are latched on the device and reported
 *     as GB_ERR_MESH / GB_ERR_NONPHYSICAL by the next synchronising call.
 */
#ifndef GB_H
#define GB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GB_OK = 0,
    GB_ERR_ARG = 1,          /* invalid argument (null pointer, size, range)      */
    GB_ERR_MESH = 2,         /* J <= 0, unmatched face, inconsistent period       */
    GB_ERR_OOM = 3,          /* device allocation failed                          */
    GB_ERR_DEVICE = 4,       /* HIP runtime error                                 */
    GB_ERR_NONPHYSICAL = 5,  /* latched on the device: density <= 0 or NaN        */
    GB_ERR_STATE = 6,        /* call out of order (e.g. stepping without a state) */
    GB_ERR_UNSUPPORTED = 7,  /* (dim, N, precision) combination not built         */
    GB_ERR_BUSY = 8          /* admission refused: over the batch's free budget   */
} gb_status;

typedef enum { GB_FP64 = 0, GB_FP32 = 1 } gb_precision;

/* Upwinding of the surface flux (Section 3, eq. upwind_flux).
 * SPLIT: the stationary part A.n and the ALE part w.n are upwinded
 *        separately, as the paper writes it.
 * RELATIVE: the characteristic speeds c*lambda_k - w.n are upwinded together. */
typedef enum { GB_FLUX_SPLIT = 0, GB_FLUX_RELATIVE = 1 } gb_flux_mode;

/* Face tags for gb_mesh_create (face_tag may be NULL: every unmatched face is
 * then an error).  Interior and periodic faces are found automatically. */
enum { GB_FACE_INTERIOR = 0, GB_FACE_WALL = 1, GB_FACE_FARFIELD = 2 };

/* Prescribed mesh motions (Section 5: the grid velocity is given at the
 * vertices and interpolated linearly; vertices move with classical RK4).
 * Displacement d(X, t) of a vertex with reference position X, x = X + d:
 *   NONE
 *   SIN_PRODUCT_2D  eq. gcl_exact_field:
 *     d = (p[0], p[1]) sin(2 pi t/p[2]) sin(2 pi (X-p[5])/p[3]) sin(2 pi (Y-p[6])/p[4])
 *   TRIPLE_PRODUCT_3D  eq. TGV_deformation, amplitude p[0], period p[1], box p[2]:
 *     d_x = p[0] sin(2 pi t/p[1]) sin(2 pi (Y+p[2]/2)/p[2]) sin(2 pi (Z+p[2]/2)/p[2]), cyclic
 *   PLUNGE_BLEND_2D  the plunge y = Y - h0 sin(omega t) of Section 7.3 times a
 *     radial weight B(r) = 1 for r <= p[2], cosine ramp to 0 at r = p[3],
 *     r = |X - (p[4], p[5])|; h0 = p[0], omega = p[1].  (The weight is this
 *     library's addition so the outer boundary stays fixed.)
 *   FISH_3D  the carangiform swimming motion of Section 7.4 (eq. fish_motion,
 *     eq. fish_amplitude_function and the blended mesh motion built on them),
 *     lengths in body lengths, only z moves:
 *       d_z = A(xt) sin(phi) B S(t),  xt = min(1, max(0, X)),
 *       A = p[0] + p[1] xt + p[2] xt^2,  phi = 2 pi X / p[3] - 2 pi p[4] t,
 *       B = exp(-p[6] d^2),  d = max(|(X - xt, Y, Z)| - p[5], 0),
 *       S = (1 - cos(pi t / p[7])) / 2 for t < p[7], else 1 (p[7] <= 0: S = 1);
 *     (a0, a1, a2, wavelength, tail-beat frequency, rigid-core radius, decay
 *     rate, ramp time).  The paper prints the displacement with a factor R
 *     where the ramp S belongs; its printed mesh velocity is d/dt of the
 *     form above. */
typedef enum {
    GB_MOTION_NONE = 0,
    GB_MOTION_SIN_PRODUCT_2D = 1,
    GB_MOTION_TRIPLE_PRODUCT_3D = 2,
    GB_MOTION_PLUNGE_BLEND_2D = 3,
    GB_MOTION_VERTEX_ARRAY = 4,    /* velocities supplied per step, gb_set_vertex_velocity */
    GB_MOTION_FISH_3D = 5
} gb_motion_kind;

typedef struct {
    int kind;          /* gb_motion_kind */
    double p[8];       /* parameters, meaning per kind above */
} gb_motion;

/* Solver parameters.  c = sqrt(RT); tau is the relaxation time (nu = tau c^2,
 * Section 2).  rho0 is the density offset of FP32 storage: the FP32 path
 * stores q1 - rho0 so O(Ma^2) density fluctuations keep their digits; it is
 * ignored for FP64.  cubature_degree: exactness degree of the collapsed
 * Gauss-Jacobi rule for the relaxation term (0 = 3N; must be >= 2N).
 * q_inf: far-field / sponge state (NF values, FP64).  The sponge adds
 * -sigma(r) (q - q_inf), sigma = sigma_max ((r - r0)/(r1 - r0))^2 for
 * r0 < r (r measured from (cx, cy)); sigma_max = 0 disables it.  Wall, far
 * field and sponge are stand-ins for the paper's wall treatment and perfectly
 * matched layer, which it names without giving their form. */
typedef struct {
    double c;
    double tau;
    int precision;         /* gb_precision */
    int flux_mode;         /* gb_flux_mode */
    double rho0;
    int cubature_degree;
    double q_inf[10];
    double sponge_cx, sponge_cy, sponge_r0, sponge_r1, sponge_sigma_max;
} gb_params;

typedef struct gb_ctx gb_ctx;
typedef struct gb_mesh gb_mesh;
typedef struct gb_solver gb_solver;
typedef struct gb_batch gb_batch;

/* Last error message of this thread (never NULL). */
const char *gb_last_error(void);

/* Library version string. */
const char *gb_version(void);

/* Create a context on HIP device `device` that enqueues all work on the HIP
 * stream `stream` (a hipStream_t, or NULL for the default stream). */
gb_status gb_ctx_create(int device, void *stream, gb_ctx **out);
void gb_ctx_destroy(gb_ctx *ctx);
/* Block until all work the context enqueued has finished. */
gb_status gb_ctx_synchronize(gb_ctx *ctx);

/* A non-blocking HIP stream (default priority) of this library's HIP
 * runtime, for gb_ctx_create.  A process can hold more than one HIP runtime
 * (another framework may bundle its own); stream handles are not
 * interchangeable between runtimes, so pass either NULL (the null stream) or
 * a stream from this call. */
gb_status gb_stream_create(int device, void **stream);
void gb_stream_destroy(void *stream);


/* Build a mesh (Section 3: K non-overlapping, straight-sided, positively
 * oriented simplices with a fixed topology).
 *   dim      2 or 3;  N  polynomial order (2D: 1..5, 3D: 1..3)
 *   vx       [nv][dim] reference (t = 0) vertex coordinates
 *   etov     [K][dim+1] vertex indices, every element with J > 0
 *   period   [dim] box period per direction, 0 = not periodic; NULL = none.
 *            Periodic images are matched modulo the period; vertices on
 *            opposite sides stay separate vertices.
 *   face_tag [K][dim+1] GB_FACE_* for faces without a partner; NULL = none.
 * Builds the reference operators, the element connectivity and the
 * node-to-node trace map (vmapP) on the host and uploads them once.
 * Errors: GB_ERR_ARG, GB_ERR_MESH (J <= 0, unmatched untagged face),
 * GB_ERR_UNSUPPORTED, GB_ERR_OOM. */
gb_status gb_mesh_create(gb_ctx *ctx, int dim, int N, int64_t nv, const double *vx,
                         int64_t K, const int32_t *etov, const double *period,
                         const int8_t *face_tag, gb_mesh **out);
void gb_mesh_destroy(gb_mesh *mesh);

/* Sizes: Np nodes per element, NF fields, Nfaces*Nfp face nodes per
 * element, Nc cubature points (for the given degree, 0 = 3N). */
gb_status gb_mesh_sizes(const gb_mesh *mesh, int64_t *K, int *Np, int *NF, int *Nfp, int *Nfaces);

/* Reference-operator export (host computation, no GPU work), for checking
 * the host setup: which = 0..2 differentiation matrix D_r, D_s, D_t [Np][Np];
 * 3 LIFT [Np][Nfaces*Nfp] (faces parametrised with reference measure 2);
 * 4 cubature interpolation [Nc][Np]; 5 projection [Np][Nc]; 6 nodes [Np][dim];
 * 7 mass matrix [Np][Np].  `out` must hold the stated size; `n_out` receives
 * the element count written. */
gb_status gb_ref_operator(int dim, int N, int cubature_degree, int which, double *out,
                          int64_t capacity, int64_t *n_out);

/* Host-only checks (no device work), for validating inputs and the library's
 * own table construction without a GPU:
 *   gb_check_mesh_tables builds the connectivity and the blocked trace map
 *   exactly as gb_mesh_create does and checks them: vertex ids in range,
 *   every trace-map entry a boundary code or a face node of another element,
 *   the map an involution on matched faces, the blocked copy equal to the
 *   flat one with padding elsewhere.  GB_ERR_MESH with the first violation.
 *   gb_check_batch_layout builds the request-table layout of a batched launch
 *   class of nmembers meshes (K[i] elements, nv[i] vertices) with the buffer
 *   sizes gb_mesh_create / gb_solver_create allocate and checks it as
 *   gb_batch_run does before every table upload: buffers cover what the
 *   kernel addresses, group offsets are the running sums, counts within
 *   limits, and the dynamic LDS of the launch (written to *lds_bytes) within
 *   lds_limit.  GB_ERR_STATE with the first violation. */
gb_status gb_check_mesh_tables(int dim, int N, int64_t nv, const double *vx, int64_t K, const int32_t *etov,
                               const double *period, const int8_t *face_tag);
gb_status gb_check_batch_layout(int dim, int N, int precision, int cubature_degree, int nmembers, const int64_t *K,
                                const int64_t *nv, size_t lds_limit, size_t *lds_bytes);

/* Current node coordinates [K][dim][Np] (host output). */
gb_status gb_mesh_nodes(const gb_mesh *mesh, double *xyz);

/* Current vertex coordinates [nv][dim] (host output). */
gb_status gb_mesh_vertices(const gb_mesh *mesh, double *vx);

/* Set the prescribed motion (Section 5).  May be called before or between
 * steps; the current vertex positions are kept. */
gb_status gb_set_motion(gb_mesh *mesh, const gb_motion *motion);

/* Grid motion given by the caller (e.g. an external mesh-motion solver):
 * w [4][nv][dim] (FP64 host, copied) holds the velocity of every vertex at
 * the stage times t_n, t_n + dt/2, t_n + dt/2 and t_n + dt of the next step;
 * the vertex positions of the stages advance from them by the classical RK4
 * of Section 5, as for the analytic motions.  Call it before every step
 * (steps run with the last values given); it waits for earlier work of the
 * mesh's context.  Sets the mesh's motion kind to GB_MOTION_VERTEX_ARRAY. */
gb_status gb_set_vertex_velocity(gb_mesh *mesh, const double *w);

/* Create a solver on a mesh.  Allocates the four resident state arrays of the
 * SARK-4 schedule in device memory.  The solver keeps a reference to the
 * mesh: destroy the solver first.  A mesh carries the vertex positions its
 * solver moves, so it takes one solver at a time: GB_ERR_STATE while another
 * solver of the mesh exists. */
gb_status gb_solver_create(gb_mesh *mesh, const gb_params *params, gb_solver **out);
void gb_solver_destroy(gb_solver *solver);

/* Device bytes gb_solver_create would allocate for this mesh and params
 * (state arrays and per-stage vertex data; the mesh's own tables are counted
 * by gb_mesh_footprint). */
gb_status gb_solver_footprint(const gb_mesh *mesh, const gb_params *params, size_t *bytes);

/* Device bytes held by the mesh (connectivity, trace map, vertex arrays). */
gb_status gb_mesh_footprint(const gb_mesh *mesh, size_t *bytes);

/* Set the state q [K][NF][Np] (FP64 host) and the time t0; resets the step
 * counter to 0 and the vertex positions to the reference positions the mesh
 * was created with (the configuration of the motion at time t0; the analytic
 * motions have zero displacement at t = 0).  To resume a run with moved
 * vertices use gb_checkpoint_load. */
gb_status gb_state_set(gb_solver *solver, const double *q, double t0);

/* Set the state to the equilibrium of the given density and velocity at
 * every node (Section 2: rho = q1, rho u = c m, and the stress moments at
 * which the collision term vanishes, S = m m^T / rho, stored with the
 * diagonal as S_ii / sqrt2), plus an optional constant offset per field.
 *   rho    [K][Np] density, > 0      u  [K][dim][Np] velocity
 *   offset [NF] added to every node's moments after the equilibrium map, or
 *          NULL (e.g. a uniform off-equilibrium stress)
 * Computed on the device; time, step counter and vertex positions are reset
 * as by gb_state_set.  GB_ERR_ARG if a density is not positive. */
gb_status gb_state_set_equilibrium(gb_solver *solver, const double *rho, const double *u, const double *offset,
                                   double t0);

/* The same equilibrium map on the host, for states such as a far-field
 * q_inf: rho [n], u [dim][n] -> q [NF][n].  No device work. */
gb_status gb_equilibrium_moments(int dim, double c, int64_t n, const double *rho, const double *u, double *q);

/* Checkpoint / resume.  A checkpoint is the solver's state in its storage
 * precision (bit for bit), the current vertex positions, the time and the
 * step counter, with a header of the mesh sizes.  Loading it into a solver
 * of the same mesh (same vertices, elements, order, precision) and stepping
 * n more steps gives bit for bit the result of stepping on without the
 * checkpoint.  gb_checkpoint_bytes gives the buffer size; save synchronises;
 * load checks the header (GB_ERR_ARG on a mismatch) and replaces state,
 * positions, time and step counter. */
gb_status gb_checkpoint_bytes(const gb_solver *solver, size_t *bytes);
gb_status gb_checkpoint_save(gb_solver *solver, void *buf, size_t bytes);
gb_status gb_checkpoint_load(gb_solver *solver, const void *buf, size_t bytes);

/* Copy the state to the host (FP64 [K][NF][Np]); also returns the time and
 * the number of steps taken.  Synchronises and reports latched errors. */
gb_status gb_state_get(gb_solver *solver, double *q, double *t, int64_t *step);

/* F = L(q) + P Ntilde(I q) for q [K][NF][Np] (FP64 host in and out) at the
 * current vertex positions, with the grid velocity at the current time: the
 * right-hand side of eq. time_split without the stiff -Lambda q part
 * (Section 4).  Does not change the solver state, its constants or its
 * later steps.  Synchronises.  GB_ERR_STATE while the solver is a member of
 * a batch. */
gb_status gb_rhs(gb_solver *solver, const double *q, double *F);

/* Kinetic energy and its dissipation rate (Section 7.2):
 *   out[0] = E_K = (1 / (rho_inf |Omega|)) integral of rho u.u / 2,
 *   out[1] = epsilon_1 = -dE_K/dt,  out[2] = |Omega| (current mesh volume),
 * at the solver's current state, vertex positions and time.  The integral is
 * taken element by element with the cubature rule of the relaxation term
 * applied to the element's density and momentum (rho u = c m); dE_K/dt is
 * the exact rate of that discrete energy along the semi-discrete system:
 * the density and momentum change by F(q) (they have no stiff part) and the
 * element Jacobians by J div(w), w the grid velocity at the current time.
 * One right-hand-side evaluation (into a state array that is free between
 * steps) and a two-pass device reduction in FP64 (deterministic: the same
 * state gives the same bits).  Synchronises.  GB_ERR_STATE without a state
 * or while the solver is a member of a batch. */
gb_status gb_energy(gb_solver *solver, double rho_inf, double out[3]);

/* gb_energy for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result bit for bit, with the reduction's
 * partial sums in a fixed 64 KiB device array that the library holds on
 * every device it runs on until the process ends, instead of a buffer the
 * solver allocates on its first gb_energy call.  The call makes no device
 * allocation or free.  That array takes at most 8192 doubles: one workgroup
 * per 4 elements up to 4 per compute unit, 4 partial sums each, and the
 * result; GB_ERR_ARG if the reduction would need more (not reached below
 * 512 compute units).  All calls on one device share the array and it keeps
 * the last call's contents (each call writes every entry it reads): calls
 * that overlap in time on one device race, so issue them from one thread,
 * one at a time.  Synchronises; errors as gb_energy. */
gb_status gb_energy_noalloc(gb_solver *solver, double rho_inf, double out[3]);

/* Force of the fluid on the body: the integral over every wall face
 * (GB_FACE_WALL) of p n (pressure, p = rho RT = c^2 rho) and of -sigma n
 * (viscous, sigma the deviatoric stress of Section 2: sigma_ab =
 * -c^2 (S_ab - m_a m_b / rho)), n the outward normal of the fluid element,
 * at the current state and vertex positions.  out[0..dim) = pressure part,
 * out[dim..2 dim) = viscous part.  The drag and lift coefficients of Section
 * 7.3 are c_D = F_x / (rho_inf u_inf^2 chord / 2) and c_L likewise with F_y.
 * Zero when the mesh has no wall face.  FP64 device reduction; synchronises.
 * GB_ERR_STATE without a state or while the solver is a member of a batch. */
gb_status gb_wall_force(gb_solver *solver, double *out);

/* Advance nsteps SARK-4 steps of size dt (Section 4) on the context's
 * stream.  Asynchronous: returns after enqueueing.  The vertex positions
 * move with the prescribed motion by classical RK4 (Section 5). */
gb_status gb_sark_step(gb_solver *solver, double dt, int64_t nsteps);

/* Same as gb_sark_step, replaying a captured HIP graph of one step; the
 * graph is rebuilt when dt changes. */
gb_status gb_sark_step_graph(gb_solver *solver, double dt, int64_t nsteps);

/* Stage-kernel timing.  gb_solver_time_stages(solver, 1) resets the counters
 * and brackets every later stage launch of gb_sark_step with a HIP event pair
 * on the context's stream (graph replays are not timed).  gb_solver_stage_time
 * synchronises on the last event and returns the average launch duration in
 * milliseconds and the number of launches measured since the reset. */
gb_status gb_solver_time_stages(gb_solver *solver, int enable);
gb_status gb_solver_stage_time(gb_solver *solver, double *avg_ms, int64_t *launches);
/* Per stage kind (0..3) average launch duration in ms, same measurement. */
gb_status gb_solver_stage_time_by_kind(gb_solver *solver, double *avg_ms4);

/* ------------------------------------------------------------------------
 * Batched form: many solvers (meshes of any size, orders and precisions on
 * one device) advanced together.  A member large
 * enough to fill the GPU (>= 2048 groups of 16 elements) is stepped on its
 * own (vertex motion, the four SARK-4 stages, end-of-step update); the
 * smaller members are stepped together from a captured HIP graph: one
 * vertex launch per dimension,
 * then for each stage one launch per class (same dimension, order,
 * precision and cubature rule) over the concatenated element groups of its
 * members.  The kernels read a device request
 * table (buffers, group offsets, constants, clock and target step of every
 * member); a member whose step counter has reached its target is skipped, so
 * members finish at different steps while the graph keeps replaying.  A
 * member's result does not depend on what else is in the batch (bit for
 * bit); it agrees with gb_sark_step to rounding (same per-element source,
 * compiled in another kernel).
 *
 * Continuous batching: members join (gb_batch_add) and leave (gb_batch_poll)
 * at step boundaries; the table and the graph are rebuilt at the next
 * gb_batch_run after a change.  The launch grid of each class is chosen by
 * timing the first stage at several grids the first time the class runs
 * (stage 0 at a step boundary only overwrites a buffer the next step
 * recomputes, so the tuning leaves every member's state unchanged); the
 * tile tried covers workgroups per CU, wavefronts per workgroup and the
 * dealing of groups to workgroups (gb_batch_class_tile, gb_tune_cache_*).
 * ------------------------------------------------------------------------ */

/* Create a batch on ctx's stream with an admission budget in bytes of device
 * memory (the sum of gb_solver_footprint + gb_mesh_footprint of its members). */
gb_status gb_batch_create(gb_ctx *ctx, size_t hbm_budget, gb_batch **out);
/* Synchronises; the members stay valid and owned by the caller. */
void gb_batch_destroy(gb_batch *batch);

/* Admit solver (state already set, same device) for nsteps >= 1 more steps of
 * size dt.  GB_ERR_BUSY if its footprint exceeds the free budget (nothing is
 * changed; retry after members leave).  The solver must not be stepped or
 * read by other calls until gb_batch_poll has returned its ticket. */
gb_status gb_batch_add(gb_batch *batch, gb_solver *solver, double dt, int64_t nsteps, uint64_t *ticket);

/* Enqueue `steps` batch steps on the batch's stream (asynchronous), in
 * rounds of k steps (k the largest divisor of `steps` up to 8): each large
 * member takes its k steps in turn (direct launches), then the small members
 * take theirs from a captured graph of k steps.  Members stop at their
 * target step. */
gb_status gb_batch_run(gb_batch *batch, int64_t steps);

/* Synchronise, retire up to `capacity` members that reached their target
 * step and write their tickets to done[0..*n_done).  A retired solver is
 * usable alone again (gb_state_get reports its time, steps and latched
 * errors). */
gb_status gb_batch_poll(gb_batch *batch, uint64_t *done, int capacity, int *n_done);

/* Members, budget in use, and budget. */
gb_status gb_batch_info(const gb_batch *batch, int *active, size_t *used_bytes, size_t *budget);

/* Members large enough to be stepped on their own run on up to `streams`
 * streams at once (library-owned, default priority), so that the last
 * workgroups of one member's kernels overlap another's; 1 (default) steps
 * them in turn on the batch's stream.  Results do not depend on it.  Waits
 * for the batch's queued work. */
gb_status gb_batch_set_concurrency(gb_batch *batch, int streams);

/* Enable (default) or disable the launch-grid tuning of new classes. */
gb_status gb_batch_set_autotune(gb_batch *batch, int enable);

/* Launch classes of the current table (valid after gb_batch_run): info[7] =
 * {dim, N, precision, members, element groups, launch grid, solo}; solo = 1
 * for a member large enough (>= 2048 groups of 16 elements) to be stepped on
 * its own, its four stages back to back so its state stays in the
 * last-level cache; the smaller members of a class share one launch per
 * stage. */
gb_status gb_batch_class_count(const gb_batch *batch, int *n);
gb_status gb_batch_class_info(const gb_batch *batch, int i, int64_t *info7);

/* Launch tile of class i: tile3 = {workgroups, wavefronts per workgroup (4,
 * or 8 for the kernels that run two wavefronts per SIMD), group dealing (0 =
 * contiguous ranges per workgroup, 1 = blocks of one group per wavefront
 * dealt round robin)}.  The tile does not change any member's result. */
gb_status gb_batch_class_tile(const gb_batch *batch, int i, int64_t *tile3);

/* Launch-tile cache of the autotuner.  The first run of a class (same device
 * architecture, dimension, order, precision, cubature size, solo or shared,
 * and power-of-two bucket of its element groups) times stage 0 for every
 * candidate tile (1, 2, 4, 8, 16 workgroups per CU; 4 or 8 wavefronts per
 * workgroup; ranges or round-robin dealing) and keeps the fastest in a
 * process-wide cache; later batches reuse it without timing.  The cache can
 * be saved to a text file and loaded in another process (entries merge,
 * loaded ones win); a malformed file is refused with GB_ERR_ARG. */
gb_status gb_tune_cache_save(const char *path);
gb_status gb_tune_cache_load(const char *path, int *entries);
void gb_tune_cache_clear(void);

#ifdef __cplusplus
}
#endif

#endif /* GB_H */
