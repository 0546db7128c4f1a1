/*
 * liblbm -- one D3Q19 lattice Boltzmann step with Smagorinsky relaxation,
 * velocity-corrected (Bouzidi) bounce-back on moving spheres and voxel walls,
 * and the momentum-exchange force/torque on every solid, for AMD Instinct
 * MI355X (gfx950).
 *
 * The operation is the fluid half of the LBM-DEM coupling of Mutabaruka &
 * Kamrin, arXiv:1703.05158: each time step the solids (DEM spheres, moving
 * rigid walls) hand their kinematics to the fluid, the fluid performs one
 * collide-stream step in which the lattice links cut by solid surfaces are
 * closed by interpolated bounce-back with the moving-boundary correction
 * (Sec. 2.3, eq. moving_boundary_velocity), and the fluid returns the
 * hydrodynamic force and torque on every solid by momentum exchange
 * (Sec. 2.3, force and torque equations; Sec. 2.5 for the coupled step).
 * Streaming and BGK collision follow Sec. 2.2 (eq. Collision_step and the
 * streaming equation), the velocity set Table 1, the equilibrium eq.
 * (Equilibre_Maxwell_Boltzmann) and the Smagorinsky relaxation time the
 * closing equation of Sec. 2.2, with the filter length and time step 1.
 *
 * Conventions shared by every call
 *   - Lattice units (Sec. 2.2): spacing = time step = 1, c_s^2 = 1/3.
 *   - Node (x, y, z) has linear index n = x + nx*(y + ny*z); every axis is
 *     index-periodic; non-periodic boundaries are solid wall voxels.
 *   - Populations are numbered as in Table 1 (opposite(i) = i +- 9).
 *   - Host arrays are read or written only during the call (copied before
 *     return).  Device pointers (the *_device calls) must stay valid until
 *     the work queued on the handle's stream has run.
 *   - Owner precedence: a node inside a wall voxel belongs to that wall;
 *     otherwise to the lowest-index sphere whose closed ball contains it
 *     (|p - X|^2 <= R^2, minimum image, evaluated in FP64 without fused
 *     multiply-add); otherwise it is fluid.
 *   - Force ordering: spheres first (index order), then walls (id order).
 *   - Every call returns a status; nothing aborts or throws across the ABI.
 *     Argument errors are detected on the host before any device work is
 *     queued; lbm_last_error() gives a per-handle description.
 *   - A handle is used by one host thread at a time.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx *lbm_handle;

typedef enum {
    LBM_OK = 0,
    LBM_ERR_ARG = 1,       /* invalid argument (null pointer, range, size) */
    LBM_ERR_OOM = 2,       /* device or pinned host allocation failed */
    LBM_ERR_HIP = 3,       /* a HIP runtime call failed (text in lbm_last_error) */
    LBM_ERR_STATE = 4,     /* call not valid in the handle's current state */
    LBM_ERR_UNSTABLE = 5,  /* NaN/Inf or non-positive density detected by the guard */
    LBM_ERR_CAPACITY = 6   /* more bodies or walls than the handle was created for */
} lbm_status;

/* Storage of the populations in HBM.  All three store deviations
 * g_i = f_i - w_i rho0 from the rest state; collision math is FP32 and each
 * link's force and torque FP64 in every mode. */
typedef enum {
    LBM_STORE_F32 = 0,     /* 4 bytes per population */
    LBM_STORE_F16_DEV = 1, /* IEEE binary16 deviations, 2 bytes */
    LBM_STORE_BF16_DEV = 2 /* bfloat16 deviations, 2 bytes */
} lbm_storage;

/* Link fraction q of Sec. 2.3.  BOUZIDI: q from the exact sphere geometry,
 * walls at q = 1/2.  HALFWAY: q = 1/2 on every link (then both Bouzidi
 * branches reduce to bounce-back at the link midpoint). */
typedef enum { LBM_BB_BOUZIDI = 0, LBM_BB_HALFWAY = 1 } lbm_bb_mode;

typedef struct lbm_config {
    int32_t nx, ny, nz;        /* box in nodes, each >= 1 */
    int32_t storage;           /* lbm_storage */
    double tau0;               /* molecular relaxation time, > 1/2 (Sec. 2.2, eq. ViscositeLBM) */
    double smag_c;             /* Smagorinsky constant C >= 0 (Sec. 2.2) */
    double rho0;               /* reference density, > 0 (1 in lattice units) */
    double body_force[3];      /* body-force density per fluid node per step (Guo forcing) */
    int32_t bb_mode;           /* lbm_bb_mode */
    int32_t max_bodies;        /* capacity of the sphere table, >= 0 */
    int32_t max_walls;         /* capacity of the wall table, 0..16 */
    int32_t nan_guard_every;   /* 0 = off; k > 0: check every k steps (syncs) */
    void *stream;              /* hipStream_t to queue work on; NULL = null stream */
} lbm_config;

typedef struct lbm_info {
    int64_t n_nodes;           /* nx*ny*nz */
    int32_t n_bodies;          /* spheres of the current state's geometry */
    int32_t n_walls;
    int32_t storage_bytes;     /* bytes per stored population: 4 or 2 */
    int32_t steps_done;
    int64_t device_bytes;      /* device memory held by the handle */
} lbm_info;

/* Version of this interface: 10000*major + 100*minor + patch. */
int32_t lbm_version(void);

/* Create a handle: validates cfg, allocates two population buffers
 * (19 * N * storage bytes each), the owner map (2 bytes per node) and the
 * body/wall tables on the current HIP device.  *out is set only on LBM_OK.
 * Errors: ARG (null pointer, sizes, tau0 <= 1/2, C < 0, rho0 <= 0, unknown
 * enum, capacities), OOM, HIP. */
lbm_status lbm_create(const lbm_config *cfg, lbm_handle *out);

/* Free every resource of the handle (waits for its queued work).  NULL is
 * ignored.  The handle must not be used afterwards. */
void lbm_destroy(lbm_handle h);

/* Text of the last error on this handle ("" if none; static text if h is
 * NULL).  Valid until the next call on the handle. */
const char *lbm_last_error(lbm_handle h);

/* Queue the handle's future work on another stream (hipStream_t or NULL). */
lbm_status lbm_set_stream(lbm_handle h, void *stream);

/* Static wall voxels (the moving rigid walls of Sec. 2.1/2.3 realised as
 * voxel objects whose links close at q = 1/2).
 *   wall_id  : N bytes, 0 = not a wall, 1..n_walls = wall object (host).
 *   wall_vel : n_walls x 3 wall velocities (host; may be NULL if n_walls = 0).
 *   wall_ref : n_walls x 3 torque reference points (host; NULL = origin).
 * Must be called before lbm_init_fields.  Errors: ARG (null map, id larger
 * than n_walls, non-finite values), CAPACITY (n_walls > max_walls), STATE
 * (after lbm_init_fields). */
lbm_status lbm_set_walls(lbm_handle h, const uint8_t *wall_id, int32_t n_walls,
                         const double *wall_vel, const double *wall_ref);

/* Sphere kinematics for the next step (Sec. 2.3: the solid velocity at a
 * boundary point is V + Omega x (x_b - X)).  Host arrays:
 *   X, V, Omega : n x 3 (centre in [0, n_axis) per axis, velocity, angular
 *                 velocity); R : n radii, 0 < R < min(nx,ny,nz)/2 - 1.
 * The bodies given before step k are the geometry and velocities of step k;
 * nodes that turn from solid to fluid are refilled with the equilibrium at
 * rho0 and the velocity they had as solids.  The copy is asynchronous on the
 * handle's stream (pinned staging).  The link pass takes the spheres in
 * Morton order of centres given here (made again when the count changes and
 * on every 32nd call, kept for device tables of the same count); no result
 * depends on that order.  Errors: ARG (null with
 * n > 0, ranges, non-finite values), CAPACITY (n > max_bodies). */
lbm_status lbm_set_bodies(lbm_handle h, int32_t n, const double *X, const double *V,
                          const double *Omega, const double *R);

/* Same from a device table d_table[n][10] = {X[3], V[3], Omega[3], R} in
 * FP64, copied on the handle's stream.  The values are not checked on the
 * host: a sphere with a radius outside (0, min(n)/2 - 1) or a centre outside
 * the box is ignored by the rasteriser.  Errors: ARG, CAPACITY. */
lbm_status lbm_set_bodies_device(lbm_handle h, int32_t n, const double *d_table);

/* Initial state: f_i = f_i^eq(rho, u) at fluid nodes (no collision), the
 * geometry of the current walls and bodies being both the initial geometry
 * and that of step 1.  rho: N densities or NULL (rho0); u: 3N velocities,
 * component-major (u[c*N + n]), or NULL (0).  Host arrays.  Resets the step
 * counter and the forces.  Errors: ARG (non-positive or non-finite rho,
 * non-finite u), HIP. */
lbm_status lbm_init_fields(lbm_handle h, const double *rho, const double *u);

/* Advance nsteps steps, asynchronously on the handle's stream.  Each step:
 * re-rasterise the spheres if they were set since the previous step (nodes
 * a sphere no longer covers are refilled, then the new spheres are
 * stamped); then, on the fused path (the default), one kernel per tile
 * closes every cut link of the tile's fluid nodes with interpolated
 * bounce-back and the moving-boundary term (Sec. 2.3), formed from the
 * current state, adds the momentum exchanged on each link to the body's
 * force and torque, and does pull streaming, moments, Smagorinsky tau*,
 * BGK + Guo collision and the store (Sec. 2.2).  The force and torque sums
 * are kept as 64-bit fixed point with a resolution of 2^-32 per link
 * contribution (sums must stay below 2^31 in magnitude), so they are the same
 * bit for bit in any launch order, tile shape or batch.  The sums of a
 * step are turned into FP64 forces by whichever comes first: the next fused
 * step kernel, or lbm_get_forces / lbm_get_forces_device.  On the split path
 * (lbm_set_step_path) a link pass writes every link value into the solid
 * node's slot of the current state and reduces the forces per body in FP64,
 * then the pull-collide kernel pulls it; the populations are the same bit
 * for bit on both paths.  Forces are those of the last step.
 * With nan_guard_every = k the call synchronises every k steps and returns
 * LBM_ERR_UNSTABLE if a fluid node had a non-finite or non-positive density
 * or a non-finite velocity.  Errors: STATE (before lbm_init_fields), ARG
 * (nsteps < 0), HIP, UNSTABLE. */
lbm_status lbm_step(lbm_handle h, int32_t nsteps);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lbm_step
 * with the fused kernel whatever the step path, whose fixed-point force sums
 * live in a static device array of the library (2 x LBM_STATIC_FIX_SUMS
 * 64-bit sums, 1 MiB, held on each device the library runs on until the
 * process ends) instead of the handle's buffers.  The call allocates
 * nothing and records no profile events; it clears what it uses of the array
 * at its start, with a kernel, and turns the sums of its last step into the
 * forces before it returns, so nothing in the array outlives the call.
 * Populations and forces are the same bit for bit as lbm_step's.  All calls
 * on one device share the array: calls that overlap on that device (two
 * handles on different streams, or threads) race and give wrong forces.
 * Limit: 6 (n_bodies + 64 n_walls) <= LBM_STATIC_FIX_SUMS, with n_bodies the
 * larger of the current and the pending sphere count.  Errors: as lbm_step,
 * CAPACITY beyond the limit, HIP if the array's address could not be found
 * on the device the handle was created on. */
#define LBM_STATIC_FIX_SUMS 65536
lbm_status lbm_step_noalloc(lbm_handle h, int32_t nsteps);

/* Force and torque on every sphere then every wall, of the last step, in
 * FP64 (host arrays of (n_bodies + n_walls) x 3).  Torques of spheres are
 * about their centre, of walls about their reference point.  Synchronises
 * the stream.  Errors: ARG, STATE, HIP. */
lbm_status lbm_get_forces(lbm_handle h, double *F, double *T);

/* Same into device memory, asynchronously: d_out[(n_bodies + n_walls) * 6]
 * holds {Fx, Fy, Fz, Tx, Ty, Tz} per body.  Errors: ARG, STATE, HIP. */
lbm_status lbm_get_forces_device(lbm_handle h, double *d_out);

/* Post-collision populations of the current state as full f (not
 * deviations), FP64, host array [19][N].  Solid nodes report the
 * equilibrium at rho0 and their solid velocity.  Synchronises.
 * Errors: ARG, STATE, HIP. */
lbm_status lbm_get_populations(lbm_handle h, double *f);

/* Overwrite the current state with full populations f [19][N] (host, FP64),
 * converted to the storage type.  Errors: ARG (non-finite), STATE, HIP. */
lbm_status lbm_set_populations(lbm_handle h, const double *f);

/* Density rho[N] and velocity u[3N] (component-major) of the current state:
 * rho = sum f, u = (sum f c - F/2)/rho, i.e. the velocity used by the last
 * collision (which added F to the momentum).  Solid nodes report rho0 and
 * their solid velocity.  Synchronises.  Errors: ARG, STATE, HIP. */
lbm_status lbm_get_macro(lbm_handle h, double *rho, double *u);

/* Owner map of the current state's geometry, int32 per node: -1 fluid,
 * 0..n_walls-1 wall, n_walls + b sphere b.  Synchronises. */
lbm_status lbm_get_owner(lbm_handle h, int32_t *owner);

/* Checkpoint: with buf == NULL, *bytes receives the size needed; otherwise
 * the populations (storage type), owner map, body and wall tables and
 * counters are written to buf (host, *bytes >= size).  lbm_set_state
 * restores a checkpoint of a handle with the same configuration; resuming
 * reproduces the populations bit for bit.  It checks the buffer on the host
 * before copying anything: size, configuration, body and wall counts within
 * the handle's capacities and wall ids within the wall count; a rejected
 * buffer leaves the handle as it was.  Errors: ARG, STATE, HIP. */
lbm_status lbm_get_state(lbm_handle h, void *buf, size_t *bytes);
lbm_status lbm_set_state(lbm_handle h, const void *buf, size_t bytes);

/* Sizes and counters of the handle (host-side values, no device work).
 * Errors: ARG. */
lbm_status lbm_get_info(lbm_handle h, lbm_info *info);

/* Number of fluid nodes of the current state's geometry (a reduction over
 * the owner map; synchronises).  Errors: ARG, HIP. */
lbm_status lbm_count_fluid(lbm_handle h, int64_t *n_fluid);

/* Timing of the step's parts with HIP events on the handle's stream:
 * lbm_profile(h, every) with every > 0 starts recording events at the
 * boundaries of the parts of every every-th step, the first one included
 * (and clears earlier records); lbm_profile(h, 0) stops.  Each event costs a profiled step a few
 * microseconds of GPU time, so a sample of the steps disturbs a long run
 * less.  The fused kernel's start and end are recorded by its own launch.
 * lbm_profile_read synchronises and returns the summed time of the step
 * kernel (the fused kernel, or the pull-collide kernel of the split path) in
 * milliseconds and the number of steps recorded.  lbm_profile_read_parts
 * returns ms[LBM_PROF_PARTS]: the summed time of each part below over the
 * recorded steps (0 for a part the path does not run), and the step count.
 * Errors: ARG (n < 0), HIP. */
enum {
    LBM_PROF_GEOMETRY = 0, /* inflow-plane update and re-rasterisation */
    LBM_PROF_LINKS = 1,    /* boundary-link pass (split path) */
    LBM_PROF_STEP = 2,     /* step kernel */
    LBM_PROF_WHOLE = 3,    /* the whole step, first event to last */
    LBM_PROF_PARTS = 4
};
lbm_status lbm_profile(lbm_handle h, int32_t every);
lbm_status lbm_profile_read(lbm_handle h, double *ms_total, int64_t *launches);
lbm_status lbm_profile_read_parts(lbm_handle h, double *ms, int64_t *steps);

/* Kernels that make a step (see lbm_step).  FUSED: one kernel per step does
 * links, streaming and collision; its fixed-point force sums become FP64
 * forces when they are read or at the start of the next fused step.  SPLIT:
 * the boundary-link pass, then the
 * pull-collide kernel.  Both give the same populations bit for bit; their
 * forces agree to rounding.  The drag gradient's reverse sweep uses the
 * split path's kernels whatever the setting.  Errors: ARG. */
typedef enum { LBM_PATH_FUSED = 0, LBM_PATH_SPLIT = 1 } lbm_step_path;
lbm_status lbm_set_step_path(lbm_handle h, int32_t path);
lbm_status lbm_get_step_path(lbm_handle h, int32_t *path);

/* Zoom-in with Effective Boundaries (Sec. 2.6): the plane z = z_s is fed
 * by a removed cylinder of volume `volume` and piston area `area` whose
 * piston moves at v_piston (lattice units, time step 1) towards +z.  The
 * whole layer z_s - 1 (periodic) must be wall voxels; it stands for the
 * removed domain, and the plane's links into it are not wall links.  Each
 * step: the mean in-flowing velocity v_f of the plane's fluid nodes (u of the
 * current state, as in lbm_get_macro) and eq. (ZIEBdesity8) give the
 * cylinder's new density rho (at the first step rho starts from the plane's
 * mean density); on the plane, the populations arriving from the removed
 * domain keep the node's own values, f_12 becomes rho - (rho* - f_12) with
 * rho* the node's density (eq. ZIEBdesity9), and all populations become the
 * equilibrium at rho and u = sum f c / rho before the collision.  The piston
 * displacement H advances by v_piston per step.  z_s < 0 removes the plane.
 * Must be called after lbm_set_walls and before lbm_init_fields; handles
 * with a plane cannot be batched.  lbm_get_zieb writes {rho, H, v_f} of the
 * last step (host, 3 doubles; synchronises).  Errors: ARG (range, the layer
 * below is not all wall), STATE (after lbm_init_fields, before the walls;
 * no plane for lbm_get_zieb), HIP. */
lbm_status lbm_set_zieb(lbm_handle h, int32_t z_s, double area, double volume, double v_piston);
lbm_status lbm_get_zieb(lbm_handle h, double *state);

/* Replace the body force (Guo source density per fluid node, Sec. 2.2 with
 * the forcing reading) for the following steps.  Errors: ARG. */
lbm_status lbm_set_body_force(lbm_handle h, const double *F);

/* Gradient of the summed sphere drag.  J = sum_b F_b,x, the x-component of
 * the momentum-exchange force on every sphere (Sec. 2.3) at the last of
 * nsteps steps from the current state, with the spheres held where they are
 * (their velocities V enter only the moving-boundary term).  The call runs
 * the nsteps steps (the handle's state advances as with lbm_step, and the
 * forces of the last step stay readable), keeping every ckpt-th state, then
 * runs the reverse-mode kernels backwards, recomputing each stretch of ckpt
 * steps from its checkpoint: the transposed collision per node, the
 * transposed streaming and the transposed boundary links.  Outputs (host):
 * J; dJdF[3] = dJ/d(body force); dJdV[3 n_bodies] = dJ/dV_b, sphere-major
 * (may be NULL with no spheres).  The square root of Q = Pi:Pi has the
 * derivative 1/(2 sqrt(Q + 1e-30)).  Device memory: ceil(nsteps/ckpt) +
 * min(ckpt, nsteps) + 2 population buffers, allocated for the call.  Needs
 * FP32 storage, no walls and no inflow plane.  Synchronises.  Errors: ARG,
 * STATE, OOM, HIP. */
lbm_status lbm_drag_gradient(lbm_handle h, int32_t nsteps, int32_t ckpt, double *J, double *dJdF,
                             double *dJdV);

/* Tile shape of the step kernel, the nodes of one 256-thread workgroup:
 * 0 = 64x2x2, 1 = 32x4x2, 2 = 32x2x4, 3 = 16x8x2 (x, y, z).  Results are the
 * same bit for bit for every shape; only the speed differs.  lbm_create
 * picks 64x2x2, or 32x4x2 when nx is a multiple of 32 but not of 64.
 * Errors: ARG (shape out of range). */
lbm_status lbm_set_tile(lbm_handle h, int32_t shape);
lbm_status lbm_get_tile(lbm_handle h, int32_t *shape);

/* Tile-shape autotuner.  Times trial_steps launches of the step kernel for
 * every tile shape on the handle's current state (the launches write only
 * the spare population buffer, so the state does not advance), twice over
 * the shapes, and keeps the shape with the fastest of its two times.  cache_path (may be NULL) names a JSON object of integer shapes
 * keyed "<gfx target>/<f32|f16|bf16>/<nx>x<ny>x<nz>": a key that is present
 * is used without timing; a new result is written back.  shape (may be
 * NULL) receives the chosen shape; us (may be NULL, 4 doubles) the faster
 * of each shape's two average kernel times in microseconds, -1 where not
 * timed.  Synchronises.
 * Errors: STATE (before lbm_init_fields, or bodies set since the last step),
 * ARG (trial_steps < 1, cache not writable), HIP. */
lbm_status lbm_autotune_tile(lbm_handle h, int32_t trial_steps, const char *cache_path, int32_t *shape,
                             double *us);

/* Batched stepping of independent lattices (a parameter sweep of many
 * boxes): a batched step runs the fused step of all members as one
 * persistent launch over their tiles (each member with its own parameters),
 * the force finish of all members, and a parity flip.  lbm_batch_step
 * replays a captured hipGraph of 50 such steps as long as at least 50
 * remain, then a graph of one step for the rest.  Each member's results are
 * bit for bit those of lbm_step on that member.
 *   members : n distinct handles, all past lbm_init_fields, same storage,
 *             no bodies set since their last step (their own tile shapes
 *             do not matter: the batch has one, see below).  The batch borrows them:
 *             they must outlive it, and their bodies, walls, body force
 *             and state must not be replaced while it is used (build a new
 *             batch after a change; lbm_batch_step refuses a member
 *             changed since the batch was built with STATE).
 *   stream  : hipStream_t for the batch's work, or NULL for a stream of its
 *             own (default priority).
 * lbm_batch_step waits for the members' queued work, replays the graphs
 * for nsteps steps, synchronises, and advances every member's state and step
 * counter; forces of the last step are then read per member as usual.  The
 * NaN guard does not run in batched steps.  Errors: ARG, STATE (a member not
 * initialised, or with bodies pending), HIP, OOM (text in
 * lbm_batch_last_error, or on the offending member's handle at creation). */
typedef struct lbm_batch_ctx *lbm_batch;
lbm_status lbm_batch_create(const lbm_handle *members, int32_t n, void *stream, lbm_batch *out);
lbm_status lbm_batch_step(lbm_batch b, int32_t nsteps);
const char *lbm_batch_last_error(lbm_batch b);
void lbm_batch_destroy(lbm_batch b);

/* Tile shape of the batched step kernel (one shape for all members, same
 * numbering as lbm_set_tile; 64x2x2 when every nx is a multiple of 64, else
 * 32x4x2 at creation).  lbm_batch_autotune times trial_steps launches of the
 * batched step kernel for every shape on the members' current states (the
 * launches write only the spare buffers, so no state advances), twice over
 * the shapes, keeps the shape with the fastest of its two times and returns
 * it in shape (may be NULL), with that time per launch in microseconds for
 * each shape in us (may be NULL, 4 doubles).  Both
 * rebuild the captured graph.  Errors: ARG, STATE, HIP. */
lbm_status lbm_batch_set_tile(lbm_batch b, int32_t shape);
lbm_status lbm_batch_get_tile(lbm_batch b, int32_t *shape);
lbm_status lbm_batch_autotune(lbm_batch b, int32_t trial_steps, int32_t *shape, double *us);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
