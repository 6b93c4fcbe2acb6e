/*
 * fvlbm.h - C ABI of the MI355X (gfx950) cell-centred finite-volume lattice
 * Boltzmann library (D2Q9, BGK) on 2D unstructured meshes.
 *
 * The method is that of Wang, Zhong, Cao and Zhuo, "A simplified finite
 * volume lattice Boltzmann method ... Part I" (arXiv 1812.00390), Section 2:
 * per-cell weighted least-squares gradients of the nine distributions
 * (Eq. 12), second-order upwind face values (Eq. 11), face-flux
 * accumulation and the BGK source (Eq. 10), forward Euler (Eq. 13), AB2
 * (Eq. 16) or the four-stage Runge-Kutta scheme (Eq. 17), with the wall,
 * inlet, outlet and symmetry treatments of Section 2.4 (Eqs. 18-26).
 *
 * Conventions
 *  - Every call returns fvlbm_status (0 = OK, < 0 = error) unless stated.
 *    No C++ exception crosses this boundary.  fvlbm_last_error() gives a
 *    thread-local text for the last failing call of the calling thread.
 *  - Host arrays passed in are read during the call only (copied).
 *  - hip_stream arguments are hipStream_t values (NULL = the null stream).
 *    Work is enqueued on that stream; only calls documented as syncing wait.
 *  - Cell indices are the caller's (input) order everywhere in this API; an
 *    internal reordering is undone on output.
 *  - Distributions are exchanged in FP64, [cell][alpha], alpha in the order
 *    of Eq. 2: e0=(0,0), e1..e4=(1,0),(0,1),(-1,0),(0,-1),
 *    e5..e8=(1,1),(-1,1),(-1,-1),(1,-1).
 */
#ifndef FVLBM_H
#define FVLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FVLBM_OK = 0,
    FVLBM_E_ARG = -1,      /* null pointer, size out of range, bad enum value */
    FVLBM_E_MESH = -2,     /* invalid mesh: non-CCW/inverted cell, open or non-manifold edge, bad periodic pair, singular stencil */
    FVLBM_E_PARAM = -3,    /* tau <= 0, dt > 2 tau without FVLBM_FLAG_FORCE_DT, bad scheme/storage, buffer too small */
    FVLBM_E_NOMEM = -4,    /* device allocation failed */
    FVLBM_E_DEVICE = -5,   /* a HIP runtime call or kernel failed */
    FVLBM_E_DIVERGED = -6, /* a non-finite density or velocity was found (fvlbm_macros) */
    FVLBM_E_STATE = -7     /* the call does not fit the object's state (a solver in an error state:
                              destroy it; the last member of a batch) */
} fvlbm_status;

/* Boundary-condition kinds, Section 2.4 (Eqs. 18-26). */
typedef enum {
    FVLBM_BC_WALL = 1,     /* Eq. 18: f_P = f_eq(rho_k, u_w) + f_k - f_eq,k; face value f_P for all alpha */
    FVLBM_BC_INLET = 2,    /* Eq. 19 ghost, Eq. 23 face; rho* = rho_inf (external) or rho_k (internal) */
    FVLBM_BC_OUTLET = 3,   /* external: Eq. 20 ghost, Eq. 25 face; internal: Eq. 21 ghost, Eq. 24 face */
    FVLBM_BC_SYMMETRY = 4  /* Eq. 22 ghost (mirrored normal velocity), Eq. 26 face */
} fvlbm_bc_kind;

typedef struct {
    int32_t kind;          /* fvlbm_bc_kind */
    int32_t internal;      /* 0 external flow, 1 internal flow (inlet/outlet only) */
    double u[2];           /* wall velocity u_w (wall) or free-stream velocity u_inf (inlet/outlet) */
    double rho;            /* rho_inf (inlet/outlet); ignored for wall/symmetry */
} fvlbm_bc;

enum { FVLBM_SCHEME_EULER = 0, FVLBM_SCHEME_RK4 = 1, FVLBM_SCHEME_AB2 = 2 };
enum { FVLBM_STORE_FP32 = 0, FVLBM_STORE_FP32_DEV = 1, FVLBM_STORE_FP16_DEV = 2, FVLBM_STORE_I16_DEV = 3 };
enum { FVLBM_REORDER_NONE = 0, FVLBM_REORDER_RCM = 1, FVLBM_REORDER_HILBERT = 2, FVLBM_REORDER_BISECT = 3 };
enum { FVLBM_FLAG_FORCE_DT = 1 };

typedef struct {
    double tau;            /* relaxation time, tau = nu / cs^2 = 3 nu (Eq. 6); > 0 */
    double dt;             /* time step; 0 = min(CFL limit of Eq. 14, 2 tau of Eq. 15) */
    double cfl;            /* CFL number used when dt == 0 */
    double u_ref;          /* |U|max of Eq. 14, used when dt == 0 */
    int32_t scheme;        /* FVLBM_SCHEME_* */
    int32_t storage;       /* FVLBM_STORE_*: f as FP32, h = f - f_eq(rho0, u_dev) as FP32, h/(w S) as FP16,
                              or h as 16-bit block-scaled values (per cell nine int16 mantissas and one
                              exponent byte: 19 bytes per cell, 15 bits for the largest deviation).
                              FP16: a cell's nine values are rounded together so that its mass and
                              momentum lose as little as the format allows, and what is left (three FP16
                              values per cell, 6 bytes) is carried to the next step's update: the state is
                              the stored values less that carry.  fvlbm_macros and the residual include
                              it; fvlbm_get_f, fvlbm_rhs and fvlbm_wall_force see the stored values;
                              fvlbm_set_f and Step 0 set it from their own rounding.
                              Accuracy of the 16-bit formats: the rounding noise left in the
                              non-conserved moments is relaxed by the collision over about tau/dt
                              steps, so it grows as sqrt(tau/dt) ulps: FP16 deviations keep
                              1e-3 U where tau/dt is below about 10 (2e-3 U at tau/dt = 78),
                              the block-scaled format about ten times better */
    double rho0;           /* reference density of the deviation storage (and of Step 0 when no field is given) */
    double fp16_scale;     /* S of the FP16 deviation storage; 0 = 3 |u_ref| (or 0.3 if u_ref = 0) */
    int32_t residual_lag;  /* steps between velocity snapshots for the residual (Eq. 32); 0 = 1000 */
    int32_t flags;         /* FVLBM_FLAG_* */
    double u_dev[2];       /* deviations are stored from f_eq(rho0, u_dev) (Eq. 3); (0,0) gives f - w rho0.
                              A free-stream value keeps far-field deviations small (FP16 storage) */
} fvlbm_params;

typedef struct fvlbm_mesh fvlbm_mesh;        /* opaque; device arrays owned by the library */
typedef struct fvlbm_solver fvlbm_solver;    /* opaque; state lives in a caller-owned device buffer */
typedef struct fvlbm_batch fvlbm_batch;      /* opaque; a set of solvers advanced by shared launches */

/*
 * Build a mesh (Section 2.2): convex polygons with 3 or 4 nodes, CCW.
 *   xy            [2*n_nodes]  node coordinates
 *   cell_ptr      [n_cells+1]  CSR offsets into cell_nodes; cell_nodes CCW node ids
 *   bface_nodes   [2*n_bfaces] node pairs of boundary edges (either order)
 *   bface_group   [n_bfaces]   index into groups, or -1 for an edge listed in periodic_pairs
 *   groups        [n_groups]   boundary-condition groups
 *   periodic_pairs[2*n_periodic] boundary-edge indices (a, b) joined by periodicity
 *   periodic_shift[2*n_periodic] vector added to positions on b's side to bring them next to a
 *   reorder       FVLBM_REORDER_*; internal cell order for locality (outputs stay in input order).
 *                 FVLBM_REORDER_BISECT (recursive graph bisection) gives the step kernel's
 *                 tiles the shortest halos on meshes of any cell aspect ratio
 * Geometry and least-squares coefficients are computed on the device in FP64
 * (Eq. 12 with w = 1/|x_n - x_i|^2; f at the area centroid) and stored as FP32.
 * Errors: FVLBM_E_ARG, FVLBM_E_MESH, FVLBM_E_NOMEM, FVLBM_E_DEVICE.  Syncs hip_stream.
 */
fvlbm_status fvlbm_create_mesh(int32_t n_nodes, const double *xy, int32_t n_cells,
                               const int32_t *cell_ptr, const int32_t *cell_nodes,
                               int32_t n_bfaces, const int32_t *bface_nodes,
                               const int32_t *bface_group, int32_t n_groups,
                               const fvlbm_bc *groups, int32_t n_periodic,
                               const int32_t *periodic_pairs, const double *periodic_shift,
                               int32_t reorder, void *hip_stream, fvlbm_mesh **out);

/* Mesh facts: out[0] n_cells, out[1] faces per cell slot (3 or 4), out[2] device bytes
 * of the mesh arrays, out[3] number of boundary-adjacent cells.  Returns FVLBM_OK or FVLBM_E_ARG. */
fvlbm_status fvlbm_mesh_info(const fvlbm_mesh *mesh, int64_t out[4]);

/* min over cells of A/(Lx+Ly) (Eq. 14's length scale, FP64), or -1 on a null mesh. */
double fvlbm_mesh_cfl_length(const fvlbm_mesh *mesh);

/* Device bytes a solver needs in its caller-owned state buffer for these params
 * (distribution buffers for the scheme plus per-cell scratch).  0 on bad arguments. */
size_t fvlbm_state_bytes(const fvlbm_mesh *mesh, const fvlbm_params *params);

/*
 * Step 0 (Section 2.4.2): f = f_eq(rho, u) per cell.  rho0_cells [n_cells] and
 * u0_cells [2*n_cells] may be NULL for the uniform values params->rho0 and (0,0).
 * device_buf must hold fvlbm_state_bytes() bytes, 256-byte aligned, and outlive
 * the solver.  The solver keeps a reference to mesh (destroy solvers first).
 * Errors: FVLBM_E_ARG, FVLBM_E_PARAM, FVLBM_E_DEVICE.
 */
fvlbm_status fvlbm_init(fvlbm_mesh *mesh, const fvlbm_params *params, const double *rho0_cells,
                        const double *u0_cells, void *device_buf, size_t buf_bytes,
                        void *hip_stream, fvlbm_solver **out);

/* Time step actually used (after the Eq. 14/15 rule), or -1 on a null solver. */
double fvlbm_solver_dt(const fvlbm_solver *s);

/* Steps 1-5 repeated n_steps times (Section 2.4.2), enqueued on the solver's stream;
 * does not sync.  The launches replay HIP graphs of 32 steps and, for the rest of
 * a call, of the largest power of two that fits, each instantiated on first use.
 * Errors: FVLBM_E_ARG (n_steps < 0), FVLBM_E_STATE, FVLBM_E_DEVICE. */
fvlbm_status fvlbm_step(fvlbm_solver *s, int64_t n_steps);

/* Instantiates the graphs that fvlbm_step(s, n_steps) would replay from the
 * solver's present position, without enqueueing anything or changing the
 * state, so that a later call of that size spends no time building them (for
 * callers that time or bound the latency of their step calls).  Optional.
 * Errors: FVLBM_E_ARG, FVLBM_E_STATE, FVLBM_E_DEVICE. */
fvlbm_status fvlbm_prepare(fvlbm_solver *s, int64_t n_steps);

/*
 * Step 6: rho [n_cells], u [2*n_cells] (either may be NULL) and
 * stats [4] = {mass = sum A_i rho_i, velocity residual of Eq. 32 against the
 * snapshot taken residual_lag steps earlier (or -1 if none yet), time, steps}
 * (may be NULL).  Reductions run in FP64 on the device.  Syncs the stream.
 * Returns FVLBM_E_DIVERGED if any rho or u is not finite.
 */
fvlbm_status fvlbm_macros(fvlbm_solver *s, double *rho, double *u, double *stats);

/*
 * For callers that cannot allocate device memory or sync (code under HIP graph
 * capture, tight serving loops): Step 6 as fvlbm_macros computes it, written
 * to the caller's device arrays and enqueued on the solver's stream, with no
 * allocation, no copy to the host and no sync.
 *   rho_dev   [n_cells] device array (may be NULL), u_dev [2*n_cells] (may be NULL)
 *   stats_dev [2] device array: {mass = sum A_i rho_i, 1 if any rho or u is not finite else 0}
 * The partial sums and the flag live in a static scratch of the library, one
 * copy per GPU: meshes of at most 16,777,216 cells (FVLBM_E_ARG beyond), and
 * calls that overlap on one GPU (several host threads or streams) race on it.
 * Errors: FVLBM_E_ARG, FVLBM_E_STATE, FVLBM_E_DEVICE (launch failures only).
 */
fvlbm_status fvlbm_macros_noalloc(fvlbm_solver *s, double *rho_dev, double *u_dev, double *stats_dev);

/* Copy the distributions out / in (FP64, [cell][alpha], input cell order).  Sync. */
fvlbm_status fvlbm_get_f(fvlbm_solver *s, double *f);
fvlbm_status fvlbm_set_f(fvlbm_solver *s, const double *f);

/* One evaluation of RHS (Eq. 10) at the current state, FP64 out, [cell][alpha]. Sync. */
fvlbm_status fvlbm_rhs(fvlbm_solver *s, double *rhs);

/* Raw checkpoint of the solver state (storage precision).  state_bytes() tells the size. */
size_t fvlbm_checkpoint_bytes(const fvlbm_solver *s);
fvlbm_status fvlbm_checkpoint(fvlbm_solver *s, void *host_buf, size_t bytes);
fvlbm_status fvlbm_restore(fvlbm_solver *s, const void *host_buf, size_t bytes);

/* Release a solver (its caller-owned state buffer is not touched) or a mesh.
 * Either order is safe: a mesh destroyed while solvers still use it stays
 * alive until the last of them is destroyed, and a solver destroyed while a
 * batch holds it stays alive until that batch is destroyed (the batch then
 * refuses to step, FVLBM_E_STATE).  A second destroy of the same handle is a
 * no-op until the memory is released; after that the handle is invalid.
 * The solver's stream is synchronized before anything is freed. */
void fvlbm_solver_destroy(fvlbm_solver *s);
void fvlbm_mesh_destroy(fvlbm_mesh *mesh);

/* Force on a wall group (post-processing for the force coefficients of Sections 3.3-3.4, whose
 * formula the paper takes from elsewhere; here the discrete momentum flux through the wall faces):
 *   F = sum over the group's faces of sum_a e_a (e_a . n dl) f_P,a,
 * with n dl the outward normal of the fluid cell times the face length and f_P the wall value of
 * Eq. 18, which is the face value of every direction at a wall (Eq. 11).  This is the force the
 * fluid exerts on the wall (pressure rho/3 plus the non-equilibrium stress), per unit depth.
 * FP64 from the stored state; syncs the stream.
 *   force[2]  (may be NULL) receives (Fx, Fy)
 *   n_faces   (may be NULL) receives the number of the group's faces
 *   face_p    (may be NULL) receives p = rho/3 of each face's border cell, n_faces values, in the
 *             order the faces appear in the bface arrays given to fvlbm_create_mesh
 * Errors: FVLBM_E_ARG (null solver, group out of range or not a wall), FVLBM_E_DEVICE. */
fvlbm_status fvlbm_wall_force(fvlbm_solver *s, int32_t group, double force[2], int32_t *n_faces, double *face_p);

/*
 * Batched solves: several solvers (each with its own mesh, parameters and
 * state) advanced by shared launches, one work unit per (solver, cell tile).
 * All solvers must use the same scheme and storage and the same stream.
 * fvlbm_batch_step() advances every member by n_steps; the launches of 8 steps
 * (and of the powers of two below for the rest of a call) are built once into
 * HIP graphs and replayed.
 * The per-cell arithmetic is the same as fvlbm_step(): a member's result does
 * not depend on the other members.  Errors: FVLBM_E_ARG, FVLBM_E_PARAM, FVLBM_E_DEVICE.
 */
fvlbm_status fvlbm_batch_create(fvlbm_solver *const *solvers, int32_t n, fvlbm_batch **out);
fvlbm_status fvlbm_batch_step(fvlbm_batch *b, int64_t n_steps);
/* The velocity residual of Eq. 32 of every member (as fvlbm_macros reports it: against the
 * snapshot residual_lag steps earlier, -1 until two snapshots exist) and its step count:
 * out[2 i] = residual, out[2 i + 1] = steps of member i, in the order given to
 * fvlbm_batch_create.  One sync of the batch's stream for all members (the residual is
 * formed on the device in FP64 when a step count reaches a multiple of the lag).
 * Errors: FVLBM_E_ARG, FVLBM_E_STATE, FVLBM_E_DEVICE. */
fvlbm_status fvlbm_batch_residuals(fvlbm_batch *b, double *out);

/* Replaces the batch's members (continuous batching: requests join and leave
 * between calls), keeping its schedule and its instantiated graphs.  The graphs'
 * kernel nodes are re-pointed in place at the new members' descriptors and work
 * units (grid and LDS size follow); a graph built when the batch held another set
 * of cell kinds (triangle, quadrilateral) is rebuilt at the next step instead.
 * Each member advances exactly as alone (Section 2.4.2 per cell; the other
 * members do not enter its arithmetic).
 *   solvers, n   the new members, the same constraints as fvlbm_batch_create and
 *                the batch's scheme, storage and stream; a member may stay, leave or
 *                join.  Members that leave and were destroyed while the batch held
 *                them are freed here.
 * Synchronizes the batch's stream.  Errors: FVLBM_E_ARG (also: the new members'
 * tiles do not fit the LDS at the batch's tile size), FVLBM_E_PARAM, FVLBM_E_NOMEM,
 * FVLBM_E_DEVICE; on error the batch keeps its old members. */
fvlbm_status fvlbm_batch_set_members(fvlbm_batch *b, fvlbm_solver *const *solvers, int32_t n);
/* Remove one member from a batch (a request that has finished): the batch keeps its
 * other members in their order and its graphs, re-pointed as by
 * fvlbm_batch_set_members, which this call is a shorthand for.  The solver itself
 * is not destroyed; it can be stepped alone or joined to a batch again.
 * Synchronizes the batch's stream.  Errors: FVLBM_E_ARG (null arguments, or the
 * solver is not a member), FVLBM_E_STATE (it is the last member: destroy the
 * batch instead), and those of fvlbm_batch_set_members; on error the batch keeps
 * its members. */
fvlbm_status fvlbm_batch_remove(fvlbm_batch *b, fvlbm_solver *s);
/* How many graphs the batch has instantiated, and how many times a membership
 * change re-pointed an instantiated graph instead (fvlbm_batch_set_members).
 * Errors: FVLBM_E_ARG. */
fvlbm_status fvlbm_batch_graph_counts(const fvlbm_batch *b, int64_t *built, int64_t *repointed);

/* Destroys the batch (not its members, which stay usable alone) and frees members
 * that were destroyed while the batch held them. */
void fvlbm_batch_destroy(fvlbm_batch *b);

/* Launch schedule: tile size in cells (one workgroup per tile: a multiple of 64
 * from 64 to 512), whether tiles are renumbered so that each XCD walks one contiguous
 * range of tiles (neighbouring tiles then share that XCD's L2), and the launch
 * form `persistent`: 0 one workgroup per tile; 1 a persistent grid sized to
 * the resident capacity takes tiles from a device work queue (one ticket
 * counter per XCD, each over its own contiguous range of tiles, stealing from
 * the others when its own is used up; Euler and RK stages, other stages as 0),
 * so fast workgroups take more tiles and none waits for a new launch; the
 * queue lives with the solver's or batch's tile tables and every launch leaves
 * it cleared, so launches of one solver or batch must stay ordered on its
 * stream (as the library issues them); 2 one workgroup per tile with one
 * more wave (two when the larger halo ring of any tile holds more than 64
 * cells) that loads the tile's halo and forms the ring-1 gradients beside
 * the tile's own (single solvers, tiles of 64 or 128 cells, Euler and RK
 * stages; elsewhere it acts as 0); with 64-cell tiles and per-value storage
 * two more waves take half of each cell's directions, so a workgroup runs four
 * waves of 64 (one halo wave).  A batch takes 0 or 1.  A schedule never
 * changes the per-cell arithmetic: results are bitwise identical under every
 * schedule.
 * Errors: FVLBM_E_ARG (unsupported tile size, or tile plus halo do not fit
 * the LDS a workgroup may use: 160 KiB on gfx950). */
fvlbm_status fvlbm_set_schedule(fvlbm_solver *s, int32_t block, int32_t xcd_remap, int32_t persistent);

/* Moves a solver's later work to another stream (after syncing the one it was
 * on), e.g. a solver prepared on a side stream and then handed to the stream
 * its batch runs on.  Errors: FVLBM_E_ARG, FVLBM_E_STATE (a batch holds it:
 * members keep the batch's stream), FVLBM_E_DEVICE. */
fvlbm_status fvlbm_set_stream(fvlbm_solver *s, void *hip_stream);
fvlbm_status fvlbm_get_schedule(const fvlbm_solver *s, int32_t *block, int32_t *xcd_remap, int32_t *persistent);
fvlbm_status fvlbm_batch_set_schedule(fvlbm_batch *b, int32_t block, int32_t xcd_remap, int32_t persistent);
/* The schedule a batch launches with (after fvlbm_batch_set_schedule, fvlbm_batch_autotune, or the
 * one fvlbm_batch_create chose).  Errors: FVLBM_E_ARG. */
fvlbm_status fvlbm_batch_get_schedule(const fvlbm_batch *b, int32_t *block, int32_t *xcd_remap, int32_t *persistent);

/* Autotuner: times every supported schedule (tile sizes 64, 128, 256, 512 and
 * the multiples of 64 that split the cells into about 1-4 tiles per compute
 * unit, each with and without XCD remap, each launch form) for trial_steps steps (HIP
 * events on the solver's or batch's stream; after one untimed run, the faster of
 * two timed runs), keeps the fastest, and restores
 * the state, step counters and residual snapshots to what they were, so the
 * solve continues exactly as without tuning.  best_ms (may be NULL) receives
 * the chosen schedule's time per step.  Syncs the stream.
 * Errors: FVLBM_E_ARG, FVLBM_E_NOMEM, FVLBM_E_DEVICE. */
fvlbm_status fvlbm_autotune(fvlbm_solver *s, int32_t trial_steps, double *best_ms);
fvlbm_status fvlbm_batch_autotune(fvlbm_batch *b, int32_t trial_steps, double *best_ms);

const char *fvlbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FVLBM_H */
