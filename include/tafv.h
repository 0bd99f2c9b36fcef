/*
 * tafv: temporal-adaptive finite volumes for the 3D Euler equations on
 * tetrahedral meshes, on one AMD Instinct MI355X (gfx950).
 *
 * The method is the explicit temporal adaptive scheme of Couteyen Carpaye,
 * Roman, Brenner, "Design and Analysis of a Task-based Parallelization over
 * a Runtime System of an Explicit Finite-Volume CFD Code with Adaptive Time
 * Stepping", J. Comput. Sci. 2017:
 *   - Sec. 2.1, Eq. (1): each cell average changes by the sum over its faces
 *     of a numerical flux taken from the Riemann problem at the face
 *     (Godunov's method).  Here: ideal gas, no source term, an exact Riemann
 *     solver (Newton on the star pressure p*), first order or MUSCL with
 *     least-squares gradients and the Barth-Jespersen limiter.
 *   - Sec. 2.2, Alg. 2: every cell gets a maximal time step from a CFL
 *     condition; the smallest one is dt_min; a cell of level tau advances
 *     with 2^tau * dt_min; one iteration is 2^theta subiterations; the level
 *     computed in subiteration s is the largest tau <= theta with 2^tau
 *     dividing s-1; neighbours differ by at most one level.  A face between
 *     two levels is computed with the faster side's step and its flux is
 *     accumulated on both sides, so the slower cell applies the sum when its
 *     own step ends and mass, momentum and energy are conserved exactly.
 *   - Sec. 2.2, cost model: the cell-update counter counts
 *     C(tau) = 2^(theta - tau) |Omega(tau)| per iteration.
 *
 * Conventions common to every call
 *   Status: every call returns a tafv_status; nothing aborts or throws.
 *     tafv_last_error() returns a message for the last failure on a context.
 *   Ownership: the caller owns every host array; the library copies inputs
 *     during the call and keeps no caller pointer.  The context owns all
 *     device memory it allocates (with hipMalloc, or with the caller's
 *     allocator: tafv_set_allocator) and frees it in tafv_destroy().
 *   Streams: all device work of a context is enqueued on the HIP stream
 *     given to tafv_create() (NULL: the null stream).  Calls that return
 *     data to the host synchronise that stream; tafv_advance() does not wait
 *     for its work to finish except once per iteration (2^theta
 *     subiterations), when it reads back the new level counts.
 *   Layout: host arrays are row-major in the caller's cell order; the device
 *     layout is internal.
 *   Threading: a context is not thread-safe; distinct contexts are
 *     independent.
 */
#ifndef TAFV_H
#define TAFV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tafv_ctx tafv_ctx;

typedef enum {
  TAFV_OK = 0,
  TAFV_E_ARG = -1,     /* a bad argument (NULL, size, unknown option)        */
  TAFV_E_MESH = -2,    /* index out of range, non-positive volume, a face
                          shared by more than two tets                      */
  TAFV_E_STATE = -3,   /* rho <= 0, p <= 0 or a non-finite initial value     */
  TAFV_E_ORDER = -4,   /* a call out of order (advance before state_init)    */
  TAFV_E_DEVICE = -5,  /* a HIP runtime error; the message has its text      */
  TAFV_E_OOM = -6,     /* device memory allocation failed                    */
  TAFV_E_NUMERIC = -7, /* a non-finite state after a subiteration            */
  TAFV_E_MLP = -8      /* learned guess: no network set, or a non-finite
                          parameter                                         */
} tafv_status;

enum { TAFV_FP64 = 0, TAFV_FP32_FLUX = 1 };
enum { TAFV_GUESS_TR = 0, TAFV_GUESS_MLP = 1 };
enum { TAFV_BC_WALL = 0, TAFV_BC_TRANSMIT = 1 };
/* How face fluxes reach the cell accumulators.  COLOUR: faces are coloured
 * so that no two faces of a colour share a cell; one launch per colour
 * updates both cells of each face with plain read-modify-writes.  GATHER:
 * one launch stores each active face's time-integrated flux, then every cell
 * adds its own faces in its fixed local face order.  Both are atomic-free
 * and deterministic; results agree to rounding. */
enum { TAFV_SCATTER_COLOUR = 0, TAFV_SCATTER_GATHER = 1 };
/* Internal cell order: the caller's order, or a Morton (Z-order) sort of
 * the cell centroids for meshes given in an order without locality.  Host
 * arrays always use the caller's order. */
enum { TAFV_ORDER_CALLER = 0, TAFV_ORDER_MORTON = 1 };

/* Method parameters.  tafv_params_default() fills: gamma 1.4, cfl 0.5,
 * newton_tol 1e-12, level_margin 1e-9, max_levels 5, order 2, precision
 * TAFV_FP64, guess TAFV_GUESS_TR, boundary TAFV_BC_WALL, newton_max_iter
 * 50, reclassify 1, scatter TAFV_SCATTER_GATHER, cell_order TAFV_ORDER_CALLER,
 * guess_stats 0, guess_gate 0, batch 0, guess_strength 0, time_order 1,
 * fuse_faces 0, pipeline_chunks 1. */
typedef struct {
  double gamma;          /* ratio of specific heats, > 1                        */
  double cfl;            /* dt_i = cfl V_i / sum_f (|u_i . n_f| + a_i) |A_f|    */
  double newton_tol;     /* stop when 2|p_{k+1}-p_k|/(p_{k+1}+p_k) < newton_tol */
  double level_margin;   /* tau_i = floor(log2(dt_i (1 - margin) / dt_min))     */
  int32_t max_levels;    /* L in 1..8: levels 0..L-1                            */
  int32_t order;         /* 1: piecewise constant; 2: MUSCL least squares       */
  int32_t precision;     /* TAFV_FP64 or TAFV_FP32_FLUX (reconstruction and flux
                            in FP32; state, accumulators, time steps, levels
                            and the p* Newton solve in FP64)                    */
  int32_t guess;         /* initial p* of the Newton solve: TAFV_GUESS_TR (the
                            two-rarefaction value p_TR), or TAFV_GUESS_MLP
                            (gamma 1.4 and TAFV_SCATTER_GATHER only): where p_TR
                            is inexact and the network's correction y exceeds
                            guess_gate in size, p_TR exp(y); the Newton
                            iteration and its stop test are unchanged          */
  int32_t boundary;      /* every boundary face: wall or transmissive           */
  int32_t newton_max_iter; /* Newton updates before bisection takes over       */
  int32_t reclassify;    /* 1: new levels at every iteration start; 0: keep the
                            first classification (and its dt_min)               */
  int32_t scatter;       /* TAFV_SCATTER_COLOUR or TAFV_SCATTER_GATHER          */
  int32_t cell_order;    /* TAFV_ORDER_CALLER or TAFV_ORDER_MORTON              */
  int32_t guess_stats;   /* 1: count the faces where the two-rarefaction start
                            is inexact (at least one shock) and their Newton
                            updates, also with TAFV_GUESS_TR                    */
  double guess_gate;     /* |y| threshold of the learned correction (>= 0)      */
  int32_t batch;         /* 0: tafv_advance() runs the meshes of the context one
                            after another, the host reading each mesh's level
                            counts once per iteration.  1: batched form (gather
                            scatter only): all meshes are merged into one set of
                            device arrays at the first tafv_state_init(), each
                            keeps its own levels, dt_min, phase and level cap
                            in a device-side schedule, and every subiteration
                            is one fixed sequence of persistent kernels over
                            all meshes, with no host synchronisation (see
                            tafv_batch_config()).  Meshes must all be uploaded
                            before the first tafv_state_init(); checkpoints
                            are read only (tafv_checkpoint_write() is not
                            available) and face logging is not available.  */
  double guess_strength; /* learned guess: the network is evaluated only on
                            faces whose jump strength |u_R - u_L|/a_m +
                            |p_L - p_R|/p_m is at least this (>= 0; 0: every
                            face where p_TR is inexact).  A wave evaluates
                            the network once if any of its faces qualifies. */
  int32_t time_order;    /* 1: each level step is one forward Euler step; the
                            faces of a subiteration are computed once, from
                            the cells' current states.  2: each level step
                            is a predictor and a corrector (Sec. 2.2, Alg. 2:
                            predictor, prediction, interpolation of the
                            slower levels, corrector, correction): predictor
                            fluxes at the step's start give each starting
                            cell a predicted change D of its step; a cell is
                            seen inside its step as U + w D, w the elapsed
                            fraction; corrector fluxes at the end of each
                            face's step give q = dt_f (phi0 + phi1) / 2,
                            added to both cells.  Heun's method on one
                            level, second order in time across levels,
                            conservative; two face solves per face step.
                            Needs TAFV_SCATTER_GATHER and batch 0;
                            checkpoints are written at phase 0 only.      */
  int32_t fuse_faces;    /* 1: at second order in gather mode with
                            time_order 1 on a fixed mesh (no face statistics
                            or logging), a gradient launch over the whole
                            mesh also computes the fluxes of the faces with
                            both cells in one block of 256 cells (and of the
                            boundary faces) from face values held on chip;
                            the face list keeps those faces apart and the
                            flux kernel takes the others.  0 (default): one
                            face list, every face through the flux kernel.
                            Either way the results are the same bits.     */
  int32_t pipeline_chunks; /* K > 1: at second order in gather mode with
                            time_order 1 on a fixed mesh, a subiteration
                            whose gradient, flux and gather launches would
                            each cover the whole mesh runs them as a
                            pipeline over K chunks of consecutive cells
                            (gradient of chunk k + 1, fluxes of the faces
                            whose first cell lies in chunk k, gather of
                            chunk k - 1), so that face values and fluxes
                            are read back soon after they are written.
                            Meshes whose faces span more than a chunk run
                            unchunked.  0 or 1 (default): no pipeline.
                            The results are the same bits either way.     */
} tafv_params;

/* Counters (int64) and schedule state.  Summed over meshes where a call
 * covers several. */
typedef struct {
  int64_t subiterations;   /* subiterations run (one dt_min unit each)        */
  int64_t cell_updates;    /* level steps completed by cells: C(tau) summed    */
  int64_t face_solves;     /* face fluxes computed                             */
  int64_t newton_updates;  /* Newton updates over all face solves              */
  int64_t newton_fallbacks;/* face solves that needed bisection                */
  int64_t vacuum_faces;    /* face solves whose data generate vacuum           */
  int64_t cells_per_level[8]; /* histogram of the latest classification        */
  int32_t theta, phase;    /* highest level; subiteration index within the
                              iteration (0 = every cell synchronised)          */
  double dt_min, t_reached;/* current dt_min; physical time advanced           */
  double wall_impulse[3];  /* time-integrated momentum flux through walls      */
  int64_t guess_faces;     /* face solves where two-rarefaction is inexact
                              (counted with guess_stats or TAFV_GUESS_MLP)     */
  int64_t guess_newton_updates; /* Newton updates on those faces               */
  int64_t guess_rejected;  /* network guesses rejected (non-finite or <= 0)    */
  int64_t guess_used;      /* face solves started from the network's guess     */
  int64_t guess_evaluated; /* faces the network was evaluated for             */
  int64_t newton_hist[3][8]; /* with guess_stats: Newton solves by category
                              and updates.  Category: [0] p* <= min(p_L, p_R)
                              (two rarefactions: the two-rarefaction value is
                              exact), [1] p* between them (one shock), [2]
                              p* above both (two shocks); a wall's mirror
                              state has p_R = p_L.  [c][b]: solves with b + 1
                              Newton updates (b < 7), [c][7]: 8 or more (the
                              bisection fallback included).  Vacuum and
                              transmissive faces are not counted.          */
  int64_t newton_hist_long_updates[3]; /* Newton updates of the [c][7] solves */
} tafv_stats;

/* Fill *p with the defaults listed above. */
tafv_status tafv_params_default(tafv_params* p);

/* Create a context on HIP device `device` (made current for every call on
 * the context).  `hip_stream` is a hipStream_t or NULL.  *out receives the
 * context; on failure *out is NULL. */
tafv_status tafv_create(int device, const tafv_params* params, void* hip_stream,
                        tafv_ctx** out);

/* Free every device buffer of the context and the context itself. */
tafv_status tafv_destroy(tafv_ctx* ctx);

/* Message of the last failed call on ctx (or of tafv_create when ctx is
 * NULL); the string lives until the next call on the context. */
const char* tafv_last_error(const tafv_ctx* ctx);

/* Device memory of the context.  By default the library allocates with
 * hipMalloc and frees with hipFree.  tafv_set_allocator routes every device
 * buffer of the context (mesh arrays, state, schedule lists, face fluxes,
 * network, face log, batch tables, and the temporary buffers of single
 * calls) through the caller's functions instead, for instance a framework's
 * caching allocator, so that the caller owns the memory policy and the
 * library only uses HIP for kernels, copies and the stream:
 *   alloc(bytes, user) returns device memory of the context's device, at
 *     least `bytes` long and 256-byte aligned, usable in stream order on the
 *     context's stream; NULL when it cannot, which the failing call reports
 *     as TAFV_E_OOM after handing back whatever it took (the context stays
 *     usable and can be destroyed);
 *   dealloc(ptr, user) takes back a pointer alloc returned.  The library
 *     calls it once for every such pointer: for a call's temporary buffer
 *     when the call returns, for the context's buffers in tafv_destroy()
 *     (after synchronising the context's stream) or when a buffer is
 *     replaced (network partial sums, face log).
 * A misaligned pointer is handed back and the call fails with
 * TAFV_E_DEVICE.  alloc and dealloc are both given or both NULL (NULL
 * restores hipMalloc / hipFree); TAFV_E_ARG otherwise.  The allocator can
 * only be set or changed while the context holds no device memory: right
 * after tafv_create() (or once everything was freed), else TAFV_E_ORDER. */
tafv_status tafv_set_allocator(tafv_ctx* ctx, void* (*alloc)(size_t bytes, void* user),
                               void (*dealloc)(void* ptr, void* user), void* user);

/* Number of device buffers the context holds (-1 for NULL): the pointers
 * its allocator gave out and has not had back. */
int64_t tafv_device_buffers(const tafv_ctx* ctx);

/* Upload a tetrahedral mesh.  xyz: host [n_nodes][3] node coordinates;
 * tets: host [n_tets][4] node ids, each tet positively oriented
 * (det[x1-x0, x2-x0, x3-x0] > 0).  Faces are the sorted vertex triples;
 * a face with one tet is a boundary face.  Builds the FP64 geometry
 * (volumes, centroids, area vectors, face centroids, least-squares
 * weights; Sec. 2.1 finite volumes), a face colouring and the device
 * arrays.  *mesh_id receives the mesh index (0, 1, ... in upload order).
 * Errors: TAFV_E_MESH as listed above, TAFV_E_OOM, TAFV_E_DEVICE. */
tafv_status tafv_mesh_upload(tafv_ctx* ctx, int64_t n_nodes, const double* xyz,
                             int64_t n_tets, const int64_t* tets, int32_t* mesh_id);

/* Host-only mesh preprocessing, for inspection and tests (no device call):
 * runs the face extraction, geometry and colouring of tafv_mesh_upload on
 * host arrays and returns the face count, boundary face count and colour
 * count.  Optional outputs (NULL to skip; sized with the counts of a first
 * call): face_cells [n_faces][2] = (lower cell, higher cell or -1) in the
 * library's face order (colour-major), face_colour [n_faces],
 * face_area [n_faces][3] (area vector out of the lower cell),
 * cell_neighbours [n_tets][4] (cell across local face m = the face opposite
 * vertex m, -1 on the boundary), recon_coef [n_tets][3][4] (a_mj = c_j . r_m
 * for m < 3: c_j the least-squares coefficient vector of neighbour j, or of
 * its mirror ghost, and r_m the offset of face centroid m from the cell
 * centroid; the reconstruction's change to face centroid m is
 * sum_j a_mj (W_j - W_i), and to face 3 minus the sum of the other three,
 * Sec. 2.1).  Errors as tafv_mesh_upload. */
tafv_status tafv_mesh_inspect(int64_t n_nodes, const double* xyz, int64_t n_tets,
                              const int64_t* tets, int64_t* n_faces, int64_t* n_boundary,
                              int32_t* n_colours, int32_t* face_cells, int8_t* face_colour,
                              double* face_area, int32_t* cell_neighbours,
                              double* recon_coef);

/* Per-mesh level cap (1..8), overriding params.max_levels for that mesh. */
tafv_status tafv_mesh_params(tafv_ctx* ctx, int32_t mesh_id, int32_t max_levels);

/* Moving mesh (Sec. 2.1: an ALE formulation in which the flux through a face
 * takes the face's own velocity into account, and cell volumes that follow
 * the geometric conservation law instead of a recomputed geometry, as for
 * slow relative motion).  node_vel [n_nodes][3] (host, the uploaded node
 * order) are the node velocities; each face moves with the mean velocity w_f
 * of its three nodes and sweeps volume at the rate w_f . A_f.  The face
 * geometry (area vectors, centroids, reconstruction weights) stays that of
 * the uploaded mesh.  From the next subiteration on:
 *   - the Riemann problem of a face is solved in the face's frame and
 *     sampled on the face's path: flux |A| (F(W) . n - xi U(W)), xi the
 *     face's normal speed; a wall moves with its face (no mass through it,
 *     momentum p* n |A|, work p* xi |A|), and so do the wall ghosts of the
 *     gradient;
 *   - a cell ending its step sets V' = V + (volume its faces swept, the
 *     slower side accumulating it like the flux) and U' = (V U + flux sum)
 *     / V';
 *   - time steps use the wave speeds relative to the faces and the current
 *     volumes.
 * The motion is kept until changed (zeros stop it); tafv_state_init() and
 * tafv_state_reset() restore the uploaded volumes.  Needs time_order 1,
 * TAFV_SCATTER_GATHER, the two-rarefaction start without statistics or face
 * logging, and no batch (TAFV_E_ARG otherwise); checkpoints are not written
 * for a moving mesh.  TAFV_E_NUMERIC if a volume becomes non-positive. */
tafv_status tafv_mesh_motion(tafv_ctx* ctx, int32_t mesh_id, const double* node_vel);
/* Current cell volumes, host vol [n_tets] in the caller's order (the
 * uploaded volumes on a fixed mesh). */
tafv_status tafv_volume_read(tafv_ctx* ctx, int32_t mesh_id, double* vol);

/* Set the initial state of a mesh from host prim [n_tets][5] =
 * (rho, u, v, w, p) and reset its schedule (phase 0, t = 0, counters 0).
 * TAFV_E_STATE if rho <= 0, p <= 0 or a value is not finite. */
tafv_status tafv_state_init(tafv_ctx* ctx, int32_t mesh_id, const double* prim);

/* Restore the state given to the last tafv_state_init() of the mesh from a
 * device-side copy (no host transfer) and reset its schedule (phase 0,
 * t = 0).  Cumulative counters are kept.  mesh_id -1: every mesh of the
 * context.  TAFV_E_ORDER without a state. */
tafv_status tafv_state_reset(tafv_ctx* ctx, int32_t mesh_id);

/* Run n_dt_min subiterations (Alg. 2) on every mesh of the context.  The
 * phase persists across calls, so a mesh is time-synchronised only when its
 * phase is 0.  If out is not NULL it receives the counters of this call
 * (summed over meshes) and the schedule state of the last mesh.
 * TAFV_E_ORDER if a mesh has no state; TAFV_E_NUMERIC if a state became
 * non-finite (the call stops at that iteration boundary). */
tafv_status tafv_advance(tafv_ctx* ctx, int64_t n_dt_min, tafv_stats* out);

/* Advance several contexts together, each by n_dt_min subiterations: the
 * same bits as calling tafv_advance() on each in turn, with the work of all
 * of them in flight at once.  This is the task-based execution of Sec. 3
 * and 4 of the paper on one GPU, with a context (its meshes) as the
 * subdomain: `workers` host threads (at most n) each drive contexts w,
 * w + workers, ..., enqueueing one subiteration of each in turn on the
 * context's own stream, so that a context never waits for the others at a
 * subiteration boundary, a quiet context runs ahead of a busy one, and the
 * GPU keeps queued work from other contexts while one waits for the
 * readback of its iteration start.  Contexts must be distinct, not batched
 * (params.batch = 0) and ready to advance; give them different streams for
 * their kernels to overlap on the GPU (contexts on one stream are
 * serialised there).  No other call may use these contexts meanwhile.
 * out (nullable) receives the counters summed over the contexts (cell
 * updates, face solves and subiterations of this call; the device counters
 * since each state_init), the largest theta, and the schedule state of the
 * last context.  On an error the call stops at a subiteration boundary and
 * returns the first failing context's status (its tafv_last_error() has the
 * message; TAFV_E_ARG for the arguments themselves: tafv_last_error(NULL)). */
tafv_status tafv_advance_group(tafv_ctx* const* ctxs, int32_t n, int64_t n_dt_min,
                               int32_t workers, tafv_stats* out);

/* Cumulative counters and schedule state of one mesh since state_init.  In
 * the batched form the face-solve counters (Newton updates, fallbacks,
 * vacuum faces, guess counters, wall impulse) are kept for the whole batch
 * and returned by tafv_advance() only; here they are 0. */
tafv_status tafv_mesh_stats(tafv_ctx* ctx, int32_t mesh_id, tafv_stats* out);

/* Copy the conserved state to host cons [n_tets][5] = (rho, rho u, rho v,
 * rho w, E) and, if levels is not NULL, the levels to host [n_tets].
 * Mid-iteration (phase != 0) a cell shows the state at the start of its
 * current level step, except that with TAFV_SCATTER_GATHER and time_order 1
 * a cell whose faces are all on its own level -- and, at second order,
 * none of whose neighbours has a face on a faster level -- shows the state
 * at the end of its current step: all fluxes of its step are known at the
 * step's start and nothing reads its state before the step ends, so it
 * applies them then.  The accumulator of such a cell is 0.  cons + accum /
 * V is the state at the end of each cell's current step in every case. */
tafv_status tafv_state_read(tafv_ctx* ctx, int32_t mesh_id, double* cons,
                            int8_t* levels);

/* Full schedule state (checkpoint): conserved state, flux accumulators
 * accum [n_tets][5] (time-integrated flux not yet applied by cells whose
 * step has not ended), levels, phase, theta, dt_min and time.  Restoring a
 * checkpoint with tafv_checkpoint_write() and advancing reproduces the
 * uninterrupted run bit for bit. */
tafv_status tafv_checkpoint_read(tafv_ctx* ctx, int32_t mesh_id, double* cons,
                                 double* accum, int8_t* levels, int32_t* phase,
                                 int32_t* theta, double* dt_min, double* t);
tafv_status tafv_checkpoint_write(tafv_ctx* ctx, int32_t mesh_id, const double* cons,
                                  const double* accum, const int8_t* levels,
                                  int32_t phase, int32_t theta, double dt_min,
                                  double t);

/* ---- learned initial guess of the star pressure ----------------------
 * A 6-32-32-1 ReLU network maps the face states, as deviations from the
 * side averages normalised by them,
 * x = (rho_L/rho_m - 1, (u_L - u_m)/a_m, p_L/p_m - 1,
 *      rho_R/rho_m - 1, (u_R - u_m)/a_m, p_R/p_m - 1)
 * (normal velocities; rho_m, u_m, p_m side averages; a_m = sqrt(g p_m/rho_m)) to
 * a correction y ~ ln(p_star / p_TR) of the two-rarefaction value p_TR,
 * p_star the exact star pressure; the Newton solve starts from
 * p_TR exp(y).  BF16 inputs, weights and activations, FP32 accumulation, on
 * the matrix cores.  Parameter vector (TAFV_MLP_PARAMS floats): W1 [32][6]
 * row-major, b1 [32], W2 [32][32] row-major, b2 [32], w3 [32], b3.  The
 * context keeps FP32 master parameters and their BF16 device copy. */
#define TAFV_MLP_PARAMS 1313

/* Change the guess settings of a context (params.guess, guess_gate,
 * guess_strength, guess_stats) between tafv_advance() calls. */
tafv_status tafv_guess_config(tafv_ctx* ctx, int32_t guess, double gate, double strength,
                              int32_t stats);

/* Set / read the FP32 parameters (n must be TAFV_MLP_PARAMS).  Setting
 * resets the optimiser state. */
tafv_status tafv_mlp_set(tafv_ctx* ctx, const float* params, int64_t n);
tafv_status tafv_mlp_get(tafv_ctx* ctx, float* params, int64_t n);

/* Network outputs y[n] for host inputs x [n][6]. TAFV_E_MLP if unset. */
tafv_status tafv_mlp_forward(tafv_ctx* ctx, const float* x, int64_t n, float* y);

/* Gradient of the mean squared error mean((y - t)^2) over the n rows of x
 * [n][6] with targets t[n], computed by the training kernels (BF16 forward,
 * MFMA backward, FP32 sums); grad[TAFV_MLP_PARAMS], *loss the mean squared
 * error (either may be NULL). */
tafv_status tafv_mlp_grad(tafv_ctx* ctx, const float* x, const float* t, int64_t n,
                          float* grad, float* loss);

/* tafv_mlp_grad for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same result, bit for bit, with the device
 * staging of x and t, the per-block partial sums, the gradient and the loss
 * in a scratch area the library holds in a static device array, one per GPU
 * (about 7.2 MB, kept from the first tafv_create() on that GPU until the
 * process ends).  The call allocates nothing; its host arrays are as in
 * tafv_mlp_grad.  n must be 1..TAFV_MLP_GRAD_NOALLOC_MAX_ROWS (TAFV_E_ARG
 * otherwise).  Every call on one GPU shares that GPU's scratch: calls that
 * overlap on one GPU (from several contexts, streams or threads) race and
 * must be serialised by the caller. */
#define TAFV_MLP_GRAD_NOALLOC_MAX_ROWS 65536
tafv_status tafv_mlp_grad_noalloc(tafv_ctx* ctx, const float* x, const float* t, int64_t n,
                                  float* grad, float* loss);

/* Train on the GPU with Adam (lr, beta1 0.9, beta2 0.999, eps 1e-8) for
 * `epochs` passes over the n rows in minibatches of `batch` rows; each
 * epoch visits the rows in the order i -> (a i + b) mod n with a, b drawn
 * from `seed` and the epoch by the splitmix64 generator.  loss[epochs]
 * (nullable) receives the mean squared error of each epoch. */
tafv_status tafv_mlp_train(tafv_ctx* ctx, const float* x, const float* t, int64_t n,
                           int32_t epochs, int32_t batch, float lr, uint64_t seed, float* loss);

/* Face logging: during tafv_advance, a hashed sample (probability `rate`,
 * hash of seed, face and subiteration) of the face solves where the
 * two-rarefaction start is inexact writes a row of 7 floats (the 6 network
 * inputs and the target ln(p_star / p_TR)) until `capacity` rows are held.
 * capacity 0 turns logging off.  Reading returns min(rows logged, cap)
 * rows, in an order fixed by their contents (sorted by their bytes), not
 * by which wave logged them first. */
tafv_status tafv_facelog_config(tafv_ctx* ctx, int64_t capacity, double rate, uint64_t seed);
tafv_status tafv_facelog_read(tafv_ctx* ctx, float* rows, int64_t cap, int64_t* n_rows);

/* ---- batched form (params.batch = 1) ---------------------------------
 * Many independent meshes with staggered level schedules advance together:
 * per subiteration, meshes at an iteration start reclassify (time step,
 * levels, sweeps, level-sorted lists; Sec. 2.2, Alg. 2) while the others
 * skip that work, a one-block kernel derives each mesh's subiteration level
 * and active counts, and the gradient, flux and cell kernels walk the
 * active prefixes of all meshes as one list of tiles.  Results equal those
 * of advancing each mesh on its own (the same per-item arithmetic).
 *
 * tafv_batch_config: graph = 1 captures the subiteration sequence of a
 * tafv_advance(n) call as HIP graphs (up to 32 subiterations each, cached
 * per length) and replays them on the context stream; graph = 0 launches
 * the kernels directly (per-kernel timing works only then).
 * autotune = 1 times candidate launch shapes of the gradient and cell
 * kernels (block size 64, 128, 256 or 512 threads; a persistent grid of 8,
 * 16 or 32 waves per CU taking 1 or 4 groups of wave-sized work units at a
 * time, or one group per block over all cell units) on the first
 * subiteration of the first advance (the cell kernel on scratch copies of
 * the state) and keeps the fastest; the flux kernel takes one tile per
 * block over the static count of face tiles; tune_cache (NULL: none) names a
 * text file that stores the choice per (GPU architecture, precision, order,
 * guess, log2 of the total cell count) and is read before timing.
 * autotune = 0 uses 4 blocks per CU and one tile per grab.  Defaults:
 * graph 1, autotune 1, no cache.  Changing the settings drops the captured
 * graphs.  TAFV_E_ARG on a context without params.batch. */
tafv_status tafv_batch_config(tafv_ctx* ctx, int32_t graph, int32_t autotune,
                              const char* tune_cache);

/* Launch settings in use (n >= 10): info[3k..3k+2] = blocks, unit groups
 * per grab (0: one group per block) and threads per block of the gradient
 * (k = 0), flux (k = 1) and cell (k = 2) kernels; info[9] = 0 defaults,
 * 1 timed by the autotuner, 2 read from the cache file. */
tafv_status tafv_batch_info(tafv_ctx* ctx, int32_t* info, int32_t n);

/* Per-kernel timing: when enabled, tafv_advance() brackets every launch of
 * each kernel class with HIP events on the context stream.
 * tafv_profile_read() returns, per class k < n, the summed launch time in
 * ms, the number of launches and the work items (faces or cells) processed,
 * and the class name in names[k] (static strings).  Reading synchronises
 * the stream and resets the sums. */
tafv_status tafv_profile_enable(tafv_ctx* ctx, int32_t on);
tafv_status tafv_profile_read(tafv_ctx* ctx, int32_t n, double* ms, int64_t* launches,
                              int64_t* items, const char** names, int32_t* n_classes);

#ifdef __cplusplus
}
#endif
#endif
