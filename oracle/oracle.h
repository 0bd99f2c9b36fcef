/*
 * Reference oracle for the temporal-adaptive finite-volume Euler path.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, sequential FP64
 * implementation written to check the GPU library against.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or constant with the GPU library.
 *
 * What it computes (Couteyen Carpaye, Roman, Brenner, J. Comput. Sci. 2017):
 *   - the finite-volume integral form with Godunov upwind fluxes, Sec. 2.1,
 *     Eq. (1), for the 3D Euler equations of an ideal gas (no source term);
 *   - one iteration of the temporal adaptive scheme, Sec. 2.2, Alg. 2:
 *     per-cell time step, classification in levels tau with
 *     dt = 2^tau * dt_min, 2^theta subiterations with the level rule of
 *     Alg. 2, neighbours at most one level apart;
 *   - the cost model C(tau) = 2^(theta-tau) |Omega(tau)| of Sec. 2.2, which
 *     is what the cell-update counter counts;
 *   - moving meshes (ALE): fluxes through faces moving with their nodes,
 *     and cell volumes that follow the swept volumes (the geometric
 *     conservation law), with the face geometry kept fixed -- the form
 *     Sec. 2.1 describes for slow relative motion;
 *   - a predictor/corrector form of every level step (time_order 2),
 *     following the order of the steps of Alg. 2: predictor fluxes,
 *     prediction, slower neighbours seen at the interpolated time, corrector
 *     fluxes, correction.  The paper takes its interface formulas from a
 *     cited report; the form here is this oracle's own reading (Heun's
 *     method per level step, linear-in-time prediction of the slower side,
 *     one shared time-integrated flux per face).
 * Readings where the paper is silent (flux accumulation for the slower side,
 * exact Riemann solver, MUSCL least squares with Barth-Jespersen limiting,
 * CFL formula, level margin) are listed in the project design notes.
 *
 * Parity pins: every function below is checked by the CPU tests against a
 * closed form, an invariant, brute force or a value printed in the paper.
 */
#ifndef TAFV_ORACLE_H
#define TAFV_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_E_ARG = -1, ORC_E_MESH = -2, ORC_E_STATE = -3,
       ORC_E_NUMERIC = -7 };
enum { ORC_BC_WALL = 0, ORC_BC_TRANSMIT = 1 };
enum { ORC_GUESS_TR = 0, ORC_GUESS_GIVEN = 1 };

typedef struct {
  double gamma;        /* ratio of specific heats */
  double cfl;          /* Courant number of the per-cell time step */
  double newton_tol;   /* relative-change stop test of the p* Newton solve */
  double level_margin; /* relative margin delta of the level classification */
  int32_t max_levels;  /* L: levels are 0..L-1 */
  int32_t order;       /* 1 = piecewise constant, 2 = MUSCL least squares */
  int32_t newton_max_iter;
  int32_t boundary;    /* ORC_BC_WALL or ORC_BC_TRANSMIT for every boundary face */
  int32_t reclassify;  /* 1: reclassify at every iteration start; 0: only once */
  int32_t time_order;  /* 1: forward Euler per level step; 2: predictor and
                          corrector per level step (see orc_advance) */
} orc_params;

typedef struct {
  int64_t subiterations, cell_updates, face_solves, newton_updates,
          newton_fallbacks, vacuum_faces;
  int64_t cells_per_level[8];
  int32_t theta, phase;
  double dt_min, t_reached;
  double wall_impulse[3];
} orc_stats;

/* Result of one exact Riemann solve in the face-normal frame. */
typedef struct {
  double p_star, u_star;
  int32_t newton_updates; /* Newton updates until the stop test passed */
  int32_t fallback;       /* 1 if bisection had to take over */
  int32_t vacuum;         /* 1 if the data generate vacuum */
} orc_riemann_out;

typedef struct orc_mesh orc_mesh;
typedef struct orc_state orc_state;

/* --- mesh ------------------------------------------------------------ */
int orc_mesh_build(int64_t n_nodes, const double* xyz, int64_t n_tets,
                   const int64_t* tets, orc_mesh** out);
void orc_mesh_free(orc_mesh* m);
int orc_mesh_counts(const orc_mesh* m, int64_t* n_cells, int64_t* n_faces,
                    int64_t* n_boundary);
/* vol[n_cells], centroid[n_cells][3], face_L[n_faces], face_R[n_faces]
 * (-1 on the boundary), face_area[n_faces][3] (outward from L),
 * face_centroid[n_faces][3], cell_faces[n_cells][4]; any may be NULL. */
int orc_mesh_geometry(const orc_mesh* m, double* vol, double* centroid,
                      int64_t* face_L, int64_t* face_R, double* face_area,
                      double* face_centroid, int64_t* cell_faces);

/* --- exact Riemann problem (normal frame: rho, u_n, p) ---------------- */
int orc_riemann_solve(double gamma, const double* wl, const double* wr,
                      double tol, int32_t max_iter, int32_t guess_mode,
                      double guess, orc_riemann_out* out);
/* Sample the solution at similarity coordinate xi = x/t: w_out = rho,u_n,p.
 * Returns 0 if the sample lies left of the contact (or in the left part of
 * a vacuum fan), 1 otherwise. */
int orc_riemann_sample(double gamma, const double* wl, const double* wr,
                       const orc_riemann_out* rs, double xi, double* w_out);
/* Godunov flux through an oriented face: wl, wr are primitive
 * (rho,u,v,w,p); area is the area vector pointing from L to R.  For a wall
 * face wr is ignored and the mirror problem is solved.  flux[5] receives
 * |A| * F(W(0)) . n.  Returns the Riemann solve diagnostics in *out. */
int orc_face_flux(double gamma, const double* wl, const double* wr,
                  const double* area, int32_t kind, double tol,
                  int32_t max_iter, int32_t guess_mode, double guess,
                  double* flux, orc_riemann_out* out);

/* ALE flux through a face moving with normal speed xi along area/|area|:
 * the Riemann problem sampled at x/t = xi, flux |A| (F(W) . n - xi U(W));
 * a wall moves with the face (no mass through it, momentum p* n |A|, work
 * p* xi |A|). */
int orc_face_flux_moving(double gamma, const double* wl, const double* wr,
                         const double* area, double xi, int32_t kind, double tol,
                         int32_t max_iter, double* flux, orc_riemann_out* out);

/* --- reconstruction --------------------------------------------------- */
/* Unlimited and limited least-squares gradients of the primitive
 * variables, grad[n_cells][3][5] (d/dx, d/dy, d/dz of rho,u,v,w,p). */
int orc_gradients(const orc_mesh* m, const orc_params* prm,
                  const double* prim, double* grad_raw, double* grad_lim);

/* --- time step and levels ------------------------------------------- */
int orc_classify(const orc_mesh* m, const orc_params* prm, const double* cons,
                 double* dt, int8_t* levels, double* dt_min, int32_t* theta);

/* --- solver state ----------------------------------------------------- */
int orc_state_new(const orc_mesh* m, const orc_params* prm,
                  const double* prim, orc_state** out);
void orc_state_free(orc_state* s);
/* Overwrite the full schedule state: conserved cons[n][5], accumulators
 * accum[n][5], levels[n], phase, theta, dt_min, time.  With time_order 2
 * only phase 0 is accepted (mid-iteration the predictions are state too). */
int orc_state_set(orc_state* s, const double* cons, const double* accum,
                  const int8_t* levels, int32_t phase, int32_t theta,
                  double dt_min, double t);
/* Run n subiterations of dt_min each.
 * time_order 1: every face whose faster side starts a step is computed once
 *   from the current states, and its flux times the faster side's step is
 *   added to both cells; a cell applies its sum when its own step ends.
 * time_order 2: each level step [a, a + 2^tau dt_min] is a predictor and a
 *   corrector.  Predictor, at the step start: fluxes phi0 from the states at
 *   that time, and the cell's prediction D = 2^tau dt_min sum(+-phi0) / V.
 *   A cell's state at a time inside its step is U + w D, w the fraction of
 *   the step elapsed (w = 1 at the step's end): this is how a slower
 *   neighbour is seen mid-step.  Corrector, at the end of the face's step
 *   (its faster side's): fluxes phi1 from the states U + w D at that time,
 *   and q = dt_f (phi0 + phi1) / 2 added to both cells as in time_order 1.
 *   On one level this is Heun's method; q is shared by both cells, so the
 *   scheme stays conservative across levels. */
int orc_advance(orc_state* s, int64_t n_subiterations);
/* Level tau computed in subiteration s (1-based) of an iteration with
 * levels 0..theta (Alg. 2). */
int32_t orc_subiteration_level(int64_t s, int32_t theta);

/* Threads the per-cell and per-face loops run on: 1 in the plain build,
 * the OpenMP thread count in the timing build (same bits either way). */
int32_t orc_threads(void);
int orc_state_read(const orc_state* s, double* cons, double* accum,
                   int8_t* levels);
int orc_state_stats(const orc_state* s, orc_stats* out);
/* Moving mesh: node velocities [n_nodes][3]; faces move with the mean of
 * their nodes, sweep volume w_f . A_f; the face geometry stays fixed and
 * the cell volumes follow the swept volumes (geometric conservation law);
 * a cell ending its step sets V' = V + swept, U' = (V U + flux sum) / V'.
 * time_order 1 only; checkpoints (orc_state_set) are refused afterwards. */
int orc_state_motion(orc_state* s, const double* node_vel);
/* current cell volumes [n_cells] */
int orc_state_volumes(const orc_state* s, double* vol);

#ifdef __cplusplus
}
#endif
#endif
