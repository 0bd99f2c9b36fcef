/*
 * Reference oracle: temporal-adaptive explicit finite volumes for the 3D
 * Euler equations on tetrahedra, plain sequential FP64 C.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written for clarity, not speed:
 * every step is taken in the order the method states it, on whole arrays,
 * with no blocking or fusion.
 *
 * Paper: Couteyen Carpaye, Roman, Brenner, "Design and Analysis of a
 * Task-based Parallelization over a Runtime System of an Explicit
 * Finite-Volume CFD Code with Adaptive Time Stepping", J. Comput. Sci. 2017.
 *   Sec. 2.1, Eq. (1): cell averages change by the sum of face fluxes,
 *                      fluxes from a Riemann problem per face (Godunov).
 *   Sec. 2.2, Alg. 2:  per-cell time step, level classification,
 *                      2^theta subiterations, level rule per subiteration,
 *                      neighbour levels differ by at most one.
 *   Sec. 2.2:          cost C(tau) = 2^(theta-tau) |Omega(tau)|.
 * Textbook pieces the paper does not spell out:
 *   exact Riemann solver, Newton on p*, sampling: E. F. Toro, "Riemann
 *     Solvers and Numerical Methods for Fluid Dynamics", 3rd ed., ch. 4;
 *   least-squares gradients and the limiter: T. J. Barth, D. C. Jespersen,
 *     AIAA paper 89-0366 (1989).
 *
 * Timing build: compiled with -fopenmp, the per-cell and per-face loops
 * marked ORC_PARALLEL_FOR or ORC_OMP run on all host threads.  Each
 * iteration of such a loop writes only its own cell's or face's entries and
 * every floating-point sum keeps its sequential order (a cell adds its faces
 * in local face order; the reductions are of integers and flags; dt_min is
 * a minimum), so the timing build computes the same bits as the sequential
 * one.  The wall-impulse sum stays sequential.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#define ORC_OMP(x) _Pragma(#x)
#else
#define ORC_OMP(x)
#endif
#define ORC_PARALLEL_FOR ORC_OMP(omp parallel for schedule(static))

int32_t orc_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

/* ====================================================================== */
/* Mesh and geometry                                                       */
/* ====================================================================== */

struct orc_mesh {
  int64_t nc, nf, nb;
  double* vol;     /* [nc]        cell volume                           */
  double* xc;      /* [nc][3]     cell centroid                         */
  int64_t* fL;     /* [nf]        lower cell id                         */
  int64_t* fR;     /* [nf]        higher cell id, -1 on the boundary    */
  double* af;      /* [nf][3]     area vector, pointing out of fL       */
  double* xf;      /* [nf][3]     face centroid                         */
  int64_t* c2f;    /* [nc][4]     face opposite local vertex m          */
  int64_t nn;      /* node count                                        */
  int64_t* fn;     /* [nf][3]     sorted node ids of the face           */
};

typedef struct {
  int64_t v[3]; /* sorted vertex ids */
  int64_t cell;
  int32_t local; /* local face index = the vertex it is opposite to */
} face_rec;

static int cmp_face_rec(const void* a, const void* b) {
  const face_rec* x = (const face_rec*)a;
  const face_rec* y = (const face_rec*)b;
  for (int k = 0; k < 3; ++k) {
    if (x->v[k] < y->v[k]) return -1;
    if (x->v[k] > y->v[k]) return 1;
  }
  if (x->cell < y->cell) return -1;
  if (x->cell > y->cell) return 1;
  return 0;
}

static void sort3(int64_t* v) {
  int64_t t;
  if (v[0] > v[1]) { t = v[0]; v[0] = v[1]; v[1] = t; }
  if (v[1] > v[2]) { t = v[1]; v[1] = v[2]; v[2] = t; }
  if (v[0] > v[1]) { t = v[0]; v[0] = v[1]; v[1] = t; }
}

static double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

void orc_mesh_free(orc_mesh* m) {
  if (!m) return;
  free(m->vol); free(m->xc); free(m->fL); free(m->fR);
  free(m->af); free(m->xf); free(m->c2f); free(m->fn);
  free(m);
}

/* Tets must be positively oriented: det[x1-x0, x2-x0, x3-x0] > 0.  A face
 * is the sorted triple of its vertex ids; one owner makes it a boundary
 * face, two an interior face, more is an error. */
int orc_mesh_build(int64_t n_nodes, const double* xyz, int64_t n_tets,
                   const int64_t* tets, orc_mesh** out) {
  if (!out || n_nodes < 4 || n_tets < 1 || !xyz || !tets) return ORC_E_ARG;
  *out = NULL;
  orc_mesh* m = (orc_mesh*)calloc(1, sizeof(orc_mesh));
  if (!m) return ORC_E_ARG;
  m->nc = n_tets;
  m->vol = (double*)malloc(sizeof(double) * n_tets);
  m->xc = (double*)malloc(sizeof(double) * 3 * n_tets);
  m->c2f = (int64_t*)malloc(sizeof(int64_t) * 4 * n_tets);
  face_rec* rec = (face_rec*)malloc(sizeof(face_rec) * 4 * n_tets);
  if (!m->vol || !m->xc || !m->c2f || !rec) {
    free(rec); orc_mesh_free(m); return ORC_E_ARG;
  }
  for (int64_t t = 0; t < n_tets; ++t) {
    const int64_t* v = tets + 4 * t;
    for (int k = 0; k < 4; ++k)
      if (v[k] < 0 || v[k] >= n_nodes) { free(rec); orc_mesh_free(m); return ORC_E_MESH; }
    const double* p0 = xyz + 3 * v[0];
    const double* p1 = xyz + 3 * v[1];
    const double* p2 = xyz + 3 * v[2];
    const double* p3 = xyz + 3 * v[3];
    double e1[3], e2[3], e3[3], c[3];
    for (int k = 0; k < 3; ++k) { e1[k] = p1[k] - p0[k]; e2[k] = p2[k] - p0[k]; e3[k] = p3[k] - p0[k]; }
    cross3(e2, e3, c);
    double det = dot3(e1, c);
    if (!(det > 0.0)) { free(rec); orc_mesh_free(m); return ORC_E_MESH; }
    m->vol[t] = det / 6.0;
    for (int k = 0; k < 3; ++k) m->xc[3 * t + k] = 0.25 * (p0[k] + p1[k] + p2[k] + p3[k]);
    for (int f = 0; f < 4; ++f) {
      face_rec* r = rec + 4 * t + f;
      int q = 0;
      for (int k = 0; k < 4; ++k) if (k != f) r->v[q++] = v[k];
      sort3(r->v);
      r->cell = t;
      r->local = f;
    }
  }
  qsort(rec, (size_t)(4 * n_tets), sizeof(face_rec), cmp_face_rec);

  /* count faces */
  int64_t nf = 0, nb = 0;
  for (int64_t i = 0; i < 4 * n_tets;) {
    int64_t j = i + 1;
    while (j < 4 * n_tets && rec[j].v[0] == rec[i].v[0] && rec[j].v[1] == rec[i].v[1] &&
           rec[j].v[2] == rec[i].v[2]) ++j;
    if (j - i > 2) { free(rec); orc_mesh_free(m); return ORC_E_MESH; }
    if (j - i == 2 && rec[i].cell == rec[i + 1].cell) { free(rec); orc_mesh_free(m); return ORC_E_MESH; }
    if (j - i == 1) ++nb;
    ++nf;
    i = j;
  }
  m->nf = nf;
  m->nb = nb;
  m->nn = n_nodes;
  m->fL = (int64_t*)malloc(sizeof(int64_t) * nf);
  m->fR = (int64_t*)malloc(sizeof(int64_t) * nf);
  m->af = (double*)malloc(sizeof(double) * 3 * nf);
  m->xf = (double*)malloc(sizeof(double) * 3 * nf);
  m->fn = (int64_t*)malloc(sizeof(int64_t) * 3 * nf);
  if (!m->fL || !m->fR || !m->af || !m->xf || !m->fn) {
    free(rec); orc_mesh_free(m); return ORC_E_ARG;
  }
  int64_t f = 0;
  for (int64_t i = 0; i < 4 * n_tets;) {
    int64_t j = i + 1;
    while (j < 4 * n_tets && rec[j].v[0] == rec[i].v[0] && rec[j].v[1] == rec[i].v[1] &&
           rec[j].v[2] == rec[i].v[2]) ++j;
    /* records are sorted by cell within a key, so rec[i] has the lower id */
    m->fL[f] = rec[i].cell;
    m->fR[f] = (j - i == 2) ? rec[i + 1].cell : -1;
    m->c2f[4 * rec[i].cell + rec[i].local] = f;
    if (j - i == 2) m->c2f[4 * rec[i + 1].cell + rec[i + 1].local] = f;
    for (int k = 0; k < 3; ++k) m->fn[3 * f + k] = rec[i].v[k];
    const double* a = xyz + 3 * rec[i].v[0];
    const double* b = xyz + 3 * rec[i].v[1];
    const double* c = xyz + 3 * rec[i].v[2];
    double ab[3], ac[3], n[3], d[3];
    for (int k = 0; k < 3; ++k) { ab[k] = b[k] - a[k]; ac[k] = c[k] - a[k]; }
    cross3(ab, ac, n);
    for (int k = 0; k < 3; ++k) {
      m->af[3 * f + k] = 0.5 * n[k];
      m->xf[3 * f + k] = (a[k] + b[k] + c[k]) / 3.0;
      d[k] = m->xf[3 * f + k] - m->xc[3 * m->fL[f] + k];
    }
    if (dot3(m->af + 3 * f, d) < 0.0)
      for (int k = 0; k < 3; ++k) m->af[3 * f + k] = -m->af[3 * f + k];
    ++f;
    i = j;
  }
  free(rec);
  *out = m;
  return ORC_OK;
}

int orc_mesh_counts(const orc_mesh* m, int64_t* n_cells, int64_t* n_faces,
                    int64_t* n_boundary) {
  if (!m) return ORC_E_ARG;
  if (n_cells) *n_cells = m->nc;
  if (n_faces) *n_faces = m->nf;
  if (n_boundary) *n_boundary = m->nb;
  return ORC_OK;
}

int orc_mesh_geometry(const orc_mesh* m, double* vol, double* centroid,
                      int64_t* face_L, int64_t* face_R, double* face_area,
                      double* face_centroid, int64_t* cell_faces) {
  if (!m) return ORC_E_ARG;
  if (vol) memcpy(vol, m->vol, sizeof(double) * m->nc);
  if (centroid) memcpy(centroid, m->xc, sizeof(double) * 3 * m->nc);
  if (face_L) memcpy(face_L, m->fL, sizeof(int64_t) * m->nf);
  if (face_R) memcpy(face_R, m->fR, sizeof(int64_t) * m->nf);
  if (face_area) memcpy(face_area, m->af, sizeof(double) * 3 * m->nf);
  if (face_centroid) memcpy(face_centroid, m->xf, sizeof(double) * 3 * m->nf);
  if (cell_faces) memcpy(cell_faces, m->c2f, sizeof(int64_t) * 4 * m->nc);
  return ORC_OK;
}

/* ====================================================================== */
/* Ideal gas                                                               */
/* ====================================================================== */

/* primitive (rho,u,v,w,p) -> conserved (rho, rho u, rho v, rho w, E) with
 * E = p/(gamma-1) + rho |u|^2 / 2 */
static void prim_to_cons(double g, const double* w, double* u) {
  u[0] = w[0];
  u[1] = w[0] * w[1];
  u[2] = w[0] * w[2];
  u[3] = w[0] * w[3];
  u[4] = w[4] / (g - 1.0) + 0.5 * w[0] * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
}

/* conserved -> primitive, p = (gamma-1)(E - |m|^2/(2 rho)) */
static void cons_to_prim(double g, const double* u, double* w) {
  w[0] = u[0];
  w[1] = u[1] / u[0];
  w[2] = u[2] / u[0];
  w[3] = u[3] / u[0];
  w[4] = (g - 1.0) * (u[4] - 0.5 * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0]);
}

/* ====================================================================== */
/* Exact Riemann solver (Toro ch. 4), normal frame                         */
/* ====================================================================== */

/* Pressure function of one side and its derivative: shock branch for
 * p > pk, rarefaction branch otherwise. */
static double pressure_fn(double g, double p, double rk, double pk, double ak,
                          double* dfdp) {
  if (p > pk) {
    double A = 2.0 / ((g + 1.0) * rk);
    double B = (g - 1.0) / (g + 1.0) * pk;
    double s = sqrt(A / (p + B));
    *dfdp = s * (1.0 - (p - pk) / (2.0 * (B + p)));
    return (p - pk) * s;
  }
  double z = (g - 1.0) / (2.0 * g);
  *dfdp = pow(p / pk, -(g + 1.0) / (2.0 * g)) / (rk * ak);
  return 2.0 * ak / (g - 1.0) * (pow(p / pk, z) - 1.0);
}

static double total_fn(double g, double p, const double* wl, const double* wr,
                       double al, double ar, double* dfdp) {
  double dl, dr;
  double f = pressure_fn(g, p, wl[0], wl[2], al, &dl) +
             pressure_fn(g, p, wr[0], wr[2], ar, &dr) + (wr[1] - wl[1]);
  if (dfdp) *dfdp = dl + dr;
  return f;
}

/* Two-rarefaction approximation of p* (Toro ch. 4). */
static double guess_two_rarefaction(double g, const double* wl, const double* wr,
                                    double al, double ar) {
  double z = (g - 1.0) / (2.0 * g);
  double num = al + ar - 0.5 * (g - 1.0) * (wr[1] - wl[1]);
  double den = al / pow(wl[2], z) + ar / pow(wr[2], z);
  return pow(num / den, 1.0 / z);
}

int orc_riemann_solve(double g, const double* wl, const double* wr, double tol,
                      int32_t max_iter, int32_t guess_mode, double guess,
                      orc_riemann_out* out) {
  if (!wl || !wr || !out) return ORC_E_ARG;
  if (!(wl[0] > 0.0) || !(wl[2] > 0.0) || !(wr[0] > 0.0) || !(wr[2] > 0.0)) return ORC_E_STATE;
  memset(out, 0, sizeof(*out));
  double al = sqrt(g * wl[2] / wl[0]);
  double ar = sqrt(g * wr[2] / wr[0]);
  /* pressure positivity condition: vacuum is generated otherwise */
  if (2.0 * (al + ar) / (g - 1.0) <= wr[1] - wl[1]) {
    out->vacuum = 1;
    out->p_star = 0.0;
    out->u_star = 0.5 * ((wl[1] + 2.0 * al / (g - 1.0)) + (wr[1] - 2.0 * ar / (g - 1.0)));
    return ORC_OK;
  }
  double p = (guess_mode == ORC_GUESS_GIVEN) ? guess : 0.0;
  if (guess_mode != ORC_GUESS_GIVEN || !(p > 0.0) || !isfinite(p))
    p = guess_two_rarefaction(g, wl, wr, al, ar);
  int converged = 0;
  for (int32_t k = 1; k <= max_iter; ++k) {
    double df;
    double f = total_fn(g, p, wl, wr, al, ar, &df);
    double pn = p - f / df;
    /* f is increasing and concave, so a non-positive Newton iterate can
     * only come from the right of the root, which then lies in (0, p):
     * step down by a fixed factor instead (the stop test cannot pass). */
    if (!(pn > 0.0)) pn = p / 16.0;
    out->newton_updates = k;
    double change = 2.0 * fabs(pn - p) / (pn + p);
    p = pn;
    if (change < tol) { converged = 1; break; }
  }
  if (!converged) {
    /* bisection on [0, hi] with f(0) < 0 < f(hi) */
    out->fallback = 1;
    double lo = 0.0, hi = fmax(wl[2], wr[2]);
    for (int k = 0; k < 2100 && total_fn(g, hi, wl, wr, al, ar, NULL) <= 0.0; ++k) hi *= 2.0;
    for (int k = 0; k < 400; ++k) {
      double mid = 0.5 * (lo + hi);
      if (total_fn(g, mid, wl, wr, al, ar, NULL) > 0.0) hi = mid; else lo = mid;
      if (hi - lo <= tol * hi) break;
    }
    p = 0.5 * (lo + hi);
  }
  double dl, dr;
  double fl = pressure_fn(g, p, wl[0], wl[2], al, &dl);
  double fr = pressure_fn(g, p, wr[0], wr[2], ar, &dr);
  out->p_star = p;
  out->u_star = 0.5 * (wl[1] + wr[1]) + 0.5 * (fr - fl);
  return ORC_OK;
}

/* Sampling of the exact solution at x/t = xi (Toro ch. 4, including the
 * vacuum-generation case). */
int orc_riemann_sample(double g, const double* wl, const double* wr,
                       const orc_riemann_out* rs, double xi, double* w) {
  double al = sqrt(g * wl[2] / wl[0]);
  double ar = sqrt(g * wr[2] / wr[0]);
  double g1 = (g - 1.0) / (g + 1.0);
  double z = (g - 1.0) / (2.0 * g);
  if (rs->vacuum) {
    double sl_tail = wl[1] + 2.0 * al / (g - 1.0);
    double sr_tail = wr[1] - 2.0 * ar / (g - 1.0);
    if (xi <= wl[1] - al) { w[0] = wl[0]; w[1] = wl[1]; w[2] = wl[2]; return 0; }
    if (xi < sl_tail) {
      double c = 2.0 / (g + 1.0) + g1 / al * (wl[1] - xi);
      w[0] = wl[0] * pow(c, 2.0 / (g - 1.0));
      w[1] = 2.0 / (g + 1.0) * (al + 0.5 * (g - 1.0) * wl[1] + xi);
      w[2] = wl[2] * pow(c, 2.0 * g / (g - 1.0));
      return 0;
    }
    if (xi <= sr_tail) { w[0] = 0.0; w[1] = 0.0; w[2] = 0.0; return xi < 0.5 * (sl_tail + sr_tail) ? 0 : 1; }
    if (xi < wr[1] + ar) {
      double c = 2.0 / (g + 1.0) - g1 / ar * (wr[1] - xi);
      w[0] = wr[0] * pow(c, 2.0 / (g - 1.0));
      w[1] = 2.0 / (g + 1.0) * (-ar + 0.5 * (g - 1.0) * wr[1] + xi);
      w[2] = wr[2] * pow(c, 2.0 * g / (g - 1.0));
      return 1;
    }
    w[0] = wr[0]; w[1] = wr[1]; w[2] = wr[2];
    return 1;
  }
  double ps = rs->p_star, us = rs->u_star;
  if (xi <= us) {
    /* left of the contact */
    if (ps > wl[2]) {
      double sl = wl[1] - al * sqrt((g + 1.0) / (2.0 * g) * ps / wl[2] + (g - 1.0) / (2.0 * g));
      if (xi <= sl) { w[0] = wl[0]; w[1] = wl[1]; w[2] = wl[2]; }
      else {
        double r = ps / wl[2];
        w[0] = wl[0] * (r + g1) / (g1 * r + 1.0);
        w[1] = us; w[2] = ps;
      }
    } else {
      double shl = wl[1] - al;
      if (xi <= shl) { w[0] = wl[0]; w[1] = wl[1]; w[2] = wl[2]; }
      else {
        double astar = al * pow(ps / wl[2], z);
        double stl = us - astar;
        if (xi >= stl) {
          w[0] = wl[0] * pow(ps / wl[2], 1.0 / g);
          w[1] = us; w[2] = ps;
        } else {
          double c = 2.0 / (g + 1.0) + g1 / al * (wl[1] - xi);
          w[0] = wl[0] * pow(c, 2.0 / (g - 1.0));
          w[1] = 2.0 / (g + 1.0) * (al + 0.5 * (g - 1.0) * wl[1] + xi);
          w[2] = wl[2] * pow(c, 2.0 * g / (g - 1.0));
        }
      }
    }
    return 0;
  }
  /* right of the contact */
  if (ps > wr[2]) {
    double sr = wr[1] + ar * sqrt((g + 1.0) / (2.0 * g) * ps / wr[2] + (g - 1.0) / (2.0 * g));
    if (xi >= sr) { w[0] = wr[0]; w[1] = wr[1]; w[2] = wr[2]; }
    else {
      double r = ps / wr[2];
      w[0] = wr[0] * (r + g1) / (g1 * r + 1.0);
      w[1] = us; w[2] = ps;
    }
  } else {
    double shr = wr[1] + ar;
    if (xi >= shr) { w[0] = wr[0]; w[1] = wr[1]; w[2] = wr[2]; }
    else {
      double astar = ar * pow(ps / wr[2], z);
      double str = us + astar;
      if (xi <= str) {
        w[0] = wr[0] * pow(ps / wr[2], 1.0 / g);
        w[1] = us; w[2] = ps;
      } else {
        double c = 2.0 / (g + 1.0) - g1 / ar * (wr[1] - xi);
        w[0] = wr[0] * pow(c, 2.0 / (g - 1.0));
        w[1] = 2.0 / (g + 1.0) * (-ar + 0.5 * (g - 1.0) * wr[1] + xi);
        w[2] = wr[2] * pow(c, 2.0 * g / (g - 1.0));
      }
    }
  }
  return 1;
}

/* Physical Euler flux through unit normal n of primitive state w. */
static void euler_flux(double g, const double* w, const double* n, double* F) {
  double un = w[1] * n[0] + w[2] * n[1] + w[3] * n[2];
  double E = w[4] / (g - 1.0) + 0.5 * w[0] * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
  F[0] = w[0] * un;
  F[1] = w[0] * un * w[1] + w[4] * n[0];
  F[2] = w[0] * un * w[2] + w[4] * n[1];
  F[3] = w[0] * un * w[3] + w[4] * n[2];
  F[4] = un * (E + w[4]);
}

/* kind: 0 interior, 1 wall (mirror state), 2 transmissive (copy state) */
int orc_face_flux(double g, const double* wl, const double* wr, const double* area,
                  int32_t kind, double tol, int32_t max_iter, int32_t guess_mode,
                  double guess, double* flux, orc_riemann_out* out) {
  orc_riemann_out dummy;
  if (!out) out = &dummy;
  memset(out, 0, sizeof(*out));
  double amag = sqrt(dot3(area, area));
  if (!(amag > 0.0)) return ORC_E_ARG;
  double n[3] = {area[0] / amag, area[1] / amag, area[2] / amag};
  if (kind == 2) {
    double F[5];
    euler_flux(g, wl, n, F);
    for (int k = 0; k < 5; ++k) flux[k] = amag * F[k];
    return ORC_OK;
  }
  double unl = wl[1] * n[0] + wl[2] * n[1] + wl[3] * n[2];
  double nl[3] = {wl[0], unl, wl[4]};
  if (kind == 1) {
    double nr[3] = {wl[0], -unl, wl[4]};
    int rc = orc_riemann_solve(g, nl, nr, tol, max_iter, guess_mode, guess, out);
    if (rc) return rc;
    /* a wall lets no mass or energy through; the star pressure pushes */
    flux[0] = 0.0;
    flux[1] = amag * out->p_star * n[0];
    flux[2] = amag * out->p_star * n[1];
    flux[3] = amag * out->p_star * n[2];
    flux[4] = 0.0;
    return ORC_OK;
  }
  double unr = wr[1] * n[0] + wr[2] * n[1] + wr[3] * n[2];
  double nr[3] = {wr[0], unr, wr[4]};
  int rc = orc_riemann_solve(g, nl, nr, tol, max_iter, guess_mode, guess, out);
  if (rc) return rc;
  double ws[3];
  int side = orc_riemann_sample(g, nl, nr, out, 0.0, ws);
  const double* src = side == 0 ? wl : wr;
  double un_src = side == 0 ? unl : unr;
  double w[5];
  w[0] = ws[0];
  for (int k = 0; k < 3; ++k) w[1 + k] = ws[1] * n[k] + (src[1 + k] - un_src * n[k]);
  w[4] = ws[2];
  double F[5];
  euler_flux(g, w, n, F);
  for (int k = 0; k < 5; ++k) flux[k] = amag * F[k];
  return ORC_OK;
}

/* ALE form of the face flux (Sec. 2.1: the face's own velocity enters the
 * flux of a moving mesh): the face moves with normal speed xi along the
 * unit normal n = A/|A|; the Riemann problem of the normal frame is sampled
 * on the face's path, x/t = xi, and the flux through the moving face is
 * |A| (F(W(xi)) . n - xi U(W(xi))).  A wall moves with the face: its mirror
 * state has normal velocity 2 xi - u_nL, so the contact follows the wall,
 * no mass crosses it, the star pressure pushes (p* n |A|) and does the
 * work p* xi |A|.  A transmissive face takes W = W_L.  xi = 0 gives the
 * fluxes of orc_face_flux up to rounding. */
int orc_face_flux_moving(double g, const double* wl, const double* wr, const double* area,
                         double xi, int32_t kind, double tol, int32_t max_iter,
                         double* flux, orc_riemann_out* out) {
  orc_riemann_out dummy;
  if (!out) out = &dummy;
  memset(out, 0, sizeof(*out));
  double amag = sqrt(dot3(area, area));
  if (!(amag > 0.0)) return ORC_E_ARG;
  double n[3] = {area[0] / amag, area[1] / amag, area[2] / amag};
  double w[5];
  if (kind == 2) {
    for (int k = 0; k < 5; ++k) w[k] = wl[k];
  } else {
    double unl = wl[1] * n[0] + wl[2] * n[1] + wl[3] * n[2];
    double nl[3] = {wl[0], unl, wl[4]};
    if (kind == 1) {
      double nr[3] = {wl[0], 2.0 * xi - unl, wl[4]};
      int rc = orc_riemann_solve(g, nl, nr, tol, max_iter, ORC_GUESS_TR, 0.0, out);
      if (rc) return rc;
      flux[0] = 0.0;
      for (int k = 0; k < 3; ++k) flux[1 + k] = amag * out->p_star * n[k];
      flux[4] = amag * out->p_star * xi;
      return ORC_OK;
    }
    double unr = wr[1] * n[0] + wr[2] * n[1] + wr[3] * n[2];
    double nr[3] = {wr[0], unr, wr[4]};
    int rc = orc_riemann_solve(g, nl, nr, tol, max_iter, ORC_GUESS_TR, 0.0, out);
    if (rc) return rc;
    double ws[3];
    int side = orc_riemann_sample(g, nl, nr, out, xi, ws);
    const double* src = side == 0 ? wl : wr;
    double un_src = side == 0 ? unl : unr;
    w[0] = ws[0];
    for (int k = 0; k < 3; ++k) w[1 + k] = ws[1] * n[k] + (src[1 + k] - un_src * n[k]);
    w[4] = ws[2];
  }
  double F[5], U[5];
  euler_flux(g, w, n, F);
  prim_to_cons(g, w, U);
  for (int k = 0; k < 5; ++k) flux[k] = amag * (F[k] - xi * U[k]);
  return ORC_OK;
}

/* ====================================================================== */
/* Least-squares gradients and Barth-Jespersen limiter                     */
/* ====================================================================== */

/* Neighbour j of cell i across its local face m: position and primitive
 * state.  A boundary face gives the mirror ghost: the cell centroid
 * reflected in the face plane, with the normal velocity reversed on a wall
 * and the state copied on a transmissive boundary. */
/* On a moving mesh (sF not NULL) a wall moves with its face: the ghost's
 * normal velocity is 2 xi - u_n, xi = sF / |A| the face's normal speed. */
static void neighbour(const orc_mesh* m, int32_t bc, const double* sF, const double* prim,
                      int64_t i, int mloc, double* pos, double* w) {
  int64_t f = m->c2f[4 * i + mloc];
  if (m->fR[f] >= 0) {
    int64_t j = (m->fL[f] == i) ? m->fR[f] : m->fL[f];
    for (int k = 0; k < 3; ++k) pos[k] = m->xc[3 * j + k];
    for (int k = 0; k < 5; ++k) w[k] = prim[5 * j + k];
    return;
  }
  const double* a = m->af + 3 * f;
  double amag = sqrt(dot3(a, a));
  double n[3] = {a[0] / amag, a[1] / amag, a[2] / amag};
  double d[3];
  for (int k = 0; k < 3; ++k) d[k] = m->xf[3 * f + k] - m->xc[3 * i + k];
  double h = dot3(d, n);
  for (int k = 0; k < 3; ++k) pos[k] = m->xc[3 * i + k] + 2.0 * h * n[k];
  const double* wi = prim + 5 * i;
  for (int k = 0; k < 5; ++k) w[k] = wi[k];
  if (bc == ORC_BC_WALL) {
    double un = wi[1] * n[0] + wi[2] * n[1] + wi[3] * n[2];
    if (sF) un -= sF[f] / amag;
    for (int k = 0; k < 3; ++k) w[1 + k] = wi[1 + k] - 2.0 * un * n[k];
  }
}

static int invert_sym3(const double* M, double* Minv) {
  /* M = [a b c; b d e; c e f] */
  double a = M[0], b = M[1], c = M[2], d = M[4], e = M[5], f = M[8];
  double A = d * f - e * e, B = c * e - b * f, C = b * e - c * d;
  double det = a * A + b * B + c * C;
  if (!(det != 0.0)) return ORC_E_MESH;
  double D = a * f - c * c, E = b * c - a * e, F = a * d - b * b;
  Minv[0] = A / det; Minv[1] = B / det; Minv[2] = C / det;
  Minv[3] = B / det; Minv[4] = D / det; Minv[5] = E / det;
  Minv[6] = C / det; Minv[7] = E / det; Minv[8] = F / det;
  return ORC_OK;
}

static int gradients_core(const orc_mesh* m, const orc_params* prm, const double* sF,
                          const double* prim, double* grad_raw, double* grad_lim) {
  int bad = 0;
  ORC_OMP(omp parallel for schedule(static) reduction(| : bad))
  for (int64_t i = 0; i < m->nc; ++i) {
    const double* xi = m->xc + 3 * i;
    const double* wi = prim + 5 * i;
    double pos[4][3], wn[4][5];
    double M[9] = {0}, b[3][5];
    memset(b, 0, sizeof(b));
    for (int j = 0; j < 4; ++j) {
      neighbour(m, prm->boundary, sF, prim, i, j, pos[j], wn[j]);
      double d[3] = {pos[j][0] - xi[0], pos[j][1] - xi[1], pos[j][2] - xi[2]};
      double wgt = 1.0 / dot3(d, d);
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[3 * r + c] += wgt * d[r] * d[c];
      for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 5; ++k) b[r][k] += wgt * d[r] * (wn[j][k] - wi[k]);
    }
    double Minv[9];
    if (invert_sym3(M, Minv)) {
      bad = 1;
      continue;
    }
    double G[3][5];
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 5; ++k)
        G[r][k] = Minv[3 * r + 0] * b[0][k] + Minv[3 * r + 1] * b[1][k] + Minv[3 * r + 2] * b[2][k];
    if (grad_raw)
      for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 5; ++k) grad_raw[15 * i + 5 * r + k] = G[r][k];
    if (!grad_lim) continue;
    for (int k = 0; k < 5; ++k) {
      double wmax = wi[k], wmin = wi[k];
      for (int j = 0; j < 4; ++j) {
        if (wn[j][k] > wmax) wmax = wn[j][k];
        if (wn[j][k] < wmin) wmin = wn[j][k];
      }
      double psi = 1.0;
      for (int j = 0; j < 4; ++j) {
        int64_t f = m->c2f[4 * i + j];
        double r[3];
        for (int q = 0; q < 3; ++q) r[q] = m->xf[3 * f + q] - xi[q];
        double delta = G[0][k] * r[0] + G[1][k] * r[1] + G[2][k] * r[2];
        double phi = 1.0;
        if (delta > 0.0) phi = fmin(1.0, (wmax - wi[k]) / delta);
        else if (delta < 0.0) phi = fmin(1.0, (wmin - wi[k]) / delta);
        if (phi < psi) psi = phi;
      }
      for (int r = 0; r < 3; ++r) grad_lim[15 * i + 5 * r + k] = psi * G[r][k];
    }
  }
  return bad ? ORC_E_MESH : ORC_OK;
}

int orc_gradients(const orc_mesh* m, const orc_params* prm, const double* prim,
                  double* grad_raw, double* grad_lim) {
  if (!m || !prm || !prim) return ORC_E_ARG;
  return gradients_core(m, prm, NULL, prim, grad_raw, grad_lim);
}

/* ====================================================================== */
/* Time step and levels (Sec. 2.2, Alg. 2: time step computation,          */
/* classification; neighbour levels differ by at most one)                 */
/* ====================================================================== */

/* vol: the cell volumes; sF (NULL on a fixed mesh): per face the rate
 * w_f . A_f of the volume it sweeps, so that its normal speed is
 * sF / |A| and the wave speeds are taken relative to it */
static int classify_core(const orc_mesh* m, const orc_params* prm, const double* cons,
                         const double* vol, const double* sF, double* dt, int8_t* levels,
                         double* dt_min_out, int32_t* theta_out) {
  double g = prm->gamma;
  double dtmin = INFINITY;
  int bad = 0;
  ORC_OMP(omp parallel for schedule(static) reduction(| : bad))
  for (int64_t i = 0; i < m->nc; ++i) {
    double w[5];
    cons_to_prim(g, cons + 5 * i, w);
    if (!(w[0] > 0.0) || !(w[4] > 0.0)) {
      bad = 1;
      dt[i] = INFINITY;
      continue;
    }
    double a = sqrt(g * w[4] / w[0]);
    double s = 0.0;
    for (int j = 0; j < 4; ++j) {
      const double* A = m->af + 3 * m->c2f[4 * i + j];
      double amag = sqrt(dot3(A, A));
      double un = (w[1] * A[0] + w[2] * A[1] + w[3] * A[2]) / amag;
      if (sF) un -= sF[m->c2f[4 * i + j]] / amag;
      s += (fabs(un) + a) * amag;
    }
    dt[i] = prm->cfl * vol[i] / s;
  }
  if (bad) return ORC_E_NUMERIC;
  for (int64_t i = 0; i < m->nc; ++i)
    if (dt[i] < dtmin) dtmin = dt[i];
  int L = prm->max_levels;
  ORC_PARALLEL_FOR
  for (int64_t i = 0; i < m->nc; ++i) {
    int e;
    double q = dt[i] * (1.0 - prm->level_margin) / dtmin;
    frexp(q, &e); /* q = mant * 2^e, mant in [0.5, 1): floor(log2 q) = e - 1 */
    int tau = e - 1;
    if (tau < 0) tau = 0;
    if (tau > L - 1) tau = L - 1;
    levels[i] = (int8_t)tau;
  }
  /* lower-only Jacobi sweeps; L-1 of them reach the fixed point */
  int8_t* tmp = (int8_t*)malloc((size_t)m->nc);
  if (!tmp) return ORC_E_ARG;
  for (int sweep = 0; sweep < L - 1; ++sweep) {
    ORC_PARALLEL_FOR
    for (int64_t i = 0; i < m->nc; ++i) {
      int t = levels[i];
      for (int j = 0; j < 4; ++j) {
        int64_t f = m->c2f[4 * i + j];
        if (m->fR[f] < 0) continue;
        int64_t nb = (m->fL[f] == i) ? m->fR[f] : m->fL[f];
        if (levels[nb] + 1 < t) t = levels[nb] + 1;
      }
      tmp[i] = (int8_t)t;
    }
    memcpy(levels, tmp, (size_t)m->nc);
  }
  free(tmp);
  int theta = 0;
  for (int64_t i = 0; i < m->nc; ++i) if (levels[i] > theta) theta = levels[i];
  if (dt_min_out) *dt_min_out = dtmin;
  if (theta_out) *theta_out = theta;
  return ORC_OK;
}

int orc_classify(const orc_mesh* m, const orc_params* prm, const double* cons,
                 double* dt, int8_t* levels, double* dt_min_out, int32_t* theta_out) {
  if (!m || !prm || !cons || !dt || !levels) return ORC_E_ARG;
  return classify_core(m, prm, cons, m->vol, NULL, dt, levels, dt_min_out, theta_out);
}

/* ====================================================================== */
/* Solver state and the subiteration loop (Alg. 2)                         */
/* ====================================================================== */

struct orc_state {
  const orc_mesh* m;
  orc_params prm;
  double* U;      /* [nc][5] conserved cell averages                     */
  double* R;      /* [nc][5] flux accumulated since the cell last moved  */
  int8_t* lev;    /* [nc]                                                */
  double* dt;     /* [nc] scratch                                        */
  double* prim;   /* [nc][5] scratch                                     */
  double* glim;   /* [nc][3][5] scratch                                  */
  double* q;      /* [nf][5] scratch: dt_f * flux of active faces        */
  uint8_t* act;   /* [nf] scratch                                        */
  /* time_order 2 only */
  double* D;      /* [nc][5] prediction of the cell's current step       */
  double* Ut;     /* [nc][5] scratch: states at one time inside the steps */
  double* phi0;   /* [nf][5] predictor flux of the face's current step   */
  double* phi1;   /* [nf][5] scratch: corrector flux                     */
  /* moving mesh only (orc_state_motion) */
  int32_t moving;
  double* V;      /* [nc] cell volumes                                   */
  double* RV;     /* [nc] swept volume accumulated since the cell moved   */
  double* sF;     /* [nf] volume rate w_f . A_f of each face              */
  double* qv;     /* [nf] scratch: -dt_f sF of the computed faces         */
  int32_t phase, theta, classified;
  double dt_min, t;
  orc_stats st;
};

void orc_state_free(orc_state* s) {
  if (!s) return;
  free(s->U); free(s->R); free(s->lev); free(s->dt); free(s->prim);
  free(s->glim); free(s->q); free(s->act);
  free(s->D); free(s->Ut); free(s->phi0); free(s->phi1);
  free(s->V); free(s->RV); free(s->sF); free(s->qv);
  free(s);
}

int orc_state_new(const orc_mesh* m, const orc_params* prm, const double* prim,
                  orc_state** out) {
  if (!m || !prm || !prim || !out) return ORC_E_ARG;
  if (prm->max_levels < 1 || prm->max_levels > 8 || (prm->order != 1 && prm->order != 2) ||
      !(prm->gamma > 1.0) || !(prm->cfl > 0.0) || prm->newton_max_iter < 1 ||
      (prm->time_order != 1 && prm->time_order != 2))
    return ORC_E_ARG;
  for (int64_t i = 0; i < m->nc; ++i) {
    const double* w = prim + 5 * i;
    for (int k = 0; k < 5; ++k) if (!isfinite(w[k])) return ORC_E_STATE;
    if (!(w[0] > 0.0) || !(w[4] > 0.0)) return ORC_E_STATE;
  }
  orc_state* s = (orc_state*)calloc(1, sizeof(orc_state));
  if (!s) return ORC_E_ARG;
  s->m = m;
  s->prm = *prm;
  s->U = (double*)malloc(sizeof(double) * 5 * m->nc);
  s->R = (double*)calloc((size_t)(5 * m->nc), sizeof(double));
  s->lev = (int8_t*)calloc((size_t)m->nc, 1);
  s->dt = (double*)malloc(sizeof(double) * m->nc);
  s->prim = (double*)malloc(sizeof(double) * 5 * m->nc);
  s->glim = (double*)malloc(sizeof(double) * 15 * m->nc);
  s->q = (double*)malloc(sizeof(double) * 5 * m->nf);
  s->act = (uint8_t*)malloc((size_t)m->nf);
  if (!s->U || !s->R || !s->lev || !s->dt || !s->prim || !s->glim || !s->q || !s->act) {
    orc_state_free(s);
    return ORC_E_ARG;
  }
  if (prm->time_order == 2) {
    s->D = (double*)calloc((size_t)(5 * m->nc), sizeof(double));
    s->Ut = (double*)malloc(sizeof(double) * 5 * m->nc);
    s->phi0 = (double*)calloc((size_t)(5 * m->nf), sizeof(double));
    s->phi1 = (double*)malloc(sizeof(double) * 5 * m->nf);
    if (!s->D || !s->Ut || !s->phi0 || !s->phi1) {
      orc_state_free(s);
      return ORC_E_ARG;
    }
  }
  for (int64_t i = 0; i < m->nc; ++i) prim_to_cons(prm->gamma, prim + 5 * i, s->U + 5 * i);
  *out = s;
  return ORC_OK;
}

int orc_state_set(orc_state* s, const double* cons, const double* accum,
                  const int8_t* levels, int32_t phase, int32_t theta, double dt_min,
                  double t) {
  if (!s || !cons || !accum || !levels) return ORC_E_ARG;
  if (theta < 0 || theta >= s->prm.max_levels || phase < 0 || phase >= (1 << theta))
    return ORC_E_ARG;
  if (s->prm.time_order == 2 && phase != 0) return ORC_E_ARG;
  if (s->moving) return ORC_E_ARG;
  memcpy(s->U, cons, sizeof(double) * 5 * s->m->nc);
  memcpy(s->R, accum, sizeof(double) * 5 * s->m->nc);
  memcpy(s->lev, levels, (size_t)s->m->nc);
  s->phase = phase;
  s->theta = theta;
  s->dt_min = dt_min;
  s->t = t;
  s->classified = 1;
  return ORC_OK;
}

/* Level computed in subiteration s = 1..2^theta (Alg. 2): start from 0
 * and take every tmp = 1..theta for which 2^tmp divides s-1. */
int32_t orc_subiteration_level(int64_t s, int32_t theta) {
  int32_t tau = 0;
  for (int32_t tmp = 1; tmp <= theta; ++tmp)
    if ((s - 1) % ((int64_t)1 << tmp) == 0) tau = tmp;
  return tau;
}

static int classify_state(orc_state* s) {
  int rc = s->moving ? classify_core(s->m, &s->prm, s->U, s->V, s->sF, s->dt, s->lev,
                                     &s->dt_min, &s->theta)
                     : orc_classify(s->m, &s->prm, s->U, s->dt, s->lev, &s->dt_min, &s->theta);
  if (rc) return rc;
  for (int k = 0; k < 8; ++k) s->st.cells_per_level[k] = 0;
  for (int64_t i = 0; i < s->m->nc; ++i) s->st.cells_per_level[s->lev[i]]++;
  s->classified = 1;
  return ORC_OK;
}

/* Godunov fluxes |A| F . n (Sec. 2.1, Eq. (1)) of every face whose faster
 * side has level <= tau_max, from the cell states cons: primitive
 * variables, limited least-squares gradients at second order (Alg. 2,
 * gradient computation and limitation), reconstruction at the face centroid,
 * exact Riemann solve (Alg. 2, Riemann solver).  act[f] marks the faces
 * computed; phi of the others is left as it was.  The solve counters are
 * added to the statistics. */
static int face_fluxes(orc_state* s, const double* cons, int tau_max, double* phi) {
  const orc_mesh* m = s->m;
  const orc_params* prm = &s->prm;
  double g = prm->gamma;
  ORC_PARALLEL_FOR
  for (int64_t i = 0; i < m->nc; ++i) cons_to_prim(g, cons + 5 * i, s->prim + 5 * i);
  if (prm->order == 2) {
    int rc = gradients_core(m, prm, s->moving ? s->sF : NULL, s->prim, NULL, s->glim);
    if (rc) return rc;
  }
  int64_t n_solves = 0, n_newton = 0, n_fallback = 0, n_vacuum = 0;
  int bad = 0;
  ORC_OMP(omp parallel for schedule(dynamic, 1024)
          reduction(+ : n_newton, n_fallback, n_vacuum) reduction(| : bad))
  for (int64_t f = 0; f < m->nf; ++f) {
    int64_t L = m->fL[f], R = m->fR[f];
    int tau_f = s->lev[L];
    if (R >= 0 && s->lev[R] < tau_f) tau_f = s->lev[R];
    s->act[f] = (uint8_t)(tau_f <= tau_max);
    if (!s->act[f]) continue;
    double wl[5], wr[5];
    for (int k = 0; k < 5; ++k) wl[k] = s->prim[5 * L + k];
    if (R >= 0) for (int k = 0; k < 5; ++k) wr[k] = s->prim[5 * R + k];
    if (prm->order == 2) {
      double rl[3], rr[3];
      for (int q = 0; q < 3; ++q) rl[q] = m->xf[3 * f + q] - m->xc[3 * L + q];
      for (int k = 0; k < 5; ++k)
        for (int q = 0; q < 3; ++q) wl[k] += s->glim[15 * L + 5 * q + k] * rl[q];
      if (R >= 0) {
        for (int q = 0; q < 3; ++q) rr[q] = m->xf[3 * f + q] - m->xc[3 * R + q];
        for (int k = 0; k < 5; ++k)
          for (int q = 0; q < 3; ++q) wr[k] += s->glim[15 * R + 5 * q + k] * rr[q];
      }
    }
    int kind = (R >= 0) ? 0 : (prm->boundary == ORC_BC_WALL ? 1 : 2);
    orc_riemann_out ro;
    int rc;
    if (s->moving) {
      const double* A = m->af + 3 * f;
      double xi = s->sF[f] / sqrt(dot3(A, A));
      rc = orc_face_flux_moving(g, wl, wr, A, xi, kind, prm->newton_tol, prm->newton_max_iter,
                                phi + 5 * f, &ro);
    } else {
      rc = orc_face_flux(g, wl, wr, m->af + 3 * f, kind, prm->newton_tol,
                         prm->newton_max_iter, ORC_GUESS_TR, 0.0, phi + 5 * f, &ro);
    }
    if (rc) {
      bad = 1;
      continue;
    }
    n_newton += ro.newton_updates;
    n_fallback += ro.fallback;
    n_vacuum += ro.vacuum;
  }
  if (bad) return ORC_E_NUMERIC;
  for (int64_t f = 0; f < m->nf; ++f) n_solves += s->act[f];
  s->st.face_solves += n_solves;
  s->st.newton_updates += n_newton;
  s->st.newton_fallbacks += n_fallback;
  s->st.vacuum_faces += n_vacuum;
  return ORC_OK;
}

/* Flow sum on cells (Alg. 2): each cell adds the time-integrated flux q of
 * its own computed faces in its local face order, -q where it is the face's
 * L side (the flux leaves it), +q otherwise; then the cells whose level
 * step ends at the end of subiteration sub apply their sum. */
static int flow_sum_and_update(orc_state* s, int64_t sub) {
  const orc_mesh* m = s->m;
  ORC_PARALLEL_FOR
  for (int64_t i = 0; i < m->nc; ++i) {
    for (int j = 0; j < 4; ++j) {
      int64_t f = m->c2f[4 * i + j];
      if (!s->act[f]) continue;
      double sign = (m->fL[f] == i) ? -1.0 : 1.0;
      for (int k = 0; k < 5; ++k) s->R[5 * i + k] += sign * s->q[5 * f + k];
      if (s->moving) s->RV[i] += sign * s->qv[f];
    }
  }
  int64_t updates = 0;
  int bad = 0;
  ORC_OMP(omp parallel for schedule(static) reduction(+ : updates) reduction(| : bad))
  for (int64_t i = 0; i < m->nc; ++i) {
    if (sub % ((int64_t)1 << s->lev[i]) != 0) continue;
    if (s->moving) {
      /* geometric conservation: the cell's content V U changes by its flux
       * sum, its volume by the volume its faces swept */
      double v = s->V[i], vn = v + s->RV[i];
      if (!(vn > 0.0)) {
        bad = 1;
        continue;
      }
      for (int k = 0; k < 5; ++k) {
        s->U[5 * i + k] = (v * s->U[5 * i + k] + s->R[5 * i + k]) / vn;
        s->R[5 * i + k] = 0.0;
        if (!isfinite(s->U[5 * i + k])) bad = 1;
      }
      s->V[i] = vn;
      s->RV[i] = 0.0;
    } else {
      for (int k = 0; k < 5; ++k) {
        s->U[5 * i + k] += s->R[5 * i + k] / m->vol[i];
        s->R[5 * i + k] = 0.0;
        if (!isfinite(s->U[5 * i + k])) bad = 1;
      }
    }
    updates++;
  }
  s->st.cell_updates += updates;
  return bad ? ORC_E_NUMERIC : ORC_OK;
}

static int faster_level(const orc_state* s, int64_t f) {
  int t = s->lev[s->m->fL[f]];
  int64_t R = s->m->fR[f];
  if (R >= 0 && s->lev[R] < t) t = s->lev[R];
  return t;
}

/* One subiteration of Alg. 2 with flux accumulation for the slower side,
 * forward Euler per level step:
 *   1. at the start of an iteration (phase 0) every cell is synchronised;
 *      compute time steps and levels;
 *   2. the level of this subiteration is theta at phase 0, else the largest
 *      tau <= theta with 2^tau dividing the phase;
 *   3. every face whose faster side has level <= that tau is computed from
 *      the current states of both cells and its time-integrated flux
 *      2^tau_f dt_min * flux is added to both cells' accumulators;
 *   4. cells whose level step ends now apply their accumulator. */
static int subiteration(orc_state* s) {
  const orc_mesh* m = s->m;
  const orc_params* prm = &s->prm;
  if (s->phase == 0 && (prm->reclassify || !s->classified)) {
    int rc = classify_state(s);
    if (rc) return rc;
  }
  int tau_s = orc_subiteration_level((int64_t)s->phase + 1, s->theta);
  int rc = face_fluxes(s, s->U, tau_s, s->q);
  if (rc) return rc;
  for (int64_t f = 0; f < m->nf; ++f) {
    if (!s->act[f]) continue;
    double dtf = ldexp(s->dt_min, faster_level(s, f));
    for (int k = 0; k < 5; ++k) s->q[5 * f + k] *= dtf;
    if (s->moving) s->qv[f] = -dtf * s->sF[f];
    if (m->fR[f] < 0 && prm->boundary == ORC_BC_WALL)
      for (int k = 0; k < 3; ++k) s->st.wall_impulse[k] += s->q[5 * f + 1 + k];
  }
  int64_t sub = (int64_t)s->phase + 1;
  rc = flow_sum_and_update(s, sub);
  if (rc) return rc;
  s->phase = (int32_t)(sub % ((int64_t)1 << s->theta));
  s->t += s->dt_min;
  s->st.subiterations++;
  return ORC_OK;
}

/* States of every cell at dt_min unit k of the iteration, into Ut.  A cell
 * of level tau is inside its step [a, a + 2^tau) with a a multiple of 2^tau;
 * its state there is U + w D with w = (k - a) / 2^tau, the elapsed fraction
 * of the step (Alg. 2, intensive interpolation).  At a step boundary
 * (k a multiple of 2^tau) the state is U (w = 0) when the step starts at k,
 * and the prediction U + D (w = 1) when the step ends at k. */
static void states_at(orc_state* s, int64_t k, int ending) {
  const orc_mesh* m = s->m;
  for (int64_t i = 0; i < m->nc; ++i) {
    int64_t per = (int64_t)1 << s->lev[i];
    int64_t r = k % per;
    double w = (r == 0) ? (ending ? 1.0 : 0.0) : (double)r / (double)per;
    for (int c = 0; c < 5; ++c)
      s->Ut[5 * i + c] = (w == 0.0) ? s->U[5 * i + c] : s->U[5 * i + c] + w * s->D[5 * i + c];
  }
}

/* One subiteration with a predictor and a corrector per level step:
 *   1. as above: levels at phase 0, the subiteration's level tau_s; the
 *      cells and faces of levels <= tau_s start a step at unit a = phase;
 *   2. predictor: fluxes phi0 of the starting faces from the states at a;
 *      each starting cell of level tau predicts the change of its step,
 *      D = 2^tau dt_min (sum of its faces' +-phi0) / V (Alg. 2, extensive
 *      prediction);
 *   3. corrector: the cells and faces of levels <= upd end a step at unit
 *      a + 1, upd the largest tau <= theta with 2^tau dividing a + 1;
 *      fluxes phi1 of those faces from the states at a + 1, the face's
 *      time-integrated flux q = 2^tau_f dt_min (phi0 + phi1) / 2, added to
 *      both cells (Alg. 2, flow sum on cells, extensive correction); the
 *      cells whose step ends apply their sum. */
static int subiteration2(orc_state* s) {
  const orc_mesh* m = s->m;
  const orc_params* prm = &s->prm;
  if (s->phase == 0 && (prm->reclassify || !s->classified)) {
    int rc = classify_state(s);
    if (rc) return rc;
  }
  int64_t a = s->phase, sub = a + 1;
  int tau_s = orc_subiteration_level(sub, s->theta);
  int upd = 0;
  while (upd < s->theta && sub % ((int64_t)1 << (upd + 1)) == 0) ++upd;

  /* predictor */
  states_at(s, a, 0);
  int rc = face_fluxes(s, s->Ut, tau_s, s->phi0);
  if (rc) return rc;
  for (int64_t i = 0; i < m->nc; ++i) {
    if (s->lev[i] > tau_s) continue;
    double acc[5] = {0, 0, 0, 0, 0};
    for (int j = 0; j < 4; ++j) {
      int64_t f = m->c2f[4 * i + j];
      double sign = (m->fL[f] == i) ? -1.0 : 1.0;
      for (int k = 0; k < 5; ++k) acc[k] += sign * s->phi0[5 * f + k];
    }
    double dtc = ldexp(s->dt_min, s->lev[i]);
    for (int k = 0; k < 5; ++k) s->D[5 * i + k] = dtc * acc[k] / m->vol[i];
  }

  /* corrector */
  states_at(s, sub, 1);
  rc = face_fluxes(s, s->Ut, upd, s->phi1);
  if (rc) return rc;
  for (int64_t f = 0; f < m->nf; ++f) {
    if (!s->act[f]) continue;
    double h = 0.5 * ldexp(s->dt_min, faster_level(s, f));
    for (int k = 0; k < 5; ++k) s->q[5 * f + k] = h * (s->phi0[5 * f + k] + s->phi1[5 * f + k]);
    if (m->fR[f] < 0 && prm->boundary == ORC_BC_WALL)
      for (int k = 0; k < 3; ++k) s->st.wall_impulse[k] += s->q[5 * f + 1 + k];
  }
  rc = flow_sum_and_update(s, sub);
  if (rc) return rc;
  s->phase = (int32_t)(sub % ((int64_t)1 << s->theta));
  s->t += s->dt_min;
  s->st.subiterations++;
  return ORC_OK;
}

int orc_advance(orc_state* s, int64_t n) {
  if (!s || n < 0) return ORC_E_ARG;
  for (int64_t k = 0; k < n; ++k) {
    int rc = s->prm.time_order == 2 ? subiteration2(s) : subiteration(s);
    if (rc) return rc;
  }
  return ORC_OK;
}

/* Moving mesh (ALE with the geometric conservation law, Sec. 2.1): node
 * velocities node_vel [n_nodes][3]; each face moves with the mean velocity
 * of its three nodes, w_f = (v_a + v_b + v_c) / 3 (sorted node ids), and
 * sweeps volume at the rate sF = w_f . A_f.  The face geometry (areas,
 * centroids, reconstruction weights) stays that of the uploaded mesh; the
 * cell volumes evolve by the swept volumes (the conservation law of the
 * geometry), and the fluxes are those of orc_face_flux_moving.  Forward
 * Euler level steps (time_order 1) only.  Takes effect at the next
 * subiteration; pass zeros to stop the motion. */
int orc_state_motion(orc_state* s, const double* node_vel) {
  if (!s || !node_vel || s->prm.time_order != 1) return ORC_E_ARG;
  const orc_mesh* m = s->m;
  for (int64_t k = 0; k < 3 * m->nn; ++k)
    if (!isfinite(node_vel[k])) return ORC_E_ARG;
  if (!s->sF) {
    s->sF = (double*)malloc(sizeof(double) * m->nf);
    s->qv = (double*)calloc((size_t)m->nf, sizeof(double));
    s->V = (double*)malloc(sizeof(double) * m->nc);
    s->RV = (double*)calloc((size_t)m->nc, sizeof(double));
    if (!s->sF || !s->qv || !s->V || !s->RV) return ORC_E_ARG;
    memcpy(s->V, m->vol, sizeof(double) * m->nc);
  }
  for (int64_t f = 0; f < m->nf; ++f) {
    const double* va = node_vel + 3 * m->fn[3 * f];
    const double* vb = node_vel + 3 * m->fn[3 * f + 1];
    const double* vc = node_vel + 3 * m->fn[3 * f + 2];
    double w[3];
    for (int k = 0; k < 3; ++k) w[k] = (va[k] + vb[k] + vc[k]) / 3.0;
    s->sF[f] = dot3(w, m->af + 3 * f);
  }
  s->moving = 1;
  return ORC_OK;
}

int orc_state_volumes(const orc_state* s, double* vol) {
  if (!s || !vol) return ORC_E_ARG;
  memcpy(vol, s->moving ? s->V : s->m->vol, sizeof(double) * s->m->nc);
  return ORC_OK;
}

int orc_state_read(const orc_state* s, double* cons, double* accum, int8_t* levels) {
  if (!s) return ORC_E_ARG;
  if (cons) memcpy(cons, s->U, sizeof(double) * 5 * s->m->nc);
  if (accum) memcpy(accum, s->R, sizeof(double) * 5 * s->m->nc);
  if (levels) memcpy(levels, s->lev, (size_t)s->m->nc);
  return ORC_OK;
}

int orc_state_stats(const orc_state* s, orc_stats* out) {
  if (!s || !out) return ORC_E_ARG;
  *out = s->st;
  out->theta = s->theta;
  out->phase = s->phase;
  out->dt_min = s->dt_min;
  out->t_reached = s->t;
  return ORC_OK;
}
