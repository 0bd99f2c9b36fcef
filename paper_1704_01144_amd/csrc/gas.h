// Ideal-gas helpers and the exact Riemann solver, device side.
//
// The Riemann problem at a face (Godunov's method, Sec. 2.1) is solved
// exactly: the star pressure p* is the root of
//   f(p) = f_L(p) + f_R(p) + (u_R - u_L),
// with, per side K, the shock branch (p > p_K)
//   f_K = (p - p_K) sqrt(A_K / (p + B_K)),  A_K = 2/((g+1) rho_K),
//   B_K = (g-1)/(g+1) p_K,
// and the rarefaction branch (p <= p_K)
//   f_K = 2 a_K/(g-1) ((p/p_K)^z - 1),  z = (g-1)/(2g).
// f is increasing and concave, so Newton converges from any positive start
// (from the left monotonically); the start is the two-rarefaction value.  A
// non-positive Newton iterate can only come from the right of the root and
// is replaced by p/16.  The solve stops when the relative change falls below
// the tolerance; after the update limit it switches to bisection.  The
// solution is sampled at x/t = 0 (E. F. Toro, Riemann Solvers and Numerical
// Methods for Fluid Dynamics, ch. 4).
//
// For g = 1.4 every power in these formulas is a power of the 7th root
// y = x^(1/7): z = 1/7, 1/z = 7, 1/g = 5/7, 2/(g-1) = 5, 2g/(g-1) = 7.
// The inverse 7th root is an FP32 exp2/log2 seed refined by Newton steps on
// z^-7 = x (two in FP64, one in FP32), which replaces the generic pow().
#pragma once

#include <hip/hip_runtime.h>

namespace tafv {

struct Gas {
  double g, gm1, z, inv_z, g1, a_shock, two_gm1, inv_g, sh1, sh2, exp_rho, exp_p;
  int is14;  // g == 1.4: kernels are instantiated with G14 = true
};

inline Gas make_gas(double g) {
  Gas G;
  G.g = g;
  G.gm1 = g - 1.0;
  G.z = (g - 1.0) / (2.0 * g);
  G.inv_z = 1.0 / G.z;
  G.g1 = (g - 1.0) / (g + 1.0);
  G.a_shock = 2.0 / (g + 1.0);
  G.two_gm1 = 2.0 / (g - 1.0);
  G.inv_g = 1.0 / g;
  G.sh1 = (g + 1.0) / (2.0 * g);
  G.sh2 = (g - 1.0) / (2.0 * g);
  G.exp_rho = 2.0 / (g - 1.0);
  G.exp_p = 2.0 * g / (g - 1.0);
  G.is14 = (g == 1.4);
  return G;
}

// ---- powers: generic pow(), or for g = 1.4 powers of the 7th root ------

template <typename T>
__device__ inline T pw(T x, T e) {
  return pow(x, e);
}
template <>
__device__ inline float pw<float>(float x, float e) {
  return powf(x, e);
}

// x^z
template <typename T>
__device__ inline T irt7(T x);

template <bool G14, typename T>
__device__ inline T pow_z(const Gas& G, T x) {
  if (G14) {
    T z = irt7(x), z2 = z * z;
    return x * z2 * z2 * z2;
  }
  return pw<T>(x, (T)G.z);
}
// x^(1/z)
template <bool G14, typename T>
__device__ inline T pow_inv_z(const Gas& G, T x) {
  if (G14) {
    T x2 = x * x, x3 = x2 * x;
    return x3 * x3 * x;
  }
  return pw<T>(x, (T)G.inv_z);
}
// x^(1/g)
template <bool G14, typename T>
__device__ inline T pow_inv_g(const Gas& G, T x) {
  if (G14) {
    T z = irt7(x);
    return x * z * z;
  }
  return pw<T>(x, (T)G.inv_g);
}
// x^(2/(g-1))
template <bool G14, typename T>
__device__ inline T pow_rho(const Gas& G, T x) {
  if (G14) {
    T x2 = x * x;
    return x2 * x2 * x;
  }
  return pw<T>(x, (T)G.exp_rho);
}
// x^(2g/(g-1))
template <bool G14, typename T>
__device__ inline T pow_p(const Gas& G, T x) {
  if (G14) {
    T x2 = x * x, x3 = x2 * x;
    return x3 * x3 * x;
  }
  return pw<T>(x, (T)G.exp_p);
}

// ---- exact Riemann solver: star pressure in FP64 ----------------------

struct Star {
  double p, u;
  int iters, fallback, vacuum;
  // gamma = 1.4 solver: (p/p_K)^(-1/7) of each side at p where that side is
  // a rarefaction (<= 0 otherwise), for the sampling
  double zl = -1.0, zr = -1.0;
};

template <bool G14>
__device__ inline double side_fn(const Gas& G, double p, double rk, double pk, double ak,
                                 double& df) {
  if (p > pk) {
    double A = G.a_shock / rk, B = G.g1 * pk;
    double s = sqrt(A / (p + B));
    df = s * (1.0 - 0.5 * (p - pk) / (B + p));
    return (p - pk) * s;
  }
  double x = p / pk;
  double y = pow_z<G14, double>(G, x);
  df = y / (x * rk * ak);
  return G.two_gm1 * ak * (y - 1.0);
}

template <bool G14>
__device__ inline double total_fn(const Gas& G, double p, double rl, double ul, double pl,
                                  double al, double rr, double ur, double pr, double ar,
                                  double& df) {
  double dl, dr;
  double f = side_fn<G14>(G, p, rl, pl, al, dl) + side_fn<G14>(G, p, rr, pr, ar, dr) + (ur - ul);
  df = dl + dr;
  return f;
}

template <bool G14>
__device__ inline double tr_guess(const Gas& G, double rl, double ul, double pl, double al,
                                  double rr, double ur, double pr, double ar) {
  (void)rl;
  (void)rr;
  double num = al + ar - 0.5 * G.gm1 * (ur - ul);
  double den = al / pow_z<G14, double>(G, pl) + ar / pow_z<G14, double>(G, pr);
  return pow_inv_z<G14, double>(G, num / den);
}

// guess <= 0 or not finite: use the two-rarefaction value
template <bool G14>
__device__ inline Star solve_star(const Gas& G, double rl, double ul, double pl, double al,
                                  double rr, double ur, double pr, double ar, double tol,
                                  int max_iter, double guess) {
  Star s;
  s.iters = 0;
  s.fallback = 0;
  s.vacuum = 0;
  if (G.two_gm1 * (al + ar) <= ur - ul) {
    s.vacuum = 1;
    s.p = 0.0;
    s.u = 0.5 * ((ul + G.two_gm1 * al) + (ur - G.two_gm1 * ar));
    return s;
  }
  double p = guess;
  if (!(p > 0.0) || !isfinite(p)) p = tr_guess<G14>(G, rl, ul, pl, al, rr, ur, pr, ar);
  bool conv = false;
  for (int k = 1; k <= max_iter; ++k) {
    double df;
    double f = total_fn<G14>(G, p, rl, ul, pl, al, rr, ur, pr, ar, df);
    double pn = p - f / df;
    if (!(pn > 0.0)) pn = p * 0.0625;
    s.iters = k;
    double change = 2.0 * fabs(pn - p) / (pn + p);
    p = pn;
    if (change < tol) {
      conv = true;
      break;
    }
  }
  if (!conv) {
    s.fallback = 1;
    double lo = 0.0, hi = fmax(pl, pr), df;
    for (int k = 0; k < 2100 && total_fn<G14>(G, hi, rl, ul, pl, al, rr, ur, pr, ar, df) <= 0.0; ++k)
      hi *= 2.0;
    for (int k = 0; k < 400; ++k) {
      double mid = 0.5 * (lo + hi);
      if (total_fn<G14>(G, mid, rl, ul, pl, al, rr, ur, pr, ar, df) > 0.0)
        hi = mid;
      else
        lo = mid;
      if (hi - lo <= tol * hi) break;
    }
    p = 0.5 * (lo + hi);
  }
  double dl, dr;
  double fl = side_fn<G14>(G, p, rl, pl, al, dl);
  double fr = side_fn<G14>(G, p, rr, pr, ar, dr);
  s.p = p;
  s.u = 0.5 * (ul + ur) + 0.5 * (fr - fl);
  return s;
}

// ---- fast reciprocal, reciprocal square root, inverse 7th root ----------
// Hardware estimates refined by Newton-Raphson steps (quadratic
// convergence): two steps give full FP64 precision for normal inputs, one
// step full FP32 precision.

__device__ inline double frcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ inline float frcp(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}
__device__ inline double frsq(double x) {
  double r = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x;
  r = r * fma(-h * r, r, 1.5);
  return r * fma(-h * r, r, 1.5);
}
__device__ inline float frsq(float x) {
  float r = __builtin_amdgcn_rsqf(x);
  return r * fmaf(-0.5f * x * r, r, 1.5f);
}

// z = x^(-1/7) for x > 0: write x = xs 2^(7q) with xs near 1, seed
// xs^(-1/7) in FP32, scale by 2^-q, then Newton on z^-7 = x,
// z <- z (8 - x z^7) / 7 (two steps in FP64, one in FP32)
template <>
__device__ inline double irt7<double>(double x) {
  int q = ilogb(x) / 7;
  double xs = ldexp(x, -7 * q);
  double z = ldexp((double)exp2f(log2f((float)xs) * (-1.0f / 7.0f)), -q);
  #pragma unroll
  for (int k = 0; k < 2; ++k) {
    double z3 = z * z * z, z7 = z3 * z3 * z;
    z = z * fma(-x, z7, 8.0) * (1.0 / 7.0);
  }
  return z;
}
template <>
__device__ inline float irt7<float>(float x) {
  int q = ilogbf(x) / 7;
  float xs = ldexpf(x, -7 * q);
  float z = ldexpf(exp2f(log2f(xs) * (-1.0f / 7.0f)), -q);
  float z3 = z * z * z, z7 = z3 * z3 * z;
  return z * fmaf(-x, z7, 8.0f) * (1.0f / 7.0f);
}

// ---- gamma = 1.4: division-light exact Riemann solver --------------------
// Per side K: p_K, 1/p_K, 2 a_K/(g-1), 1/(rho_K a_K), sqrt(A_K), B_K.
// Shock branch:       f = (p - p_K) s,  s = sqrt(A_K) / sqrt(p + B_K),
//                     f' = s (1 - (p - p_K) / (2 (p + B_K)));
// rarefaction branch: with x = p/p_K and z = x^(-1/7),
//                     f = 2 a_K/(g-1) (x z^6 - 1),  f' = z^6 / (rho_K a_K).

struct K14 {
  double p, ip, c, iria, sA, B;
};

__device__ inline K14 make_k14(const Gas& G, double p, double a, double ir, double ra) {
  K14 k;
  k.p = p;
  k.ip = frcp(p);
  k.c = G.two_gm1 * a;
  k.iria = ir * ra;
  double t = G.a_shock * ir;
  k.sA = t * frsq(t);
  k.B = G.g1 * p;
  return k;
}

__device__ inline double side14(double p, const K14& k, double& df) {
  if (p > k.p) {
    double r = frsq(p + k.B);
    double s = k.sA * r;
    double d = p - k.p;
    df = s * fma(-0.5 * d, r * r, 1.0);
    return d * s;
  }
  double x = p * k.ip;
  double z = irt7(x);
  double z2 = z * z, z6 = z2 * z2 * z2;
  df = z6 * k.iria;
  return k.c * fma(x, z6, -1.0);
}

// One side at p with z = (p/p_K)^(-1/7) carried along: on the rarefaction
// branch a known z (> 0) is used, an unknown one is computed; on the shock
// branch z is not needed and is reset.
__device__ inline double side14z(double p, const K14& k, double& z, double& df) {
  if (p > k.p) {
    z = -1.0;
    return side14(p, k, df);
  }
  double x = p * k.ip;
  if (!(z > 0.0)) z = irt7(x);
  double z2 = z * z, z6 = z2 * z2 * z2;
  df = z6 * k.iria;
  return k.c * fma(x, z6, -1.0);
}

// The two-rarefaction value p_TR = x^7, x = (a_L + a_R - (g-1)/2 (u_R - u_L))
// / (a_L w_L + a_R w_R), w_K = p_K^(-1/7).  At p = p_TR the rarefaction
// variable of side K is (p_TR/p_K)^(-1/7) = 1 / (x w_K), with no root.
struct TR14 {
  double x, wl, wr, p;
};

__device__ inline TR14 tr14(const Gas& G, double ul, double ur, double al, double ar,
                            const K14& L, const K14& R) {
  TR14 t;
  t.wl = irt7(L.p);
  t.wr = irt7(R.p);
  double num = al + ar - 0.5 * G.gm1 * (ur - ul);
  double den = al * t.wl + ar * t.wr;
  t.x = num * frcp(den);
  double x2 = t.x * t.x, x3 = x2 * t.x;
  t.p = x3 * x3 * t.x;
  return t;
}

// bisection on [0, hi] with f(0) < 0 < f(hi)
__device__ inline double bisect14(const K14& L, const K14& R, double du, double tol) {
  double lo = 0.0, hi = fmax(L.p, R.p), dl, dr;
  for (int k = 0; k < 2100 && side14(hi, L, dl) + side14(hi, R, dr) + du <= 0.0; ++k) hi *= 2.0;
  for (int k = 0; k < 400; ++k) {
    double mid = 0.5 * (lo + hi);
    if (side14(mid, L, dl) + side14(mid, R, dr) + du > 0.0)
      hi = mid;
    else
      lo = mid;
    if (hi - lo <= tol * hi) break;
  }
  return 0.5 * (lo + hi);
}

// guess <= 0 or not finite: the two-rarefaction value (tr, when given,
// holds it).  The rarefaction variables z = (p/p_K)^(-1/7) are carried from
// one Newton iterate to the next: exactly at the two-rarefaction start, and
// across an update p -> p' with |p' - p| < 1e-9 p as z (1 - (p' - p)/(7 p))
// (the dropped term is below 1e-19 relative); otherwise recomputed.
__device__ inline Star solve_star14(const Gas& G, double ul, double ur, double al, double ar,
                                    const K14& L, const K14& R, double tol, int max_iter,
                                    double guess, const TR14* tr = nullptr) {
  Star s;
  s.iters = 0;
  s.fallback = 0;
  s.vacuum = 0;
  if (G.two_gm1 * (al + ar) <= ur - ul) {
    s.vacuum = 1;
    s.p = 0.0;
    s.u = 0.5 * ((ul + G.two_gm1 * al) + (ur - G.two_gm1 * ar));
    return s;
  }
  double p = guess, zl = -1.0, zr = -1.0;
  if (!(p > 0.0) || !isfinite(p)) {
    TR14 t = tr ? *tr : tr14(G, ul, ur, al, ar, L, R);
    p = t.p;
    zl = frcp(t.x * t.wl);
    zr = frcp(t.x * t.wr);
  } else if (tr && p == tr->p) {
    zl = frcp(tr->x * tr->wl);
    zr = frcp(tr->x * tr->wr);
  }
  const double du = ur - ul;
  bool conv = false;
  for (int k = 1; k <= max_iter; ++k) {
    double dl, dr;
    double f = side14z(p, L, zl, dl) + side14z(p, R, zr, dr) + du;
    double pn = p - f * frcp(dl + dr);
    if (!(pn > 0.0)) pn = p * 0.0625;
    s.iters = k;
    conv = 2.0 * fabs(pn - p) < tol * (pn + p);
    if (fabs(pn - p) < 1e-9 * p) {
      double c = 1.0 - (pn - p) * frcp(7.0 * p);
      zl *= c;  // an unknown (negative) z stays unknown
      zr *= c;
    } else {
      zl = zr = -1.0;
    }
    p = pn;
    if (conv) break;
  }
  if (!conv) {
    s.fallback = 1;
    p = bisect14(L, R, du, tol);
    zl = zr = -1.0;
  }
  double dl, dr;
  double fl = side14z(p, L, zl, dl), fr = side14z(p, R, zr, dr);
  s.p = p;
  s.u = 0.5 * (ul + ur) + 0.5 * (fr - fl);
  s.zl = zl;
  s.zr = zr;
  return s;
}

// Sampling at x/t = 0 for gamma = 1.4, precision T.  Per side: rho, u_n, p,
// a, 1/p, 1/a.  Star densities: rarefaction rho_K x^(5/7) = rho_K x z^2,
// shock rho_K (q + g1)/(g1 q + 1); fan states: rho_K c^5, p_K c^7.
template <typename T>
__device__ inline int sample14(const Gas& G, T rl, T ul, T pl, T al, T ipl, T ral, T rr, T ur,
                               T pr, T ar, T ipr, T rar, T ps, T us, T& r, T& u, T& p,
                               double zl = -1.0, double zr = -1.0) {
  const T g1 = (T)G.g1, ash = (T)G.a_shock, sh1 = (T)G.sh1, sh2 = (T)G.sh2;
  const T hg = (T)(0.5 * G.gm1);
  if (0 <= us) {
    if (ps > pl) {
      T q = ps * ipl, t = sh1 * q + sh2;
      T sl = ul - al * (t * frsq(t));
      if (0 <= sl) { r = rl; u = ul; p = pl; }
      else { r = rl * (q + g1) * frcp(g1 * q + 1); u = us; p = ps; }
    } else {
      if (0 <= ul - al) { r = rl; u = ul; p = pl; }
      else {
        T x = ps * ipl, z = zl > 0.0 ? (T)zl : irt7(x), z2 = z * z, z6 = z2 * z2 * z2;
        if (0 >= us - al * x * z6) { r = rl * x * z2; u = us; p = ps; }
        else {
          T c = ash + g1 * ral * ul, c2 = c * c, c5 = c2 * c2 * c;
          r = rl * c5;
          u = ash * (al + hg * ul);
          p = pl * c5 * c2;
        }
      }
    }
    return 0;
  }
  if (ps > pr) {
    T q = ps * ipr, t = sh1 * q + sh2;
    T sr = ur + ar * (t * frsq(t));
    if (0 >= sr) { r = rr; u = ur; p = pr; }
    else { r = rr * (q + g1) * frcp(g1 * q + 1); u = us; p = ps; }
  } else {
    if (0 >= ur + ar) { r = rr; u = ur; p = pr; }
    else {
      T x = ps * ipr, z = zr > 0.0 ? (T)zr : irt7(x), z2 = z * z, z6 = z2 * z2 * z2;
      if (0 <= us + ar * x * z6) { r = rr * x * z2; u = us; p = ps; }
      else {
        T c = ash - g1 * rar * ur, c2 = c * c, c5 = c2 * c2 * c;
        r = rr * c5;
        u = ash * (-ar + hg * ur);
        p = pr * c5 * c2;
      }
    }
  }
  return 1;
}

// ---- sampling at x/t = 0 in precision T --------------------------------
// returns 0 for the left side of the contact, 1 for the right side

template <bool G14, typename T>
__device__ inline int sample0(const Gas& G, T rl, T ul, T pl, T al, T rr, T ur, T pr, T ar,
                              T ps, T us, int vacuum, T& r, T& u, T& p) {
  const T g1 = (T)G.g1, ash = (T)G.a_shock, gm1 = (T)G.gm1;
  if (vacuum) {
    T tl = ul + (T)G.two_gm1 * al, tr = ur - (T)G.two_gm1 * ar;
    if (0 <= ul - al) { r = rl; u = ul; p = pl; return 0; }
    if (0 < tl) {
      T c = ash + g1 / al * ul;
      r = rl * pow_rho<G14, T>(G, c);
      u = ash * (al + (T)0.5 * gm1 * ul);
      p = pl * pow_p<G14, T>(G, c);
      return 0;
    }
    if (0 <= tr) { r = 0; u = 0; p = 0; return 0; }
    if (0 < ur + ar) {
      T c = ash - g1 / ar * ur;
      r = rr * pow_rho<G14, T>(G, c);
      u = ash * (-ar + (T)0.5 * gm1 * ur);
      p = pr * pow_p<G14, T>(G, c);
      return 1;
    }
    r = rr; u = ur; p = pr;
    return 1;
  }
  if (0 <= us) {
    if (ps > pl) {
      T sl = ul - al * sqrt((T)G.sh1 * ps / pl + (T)G.sh2);
      if (0 <= sl) { r = rl; u = ul; p = pl; }
      else {
        T q = ps / pl;
        r = rl * (q + g1) / (g1 * q + 1);
        u = us; p = ps;
      }
    } else {
      if (0 <= ul - al) { r = rl; u = ul; p = pl; }
      else {
        T y = pow_z<G14, T>(G, ps / pl);
        if (0 >= us - al * y) {
          r = rl * pow_inv_g<G14, T>(G, ps / pl);
          u = us; p = ps;
        } else {
          T c = ash + g1 / al * ul;
          r = rl * pow_rho<G14, T>(G, c);
          u = ash * (al + (T)0.5 * gm1 * ul);
          p = pl * pow_p<G14, T>(G, c);
        }
      }
    }
    return 0;
  }
  if (ps > pr) {
    T sr = ur + ar * sqrt((T)G.sh1 * ps / pr + (T)G.sh2);
    if (0 >= sr) { r = rr; u = ur; p = pr; }
    else {
      T q = ps / pr;
      r = rr * (q + g1) / (g1 * q + 1);
      u = us; p = ps;
    }
  } else {
    if (0 >= ur + ar) { r = rr; u = ur; p = pr; }
    else {
      T y = pow_z<G14, T>(G, ps / pr);
      if (0 <= us + ar * y) {
        r = rr * pow_inv_g<G14, T>(G, ps / pr);
        u = us; p = ps;
      } else {
        T c = ash - g1 / ar * ur;
        r = rr * pow_rho<G14, T>(G, c);
        u = ash * (-ar + (T)0.5 * gm1 * ur);
        p = pr * pow_p<G14, T>(G, c);
      }
    }
  }
  return 1;
}

}  // namespace tafv
