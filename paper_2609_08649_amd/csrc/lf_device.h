// Device-side lens profile mathematics for gfx950.
//
// Every profile returns its deflection alpha, deformation tensor psi_ij and, on request,
// third potential derivatives psi_ijk in closed form (hand-derived, verified against
// finite differences); all quantities are a_dis-free (Sec. 2.1).  T is float (member
// galaxies in the mixed-precision path) or double.
#pragma once
#include <hip/hip_runtime.h>

#include "lf_internal.h"

namespace lf {

enum { T_POINT = 0, T_SIS = 1, T_SIE = 2, T_PJE = 3, T_NFW = 4, T_ENFW = 5, T_SHEAR = 6, T_MPOLE3 = 7 };
enum { FL_SINGULAR = 1, FL_GSING = 2, FL_NOCONV = 4, FL_REJECT = 8, FL_MERGED = 16,
       FL_OVERFLOW = 32, FL_UMBILIC = 64, FL_INVALID = 128 };

// Reciprocal and reciprocal square root.  FP32: the hardware instructions (1 ulp).  FP64:
// the hardware estimate refined by two Newton-Raphson steps (each doubles the number of
// correct bits; the result is within about 1 ulp, not correctly rounded), several times
// cheaper than the correctly rounded division and square-root sequences.  Arguments are
// finite and positive (rsq) or finite and non-zero (rcp) wherever these are called.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double frsq(double x) {
  // y <- y + y (1 - x y^2) / 2
  double y = __builtin_amdgcn_rsq(x);
  double hx = 0.5 * x;
  double r = fma(-hx * y, y, 0.5);
  y = fma(y, r, y);
  r = fma(-hx * y, y, 0.5);
  return fma(y, r, y);
}
__device__ __forceinline__ float fatan(float x) { return atanf(x); }
__device__ __forceinline__ double fatan(double x) { return atan(x); }
__device__ __forceinline__ float fatanh(float x) { return atanhf(x); }
__device__ __forceinline__ double fatanh(double x) { return atanh(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
// FP64 square root from the refined reciprocal square root y: s = x y, corrected once by
// s + (y/2)(x - s^2) (the residual taken with an FMA); x >= 0, finite.
__device__ __forceinline__ double fsqrt(double x) {
  const double y = frsq(x);
  const double s = x * y;
  const double r = fma(-s, s, x);
  return x > 0.0 ? fma(0.5 * y, r, s) : 0.0;
}

// Per-point FP64 accumulators.
struct Acc {
  double ax, ay, h11, h12, h22, t111, t112, t122, t222;
  int flags;
  __device__ void zero() { ax = ay = h11 = h12 = h22 = t111 = t112 = t122 = t222 = 0.0; flags = 0; }
};

template <class T>
struct Term {
  T ax, ay, h11, h12, h22, t111, t112, t122, t222;
};

template <bool D3, class T>
__device__ __forceinline__ void add(Acc& a, const Term<T>& t) {
  a.ax += (double)t.ax; a.ay += (double)t.ay;
  a.h11 += (double)t.h11; a.h12 += (double)t.h12; a.h22 += (double)t.h22;
  if (D3) { a.t111 += (double)t.t111; a.t112 += (double)t.t112; a.t122 += (double)t.t122; a.t222 += (double)t.t222; }
}

// ---------------------------------------------------------------------------------------
// Circularly symmetric profiles: alpha = m(r^2) r_vec, psi_ij = m delta_ij + w x_i x_j with
// w = 2 dm/d(r^2), psi_ijk = w (delta_ij x_k + delta_ik x_j + delta_jk x_i) + 2 w' x_i x_j x_k.
// ---------------------------------------------------------------------------------------
template <bool D3, class T>
__device__ __forceinline__ void radial(T dx, T dy, T m, T w, T wp, Term<T>& t) {
  t.ax = m * dx; t.ay = m * dy;
  T wx = w * dx, wy = w * dy;
  t.h11 = fma(wx, dx, m); t.h22 = fma(wy, dy, m); t.h12 = wx * dy;
  if (D3) {
    T q = (T)2 * wp;
    T qx2 = q * dx * dx, qy2 = q * dy * dy;
    t.t111 = dx * ((T)3 * w + qx2); t.t112 = dy * (w + qx2);
    t.t122 = dx * (w + qy2); t.t222 = dy * ((T)3 * w + qy2);
  }
}

// Cored isothermal term b / (R + s) with R = sqrt(s^2 + r^2): returns m, w (and w').
template <bool D3, class T>
__device__ __forceinline__ void cored_mw(T b, T s, T s2, T r2, T& m, T& w, T& wp) {
  T S2 = s2 + r2;
  T is = frsq(S2);
  T R = S2 * is;
  T u = frcp(R + s);
  T uu = u * u;
  m = b * u;
  T wt = uu * is;
  w = -b * wt;
  if (D3) wp = (T)0.5 * b * wt * fma((T)2 * u, R, (T)1) * is * is;
}

// Circular pseudo-Jaffe (dPIE, Sec. 3.4): the cored term with core s minus the same with
// core a > s, written without cancellation.  With R_c = sqrt(c^2 + r^2), D_c = R_c + c,
// Sg = R_s + R_a and G = D_s + D_a = Sg + a + s:
//   R_a - R_s = (a^2 - s^2) / Sg,   D_a - D_s = (a - s) G / Sg,
//   m = b/D_s - b/D_a = b (a - s) G / (Sg D_s D_a),
//   w = -b/(D_s^2 R_s) + b/(D_a^2 R_a) = -b (a - s) (D_a^2 (a + s) + R_s G^2) / (Sg (D_s D_a)^2 R_s R_a),
// every term positive, and one reciprocal, 1/(Sg D_s D_a), serves m, w and 1/(D_s D_a).  With
// R_s (1/R_s) = 1 the last form is w = -b (a - s) (D_a^2 (a + s)/R_s + G^2) / (Sg (D_s D_a)^2 R_a),
// one product fewer.  Subtracting two cored terms instead loses about log2(r/a) bits far from
// the member, where both terms are ~ b/r and their difference ~ b (a - s)/r^2.  bd = b (a - s)
// and apls = a + s are supplied by the caller.  Sg D_s D_a ~ 2 r^3 must stay finite: FP32
// callers keep r^2 < 1e25.  w' (third derivatives only) is the difference of the per-core
// derivatives b u^2 is^2 (u + is/2), u = 1/D, is = 1/R.
template <bool D3, class T>
__device__ __forceinline__ void pje_mw(T b, T s, T a, T s2, T a2, T bd, T apls, T r2, T& m, T& w, T& wp) {
  T Ss = s2 + r2, Sa = a2 + r2;
  T is = frsq(Ss), ia = frsq(Sa);
  T Rs = Ss * is, Ra = Sa * ia;
  T Ds = Rs + s, Da = Ra + a;
  T Sg = Rs + Ra, G = Sg + apls;
  T Z = frcp(Sg * (Ds * Da));
  T eZ = bd * Z;
  m = eZ * G;
  T iP = Sg * Z;
  T num = fma((Da * apls) * is, Da, G * G);
  w = -(eZ * iP) * ia * num;
  if (D3) {
    T us = Da * iP, ua = Ds * iP;                 // u of each core
    T xs = us * is, xa = ua * ia;
    wp = b * fma(xs * xs, fma((T)0.5, is, us), -(xa * xa * fma((T)0.5, ia, ua)));
  }
}
template <bool D3, class T>
__device__ __forceinline__ void cpje(T dx, T dy, T b, T s, T a, T s2, T a2, T bd, T apls, Term<T>& t) {
  T r2 = fma(dx, dx, dy * dy);
  T m, w, p = 0;
  pje_mw<D3>(b, s, a, s2, a2, bd, apls, r2, m, w, p);
  radial<D3>(dx, dy, m, w, p, t);
}
template <bool D3, class T>
__device__ __forceinline__ void csie(T dx, T dy, T b, T s, T s2, Term<T>& t) {
  T r2 = fma(dx, dx, dy * dy);
  T m, w, p = 0;
  cored_mw<D3>(b, s, s2, r2, m, w, p);
  radial<D3>(dx, dy, m, w, p, t);
}
template <bool D3, class T>
__device__ __forceinline__ void point_mass(T dx, T dy, T b, Term<T>& t) {
  T r2 = fma(dx, dx, dy * dy);
  T ir2 = frcp(r2);
  T b2 = b * b;
  T m = b2 * ir2;
  T w = (T)-2 * m * ir2;
  T wp = (T)-2 * w * ir2;
  radial<D3>(dx, dy, m, w, wp, t);
}

// ---------------------------------------------------------------------------------------
// Elliptical cored isothermal (SIE) in its own frame (major axis on x'):
//   psi~ = sqrt(q^2 (s^2 + x^2) + y^2),  alpha_x = (b q/e) atan(e x / (psi~ + s)),
//   alpha_y = (b q/e) atanh(e y / (psi~ + q^2 s)),  e = sqrt(1 - q^2);
//   psi_ij = b q N_ij / (psi~ D), D = (1+q^2) s^2 + 2 psi~ s + x^2 + y^2,
//   N_xx = q^2 s^2 + y^2 + s psi~, N_yy = s^2 + x^2 + s psi~, N_xy = -x y;
//   d_k psi_ij = b q / (psi~ D) (d_k N_ij - N_ij L_k), L_k = d_k psi~/psi~ + d_k D / D.
// ---------------------------------------------------------------------------------------
// Second and third derivatives of one core, psi~ given.
template <bool D3, class T>
__device__ __forceinline__ void esie_hess(T xp, T yp, T xx, T yy, T bqe, T e, T q2, T s, T psi, Term<T>& t) {
  T ss = s * s;
  T ip = frcp(psi);
  T D = fma((T)1 + q2, ss, fma((T)2 * psi, s, xx + yy));
  T iD = frcp(D);
  T Tn = bqe * e * ip * iD;
  T sp = s * psi;
  T Nxx = fma(q2, ss, yy + sp), Nyy = ss + xx + sp, Nxy = -xp * yp;
  t.h11 = Tn * Nxx; t.h22 = Tn * Nyy; t.h12 = Tn * Nxy;
  if (D3) {
    T dpx = q2 * xp * ip, dpy = yp * ip;
    T Lx = fma(dpx, ip, (T)2 * fma(s, dpx, xp) * iD);
    T Ly = fma(dpy, ip, (T)2 * fma(s, dpy, yp) * iD);
    t.t111 = Tn * (s * dpx - Nxx * Lx);
    t.t112 = Tn * ((T)2 * yp + s * dpy - Nxx * Ly);
    t.t122 = Tn * ((T)2 * xp + s * dpx - Nyy * Lx);
    t.t222 = Tn * (s * dpy - Nyy * Ly);
  }
}
template <bool D3, class T>
__device__ __forceinline__ void esie_prime(T xp, T yp, T bqe, T e, T q2, T s, Term<T>& t) {
  T xx = xp * xp, yy = yp * yp;
  T psi = fsqrt(fma(q2, fma(s, s, xx), yy));
  t.ax = bqe * fatan(e * xp * frcp(psi + s));
  t.ay = bqe * fatanh(e * yp * frcp(fma(q2, s, psi)));
  esie_hess<D3>(xp, yp, xx, yy, bqe, e, q2, s, psi, t);
}
// The dPIE pair (core s minus core a) in its own frame.  The deflection takes one arctangent
// and one inverse hyperbolic tangent for both cores: atan u1 - atan u2 = atan((u1 - u2) /
// (1 + u1 u2)) with u1 u2 >= 0 (both have the sign of x'), and atanh v1 - atanh v2 =
// atanh((v1 - v2) / (1 - v1 v2)) with v1 v2 >= 0 and |v| <= e < 1; the difference u1 - u2 is
// as exact as the difference of the two arctangents it replaces.
// In FP64 the two arguments are formed with one reciprocal each: with A_c = psi~_c + c and
// B_c = psi~_c + q^2 c, psi~_a - psi~_s = q^2 (a^2 - s^2) / (psi~_a + psi~_s) (no cancellation),
//   (u1 - u2) / (1 + u1 u2) = e x' [q^2 (a^2 - s^2) + (a - s) P] / (P (A_s A_a + e^2 x'^2)),
//   (v1 - v2) / (1 - v1 v2) = e y' q^2 (a - s) (P + a + s) / (P (B_s B_a - e^2 y'^2)),
// P = psi~_s + psi~_a; B_s B_a - e^2 y'^2 >= q^2 y'^2 (psi~ >= |y'|).
template <bool D3, class T>
__device__ __forceinline__ void epje_prime(T xp, T yp, T bqe, T e, T q2, T s, T a, Term<T>& t) {
  T xx = xp * xp, yy = yp * yp;
  T psi_s = fsqrt(fma(q2, fma(s, s, xx), yy)), psi_a = fsqrt(fma(q2, fma(a, a, xx), yy));
  T zx, zy;
  if constexpr (sizeof(T) == 8) {
    const T P = psi_s + psi_a, as = a - s, ee = e * e;
    const T As = psi_s + s, Aa = psi_a + a, Bs = fma(q2, s, psi_s), Ba = fma(q2, a, psi_a);
    zx = e * xp * fma(q2 * as, a + s, as * P) * frcp(P * fma(ee, xx, As * Aa));
    zy = e * yp * q2 * as * (P + (a + s)) * frcp(P * fma(-ee, yy, Bs * Ba));
  } else {
    T u1 = e * xp * frcp(psi_s + s), u2 = e * xp * frcp(psi_a + a);
    T v1 = e * yp * frcp(fma(q2, s, psi_s)), v2 = e * yp * frcp(fma(q2, a, psi_a));
    zx = (u1 - u2) * frcp(fma(u1, u2, (T)1));
    zy = (v1 - v2) * frcp(fma(-v1, v2, (T)1));
  }
  // the derivatives first, so that few values stay live across the two library calls
  Term<T> hs, ha;
  esie_hess<D3>(xp, yp, xx, yy, bqe, e, q2, s, psi_s, hs);
  esie_hess<D3>(xp, yp, xx, yy, bqe, e, q2, a, psi_a, ha);
  t.h11 = hs.h11 - ha.h11; t.h12 = hs.h12 - ha.h12; t.h22 = hs.h22 - ha.h22;
  if (D3) {
    t.t111 = hs.t111 - ha.t111; t.t112 = hs.t112 - ha.t112; t.t122 = hs.t122 - ha.t122; t.t222 = hs.t222 - ha.t222;
  }
  t.ax = bqe * fatan(zx);
  t.ay = bqe * fatanh(zy);
}

template <class T>
__device__ __forceinline__ T t3eval(const Term<T>& t, T u0, T u1, T v0, T v1, T w0, T w1) {
  return t.t111 * u0 * v0 * w0 + t.t112 * (u0 * v0 * w1 + u0 * v1 * w0 + u1 * v0 * w0) +
         t.t122 * (u0 * v1 * w1 + u1 * v0 * w1 + u1 * v1 * w0) + t.t222 * u1 * v1 * w1;
}

// Rotate a primed-frame term back to the sky frame (x' = c dx + s dy, y' = -s dx + c dy).
template <bool D3, class T>
__device__ __forceinline__ void rotate_back(T c, T s, const Term<T>& p, Term<T>& t) {
  t.ax = c * p.ax - s * p.ay;
  t.ay = s * p.ax + c * p.ay;
  T cc = c * c, ss = s * s, cs = c * s;
  t.h11 = cc * p.h11 - (T)2 * cs * p.h12 + ss * p.h22;
  t.h22 = ss * p.h11 + (T)2 * cs * p.h12 + cc * p.h22;
  t.h12 = cs * (p.h11 - p.h22) + (cc - ss) * p.h12;
  if (D3) {
    // unit vectors e_x -> (c, -s), e_y -> (s, c) in the primed frame
    t.t111 = t3eval(p, c, -s, c, -s, c, -s);
    t.t112 = t3eval(p, c, -s, c, -s, s, c);
    t.t122 = t3eval(p, c, -s, s, c, s, c);
    t.t222 = t3eval(p, s, c, s, c, s, c);
  }
}

template <bool D3, class T>
__device__ __forceinline__ void sub_term(Term<T>& a, const Term<T>& b) {
  a.ax -= b.ax; a.ay -= b.ay; a.h11 -= b.h11; a.h12 -= b.h12; a.h22 -= b.h22;
  if (D3) { a.t111 -= b.t111; a.t112 -= b.t112; a.t122 -= b.t122; a.t222 -= b.t222; }
}

// PAIR: the dPIE by epje_prime (one arctangent and one inverse hyperbolic tangent); otherwise
// as the difference of two cored isothermal terms.  The main-halo passes of the maps and of the
// chi^2 take the pair form (19% and ~4% faster there); in the image-plane Newton kernel the
// pair form measured 2.2x slower (its code around the per-lane member loop compiles
// differently), so the other callers keep the two-term form.
template <bool D3, class T, bool PAIR = false>
__device__ __forceinline__ void epje(T dx, T dy, T c, T sn, T bqe, T e, T q2, T s, T a, bool pje, Term<T>& t) {
  T xp = c * dx + sn * dy, yp = c * dy - sn * dx;
  Term<T> p;
  if (PAIR && pje) {
    epje_prime<D3>(xp, yp, bqe, e, q2, s, a, p);
  } else {
    esie_prime<D3>(xp, yp, bqe, e, q2, s, p);
    if (pje) {
      Term<T> p2;
      esie_prime<D3>(xp, yp, bqe, e, q2, a, p2);
      sub_term<D3>(p, p2);
    }
  }
  rotate_back<D3>(c, sn, p, t);
}

// ---------------------------------------------------------------------------------------
// NFW.  With X^2 = xi^2 / r_s^2 and z = 1 - X^2:  F = arccosh(1/X)/sqrt(1-X^2) (X < 1),
// arccos(1/X)/sqrt(X^2-1) (X > 1); kappa = 2 k_s G(z), G = (F - 1)/z (series near z = 0).
// Returns G and dG/dz (D2: d^2G/dz^2 too).  For X < 1, arccosh(1/X) = log((1 + w)/X) =
// log((1 + w)^2 / X^2) / 2 with w = sqrt(z) >= 0.3 outside the series range: one logarithm,
// no cancellation.  Outside the series range the derivatives follow from F' = (1/(1-z) - F) / 2z,
// F'' = (1/(1-z)^2 - 3 F') / 2z, G' = (F' - G) / z and G'' = (F'' - 2 G') / z.
// ---------------------------------------------------------------------------------------
template <bool D2>
__device__ __forceinline__ void nfw_G(double X2, double& F, double& G, double& Gp, double& Gpp) {
  double z = 1.0 - X2;
  if (fabs(z) < 0.1) {
    // F = sum z^k/(2k+1); G = sum_{k>=1} z^(k-1)/(2k+1); G' = sum_{k>=2} (k-1) z^(k-2)/(2k+1);
    // G'' = sum_{k>=3} (k-1)(k-2) z^(k-3)/(2k+1)
    double g = 0.0, gp = 0.0;
#pragma unroll
    for (int k = 18; k >= 2; --k) { g = fma(g, z, 1.0 / (2 * k + 1)); gp = fma(gp, z, (double)(k - 1) / (2 * k + 1)); }
    G = fma(g, z, 1.0 / 3.0);
    Gp = gp;
    F = fma(G, z, 1.0);
    if (D2) {
      double gpp = 0.0;
#pragma unroll
      for (int k = 21; k >= 3; --k) gpp = fma(gpp, z, (double)((k - 1) * (k - 2)) / (2 * k + 1));
      Gpp = gpp;
    }
  } else {
    // one reciprocal square root y = 1/sqrt(|z|) gives w = sqrt(|z|) = |z| y, 1/w = y and
    // 1/z = +-y^2
    const double iX2 = frcp(X2);
    const double az = fabs(z), y = frsq(az);
    const double w = fma(0.5 * y, fma(-az * y, az * y, az), az * y);   // |z| y, one Newton step
    if (z > 0) {
      const double w1 = 1.0 + w;
      F = 0.5 * log(w1 * w1 * iX2) * y;
    } else {
      F = atan(w) * y;
    }
    const double iz = z > 0 ? y * y : -(y * y);
    G = (F - 1.0) * iz;
    const double Fp = 0.5 * (iX2 - F) * iz;
    Gp = (Fp - G) * iz;
    if (D2) {
      const double Fpp = 0.5 * fma(iX2, iX2, -3.0 * Fp) * iz;
      Gpp = (Fpp - 2.0 * Gp) * iz;
    }
  }
}
__device__ __forceinline__ void nfw_G(double X2, double& F, double& G, double& Gp) {
  double unused;
  nfw_G<false>(X2, F, G, Gp, unused);
}

template <bool D3>
__device__ __forceinline__ void nfw_circ(double dx, double dy, double ks, double rs, Term<double>& t) {
  double r2 = fma(dx, dx, dy * dy);
  double irs2 = 1.0 / (rs * rs);
  double X2 = r2 * irs2;
  double F, G, Gp;
  nfw_G(X2, F, G, Gp);
  double ir2 = frcp(r2);
  double h = 0.5 * log(0.25 * X2) + F;
  double m = 4.0 * ks * rs * rs * h * ir2;
  double kap = 2.0 * ks * G;
  double w = 2.0 * (kap - m) * ir2;
  double wp = 0.0;
  if (D3) { double kp = -2.0 * ks * Gp * irs2; wp = 2.0 * (kp - w) * ir2; }
  radial<D3>(dx, dy, m, w, wp, t);
}

// Elliptical NFW in its own frame from the integrals
//   J_n = int_0^1 kappa(xi^2(u)) (1 - e^2 u)^-(n+1/2) du,  K_n = int_0^1 u kappa'(xi^2(u)) (...)^-(n+1/2) du,
//   L_n = int_0^1 u^2 kappa''(xi^2(u)) (...)^-(n+1/2) du  (derivatives in xi^2)
// with xi^2(u) = u (x^2 + y^2/(1 - e^2 u)):  alpha = q (x J0, y J1),
// psi_xx = 2 q x^2 K0 + q J0, psi_yy = 2 q y^2 K2 + q J1, psi_xy = 2 q x y K1.  Since
// d(xi^2)/dx = 2 u x and d(xi^2)/dy = 2 u y / (1 - e^2 u), d/dx of an integral of order n
// brings 2 x times the next kind at the same order and d/dy 2 y times it at order n + 1:
// psi_xxx = q x (6 K0 + 4 x^2 L0), psi_xxy = q y (2 K1 + 4 x^2 L1), psi_xyy = q x (2 K1 + 4 y^2 L2),
// psi_yyy = q y (6 K2 + 4 y^2 L3).
// Fixed Gauss-Legendre nodes in t with u = t^6 (u_node, w_node carry the Jacobian).
struct Quad {
  int n;
  const double* u;
  const double* w;
};
template <bool D3 = false>
__device__ __forceinline__ void enfw_prime(double xp, double yp, double ks, double rs, double q,
                                           const Quad& qd, Term<double>& t) {
  double e2 = 1.0 - q * q;
  double xx = xp * xp, yy = yp * yp;
  double irs2 = 1.0 / (rs * rs);
  double J0 = 0, J1 = 0, K0 = 0, K1 = 0, K2 = 0;
  double L0 = 0, L1 = 0, L2 = 0, L3 = 0;
  for (int i = 0; i < qd.n; ++i) {
    double u = qd.u[i], wq = qd.w[i];
    double W = fma(-e2, u, 1.0);
    const double rW = frsq(W), iW = rW * rW;
    double X2 = u * fma(yy, iW, xx) * irs2;
    double F, G, Gp, Gpp;
    nfw_G<D3>(X2, F, G, Gp, Gpp);
    double kap = 2.0 * ks * G;
    double ukp = -2.0 * ks * Gp * irs2 * u;
    double f0 = wq * rW;
    double f1 = f0 * iW, f2 = f1 * iW;
    J0 = fma(f0, kap, J0); J1 = fma(f1, kap, J1);
    K0 = fma(f0, ukp, K0); K1 = fma(f1, ukp, K1); K2 = fma(f2, ukp, K2);
    if (D3) {
      const double uukpp = 2.0 * ks * Gpp * (irs2 * u) * (irs2 * u);
      const double f3 = f2 * iW;
      L0 = fma(f0, uukpp, L0); L1 = fma(f1, uukpp, L1); L2 = fma(f2, uukpp, L2); L3 = fma(f3, uukpp, L3);
    }
  }
  t.ax = q * xp * J0; t.ay = q * yp * J1;
  t.h11 = 2.0 * q * xx * K0 + q * J0;
  t.h22 = 2.0 * q * yy * K2 + q * J1;
  t.h12 = 2.0 * q * xp * yp * K1;
  if (D3) {
    t.t111 = q * xp * fma(4.0 * xx, L0, 6.0 * K0);
    t.t112 = q * yp * fma(4.0 * xx, L1, 2.0 * K1);
    t.t122 = q * xp * fma(4.0 * yy, L2, 2.0 * K1);
    t.t222 = q * yp * fma(4.0 * yy, L3, 6.0 * K2);
  } else {
    t.t111 = t.t112 = t.t122 = t.t222 = 0.0;
  }
}

// ---------------------------------------------------------------------------------------
// Lensing potential psi (Sec. 2.1, defined without a_dis), FP64, for the time-delay terms;
// each profile up to its own additive constant (delays use differences within a family):
//   circular cored  b (R - s ln(R + s));  circular dPIE  b (-(R_a - R_s) - s ln D_s + a ln D_a)
//   (R_a - R_s as in pje_mw);  elliptical SIE  x alpha_x + y alpha_y - b q s ln sqrt((psi~ + s)^2
//   + e^2 x^2) in the halo frame;  point mass  b^2 ln r;  NFW  2 k_s r_s^2 h(X) with
//   h = ln^2(X/2) - arccosh^2(1/X) (X < 1), ln^2(X/2) + arccos^2(1/X) (X > 1);  elliptical NFW
//   (q/2) int_0^1 xi alpha_c(xi) / (u sqrt(1 - e^2 u)) du, xi alpha_c = 4 k_s r_s^2 (ln(X/2) + F).
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double pot_cored(double b, double s, double r2) {
  const double R = sqrt(fma(s, s, r2));
  return s > 0.0 ? b * (R - s * log(R + s)) : b * R;
}
__device__ __forceinline__ double pot_cpje(double b, double s, double a, double r2) {
  const double Rs = sqrt(fma(s, s, r2)), Ra = sqrt(fma(a, a, r2));
  const double dR = (a - s) * (a + s) / (Ra + Rs);
  double v = a * log(Ra + a) - dR;
  if (s > 0.0) v -= s * log(Rs + s);
  return b * v;
}
__device__ __forceinline__ double pot_esie(double xp, double yp, double bqe, double e, double q2, double s) {
  const double psi = sqrt(fma(q2, fma(s, s, xp * xp), yp * yp));
  const double ax = bqe * atan(e * xp / (psi + s)), ay = bqe * atanh(e * yp / fma(q2, s, psi));
  double v = xp * ax + yp * ay;
  if (s > 0.0) {
    const double ps = psi + s;
    v -= bqe * e * s * 0.5 * log(fma(ps, ps, e * e * xp * xp));   // b q s = bqe e s
  }
  return v;
}
__device__ __forceinline__ double pot_nfw(double r2, double ks, double rs) {
  const double X2 = r2 / (rs * rs), X = sqrt(X2);
  const double l = log(0.5 * X);
  double h;
  if (X < 1.0) { const double ac = log((1.0 + sqrt(1.0 - X2)) / X); h = l * l - ac * ac; }
  else { const double ac = acos(1.0 / X); h = l * l + ac * ac; }
  return 2.0 * ks * rs * rs * h;
}
__device__ __forceinline__ double pot_enfw(double xp, double yp, double ks, double rs, double q, const Quad& qd) {
  const double e2 = 1.0 - q * q, xx = xp * xp, yy = yp * yp, irs2 = 1.0 / (rs * rs);
  double I = 0.0;
  for (int i = 0; i < qd.n; ++i) {
    const double u = qd.u[i], W = fma(-e2, u, 1.0);
    const double X2 = u * (xx + yy / W) * irs2;
    double F, G, Gp;
    nfw_G(X2, F, G, Gp);
    const double xa = 4.0 * ks * rs * rs * (0.5 * log(0.25 * X2) + F);
    I = fma(qd.w[i], xa / (u * sqrt(W)), I);
  }
  return 0.5 * q * I;
}
// Potential of one main component (0 on a singular centre, where its deflection is 0 too).
// A point exactly on the centre of a profile whose derivatives diverge there gets no term.
__device__ __forceinline__ bool main_singular(const MainRec& r) {
  return r.type == T_POINT || r.type == T_SIS || r.type == T_NFW || r.type == T_ENFW || r.type == T_MPOLE3 ||
         ((r.type == T_SIE || r.type == T_PJE) && r.s == 0.0);
}

// External shear about the component's centre: gamma_1 = b cos 2pa, gamma_2 = b sin 2pa
// (from the cosine and sine of pa: cos 2pa = c^2 - s^2, sin 2pa = 2 c s).
template <bool D3>
__device__ __forceinline__ void ext_shear(double dx, double dy, double b, double c, double sn, Term<double>& t) {
  const double g1 = b * (c * c - sn * sn), g2 = b * (2.0 * c * sn);
  t.ax = g1 * dx + g2 * dy;
  t.ay = g2 * dx - g1 * dy;
  t.h11 = g1; t.h12 = g2; t.h22 = -g1;
  t.t111 = t.t112 = t.t122 = t.t222 = 0.0;
}
// m = 3 multipole psi = A r^2 cos 3phi' (A = b/3) in the frame turned by pa, x = x', y = y':
// alpha = A (2x^4 + 3x^2y^2 - 3y^4, -7x^3y - 3xy^3) / r^3,
// psi_11 = A (2x^5 + 5x^3y^2 + 15xy^4) / r^5, psi_12 = -A (15x^2y^3 + 3y^5) / r^5,
// psi_22 = A (5x^3y^2 - 7x^5) / r^5, psi_111 = 15A y^4 (y^2 - 3x^2) / r^7,
// psi_112 = 15A x y^3 (3x^2 - y^2) / r^7, psi_122 = 15A x^2 y^2 (y^2 - 3x^2) / r^7,
// psi_222 = 15A x^3 y (3x^2 - y^2) / r^7; then rotated back.
template <bool D3>
__device__ __forceinline__ void mpole3(double dx, double dy, double b, double c, double sn, Term<double>& t) {
  const double x = c * dx + sn * dy, y = c * dy - sn * dx;
  const double A = b / 3.0, x2 = x * x, y2 = y * y, r2 = x2 + y2;
  const double ir = frsq(r2), ir2 = ir * ir, ir3 = ir2 * ir, ir5 = ir3 * ir2;
  Term<double> p;
  p.ax = A * (2.0 * x2 * x2 + 3.0 * x2 * y2 - 3.0 * y2 * y2) * ir3;
  p.ay = -A * x * y * (7.0 * x2 + 3.0 * y2) * ir3;
  p.h11 = A * x * (2.0 * x2 * x2 + 5.0 * x2 * y2 + 15.0 * y2 * y2) * ir5;
  p.h12 = -A * y * y2 * (15.0 * x2 + 3.0 * y2) * ir5;
  p.h22 = A * x * x2 * (5.0 * y2 - 7.0 * x2) * ir5;
  p.t111 = p.t112 = p.t122 = p.t222 = 0.0;
  if (D3) {
    const double k = 15.0 * A * ir5 * ir2;
    p.t111 = k * y2 * y2 * (y2 - 3.0 * x2);
    p.t112 = k * x * y * y2 * (3.0 * x2 - y2);
    p.t122 = k * x2 * y2 * (y2 - 3.0 * x2);
    p.t222 = k * x * x2 * y * (3.0 * x2 - y2);
  }
  rotate_back<D3>(c, sn, p, t);
}

__device__ __forceinline__ double pot_main(const MainRec& r, double px, double py, const Quad& qd) {
  const double dx = px - r.x, dy = py - r.y, r2 = fma(dx, dx, dy * dy);
  if (main_singular(r) && r2 < 1e-24) return 0.0;
  switch (r.type) {
    case T_SHEAR: {
      const double c2 = r.c * r.c - r.sn * r.sn, s2 = 2.0 * r.c * r.sn;
      return 0.5 * r.b * ((dx * dx - dy * dy) * c2 + 2.0 * dx * dy * s2);
    }
    case T_MPOLE3: {
      const double x = r.c * dx + r.sn * dy, y = r.c * dy - r.sn * dx;
      return (r.b / 3.0) * x * (x * x - 3.0 * y * y) * frsq(r2);
    }
    case T_POINT: return r.b * r.b * 0.5 * log(r2);
    case T_SIS: return r.b * sqrt(r2);
    case T_NFW: return pot_nfw(r2, r.b, r.s);
    default: break;
  }
  if (r.q >= 1.0) {
    if (r.type == T_SIE) return pot_cored(r.b, r.s, r2);
    if (r.type == T_PJE) return pot_cpje(r.b, r.s, r.a, r2);
    return pot_nfw(r2, r.b, r.s);
  }
  const double xp = r.c * dx + r.sn * dy, yp = r.c * dy - r.sn * dx;
  if (r.type == T_SIE) return pot_esie(xp, yp, r.bqe, r.e, r.q2, r.s);
  if (r.type == T_PJE) return pot_esie(xp, yp, r.bqe, r.e, r.q2, r.s) - pot_esie(xp, yp, r.bqe, r.e, r.q2, r.a);
  return pot_enfw(xp, yp, r.b, r.s, r.q, qd);
}

// ---------------------------------------------------------------------------------------
// One main component (FP64) at one point.
// ---------------------------------------------------------------------------------------
// ENFW = false compiles the elliptical NFW quadrature out (a kernel variant for models without
// elliptical NFW halos, which then needs far fewer registers); such a halo reaching it is
// flagged invalid.
template <bool D3, bool ENFW = true, bool PAIR = false>
__device__ __forceinline__ void eval_main(const MainRec& r, double px, double py, const Quad& qd, Acc& acc) {
  double dx = px - r.x, dy = py - r.y;
  double r2 = fma(dx, dx, dy * dy);
  Term<double> t;
  t.t111 = t.t112 = t.t122 = t.t222 = 0.0;
  if (main_singular(r) && r2 < 1e-24) { acc.flags |= FL_SINGULAR; return; }
  switch (r.type) {
    case T_SHEAR: ext_shear<D3>(dx, dy, r.b, r.c, r.sn, t); break;
    case T_MPOLE3: mpole3<D3>(dx, dy, r.b, r.c, r.sn, t); break;
    case T_POINT: point_mass<D3>(dx, dy, r.b, t); break;
    case T_SIS: csie<D3>(dx, dy, r.b, 0.0, 0.0, t); break;
    case T_SIE:
      if (r.q >= 1.0) csie<D3>(dx, dy, r.b, r.s, r.s * r.s, t);
      else epje<D3>(dx, dy, r.c, r.sn, r.bqe, r.e, r.q2, r.s, r.a, false, t);
      break;
    case T_PJE:
      if (r.q >= 1.0) cpje<D3>(dx, dy, r.b, r.s, r.a, r.s * r.s, r.a * r.a, r.b * (r.a - r.s), r.a + r.s, t);
      else epje<D3, double, PAIR>(dx, dy, r.c, r.sn, r.bqe, r.e, r.q2, r.s, r.a, true, t);
      break;
    case T_NFW: nfw_circ<D3>(dx, dy, r.b, r.s, t); break;
    default:
      if (r.q >= 1.0) nfw_circ<D3>(dx, dy, r.b, r.s, t);
      else if constexpr (ENFW) {
        double xp = r.c * dx + r.sn * dy, yp = r.c * dy - r.sn * dx;
        Term<double> p;
        enfw_prime<D3>(xp, yp, r.b, r.s, r.q, qd, p);
        rotate_back<D3>(r.c, r.sn, p, t);
      } else {
        acc.flags |= FL_INVALID;
        return;
      }
      break;
  }
  add<D3>(acc, t);
}

// Unit eigenvectors of the deformation tensor (Sec. 6): v of e_1 = kappa + |gamma| is the
// larger of (g1 + |g|, g2) and (g2, |g| - g1), normalised; w (of e_2) is v turned by +90
// degrees; each with a non-negative x component (then y).
__device__ __forceinline__ void a3_vectors(double g1, double g2, double gm, double& vx, double& vy, double& wx,
                                           double& wy) {
  double vax = g1 + gm, vay = g2, vbx = g2, vby = gm - g1;
  double na = vax * vax + vay * vay, nb = vbx * vbx + vby * vby;
  if (na >= nb) { double n = 1.0 / sqrt(na); vx = vax * n; vy = vay * n; }
  else { double n = 1.0 / sqrt(nb); vx = vbx * n; vy = vby * n; }
  if (vx < 0 || (vx == 0 && vy < 0)) { vx = -vx; vy = -vy; }
  wx = -vy; wy = vx;
  if (wx < 0 || (wx == 0 && wy < 0)) { wx = -wx; wy = -wy; }
}
// A3-line fields f_k = v_k . grad e_k (Sec. 6) from kappa, gamma and the third derivatives;
// false (umbilic: |gamma| <= 1e-12 |kappa|, f undefined) leaves f1, f2 untouched.
__device__ __forceinline__ bool a3_fields(double kap, double g1, double g2, double t111, double t112, double t122,
                                          double t222, double& f1, double& f2, double& vx, double& vy, double& wx,
                                          double& wy) {
  double gm = sqrt(g1 * g1 + g2 * g2);
  if (!(gm > 1e-12 * fabs(kap)) || gm == 0.0) return false;
  double gkx = 0.5 * (t111 + t122), gky = 0.5 * (t112 + t222);
  double g1x = 0.5 * (t111 - t122), g1y = 0.5 * (t112 - t222);
  double g2x = t112, g2y = t122;
  double igm = 1.0 / gm;
  double ggx = (g1 * g1x + g2 * g2x) * igm, ggy = (g1 * g1y + g2 * g2y) * igm;
  a3_vectors(g1, g2, gm, vx, vy, wx, wy);
  f1 = vx * (gkx + ggx) + vy * (gky + ggy);
  f2 = wx * (gkx - ggx) + wy * (gky - ggy);
  return true;
}

// FP64 epilogue of a single-plane point (Sec. 2.1): kappa, gamma, det A, mu, beta,
// eigenvalues and the A3-line fields f_k = v_k . grad e_k (Sec. 6).
struct Epi {
  double kappa, g1, g2, detA, mu, bx, by, e1, e2, f1, f2;
  int flags;
};
template <bool D3>
__device__ __forceinline__ void epilogue(double x, double y, double a, const Acc& h, Epi& o) {
  o.kappa = 0.5 * (h.h11 + h.h22);
  o.g1 = 0.5 * (h.h11 - h.h22);
  o.g2 = h.h12;
  double A11 = fma(-a, h.h11, 1.0), A22 = fma(-a, h.h22, 1.0), A12 = -a * h.h12;
  o.detA = A11 * A22 - A12 * A12;
  o.mu = 1.0 / o.detA;
  o.bx = fma(-a, h.ax, x);
  o.by = fma(-a, h.ay, y);
  double gm = sqrt(o.g1 * o.g1 + o.g2 * o.g2);
  o.e1 = o.kappa + gm;
  o.e2 = o.kappa - gm;
  o.flags = h.flags;
  o.f1 = o.f2 = 0.0;
  if (D3) {
    double vx, vy, wx, wy;
    if (!a3_fields(o.kappa, o.g1, o.g2, h.t111, h.t112, h.t122, h.t222, o.f1, o.f2, vx, vy, wx, wy))
      o.flags |= FL_UMBILIC;
  }
}

}  // namespace lf
