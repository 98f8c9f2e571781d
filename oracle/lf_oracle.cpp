// FP64 CPU oracle for the lens-equation hot path.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library may call, link or
// load this file; only the test suite, the smoke check and the benchmark's
// CPU-baseline leg do.  It shares no code with the GPU library.
//
// Plain, slow and obviously correct: every sum runs over halos in table order,
// every quantity is computed in IEEE double precision (no fast-math), and all
// derivatives of the lensing potential come from forward-mode automatic
// differentiation of the closed-form deflection (a second-order "jet" in the two
// image-plane coordinates).  Hessian = first derivatives of alpha, third
// potential derivatives = second derivatives of alpha.
//
// Paper passages followed (arXiv 2609.08649):
//   * Sec. 2.1 Eq. (lens_eq), Eq. (jac), deformation tensor, kappa/gamma and mu
//     definitions (potential defined without the distance ratio a_dis).
//   * Sec. 2.2 multi-plane lens equation and the recursion for theta_j.
//   * Sec. 2.3 lens-equation solving (replaced here by triangle mapping with exact
//     orientation predicates; accuracy O(h^2) before polishing).
//   * Sec. 3.1 Eq. (chi2_img), Eq. (chi2_src), Eq. (delta), beta_model = G^-1 g.
//   * Sec. 2.1 Eq. (time_delay) (Fermat potential, lensing potential psi without a_dis);
//     Sec. 3.2 Eq. (chi2_flux), Eq. (msrc) and the linear magnification expansion;
//     Sec. 3.3 Eq. (chi2_td), Eq. (dt0), Eq. (td_approx).
//   * Sec. 3.4 Eq. (scaling) for member galaxies.
//   * Sec. 3.5 Newton-Raphson image-plane solve started at the observed images.
//   * Sec. 6 singularity maps: A3-line fields from third derivatives, and the
//     extraction of A3 lines, umbilics (D4) and swallowtails (A4) from a vertex grid
//     with refinement of every crossing and point (the refinement the paper plans).
// Readings where the paper is silent (profile formulas, sigma->b, eNFW, tie rules,
// Newton stopping rules) are listed in the design notes of the repository.
//
// Parity pins for every function live in tests/test_oracle_*.py.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <thread>
#include <vector>

namespace orc {

// ----------------------------------------------------------------------------
// Physical constants
// ----------------------------------------------------------------------------
static const double C_KMS = 299792.458;               // speed of light [km/s]
static const double G_MPC = 4.30091727e-9;            // G [Mpc (km/s)^2 / Msun]
static const double ARCSEC = 206264.80624709636;      // arcsec per radian
static const double PI = 3.14159265358979323846;

// ----------------------------------------------------------------------------
// Second-order jet in (x, y): value, gradient and Hessian of a scalar.
// ----------------------------------------------------------------------------
struct J {
  double v = 0, dx = 0, dy = 0, hxx = 0, hxy = 0, hyy = 0;
  J() {}
  J(double c) : v(c) {}
};
static inline J var_x(double x) { J r(x); r.dx = 1; return r; }
static inline J var_y(double y) { J r(y); r.dy = 1; return r; }
static inline J operator+(const J& a, const J& b) {
  J r; r.v = a.v + b.v; r.dx = a.dx + b.dx; r.dy = a.dy + b.dy;
  r.hxx = a.hxx + b.hxx; r.hxy = a.hxy + b.hxy; r.hyy = a.hyy + b.hyy; return r;
}
static inline J operator-(const J& a, const J& b) {
  J r; r.v = a.v - b.v; r.dx = a.dx - b.dx; r.dy = a.dy - b.dy;
  r.hxx = a.hxx - b.hxx; r.hxy = a.hxy - b.hxy; r.hyy = a.hyy - b.hyy; return r;
}
static inline J operator-(const J& a) { return J(0.0) - a; }
static inline J operator*(const J& a, const J& b) {
  J r; r.v = a.v * b.v;
  r.dx = a.dx * b.v + a.v * b.dx; r.dy = a.dy * b.v + a.v * b.dy;
  r.hxx = a.hxx * b.v + 2 * a.dx * b.dx + a.v * b.hxx;
  r.hxy = a.hxy * b.v + a.dx * b.dy + a.dy * b.dx + a.v * b.hxy;
  r.hyy = a.hyy * b.v + 2 * a.dy * b.dy + a.v * b.hyy; return r;
}
static inline J operator*(const J& a, double c) {
  J r; r.v = a.v * c; r.dx = a.dx * c; r.dy = a.dy * c;
  r.hxx = a.hxx * c; r.hxy = a.hxy * c; r.hyy = a.hyy * c; return r;
}
static inline J operator*(double c, const J& a) { return a * c; }
static inline J operator+(const J& a, double c) { J r = a; r.v += c; return r; }
static inline J operator+(double c, const J& a) { return a + c; }
static inline J operator-(const J& a, double c) { J r = a; r.v -= c; return r; }
static inline J operator-(double c, const J& a) { return J(c) - a; }
// chain rule for a scalar function with value f, first derivative f1, second f2
static inline J chain(const J& u, double f, double f1, double f2) {
  J r; r.v = f; r.dx = f1 * u.dx; r.dy = f1 * u.dy;
  r.hxx = f1 * u.hxx + f2 * u.dx * u.dx;
  r.hxy = f1 * u.hxy + f2 * u.dx * u.dy;
  r.hyy = f1 * u.hyy + f2 * u.dy * u.dy; return r;
}
static inline J recip(const J& u) { double i = 1.0 / u.v; return chain(u, i, -i * i, 2 * i * i * i); }
static inline J operator/(const J& a, const J& b) { return a * recip(b); }
static inline J operator/(const J& a, double c) { return a * (1.0 / c); }
static inline J operator/(double c, const J& a) { return c * recip(a); }
static inline J sqrt(const J& u) { double s = std::sqrt(u.v); return chain(u, s, 0.5 / s, -0.25 / (s * u.v)); }
static inline J atan(const J& u) { double d = 1 + u.v * u.v; return chain(u, std::atan(u.v), 1 / d, -2 * u.v / (d * d)); }
static inline J atanh(const J& u) { double d = 1 - u.v * u.v; return chain(u, std::atanh(u.v), 1 / d, 2 * u.v / (d * d)); }
static inline J log(const J& u) { return chain(u, std::log(u.v), 1 / u.v, -1 / (u.v * u.v)); }
static inline double val(double x) { return x; }
static inline double val(const J& x) { return x.v; }
using std::sqrt; using std::atan; using std::atanh; using std::log;

// ----------------------------------------------------------------------------
// Gauss-Legendre nodes (Newton iteration on P_n) and adaptive quadrature.
// ----------------------------------------------------------------------------
struct GL {
  int n; std::vector<double> x, w;
  explicit GL(int n_) : n(n_), x(n_), w(n_) {
    for (int i = 0; i < n; ++i) {
      double z = std::cos(PI * (i + 0.75) / (n + 0.5)), pp = 0;
      for (int it = 0; it < 100; ++it) {
        double p1 = 1, p2 = 0;
        for (int k = 1; k <= n; ++k) { double p3 = p2; p2 = p1; p1 = ((2 * k - 1) * z * p2 - (k - 1) * p3) / k; }
        pp = n * (z * p1 - p2) / (z * z - 1);
        double z1 = z; z = z1 - p1 / pp;
        if (std::fabs(z - z1) < 1e-16) break;
      }
      x[i] = z; w[i] = 2 / ((1 - z * z) * pp * pp);
    }
  }
};
static const GL& gl10() { static GL g(10); return g; }

// Integrate a vector-valued function (K components of type T) over [lo, hi];
// error control on the value parts of all components.
template <class T, int K>
static void gl_panel(const std::function<void(double, T*)>& f, double lo, double hi, T* out) {
  const GL& g = gl10();
  for (int k = 0; k < K; ++k) out[k] = T(0.0);
  double m = 0.5 * (hi + lo), r = 0.5 * (hi - lo);
  T tmp[K];
  for (int i = 0; i < g.n; ++i) {
    f(m + r * g.x[i], tmp);
    for (int k = 0; k < K; ++k) out[k] = out[k] + tmp[k] * (g.w[i] * r);
  }
}
template <class T, int K>
static void adapt(const std::function<void(double, T*)>& f, double lo, double hi, const T* whole,
                  double tol, int depth, T* acc, long* budget) {
  double m = 0.5 * (lo + hi);
  T L[K], R[K];
  gl_panel<T, K>(f, lo, m, L);
  gl_panel<T, K>(f, m, hi, R);
  double err = 0, mag = 0;
  for (int k = 0; k < K; ++k) {
    err += std::fabs(val(L[k]) + val(R[k]) - val(whole[k]));
    mag += std::fabs(val(L[k])) + std::fabs(val(R[k]));
  }
  // stop at the requested tolerance, at the rounding floor of this panel, or at a
  // depth cap (panel width 2^-40 of the interval)
  --*budget;
  if (err <= tol || err <= 64 * 2.2e-16 * mag || depth >= 40 || *budget <= 0 || !(err == err)) {
    for (int k = 0; k < K; ++k) acc[k] = acc[k] + L[k] + R[k];
    return;
  }
  adapt<T, K>(f, lo, m, L, 0.5 * tol, depth + 1, acc, budget);
  adapt<T, K>(f, m, hi, R, 0.5 * tol, depth + 1, acc, budget);
}
template <class T, int K>
static void integrate(const std::function<void(double, T*)>& f, double lo, double hi, double rel, T* out) {
  T whole[K];
  gl_panel<T, K>(f, lo, hi, whole);
  double scale = 0;
  for (int k = 0; k < K; ++k) scale += std::fabs(val(whole[k]));
  for (int k = 0; k < K; ++k) out[k] = T(0.0);
  long budget = 100000;
  adapt<T, K>(f, lo, hi, whole, rel * scale + 1e-300, 0, out, &budget);
}

// ----------------------------------------------------------------------------
// Cosmology: flat LCDM, Omega_r = 0, w = -1 (defaults of Sec. 1: H0=70, Om=0.3).
// ----------------------------------------------------------------------------
static double comoving(double z1, double z2, double H0, double Om) {
  if (z2 == z1) return 0.0;
  std::function<void(double, double*)> f = [&](double z, double* o) {
    o[0] = 1.0 / std::sqrt(Om * (1 + z) * (1 + z) * (1 + z) + (1 - Om));
  };
  double r;
  integrate<double, 1>(f, z1, z2, 1e-15, &r);
  return C_KMS / H0 * r;
}
// angular diameter distance from z1 to z2 [Mpc]
static double dist(double z1, double z2, double H0, double Om) {
  return comoving(z1, z2, H0, Om) / (1 + z2);
}

// ----------------------------------------------------------------------------
// Profiles: deflection in the halo frame (a_dis-free, arcsec).
// Halo table row: type, x, y, b, q, pa, s, a.
//   POINT: b = Einstein radius;  SIS: b;  SIE: b, q, s (core);  PJE: b, q, s, a;
//   NFW: b = kappa_s, s = r_s;  ENFW: b = kappa_s, s = r_s, q, pa.
// ----------------------------------------------------------------------------
enum { POINT = 0, SIS = 1, SIE = 2, PJE = 3, NFW = 4, ENFW = 5, SHEAR = 6, MPOLE3 = 7 };
enum { F_SINGULAR = 1, F_GSING = 2, F_NOCONV = 4, F_REJECT = 8, F_MERGED = 16, F_OVERFLOW = 32, F_UMBILIC = 64 };

// Cored isothermal ellipsoid, kappa = (b/2) / sqrt(s^2 + x^2 + y^2/q^2), major axis on x.
template <class T>
static void sie_alpha(const T& x, const T& y, double b, double q, double s, T& ax, T& ay) {
  if (q >= 1.0) {
    T r2 = x * x + y * y;
    T d = sqrt(s * s + r2) + s;         // b x (sqrt(s^2+r^2) - s) / r^2 written without the 0/0
    ax = b * x / d; ay = b * y / d;
    return;
  }
  double e = std::sqrt(1 - q * q);
  T psi = sqrt(q * q * (s * s + x * x) + y * y);
  ax = (b * q / e) * atan(e * x / (psi + s));
  ay = (b * q / e) * atanh(e * y / (psi + q * q * s));
}

// NFW helper F(X) through z = 1 - X^2 (series near X = 1, closed forms elsewhere),
// and (F - 1)/z which gives kappa = 2 kappa_s (F - 1)/z without cancellation.
template <class T>
static void nfw_F(const T& z, T& F, T& Fm1_over_z, const T& X2in) {
  if (std::fabs(val(z)) < 0.1) {
    // F = sum_k z^k / (2k+1);  (F-1)/z = sum_{k>=1} z^(k-1)/(2k+1)
    T acc(0.0);
    for (int k = 40; k >= 1; --k) acc = acc * z + 1.0 / (2 * k + 1);
    Fm1_over_z = acc;
    F = 1.0 + z * acc;
  } else if (val(z) > 0) {          // X < 1: arccosh(1/X)/sqrt(1-X^2)
    // arccosh(1/X) = ln((1 + w)/X) with w = sqrt(1 - X^2): no overflow as X -> 0
    T w = sqrt(z);
    F = (log(1.0 + w) - 0.5 * log(X2in)) / w;
    Fm1_over_z = (F - 1.0) / z;
  } else {                          // X > 1: arccos(1/X)/sqrt(X^2-1)
    T w = sqrt(-1.0 * z);
    F = atan(w) / w;
    Fm1_over_z = (F - 1.0) / z;
  }
}
// circular NFW: alpha = 4 kappa_s r_s^2 h(X) / r^2 * (x, y), h = ln(X/2) + F(X)
template <class T>
static void nfw_alpha(const T& x, const T& y, double ks, double rs, T& ax, T& ay) {
  T r2 = x * x + y * y;
  T X2 = r2 / (rs * rs);
  T F, G;
  nfw_F(1.0 - X2, F, G, X2);
  T h = 0.5 * log(X2 / 4.0) + F;
  T m = 4.0 * ks * rs * rs * h / r2;
  ax = m * x; ay = m * y;
}
// NFW convergence as a function of xi^2 (elliptical radius squared)
template <class T>
static T nfw_kappa_xi2(const T& xi2, double ks, double rs) {
  T F, G;
  T X2 = xi2 / (rs * rs);
  nfw_F(1.0 - X2, F, G, X2);
  return 2.0 * ks * G;   // 2 ks (1 - F)/(X^2 - 1) = 2 ks (F - 1)/z
}
// Elliptical NFW with kappa(xi), xi^2 = x^2 + y^2/q^2, through the integrals
// J_n = int_0^1 kappa(xi^2(u)) (1 - e^2 u)^-(n+1/2) du, xi^2(u) = u (x^2 + y^2/(1-e^2 u)),
// alpha_x = q x J_0, alpha_y = q y J_1;  u = t^2 removes the endpoint singularity.
template <class T>
static void enfw_alpha(const T& x, const T& y, double ks, double rs, double q, T& ax, T& ay) {
  double e2 = 1 - q * q;
  T x2 = x * x, y2 = y * y;
  std::function<void(double, T*)> f = [&](double t, T* o) {
    double u = t * t;
    double w = 1 - e2 * u;
    T xi2 = u * (x2 + y2 / w);
    T k = nfw_kappa_xi2(xi2, ks, rs);
    double jac = 2 * t;
    o[0] = k * (jac / std::sqrt(w));
    o[1] = k * (jac / (w * std::sqrt(w)));
  };
  T Jn[2];
  integrate<T, 2>(f, 0.0, 1.0, 1e-14, Jn);
  ax = q * x * Jn[0];
  ay = q * y * Jn[1];
}

// One halo's deflection at image-plane point (X, Y).  Returns true if the point
// sits on a singular centre (then alpha = 0 and no derivatives).
template <class T>
static bool halo_alpha(const double* row, const T& X, const T& Y, T& ax, T& ay) {
  int type = (int)row[0];
  double xc = row[1], yc = row[2], b = row[3], q = row[4], pa = row[5], s = row[6], a = row[7];
  T dx = X - xc, dy = Y - yc;
  double r2v = val(dx) * val(dx) + val(dy) * val(dy);
  bool singular_type = (type == POINT || type == SIS || type == NFW || type == ENFW || type == MPOLE3 ||
                        ((type == SIE || type == PJE) && s == 0.0));
  if (singular_type && r2v < 1e-24) { ax = T(0.0); ay = T(0.0); return true; }
  if (type == SHEAR) {
    // external shear of amplitude b and angle pa: psi = (b/2) [(x^2 - y^2) cos 2pa + 2 x y sin 2pa]
    double c2 = std::cos(2 * pa), s2 = std::sin(2 * pa);
    ax = b * (c2 * dx + s2 * dy);
    ay = b * (s2 * dx - c2 * dy);
    return false;
  }
  if (type == MPOLE3) {
    // m = 3 multipole with psi ~ r^2: psi = (b/3) r^2 cos 3(phi - pa) = (b/3) (x'^3 - 3 x' y'^2) / r
    // in the frame turned by pa; alpha = grad psi
    double c = std::cos(pa), sn = std::sin(pa);
    T xp = c * dx + sn * dy, yp = -sn * dx + c * dy;
    T r = sqrt(xp * xp + yp * yp);
    T u = xp * xp * xp - 3.0 * xp * yp * yp;
    T ux = 3.0 * xp * xp - 3.0 * yp * yp, uy = -6.0 * xp * yp;
    double A = b / 3.0;
    T r3 = r * r * r;
    T axp = A * (ux / r - u * xp / r3), ayp = A * (uy / r - u * yp / r3);
    ax = c * axp - sn * ayp;
    ay = sn * axp + c * ayp;
    return false;
  }
  if (type == POINT) {
    T r2 = dx * dx + dy * dy;
    ax = b * b * dx / r2; ay = b * b * dy / r2; return false;
  }
  if (type == SIS) {
    T r = sqrt(dx * dx + dy * dy);
    ax = b * dx / r; ay = b * dy / r; return false;
  }
  if (type == NFW) { nfw_alpha(dx, dy, b, s, ax, ay); return false; }
  double c = std::cos(pa), sn = std::sin(pa);
  T xp = c * dx + sn * dy, yp = -sn * dx + c * dy;
  T axp, ayp;
  if (type == SIE) {
    sie_alpha(xp, yp, b, q, s, axp, ayp);
  } else if (type == PJE) {
    T a1x, a1y, a2x, a2y;
    sie_alpha(xp, yp, b, q, s, a1x, a1y);
    sie_alpha(xp, yp, b, q, a, a2x, a2y);
    axp = a1x - a2x; ayp = a1y - a2y;
  } else {  // ENFW
    if (q >= 1.0) nfw_alpha(xp, yp, b, s, axp, ayp);
    else enfw_alpha(xp, yp, b, s, q, axp, ayp);
  }
  ax = c * axp - sn * ayp;
  ay = sn * axp + c * ayp;
  return false;
}

// Sum over halos in table order at point (x, y).
// out: ax, ay, p11, p12, p22, p111, p112, p122, p222 ; returns flags.
static int halo_sum(const double* tab, int H, double x, double y, double* out) {
  J X = var_x(x), Y = var_y(y);
  J ax(0.0), ay(0.0);
  int flags = 0;
  for (int h = 0; h < H; ++h) {
    J hx, hy;
    if (halo_alpha(tab + 8 * h, X, Y, hx, hy)) flags |= F_SINGULAR;
    ax = ax + hx; ay = ay + hy;
  }
  out[0] = ax.v; out[1] = ay.v;
  out[2] = ax.dx; out[3] = ax.dy; out[4] = ay.dy;
  out[5] = ax.hxx; out[6] = ax.hxy; out[7] = ax.hyy; out[8] = ay.hyy;
  return flags;
}
// value-only deflection (fast path used where derivatives are not needed)
static int halo_sum_alpha(const double* tab, int H, double x, double y, double* ax, double* ay) {
  double sx = 0, sy = 0; int flags = 0;
  for (int h = 0; h < H; ++h) {
    double hx, hy;
    if (halo_alpha<double>(tab + 8 * h, x, y, hx, hy)) flags |= F_SINGULAR;
    sx += hx; sy += hy;
  }
  *ax = sx; *ay = sy; return flags;
}

// ----------------------------------------------------------------------------
// Lensing potential psi (Sec. 2.1, defined without a_dis), one halo, FP64, each profile
// up to its own additive constant (time delays only use differences within a family,
// whose common offset is the fitted zero point).  Closed forms, textbook derivations:
//   point mass  b^2 ln r;  SIS  b r;  circular cored  b (R - s ln(R + s)), R = sqrt(s^2 + r^2);
//   elliptical cored SIE  x alpha_x + y alpha_y - b q s ln sqrt((psi~ + s)^2 + e^2 x^2)
//     (halo frame, psi~ = sqrt(q^2 (s^2 + x^2) + y^2), e^2 = 1 - q^2);
//   PJE = SIE(s) - SIE(a);  NFW  2 kappa_s r_s^2 h(X), h = ln^2(X/2) - arccosh^2(1/X) (X < 1),
//     ln^2(X/2) + arccos^2(1/X) (X > 1);
//   elliptical NFW  (q/2) int_0^1 xi(u) alpha_c(xi(u)) / (u sqrt(1 - e^2 u)) du with
//     xi alpha_c(xi) = 4 kappa_s r_s^2 (ln(X/2) + F(X)), X = xi / r_s (the deflection of the
//     circular profile with the same kappa), u = t^2.
// Pinned in the tests by grad psi = alpha (central differences) for every profile.
// ----------------------------------------------------------------------------
static double sie_potential(double x, double y, double b, double q, double s) {
  if (q >= 1.0) {
    double R = std::sqrt(s * s + x * x + y * y);
    return b * (R - (s > 0 ? s * std::log(R + s) : 0.0));
  }
  double e2 = 1 - q * q;
  double psi = std::sqrt(q * q * (s * s + x * x) + y * y);
  double ax, ay;
  sie_alpha<double>(x, y, b, q, s, ax, ay);
  double v = x * ax + y * ay;
  if (s > 0) v -= b * q * s * 0.5 * std::log((psi + s) * (psi + s) + e2 * x * x);
  return v;
}
// ln(X/2) + F(X) (the bracket of the circular NFW deflection)
static double nfw_g(double X2) {
  double F, G;
  nfw_F<double>(1.0 - X2, F, G, X2);
  return 0.5 * std::log(X2 / 4.0) + F;
}
static double nfw_potential(double r2, double ks, double rs) {
  double X2 = r2 / (rs * rs);
  double X = std::sqrt(X2);
  double l = std::log(X / 2);
  double h;
  if (X < 1) { double ac = std::log((1 + std::sqrt(1 - X2)) / X); h = l * l - ac * ac; }
  else { double ac = std::acos(1 / X); h = l * l + ac * ac; }
  return 2 * ks * rs * rs * h;
}
static double enfw_potential(double x, double y, double ks, double rs, double q) {
  double e2 = 1 - q * q;
  std::function<void(double, double*)> f = [&](double t, double* o) {
    if (t <= 0) { o[0] = 0; return; }
    double u = t * t, w = 1 - e2 * u;
    double xi2 = u * (x * x + y * y / w);
    double xa = 4 * ks * rs * rs * nfw_g(xi2 / (rs * rs));
    o[0] = xa * 2 * t / (u * std::sqrt(w));
  };
  double I[1];
  integrate<double, 1>(f, 0.0, 1.0, 1e-13, I);
  return 0.5 * q * I[0];
}
static double halo_potential(const double* row, double X, double Y, bool* singular) {
  int type = (int)row[0];
  double xc = row[1], yc = row[2], b = row[3], q = row[4], pa = row[5], s = row[6], a = row[7];
  double dx = X - xc, dy = Y - yc;
  double r2 = dx * dx + dy * dy;
  bool singular_type = (type == POINT || type == SIS || type == NFW || type == ENFW || type == MPOLE3 ||
                        ((type == SIE || type == PJE) && s == 0.0));
  *singular = singular_type && r2 < 1e-24;
  if (*singular) return 0.0;
  if (type == SHEAR)
    return 0.5 * b * ((dx * dx - dy * dy) * std::cos(2 * pa) + 2 * dx * dy * std::sin(2 * pa));
  if (type == MPOLE3) {
    double c = std::cos(pa), sn = std::sin(pa);
    double xp = c * dx + sn * dy, yp = -sn * dx + c * dy;
    return (b / 3.0) * (xp * xp * xp - 3 * xp * yp * yp) / std::sqrt(r2);
  }
  if (type == POINT) return b * b * 0.5 * std::log(r2);
  if (type == SIS) return b * std::sqrt(r2);
  if (type == NFW) return nfw_potential(r2, b, s);
  double c = std::cos(pa), sn = std::sin(pa);
  double xp = c * dx + sn * dy, yp = -sn * dx + c * dy;
  if (type == SIE) return sie_potential(xp, yp, b, q, s);
  if (type == PJE) return sie_potential(xp, yp, b, q, s) - sie_potential(xp, yp, b, q, a);
  if (q >= 1.0) return nfw_potential(r2, b, s);
  return enfw_potential(xp, yp, b, s, q);
}
static int potential_sum(const double* tab, int H, double x, double y, double* pot) {
  double acc = 0; int flags = 0;
  for (int h = 0; h < H; ++h) {
    bool sg;
    acc += halo_potential(tab + 8 * h, x, y, &sg);
    if (sg) flags |= F_SINGULAR;
  }
  *pot = acc;
  return flags;
}

// ----------------------------------------------------------------------------
// Halo-table expansion (Sec. 3.4 Eq. scaling; unit conversions).
// ----------------------------------------------------------------------------
enum { XF_NONE = 0, XF_SIGMA_TO_B = 1, XF_KPC = 2, XF_EPS_TO_Q = 3, XF_DEG = 4, XF_M200 = 5, XF_C200 = 6 };

static void nfw_params(double H0, double Om, double zd, double m200, double c200, double* ks, double* rs_arcsec) {
  double Hz = H0 * std::sqrt(Om * std::pow(1 + zd, 3) + 1 - Om);
  double rho_c = 3 * Hz * Hz / (8 * PI * G_MPC);                 // Msun / Mpc^3
  double r200 = std::cbrt(3 * m200 / (4 * PI * 200 * rho_c));     // Mpc
  double rs = r200 / c200;
  double dc = (200.0 / 3.0) * c200 * c200 * c200 / (std::log(1 + c200) - c200 / (1 + c200));
  double Dd = dist(0, zd, H0, Om);
  double sigma_cr = C_KMS * C_KMS / (4 * PI * G_MPC * Dd);        // Msun / Mpc^2 (a_dis-free)
  *ks = dc * rho_c * rs / sigma_cr;
  *rs_arcsec = rs / Dd * ARCSEC;
}

struct Binding { int kind, index, xf; double value; };

static double apply_xf(int xf, double raw, double Dd) {
  switch (xf) {
    case XF_NONE: return raw;
    case XF_SIGMA_TO_B: return 4 * PI * (raw / C_KMS) * (raw / C_KMS) * ARCSEC;
    case XF_KPC: return raw / 1000.0 / Dd * ARCSEC;
    case XF_EPS_TO_Q: return (1 - raw) / (1 + raw);
    case XF_DEG: return raw * PI / 180.0;
    default: return raw;   // M200 / C200 are handled jointly by the caller
  }
}
static double raw_value(const Binding& bd, const double* params, int n_free, int* err) {
  if (bd.kind == 0) return bd.value;
  if (bd.index < 0 || bd.index >= n_free) { *err = -1; return 0; }
  return params[bd.index];
}

}  // namespace orc

using namespace orc;

extern "C" {

int orc_version() { return 1; }

double orc_dist(double z1, double z2, double H0, double Om) { return dist(z1, z2, H0, Om); }

double orc_comoving(double z1, double z2, double H0, double Om) { return comoving(z1, z2, H0, Om); }

double orc_adis(double zd, double zs, double H0, double Om) {
  return dist(zd, zs, H0, Om) / dist(0, zs, H0, Om);
}

double orc_sigma_to_b(double sigma) { return apply_xf(XF_SIGMA_TO_B, sigma, 1.0); }

void orc_nfw_params(double H0, double Om, double zd, double m200, double c200, double* ks, double* rs) {
  nfw_params(H0, Om, zd, m200, c200, ks, rs);
}

// Expand one parameter sample of a model into a flat halo table [H x 8]
// (type, x, y, b, q, pa, s, a), main components first then members in catalog order.
// Bindings are packed as int[4] {kind, index, xf, 0} + double value.
// Returns 0 on success, negative on invalid input.
int orc_expand(int n_main, const int* main_type, const int* main_bind /*[n_main*7*3]*/,
               const double* main_val /*[n_main*7]*/,
               int n_mem, const int* mem_type, const double* mem_x, const double* mem_y,
               const double* mem_q, const double* mem_pa,
               const double* mem_lum, const double* exps /*lam,bet,alp*/,
               const double* mem_b0, const double* mem_s0, const double* mem_a0,
               const int* mul_bind /*[3*3]*/, const double* mul_val /*[3]*/,
               double zd, double H0, double Om,
               const double* params, int n_free, double* out) {
  int err = 0;
  double Dd = dist(0, zd, H0, Om);
  for (int m = 0; m < n_main; ++m) {
    double f[7];
    int xfs[7];
    for (int k = 0; k < 7; ++k) {
      Binding bd{main_bind[(m * 7 + k) * 3 + 0], main_bind[(m * 7 + k) * 3 + 1],
                 main_bind[(m * 7 + k) * 3 + 2], main_val[m * 7 + k]};
      double raw = raw_value(bd, params, n_free, &err);
      xfs[k] = bd.xf;
      f[k] = (bd.xf == XF_M200 || bd.xf == XF_C200) ? raw : apply_xf(bd.xf, raw, Dd);
    }
    if (xfs[2] == XF_M200 || xfs[5] == XF_C200) {
      if (!(xfs[2] == XF_M200 && xfs[5] == XF_C200)) return -2;
      double ks, rs;
      nfw_params(H0, Om, zd, f[2], f[5], &ks, &rs);
      f[2] = ks; f[5] = rs;
    }
    double* row = out + 8 * m;
    row[0] = main_type[m];
    for (int k = 0; k < 7; ++k) row[1 + k] = f[k];
  }
  double mul[3];
  for (int k = 0; k < 3; ++k) {
    Binding bd{mul_bind[k * 3 + 0], mul_bind[k * 3 + 1], mul_bind[k * 3 + 2], mul_val[k]};
    mul[k] = apply_xf(bd.xf, raw_value(bd, params, n_free, &err), Dd);
  }
  for (int i = 0; i < n_mem; ++i) {
    double fb, fs, fa;
    if (mem_lum) {   // Eq. (scaling): v_d ~ L^lam (b ~ v_d^2), core ~ L^bet, cut ~ L^alp
      fb = std::pow(mem_lum[i], 2 * exps[0]);
      fs = std::pow(mem_lum[i], exps[1]);
      fa = std::pow(mem_lum[i], exps[2]);
    } else {
      fb = mem_b0[i]; fs = mem_s0[i]; fa = mem_a0[i];
    }
    double* row = out + 8 * (n_main + i);
    row[0] = mem_type[i]; row[1] = mem_x[i]; row[2] = mem_y[i];
    row[3] = mul[0] * fb; row[4] = mem_q ? mem_q[i] : 1.0; row[5] = mem_pa ? mem_pa[i] : 0.0;
    row[6] = mul[1] * fs; row[7] = mul[2] * fa;
  }
  if (err) return err;
  // validation
  int H = n_main + n_mem;
  for (int h = 0; h < H; ++h) {
    const double* r = out + 8 * h;
    for (int k = 1; k < 8; ++k) if (!std::isfinite(r[k])) return -3;
    int t = (int)r[0];
    if (t < 0 || t > 7) return -4;
    if (!(r[4] > 0 && r[4] <= 1)) return -5;
    if (r[3] < 0 || r[6] < 0) return -6;
    if (t == PJE && !(r[7] > r[6])) return -7;
    if ((t == NFW || t == ENFW) && !(r[6] > 0)) return -8;
  }
  return 0;
}

// Per-point maps.  out row (stride 20):
//  0 ax 1 ay 2 p11 3 p12 4 p22 5 p111 6 p112 7 p122 8 p222
//  9 kappa 10 gamma1 11 gamma2 12 detA 13 mu 14 beta_x 15 beta_y
//  16 e1 17 e2 18 f1 19 f2     ; flags[P]
static void epilogue_single(double x, double y, double a, const double* h, double* o, int* flags) {
  for (int k = 0; k < 9; ++k) o[k] = h[k];
  double p11 = h[2], p12 = h[3], p22 = h[4];
  double kap = 0.5 * (p11 + p22), g1 = 0.5 * (p11 - p22), g2 = p12;
  o[9] = kap; o[10] = g1; o[11] = g2;
  double A11 = 1 - a * p11, A22 = 1 - a * p22, A12 = -a * p12;   // Eq. (jac)
  double det = A11 * A22 - A12 * A12;
  o[12] = det; o[13] = 1.0 / det;
  o[14] = x - a * h[0]; o[15] = y - a * h[1];                      // Eq. (lens_eq)
  double gm = std::sqrt(g1 * g1 + g2 * g2);
  o[16] = kap + gm; o[17] = kap - gm;
  // A3-line fields: f_k = v_k . grad e_k (derivatives from the third-order terms)
  double p111 = h[5], p112 = h[6], p122 = h[7], p222 = h[8];
  double gkx = 0.5 * (p111 + p122), gky = 0.5 * (p112 + p222);
  double g1x = 0.5 * (p111 - p122), g1y = 0.5 * (p112 - p222);
  double g2x = p112, g2y = p122;
  if (gm <= 1e-12 * (std::fabs(kap) + 1e-300) || gm == 0.0) {
    o[18] = 0; o[19] = 0; *flags |= F_UMBILIC;
  } else {
    double ggx = (g1 * g1x + g2 * g2x) / gm, ggy = (g1 * g1y + g2 * g2y) / gm;
    double e1x = gkx + ggx, e1y = gky + ggy, e2x = gkx - ggx, e2y = gky - ggy;
    double vax = g1 + gm, vay = g2, vbx = g2, vby = gm - g1;
    double na = vax * vax + vay * vay, nb = vbx * vbx + vby * vby;
    double vx, vy;
    if (na >= nb) { double n = std::sqrt(na); vx = vax / n; vy = vay / n; }
    else { double n = std::sqrt(nb); vx = vbx / n; vy = vby / n; }
    if (vx < 0 || (vx == 0 && vy < 0)) { vx = -vx; vy = -vy; }
    double wx = -vy, wy = vx;    // eigenvector of e2 (perpendicular)
    if (wx < 0 || (wx == 0 && wy < 0)) { wx = -wx; wy = -wy; }
    o[18] = vx * e1x + vy * e1y;
    o[19] = wx * e2x + wy * e2y;
  }
}

static void parallel_for(int n, int nthreads, const std::function<void(int, int)>& body) {
  if (nthreads <= 1 || n < 2) { body(0, n); return; }
  nthreads = std::min(nthreads, n);
  std::vector<std::thread> th;
  int chunk = (n + nthreads - 1) / nthreads;
  for (int t = 0; t < nthreads; ++t) {
    int lo = t * chunk, hi = std::min(n, lo + chunk);
    if (lo >= hi) break;
    th.emplace_back([=, &body]() { body(lo, hi); });
  }
  for (auto& t : th) t.join();
}

int orc_maps(const double* tab, int H, const double* px, const double* py, int P, double a_dis,
             double* out, int* flags, int nthreads) {
  parallel_for(P, nthreads, [&](int lo, int hi) {
    for (int p = lo; p < hi; ++p) {
      double h[9];
      int fl = halo_sum(tab, H, px[p], py[p], h);
      epilogue_single(px[p], py[p], a_dis, h, out + 20 * p, &fl);
      flags[p] = fl;
    }
  });
  return 0;
}

// deflection only (for tests and the CPU-baseline timing of alpha-only maps)
int orc_alpha(const double* tab, int H, const double* px, const double* py, int P,
              double* ax, double* ay, int nthreads) {
  parallel_for(P, nthreads, [&](int lo, int hi) {
    for (int p = lo; p < hi; ++p) halo_sum_alpha(tab, H, px[p], py[p], ax + p, ay + p);
  });
  return 0;
}

// ----------------------------------------------------------------------------
// Multi-plane (Sec. 2.2).  Planes are sorted by redshift.  For each point and each
// requested source redshift: beta (2), A (4: A11 A12 A21 A22), mu.  Planes at or
// behind the source do not deflect it.  Also returns per-plane alpha at theta_j.
// ----------------------------------------------------------------------------
int orc_multiplane(int n_planes, const double* const* tabs, const int* Hs, const double* zp,
                   double H0, double Om, const double* zs, int n_zs,
                   const double* px, const double* py, int P,
                   double* beta /*[n_zs][P][2]*/, double* Aout /*[n_zs][P][4]*/, double* mu /*[n_zs][P]*/,
                   double* alpha_planes /*[n_planes][P][2] or null*/, int* flags, int nthreads) {
  int N = n_planes;
  std::vector<double> Dj(N), Dij(N * N, 0.0), Ds(n_zs), Djs(N * n_zs);
  for (int j = 0; j < N; ++j) {
    Dj[j] = dist(0, zp[j], H0, Om);
    for (int i = 0; i < j; ++i) Dij[i * N + j] = dist(zp[i], zp[j], H0, Om);
  }
  for (int k = 0; k < n_zs; ++k) {
    Ds[k] = dist(0, zs[k], H0, Om);
    for (int j = 0; j < N; ++j) Djs[j * n_zs + k] = (zp[j] < zs[k]) ? dist(zp[j], zs[k], H0, Om) : 0.0;
  }
  parallel_for(P, nthreads, [&](int lo, int hi) {
    std::vector<double> al(2 * N), Hm(3 * N), Am(4 * N);
    for (int p = lo; p < hi; ++p) {
      int fl = 0;
      for (int j = 0; j < N; ++j) {
        // theta_j = theta_1 - sum_{i<j} D_ij/D_j alpha_i(theta_i)
        double tx = px[p], ty = py[p];
        double A11 = 1, A12 = 0, A21 = 0, A22 = 1;
        for (int i = 0; i < j; ++i) {
          double w = Dij[i * N + j] / Dj[j];
          tx -= w * al[2 * i]; ty -= w * al[2 * i + 1];
          // A_j = I - sum_{i<j} w H_i A_i
          const double* Hh = &Hm[3 * i]; const double* Ai = &Am[4 * i];
          A11 -= w * (Hh[0] * Ai[0] + Hh[1] * Ai[2]);
          A12 -= w * (Hh[0] * Ai[1] + Hh[1] * Ai[3]);
          A21 -= w * (Hh[1] * Ai[0] + Hh[2] * Ai[2]);
          A22 -= w * (Hh[1] * Ai[1] + Hh[2] * Ai[3]);
        }
        double h[9];
        fl |= halo_sum(tabs[j], Hs[j], tx, ty, h);
        al[2 * j] = h[0]; al[2 * j + 1] = h[1];
        Hm[3 * j] = h[2]; Hm[3 * j + 1] = h[3]; Hm[3 * j + 2] = h[4];
        Am[4 * j] = A11; Am[4 * j + 1] = A12; Am[4 * j + 2] = A21; Am[4 * j + 3] = A22;
        if (alpha_planes) {
          alpha_planes[(size_t)(j * P + p) * 2] = h[0];
          alpha_planes[(size_t)(j * P + p) * 2 + 1] = h[1];
        }
      }
      for (int k = 0; k < n_zs; ++k) {
        double bx = px[p], by = py[p];
        double A11 = 1, A12 = 0, A21 = 0, A22 = 1;
        for (int j = 0; j < N; ++j) {
          if (!(zp[j] < zs[k])) continue;
          double w = Djs[j * n_zs + k] / Ds[k];
          bx -= w * al[2 * j]; by -= w * al[2 * j + 1];
          const double* Hh = &Hm[3 * j]; const double* Aj = &Am[4 * j];
          A11 -= w * (Hh[0] * Aj[0] + Hh[1] * Aj[2]);
          A12 -= w * (Hh[0] * Aj[1] + Hh[1] * Aj[3]);
          A21 -= w * (Hh[1] * Aj[0] + Hh[2] * Aj[2]);
          A22 -= w * (Hh[1] * Aj[1] + Hh[2] * Aj[3]);
        }
        size_t o = (size_t)k * P + p;
        beta[2 * o] = bx; beta[2 * o + 1] = by;
        Aout[4 * o] = A11; Aout[4 * o + 1] = A12; Aout[4 * o + 2] = A21; Aout[4 * o + 3] = A22;
        mu[o] = 1.0 / (A11 * A22 - A12 * A21);
      }
      flags[p] = fl;
    }
  });
  return 0;
}

// ----------------------------------------------------------------------------
// chi^2 (Sec. 3.1).  Constraint images grouped by family id (any order).
// Writes chi2_src, chi2_img (if img_mode), flags, beta_model [n_fam*2],
// theta_model [n_img*2] for one halo table.
// ----------------------------------------------------------------------------
static void sinv(double s1, double s2, double phi, double* S) {
  // S = R^T diag(s1^2, s2^2) R with R = [[c, s], [-s, c]];  inverse has 1/s^2 on the diagonal
  double c = std::cos(phi), s = std::sin(phi);
  double i1 = 1 / (s1 * s1), i2 = 1 / (s2 * s2);
  S[0] = c * c * i1 + s * s * i2;          // (0,0)
  S[1] = c * s * i1 - s * c * i2;          // (0,1) = (1,0)
  S[2] = s * s * i1 + c * c * i2;          // (1,1)
}

// Per-image quantities kept for the flux and time-delay terms.
struct ImgInfo {
  std::vector<double> h;    // [n][9] halo sums at theta_obs (alpha, psi_ij, psi_ijk)
  std::vector<int> ok;      // image-plane solution converged and accepted
};

static int chi2_one(const double* tab, int H, const double* th, const int* fam, const double* s1,
                    const double* s2, const double* phi, int n, const double* afam, int n_fam,
                    int img_mode, double newton_tol, double* chi_src, double* chi_img,
                    double* bmod, double* tmod, ImgInfo* info = nullptr, int* img_flags = nullptr) {
  int flags = 0;
  std::vector<double> bo(2 * n), W(3 * n), M(3 * n), Si(3 * n), detA0(n), csrc_i(n);
  if (info) { info->h.assign(9 * n, 0.0); info->ok.assign(n, 0); }
  for (int i = 0; i < n; ++i) {
    double h[9];
    flags |= halo_sum(tab, H, th[2 * i], th[2 * i + 1], h);
    if (info) std::copy(h, h + 9, info->h.begin() + 9 * i);
    double a = afam[fam[i]];
    bo[2 * i] = th[2 * i] - a * h[0]; bo[2 * i + 1] = th[2 * i + 1] - a * h[1];
    double A11 = 1 - a * h[2], A12 = -a * h[3], A22 = 1 - a * h[4];
    double det = A11 * A22 - A12 * A12;
    detA0[i] = det;
    double m11 = A22 / det, m12 = -A12 / det, m22 = A11 / det;      // mu = A^-1 (symmetric)
    double* S = &Si[3 * i];
    sinv(s1[i], s2[i], phi[i], S);
    M[3 * i] = m11; M[3 * i + 1] = m12; M[3 * i + 2] = m22;
    // W = mu^T S^-1 mu
    double t11 = S[0] * m11 + S[1] * m12, t12 = S[0] * m12 + S[1] * m22;
    double t21 = S[1] * m11 + S[2] * m12, t22 = S[1] * m12 + S[2] * m22;
    W[3 * i] = m11 * t11 + m12 * t21;
    W[3 * i + 1] = m11 * t12 + m12 * t22;
    W[3 * i + 2] = m12 * t12 + m22 * t22;
  }
  double total = 0;
  for (int f = 0; f < n_fam; ++f) {
    double G11 = 0, G12 = 0, G22 = 0, g1 = 0, g2 = 0;
    int cnt = 0;
    for (int i = 0; i < n; ++i) {
      if (fam[i] != f) continue;
      ++cnt;
      G11 += W[3 * i]; G12 += W[3 * i + 1]; G22 += W[3 * i + 2];
      g1 += W[3 * i] * bo[2 * i] + W[3 * i + 1] * bo[2 * i + 1];
      g2 += W[3 * i + 1] * bo[2 * i] + W[3 * i + 2] * bo[2 * i + 1];
    }
    double bx = 0, by = 0;
    if (cnt > 0) {
      double det = G11 * G22 - G12 * G12;
      double tr = G11 + G22;
      if (!(std::fabs(det) > 1e-12 * tr * tr)) {
        flags |= F_GSING;
        // pseudo-inverse along the dominant eigen-direction
        double lam = 0.5 * tr + std::sqrt(0.25 * (G11 - G22) * (G11 - G22) + G12 * G12);
        double vx = G12, vy = lam - G11;
        if (std::fabs(vx) + std::fabs(vy) == 0) { vx = 1; vy = 0; }
        double nv = std::sqrt(vx * vx + vy * vy); vx /= nv; vy /= nv;
        double proj = (vx * g1 + vy * g2) / (lam > 0 ? lam : 1);
        bx = proj * vx; by = proj * vy;
      } else {
        bx = (G22 * g1 - G12 * g2) / det;
        by = (-G12 * g1 + G11 * g2) / det;
      }
    }
    bmod[2 * f] = bx; bmod[2 * f + 1] = by;
    for (int i = 0; i < n; ++i) {
      if (fam[i] != f) continue;
      double dx = bo[2 * i] - bx, dy = bo[2 * i + 1] - by;
      // d^T W d = (mu d)^T S^-1 (mu d): the image-plane offset weighted by the error ellipse,
      // evaluated in the second form, which rounding cannot make negative when mu is huge
      const double* m = &M[3 * i];
      const double* S = &Si[3 * i];
      double vx = m[0] * dx + m[1] * dy, vy = m[1] * dx + m[2] * dy;
      double c = S[0] * vx * vx + 2 * S[1] * vx * vy + S[2] * vy * vy;
      csrc_i[i] = c;
      total += c;
    }
  }
  *chi_src = total;
  if (!img_mode) return flags;
  // image-plane: Newton from the observed position towards beta_model (Sec. 3.5)
  double tot_img = 0;
  for (int i = 0; i < n; ++i) {
    double a = afam[fam[i]];
    double bmx = bmod[2 * fam[i]], bmy = bmod[2 * fam[i] + 1];
    double tx = th[2 * i], ty = th[2 * i + 1];
    bool conv = false;
    double det_last = detA0[i];
    for (int it = 0; it < 20; ++it) {
      double h[9];
      halo_sum(tab, H, tx, ty, h);
      double rx = bmx - (tx - a * h[0]), ry = bmy - (ty - a * h[1]);
      double A11 = 1 - a * h[2], A12 = -a * h[3], A22 = 1 - a * h[4];
      double det = A11 * A22 - A12 * A12;
      det_last = det;
      double dx = (A22 * rx - A12 * ry) / det, dy = (-A12 * rx + A11 * ry) / det;
      tx += dx; ty += dy;
      if (std::sqrt(dx * dx + dy * dy) < newton_tol) { conv = true; break; }
    }
    double sig = std::max(s1[i], s2[i]);
    double ox = th[2 * i] - tx, oy = th[2 * i + 1] - ty;
    bool reject = !(std::sqrt(ox * ox + oy * oy) <= 10 * sig) || ((det_last > 0) != (detA0[i] > 0));
    tmod[2 * i] = tx; tmod[2 * i + 1] = ty;
    if (!conv) flags |= F_NOCONV;
    if (reject) flags |= F_REJECT;
    if (img_flags) img_flags[i] = (conv ? 0 : F_NOCONV) | (reject ? F_REJECT : 0);
    if (!conv || reject) {
      tot_img += csrc_i[i];
    } else {
      double S[3];
      sinv(s1[i], s2[i], phi[i], S);
      tot_img += ox * (S[0] * ox + S[1] * oy) + oy * (S[1] * ox + S[2] * oy);    // Eq. (chi2_img)
      if (info) info->ok[i] = 1;
    }
  }
  *chi_img = tot_img;
  return flags;
}

// Flux and time-delay terms (Sec. 3.2, 3.3) of one halo table, after the position fit.
// Per image i of family f (distance ratio a, time scale T = (1+z_d)/c D_d D_s/D_ds theta_0^2):
//   mu = 1/det A(theta_obs); grad mu = -mu^2 grad det A (third derivatives);
//   source plane (and images the image-plane solve did not accept):
//     mu_model = mu + (A^-1 (beta_model - beta_obs)) . grad mu          (linear expansion),
//     dt_model = T [|theta_obs - beta_obs|^2 / 2 - a psi(theta_obs)]
//                + T (beta_model - beta_obs) . (beta_obs - theta_obs)   Eq. (td_approx);
//   image plane (accepted images): mu_model = mu(theta_model),
//     dt_model = T [|theta_model - beta_model|^2 / 2 - a psi(theta_model)]   Eq. (time_delay);
//   per family: m_src by Eq. (msrc), chi2_f by Eq. (chi2_flux) (magnitudes: 2.5 log10 |mu|);
//   dt_0 by Eq. (dt0), chi2_dt by Eq. (chi2_td).
// An image enters a term only where its error (sig_mag, sig_dt) is positive.
static int obs_terms(const double* tab, int H, const double* th, const int* fam, int n, const double* afam,
                     int n_fam, const double* bmod, const double* tmod, const ImgInfo& I, int img_mode,
                     const double* mag, const double* smag, const double* dt, const double* sdt,
                     const double* tsc, double* chi_f, double* chi_t) {
  int flags = 0;
  std::vector<double> mval(n, 0.0), tval(n, 0.0);
  for (int i = 0; i < n; ++i) {
    bool want_f = mag && smag[i] > 0, want_t = dt && sdt[i] > 0;
    if (!want_f && !want_t) continue;
    int f = fam[i];
    double a = afam[f];
    const double* h = &I.h[9 * i];
    double tx = th[2 * i], ty = th[2 * i + 1];
    double bx = tx - a * h[0], by = ty - a * h[1];
    double A11 = 1 - a * h[2], A12 = -a * h[3], A22 = 1 - a * h[4];
    double det = A11 * A22 - A12 * A12, mu = 1 / det;
    double dbx = bmod[2 * f] - bx, dby = bmod[2 * f + 1] - by;
    double mu_m, t_m;
    bool img = img_mode && I.ok[i];
    if (img) {
      double mx = tmod[2 * i], my = tmod[2 * i + 1];
      double g[9], pot;
      flags |= halo_sum(tab, H, mx, my, g);
      flags |= potential_sum(tab, H, mx, my, &pot);
      double B11 = 1 - a * g[2], B12 = -a * g[3], B22 = 1 - a * g[4];
      mu_m = 1 / (B11 * B22 - B12 * B12);
      double ex = mx - bmod[2 * f], ey = my - bmod[2 * f + 1];
      t_m = want_t ? tsc[f] * (0.5 * (ex * ex + ey * ey) - a * pot) : 0.0;
    } else {
      double gdx = -a * (h[5] * A22 + A11 * h[7] - 2 * A12 * h[6]);
      double gdy = -a * (h[6] * A22 + A11 * h[8] - 2 * A12 * h[7]);
      double dthx = (A22 * dbx - A12 * dby) / det, dthy = (-A12 * dbx + A11 * dby) / det;
      mu_m = mu - mu * mu * (dthx * gdx + dthy * gdy);
      t_m = 0.0;
      if (want_t) {
        double pot;
        flags |= potential_sum(tab, H, tx, ty, &pot);
        double ex = tx - bx, ey = ty - by;
        t_m = tsc[f] * (0.5 * (ex * ex + ey * ey) - a * pot) + tsc[f] * (dbx * (bx - tx) + dby * (by - ty));
      }
    }
    if (want_f) mval[i] = mag[i] + 2.5 * std::log10(std::fabs(mu_m));
    if (want_t) tval[i] = dt[i] - t_m;
  }
  double cf = 0, ct = 0;
  for (int f = 0; f < n_fam; ++f) {
    double wf = 0, sf = 0, wt = 0, st = 0;
    for (int i = 0; i < n; ++i) {
      if (fam[i] != f) continue;
      if (mag && smag[i] > 0) { double w = 1 / (smag[i] * smag[i]); wf += w; sf += w * mval[i]; }
      if (dt && sdt[i] > 0) { double w = 1 / (sdt[i] * sdt[i]); wt += w; st += w * tval[i]; }
    }
    double msrc = wf > 0 ? sf / wf : 0, dt0 = wt > 0 ? st / wt : 0;      // Eq. (msrc), Eq. (dt0)
    for (int i = 0; i < n; ++i) {
      if (fam[i] != f) continue;
      if (mag && smag[i] > 0) { double d = mval[i] - msrc; cf += d * d / (smag[i] * smag[i]); }
      if (dt && sdt[i] > 0) { double d = tval[i] - dt0; ct += d * d / (sdt[i] * sdt[i]); }
    }
  }
  *chi_f = cf; *chi_t = ct;
  return flags;
}

// Position, flux and time-delay chi^2 terms of S halo tables (Sec. 3.1-3.3): chi_pos is
// the source-plane or image-plane position term; mag/smag and dt/sdt/tsc may be null.
int orc_chi2_obs(const double* tabs, int S, int H, const double* th, const int* fam,
                 const double* s1, const double* s2, const double* phi, int n,
                 const double* afam, int n_fam, int img_mode, double newton_tol,
                 const double* mag, const double* smag, const double* dt, const double* sdt,
                 const double* tsc, double* chi_pos, double* chi_f, double* chi_t, int* flags, int nthreads) {
  parallel_for(S, nthreads, [&](int lo, int hi) {
    std::vector<double> bm(2 * n_fam), tm(2 * n);
    ImgInfo I;
    for (int s = lo; s < hi; ++s) {
      const double* tab = tabs + (size_t)s * H * 8;
      double cs = 0, ci = 0;
      int fl = chi2_one(tab, H, th, fam, s1, s2, phi, n, afam, n_fam, img_mode, newton_tol, &cs, &ci,
                        bm.data(), tm.data(), &I);
      chi_pos[s] = img_mode ? ci : cs;
      fl |= obs_terms(tab, H, th, fam, n, afam, n_fam, bm.data(), tm.data(), I, img_mode, mag, smag, dt, sdt,
                      tsc, chi_f + s, chi_t + s);
      flags[s] = fl;
    }
  });
  return 0;
}

// Lensing potential sum at P points.
int orc_potential(const double* tab, int H, const double* px, const double* py, int P, double* pot, int* flags,
                  int nthreads) {
  parallel_for(P, nthreads, [&](int lo, int hi) {
    for (int p = lo; p < hi; ++p) flags[p] = potential_sum(tab, H, px[p], py[p], pot + p);
  });
  return 0;
}

// Time-delay scale (1 + z_d)/c D_d D_s / D_ds theta_0^2 with theta_0 = 1", in days per arcsec^2.
double orc_tdscale(double zd, double zs, double H0, double Om) {
  const double MPC_M = 3.0856775814913673e22, C_MS = 299792458.0, DAY = 86400.0;
  double Dd = dist(0, zd, H0, Om), Ds = dist(0, zs, H0, Om), Dds = dist(zd, zs, H0, Om);
  double th0 = 1.0 / ARCSEC;
  return (1 + zd) / C_MS * (Dd * Ds / Dds) * MPC_M * th0 * th0 / DAY;
}

// Batched over S halo tables (each [H x 8]).
int orc_chi2_batch(const double* tabs, int S, int H, const double* th, const int* fam,
                   const double* s1, const double* s2, const double* phi, int n,
                   const double* afam, int n_fam, int img_mode, double newton_tol,
                   double* chi_src, double* chi_img, int* flags, double* bmod, double* tmod,
                   int* img_flags, int nthreads) {
  parallel_for(S, nthreads, [&](int lo, int hi) {
    for (int s = lo; s < hi; ++s) {
      double ci = 0;
      flags[s] = chi2_one(tabs + (size_t)s * H * 8, H, th, fam, s1, s2, phi, n, afam, n_fam, img_mode,
                          newton_tol, chi_src + s, &ci, bmod + (size_t)s * n_fam * 2,
                          tmod + (size_t)s * n * 2, nullptr, img_flags + (size_t)s * n);
      if (img_mode) chi_img[s] = ci;
    }
  });
  return 0;
}

}  // extern "C"

// ----------------------------------------------------------------------------
// Exact orientation predicate (expansion arithmetic: error-free sums and
// products, Shewchuk-style), used for triangle containment.
// ----------------------------------------------------------------------------
namespace orc {
static inline void two_sum(double a, double b, double& x, double& y) {
  x = a + b; double bv = x - a; double av = x - bv; y = (a - av) + (b - bv);
}
static inline void two_prod(double a, double b, double& x, double& y) {
  x = a * b; y = std::fma(a, b, -x);
}
// e + b (e non-overlapping, increasing magnitude) -> h, zero-eliminated
static int grow(const double* e, int n, double b, double* h) {
  double Q = b; int k = 0;
  for (int i = 0; i < n; ++i) {
    double Qn, hh; two_sum(Q, e[i], Qn, hh); Q = Qn;
    if (hh != 0) h[k++] = hh;
  }
  if (Q != 0 || k == 0) h[k++] = Q;
  return k;
}
static int exp_sum(const double* e, int n, const double* f, int m, double* h) {
  std::vector<double> cur(e, e + n), nxt(n + m + 1);
  int len = n;
  for (int j = 0; j < m; ++j) { len = grow(cur.data(), len, f[j], nxt.data()); cur.assign(nxt.begin(), nxt.begin() + len); }
  for (int i = 0; i < len; ++i) h[i] = cur[i];
  return len;
}
static int scale(const double* e, int n, double b, double* h) {
  // exact e * b as an expansion (sum of error-free products, then summed exactly)
  std::vector<double> acc(1, 0.0), tmp;
  int len = 1;
  for (int i = 0; i < n; ++i) {
    double p, q; two_prod(e[i], b, p, q);
    double pr[2] = {q, p};
    tmp.assign(len + 3, 0.0);
    int l2 = exp_sum(acc.data(), len, pr, 2, tmp.data());
    acc.assign(tmp.begin(), tmp.begin() + l2); len = l2;
  }
  for (int i = 0; i < len; ++i) h[i] = acc[i];
  return len;
}
static int exp_sign(const double* e, int n) {
  for (int i = n - 1; i >= 0; --i) if (e[i] != 0) return e[i] > 0 ? 1 : -1;
  return 0;
}
// sign of (bx-ax)(cy-ay) - (by-ay)(cx-ax), exactly
static int orient_exact(double ax, double ay, double bx, double by, double cx, double cy) {
  double A[2], B[2], C[2], D[2];
  two_sum(bx, -ax, A[1], A[0]);
  two_sum(cy, -ay, B[1], B[0]);
  two_sum(by, -ay, C[1], C[0]);
  two_sum(cx, -ax, D[1], D[0]);
  double t1[16], t2[16], u[16], v[16], w[40];
  int n1 = scale(A, 2, B[0], t1), n2 = scale(A, 2, B[1], t2);
  int nu = exp_sum(t1, n1, t2, n2, u);
  n1 = scale(C, 2, -D[0], t1); n2 = scale(C, 2, -D[1], t2);
  int nv = exp_sum(t1, n1, t2, n2, v);
  int nw = exp_sum(u, nu, v, nv, w);
  return exp_sign(w, nw);
}
// lexicographic positivity of sigma * (q - p), decided by comparisons only
static bool edge_closed(int sigma, double px, double py, double qx, double qy) {
  if (sigma > 0) return qx > px || (qx == px && qy > py);
  return px > qx || (px == qx && py > qy);
}
static bool tri_contains(const double* B, double sx, double sy) {
  int sg = orient_exact(B[0], B[1], B[2], B[3], B[4], B[5]);
  if (sg == 0) return false;
  for (int e = 0; e < 3; ++e) {
    int a = e, b = (e + 1) % 3;
    int o = orient_exact(B[2 * a], B[2 * a + 1], B[2 * b], B[2 * b + 1], sx, sy);
    if (o == 0) { if (!edge_closed(sg, B[2 * a], B[2 * a + 1], B[2 * b], B[2 * b + 1])) return false; }
    else if (o != sg) return false;
  }
  return true;
}
}  // namespace orc

extern "C" {

int orc_orient(double ax, double ay, double bx, double by, double cx, double cy) {
  return orient_exact(ax, ay, bx, by, cx, cy);
}
int orc_tri_contains(const double* B, double sx, double sy) { return tri_contains(B, sx, sy) ? 1 : 0; }

// ----------------------------------------------------------------------------
// Image finder (triangle mapping).  Vertices at pixel centres x0 + (i+1/2)h.
// Cell (i, j) splits along its (i,j)-(i+1,j+1) diagonal:
//   tri 2c   = v(i,j), v(i+1,j), v(i+1,j+1);   tri 2c+1 = v(i,j), v(i+1,j+1), v(i,j+1),
//   c = j (nx-1) + i.
// A lens is either one halo table with a per-source distance ratio, or a list
// of planes with per-source plane weights (multi-plane).
// ----------------------------------------------------------------------------
struct Lens {
  // single plane
  const double* tab = nullptr; int H = 0;
  // multi-plane
  int N = 0; const double* const* tabs = nullptr; const int* Hs = nullptr;
  std::vector<double> wij;   // D_ij / D_j  [N*N]
};

// beta(theta) and A(theta) for source weights w (single plane: w[0] = a_dis;
// multi-plane: w[j] = D_js / D_s, zero for planes at or behind the source)
static int lens_eval(const Lens& L, const double* w, double x, double y, double* bx, double* by, double* A) {
  int fl = 0;
  if (L.N == 0) {
    double h[9];
    fl = halo_sum(L.tab, L.H, x, y, h);
    double a = w[0];
    *bx = x - a * h[0]; *by = y - a * h[1];
    A[0] = 1 - a * h[2]; A[1] = -a * h[3]; A[2] = -a * h[3]; A[3] = 1 - a * h[4];
    return fl;
  }
  int N = L.N;
  std::vector<double> al(2 * N), Hm(3 * N), Am(4 * N);
  double Bx = x, By = y, F11 = 1, F12 = 0, F21 = 0, F22 = 1;
  for (int j = 0; j < N; ++j) {
    double tx = x, ty = y, A11 = 1, A12 = 0, A21 = 0, A22 = 1;
    for (int i = 0; i < j; ++i) {
      double wi = L.wij[i * N + j];
      tx -= wi * al[2 * i]; ty -= wi * al[2 * i + 1];
      const double* Hh = &Hm[3 * i]; const double* Ai = &Am[4 * i];
      A11 -= wi * (Hh[0] * Ai[0] + Hh[1] * Ai[2]); A12 -= wi * (Hh[0] * Ai[1] + Hh[1] * Ai[3]);
      A21 -= wi * (Hh[1] * Ai[0] + Hh[2] * Ai[2]); A22 -= wi * (Hh[1] * Ai[1] + Hh[2] * Ai[3]);
    }
    double h[9];
    fl |= halo_sum(L.tabs[j], L.Hs[j], tx, ty, h);
    al[2 * j] = h[0]; al[2 * j + 1] = h[1];
    Hm[3 * j] = h[2]; Hm[3 * j + 1] = h[3]; Hm[3 * j + 2] = h[4];
    Am[4 * j] = A11; Am[4 * j + 1] = A12; Am[4 * j + 2] = A21; Am[4 * j + 3] = A22;
    if (w[j] == 0) continue;
    Bx -= w[j] * h[0]; By -= w[j] * h[1];
    F11 -= w[j] * (h[2] * A11 + h[3] * A21); F12 -= w[j] * (h[2] * A12 + h[3] * A22);
    F21 -= w[j] * (h[3] * A11 + h[4] * A21); F22 -= w[j] * (h[3] * A12 + h[4] * A22);
  }
  *bx = Bx; *by = By; A[0] = F11; A[1] = F12; A[2] = F21; A[3] = F22;
  return fl;
}

// per-plane deflections at a vertex (value only): single plane -> 1 pair,
// multi-plane -> alpha_j(theta_j) for every plane, from the recursion of Sec. 2.2
static void vertex_alphas(const Lens& L, double x, double y, double* al) {
  if (L.N == 0) { halo_sum_alpha(L.tab, L.H, x, y, al, al + 1); return; }
  int N = L.N;
  for (int j = 0; j < N; ++j) {
    double tx = x, ty = y;
    for (int i = 0; i < j; ++i) { tx -= L.wij[i * N + j] * al[2 * i]; ty -= L.wij[i * N + j] * al[2 * i + 1]; }
    halo_sum_alpha(L.tabs[j], L.Hs[j], tx, ty, al + 2 * j, al + 2 * j + 1);
  }
}

static int find_images(const Lens& L, const double* W /*[n_src * nw]*/, int nw,
                       double x0, double y0, double h, int nx, int ny,
                       const double* beta, int n_src, int max_img,
                       double* theta_out, double* mu_out, int* count, int* flags,
                       int* cand_src, int* cand_tri, int* cand_status, int max_cand, int* n_cand,
                       int nthreads) {
  size_t NV = (size_t)nx * ny;
  std::vector<double> vx(NV), vy(NV), val_al(NV * 2 * nw);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) { vx[(size_t)j * nx + i] = x0 + (i + 0.5) * h; vy[(size_t)j * nx + i] = y0 + (j + 0.5) * h; }
  parallel_for((int)NV, nthreads, [&](int lo, int hi) {
    for (int v = lo; v < hi; ++v) vertex_alphas(L, vx[v], vy[v], &val_al[(size_t)v * 2 * nw]);
  });
  // sources are independent items: each thread takes a range of them; candidates are listed
  // afterwards in source order
  std::vector<std::vector<int>> src_tris(n_src), src_status(n_src);
  parallel_for(n_src, nthreads, [&](int s_lo, int s_hi) {
    std::vector<double> bx(NV), by(NV);
    for (int s = s_lo; s < s_hi; ++s) {
      const double* w = W + (size_t)s * nw;
      for (size_t v = 0; v < NV; ++v) {
        double ex = vx[v], ey = vy[v];
        for (int j = 0; j < nw; ++j) { ex -= w[j] * val_al[v * 2 * nw + 2 * j]; ey -= w[j] * val_al[v * 2 * nw + 2 * j + 1]; }
        bx[v] = ex; by[v] = ey;
      }
      double sx = beta[2 * s], sy = beta[2 * s + 1];
      // candidates in triangle order
      std::vector<int> tris;
      for (int j = 0; j + 1 < ny; ++j)
        for (int i = 0; i + 1 < nx; ++i) {
          size_t v00 = (size_t)j * nx + i, v10 = v00 + 1, v01 = v00 + nx, v11 = v01 + 1;
          size_t vs[2][3] = {{v00, v10, v11}, {v00, v11, v01}};
          for (int k = 0; k < 2; ++k) {
            double B[6];
            double mnx = 1e300, mxx = -1e300, mny = 1e300, mxy = -1e300;
            for (int t = 0; t < 3; ++t) {
              B[2 * t] = bx[vs[k][t]]; B[2 * t + 1] = by[vs[k][t]];
              mnx = std::min(mnx, B[2 * t]); mxx = std::max(mxx, B[2 * t]);
              mny = std::min(mny, B[2 * t + 1]); mxy = std::max(mxy, B[2 * t + 1]);
            }
            if (sx < mnx || sx > mxx || sy < mny || sy > mxy) continue;   // exact prefilter
            if (tri_contains(B, sx, sy)) tris.push_back(2 * (j * (nx - 1) + i) + k);
          }
        }
      // polish each candidate (FP64 Newton, Sec. 3.5), accept, merge
      int cnt = 0, fl = 0;
      std::vector<double> acc_t;
      for (size_t c = 0; c < tris.size(); ++c) {
        int tri = tris[c], cell = tri / 2, k = tri % 2;
        int i = cell % (nx - 1), j = cell / (nx - 1);
        size_t v00 = (size_t)j * nx + i, v10 = v00 + 1, v01 = v00 + nx, v11 = v01 + 1;
        size_t vv[3];
        if (k == 0) { vv[0] = v00; vv[1] = v10; vv[2] = v11; } else { vv[0] = v00; vv[1] = v11; vv[2] = v01; }
        double B[6], T[6];
        for (int t = 0; t < 3; ++t) { B[2 * t] = bx[vv[t]]; B[2 * t + 1] = by[vv[t]]; T[2 * t] = vx[vv[t]]; T[2 * t + 1] = vy[vv[t]]; }
        // barycentric initial guess
        double area = (B[2] - B[0]) * (B[5] - B[1]) - (B[3] - B[1]) * (B[4] - B[0]);
        double l1 = ((B[4] - B[2]) * (sy - B[3]) - (B[5] - B[3]) * (sx - B[2])) / area;
        double l2 = ((B[0] - B[4]) * (sy - B[5]) - (B[1] - B[5]) * (sx - B[4])) / area;
        double l3 = 1 - l1 - l2;
        double tx0 = l1 * T[0] + l2 * T[2] + l3 * T[4], ty0 = l1 * T[1] + l2 * T[3] + l3 * T[5];
        double tx = tx0, ty = ty0, A[4] = {1, 0, 0, 1};
        bool conv = false;
        for (int it = 0; it <= 30; ++it) {
          double ex, ey;
          lens_eval(L, w, tx, ty, &ex, &ey, A);
          double rx = sx - ex, ry = sy - ey;
          if (std::fabs(rx) < 1e-10 && std::fabs(ry) < 1e-10) { conv = true; break; }
          if (it == 30) break;
          double det = A[0] * A[3] - A[1] * A[2];
          tx += (A[3] * rx - A[1] * ry) / det;
          ty += (-A[2] * rx + A[0] * ry) / det;
        }
        int status;
        if (!conv) status = 1;
        else if (std::fabs(tx - tx0) > 2 * h || std::fabs(ty - ty0) > 2 * h) status = 2;
        else {
          bool dup = false;
          for (size_t m = 0; m < acc_t.size(); m += 2) {
            double dx = tx - acc_t[m], dy = ty - acc_t[m + 1];
            if (std::sqrt(dx * dx + dy * dy) < 1e-6) { dup = true; break; }
          }
          if (dup) { status = 3; fl |= F_MERGED; }
          else {
            status = 0;
            acc_t.push_back(tx); acc_t.push_back(ty);
            if (cnt < max_img) {
              theta_out[((size_t)s * max_img + cnt) * 2] = tx;
              theta_out[((size_t)s * max_img + cnt) * 2 + 1] = ty;
              mu_out[(size_t)s * max_img + cnt] = 1.0 / (A[0] * A[3] - A[1] * A[2]);
            } else fl |= F_OVERFLOW;
            ++cnt;
          }
        }
        src_tris[s].push_back(tri);
        src_status[s].push_back(status);
      }
      count[s] = cnt;
      flags[s] = fl;
    }
  });
  int ncand_total = 0;
  for (int s = 0; s < n_src; ++s)
    for (size_t c = 0; c < src_tris[s].size(); ++c) {
      if (ncand_total < max_cand) {
        cand_src[ncand_total] = s; cand_tri[ncand_total] = src_tris[s][c]; cand_status[ncand_total] = src_status[s][c];
      }
      ++ncand_total;
    }
  *n_cand = ncand_total;
  return 0;
}

int orc_find_images(const double* tab, int H, double x0, double y0, double h, int nx, int ny,
                    const double* beta, const double* a_src, int n_src, int max_img,
                    double* theta_out, double* mu_out, int* count, int* flags,
                    int* cand_src, int* cand_tri, int* cand_status, int max_cand, int* n_cand, int nthreads) {
  Lens L; L.tab = tab; L.H = H;
  return find_images(L, a_src, 1, x0, y0, h, nx, ny, beta, n_src, max_img, theta_out, mu_out,
                     count, flags, cand_src, cand_tri, cand_status, max_cand, n_cand, nthreads);
}

int orc_find_images_mp(int n_planes, const double* const* tabs, const int* Hs, const double* zp,
                       double H0, double Om, double x0, double y0, double h, int nx, int ny,
                       const double* beta, const double* zs, int n_src, int max_img,
                       double* theta_out, double* mu_out, int* count, int* flags,
                       int* cand_src, int* cand_tri, int* cand_status, int max_cand, int* n_cand, int nthreads) {
  Lens L; L.N = n_planes; L.tabs = tabs; L.Hs = Hs;
  int N = n_planes;
  L.wij.assign(N * N, 0.0);
  for (int j = 0; j < N; ++j)
    for (int i = 0; i < j; ++i) L.wij[i * N + j] = dist(zp[i], zp[j], H0, Om) / dist(0, zp[j], H0, Om);
  std::vector<double> W((size_t)n_src * N, 0.0);
  for (int s = 0; s < n_src; ++s) {
    double Ds = dist(0, zs[s], H0, Om);
    for (int j = 0; j < N; ++j) W[(size_t)s * N + j] = (zp[j] < zs[s]) ? dist(zp[j], zs[s], H0, Om) / Ds : 0.0;
  }
  return find_images(L, W.data(), N, x0, y0, h, nx, ny, beta, n_src, max_img, theta_out, mu_out,
                     count, flags, cand_src, cand_tri, cand_status, max_cand, n_cand, nthreads);
}

// Image finder of Sec. 2.3: zero contours of f = beta - theta + a alpha (both components)
// by marching squares on the vertex grid x0 + (i+1/2)h, images at the exact intersections of
// pairs of contour segments in a cell.  Per cell (corners c0 = (i,j), c1 = (i+1,j),
// c2 = (i+1,j+1), c3 = (i,j+1); edges in loop order bottom c0-c1, right c1-c2, top c3-c2,
// left c0-c3), a component with two sign changes on the edges gives one segment joining the
// two linear-interpolation points, with four the asymptotic decider of its bilinear
// interpolant pairs them (zero counts as positive).  Intersections are taken for each
// f_1 segment with each f_2 segment, in that order, cells in row-major order.  polish: each
// intersection refined by FP64 Newton (<= 30 steps to |d beta| < 1e-10") and kept if it
// converged within 2h (max-norm) of it; images closer than 1e-6" to an earlier one are merged.
// Without polish the intersections themselves are the images (accuracy O(h^2)).
static int ms_segments(const double F[4], double seg[2][4]) {
  // crossing points on the loop edges in cell coordinates (xi, eta) in [0, 1]^2
  const double P[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
  const int ea[4] = {0, 1, 3, 0}, eb[4] = {1, 2, 2, 3};
  double X[4][2];
  int has[4], n = 0;
  for (int m = 0; m < 4; ++m) {
    double fa = F[ea[m]], fb = F[eb[m]];
    has[m] = (fa < 0) != (fb < 0);
    if (has[m]) {
      double t = fa / (fa - fb);
      X[m][0] = P[ea[m]][0] + t * (P[eb[m]][0] - P[ea[m]][0]);
      X[m][1] = P[ea[m]][1] + t * (P[eb[m]][1] - P[ea[m]][1]);
      ++n;
    }
  }
  auto put = [&](int k, int a, int b) { seg[k][0] = X[a][0]; seg[k][1] = X[a][1]; seg[k][2] = X[b][0]; seg[k][3] = X[b][1]; };
  if (n == 2) {
    int a = -1, b = -1;
    for (int m = 0; m < 4; ++m) if (has[m]) { if (a < 0) a = m; else b = m; }
    put(0, a, b);
    return 1;
  }
  if (n == 4) {
    double D = F[0] + F[2] - F[1] - F[3];
    bool cpos = D == 0.0 ? true : !((F[0] * F[2] - F[1] * F[3]) / D < 0);
    if (cpos == !(F[0] < 0)) { put(0, 0, 1); put(1, 2, 3); }
    else { put(0, 0, 3); put(1, 1, 2); }
    return 2;
  }
  return 0;
}

int orc_find_images_ms(const double* tab, int H, double x0, double y0, double h, int nx, int ny, const double* beta,
                       const double* a_src, int n_src, int max_img, int polish, double* theta_out, double* mu_out,
                       int* count, int* flags, int nthreads) {
  std::vector<double> vax((size_t)nx * ny), vay((size_t)nx * ny);
  parallel_for(ny, nthreads, [&](int lo, int hi) {
    for (int j = lo; j < hi; ++j)
      for (int i = 0; i < nx; ++i)
        halo_sum_alpha(tab, H, x0 + (i + 0.5) * h, y0 + (j + 0.5) * h, &vax[(size_t)j * nx + i], &vay[(size_t)j * nx + i]);
  });
  parallel_for(n_src, nthreads, [&](int lo, int hi) {
    for (int s = lo; s < hi; ++s) {
      const double a = a_src[s], sx = beta[2 * s], sy = beta[2 * s + 1];
      int cnt = 0, fl = 0;
      std::vector<double> got;
      for (int j = 0; j + 1 < ny; ++j)
        for (int i = 0; i + 1 < nx; ++i) {
          const int ci[4] = {i, i + 1, i + 1, i}, cj[4] = {j, j, j + 1, j + 1};
          double F1[4], F2[4];
          for (int k = 0; k < 4; ++k) {
            size_t v = (size_t)cj[k] * nx + ci[k];
            double tx = x0 + (ci[k] + 0.5) * h, ty = y0 + (cj[k] + 0.5) * h;
            F1[k] = sx - (tx - a * vax[v]);
            F2[k] = sy - (ty - a * vay[v]);
          }
          double S1[2][4], S2[2][4];
          int n1 = ms_segments(F1, S1);
          if (!n1) continue;
          int n2 = ms_segments(F2, S2);
          for (int p = 0; p < n1; ++p)
            for (int q = 0; q < n2; ++q) {
              double d1x = S1[p][2] - S1[p][0], d1y = S1[p][3] - S1[p][1];
              double d2x = S2[q][2] - S2[q][0], d2y = S2[q][3] - S2[q][1];
              double wx = S2[q][0] - S1[p][0], wy = S2[q][1] - S1[p][1];
              double den = d1x * d2y - d1y * d2x;
              if (den == 0.0) continue;
              double tp = (wx * d2y - wy * d2x) / den, tq = (wx * d1y - wy * d1x) / den;
              if (!(tp >= 0 && tp <= 1 && tq >= 0 && tq <= 1)) continue;
              double tx = x0 + (i + 0.5) * h + h * (S1[p][0] + tp * d1x);
              double ty = y0 + (j + 0.5) * h + h * (S1[p][1] + tp * d1y);
              double d[9];
              if (polish) {
                double px = tx, py = ty;
                bool conv = false;
                for (int it = 0; it <= 30; ++it) {
                  halo_sum(tab, H, px, py, d);
                  double rx = sx - (px - a * d[0]), ry = sy - (py - a * d[1]);
                  if (std::fabs(rx) < 1e-10 && std::fabs(ry) < 1e-10) { conv = true; break; }
                  if (it == 30) break;
                  double A11 = 1 - a * d[2], A12 = -a * d[3], A22 = 1 - a * d[4];
                  double det = A11 * A22 - A12 * A12;
                  px += (A22 * rx - A12 * ry) / det;
                  py += (-A12 * rx + A11 * ry) / det;
                }
                if (!conv || std::fabs(px - tx) > 2 * h || std::fabs(py - ty) > 2 * h) continue;
                tx = px; ty = py;
              } else {
                halo_sum(tab, H, tx, ty, d);
              }
              bool dup = false;
              for (size_t k = 0; k < got.size(); k += 2)
                if (std::sqrt((tx - got[k]) * (tx - got[k]) + (ty - got[k + 1]) * (ty - got[k + 1])) < 1e-6) dup = true;
              if (dup) { fl |= F_MERGED; continue; }
              got.push_back(tx); got.push_back(ty);
              double A11 = 1 - a * d[2], A12 = -a * d[3], A22 = 1 - a * d[4];
              if (cnt < max_img) {
                theta_out[((size_t)s * max_img + cnt) * 2] = tx;
                theta_out[((size_t)s * max_img + cnt) * 2 + 1] = ty;
                mu_out[(size_t)s * max_img + cnt] = 1.0 / (A11 * A22 - A12 * A12);
              } else {
                fl |= F_OVERFLOW;
              }
              ++cnt;
            }
        }
      count[s] = cnt;
      flags[s] = fl;
    }
  });
  return 0;
}

// vertex beta map of a single-plane lens (test helper for brute-force containment)
int orc_vertex_beta(const double* tab, int H, double x0, double y0, double h, int nx, int ny,
                    double a, double* bx, double* by) {
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      double x = x0 + (i + 0.5) * h, y = y0 + (j + 0.5) * h, ax, ay;
      halo_sum_alpha(tab, H, x, y, &ax, &ay);
      bx[(size_t)j * nx + i] = x - a * ax; by[(size_t)j * nx + i] = y - a * ay;
    }
  return 0;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// Singularity maps (Sec. 6): A3 lines, umbilics (D4) and swallowtails (A4) of a
// single-plane lens, extracted from the fields on a grid of vertices x0 + (i+1/2)h.
//
// Definitions (the cited formalism is not available; these follow from the cusp
// condition): e_1,2 = kappa +- |gamma| are the eigenvalues of the deformation tensor psi_ij
// and v_1,2 their unit eigenvectors.  A critical curve at distance ratio a is 1 - a e_k = 0,
// and it has a cusp where v_k is tangent to it, i.e. f_k = v_k . grad e_k = 0: the A3 line of
// e_k is the zero set of f_k (independent of a; the cusp there forms for a = 1/e_k).  v_k is
// a line field (defined up to sign), so f_k is compared between two points only after the
// second point's eigenvector has been aligned with the first's.  Around a point where
// gamma = 0 (an umbilic, D4: e_1 = e_2, the two A3 lines meet) the line field turns by a half
// turn, so the orientation product around a grid cell is -1 exactly for cells holding such a
// point.  A swallowtail (A4) lies on an A3 line where v_k is tangent to the line: there
// g_k = v_k . grad f_k (orientation independent) changes sign along the line.
// ---------------------------------------------------------------------------------------
struct SingVal {
  double kap, g1, g2, e[2], f[2], v[2][2];
  bool umb;
  int flags;
};

// Fields at one point.  Eigenvector of e_1: angle phi = atan2(gamma_2, gamma_1) / 2, the
// sign chosen with a positive x component (then y); v_2 is v_1 turned by +90 degrees with
// the same sign rule.  f_k = v_k . grad e_k with grad e_1,2 = grad kappa +- grad |gamma|.
static SingVal sing_at(const double* tab, int H, double x, double y) {
  double d[9];
  SingVal o;
  o.flags = halo_sum(tab, H, x, y, d);
  double p11 = d[2], p12 = d[3], p22 = d[4], p111 = d[5], p112 = d[6], p122 = d[7], p222 = d[8];
  o.kap = 0.5 * (p11 + p22);
  o.g1 = 0.5 * (p11 - p22);
  o.g2 = p12;
  double gm = std::hypot(o.g1, o.g2);
  o.e[0] = o.kap + gm;
  o.e[1] = o.kap - gm;
  o.umb = gm == 0.0 || gm <= 1e-12 * std::fabs(o.kap);
  if (o.umb) {
    o.f[0] = o.f[1] = 0.0;
    o.v[0][0] = 1; o.v[0][1] = 0; o.v[1][0] = 0; o.v[1][1] = 1;
    return o;
  }
  double phi = 0.5 * std::atan2(o.g2, o.g1);
  double vx = std::cos(phi), vy = std::sin(phi);
  if (vx < 0 || (vx == 0 && vy < 0)) { vx = -vx; vy = -vy; }
  double wx = -vy, wy = vx;
  if (wx < 0 || (wx == 0 && wy < 0)) { wx = -wx; wy = -wy; }
  o.v[0][0] = vx; o.v[0][1] = vy; o.v[1][0] = wx; o.v[1][1] = wy;
  double dkx = 0.5 * (p111 + p122), dky = 0.5 * (p112 + p222);       // grad kappa
  double d1x = 0.5 * (p111 - p122), d1y = 0.5 * (p112 - p222);       // grad gamma_1
  double d2x = p112, d2y = p122;                                     // grad gamma_2
  double dgx = (o.g1 * d1x + o.g2 * d2x) / gm, dgy = (o.g1 * d1y + o.g2 * d2y) / gm;
  o.f[0] = vx * (dkx + dgx) + vy * (dky + dgy);
  o.f[1] = wx * (dkx - dgx) + wy * (dky - dgy);
  return o;
}

static inline double vdot(const SingVal& a, const SingVal& b, int k) {
  return a.v[k][0] * b.v[k][0] + a.v[k][1] * b.v[k][1];
}
// +1 when b's eigenvector k points the same way as a's (dot >= 0), else -1
static inline double align(const SingVal& a, const SingVal& b, int k) { return vdot(a, b, k) >= 0 ? 1.0 : -1.0; }
// sign classes: zero counts as positive
static inline bool neg(double v) { return v < 0; }

struct SingGrid {
  const double* tab; int H;
  double x0, y0, h; int nx, ny;
  std::vector<SingVal> V;
  double X(int i) const { return x0 + (i + 0.5) * h; }
  double Y(int j) const { return y0 + (j + 0.5) * h; }
  const SingVal& at(int i, int j) const { return V[(size_t)j * nx + i]; }
};

// Edge test: does f_k change sign (after alignment) between vertices a and b?
static bool edge_cross(const SingVal& a, const SingVal& b, int k) {
  if (a.umb || b.umb) return false;
  return neg(a.f[k]) != neg(align(a, b, k) * b.f[k]);
}

// f_k at q aligned with reference eigenvector r
static double f_aligned(const double* tab, int H, double qx, double qy, const SingVal& r, int k, bool* umb) {
  SingVal q = sing_at(tab, H, qx, qy);
  if (q.umb) *umb = true;
  return align(r, q, k) * q.f[k];
}

struct Crossing { double x, y, e, g; int k, flags; int64_t key; };

// Crossing on the edge from vertex a = (ax, ay) to b = a + h (dir): linear interpolation, then
// (refine) the Illinois variant of regula falsi on t in [0, 1] until the bracket is below
// tol arcsec.  Then e_k and g_k = v_k . grad f_k (central differences, step 1e-3 h, f aligned
// with v_k at the crossing) at the crossing.  Flags: 1 an evaluation met an umbilic-flagged
// point, 2 no convergence in 100 steps, 4 (refine) |f_k| at the result above 1e-3 of its
// larger end value: a jump, not a root.
static Crossing refine_crossing(const SingGrid& G, double ax, double ay, double dxh, double dyh,
                                const SingVal& A, const SingVal& B, int k, bool refine, double tol) {
  Crossing c; c.k = k; c.flags = 0;
  double F0 = A.f[k], F1 = align(A, B, k) * B.f[k];
  const double Fend = std::max(std::fabs(F0), std::fabs(F1));
  double t0 = 0.0, t1 = 1.0;
  double t = F0 / (F0 - F1);
  if (refine) {
    int side = 0;
    bool done = false;
    for (int it = 0; it < 100 && !done; ++it) {
      double tn = (t0 * F1 - t1 * F0) / (F1 - F0);
      if (!(tn > t0 && tn < t1)) tn = 0.5 * (t0 + t1);
      bool u = false;
      double F = f_aligned(G.tab, G.H, ax + tn * dxh, ay + tn * dyh, A, k, &u);
      if (u) c.flags |= 1;
      t = tn;
      if (F == 0.0) { done = true; break; }
      if (neg(F) == neg(F0)) { t0 = tn; F0 = F; if (side == -1) F1 *= 0.5; side = -1; }
      else { t1 = tn; F1 = F; if (side == 1) F0 *= 0.5; side = 1; }
      if ((t1 - t0) * G.h < tol) { t = 0.5 * (t0 + t1); done = true; }
    }
    if (!done) c.flags |= 2;
  }
  c.x = ax + t * dxh;
  c.y = ay + t * dyh;
  SingVal P = sing_at(G.tab, G.H, c.x, c.y);
  if (P.umb) { c.flags |= 1; c.e = P.e[k]; c.g = 0.0; return c; }
  c.e = P.e[k];
  // a sign change that is not a root: f (aligned) jumps where the eigenvector turns by more
  // than a quarter turn along the edge (next to an umbilic) or across a singular centre
  if (refine && std::fabs(P.f[k]) > 1e-3 * Fend) c.flags |= 4;
  double d = 1e-3 * G.h;
  bool u = false;
  double fxp = f_aligned(G.tab, G.H, c.x + d, c.y, P, k, &u), fxm = f_aligned(G.tab, G.H, c.x - d, c.y, P, k, &u);
  double fyp = f_aligned(G.tab, G.H, c.x, c.y + d, P, k, &u), fym = f_aligned(G.tab, G.H, c.x, c.y - d, P, k, &u);
  if (u) c.flags |= 1;
  c.g = P.v[k][0] * (fxp - fxm) / (2 * d) + P.v[k][1] * (fyp - fym) / (2 * d);
  return c;
}

// g_k = v_k . grad f_k at q: f aligned with v_k(q), central differences with step d
static double g_at(const double* tab, int H, double x, double y, int k, double d, bool* umb, double* f,
                   double* fx, double* fy) {
  SingVal P = sing_at(tab, H, x, y);
  if (P.umb) *umb = true;
  double fxp = f_aligned(tab, H, x + d, y, P, k, umb), fxm = f_aligned(tab, H, x - d, y, P, k, umb);
  double fyp = f_aligned(tab, H, x, y + d, P, k, umb), fym = f_aligned(tab, H, x, y - d, P, k, umb);
  *f = P.f[k];
  *fx = (fxp - fxm) / (2 * d);
  *fy = (fyp - fym) / (2 * d);
  return P.v[k][0] * *fx + P.v[k][1] * *fy;
}

// Swallowtail refinement: Newton on (f_k, g_k) = 0 from the interpolated point; grad f from
// the differences inside g (step 1e-3 h), grad g from central differences of g (step
// 1e-2 h).  The iteration stops after a step below 1e-10", after 20 steps, or as soon as it
// leaves the disc of radius h about the start.  Status 0 converged (the last step is below
// 1e-8") within h of the start, 1 no convergence, 2 left the disc.  The acceptance test sits
// two decades above the stopping step: the finite-difference g leaves a rounding noise of up
// to ~1e-9" under the steps, so a test at 1e-10" would decide by that noise; and an iteration
// that wanders off is stopped while its path is still set by the lens rather than by rounding.
static int swallowtail_newton(const SingGrid& G, int k, double* px, double* py) {
  double x = *px, y = *py, d = 1e-3 * G.h, dg = 1e-2 * G.h;
  bool umb = false;
  double last = HUGE_VAL;
  for (int it = 0; it < 20; ++it) {
    double f, fx, fy, t0, t1, t2;
    double g = g_at(G.tab, G.H, x, y, k, d, &umb, &f, &fx, &fy);
    double gxp = g_at(G.tab, G.H, x + dg, y, k, d, &umb, &t0, &t1, &t2);
    double gxm = g_at(G.tab, G.H, x - dg, y, k, d, &umb, &t0, &t1, &t2);
    double gyp = g_at(G.tab, G.H, x, y + dg, k, d, &umb, &t0, &t1, &t2);
    double gym = g_at(G.tab, G.H, x, y - dg, k, d, &umb, &t0, &t1, &t2);
    double gx = (gxp - gxm) / (2 * dg), gy = (gyp - gym) / (2 * dg);
    double det = fx * gy - fy * gx;
    double sx = -(gy * f - fy * g) / det, sy = -(-gx * f + fx * g) / det;
    x += sx; y += sy;
    if (!std::isfinite(x) || !std::isfinite(y)) { last = HUGE_VAL; break; }
    last = std::sqrt(sx * sx + sy * sy);
    if (last < 1e-10) break;
    if (std::hypot(x - *px, y - *py) > G.h) break;
  }
  int st = last < 1e-8 ? 0 : 1;
  if (std::hypot(x - *px, y - *py) > G.h) st = 2;
  if (umb) st |= 8;
  if (st == 0) { *px = x; *py = y; }
  return st;
}

// Umbilic of a cell: Newton on (gamma_1, gamma_2) = 0 from the cell centre with the Jacobian
// from the third derivatives; status 0 accepted (converged inside the closed cell), 1 no
// convergence in 30 steps, 2 converged outside the cell.
static int umbilic_newton(const SingGrid& G, int i, int j, double* ux, double* uy, double* kap) {
  double x = G.X(i) + 0.5 * G.h, y = G.Y(j) + 0.5 * G.h;
  bool conv = false;
  for (int it = 0; it < 30; ++it) {
    double d[9];
    halo_sum(G.tab, G.H, x, y, d);
    double g1 = 0.5 * (d[2] - d[4]), g2 = d[3];
    double J11 = 0.5 * (d[5] - d[7]), J12 = 0.5 * (d[6] - d[8]), J21 = d[6], J22 = d[7];
    double det = J11 * J22 - J12 * J21;
    double sx = -(J22 * g1 - J12 * g2) / det, sy = -(-J21 * g1 + J11 * g2) / det;
    x += sx; y += sy;
    if (std::sqrt(sx * sx + sy * sy) < 1e-10) { conv = true; break; }
    if (!std::isfinite(x) || !std::isfinite(y)) break;
  }
  double d[9];
  halo_sum(G.tab, G.H, x, y, d);
  *ux = x; *uy = y; *kap = 0.5 * (d[2] + d[4]);
  if (!conv) return 1;
  bool inside = x >= G.X(i) && x <= G.X(i + 1) && y >= G.Y(j) && y <= G.Y(j + 1);
  return inside ? 0 : 2;
}

extern "C" {
// Singularity map of one single-plane lens on an nx x ny vertex grid.
// Crossings (ordered by row j; in a row the horizontal edges (i,j)-(i+1,j) by i, then the
// vertical edges (i,j)-(i,j+1) by i; per edge k = 1 then 2): cx [2n], ck, ce (e_k), cg (g_k),
// cfl.  Segments (cells in row-major order, k = 1 then 2): ends sa, sb (crossing index, or
// -(umbilic index) - 1), sk.  Umbilics (cells with orientation product -1, row-major): ux
// [2n], ukap, ustat (0 ok, 1 no convergence, 2 outside the cell; +4 a family's crossings
// could not be joined to it).  Swallowtails (segments in order): wx [2n], wk, we, wseg, wstat
// (refine: the interpolated point polished by Newton on (f_k, g_k); 0 ok, 1 no convergence,
// 2 moved > h (the interpolated point is kept), +8 an umbilic-flagged evaluation).
// counts[0..3] = crossings, segments, umbilics, swallowtails (true counts; arrays hold at most
// cap of each); counts[4] = cells skipped next to umbilic-flagged vertices; counts[5] = cells
// whose crossings could not be paired.
int orc_sing_map(const double* tab, int H, double x0, double y0, double h, int nx, int ny, int refine,
                 double tol, int cap, double* cx, int* ck, double* ce, double* cg, int* cfl, int* sa, int* sb,
                 int* sk, double* ux, double* ukap, int* ustat, double* wx, int* wk, double* we, int* wseg,
                 int* wstat, int* counts, int nthreads) {
  SingGrid G;
  G.tab = tab; G.H = H; G.x0 = x0; G.y0 = y0; G.h = h; G.nx = nx; G.ny = ny;
  G.V.resize((size_t)nx * ny);
  parallel_for(ny, nthreads, [&](int lo, int hi) {
    for (int j = lo; j < hi; ++j)
      for (int i = 0; i < nx; ++i) G.V[(size_t)j * nx + i] = sing_at(tab, H, G.X(i), G.Y(j));
  });
  // 1. crossings in canonical order, then their refinement
  struct Raw { int i, j, dir, k; };
  std::vector<Raw> raw;
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i + 1 < nx; ++i)
      for (int k = 0; k < 2; ++k)
        if (edge_cross(G.at(i, j), G.at(i + 1, j), k)) raw.push_back({i, j, 0, k});
    if (j + 1 < ny)
      for (int i = 0; i < nx; ++i)
        for (int k = 0; k < 2; ++k)
          if (edge_cross(G.at(i, j), G.at(i, j + 1), k)) raw.push_back({i, j, 1, k});
  }
  std::vector<Crossing> X(raw.size());
  parallel_for((int)raw.size(), nthreads, [&](int lo, int hi) {
    for (int n = lo; n < hi; ++n) {
      const Raw& r = raw[n];
      const SingVal& A = G.at(r.i, r.j);
      const SingVal& B = r.dir == 0 ? G.at(r.i + 1, r.j) : G.at(r.i, r.j + 1);
      X[n] = refine_crossing(G, G.X(r.i), G.Y(r.j), r.dir == 0 ? h : 0.0, r.dir == 0 ? 0.0 : h, A, B, r.k,
                             refine != 0, tol);
      X[n].key = ((((int64_t)r.j * 2 + r.dir) * nx + r.i) * 2 + r.k);
    }
  });
  auto find_x = [&](int i, int j, int dir, int k) -> int {
    int64_t key = ((((int64_t)j * 2 + dir) * nx + i) * 2 + k);
    int lo = 0, hi = (int)X.size();
    while (lo < hi) { int m = (lo + hi) / 2; if (X[m].key < key) lo = m + 1; else hi = m; }
    return (lo < (int)X.size() && X[lo].key == key) ? lo : -1;
  };
  // 2. cells: segments and umbilic cells
  struct Seg { int a, b, k; };
  std::vector<Seg> S;
  struct Umb { int i, j, stat; double x, y, kap; };
  std::vector<Umb> U;
  int skipped = 0, unpaired = 0;
  for (int j = 0; j + 1 < ny; ++j)
    for (int i = 0; i + 1 < nx; ++i) {
      const SingVal* c[4] = {&G.at(i, j), &G.at(i + 1, j), &G.at(i + 1, j + 1), &G.at(i, j + 1)};
      if (c[0]->umb || c[1]->umb || c[2]->umb || c[3]->umb) { ++skipped; continue; }
      // loop edges: bottom, right, top, left (crossing lookups by their stored edge)
      const int ei[4] = {i, i + 1, i, i}, ej[4] = {j, j, j + 1, j}, ed[4] = {0, 1, 0, 1};
      double P = align(*c[0], *c[1], 0) * align(*c[1], *c[2], 0) * align(*c[2], *c[3], 0) * align(*c[3], *c[0], 0);
      int uidx = -1;
      if (P < 0) { uidx = (int)U.size(); U.push_back({i, j, 0, 0, 0, 0}); }
      for (int k = 0; k < 2; ++k) {
        int xs[4], n = 0;
        for (int m = 0; m < 4; ++m) {
          xs[m] = find_x(ei[m], ej[m], ed[m], k);
          if (xs[m] >= 0) ++n;
        }
        if (P > 0) {
          if (n == 2) {
            int a = -1, b = -1;
            for (int m = 0; m < 4; ++m) if (xs[m] >= 0) { if (a < 0) a = xs[m]; else b = xs[m]; }
            S.push_back({a, b, k});
          } else if (n == 4) {
            double F0 = c[0]->f[k];
            double F1 = align(*c[0], *c[1], k) * c[1]->f[k];
            double F2 = align(*c[0], *c[1], k) * align(*c[1], *c[2], k) * c[2]->f[k];
            double F3 = align(*c[0], *c[3], k) * c[3]->f[k];
            double D = F0 + F2 - F1 - F3;
            bool cpos = D == 0.0 ? true : !neg((F0 * F2 - F1 * F3) / D);
            if (cpos == !neg(F0)) { S.push_back({xs[0], xs[1], k}); S.push_back({xs[2], xs[3], k}); }
            else { S.push_back({xs[0], xs[3], k}); S.push_back({xs[1], xs[2], k}); }
          } else if (n != 0) {
            ++unpaired;
          }
        } else {
          // an odd number of lines of the family ends at the umbilic (one at a hyperbolic,
          // one or three at an elliptic umbilic)
          if (n == 1 || n == 3) {
            for (int m = 0; m < 4; ++m)
              if (xs[m] >= 0) S.push_back({xs[m], -uidx - 1, k});
          } else {
            U[uidx].stat |= 4;
            if (n != 0) ++unpaired;
          }
        }
      }
    }
  parallel_for((int)U.size(), nthreads, [&](int lo, int hi) {
    for (int n = lo; n < hi; ++n) {
      double x, y, kap;
      int st = umbilic_newton(G, U[n].i, U[n].j, &x, &y, &kap);
      U[n].stat |= st; U[n].x = x; U[n].y = y; U[n].kap = kap;
    }
  });
  // 3. swallowtails: g_k changes sign between the two crossings of a segment
  struct Sw { double x, y, e; int k, seg, stat; };
  std::vector<Sw> W;
  for (int n = 0; n < (int)S.size(); ++n) {
    const Seg& s = S[n];
    if (s.a < 0 || s.b < 0) continue;
    const Crossing &A = X[s.a], &B = X[s.b];
    if ((A.flags | B.flags) & 5) continue;        // umbilic-flagged evaluation or a jump
    if (neg(A.g) == neg(B.g)) continue;
    double u = A.g / (A.g - B.g);
    W.push_back({A.x + u * (B.x - A.x), A.y + u * (B.y - A.y), 0.0, s.k, n, 0});
  }
  parallel_for((int)W.size(), nthreads, [&](int lo, int hi) {
    for (int n = lo; n < hi; ++n) {
      if (refine) W[n].stat = swallowtail_newton(G, W[n].k, &W[n].x, &W[n].y);
      W[n].e = sing_at(tab, H, W[n].x, W[n].y).e[W[n].k];
    }
  });
  counts[0] = (int)X.size(); counts[1] = (int)S.size(); counts[2] = (int)U.size(); counts[3] = (int)W.size();
  counts[4] = skipped; counts[5] = unpaired;
  for (int n = 0; n < (int)X.size() && n < cap; ++n) {
    cx[2 * n] = X[n].x; cx[2 * n + 1] = X[n].y; ck[n] = X[n].k + 1; ce[n] = X[n].e; cg[n] = X[n].g; cfl[n] = X[n].flags;
  }
  for (int n = 0; n < (int)S.size() && n < cap; ++n) { sa[n] = S[n].a; sb[n] = S[n].b; sk[n] = S[n].k + 1; }
  for (int n = 0; n < (int)U.size() && n < cap; ++n) {
    ux[2 * n] = U[n].x; ux[2 * n + 1] = U[n].y; ukap[n] = U[n].kap; ustat[n] = U[n].stat;
  }
  for (int n = 0; n < (int)W.size() && n < cap; ++n) {
    wx[2 * n] = W[n].x; wx[2 * n + 1] = W[n].y; wk[n] = W[n].k + 1; we[n] = W[n].e; wseg[n] = W[n].seg;
    wstat[n] = W[n].stat;
  }
  return 0;
}
}  // extern "C"
