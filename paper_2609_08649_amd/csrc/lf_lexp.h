// Local expansion of the far members of a grid block (the lean maps passes on a grid).
//
// A circular dPIE member (Sec. 3.4) that lies far from a block (the far-field series of its
// closed form holds over the whole block, and the block is small next to its distance) is not
// summed point by point: every such member adds the Taylor coefficients of its potential about
// the block centre X to the lane that holds it, the wave sums the coefficients once, and every
// lane evaluates the summed polynomial (and its derivatives) at its points.  The deflection is
// still the sum over all halos of Sec. 2.1; the truncation of the expansion lies far below the
// FP32 rounding of the point-by-point form.
//
// Potential of the far-field series (m = alpha_r / r = fm0 t^2 + sum_{k>=1} fm_k t^(2k+1),
// t = 1/r): psi(r) = fm0 ln r - sum_{k=1..5} fm_k r^-(2k-1) / (2k-1).  In complex form, with
// zeta0 = X - c (block centre minus member centre), delta = point - X and q = 1 / zeta0:
//   ln r  = Re ln(zeta0 + delta) = const + Re sum_{i>=1} (-1)^(i+1) / i (q delta)^i,
//   r^-n  = |zeta0|^-n sum_{i,j} C(-n/2, i) C(-n/2, j) (q delta)^i conj(q delta)^j,
// so psi = sum_{i,j} G_ij delta^i conj(delta)^j with G_ji = conj(G_ij); the coefficients of a
// member are q^(i-j) |q|^(2j) times real sums of its fm.  Derivatives by the Wirtinger rules
// (d/d conj(delta) = (d/dx + i d/dy) / 2):
//   alpha_x + i alpha_y        = 2 d psi / d conj(delta),
//   psi_xx + psi_yy            = 4 d^2 psi / d delta d conj(delta),
//   psi_xx - psi_yy + 2i psi_xy = 4 d^2 psi / d conj(delta)^2.
// Terms up to total degree LX_K = 7 are kept.  Members are taken at distances of at least
// LX_DIST block radii (|delta| / |zeta0| <= 1/8): the truncation is then below 1e-9 arcsec in
// alpha and 1e-9 in the Hessian on cluster members, against 1e-7 for the FP32 rounding of one
// member term; the third derivatives (of the same polynomial, to degree 4) stay within 3e-8 of
// the exact member sums.  Coefficients are formed and summed in FP32 except G_10 (the block centre's
// deflection, the one term of the size of the total), which the lanes keep in FP64.
#pragma once
#include <hip/hip_runtime.h>

#include "lf_device.h"

namespace lf {

static constexpr int LX_K = 7;
static constexpr double LX_DIST = 8.0;

// pairs (i, j), i >= j, i + j <= LX_K, without (0, 0): column j starts at i = max(j, 1)
constexpr int lx_count(int j) { return j == 0 ? LX_K : LX_K - 2 * j + 1; }
constexpr int lx_base(int j) { return j == 0 ? 0 : lx_base(j - 1) + lx_count(j - 1); }
constexpr int lx_idx(int i, int j) { return lx_base(j) + i - (j == 0 ? 1 : j); }
static constexpr int LX_J = LX_K / 2;                 // largest j of a pair
static constexpr int LX_NP = lx_base(LX_J + 1);       // 19 pairs

// C(-n/2, i): binomial coefficient of a negative half-integer power
constexpr double lx_bin(int n, int i) {
  double r = 1.0;
  for (int k = 0; k < i; ++k) r *= (-0.5 * n - k) / (k + 1);
  return r;
}
struct LxTab {
  float t[6][LX_NP];   // t[k][pair] = -C(-n/2, i) C(-n/2, j) / n for the fm_k term, n = 2k - 1
  float lam[LX_K + 1]; // (-1)^(i+1) / (2 i): the logarithm's coefficients (j = 0)
};
constexpr LxTab lx_make() {
  LxTab T{};
  for (int k = 1; k <= 5; ++k) {
    const int n = 2 * k - 1;
    for (int j = 0; j <= LX_J; ++j)
      for (int i = (j == 0 ? 1 : j); i <= LX_K - j; ++i)
        T.t[k][lx_idx(i, j)] = (float)(-lx_bin(n, i) * lx_bin(n, j) / n);
  }
  for (int i = 1; i <= LX_K; ++i) T.lam[i] = (float)((i % 2 ? 0.5 : -0.5) / i);
  return T;
}
static constexpr LxTab LX_TAB = lx_make();

// Summed coefficients: re/im of every pair but (1, 0) (im of the diagonal pairs is zero), and
// G_10 in FP64.
struct LxAcc {
  float re[LX_NP], im[LX_NP];
  double c10r, c10i;
};
__device__ __forceinline__ void lx_zero(LxAcc& g) {
#pragma unroll
  for (int p = 0; p < LX_NP; ++p) g.re[p] = g.im[p] = 0.f;
  g.c10r = g.c10i = 0.0;
}

// Adds the coefficients of one member at offset (dx, dy) = c - X (FP32) with far-field
// coefficients fm[0..5].
__device__ __forceinline__ void lx_member(float dx, float dy, const float (&fm)[6], LxAcc& g) {
  const float r2 = fmaf(dx, dx, dy * dy);
  const float t0 = frsq(r2), inv = t0 * t0;
  float pr[LX_K + 1], pi[LX_K + 1];           // q^p, q = 1 / zeta0 = -(dx - i dy) / r^2
  pr[0] = 1.f; pi[0] = 0.f;
  pr[1] = -dx * inv; pi[1] = dy * inv;
#pragma unroll
  for (int p = 2; p <= LX_K; ++p) {
    pr[p] = fmaf(pr[p - 1], pr[1], -pi[p - 1] * pi[1]);
    pi[p] = fmaf(pr[p - 1], pi[1], pi[p - 1] * pr[1]);
  }
  float b[6];                                  // fm_k t0^(2k-1) |q|^(2j)
  b[0] = 0.f;
  b[1] = fm[1] * t0;
  float tp = t0;
#pragma unroll
  for (int k = 2; k <= 5; ++k) { tp *= inv; b[k] = fm[k] * tp; }
#pragma unroll
  for (int j = 0; j <= LX_J; ++j) {
    if (j > 0) {
#pragma unroll
      for (int k = 1; k <= 5; ++k) b[k] *= inv;
    }
#pragma unroll
    for (int i = 1; i <= LX_K; ++i) {
      if (i < j || i > LX_K - j) continue;     // constant trip counts: the loops unroll fully
      const int p = lx_idx(i, j);
      float S = j == 0 ? fm[0] * LX_TAB.lam[i] : b[1] * LX_TAB.t[1][p];
#pragma unroll
      for (int k = (j == 0 ? 1 : 2); k <= 5; ++k) S = fmaf(b[k], LX_TAB.t[k][p], S);
      if (i == j) {
        g.re[p] += S;
      } else if (p == 0) {
        g.c10r += (double)(S * pr[1]);
        g.c10i += (double)(S * pi[1]);
      } else {
        g.re[p] = fmaf(S, pr[i - j], g.re[p]);
        g.im[p] = fmaf(S, pi[i - j], g.im[p]);
      }
    }
  }
}

// Wave sums by DPP lane moves: quad permutations and row rotations give every lane its row's
// total, and row broadcasts carry the row totals into the last row, so lane 63 ends with the
// wave's sum.  Lanes that a move leaves out add zero.
template <int CTRL, int ROWS>
__device__ __forceinline__ int lx_dpp(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xf, true);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float lx_dpp_f32(float v) {
  return __int_as_float(lx_dpp<CTRL, ROWS>(__float_as_int(v)));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double lx_dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lx_dpp<CTRL, ROWS>((int)b), hi = lx_dpp<CTRL, ROWS>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <class T>
__device__ __forceinline__ T lx_wsum63(T v) {
  if constexpr (sizeof(T) == 4) {
    v += lx_dpp_f32<0xb1, 0xf>(v);     // quad_perm [1, 0, 3, 2]
    v += lx_dpp_f32<0x4e, 0xf>(v);     // quad_perm [2, 3, 0, 1]
    v += lx_dpp_f32<0x124, 0xf>(v);    // row_ror 4
    v += lx_dpp_f32<0x128, 0xf>(v);    // row_ror 8
    v += lx_dpp_f32<0x142, 0xa>(v);    // row_bcast 15 into rows 1 and 3
    v += lx_dpp_f32<0x143, 0xc>(v);    // row_bcast 31 into rows 2 and 3
  } else {
    v += lx_dpp_f64<0xb1, 0xf>(v);
    v += lx_dpp_f64<0x4e, 0xf>(v);
    v += lx_dpp_f64<0x124, 0xf>(v);
    v += lx_dpp_f64<0x128, 0xf>(v);
    v += lx_dpp_f64<0x142, 0xa>(v);
    v += lx_dpp_f64<0x143, 0xc>(v);
  }
  return v;
}

// LDS image of the summed coefficients (floats): G_10 as two doubles, then re and im of the
// pairs.  Every lane reads them back (broadcast reads), so that they do not occupy registers
// through the evaluation.
static constexpr int LX_RE = 4, LX_IM = LX_RE + LX_NP, LX_LDS = LX_IM + LX_NP;

// Sums the lanes' coefficients over the wave; lane 63 writes the sums to c[0, LX_LDS).  The
// caller orders the writes before the reads (wave_sync).
__device__ __forceinline__ void lx_reduce_store(const LxAcc& g, float* c) {
  const bool last = (threadIdx.x & 63) == 63;
#pragma unroll
  for (int j = 0; j <= LX_J; ++j) {
#pragma unroll
    for (int i = 1; i <= LX_K; ++i) {
      if (i < j || i > LX_K - j || (i == 1 && j == 0)) continue;
      const int p = lx_idx(i, j);
      const float re = lx_wsum63(g.re[p]);
      if (last) c[LX_RE + p] = re;
      if (i != j) {
        const float im = lx_wsum63(g.im[p]);
        if (last) c[LX_IM + p] = im;
      }
    }
  }
  const double r = lx_wsum63(g.c10r), i = lx_wsum63(g.c10i);
  if (last) { ((double*)c)[0] = r; ((double*)c)[1] = i; }
}

// G_ij for i + j <= LX_K from the LDS image c, except G_10 and G_01 (held in FP64).
template <int I, int J>
__device__ __forceinline__ void lx_get(const float* c, float& re, float& im) {
  if constexpr (I + J > LX_K) {
    re = im = 0.f;
  } else if constexpr (I >= J) {
    re = c[LX_RE + lx_idx(I, J)];
    im = I == J ? 0.f : c[LX_IM + lx_idx(I, J)];
  } else {
    re = c[LX_RE + lx_idx(J, I)];
    im = -c[LX_IM + lx_idx(J, I)];
  }
}

// Horner step z = z w + c in complex arithmetic, w = u + i v (CONJ: w = u - i v).
template <bool CONJ>
__device__ __forceinline__ void lx_horner(float& zr, float& zi, float u, float v, float cr, float ci) {
  const float vv = CONJ ? -v : v;
  const float t = fmaf(zr, u, fmaf(-zi, vv, cr));
  zi = fmaf(zr, vv, fmaf(zi, u, ci));
  zr = t;
}

// Inner polynomials in delta for the power B of conj(delta), from the power A of delta down:
// alpha: 2 (B+1) G(A, B+1) (the constant G_01 is added in FP64 by lx_eval), Laplacian:
// 4 (A+1)(B+1) G(A+1, B+1), Gamma: 4 (B+2)(B+1) G(A, B+2) and, with third derivatives (D3),
// T = 8 d^3 psi / d conj(delta)^3: 8 (B+3)(B+2)(B+1) G(A, B+3) and
// U = 8 d^3 psi / d delta d conj(delta)^2: 8 (A+1)(B+2)(B+1) G(A+1, B+2).  All NP points of the
// lane at once, so that each coefficient is read and scaled once.
template <int NQ>
__device__ __forceinline__ void lx_step(float (&q)[NQ], int o, bool first, float u, float v, float cr, float ci) {
  if (first) { q[o] = cr; q[o + 1] = ci; }
  else lx_horner<false>(q[o], q[o + 1], u, v, cr, ci);
}
template <int A, int B, int NP, bool D3, int NQ>
__device__ __forceinline__ void lx_inner(const float* g, float u, const float (&v)[NP], float (&q)[NP][NQ]) {
  constexpr int K = LX_K;
  float cr = 0.f, ci = 0.f;
  if constexpr (A + B > 0) {
    lx_get<A, B + 1>(g, cr, ci);
    cr *= 2.f * (B + 1); ci *= 2.f * (B + 1);
  }
#pragma unroll
  for (int k = 0; k < NP; ++k) lx_step(q[k], 0, A == K - 1 - B, u, v[k], cr, ci);
  if constexpr (A + B <= K - 2) {
    float c2r, c2i, c3r, c3i;
    lx_get<A + 1, B + 1>(g, c2r, c2i);
    lx_get<A, B + 2>(g, c3r, c3i);
    constexpr float f2 = 4.f * (A + 1) * (B + 1), f3 = 4.f * (B + 2) * (B + 1);
    c2r *= f2; c2i *= f2; c3r *= f3; c3i *= f3;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      lx_step(q[k], 2, A == K - 2 - B, u, v[k], c2r, c2i);
      lx_step(q[k], 4, A == K - 2 - B, u, v[k], c3r, c3i);
    }
  }
  if constexpr (D3 && A + B <= K - 3) {
    float c4r, c4i, c5r, c5i;
    lx_get<A, B + 3>(g, c4r, c4i);
    lx_get<A + 1, B + 2>(g, c5r, c5i);
    constexpr float f4 = 8.f * (B + 3) * (B + 2) * (B + 1), f5 = 8.f * (A + 1) * (B + 2) * (B + 1);
    c4r *= f4; c4i *= f4; c5r *= f5; c5i *= f5;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      lx_step(q[k], 6, A == K - 3 - B, u, v[k], c4r, c4i);
      lx_step(q[k], 8, A == K - 3 - B, u, v[k], c5r, c5i);
    }
  }
  if constexpr (A > 0) lx_inner<A - 1, B, NP, D3, NQ>(g, u, v, q);
}

// Outer Horner steps in conj(delta), from the power B down; P = {alpha, Laplacian, Gamma, T, U}.
template <int NQ>
__device__ __forceinline__ void lx_ostep(float (&P)[NQ], const float (&q)[NQ], int o, bool first, float u, float v) {
  if (first) { P[o] = q[o]; P[o + 1] = q[o + 1]; }
  else lx_horner<true>(P[o], P[o + 1], u, v, q[o], q[o + 1]);
}
template <int B, int NP, bool D3, int NQ>
__device__ __forceinline__ void lx_outer(const float* g, float u, const float (&v)[NP], float (&P)[NP][NQ]) {
  constexpr int K = LX_K;
  float q[NP][NQ];
  lx_inner<K - 1 - B, B, NP, D3, NQ>(g, u, v, q);
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    lx_ostep(P[k], q[k], 0, B == K - 1, u, v[k]);
    if constexpr (B <= K - 2) {
      lx_ostep(P[k], q[k], 2, B == K - 2, u, v[k]);
      lx_ostep(P[k], q[k], 4, B == K - 2, u, v[k]);
    }
    if constexpr (D3 && B <= K - 3) {
      lx_ostep(P[k], q[k], 6, B == K - 3, u, v[k]);
      lx_ostep(P[k], q[k], 8, B == K - 3, u, v[k]);
    }
  }
  if constexpr (B > 0) lx_outer<B - 1, NP, D3, NQ>(g, u, v, P);
}

// Adds the summed expansion's (LDS image c) deflection and Hessian (D3: and third derivatives)
// at the offsets (u, v[k]) from the block centre.  Each of alpha_x + i alpha_y, the Laplacian,
// Gamma = psi_xx - psi_yy + 2i psi_xy, T = psi_xxx - 3 psi_xyy + i (3 psi_xxy - psi_yyy) and
// U = psi_xxx + psi_xyy + i (psi_xxy + psi_yyy) is a polynomial sum_{a,b} c_ab delta^a
// conj(delta)^b, evaluated by Horner's rule in delta (inner) and conj(delta) (outer).  The
// Laplacian is real (its imaginary part cancels).
template <bool D3, int NP>
__device__ __forceinline__ void lx_eval(const float* c, float u, const float (&v)[NP], Acc (&acc)[NP]) {
  constexpr int NQ = D3 ? 10 : 6;
  float P[NP][NQ];
  lx_outer<LX_K - 1, NP, D3, NQ>(c, u, v, P);
  // constant term of alpha: 2 G_01 = 2 conj(G_10)
  const double c10r = ((const double*)c)[0], c10i = ((const double*)c)[1];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    acc[k].ax += 2.0 * c10r + (double)P[k][0];
    acc[k].ay += (double)P[k][1] - 2.0 * c10i;
    acc[k].h11 += 0.5 * ((double)P[k][2] + (double)P[k][4]);
    acc[k].h22 += 0.5 * ((double)P[k][2] - (double)P[k][4]);
    acc[k].h12 += 0.5 * (double)P[k][5];
    if constexpr (D3) {
      const double Tr = P[k][6], Ti = P[k][7], Ur = P[k][8], Ui = P[k][9];
      acc[k].t111 += 0.25 * (3.0 * Ur + Tr);
      acc[k].t122 += 0.25 * (Ur - Tr);
      acc[k].t112 += 0.25 * (Ui + Ti);
      acc[k].t222 += 0.25 * (3.0 * Ui - Ti);
    }
  }
}

}  // namespace lf
