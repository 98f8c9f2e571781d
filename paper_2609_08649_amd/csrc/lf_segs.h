// Member-galaxy segment loops shared by the maps, finder and multi-plane kernels.
#pragma once
#include "lf_device.h"
#include "lf_lexp.h"

namespace lf {

// ---------------------------------------------------------------------------------------
// Member segment loops over pre-scaled records (MemRec32: FP32 maths; MemRec64: FP64
// throughout).  One loop per profile segment.
//
// FP32 offsets: the lane point and the member centre are both FP32 pairs (hi + lo), and
// dx = (px_hi - cx_hi) + (px_lo - cx_lo) carries a relative error of a few FP32 ulp of dx
// itself, whatever the absolute coordinates (the FP32 maths starts from an accurate offset).
//
// FP32 accumulation of the bulk segments (circular dPIE / cored SIE): the terms of LF_CHUNK
// consecutive members are summed in FP32 and each chunk sum is added to the FP64
// accumulators, so rounding in FP32 sums is confined to short runs while most of the FP64
// conversion and addition work disappears.  The chunk boundaries depend only on the segment
// range, never on the launch shape, so results do not depend on batching.
// ---------------------------------------------------------------------------------------
static constexpr int LF_CHUNK = 16;

__device__ __forceinline__ void split32(double v, float& hi, float& lo) {
  hi = (float)v;
  lo = (float)(v - (double)hi);
}
__device__ __forceinline__ float off32(float ph, float pl, float ch, float cl) { return (ph - ch) + (pl - cl); }

// One member of segment SEG at offset (dx, dy); false if the point sits on a singular centre.
template <int SEG, bool D3, class T, class R>
__device__ __forceinline__ bool seg_term(const R& r, T dx, T dy, const Quad& qd, Term<T>& t) {
  constexpr bool F32 = sizeof(T) == 4;
  t.t111 = t.t112 = t.t122 = t.t222 = (T)0;
  if constexpr (SEG == SEG_CPJE || SEG == SEG_CSIE) {
    T r2 = fma(dx, dx, dy * dy);
    if constexpr (F32) {
      // FP32: a point within 1e-6" of a member centre is evaluated at r = 1e-6"
      r2 = fmaxf(r2, 1e-12f);
    } else {
      if (r.s == 0.0 && r2 < 1e-24) return false;
    }
    T m, w, p = 0;
    if constexpr (SEG == SEG_CPJE) pje_mw<D3>(r.b, r.s, r.a, r.s2, r.a2, r.bd, r.apls, r2, m, w, p);
    else cored_mw<D3>(r.b, r.s, r.s2, r2, m, w, p);
    radial<D3>(dx, dy, m, w, p, t);
  } else if constexpr (SEG == SEG_EPJE || SEG == SEG_ESIE) {
    if (r.s == (T)0 && dx == (T)0 && dy == (T)0) return false;
    epje<D3>(dx, dy, r.c, r.sn, r.bqe, r.e, r.q2, r.s, r.a, SEG == SEG_EPJE, t);
  } else if constexpr (SEG == SEG_POINT) {
    if (dx == (T)0 && dy == (T)0) return false;
    point_mass<D3>(dx, dy, r.b, t);
  } else if constexpr (SEG == SEG_NFW) {
    if (dx == (T)0 && dy == (T)0) return false;
    nfw_circ<D3>((double)dx, (double)dy, (double)r.b, (double)r.s, *(Term<double>*)&t);
  } else {
    if (dx == (T)0 && dy == (T)0) return false;
    double xp = r.c * dx + r.sn * dy, yp = r.c * dy - r.sn * dx;
    Term<double> pr;
    enfw_prime<D3>(xp, yp, r.b, r.s, sqrt((double)r.q2), qd, pr);
    rotate_back<D3>((double)r.c, (double)r.sn, pr, *(Term<double>*)&t);
  }
  return true;
}

// FP32 run sums of the circular segments.  The Hessian is kept as its isotropic part
// sum(m) and the anisotropic part sum(w x_i x_j), so every term enters through one FMA:
// psi_ij = sum(m) delta_ij + sum(w x_i x_j); alpha_i = sum(m x_i).  sum(w y^2) is taken as
// sum(w r^2) - sum(w x^2) when a run is flushed (in FP64).  m is the mean convergence inside r
// and w r^2 = 2 (kappa - m), so 0 <= kappa <= m (decreasing profiles) gives |w| r^2 <= 2 m: the
// rounding of sum(w r^2) stays of the order of that of sum(m).  The third derivatives of a
// circular term are psi_ijk = w (delta_ij x_k + delta_ik x_j + delta_jk x_i) + 2 w' x_i x_j x_k:
// kept as sum(w x_i) (w x reuses the Hessian's product) and sum(w' x_i x_j x_k), combined at the
// flush.
struct Run32 {
  float ax, ay, m, h11, h12, wr2, wx, wy, qxxx, qxxy, qxyy, qyyy;
};
template <bool D3>
__device__ __forceinline__ void run_zero(Run32& s) {
  s.ax = s.ay = s.m = s.h11 = s.h12 = s.wr2 = 0.f;
  if (D3) s.wx = s.wy = s.qxxx = s.qxxy = s.qxyy = s.qyyy = 0.f;
}
template <bool D3>
__device__ __forceinline__ void run_add(float dx, float dy, float r2, float m, float w, float wp, Run32& s) {
  s.ax = fmaf(m, dx, s.ax);
  s.ay = fmaf(m, dy, s.ay);
  s.m += m;
  float wx = w * dx;
  s.h11 = fmaf(wx, dx, s.h11);
  s.h12 = fmaf(wx, dy, s.h12);
  s.wr2 = fmaf(w, r2, s.wr2);
  if (D3) {
    s.wx += wx;
    s.wy = fmaf(w, dy, s.wy);
    float pxx = wp * dx * dx, pyy = wp * dy * dy;
    s.qxxx = fmaf(pxx, dx, s.qxxx);
    s.qxxy = fmaf(pxx, dy, s.qxxy);
    s.qxyy = fmaf(pyy, dx, s.qxyy);
    s.qyyy = fmaf(pyy, dy, s.qyyy);
  }
}
template <bool D3>
__device__ __forceinline__ void run_flush(const Run32& s, Acc& a) {
  const double m = (double)s.m;
  a.ax += (double)s.ax; a.ay += (double)s.ay;
  const double h11 = (double)s.h11;
  a.h11 += m + h11; a.h12 += (double)s.h12; a.h22 += m + ((double)s.wr2 - h11);
  if (D3) {
    const double wx = (double)s.wx, wy = (double)s.wy;
    a.t111 += 3.0 * wx + 2.0 * (double)s.qxxx;
    a.t112 += wy + 2.0 * (double)s.qxxy;
    a.t122 += wx + 2.0 * (double)s.qxyy;
    a.t222 += 3.0 * wy + 2.0 * (double)s.qyyy;
  }
}

// m, w (and w') of a circular member at squared radius r2 > 0 (FP32 records).
template <int SEG, bool D3, class R>
__device__ __forceinline__ void circ_mw(const R& r, float r2, float& m, float& w, float& wp) {
  wp = 0.f;
  if constexpr (SEG == SEG_CPJE) pje_mw<D3>(r.b, r.s, r.a, r.s2, r.a2, r.bd, r.apls, r2, m, w, wp);
  else cored_mw<D3>(r.b, r.s, r.s2, r2, m, w, wp);
}

// Squared radius at which the FP32 term of a near-field lane is evaluated instead of its own:
// every circular term there is below 1e-14 (and finite), so the lane's FP32 run sum is
// unaffected while its exact term is added from the FP64 record.  A dPIE term falls off as
// 1/r^2 and its closed form needs r^2 < 1e25; a cored isothermal term falls off as 1/r.
template <int SEG>
static constexpr float FAR_R2 = SEG == SEG_CPJE ? 1e24f : 1e30f;

// near64: the FP64 records of the same members (FP32 path: near-field terms); unused for
// FP64 records.
template <int SEG, bool D3, int PPL, class R>
__device__ __forceinline__ void seg_loop(const R* __restrict__ rec, const MemRec64* __restrict__ near64, int lo,
                                         int hi, const double (&px)[PPL], const double (&py)[PPL],
                                         Acc (&acc)[PPL], const Quad& qd) {
  using T = decltype(R::b);
  constexpr bool F32 = sizeof(T) == 4;
  if constexpr (F32) {
    static_assert(SEG != SEG_NFW && SEG != SEG_ENFW, "NFW members are evaluated from FP64 records");
    float xh[PPL], xl[PPL], yh[PPL], yl[PPL];
#pragma unroll
    for (int k = 0; k < PPL; ++k) { split32(px[k], xh[k], xl[k]); split32(py[k], yh[k], yl[k]); }
    if constexpr (SEG == SEG_CPJE || SEG == SEG_CSIE) {
      // Members are taken two at a time: both FP32 terms are straight-line code the compiler
      // can interleave, and the rare near-field branches come after them.
      auto near_term = [&](int h, int k) {
        const MemRec64 q = near64[h];
        Term<double> t;
        if (seg_term<SEG, D3>(q, px[k] - q.x, py[k] - q.y, qd, t)) add<D3>(acc[k], t);
        else acc[k].flags |= FL_SINGULAR;
      };
      auto far_term = [&](const R& r, int k, Run32& ps) -> bool {
        float dx = off32(xh[k], xl[k], r.xh, r.xl), dy = off32(yh[k], yl[k], r.yh, r.yl);
        float r2 = fmaf(dx, dx, dy * dy);
        const bool nr = r2 < r.rn2;
        float m, w, wp;
        circ_mw<SEG, D3>(r, nr ? FAR_R2<SEG> : r2, m, w, wp);
        run_add<D3>(dx, dy, r2, m, w, wp, ps);
        return nr;
      };
      for (int h0 = lo; h0 < hi; h0 += LF_CHUNK) {
        const int h1 = min(h0 + LF_CHUNK, hi);
        Run32 ps[PPL];
#pragma unroll
        for (int k = 0; k < PPL; ++k) run_zero<D3>(ps[k]);
        int h = h0;
        for (; h + 1 < h1; h += 2) {
          const R r0 = rec[h], r1 = rec[h + 1];
          bool n0[PPL], n1[PPL];
#pragma unroll
          for (int k = 0; k < PPL; ++k) {
            n0[k] = far_term(r0, k, ps[k]);
            n1[k] = far_term(r1, k, ps[k]);
          }
#pragma unroll
          for (int k = 0; k < PPL; ++k) {
            if (n0[k]) near_term(h, k);
            if (n1[k]) near_term(h + 1, k);
          }
        }
        if (h < h1) {
          const R r0 = rec[h];
#pragma unroll
          for (int k = 0; k < PPL; ++k)
            if (far_term(r0, k, ps[k])) near_term(h, k);
        }
#pragma unroll
        for (int k = 0; k < PPL; ++k) run_flush<D3>(ps[k], acc[k]);
      }
    } else {
      for (int h = lo; h < hi; ++h) {
        const R r = rec[h];
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
          float dx = off32(xh[k], xl[k], r.xh, r.xl), dy = off32(yh[k], yl[k], r.yh, r.yl);
          bool ok;
          if (fmaf(dx, dx, dy * dy) < r.rn2) {
            const MemRec64 q = near64[h];
            Term<double> t;
            ok = seg_term<SEG, D3>(q, px[k] - q.x, py[k] - q.y, qd, t);
            if (ok) add<D3>(acc[k], t);
          } else {
            Term<float> t;
            ok = seg_term<SEG, D3>(r, dx, dy, qd, t);
            if (ok) add<D3>(acc[k], t);
          }
          if (!ok) acc[k].flags |= FL_SINGULAR;
        }
      }
    }
  } else {
    for (int h = lo; h < hi; ++h) {
      const R r = rec[h];
#pragma unroll
      for (int k = 0; k < PPL; ++k) {
        Term<double> t;
        if (seg_term<SEG, D3>(r, px[k] - r.x, py[k] - r.y, qd, t))
          add<D3>(acc[k], t);
        else
          acc[k].flags |= FL_SINGULAR;
      }
    }
  }
}


// ---------------------------------------------------------------------------------------
// Grid tiles of the FP32 member path.  A wave owns a TILE_W x TILE_H block of grid points
// aligned to the global grid; its lanes evaluate the member terms at X + (u, v), X the block
// centre (FP64) and (u, v) the lane's offset from it rounded to FP32 (|u|, |v| <= 7.5 h, so
// the rounding moves a lane by at most 2^-24 7.5 h, the same for every member).  The offset of
// a member from X, D = c - X, is formed once per wave in FP64 and rounded to FP32, so a lane's
// offset is dx = u - D_x: one FP32 subtraction per coordinate, with an error of a few ulp of
// |dx| + |u| (the block is small next to the near-field radius of the members it holds).
// ---------------------------------------------------------------------------------------
static constexpr int TILE_W = 16, TILE_H = 4;

// A lane of a tile: TP points of one column, TILE_H rows apart.
template <int TP>
struct TileLane {
  float u, v[TP];      // offsets from the block centre (FP32)
  double X, Y;         // block centre (FP64)
  double hwx, hwy;     // half extent of the block's lane points about the centre
  double px, py[TP];   // the lane's grid points (FP64)
  float* dsh;          // this wave's 64 member records in LDS
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS record of one member for one wave: its offset from the block centre and the constants of
// the evaluation the wave uses for it.  The member loop reads them into VGPRs: on gfx950 a VALU
// instruction with an SGPR operand issues at about half the rate of one whose operands are all
// VGPRs, so constants held in SGPRs (scalar loads) would halve the rate of every instruction
// that reads one.  Floats: Dx, Dy, then either the closed form's s^2, a^2, s, a, b (a - s),
// a + s, b, or (circular dPIE members at least FAR_K cut radii from the whole block, without
// third derivatives) the twelve far-field coefficients fm, fw.
struct MemL {
  float b, s, a, s2, a2, bd, apls;
};
template <int SEG, bool D3>
static constexpr bool TILE_FAR = SEG == SEG_CPJE;
template <int SEG, bool D3>
static constexpr int TILE_LSTRIDE = TILE_FAR<SEG, D3> ? (D3 ? 20 : 16) : 12;

// closed form (three transcendentals per point)
template <int SEG, bool D3, int TP>
__device__ __forceinline__ void tile_term_l(const float* l, const TileLane<TP>& L, Run32 (&ps)[TP]) {
  const float4 q0 = *(const float4*)l, q1 = *(const float4*)(l + 4);
  MemL r;
  r.s2 = q0.z; r.a2 = q0.w; r.s = q1.x; r.a = q1.y; r.bd = q1.z; r.apls = q1.w;
  r.b = (SEG == SEG_CPJE && !D3) ? 0.f : l[8];
  const float dx = L.u - q0.x;
  const float dx2 = dx * dx;
#pragma unroll
  for (int k = 0; k < TP; ++k) {
    const float dy = L.v[k] - q0.y;
    const float r2 = fmaf(dy, dy, dx2);
    float m, w, wp;
    circ_mw<SEG, D3>(r, r2, m, w, wp);
    run_add<D3>(dx, dy, r2, m, w, wp, ps[k]);
  }
}

// far-field expansion of a circular dPIE (one transcendental per point), NT = 4, 5 or 6 terms:
// with t = 1/r and u = t^2, m = u (fm0 + t (fm1 + u (fm2 + ...))), w = u^2 (fw0 + t (fw1 + ...))
// and, with third derivatives, w' = u^3 (fwp0 + t (fwp1 + ...)).  The record holds Dx, Dy,
// fm0..fm(NT-1), fw0..fw(NT-1) (and fwp0..fwp(NT-1)) contiguously.
template <int NT>
__device__ __forceinline__ float far_poly(const float* c, float t, float uu) {
  float p = fmaf(uu, c[NT - 1], c[NT - 2]);
#pragma unroll
  for (int j = NT - 3; j >= 1; --j) p = fmaf(uu, p, c[j]);
  return fmaf(t, p, c[0]);
}
template <int TP, int NT, bool D3>
__device__ __forceinline__ void tile_term_far(const float* l, const TileLane<TP>& L, Run32 (&ps)[TP]) {
  static_assert(NT >= 4 && NT <= 6, "four to six terms");
  // 16-byte reads, and an 8- or 4-byte one for a short tail (a broadcast read moves its size
  // times 64 lanes through the LDS return path)
  constexpr int NF = 2 + (D3 ? 3 : 2) * NT;
  float f[20];
#pragma unroll
  for (int q = 0; q < NF / 4; ++q) {
    const float4 v = *(const float4*)(l + 4 * q);
    f[4 * q] = v.x; f[4 * q + 1] = v.y; f[4 * q + 2] = v.z; f[4 * q + 3] = v.w;
  }
  if constexpr (NF % 4 == 2) {
    const float2 v = *(const float2*)(l + NF - 2);
    f[NF - 2] = v.x; f[NF - 1] = v.y;
  } else if constexpr (NF % 4 == 1) {
    f[NF - 1] = l[NF - 1];
  } else if constexpr (NF % 4 == 3) {
    const float2 v = *(const float2*)(l + NF - 3);
    f[NF - 3] = v.x; f[NF - 2] = v.y; f[NF - 1] = l[NF - 1];
  }
  const float dx = L.u - f[0];
  const float dx2 = dx * dx;
#pragma unroll
  for (int k = 0; k < TP; ++k) {
    const float dy = L.v[k] - f[1];
    const float r2 = fmaf(dy, dy, dx2);
    const float t = frsq(r2), uu = t * t, uu2 = uu * uu;
    const float pm = far_poly<NT>(f + 2, t, uu), pw = far_poly<NT>(f + 2 + NT, t, uu);
    const float wp = D3 ? (uu2 * uu) * far_poly<NT>(f + 2 + 2 * NT, t, uu) : 0.f;
    run_add<D3>(dx, dy, r2, uu * pm, uu2 * pw, wp, ps[k]);
  }
}

// The runs of one far-field tier: records [c_begin, c_end) of the wave's LDS list.
template <int TP, int NT, int LS, bool D3>
__device__ __forceinline__ void far_runs(int c_begin, int c_end, const TileLane<TP>& L, Acc (&acc)[TP]) {
  for (int c0 = c_begin; c0 < c_end; c0 += LF_CHUNK) {
    const int n = min(LF_CHUNK, c_end - c0);
    const float* lr = L.dsh + LS * c0;
    Run32 ps[TP];
#pragma unroll
    for (int k = 0; k < TP; ++k) run_zero<D3>(ps[k]);
    if (n == LF_CHUNK) {
#pragma unroll
      for (int k = 0; k < LF_CHUNK; ++k) tile_term_far<TP, NT, D3>(lr + LS * k, L, ps);
    } else {
      for (int k = 0; k < n; ++k) tile_term_far<TP, NT, D3>(lr + LS * k, L, ps);
    }
#pragma unroll
    for (int k = 0; k < TP; ++k) run_flush<D3>(ps[k], acc[k]);
  }
}

// One far record with third derivatives (Dx, Dy and the first NT coefficients of m, w and w')
// written to LDS at lw, in 16-byte stores.
template <int NT>
__device__ __forceinline__ void put_far_d3_n(float* lw, float dx, float dy, const MemRec32& r) {
  constexpr int NF = 2 + 3 * NT;
  float f[(NF + 3) / 4 * 4];
  f[0] = dx; f[1] = dy;
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    f[2 + k] = r.fm[k];
    f[2 + NT + k] = r.fw[k];
    f[2 + 2 * NT + k] = FAR_WP[k] * r.fm[k];
  }
#pragma unroll
  for (int k = NF; k < (NF + 3) / 4 * 4; ++k) f[k] = 0.f;
#pragma unroll
  for (int q = 0; q < (NF + 3) / 4; ++q) *(float4*)(lw + 4 * q) = make_float4(f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]);
}
__device__ __forceinline__ void put_far_d3(float* lw, int nt, float dx, float dy, const MemRec32& r) {
  if (nt == 4) put_far_d3_n<4>(lw, dx, dy, r);
  else if (nt == 5) put_far_d3_n<5>(lw, dx, dy, r);
  else put_far_d3_n<6>(lw, dx, dy, r);
}

// Classification of member h for the wave's block: whether its near-field disc (radius^2 rn2,
// with a relative margin of 1e-5 for the FP32 rounding of a lane's r^2) meets the block, how
// many cut radii away the whole block lies (far field with four terms at FAR_K4, five at FAR_K5,
// six at FAR_K; 0: closed form), and (EXP) whether the member joins the block's local expansion
// (a far member at least LX_DIST block radii from the centre).  Every result depends only on the
// global block and the member.
struct TileCls {
  bool flag, ex;
  int tier;
  double ddx, ddy;      // offset of the member from the block centre
};
template <bool FAR, bool D3, bool EXP, int TP>
__device__ __forceinline__ TileCls tile_class(double x, double y, double ar, float rn2, const TileLane<TP>& L) {
  TileCls c;
  c.ddx = x - L.X; c.ddy = y - L.Y;
  const double ex = fmax(fabs(c.ddx) - L.hwx, 0.0), ey = fmax(fabs(c.ddy) - L.hwy, 0.0);
  const double e2 = fma(ex, ex, ey * ey);
  c.flag = e2 < (double)rn2 * (1.0 + 1e-5);
  const double a2r = ar * ar;
  constexpr double K4 = D3 ? FAR_D3_K4 : FAR_K4, K5 = D3 ? FAR_D3_K5 : FAR_K5, K6 = D3 ? FAR_D3_K : FAR_K;
  c.tier = 0;
  if (FAR && !c.flag && ar <= FAR_AMAX)
    c.tier = e2 >= K4 * K4 * a2r ? 4 : e2 >= K5 * K5 * a2r ? 5 : e2 >= K6 * K6 * a2r ? 6 : 0;
  c.ex = EXP && c.tier != 0 &&
         fma(c.ddx, c.ddx, c.ddy * c.ddy) >= LX_DIST * LX_DIST * fma(L.hwx, L.hwx, L.hwy * L.hwy);
  return c;
}

// The block's local expansion (lf_lexp.h): every member of [lo, hi) that tile_class puts in it
// adds its coefficients on the lane that holds it; the wave sums them into its LDS area (the
// member loop's first wave_sync orders these reads before the records are written there) and
// adds the expansion's deflection and Hessian at each of the lane's points.
template <bool D3, int TP>
__device__ __forceinline__ void lexp_pass(const MemSoA& so, int lo, int hi, const TileLane<TP>& L, Acc (&acc)[TP]) {
  const int lane = threadIdx.x & 63;
  LxAcc g;
  lx_zero(g);
  bool any = false;
  for (int b0 = lo; b0 < hi; b0 += 64) {
    const int h = b0 + lane;
    if (h < hi) {
      const TileCls c = tile_class<true, D3, true, TP>(so.x[h], so.y[h], so.a[h], so.rn2[h], L);
      if (c.ex) {
        float fm[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) fm[k] = so.fm[k * so.pad + h];
        lx_member((float)c.ddx, (float)c.ddy, fm, g);
        any = true;
      }
    }
  }
  if (__ballot(any) == 0) return;
  lx_reduce_store(g, L.dsh);
  wave_sync();
  lx_eval<D3, TP>(L.dsh, L.u, L.v, acc);
}

// Members are taken in blocks of 64.  Lane j of the wave takes member j of the block and
// classifies it (tile_class).  The far dPIE members at least LX_DIST
// block radii away are summed by the block's local expansion first (lexp_pass) and skipped
// here.  Ballots give the wave's near, far and closed-form sets, and the records are written to
// LDS in the order four-term, five-term, six-term far members, then closed-form ones (each set
// in member order), so that every run of LF_CHUNK members has one evaluation (full runs
// unrolled).  Runs are counted from the start of each set; near-field members are evaluated
// after the block lane by lane, exactly as in seg_loop: in FP64 from the FP64 record where the
// lane's r^2 < rn2, otherwise in FP32 from the pair offsets, each term added to the FP64
// accumulators.  Every set depends only on the global block and the member, so results do not
// depend on the launch shape.
template <int SEG, bool D3, int TP>
__device__ __forceinline__ void seg_loop_tile(const MemRec32* __restrict__ rec, const MemRec64* __restrict__ near64,
                                              const MemSoA& so, int lo, int hi, const TileLane<TP>& L,
                                              Acc (&acc)[TP], const Quad& qd) {
  static_assert(SEG == SEG_CPJE || SEG == SEG_CSIE, "tiles hold the circular segments");
  constexpr int LS = TILE_LSTRIDE<SEG, D3>;
  constexpr bool FAR = TILE_FAR<SEG, D3>;
  constexpr bool EXP = FAR;
  if constexpr (EXP) lexp_pass<D3, TP>(so, lo, hi, L, acc);
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int b0 = lo; b0 < hi; b0 += 64) {
    const int nb = min(64, hi - b0);
    bool flag = false;
    int tier = 0;                       // far-field terms (4, 5 or 6), 0: closed form
    bool ex = false;                    // summed by the local expansion
    float dxf = 0.f, dyf = 0.f;
    float4 w0 = make_float4(0.f, 0.f, 0.f, 0.f), w1 = w0, w2 = w0, w3 = w0;
    if (lane < nb) {
      const int h = b0 + lane;
      const TileCls c = tile_class<FAR, D3, EXP, TP>(so.x[h], so.y[h], so.a[h], so.rn2[h], L);
      flag = c.flag;
      ex = c.ex;
      tier = ex ? 0 : c.tier;
      dxf = (float)c.ddx; dyf = (float)c.ddy;
    }
    // the records of the members this wave stages (LDS) are read by those lanes only
    if (lane < nb && !flag && !ex) {
      const MemRec32& r = rec[b0 + lane];
      w0 = make_float4(dxf, dyf, r.s2, r.a2);
      w1 = make_float4(r.s, r.a, r.bd, r.apls);
      w2 = make_float4(r.b, 0.f, 0.f, 0.f);
      if constexpr (!D3) {
        // without third derivatives a far record fits the closed form's three 16-byte words
        // (four with six terms), selected here and written by one store sequence below
        if (tier == 4) {
          w0 = make_float4(dxf, dyf, r.fm[0], r.fm[1]);
          w1 = make_float4(r.fm[2], r.fm[3], r.fw[0], r.fw[1]);
          w2 = make_float4(r.fw[2], r.fw[3], 0.f, 0.f);
        } else if (tier == 5) {
          w0 = make_float4(dxf, dyf, r.fm[0], r.fm[1]);
          w1 = make_float4(r.fm[2], r.fm[3], r.fm[4], r.fw[0]);
          w2 = make_float4(r.fw[1], r.fw[2], r.fw[3], r.fw[4]);
        } else if (tier == 6) {
          w0 = make_float4(dxf, dyf, r.fm[0], r.fm[1]);
          w1 = make_float4(r.fm[2], r.fm[3], r.fm[4], r.fm[5]);
          w2 = make_float4(r.fw[0], r.fw[1], r.fw[2], r.fw[3]);
          w3 = make_float4(r.fw[4], r.fw[5], 0.f, 0.f);
        }
      }
    }
    const bool closed = lane < nb && !flag && !ex && tier == 0;
    const unsigned long long nmask = __ballot(flag), m4 = __ballot(tier == 4), m5 = __ballot(tier == 5),
                             m6 = __ballot(tier == 6), cmask = __ballot(closed);
    const int n4 = __popcll(m4), n5 = __popcll(m5), n6 = __popcll(m6), ncl = __popcll(cmask);
    const int nfar = n4 + n5 + n6;
    const int slot = tier == 4 ? __popcll(m4 & below)
                   : tier == 5 ? n4 + __popcll(m5 & below)
                   : tier == 6 ? n4 + n5 + __popcll(m6 & below)
                               : nfar + __popcll(cmask & below);
    wave_sync();                        // the previous block's reads precede these writes
    if (D3 && tier != 0) {
      put_far_d3(L.dsh + LS * slot, tier, dxf, dyf, rec[b0 + lane]);
    } else if (tier != 0 || closed) {
      float* lw = L.dsh + LS * slot;
      *(float4*)lw = w0;
      *(float4*)(lw + 4) = w1;
      *(float4*)(lw + 8) = w2;
      if (!D3 && LS > 12 && tier == 6) *(float4*)(lw + 12) = w3;
    }
    wave_sync();
    if constexpr (FAR) {
      far_runs<TP, 4, LS, D3>(0, n4, L, acc);
      far_runs<TP, 5, LS, D3>(n4, n4 + n5, L, acc);
      far_runs<TP, 6, LS, D3>(n4 + n5, nfar, L, acc);
    }
    for (int c0 = nfar; c0 < nfar + ncl; c0 += LF_CHUNK) {
      const int n = min(LF_CHUNK, nfar + ncl - c0);
      const float* lr = L.dsh + LS * c0;
      Run32 ps[TP];
#pragma unroll
      for (int k = 0; k < TP; ++k) run_zero<D3>(ps[k]);
      if (!D3 && TP == 1 && n == LF_CHUNK) {
#pragma unroll
        for (int k = 0; k < LF_CHUNK; ++k) tile_term_l<SEG, D3, TP>(lr + LS * k, L, ps);
      } else {
        for (int k = 0; k < n; ++k) tile_term_l<SEG, D3, TP>(lr + LS * k, L, ps);
      }
#pragma unroll
      for (int k = 0; k < TP; ++k) run_flush<D3>(ps[k], acc[k]);
    }
    // near-field members of the block, lane by lane
    unsigned long long fm = nmask;
    while (fm) {
      const int h = b0 + __builtin_ctzll(fm);
      fm &= fm - 1;
      const MemRec32 r = rec[h];
      float xh, xl;
      split32(L.px, xh, xl);
      const float dx = off32(xh, xl, r.xh, r.xl);
#pragma unroll
      for (int k = 0; k < TP; ++k) {
        float yh, yl;
        split32(L.py[k], yh, yl);
        const float dy = off32(yh, yl, r.yh, r.yl);
        if (fmaf(dx, dx, dy * dy) < r.rn2) {
          const MemRec64 q = near64[h];
          Term<double> t;
          if (seg_term<SEG, D3>(q, L.px - q.x, L.py[k] - q.y, qd, t)) add<D3>(acc[k], t);
          else acc[k].flags |= FL_SINGULAR;
        } else {
          Term<float> t;
          seg_term<SEG, D3>(r, dx, dy, qd, t);
          add<D3>(acc[k], t);
        }
      }
    }
  }
}

// All components of one sample in FP64 at one point (main halos + every member segment).
struct Plane64 {
  const MainRec* mains;
  int n_main;
  const MemRec64* mem;
  SegOff seg;
};
// ENFW = false: no elliptical NFW halos in the lens (their quadrature is compiled out).
template <bool D3, bool ENFW = true>
__device__ __forceinline__ void full_sum64(const Plane64& P, double x, double y, const Quad& qd, Acc& acc) {
  for (int c = 0; c < P.n_main; ++c) {
    const MainRec r = P.mains[c];
    eval_main<D3, ENFW>(r, x, y, qd, acc);
    acc.flags |= r.flags;
  }
  double px[1] = {x}, py[1] = {y};
  Acc a1[1];
  a1[0] = acc;
  const SegOff& so = P.seg;
  seg_loop<SEG_CPJE, D3, 1>(P.mem, nullptr, so.off[SEG_CPJE], so.off[SEG_CPJE + 1], px, py, a1, qd);
  seg_loop<SEG_EPJE, D3, 1>(P.mem, nullptr, so.off[SEG_EPJE], so.off[SEG_EPJE + 1], px, py, a1, qd);
  seg_loop<SEG_CSIE, D3, 1>(P.mem, nullptr, so.off[SEG_CSIE], so.off[SEG_CSIE + 1], px, py, a1, qd);
  seg_loop<SEG_ESIE, D3, 1>(P.mem, nullptr, so.off[SEG_ESIE], so.off[SEG_ESIE + 1], px, py, a1, qd);
  seg_loop<SEG_POINT, D3, 1>(P.mem, nullptr, so.off[SEG_POINT], so.off[SEG_POINT + 1], px, py, a1, qd);
  seg_loop<SEG_NFW, D3, 1>(P.mem, nullptr, so.off[SEG_NFW], so.off[SEG_NFW + 1], px, py, a1, qd);
  if constexpr (ENFW) seg_loop<SEG_ENFW, D3, 1>(P.mem, nullptr, so.off[SEG_ENFW], so.off[SEG_ENFW + 1], px, py, a1, qd);
  acc = a1[0];
}

}  // namespace lf
