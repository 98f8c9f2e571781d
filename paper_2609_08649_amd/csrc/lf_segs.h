// Member-galaxy segment loops shared by the maps, finder and multi-plane kernels.
#pragma once
#include "lf_device.h"

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
    enfw_prime(xp, yp, r.b, r.s, sqrt((double)r.q2), qd, pr);
    rotate_back<false>((double)r.c, (double)r.sn, pr, *(Term<double>*)&t);
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


// All components of one sample in FP64 at one point (main halos + every member segment).
struct Plane64 {
  const MainRec* mains;
  int n_main;
  const MemRec64* mem;
  SegOff seg;
};
template <bool D3>
__device__ __forceinline__ void full_sum64(const Plane64& P, double x, double y, const Quad& qd, Acc& acc) {
  for (int c = 0; c < P.n_main; ++c) {
    const MainRec r = P.mains[c];
    eval_main<D3>(r, x, y, qd, acc);
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
  seg_loop<SEG_ENFW, false, 1>(P.mem, nullptr, so.off[SEG_ENFW], so.off[SEG_ENFW + 1], px, py, a1, qd);
  acc = a1[0];
}

}  // namespace lf
