// Member-galaxy segment loops shared by the maps, finder and multi-plane kernels.
#pragma once
#include "lf_device.h"

namespace lf {

// ---------------------------------------------------------------------------------------
// Member segment loops over pre-scaled records (MemRec32: FP32 maths on an offset formed
// in FP64; MemRec64: FP64 throughout).  One loop per profile segment.
// ---------------------------------------------------------------------------------------
template <int SEG, bool D3, int PPL, class R>
__device__ __forceinline__ void seg_loop(const R* __restrict__ rec, int lo, int hi,
                                         const double (&px)[PPL], const double (&py)[PPL],
                                         Acc (&acc)[PPL], const Quad& qd) {
  using T = decltype(R::b);
  constexpr bool F32 = sizeof(T) == 4;
  for (int h = lo; h < hi; ++h) {
    const R r = rec[h];
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      T dx = (T)(px[k] - r.x), dy = (T)(py[k] - r.y);
      Term<T> t;
      t.t111 = t.t112 = t.t122 = t.t222 = (T)0;
      if constexpr (SEG == SEG_CPJE || SEG == SEG_CSIE) {
        T r2 = fma(dx, dx, dy * dy);
        if constexpr (F32) {
          // FP32: a point within 1e-6" of a member centre is evaluated at r = 1e-6"
          r2 = fmaxf(r2, 1e-12f);
        } else {
          if (r.s == 0.0 && r2 < 1e-24) { acc[k].flags |= FL_SINGULAR; continue; }
        }
        T m1, w1, p1 = 0;
        cored_mw<D3>(r.b, r.s, r.s2, r2, m1, w1, p1);
        if constexpr (SEG == SEG_CPJE) {
          T m2, w2, p2 = 0;
          cored_mw<D3>(r.b, r.a, r.a2, r2, m2, w2, p2);
          m1 -= m2; w1 -= w2; p1 -= p2;
        }
        radial<D3>(dx, dy, m1, w1, p1, t);
      } else if constexpr (SEG == SEG_EPJE || SEG == SEG_ESIE) {
        if (r.s == (T)0 && dx == (T)0 && dy == (T)0) { acc[k].flags |= FL_SINGULAR; continue; }
        epje<D3>(dx, dy, r.c, r.sn, r.bqe, r.e, r.q2, r.s, r.a, SEG == SEG_EPJE, t);
      } else if constexpr (SEG == SEG_POINT) {
        if (dx == (T)0 && dy == (T)0) { acc[k].flags |= FL_SINGULAR; continue; }
        point_mass<D3>(dx, dy, r.b, t);
      } else if constexpr (SEG == SEG_NFW) {
        if (dx == (T)0 && dy == (T)0) { acc[k].flags |= FL_SINGULAR; continue; }
        nfw_circ<D3>((double)dx, (double)dy, (double)r.b, (double)r.s, *(Term<double>*)&t);
      } else {
        if (dx == (T)0 && dy == (T)0) { acc[k].flags |= FL_SINGULAR; continue; }
        double xp = r.c * dx + r.sn * dy, yp = r.c * dy - r.sn * dx;
        Term<double> pr;
        enfw_prime(xp, yp, r.b, r.s, sqrt(r.q2), qd, pr);
        rotate_back<false>((double)r.c, (double)r.sn, pr, *(Term<double>*)&t);
      }
      add<D3>(acc[k], t);
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
  seg_loop<SEG_CPJE, D3, 1>(P.mem, so.off[SEG_CPJE], so.off[SEG_CPJE + 1], px, py, a1, qd);
  seg_loop<SEG_EPJE, D3, 1>(P.mem, so.off[SEG_EPJE], so.off[SEG_EPJE + 1], px, py, a1, qd);
  seg_loop<SEG_CSIE, D3, 1>(P.mem, so.off[SEG_CSIE], so.off[SEG_CSIE + 1], px, py, a1, qd);
  seg_loop<SEG_ESIE, D3, 1>(P.mem, so.off[SEG_ESIE], so.off[SEG_ESIE + 1], px, py, a1, qd);
  seg_loop<SEG_POINT, D3, 1>(P.mem, so.off[SEG_POINT], so.off[SEG_POINT + 1], px, py, a1, qd);
  seg_loop<SEG_NFW, D3, 1>(P.mem, so.off[SEG_NFW], so.off[SEG_NFW + 1], px, py, a1, qd);
  seg_loop<SEG_ENFW, false, 1>(P.mem, so.off[SEG_ENFW], so.off[SEG_ENFW + 1], px, py, a1, qd);
  acc = a1[0];
}

}  // namespace lf
