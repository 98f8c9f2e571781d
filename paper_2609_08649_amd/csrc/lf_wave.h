// FP64 lens evaluation for a handful of points (polishing and refinement passes): one wave per
// point, the halos of a plane split over the 64 lanes, partial sums combined by a butterfly
// of shuffles (every lane ends with the same bits), the iteration logic run redundantly by
// all lanes.  D3: third derivatives too.  ENFW = false compiles the elliptical NFW quadrature
// out (for lenses without such halos; their kernels then need fewer registers).
#pragma once
#include <hip/hip_runtime.h>

#include "lf_segs.h"

namespace lf {

template <bool D3, bool ENFW = true>
__device__ void member64_term(const Plane64& P, int m, double x, double y, const Quad& qd, Acc& acc) {
  int sg = 0;
  while (sg + 1 < NSEG && m >= P.seg.off[sg + 1]) ++sg;
  const MemRec64 r = P.mem[m];
  double dx = x - r.x, dy = y - r.y;
  double r2 = fma(dx, dx, dy * dy);
  Term<double> t;
  t.t111 = t.t112 = t.t122 = t.t222 = 0.0;
  bool sing = (r2 < 1e-24) && (r.s == 0.0 || sg == SEG_POINT || sg == SEG_NFW || sg == SEG_ENFW);
  if (sing) { acc.flags |= FL_SINGULAR; return; }
  switch (sg) {
    case SEG_CPJE: cpje<D3>(dx, dy, r.b, r.s, r.a, r.s2, r.a2, r.bd, r.apls, t); break;
    case SEG_EPJE: epje<D3>(dx, dy, r.c, r.sn, r.bqe, r.e, r.q2, r.s, r.a, true, t); break;
    case SEG_CSIE: csie<D3>(dx, dy, r.b, r.s, r.s2, t); break;
    case SEG_ESIE: epje<D3>(dx, dy, r.c, r.sn, r.bqe, r.e, r.q2, r.s, r.a, false, t); break;
    case SEG_POINT: point_mass<D3>(dx, dy, r.b, t); break;
    case SEG_NFW: nfw_circ<D3>(dx, dy, r.b, r.s, t); break;
    default: {
      if constexpr (ENFW) {
        double xp = r.c * dx + r.sn * dy, yp = r.c * dy - r.sn * dx;
        Term<double> pr;
        enfw_prime<D3>(xp, yp, r.b, r.s, sqrt(r.q2), qd, pr);
        rotate_back<D3>(r.c, r.sn, pr, t);
      } else {
        acc.flags |= FL_INVALID;
        return;
      }
    }
  }
  add<D3>(acc, t);
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wor(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v |= __shfl_xor(v, o, 64);
  return v;
}

template <bool D3, bool ENFW = true>
__device__ void plane_sum_wave(const Plane64& P, double x, double y, const Quad& qd, Acc& out) {
  Acc acc;
  acc.zero();
  const int lane = threadIdx.x & 63;
  const int H = P.n_main + P.seg.off[NSEG];
  for (int h = lane; h < H; h += 64) {
    if (h < P.n_main) {
      const MainRec r = P.mains[h];
      eval_main<D3, ENFW>(r, x, y, qd, acc);
      acc.flags |= r.flags;
    } else {
      member64_term<D3, ENFW>(P, h - P.n_main, x, y, qd, acc);
    }
  }
  out.ax = wsum(acc.ax); out.ay = wsum(acc.ay);
  out.h11 = wsum(acc.h11); out.h12 = wsum(acc.h12); out.h22 = wsum(acc.h22);
  if (D3) {
    out.t111 = wsum(acc.t111); out.t112 = wsum(acc.t112); out.t122 = wsum(acc.t122); out.t222 = wsum(acc.t222);
  } else {
    out.t111 = out.t112 = out.t122 = out.t222 = 0.0;
  }
  out.flags = wor(acc.flags);
}

}  // namespace lf
