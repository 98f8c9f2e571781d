// Internal launch interface between the host runtime (lf_api.cpp) and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "lf_internal.h"

namespace lf {

struct DevModel {          // device view of a resident model
  const MainDesc* main;    // [n_main]
  int n_main;
  const MemCat* mem;       // [n_mem], sorted by segment
  int n_mem;
  SegOff seg;
  Bind mul[3];             // bmul, smul, amul
  XfConst xc;
  int n_free;
  int has_enfw;            // an elliptical NFW main component or member (selects kernel variants)
  int has_rare;            // members outside the circular segments
};

struct QuadTab {           // eNFW quadrature nodes (device)
  int n;
  const double* u;
  const double* w;
};

struct PointsSpec {
  int grid;                // 1: regular grid, 0: explicit arrays
  double x0, y0, h;
  int nx, ny;
  const double* px;
  const double* py;
  long long P;
  long long p0;            // grid: global index of point 0 (row chunks of a larger grid)
};

struct MapsOut {
  double *ax, *ay, *p11, *p12, *p22, *kappa, *g1, *g2, *detA, *mu, *bx, *by;
  double *t111, *t112, *t122, *t222, *e1, *e2, *f1, *f2;
  int* flags;
};

// a1: per-sample expansion of main components, multipliers and (optionally) pre-scaled
// member tables.  Writes mains [S*n_main], muls [S], m32/m64 [S*n_mem] (each may be null; m32
// is followed by the S structure-of-arrays blocks of mem_soa, mem32_bytes(S, n_mem) in all).
hipError_t launch_expand(const DevModel& m, const double* params, int S, MainRec* mains,
                         MulRec* muls, MemRec32* m32, MemRec64* m64, hipStream_t st);

// Halo sums and fused epilogue over points for S samples.
hipError_t launch_maps(const DevModel& m, const MainRec* mains, const MemRec32* m32,
                       const MemRec64* m64, int S, const PointsSpec& pts, double a_dis,
                       bool mixed, bool d3, const MapsOut& out, const QuadTab& q, int ppl,
                       double* part, int which /*1 heavy, 2 lean*/, hipStream_t st);

// true when a model has components evaluated by the heavy (register-hungry) pass
inline bool has_heavy(const DevModel& m) {
  return m.n_main > 0 || m.seg.off[NSEG] > m.seg.off[SEG_CSIE + 1] || m.seg.off[SEG_EPJE + 1] > m.seg.off[SEG_EPJE];
}

}  // namespace lf
