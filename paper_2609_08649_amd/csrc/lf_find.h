// Launch interface of the image finder and multi-plane kernels (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "lf_segs.h"

#define LF_MAX_PLANES 8
#define LF_SORT_CAP 8192

namespace lf {

struct LensDev {           // FP64 lens for polishing: 1 plane, or planes with D_ij/D_j
  int n_planes;
  Plane64 pl[LF_MAX_PLANES];
  double wij[LF_MAX_PLANES * LF_MAX_PLANES];
  Quad qd;
};

struct FindArgs {
  double x0, y0, h;
  int nx, ny;
  int n_planes, va_pstride;  // vertex deflection of plane p: va + (pstride p) P (x), +1 (y)
  const double* va;
  int n_src;
  const double* beta;        // [n_src*2]
  const double* w;           // [n_src*n_planes] plane weights (single plane: a_dis)
  double eps;                // candidate margin [arcsec]
  unsigned long long* cand;  // [cap]
  int* n_cand;
  int cap;
  int* c_status;             // [cap] 0 accepted, 1 no convergence, 2 moved > 2h, 3 merged, 4 outside
  double* c_theta;           // [cap*2]
  double* c_mu;              // [cap]
  int max_img;
  double* theta_out;
  double* mu_out;
  int* count_out;
  int* flags_out;
};

struct MPArgs {
  long long P;
  int grid;
  double x0, y0, h;
  int nx;
  const double* px;
  const double* py;
  int n_planes;
  double wij[LF_MAX_PLANES * LF_MAX_PLANES];
  int n_zs;
  const double* wjs;         // [n_zs * LF_MAX_PLANES] D_js / D_s (0 for planes at/behind z_s)
  double* al;                // [N][5][P]: alpha_x, alpha_y, psi11, psi12, psi22 of plane j at theta_j
  double* tx;
  double* ty;
  double* beta;
  double* A;
  double* mu;
};

hipError_t launch_find(const FindArgs& F, const LensDev& L, hipStream_t st,
                       void (*mark)(void*, const char*, int), void* ctx);
hipError_t launch_find_ms(const FindArgs& F, const LensDev& L, int polish, hipStream_t st,
                          void (*mark)(void*, const char*, int), void* ctx);
hipError_t launch_mp_theta(const MPArgs& M, int j, hipStream_t st);
hipError_t launch_mp_final(const MPArgs& M, hipStream_t st);

}  // namespace lf
