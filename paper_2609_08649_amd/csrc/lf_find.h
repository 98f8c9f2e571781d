// Launch interface of the image finder and multi-plane kernels (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "lf_segs.h"

#define LF_MAX_PLANES 8
// Candidate lists: capacity max(LF_FIND_CAP_MIN, LF_FIND_CAP_PER_SRC n_src) unless the context
// sets another; a source's list is sorted in LDS up to LF_SEG_LDS keys, in global memory beyond.
#define LF_FIND_CAP_MIN (1 << 16)
#define LF_FIND_CAP_PER_SRC 64
#define LF_SEG_LDS 4096

namespace lf {

struct LensDev {           // FP64 lens for polishing: 1 plane, or planes with D_ij/D_j
  int n_planes;
  int enfw;                  // some plane holds an elliptical NFW halo (selects kernel variants)
  Plane64 pl[LF_MAX_PLANES];
  double wij[LF_MAX_PLANES * LF_MAX_PLANES];
  Quad qd;
};

struct FindArgs {
  double x0, y0, h;
  int nx, ny;
  int n_planes;
  long long va_pstride;      // vertex deflection of plane p: vax + pstride p (x), vay + pstride p (y)
  const double* vax;
  const double* vay;
  int n_src;
  const double* beta;        // [n_src*2]
  const double* w;           // [n_src*n_planes] plane weights (single plane: a_dis)
  double eps;                // candidate margin [arcsec]
  // Candidates, key (source << 32) | triangle or cell code.  The candidate pass appends them
  // in any order to cand_raw and counts them per source; they are then placed in per-source
  // segments of cand (src_off, the exclusive prefix sum of src_cnt) and each segment sorted,
  // so cand is ordered by key whatever the order of the atomics.  When the total exceeds cap,
  // a second candidate pass writes only the sources whose segment fits (a prefix of the
  // sources; the others are flagged), so which results survive does not depend on timing.
  unsigned long long* cand_raw;  // [cap]
  unsigned long long* cand;      // [cap]
  int* n_cand;                   // [0] all candidates found, [1] candidates kept (n_fit), [2] overflow
  int* src_cnt;                  // [n_src]
  int* src_off;                  // [n_src + 1]
  int* src_cur;                  // [n_src]
  int cap;
  int n_cu;                      // compute units (grids of the strided passes)
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
