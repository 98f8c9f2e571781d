// Launch interface of the singularity-map extraction kernels (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "lf_segs.h"

namespace lf {

struct SingArgs {
  double x0, y0, h;          // vertex (i, j) at (x0 + (i + 1/2) h, y0 + (j + 1/2) h)
  int nx, ny;
  // vertex fields [nx*ny] (row-major): gamma_1, gamma_2, f_1, f_2, flags (umbilic bit)
  const double* g1;
  const double* g2;
  const double* f1;
  const double* f2;
  const int* vflags;
  Plane64 pl;                // FP64 lens for the refinement evaluations
  int enfw;                  // the lens has elliptical NFW halos (selects the kernel variants)
  Quad qd;
  int refine;
  double tol;                // crossing bracket [arcsec]
  int cap;                   // capacity of each output list
  // per-row counts and offsets (rows of vertices for crossings, rows of cells for the rest)
  int* xrow_cnt; int* xrow_off;    // [ny], [ny+1]
  int* srow_cnt; int* srow_off;    // segments per cell row
  int* urow_cnt; int* urow_off;    // umbilic cells per cell row
  int* krow_cnt; int* krow_off;    // cells skipped next to umbilic-flagged vertices
  int* prow_cnt; int* prow_off;    // cells whose crossings could not be paired
  int* wch_cnt; int* wch_off;      // swallowtails per chunk of 256 segments, [cap/256 + 1]
  unsigned short* ebits;     // [nx*ny] per vertex: edge crossings, alignments, umbilic flag
  long long* ckey;           // [cap] crossing keys ((j * 2 + dir) * nx + i) * 2 + k - 1, ascending
  int* xpre;                 // [2 * nx * ny] per direction and vertex: index of its edge's first crossing
  int* ucell;                // [cap*2] cell (i, j) of each umbilic
  // outputs
  double* cpos; int* ck; double* ce; double* cg; int* cfl;
  int* sa; int* sb; int* sk;
  double* upos; double* ukap; int* ustat;
  double* wpos; int* wk; double* we; int* wseg; int* wstat;
  int* counts;               // [6]
};

hipError_t launch_sing(const SingArgs& A, int n_cu, hipStream_t st,
                       void (*mark)(void*, const char*, int), void* ctx);

}  // namespace lf
