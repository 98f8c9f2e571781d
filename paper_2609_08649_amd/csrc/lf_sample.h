// Launch interface of the on-device inference kernels (internal).
#pragma once
#include <hip/hip_runtime.h>

namespace lf {

struct AiesArgs {
  int K, D;                  // walkers (even), parameters per walker
  double* X;                 // [K * D] walkers
  double* lp;                // [K] log-probabilities
  const double* lo;          // [D] prior box
  const double* hi;
  double a;                  // stretch scale
  unsigned long long seed;
  double* Y;                 // [K/2 * D] proposals of a half (the chi^2 parameter batch)
  int* acc;                  // [K] accepted moves (accumulated; may be null)
  double* chain;             // [n_steps * K * D] (may be null)
  double* lp_chain;          // [n_steps * K] (may be null)
};

struct NMArgs {
  int R, D;                  // runs, parameters
  double* x;                 // [R * (D+1) * D] simplices, sorted by f
  double* f;                 // [R * (D+1)]
  double* xr;                // [R * D] reflection points
  double* fr;                // [R]
  int* state;                // [R] 0 reflect, 1 expand, 2 contract outside, 3 contract inside, 4 shrink
  int* idx;                  // [R] shrink vertex
  double* pend;              // [R * D] pending points (the chi^2 parameter batch)
  const double* lo;          // [D] prior box
  const double* hi;
  int* nev;                  // [R] evaluations (may be null)
  int team;                  // lanes per run: the power of two >= D (<= 64)
};

hipError_t launch_aies_lp(const AiesArgs& A, const double* chi2, hipStream_t st);
hipError_t launch_aies_propose(const AiesArgs& A, long long t, int h, hipStream_t st);
hipError_t launch_aies_accept(const AiesArgs& A, long long t, int h, const double* chi2, hipStream_t st);
hipError_t launch_aies_record(const AiesArgs& A, long long row, hipStream_t st);
hipError_t launch_nm_init(const NMArgs& A, const double* chi2, hipStream_t st);
hipError_t launch_nm_step(const NMArgs& A, const double* chi2, hipStream_t st);

}  // namespace lf
