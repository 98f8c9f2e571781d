// Inference on the device (Sec. 3.5): the affine-invariant ensemble sampler's stretch move and
// the Nelder-Mead downhill simplex, around batched chi^2 evaluations, so that walkers and
// simplices never leave the GPU.
//
// AIES: walkers update in two halves, each half using the other as its complementary
// ensemble: k_aies_propose writes the half's proposals Y = X_j + z (X_k - X_j) into the
// parameter batch, the chi^2 kernels evaluate them, k_aies_accept takes Y with probability
// min(1, z^(D-1) p(Y) / p(X_k)) (log p = -chi^2 / 2 inside the prior box, -inf outside or where
// chi^2 is undefined).  Random numbers: u(seed, n) = top 53 bits of output n of the SplitMix64
// generator seeded with seed (Steele, Lea & Flood 2014), draw n = ((t * 2 + half) * K + k) * 3
// + d for step t, walker k and draw d (0 complementary walker, 1 stretch factor, 2 acceptance).
//
// Nelder-Mead: one state machine per run (a team of lanes, one per coordinate), coefficients
// 1, 2, 1/2, 1/2 and the rules of Lagarias, Reeds, Wright & Wright (1998); vertices kept sorted
// by f (a new vertex goes after those with equal f, a shrink re-sorts stably); one evaluation
// per run and round (the pending point of each run forms the next chi^2 batch; a shrink takes D
// rounds).
//
// Contraction of multiply-adds into fused ones is off in this file, so proposals, centroids
// and simplex moves round exactly as their plain definitions.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include "lf_sample.h"

namespace lf {

namespace {
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long seed, unsigned long long n) {
  unsigned long long z = seed + (n + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ double uniform(unsigned long long seed, unsigned long long n) {
  return (double)(splitmix64(seed, n) >> 11) * 0x1.0p-53;
}
__device__ __forceinline__ bool in_box(const double* p, const double* lo, const double* hi, int D) {
  bool in = true;
  for (int d = 0; d < D; ++d) in = in && p[d] >= lo[d] && p[d] <= hi[d];
  return in;
}
}  // namespace

// ---------------------------------------------------------------------------------------
// AIES
// ---------------------------------------------------------------------------------------
__global__ void k_aies_lp(const AiesArgs A, const double* chi2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= A.K) return;
  const double c = chi2[k];
  A.lp[k] = (in_box(A.X + (size_t)k * A.D, A.lo, A.hi, A.D) && isfinite(c)) ? -0.5 * c : -INFINITY;
}

__global__ void k_aies_propose(const AiesArgs A, long long t, int h) {
  const int H = A.K / 2, w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= H) return;
  const int k = h * H + w;
  const unsigned long long base = (((unsigned long long)t * 2ull + (unsigned long long)h) * A.K + k) * 3ull;
  const double u0 = uniform(A.seed, base), u1 = uniform(A.seed, base + 1);
  int jj = (int)(u0 * H);
  if (jj > H - 1) jj = H - 1;
  const int j = (1 - h) * H + jj;
  const double s = (A.a - 1.0) * u1 + 1.0, z = s * s / A.a;
  const double* xj = A.X + (size_t)j * A.D;
  const double* xk = A.X + (size_t)k * A.D;
  double* y = A.Y + (size_t)w * A.D;
  for (int d = 0; d < A.D; ++d) y[d] = xj[d] + z * (xk[d] - xj[d]);
}

__global__ void k_aies_accept(const AiesArgs A, long long t, int h, const double* chi2) {
  const int H = A.K / 2, w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= H) return;
  const int k = h * H + w;
  const unsigned long long base = (((unsigned long long)t * 2ull + (unsigned long long)h) * A.K + k) * 3ull;
  const double u1 = uniform(A.seed, base + 1), u2 = uniform(A.seed, base + 2);
  const double s = (A.a - 1.0) * u1 + 1.0, z = s * s / A.a;
  const double* y = A.Y + (size_t)w * A.D;
  const double c = chi2[w];
  const double lpY = (in_box(y, A.lo, A.hi, A.D) && isfinite(c)) ? -0.5 * c : -INFINITY;
  const double lnr = (double)(A.D - 1) * log(z) + lpY - A.lp[k];
  if (log(u2) < lnr) {
    double* x = A.X + (size_t)k * A.D;
    for (int d = 0; d < A.D; ++d) x[d] = y[d];
    A.lp[k] = lpY;
    if (A.acc) A.acc[k] += 1;
  }
}

__global__ void k_aies_record(const AiesArgs A, long long row) {
  const long long n = (long long)A.K * A.D, i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (A.chain && i < n) A.chain[row * n + i] = A.X[i];
  if (A.lp_chain && i < A.K) A.lp_chain[row * A.K + i] = A.lp[i];
}

// ---------------------------------------------------------------------------------------
// Nelder-Mead.  A run is handled by a team of TS lanes of one wave (TS = the power of two >= D,
// at most 64): lane d owns coordinate d of every vertex, so centroids, moves and row shifts are
// per-coordinate (coalesced within the team); the values f, the state and the decisions are
// computed redundantly by every lane of the team (each lane only reads what it wrote itself).
// ---------------------------------------------------------------------------------------
namespace {
struct Team {
  double* x;      // [(D+1) * D] vertices, sorted by f
  double* f;      // [D+1]
  double* xr;     // [D]
  double* p;      // [D] pending point
  int D, d;       // parameters, this lane's coordinate (d >= D: idle column)
  unsigned long long mask;   // the team's lanes in the wave
};
__device__ __forceinline__ bool team_all(const Team& t, bool v) {
  return (__ballot(v) & t.mask) == t.mask;
}
__device__ __forceinline__ double nm_value(const Team& t, const double* lo, const double* hi, double c) {
  const bool in = t.d >= t.D || (t.p[t.d] >= lo[t.d] && t.p[t.d] <= hi[t.d]);
  return (team_all(t, in) && isfinite(c)) ? c : INFINITY;
}
__device__ __forceinline__ double centroid(const Team& t) {
  double s = 0.0;
  for (int i = 0; i < t.D; ++i) s += t.x[(size_t)i * t.D + t.d];
  return s / t.D;
}
// pending = c + coef (q - c), q = the reflection (expansion, outside contraction) or the worst
// vertex (inside contraction)
__device__ void set_pending(Team& t, const double* q, double coef) {
  if (t.d >= t.D) return;
  const double c = centroid(t);
  t.p[t.d] = c + coef * (q[t.d] - c);
}
__device__ void set_reflection(Team& t) {
  if (t.d >= t.D) return;
  const double c = centroid(t);
  t.p[t.d] = c + (c - t.x[(size_t)t.D * t.D + t.d]);
}
__device__ void set_shrink(Team& t, int i) {
  if (t.d >= t.D) return;
  t.p[t.d] = t.x[t.d] + 0.5 * (t.x[(size_t)i * t.D + t.d] - t.x[t.d]);
}
// replace the worst vertex by (q, fq), placed after the vertices with f <= fq
__device__ void insert(Team& t, const double* q, double fq) {
  const int D = t.D;
  int k = 0;
  while (k < D && t.f[k] <= fq) ++k;
  const double qd = t.d < D ? q[t.d] : 0.0;
  for (int i = D; i > k; --i) {
    t.f[i] = t.f[i - 1];
    if (t.d < D) t.x[(size_t)i * D + t.d] = t.x[(size_t)(i - 1) * D + t.d];
  }
  t.f[k] = fq;
  if (t.d < D) t.x[(size_t)k * D + t.d] = qd;
}
// stable insertion sort of all D+1 vertices by f
__device__ void sort_all(Team& t) {
  const int D = t.D;
  for (int i = 1; i <= D; ++i) {
    int k = i;
    while (k > 0 && t.f[k - 1] > t.f[k]) {
      const double tf = t.f[k]; t.f[k] = t.f[k - 1]; t.f[k - 1] = tf;
      if (t.d < D) {
        const double tx = t.x[(size_t)k * D + t.d];
        t.x[(size_t)k * D + t.d] = t.x[(size_t)(k - 1) * D + t.d];
        t.x[(size_t)(k - 1) * D + t.d] = tx;
      }
      --k;
    }
  }
}
// the run and coordinate of this lane; false for lanes beyond the last run
__device__ bool team_of(const NMArgs& A, Team& t, int& r) {
  const int TS = A.team, lane = threadIdx.x & 63;
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  r = (int)(g / TS);
  t.d = (int)(g % TS);
  t.D = A.D;
  const int first = lane - t.d;
  t.mask = (TS == 64 ? ~0ull : ((1ull << TS) - 1ull)) << first;
  if (r >= A.R) return false;
  t.x = A.x + (size_t)r * (A.D + 1) * A.D;
  t.f = A.f + (size_t)r * (A.D + 1);
  t.xr = A.xr + (size_t)r * A.D;
  t.p = A.pend + (size_t)r * A.D;
  return true;
}
}  // namespace

// vertices evaluated together (chi2 [R * (D+1)], the parameter batch being the simplices)
__global__ void k_nm_init(const NMArgs A, const double* chi2) {
  Team t;
  int r;
  const bool act = team_of(A, t, r);
  if (!act) return;                   // whole teams leave together (runs are team-aligned)
  for (int v = 0; v <= A.D; ++v) {
    const double c = chi2[(size_t)r * (A.D + 1) + v];
    const bool in = t.d >= t.D || (t.x[(size_t)v * A.D + t.d] >= A.lo[t.d] && t.x[(size_t)v * A.D + t.d] <= A.hi[t.d]);
    t.f[v] = (team_all(t, in) && isfinite(c)) ? c : INFINITY;
  }
  sort_all(t);
  A.state[r] = 0;
  A.idx[r] = 0;
  if (A.nev) A.nev[r] = A.D + 1;
  set_reflection(t);
}

// consume f at each run's pending point (chi2 [R]) and set the next pending point
__global__ void k_nm_step(const NMArgs A, const double* chi2) {
  Team t;
  int r;
  if (!team_of(A, t, r)) return;
  const int D = A.D;
  const double fp = nm_value(t, A.lo, A.hi, chi2[r]);
  if (A.nev && t.d == 0) A.nev[r] += 1;
  const int st = A.state[r];
  const double fr = A.fr[r];
  int nst = 0, nidx = A.idx[r];
  if (st == 0) {                                   // reflection evaluated
    if (t.f[0] <= fp && fp < t.f[D - 1]) {
      insert(t, t.p, fp);
      set_reflection(t);
    } else if (fp < t.f[0]) {
      if (t.d < D) t.xr[t.d] = t.p[t.d];
      if (t.d == 0) A.fr[r] = fp;
      nst = 1;
      set_pending(t, t.xr, 2.0);
    } else if (fp < t.f[D]) {
      if (t.d < D) t.xr[t.d] = t.p[t.d];
      if (t.d == 0) A.fr[r] = fp;
      nst = 2;
      set_pending(t, t.xr, 0.5);
    } else {
      nst = 3;
      set_pending(t, t.x + (size_t)D * D, 0.5);
    }
  } else if (st == 1) {                            // expansion
    if (fp < fr) insert(t, t.p, fp);
    else insert(t, t.xr, fr);
    set_reflection(t);
  } else if (st == 2 || st == 3) {                 // outside / inside contraction
    const bool take = st == 2 ? fp <= fr : fp < t.f[D];
    if (take) {
      insert(t, t.p, fp);
      set_reflection(t);
    } else {
      nst = 4;
      nidx = 1;
      set_shrink(t, 1);
    }
  } else {                                         // shrink: vertex i evaluated
    const int i = nidx;
    if (t.d < D) t.x[(size_t)i * D + t.d] = t.p[t.d];
    t.f[i] = fp;
    if (i < D) {
      nst = 4;
      nidx = i + 1;
      set_shrink(t, i + 1);
    } else {
      sort_all(t);
      set_reflection(t);
    }
  }
  if (t.d == 0) {
    A.state[r] = nst;
    A.idx[r] = nidx;
  }
}

hipError_t launch_aies_lp(const AiesArgs& A, const double* chi2, hipStream_t st) {
  hipLaunchKernelGGL(k_aies_lp, dim3((A.K + 255) / 256), dim3(256), 0, st, A, chi2);
  return hipGetLastError();
}
hipError_t launch_aies_propose(const AiesArgs& A, long long t, int h, hipStream_t st) {
  hipLaunchKernelGGL(k_aies_propose, dim3((A.K / 2 + 255) / 256), dim3(256), 0, st, A, t, h);
  return hipGetLastError();
}
hipError_t launch_aies_accept(const AiesArgs& A, long long t, int h, const double* chi2, hipStream_t st) {
  hipLaunchKernelGGL(k_aies_accept, dim3((A.K / 2 + 255) / 256), dim3(256), 0, st, A, t, h, chi2);
  return hipGetLastError();
}
hipError_t launch_aies_record(const AiesArgs& A, long long row, hipStream_t st) {
  const long long n = (long long)A.K * A.D;
  hipLaunchKernelGGL(k_aies_record, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, A, row);
  return hipGetLastError();
}
hipError_t launch_nm_init(const NMArgs& A, const double* chi2, hipStream_t st) {
  const long long n = (long long)A.R * A.team;
  hipLaunchKernelGGL(k_nm_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, A, chi2);
  return hipGetLastError();
}
hipError_t launch_nm_step(const NMArgs& A, const double* chi2, hipStream_t st) {
  const long long n = (long long)A.R * A.team;
  hipLaunchKernelGGL(k_nm_step, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, A, chi2);
  return hipGetLastError();
}

}  // namespace lf
