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
// Nelder-Mead: one state machine per run (one thread), coefficients 1, 2, 1/2, 1/2 and the
// rules of Lagarias, Reeds, Wright & Wright (1998); vertices kept sorted by f (a new vertex goes
// after those with equal f, a shrink re-sorts stably); one evaluation per run and round (the
// pending point of each run forms the next chi^2 batch; a shrink takes D rounds).
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
// Nelder-Mead
// ---------------------------------------------------------------------------------------
namespace {
struct Run {
  double* x;      // [(D+1) * D] vertices, sorted by f
  double* f;      // [D+1]
  double* xr;     // [D] reflection kept for the expansion / outside-contraction decision
  double* p;      // [D] pending point
  int D;
};
__device__ __forceinline__ double nm_value(const double* p, const double* lo, const double* hi, int D, double c) {
  return (in_box(p, lo, hi, D) && isfinite(c)) ? c : INFINITY;
}
__device__ __forceinline__ double centroid(const Run& r, int d) {
  double s = 0.0;
  for (int i = 0; i < r.D; ++i) s += r.x[(size_t)i * r.D + d];
  return s / r.D;
}
// pending = c + coef (q - c) with q = the reflection (state 1, 2) or the worst vertex (3)
__device__ void set_pending(Run& r, const double* q, double coef) {
  for (int d = 0; d < r.D; ++d) {
    const double c = centroid(r, d);
    r.p[d] = c + coef * (q[d] - c);
  }
}
__device__ void set_reflection(Run& r) {
  const double* w = r.x + (size_t)r.D * r.D;
  for (int d = 0; d < r.D; ++d) {
    const double c = centroid(r, d);
    r.p[d] = c + (c - w[d]);
  }
}
__device__ void set_shrink(Run& r, int i) {
  for (int d = 0; d < r.D; ++d) r.p[d] = r.x[d] + 0.5 * (r.x[(size_t)i * r.D + d] - r.x[d]);
}
// replace the worst vertex by (q, fq), placed after the vertices with f <= fq
__device__ void insert(Run& r, const double* q, double fq) {
  const int D = r.D;
  int k = 0;
  while (k < D && r.f[k] <= fq) ++k;
  for (int i = D; i > k; --i) {
    r.f[i] = r.f[i - 1];
    for (int d = 0; d < D; ++d) r.x[(size_t)i * D + d] = r.x[(size_t)(i - 1) * D + d];
  }
  r.f[k] = fq;
  for (int d = 0; d < D; ++d) r.x[(size_t)k * D + d] = q[d];
}
// stable insertion sort of all D+1 vertices by f
__device__ void sort_all(Run& r) {
  const int D = r.D;
  for (int i = 1; i <= D; ++i) {
    int k = i;
    while (k > 0 && r.f[k - 1] > r.f[k]) {
      const double tf = r.f[k]; r.f[k] = r.f[k - 1]; r.f[k - 1] = tf;
      for (int d = 0; d < D; ++d) {
        const double tx = r.x[(size_t)k * D + d];
        r.x[(size_t)k * D + d] = r.x[(size_t)(k - 1) * D + d];
        r.x[(size_t)(k - 1) * D + d] = tx;
      }
      --k;
    }
  }
}
__device__ Run run_of(const NMArgs& A, int r) {
  Run u;
  u.D = A.D;
  u.x = A.x + (size_t)r * (A.D + 1) * A.D;
  u.f = A.f + (size_t)r * (A.D + 1);
  u.xr = A.xr + (size_t)r * A.D;
  u.p = A.pend + (size_t)r * A.D;
  return u;
}
}  // namespace

// vertices evaluated together (chi2 [R * (D+1)], the parameter batch being the simplices)
__global__ void k_nm_init(const NMArgs A, const double* chi2) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= A.R) return;
  Run u = run_of(A, r);
  for (int v = 0; v <= A.D; ++v)
    u.f[v] = nm_value(u.x + (size_t)v * A.D, A.lo, A.hi, A.D, chi2[(size_t)r * (A.D + 1) + v]);
  sort_all(u);
  A.state[r] = 0;
  A.idx[r] = 0;
  if (A.nev) A.nev[r] = A.D + 1;
  set_reflection(u);
}

// consume f at each run's pending point (chi2 [R]) and set the next pending point
__global__ void k_nm_step(const NMArgs A, const double* chi2) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= A.R) return;
  Run u = run_of(A, r);
  const int D = A.D;
  const double fp = nm_value(u.p, A.lo, A.hi, D, chi2[r]);
  if (A.nev) A.nev[r] += 1;
  int st = A.state[r];
  if (st == 0) {                                   // reflection evaluated
    if (u.f[0] <= fp && fp < u.f[D - 1]) {
      insert(u, u.p, fp);
    } else if (fp < u.f[0]) {
      for (int d = 0; d < D; ++d) u.xr[d] = u.p[d];
      A.fr[r] = fp;
      A.state[r] = 1;
      set_pending(u, u.xr, 2.0);
      return;
    } else if (fp < u.f[D]) {
      for (int d = 0; d < D; ++d) u.xr[d] = u.p[d];
      A.fr[r] = fp;
      A.state[r] = 2;
      set_pending(u, u.xr, 0.5);
      return;
    } else {
      A.state[r] = 3;
      set_pending(u, u.x + (size_t)D * D, 0.5);
      return;
    }
  } else if (st == 1) {                            // expansion
    if (fp < A.fr[r]) insert(u, u.p, fp);
    else insert(u, u.xr, A.fr[r]);
  } else if (st == 2 || st == 3) {                 // outside / inside contraction
    const bool take = st == 2 ? fp <= A.fr[r] : fp < u.f[D];
    if (take) {
      insert(u, u.p, fp);
    } else {
      A.state[r] = 4;
      A.idx[r] = 1;
      set_shrink(u, 1);
      return;
    }
  } else {                                         // shrink: vertex i evaluated
    const int i = A.idx[r];
    for (int d = 0; d < D; ++d) u.x[(size_t)i * D + d] = u.p[d];
    u.f[i] = fp;
    if (i < D) {
      A.idx[r] = i + 1;
      set_shrink(u, i + 1);
      return;
    }
    sort_all(u);
  }
  A.state[r] = 0;
  set_reflection(u);
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
  hipLaunchKernelGGL(k_nm_init, dim3((A.R + 63) / 64), dim3(64), 0, st, A, chi2);
  return hipGetLastError();
}
hipError_t launch_nm_step(const NMArgs& A, const double* chi2, hipStream_t st) {
  hipLaunchKernelGGL(k_nm_step, dim3((A.R + 63) / 64), dim3(64), 0, st, A, chi2);
  return hipGetLastError();
}

}  // namespace lf
