// Singularity-map extraction (Sec. 6): A3 lines, umbilics (D4) and swallowtails (A4) of a
// single-plane lens from its fields on a vertex grid, each point refined with FP64 halo sums.
//
// A3 line of e_k: zero set of f_k = v_k . grad e_k (the cusp condition; independent of the
// distance ratio, the cusp there forming for a = 1/e_k).  v_k is a line field, so f_k is
// compared between two points only after aligning the second eigenvector with the first.
// Around an umbilic (gamma = 0) the line field turns by a half turn: the product of the four
// edge alignments of a cell is -1 exactly when the cell holds one, and an odd number of lines
// of each family ends there.  A swallowtail lies on an A3 line where v_k is tangent to it:
// g_k = v_k . grad f_k (orientation independent) changes sign along the line.
//
// Pipeline (one stream, no host synchronisation; every list is compacted by prefix sums in a
// fixed order, so results do not depend on the launch shape):
//   1. k_sing_bits / k_sing_keys: per vertex row, every grid edge and family: does f_k change
//      sign after alignment?  One 16-bit word per vertex (crossings, alignments, umbilic
//      flag), a scan, then the crossings in the order (row j; horizontal edges by i, then
//      vertical edges by i; k = 1, 2), stored as ascending keys, with each vertex's index of
//      its edges' first crossings (a prefix count);
//   2. k_sing_refine: one lane per crossing: Illinois regula falsi on the edge with FP64
//      evaluations, then e_k and g_k (central differences);
//   3. k_sing_cells: per cell row, per family, from the four vertex words: segments (two
//      crossings; four: the asymptotic decider of the bilinear interpolant), umbilic cells and
//      the segments that end at them; crossing indices read from the prefix counts;
//   4. k_sing_umb: one wave per umbilic cell: Newton on (gamma_1, gamma_2) = 0;
//   5. k_sing_swt: segments whose ends' g_k differ in sign give swallowtails (interpolated),
//      refined by Newton on (f_k, g_k) = 0 with difference Jacobians (a workgroup of eight
//      waves per point).
#include <hip/hip_runtime.h>

#include "lf_sing.h"
#include "lf_wave.h"

namespace lf {

namespace {

constexpr int NT = 256;

struct VA3 {                 // eigenvectors and A3 fields at a point (family k = 0, 1)
  double f0, f1, v0x, v0y, v1x, v1y, e0, e1;
  bool umb;
  // family selection by value (no indexed arrays: they would live in scratch memory)
  __device__ __forceinline__ double f(int k) const { return k ? f1 : f0; }
  __device__ __forceinline__ double e(int k) const { return k ? e1 : e0; }
  __device__ __forceinline__ double vx(int k) const { return k ? v1x : v0x; }
  __device__ __forceinline__ double vy(int k) const { return k ? v1y : v0y; }
};

__device__ __forceinline__ void default_vectors(VA3& o) {
  o.v0x = 1.0; o.v0y = 0.0; o.v1x = 0.0; o.v1y = 1.0;
}

__device__ __forceinline__ VA3 vertex_a3(const SingArgs& A, int i, int j) {
  const size_t p = (size_t)j * A.nx + i;
  VA3 o;
  o.umb = (A.vflags[p] & FL_UMBILIC) != 0;
  o.f0 = A.f1[p];
  o.f1 = A.f2[p];
  o.e0 = o.e1 = 0.0;
  if (o.umb) { default_vectors(o); return o; }
  const double g1 = A.g1[p], g2 = A.g2[p];
  a3_vectors(g1, g2, sqrt(g1 * g1 + g2 * g2), o.v0x, o.v0y, o.v1x, o.v1y);
  return o;
}

// FP64 evaluation at one point: by the whole wave (LANE = false; every lane returns the same
// bits) or by each lane at its own point (LANE = true; every lane walks the same halo list).
// E = false: the lens has no elliptical NFW halo (their quadrature is compiled out).
template <bool LANE, bool E>
__device__ VA3 point_a3(const SingArgs& A, double x, double y) {
  Acc acc;
  if (LANE) {
    acc.zero();
    full_sum64<true, E>(A.pl, x, y, A.qd, acc);
  } else {
    plane_sum_wave<true, E>(A.pl, x, y, A.qd, acc);
  }
  VA3 o;
  const double kap = 0.5 * (acc.h11 + acc.h22), g1 = 0.5 * (acc.h11 - acc.h22), g2 = acc.h12;
  const double gm = sqrt(g1 * g1 + g2 * g2);
  o.e0 = kap + gm;
  o.e1 = kap - gm;
  o.f0 = o.f1 = 0.0;
  o.umb = !a3_fields(kap, g1, g2, acc.t111, acc.t112, acc.t122, acc.t222, o.f0, o.f1, o.v0x, o.v0y, o.v1x, o.v1y);
  if (o.umb) default_vectors(o);
  return o;
}

// +1 when b's eigenvector k points the same way as a's (dot >= 0), else -1
__device__ __forceinline__ double align(const VA3& a, const VA3& b, int k) {
  return a.vx(k) * b.vx(k) + a.vy(k) * b.vy(k) >= 0.0 ? 1.0 : -1.0;
}
__device__ __forceinline__ bool neg(double v) { return v < 0.0; }   // zero counts as positive
__device__ __forceinline__ bool edge_cross(const VA3& a, const VA3& b, int k) {
  if (a.umb || b.umb) return false;
  return neg(a.f(k)) != neg(align(a, b, k) * b.f(k));
}
__device__ __forceinline__ long long edge_key(int nx, int i, int j, int dir, int k) {
  return (((long long)j * 2 + dir) * nx + i) * 2 + k;
}

// Central differences of f_k aligned with P's eigenvector, at (x +- d, y) and (x, y +- d):
// returns (f(x+d) - f(x-d)) / 2d and (f(y+d) - f(y-d)) / 2d.  One evaluation site in a loop
// keeps the register footprint of a single halo sum.
template <bool LANE, bool E>
__device__ void fd_grad(const SingArgs& A, const VA3& P, double x, double y, int k, double d, bool& umb,
                        double& fx, double& fy) {
  double sx = 0.0, sy = 0.0;
#pragma unroll 1
  for (int m = 0; m < 4; ++m) {
    const double qx = m == 0 ? x + d : m == 1 ? x - d : x;
    const double qy = m == 2 ? y + d : m == 3 ? y - d : y;
    const VA3 q = point_a3<LANE, E>(A, qx, qy);
    if (q.umb) umb = true;
    const double F = align(P, q, k) * q.f(k);
    if (m == 0) sx = F;
    else if (m == 1) sx = sx - F;
    else if (m == 2) sy = F;
    else sy = sy - F;
  }
  fx = sx / (2 * d);
  fy = sy / (2 * d);
}

// exclusive prefix sum over the 256 threads of a block (all threads call it)
__device__ int block_scan(int v, int* lds, int& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[w] = x;
  __syncthreads();
  int off = 0;
  for (int q = 0; q < w; ++q) off += lds[q];
  total = lds[0] + lds[1] + lds[2] + lds[3];
  __syncthreads();
  return off + x - v;
}

__device__ __forceinline__ int n_cross(const SingArgs& A) { return min(A.counts[0], A.cap); }

}  // namespace

// ---------------------------------------------------------------------------------------
// scan of per-row counts: off[0..n], total
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_sing_scan(const int* cnt, int n, int* off, int* total) {
  __shared__ int lds[4];
  int run = 0;
  for (int base = 0; base < n; base += NT) {
    const int t = base + threadIdx.x;
    const int v = t < n ? cnt[t] : 0;
    int tot;
    const int pre = block_scan(v, lds, tot);
    if (t < n) off[t] = run + pre;
    run += tot;
  }
  if (threadIdx.x == 0) {
    off[n] = run;
    *total = run;
  }
}

// ---------------------------------------------------------------------------------------
// 1. crossings.  k_sing_bits: one thread per vertex computes a 16-bit word for its right
//    (horizontal) and upper (vertical) edges: bit 0/1 horizontal crossing k = 1/2, bit 2/3
//    vertical crossing, bit 4/5 horizontal / vertical alignment of family 1 (dot >= 0), bit
//    6/7 the same for family 2, bit 8 the vertex is umbilic-flagged; and the row's crossing
//    count.  k_sing_keys writes the crossing keys in the canonical order.
// ---------------------------------------------------------------------------------------
namespace {
constexpr unsigned B_UMB = 0x100;
__device__ __forceinline__ double bsign(unsigned b, int bit) { return (b >> bit) & 1 ? 1.0 : -1.0; }
}  // namespace

__global__ __launch_bounds__(NT) void k_sing_bits(const SingArgs A) {
  __shared__ int lds[4];
  const int j = blockIdx.x;
  int run = 0;
  for (int base = 0; base < A.nx; base += NT) {
    const int i = base + threadIdx.x;
    int c = 0;
    if (i < A.nx) {
      const VA3 a = vertex_a3(A, i, j);
      unsigned bits = a.umb ? B_UMB : 0u;
      if (i + 1 < A.nx) {
        const VA3 b = vertex_a3(A, i + 1, j);
        for (int k = 0; k < 2; ++k) {
          if (edge_cross(a, b, k)) bits |= 1u << k;
          if (align(a, b, k) > 0.0) bits |= 0x10u << (2 * k);
        }
      }
      if (j + 1 < A.ny) {
        const VA3 b = vertex_a3(A, i, j + 1);
        for (int k = 0; k < 2; ++k) {
          if (edge_cross(a, b, k)) bits |= 4u << k;
          if (align(a, b, k) > 0.0) bits |= 0x20u << (2 * k);
        }
      }
      A.ebits[(size_t)j * A.nx + i] = (unsigned short)bits;
      c = __popc(bits & 0xFu);
    }
    int tot;
    block_scan(c, lds, tot);
    run += tot;
  }
  if (threadIdx.x == 0) A.xrow_cnt[j] = run;
}

__global__ __launch_bounds__(NT) void k_sing_keys(const SingArgs A) {
  __shared__ int lds[4];
  const int j = blockIdx.x;
  int run = A.xrow_off[j];
  for (int dir = 0; dir < 2; ++dir)
    for (int base = 0; base < A.nx; base += NT) {
      const int i = base + threadIdx.x;
      const unsigned m = i < A.nx ? (A.ebits[(size_t)j * A.nx + i] >> (2 * dir)) & 3u : 0u;
      int tot;
      int idx = run + block_scan(__popc(m), lds, tot);
      if (i < A.nx) A.xpre[(size_t)dir * A.nx * A.ny + (size_t)j * A.nx + i] = idx;
      for (int k = 0; k < 2; ++k)
        if ((m >> k) & 1u) {
          if (idx < A.cap) A.ckey[idx] = edge_key(A.nx, i, j, dir, k);
          ++idx;
        }
      run += tot;
    }
}

// ---------------------------------------------------------------------------------------
// 2. refinement of each crossing (one wave per crossing, persistent waves)
// ---------------------------------------------------------------------------------------
template <bool LANE, bool E>
__device__ void refine_crossing(const SingArgs& A, int n) {
  const long long key = A.ckey[n];
  const int k = (int)(key & 1);
  long long r = key >> 1;
  const int i = (int)(r % A.nx);
  r /= A.nx;
  const int dir = (int)(r & 1), j = (int)(r >> 1);
  const VA3 a = vertex_a3(A, i, j);
  const VA3 b = dir == 0 ? vertex_a3(A, i + 1, j) : vertex_a3(A, i, j + 1);
  const double ax = A.x0 + (i + 0.5) * A.h, ay = A.y0 + (j + 0.5) * A.h;
  const double dxh = dir == 0 ? A.h : 0.0, dyh = dir == 0 ? 0.0 : A.h;
  double F0 = a.f(k), F1 = align(a, b, k) * b.f(k);
  const double Fend = fmax(fabs(F0), fabs(F1));
  double t0 = 0.0, t1 = 1.0, t = F0 / (F0 - F1);
  int flags = 0;
  if (A.refine) {
    int side = 0;
    bool done = false;
    for (int it = 0; it < 100 && !done; ++it) {
      double tn = (t0 * F1 - t1 * F0) / (F1 - F0);
      if (!(tn > t0 && tn < t1)) tn = 0.5 * (t0 + t1);
      const VA3 q = point_a3<LANE, E>(A, ax + tn * dxh, ay + tn * dyh);
      if (q.umb) flags |= 1;
      const double F = align(a, q, k) * q.f(k);
      t = tn;
      if (F == 0.0) { done = true; break; }
      if (neg(F) == neg(F0)) {
        t0 = tn; F0 = F;
        if (side == -1) F1 *= 0.5;
        side = -1;
      } else {
        t1 = tn; F1 = F;
        if (side == 1) F0 *= 0.5;
        side = 1;
      }
      if ((t1 - t0) * A.h < A.tol) { t = 0.5 * (t0 + t1); done = true; }
    }
    if (!done) flags |= 2;
  }
  const double cx = ax + t * dxh, cy = ay + t * dyh;
  const VA3 P = point_a3<LANE, E>(A, cx, cy);
  const double e = P.e(k);
  double g = 0.0;
  if (P.umb) {
    flags |= 1;
  } else {
    if (A.refine && fabs(P.f(k)) > 1e-3 * Fend) flags |= 4;     // a jump, not a root
    bool u = false;
    double fx, fy;
    fd_grad<LANE, E>(A, P, cx, cy, k, 1e-3 * A.h, u, fx, fy);
    if (u) flags |= 1;
    g = P.vx(k) * fx + P.vy(k) * fy;
  }
  if (LANE || (threadIdx.x & 63) == 0) {
    A.cpos[2 * (size_t)n] = cx;
    A.cpos[2 * (size_t)n + 1] = cy;
    A.ck[n] = k + 1;
    A.ce[n] = e;
    A.cg[n] = g;
    A.cfl[n] = flags;
  }
}
// one lane per crossing: lanes of a wave hold neighbouring edges of a row, iterate alike and
// read every halo record at the same time (scalar loads)
template <bool E>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_sing_refine(const SingArgs A) {
  const int n = blockIdx.x * NT + threadIdx.x;
  if (n < n_cross(A)) refine_crossing<true, E>(A, n);
}

// ---------------------------------------------------------------------------------------
// 3. cells: segments and umbilic cells
// ---------------------------------------------------------------------------------------
namespace {
// index in the crossing list of crossing k of the edge of vertex (i, j) in direction dir (w:
// that vertex's word): the keys are in canonical order, so it is the vertex's prefix count
// from the key pass, plus one for k = 1 when the edge also holds crossing k = 0
__device__ __forceinline__ int cross_index(const SingArgs& A, int i, int j, int dir, int k, unsigned w) {
  const int base = A.xpre[(size_t)dir * A.nx * A.ny + (size_t)j * A.nx + i];
  return base + (k == 1 ? (int)((w >> (2 * dir)) & 1u) : 0);
}
struct CellRes {
  int nseg, umb, stat4, skipped, unpaired;
};
// Marching squares of one cell for both families from the vertex words; emit(a, b, k) for
// each segment in order.
template <class Emit>
__device__ CellRes cell_logic(const SingArgs& A, int i, int j, int uidx, Emit&& emit) {
  CellRes r{0, 0, 0, 0, 0};
  const size_t p0 = (size_t)j * A.nx + i;
  const unsigned b0 = A.ebits[p0], b1 = A.ebits[p0 + 1], b3 = A.ebits[p0 + A.nx], b2 = A.ebits[p0 + A.nx + 1];
  if ((b0 | b1 | b2 | b3) & B_UMB) { r.skipped = 1; return r; }
  // loop c0-c1 (bottom: b0 horizontal), c1-c2 (right: b1 vertical), c2-c3 (top: b3
  // horizontal), c3-c0 (left: b0 vertical)
  const double P = bsign(b0, 4) * bsign(b1, 5) * bsign(b3, 4) * bsign(b0, 5);
  r.umb = P < 0.0 ? 1 : 0;
  for (int k = 0; k < 2; ++k) {
    int xs[4];
    xs[0] = (b0 >> k) & 1u ? cross_index(A, i, j, 0, k, b0) : -1;
    xs[1] = (b1 >> (2 + k)) & 1u ? cross_index(A, i + 1, j, 1, k, b1) : -1;
    xs[2] = (b3 >> k) & 1u ? cross_index(A, i, j + 1, 0, k, b3) : -1;
    xs[3] = (b0 >> (2 + k)) & 1u ? cross_index(A, i, j, 1, k, b0) : -1;
    int n = 0;
    for (int m = 0; m < 4; ++m) n += xs[m] >= 0 ? 1 : 0;
    if (P > 0.0) {
      if (n == 2) {
        int a = -1, b = -1;
        for (int m = 0; m < 4; ++m)
          if (xs[m] >= 0) { if (a < 0) a = xs[m]; else b = xs[m]; }
        emit(a, b, k);
        r.nseg += 1;
      } else if (n == 4) {
        const double* f = k ? A.f2 : A.f1;
        const double a01 = bsign(b0, 4 + 2 * k), a12 = bsign(b1, 5 + 2 * k), a03 = bsign(b0, 5 + 2 * k);
        const double F0 = f[p0];
        const double F1 = a01 * f[p0 + 1];
        const double F2 = a01 * a12 * f[p0 + A.nx + 1];
        const double F3 = a03 * f[p0 + A.nx];
        const double D = F0 + F2 - F1 - F3;
        const bool cpos = D == 0.0 ? true : !neg((F0 * F2 - F1 * F3) / D);
        if (cpos == !neg(F0)) { emit(xs[0], xs[1], k); emit(xs[2], xs[3], k); }
        else { emit(xs[0], xs[3], k); emit(xs[1], xs[2], k); }
        r.nseg += 2;
      } else if (n != 0) {
        r.unpaired += 1;
      }
    } else {
      if (n == 1 || n == 3) {
        for (int m = 0; m < 4; ++m)
          if (xs[m] >= 0) { emit(xs[m], -uidx - 1, k); r.nseg += 1; }
      } else {
        r.stat4 = 1;
        if (n != 0) r.unpaired += 1;
      }
    }
  }
  return r;
}
}  // namespace

template <bool WRITE>
__global__ __launch_bounds__(NT) void k_sing_cells(const SingArgs A) {
  __shared__ int lds[4];
  const int j = blockIdx.x;            // cell row
  const bool over = A.counts[0] > A.cap;
  if (over) {                          // crossing list incomplete: no cell output
    if (!WRITE && threadIdx.x == 0) {
      A.srow_cnt[j] = 0; A.urow_cnt[j] = 0; A.krow_cnt[j] = 0; A.prow_cnt[j] = 0;
    }
    return;
  }
  const int T = A.nx - 1;
  int srun = WRITE ? A.srow_off[j] : 0, urun = WRITE ? A.urow_off[j] : 0, krun = 0, prun = 0;
  for (int base = 0; base < T; base += NT) {
    const int i = base + threadIdx.x;
    CellRes c{0, 0, 0, 0, 0};
    if (i < T) c = cell_logic(A, i, j, 0, [](int, int, int) {});
    int ts, tu, tk, tp;
    const int ps = block_scan(c.nseg, lds, ts);
    const int pu = block_scan(c.umb, lds, tu);
    if (WRITE) {
      if (i < T && (c.nseg || c.umb)) {
        const int uidx = urun + pu;
        int s = srun + ps;
        cell_logic(A, i, j, uidx, [&](int a, int b, int k) {
          if (s < A.cap) { A.sa[s] = a; A.sb[s] = b; A.sk[s] = k + 1; }
          ++s;
        });
        if (c.umb && uidx < A.cap) {
          A.ucell[2 * (size_t)uidx] = i;
          A.ucell[2 * (size_t)uidx + 1] = j;
          A.ustat[uidx] = c.stat4 ? 4 : 0;
        }
      }
    } else {
      block_scan(c.skipped, lds, tk);
      block_scan(c.unpaired, lds, tp);
      krun += tk;
      prun += tp;
    }
    srun += ts;
    urun += tu;
  }
  if (!WRITE && threadIdx.x == 0) {
    A.srow_cnt[j] = srun; A.urow_cnt[j] = urun; A.krow_cnt[j] = krun; A.prow_cnt[j] = prun;
  }
}

// ---------------------------------------------------------------------------------------
// 4. umbilics: Newton on (gamma_1, gamma_2) = 0 from the cell centre; status 0 accepted
//    (converged inside the closed cell), 1 no convergence in 30 steps, 2 outside (| 4 from
//    the cell pass: a family's crossings could not be joined to it)
// ---------------------------------------------------------------------------------------
template <bool E>
__device__ void umbilic_one(const SingArgs& A, int n) {
  const int i = A.ucell[2 * (size_t)n], j = A.ucell[2 * (size_t)n + 1];
  const double xl = A.x0 + (i + 0.5) * A.h, xr = A.x0 + (i + 1.5) * A.h;
  const double yl = A.y0 + (j + 0.5) * A.h, yr = A.y0 + (j + 1.5) * A.h;
  double x = xl + 0.5 * A.h, y = yl + 0.5 * A.h;
  bool conv = false;
  Acc acc;
  for (int it = 0; it < 30; ++it) {
    plane_sum_wave<true, E>(A.pl, x, y, A.qd, acc);
    const double g1 = 0.5 * (acc.h11 - acc.h22), g2 = acc.h12;
    const double J11 = 0.5 * (acc.t111 - acc.t122), J12 = 0.5 * (acc.t112 - acc.t222);
    const double J21 = acc.t112, J22 = acc.t122;
    const double det = J11 * J22 - J12 * J21;
    const double sx = -(J22 * g1 - J12 * g2) / det, sy = -(-J21 * g1 + J11 * g2) / det;
    x += sx;
    y += sy;
    if (sqrt(sx * sx + sy * sy) < 1e-10) { conv = true; break; }
    if (!isfinite(x) || !isfinite(y)) break;
  }
  plane_sum_wave<true, E>(A.pl, x, y, A.qd, acc);
  int st = 1;
  if (conv) st = (x >= xl && x <= xr && y >= yl && y <= yr) ? 0 : 2;
  if ((threadIdx.x & 63) == 0) {
    A.upos[2 * (size_t)n] = x;
    A.upos[2 * (size_t)n + 1] = y;
    A.ukap[n] = 0.5 * (acc.h11 + acc.h22);
    A.ustat[n] |= st;
  }
}
template <bool E>
__global__ __launch_bounds__(NT) void k_sing_umb(const SingArgs A) {
  const int nU = min(A.counts[2], A.cap);
  const int nw = gridDim.x * (NT / 64);
  for (int n = blockIdx.x * (NT / 64) + (threadIdx.x >> 6); n < nU; n += nw) umbilic_one<E>(A, n);
}

// ---------------------------------------------------------------------------------------
// 5. swallowtails
// ---------------------------------------------------------------------------------------
namespace {
__device__ bool swt_flag(const SingArgs& A, int s) {
  const int a = A.sa[s], b = A.sb[s];
  if (a < 0 || b < 0) return false;
  if ((A.cfl[a] | A.cfl[b]) & 5) return false;           // umbilic-flagged evaluation or a jump
  return neg(A.cg[a]) != neg(A.cg[b]);
}
}  // namespace

// chunks of 256 segments: count pass, then write pass (interpolated points in segment order)
template <bool WRITE>
__global__ __launch_bounds__(NT) void k_sing_swt(const SingArgs A) {
  __shared__ int lds[4];
  const int nS = min(A.counts[1], A.cap);
  const int s = blockIdx.x * NT + threadIdx.x;
  const int f = (s < nS && swt_flag(A, s)) ? 1 : 0;
  int tot;
  const int pre = block_scan(f, lds, tot);
  if (!WRITE) {
    if (threadIdx.x == 0) A.wch_cnt[blockIdx.x] = tot;
    return;
  }
  if (!f) return;
  const int w = A.wch_off[blockIdx.x] + pre;
  if (w >= A.cap) return;
  const int a = A.sa[s], b = A.sb[s];
  const double ga = A.cg[a], gb = A.cg[b], u = ga / (ga - gb);
  const double ax = A.cpos[2 * (size_t)a], ay = A.cpos[2 * (size_t)a + 1];
  const double bx = A.cpos[2 * (size_t)b], by = A.cpos[2 * (size_t)b + 1];
  A.wpos[2 * (size_t)w] = ax + u * (bx - ax);
  A.wpos[2 * (size_t)w + 1] = ay + u * (by - ay);
  A.wk[w] = A.sk[s];
  A.wseg[w] = s;
  A.wstat[w] = 0;
}

// Newton on (f_k, g_k) = 0 from the interpolated point, g_k = v_k . grad f_k with grad f_k by
// central differences (step 1e-3 h) and grad g_k by central differences of g (step 1e-2 h),
// stopped after a step below 1e-10", after 20 steps or on leaving the disc of radius h about
// the start: status 0 converged (last step below 1e-8", two decades above the stopping step and
// the ~1e-9" rounding noise that the finite-difference g leaves under the steps) within h of
// the start, 1 no convergence, 2 left the disc (the interpolated point is kept), | 8 an
// umbilic-flagged evaluation; then e_k at the point.  One workgroup per swallowtail: a step needs 25 evaluations (g at the
// point and at (x +- dg, y), (x, y +- dg), each from its point and four difference points),
// spread over SWT_WAVES waves (four rounds); each wave keeps f_k, v_k and the umbilic flag of
// its evaluations in LDS, and every thread then forms the differences in the same order.
constexpr int SWT_WAVES = 8;
template <bool E>
__global__ __launch_bounds__(64 * SWT_WAVES) void k_sing_swt_refine(const SingArgs A) {
  __shared__ double ev[25][3];
  __shared__ int eu[25];
  const int nW = min(A.counts[3], A.cap);
  const int wv = threadIdx.x >> 6;
  for (int n = blockIdx.x; n < nW; n += gridDim.x) {
    const int k = A.wk[n] - 1;
    const double x0 = A.wpos[2 * (size_t)n], y0 = A.wpos[2 * (size_t)n + 1];
    double x = x0, y = y0;
    int st = 0;
    if (A.refine) {
      const double d = 1e-3 * A.h, dg = 1e-2 * A.h;
      bool umb = false;
      double last = HUGE_VAL;
      for (int it = 0; it < 20; ++it) {
        // evaluation e = 5 m + c: stencil point m of g (0 the point, 1/2 x +- dg, 3/4 y +- dg),
        // c = 0 that point, 1..4 its f stencil (x + d, x - d, y + d, y - d)
        for (int e = wv; e < 25; e += SWT_WAVES) {
          const int m = e / 5, c = e - 5 * (e / 5);
          const double qx = m == 1 ? x + dg : m == 2 ? x - dg : x;
          const double qy = m == 3 ? y + dg : m == 4 ? y - dg : y;
          const double px = c == 1 ? qx + d : c == 2 ? qx - d : qx;
          const double py = c == 3 ? qy + d : c == 4 ? qy - d : qy;
          const VA3 P = point_a3<false, E>(A, px, py);
          if ((threadIdx.x & 63) == 0) {
            ev[e][0] = P.f(k); ev[e][1] = P.vx(k); ev[e][2] = P.vy(k);
            eu[e] = P.umb ? 1 : 0;
          }
        }
        __syncthreads();
        double g[5], f = 0.0, fx = 0.0, fy = 0.0;
        for (int m = 0; m < 5; ++m) {
          const int e0 = 5 * m;
          double F[4];
          for (int c = 0; c < 4; ++c) {
            const int e = e0 + 1 + c;
            const double al = ev[e0][1] * ev[e][1] + ev[e0][2] * ev[e][2] >= 0.0 ? 1.0 : -1.0;
            F[c] = al * ev[e][0];
            umb = umb || eu[e] != 0;
          }
          umb = umb || eu[e0] != 0;
          const double gx_ = (F[0] - F[1]) / (2 * d), gy_ = (F[2] - F[3]) / (2 * d);
          g[m] = ev[e0][1] * gx_ + ev[e0][2] * gy_;
          if (m == 0) { f = ev[0][0]; fx = gx_; fy = gy_; }
        }
        __syncthreads();
        const double gx = (g[1] - g[2]) / (2 * dg), gy = (g[3] - g[4]) / (2 * dg);
        const double det = fx * gy - fy * gx;
        const double sx = -(gy * f - fy * g[0]) / det, sy = -(-gx * f + fx * g[0]) / det;
        x += sx;
        y += sy;
        if (!isfinite(x) || !isfinite(y)) { last = HUGE_VAL; break; }
        last = sqrt(sx * sx + sy * sy);
        if (last < 1e-10) break;
        if (hypot(x - x0, y - y0) > A.h) break;
      }
      st = last < 1e-8 ? 0 : 1;
      if (hypot(x - x0, y - y0) > A.h) st = 2;
      if (umb) st |= 8;
      if (st != 0) { x = x0; y = y0; }
    }
    if (wv == 0) {
      const VA3 P = point_a3<false, E>(A, x, y);
      if (threadIdx.x == 0) {
        A.wpos[2 * (size_t)n] = x;
        A.wpos[2 * (size_t)n + 1] = y;
        A.we[n] = P.e(k);
        A.wstat[n] = st;
      }
    }
    __syncthreads();
  }
}

hipError_t launch_sing(const SingArgs& A, int n_cu, hipStream_t st, void (*mark)(void*, const char*, int),
                       void* ctx) {
  const int waves_grid = n_cu * 8;
  const unsigned chunks = (unsigned)((A.cap + NT - 1) / NT);
  mark(ctx, "sing_edges", 0);
  hipLaunchKernelGGL(k_sing_bits, dim3(A.ny), dim3(NT), 0, st, A);
  hipLaunchKernelGGL(k_sing_scan, dim3(1), dim3(NT), 0, st, A.xrow_cnt, A.ny, A.xrow_off, A.counts + 0);
  hipLaunchKernelGGL(k_sing_keys, dim3(A.ny), dim3(NT), 0, st, A);
  mark(ctx, "sing_edges", 1);
  mark(ctx, "sing_refine", 0);
  const dim3 g_ref((unsigned)((A.cap + NT - 1) / NT));
  if (A.enfw) hipLaunchKernelGGL(k_sing_refine<true>, g_ref, dim3(NT), 0, st, A);
  else hipLaunchKernelGGL(k_sing_refine<false>, g_ref, dim3(NT), 0, st, A);
  mark(ctx, "sing_refine", 1);
  mark(ctx, "sing_cells", 0);
  hipLaunchKernelGGL(k_sing_cells<false>, dim3(A.ny - 1), dim3(NT), 0, st, A);
  hipLaunchKernelGGL(k_sing_scan, dim3(1), dim3(NT), 0, st, A.srow_cnt, A.ny - 1, A.srow_off, A.counts + 1);
  hipLaunchKernelGGL(k_sing_scan, dim3(1), dim3(NT), 0, st, A.urow_cnt, A.ny - 1, A.urow_off, A.counts + 2);
  hipLaunchKernelGGL(k_sing_scan, dim3(1), dim3(NT), 0, st, A.krow_cnt, A.ny - 1, A.krow_off, A.counts + 4);
  hipLaunchKernelGGL(k_sing_scan, dim3(1), dim3(NT), 0, st, A.prow_cnt, A.ny - 1, A.prow_off, A.counts + 5);
  hipLaunchKernelGGL(k_sing_cells<true>, dim3(A.ny - 1), dim3(NT), 0, st, A);
  mark(ctx, "sing_cells", 1);
  mark(ctx, "sing_umb", 0);
  if (A.enfw) hipLaunchKernelGGL(k_sing_umb<true>, dim3(waves_grid), dim3(NT), 0, st, A);
  else hipLaunchKernelGGL(k_sing_umb<false>, dim3(waves_grid), dim3(NT), 0, st, A);
  mark(ctx, "sing_umb", 1);
  mark(ctx, "sing_swt", 0);
  hipLaunchKernelGGL(k_sing_swt<false>, dim3(chunks), dim3(NT), 0, st, A);
  hipLaunchKernelGGL(k_sing_scan, dim3(1), dim3(NT), 0, st, A.wch_cnt, (int)chunks, A.wch_off, A.counts + 3);
  hipLaunchKernelGGL(k_sing_swt<true>, dim3(chunks), dim3(NT), 0, st, A);
  if (A.enfw) hipLaunchKernelGGL(k_sing_swt_refine<true>, dim3(n_cu * 4), dim3(64 * SWT_WAVES), 0, st, A);
  else hipLaunchKernelGGL(k_sing_swt_refine<false>, dim3(n_cu * 4), dim3(64 * SWT_WAVES), 0, st, A);
  mark(ctx, "sing_swt", 1);
  return hipGetLastError();
}

}  // namespace lf
