// Image finder by triangle mapping and the multi-plane passes.
//
// Finder pipeline (all on the device, no host synchronisation):
//   1. vertex deflections on the grid (maps kernels, FP32 members in MIXED);
//   2. k_find_cand: one lane per grid cell (a wave per 8 x 8 tile) keeps FP32 copies of its
//      four corners in registers; mapped corners beta_v = theta_v - sum_j w_j alpha_j(v);
//      the wave's lanes first test 64 sources (staged in LDS) at a time against a box that
//      holds every mapped corner of the tile, then the sources that pass go through two
//      per-cell FP32 prefilters (the mapped cell centre with a radius, then the bounding box)
//      and the FP64 test: a triangle is a candidate when the source lies within eps of it (eps
//      covers the vertex error of the precision in use), appended with one atomic per wave
//      and counted per source;
//   3. k_find_scan / k_find_scatter / k_find_segsort: per-source segments of the candidate
//      list (prefix sum of the counts), each sorted by triangle, so the list is ordered by
//      (source, triangle) whatever the order of the atomics; past the capacity a second
//      candidate pass fills the segments of the sources that fit and the rest are flagged;
//   4. k_find_polish: per candidate (one workgroup each), FP64 vertex deflections, exact
//      orientation signs with the watertight tie rule, barycentric start, FP64 Newton polish
//      and acceptance;
//   5. k_find_final: per source, merge duplicates in candidate order, write images.
#include <hip/hip_runtime.h>

#include "lf_find.h"
#include "lf_segs.h"
#include "lf_wave.h"

namespace lf {

// ---------------------------------------------------------------------------------------
// Exact orientation: sign of (bx-ax)(cy-ay) - (by-ay)(cx-ax).  A floating-point filter with
// the (3 + 16 eps) eps bound, and when it cannot decide, the exact sign of the sum of the
// 16 error-free partial products (expansion arithmetic: two-sum / fma two-product).
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ void d_two_sum(double a, double b, double& x, double& y) {
  x = a + b;
  double bv = x - a, av = x - bv;
  y = (a - av) + (b - bv);
}
__device__ int d_sign_of_sum(const double* t, int n) {
  double e[40];
  int m = 0;
  for (int k = 0; k < n; ++k) {
    double q = t[k];
    int w = 0;
    for (int i = 0; i < m; ++i) {
      double qn, h;
      d_two_sum(q, e[i], qn, h);
      q = qn;
      if (h != 0.0) e[w++] = h;
    }
    if (q != 0.0) e[w++] = q;
    m = w;
  }
  for (int i = m - 1; i >= 0; --i)
    if (e[i] != 0.0) return e[i] > 0 ? 1 : -1;
  return 0;
}
__device__ int d_orient(double ax, double ay, double bx, double by, double cx, double cy) {
  double l = (bx - ax) * (cy - ay), r = (by - ay) * (cx - ax);
  double det = l - r;
  double bound = 3.3306690738754716e-16 * (fabs(l) + fabs(r));
  if (det > bound) return 1;
  if (-det > bound) return -1;
  double A[2], B[2], C[2], D[2];
  d_two_sum(bx, -ax, A[1], A[0]);
  d_two_sum(cy, -ay, B[1], B[0]);
  d_two_sum(by, -ay, C[1], C[0]);
  d_two_sum(cx, -ax, D[1], D[0]);
  double t[16];
  int n = 0;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      double p = A[i] * B[j];
      t[n++] = fma(A[i], B[j], -p);
      t[n++] = p;
      double q = -C[i] * D[j];
      t[n++] = fma(-C[i], D[j], -q);
      t[n++] = q;
    }
  return d_sign_of_sum(t, n);
}
// an edge whose direction, oriented so that the inside is on its left, is lexicographically
// positive owns the points lying exactly on it
__device__ __forceinline__ bool d_edge_closed(int sg, double px, double py, double qx, double qy) {
  if (sg > 0) return qx > px || (qx == px && qy > py);
  return px > qx || (px == qx && py > qy);
}
__device__ bool d_tri_contains(const double* B, double sx, double sy) {
  int sg = d_orient(B[0], B[1], B[2], B[3], B[4], B[5]);
  if (sg == 0) return false;
  for (int e = 0; e < 3; ++e) {
    int a = e, b = (e + 1) % 3;
    int o = d_orient(B[2 * a], B[2 * a + 1], B[2 * b], B[2 * b + 1], sx, sy);
    if (o == 0) {
      if (!d_edge_closed(sg, B[2 * a], B[2 * a + 1], B[2 * b], B[2 * b + 1])) return false;
    } else if (o != sg) {
      return false;
    }
  }
  return true;
}

// FP64 lens evaluation by a whole workgroup (the polishing passes take one candidate per
// workgroup: a few hundred candidates would leave most of the chip idle at one wave each, and
// the evaluation is a chain of dependent sums).  The halos of a plane are split over the
// threads, each wave's partial sums combined by DPP lane moves and the waves' sums added in LDS
// in wave order, so every thread ends with the same bits and runs the iteration
// logic alike (measured: 256 threads per workgroup beat 512 on the cluster lens, whose 304
// work items then leave most threads one item).  ENFW = false compiles the elliptical NFW
// quadrature out.
constexpr int POL_T = 256;
constexpr int POL_W = POL_T / 64;
// Single-plane lenses with at most this many main halos and members have their FP64 records
// copied to LDS once per workgroup (every evaluation of every candidate reads them; 5% off
// the cluster finder's time).
constexpr int POL_LDS_MAIN = 16, POL_LDS_MEM = 320;
struct PolRed {
  double v[POL_W][5];
  int f[POL_W];
};

// Wave sums by DPP lane moves (no LDS round trips, which the butterfly of shuffles takes six of
// in a row): two quad permutations and two row rotations give every lane its row's total, two
// row broadcasts carry the row totals into the last row, and lane 63's value is read out, so
// every lane gets the same bits.  Lanes of rows a move leaves out add zero.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xf, true);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i32<CTRL, ROWS>((int)b), hi = dpp_i32<CTRL, ROWS>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_f64<0xb1, 0xf>(v);     // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4e, 0xf>(v);     // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x124, 0xf>(v);    // row_ror 4
  v += dpp_f64<0x128, 0xf>(v);    // row_ror 8
  v += dpp_f64<0x142, 0xa>(v);    // row_bcast 15 into rows 1 and 3
  v += dpp_f64<0x143, 0xc>(v);    // row_bcast 31 into rows 2 and 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ int wave_or_dpp(int v) {
  v |= dpp_i32<0xb1, 0xf>(v);
  v |= dpp_i32<0x4e, 0xf>(v);
  v |= dpp_i32<0x124, 0xf>(v);
  v |= dpp_i32<0x128, 0xf>(v);
  v |= dpp_i32<0x142, 0xa>(v);
  v |= dpp_i32<0x143, 0xc>(v);
  return __builtin_amdgcn_readlane(v, 63);
}

// Half of a main halo: an elliptical dPIE is the difference of two cored isothermal terms
// (cores s and a), taken as part 0 and part 1 by two threads; any other halo is part 0 whole.
template <bool ENFW>
__device__ __forceinline__ void eval_main_part(const MainRec& r, int part, double px, double py, const Quad& qd,
                                               Acc& acc) {
  if (r.type != T_PJE || r.q >= 1.0) {
    if (part == 0) {
      eval_main<false, ENFW>(r, px, py, qd, acc);
      acc.flags |= r.flags;
    }
    return;
  }
  const double dx = px - r.x, dy = py - r.y;
  if (part == 0) {
    acc.flags |= r.flags;
    if (main_singular(r) && fma(dx, dx, dy * dy) < 1e-24) { acc.flags |= FL_SINGULAR; return; }
  } else if (main_singular(r) && fma(dx, dx, dy * dy) < 1e-24) {
    return;
  }
  const double xp = r.c * dx + r.sn * dy, yp = r.c * dy - r.sn * dx;
  Term<double> p, t;
  esie_prime<false>(xp, yp, r.bqe, r.e, r.q2, part == 0 ? r.s : r.a, p);
  if (part) { p.ax = -p.ax; p.ay = -p.ay; p.h11 = -p.h11; p.h12 = -p.h12; p.h22 = -p.h22; }
  rotate_back<false>(r.c, r.sn, p, t);
  t.t111 = t.t112 = t.t122 = t.t222 = 0.0;
  add<false>(acc, t);
}

// Work items: the main halos' parts (two each), then the members.  With at most 64 main parts
// they take the last wave, one part per lane, and the members are strided over the other
// waves: a wave that held both would run the two code paths one after the other (measured on
// the cluster lens: 2.15 us per evaluation with the parts on the last lanes of a mixed wave).
// Otherwise all items are strided over all threads.  (One call site per halo kind keeps the
// kernel's code, and its registers, small.)
template <bool ENFW>
__device__ void plane_sum_block(const Plane64& P, double x, double y, const Quad& qd, Acc& out, PolRed& R) {
  Acc acc;
  acc.zero();
  constexpr int nt = POL_T, mt = POL_T - 64;
  const int nmem = P.seg.off[NSEG], msl = 2 * P.n_main;
  const int tid = threadIdx.x;
  int first, stride, end;
  if (msl > 64) { first = tid; stride = nt; end = msl + nmem; }
  else if (tid >= mt) { first = tid - mt; stride = nt; end = min(first + 1, msl); }
  else { first = msl + tid; stride = mt; end = msl + nmem; }
  for (int it = first; it < end; it += stride) {
    if (it < msl) eval_main_part<ENFW>(P.mains[it >> 1], it & 1, x, y, qd, acc);
    else member64_term<false, ENFW>(P, it - msl, x, y, qd, acc);
  }
  const double s0 = wave_sum_dpp(acc.ax), s1 = wave_sum_dpp(acc.ay), s2 = wave_sum_dpp(acc.h11),
               s3 = wave_sum_dpp(acc.h12), s4 = wave_sum_dpp(acc.h22);
  const int fl = wave_or_dpp(acc.flags);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    R.v[wv][0] = s0; R.v[wv][1] = s1; R.v[wv][2] = s2; R.v[wv][3] = s3; R.v[wv][4] = s4;
    R.f[wv] = fl;
  }
  __syncthreads();
  double t[5];
  int f = R.f[0];
#pragma unroll
  for (int k = 0; k < 5; ++k) t[k] = R.v[0][k];
#pragma unroll
  for (int q = 1; q < POL_W; ++q) {
#pragma unroll
    for (int k = 0; k < 5; ++k) t[k] += R.v[q][k];
    f |= R.f[q];
  }
  __syncthreads();                      // R is written again by the next evaluation
  out.ax = t[0]; out.ay = t[1]; out.h11 = t[2]; out.h12 = t[3]; out.h22 = t[4];
  out.t111 = out.t112 = out.t122 = out.t222 = 0.0;
  out.flags = f;
}

// MULTI = false compiles the single-plane case alone: the multi-plane recursion's per-plane
// arrays are indexed at run time and would otherwise hold scratch memory and registers in
// every kernel that calls this.
// P0: the lens's first plane (its records possibly in LDS).
template <bool MULTI, bool ENFW>
__device__ void lens_eval64(const LensDev& L, const Plane64& P0, const double* w, double x, double y, double& bx,
                            double& by, double* Aout, int& flags, PolRed& R) {
  if (!MULTI || L.n_planes == 1) {
    Acc acc;
    plane_sum_block<ENFW>(P0, x, y, L.qd, acc, R);
    double a = w[0];
    bx = x - a * acc.ax;
    by = y - a * acc.ay;
    Aout[0] = 1.0 - a * acc.h11; Aout[1] = -a * acc.h12; Aout[2] = -a * acc.h12; Aout[3] = 1.0 - a * acc.h22;
    flags |= acc.flags;
    return;
  }
  const int N = L.n_planes;
  double al[2 * LF_MAX_PLANES], Hm[3 * LF_MAX_PLANES], Am[4 * LF_MAX_PLANES];
  double Bx = x, By = y, F11 = 1, F12 = 0, F21 = 0, F22 = 1;
  for (int j = 0; j < N; ++j) {
    double tx = x, ty = y, A11 = 1, A12 = 0, A21 = 0, A22 = 1;
    for (int i = 0; i < j; ++i) {
      double wi = L.wij[i * LF_MAX_PLANES + j];
      tx -= wi * al[2 * i]; ty -= wi * al[2 * i + 1];
      const double* H = &Hm[3 * i];
      const double* Ai = &Am[4 * i];
      A11 -= wi * (H[0] * Ai[0] + H[1] * Ai[2]); A12 -= wi * (H[0] * Ai[1] + H[1] * Ai[3]);
      A21 -= wi * (H[1] * Ai[0] + H[2] * Ai[2]); A22 -= wi * (H[1] * Ai[1] + H[2] * Ai[3]);
    }
    Acc acc;
    plane_sum_block<ENFW>(L.pl[j], tx, ty, L.qd, acc, R);
    flags |= acc.flags;
    al[2 * j] = acc.ax; al[2 * j + 1] = acc.ay;
    Hm[3 * j] = acc.h11; Hm[3 * j + 1] = acc.h12; Hm[3 * j + 2] = acc.h22;
    Am[4 * j] = A11; Am[4 * j + 1] = A12; Am[4 * j + 2] = A21; Am[4 * j + 3] = A22;
    double wj = w[j];
    if (wj == 0.0) continue;
    Bx -= wj * acc.ax; By -= wj * acc.ay;
    F11 -= wj * (acc.h11 * A11 + acc.h12 * A21); F12 -= wj * (acc.h11 * A12 + acc.h12 * A22);
    F21 -= wj * (acc.h12 * A11 + acc.h22 * A21); F22 -= wj * (acc.h12 * A12 + acc.h22 * A22);
  }
  bx = Bx; by = By;
  Aout[0] = F11; Aout[1] = F12; Aout[2] = F21; Aout[3] = F22;
}

// ---------------------------------------------------------------------------------------
// 2. candidates
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ bool near_tri(const double* B, double sx, double sy, double eps) {
  double mnx = fmin(B[0], fmin(B[2], B[4])) - eps, mxx = fmax(B[0], fmax(B[2], B[4])) + eps;
  double mny = fmin(B[1], fmin(B[3], B[5])) - eps, mxy = fmax(B[1], fmax(B[3], B[5])) + eps;
  if (sx < mnx || sx > mxx || sy < mny || sy > mxy) return false;
  double area = (B[2] - B[0]) * (B[5] - B[1]) - (B[3] - B[1]) * (B[4] - B[0]);
  double e0 = hypot(B[2] - B[0], B[3] - B[1]), e1 = hypot(B[4] - B[2], B[5] - B[3]), e2 = hypot(B[0] - B[4], B[1] - B[5]);
  if (fabs(area) <= eps * (e0 + e1 + e2)) return true;          // nearly degenerate: bbox decides
  double sg = area > 0 ? 1.0 : -1.0;
  double o0 = sg * ((B[2] - B[0]) * (sy - B[1]) - (B[3] - B[1]) * (sx - B[0]));
  double o1 = sg * ((B[4] - B[2]) * (sy - B[3]) - (B[5] - B[3]) * (sx - B[2]));
  double o2 = sg * ((B[0] - B[4]) * (sy - B[5]) - (B[1] - B[5]) * (sx - B[4]));
  return o0 >= -eps * e0 && o1 >= -eps * e1 && o2 >= -eps * e2;
}

// A wave's hits for its source s (low: each lane's triangle or cell code).  FILL = false (the
// candidate pass): appended to the unordered list, counted per source.  FILL = true (the
// second pass after an overflow): written straight into the source's segment, for the sources
// whose segment fits the capacity.
template <bool FILL>
__device__ __forceinline__ void emit_cand(const FindArgs& F, int s, bool hit, unsigned long long low, int lane) {
  const unsigned long long mask = __ballot(hit);
  if (!mask) return;
  if (FILL && F.src_off[s + 1] > F.cap) return;
  const int leader = __ffsll((long long)mask) - 1;
  int base = 0;
  if (lane == leader) {
    const int c = __popcll(mask);
    if (FILL) {
      base = F.src_off[s] + atomicAdd(F.src_cur + s, c);
    } else {
      base = atomicAdd(F.n_cand, c);
      atomicAdd(F.src_cnt + s, c);
    }
  }
  base = __shfl(base, leader, 64);
  if (hit) {
    const int idx = base + __popcll(mask & ((1ull << lane) - 1ull));
    const unsigned long long key = ((unsigned long long)s << 32) | low;
    if (FILL) {
      if (idx < F.src_off[s + 1]) F.cand[idx] = key;   // (the pass finds what the first found)
    } else if (idx < F.cap) {
      F.cand_raw[idx] = key;
    }
  }
}

// Wave minimum and maximum by the lane moves of wave_sum_dpp; lanes of rows a move leaves out
// take the identity (+inf, -inf).
template <int CTRL, int ROWS, int OLD>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(OLD, __float_as_int(v), CTRL, ROWS, 0xf, false));
}
template <bool MAX>
__device__ __forceinline__ float wave_ext(float v) {
  constexpr int ID = MAX ? (int)0xff800000 : 0x7f800000;
  auto op = [](float a, float b) { return MAX ? fmaxf(a, b) : fminf(a, b); };
  v = op(v, dpp_f32<0xb1, 0xf, ID>(v));
  v = op(v, dpp_f32<0x4e, 0xf, ID>(v));
  v = op(v, dpp_f32<0x124, 0xf, ID>(v));
  v = op(v, dpp_f32<0x128, 0xf, ID>(v));
  v = op(v, dpp_f32<0x142, 0xa, ID>(v));
  v = op(v, dpp_f32<0x143, 0xc, ID>(v));
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ float wave_min(float v) { return wave_ext<false>(v); }
__device__ __forceinline__ float wave_max(float v) { return wave_ext<true>(v); }

// A wave takes a tile of FIND_TW x FIND_TH cells (lane l: cell (l % FIND_TW, l / FIND_TW) of
// the tile), a workgroup FIND_WG of them side by side.
constexpr int FIND_TW = 8, FIND_TH = 8, FIND_WG = 4;

// NP = 1..4: that many planes, corners in registers; 0: any count up to LF_MAX_PLANES (the
// corner arrays are then indexed at run time and live in scratch memory).  FILL: the second
// pass after an overflow (returns at once otherwise).
//
// Three FP32 filters narrow the (cell, source) pairs before the FP64 test, each keeping a
// superset of what the next keeps:
//   * per wave, lanes over sources: the source against the box that holds every mapped corner
//     of the wave's tile, theta in [min, max] - sum_p w_p alpha_p in [w_p min, w_p max]
//     (bounds reduced over the tile), widened by twice the bounding-box margin below, which
//     covers the box's own margin and the at most 3 np + 2 further roundings of these bounds;
//   * per lane, the mapped cell centre with a radius (the coarse test);
//   * per lane, the bounding box of the cell's four mapped corners.
// Only the sources that pass the first filter for some lane's tile are taken one by one.
template <int NP, bool FILL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NP == 1 ? 4 : 1))) void k_find_cand(const FindArgs F) {
  constexpr int MP = NP > 0 ? NP : LF_MAX_PLANES;
  const int np = NP > 0 ? NP : F.n_planes;
  if (FILL && F.n_cand[2] == 0) return;
  const int ncx = F.nx - 1, ncy = F.ny - 1;
  const int tiles_x = (ncx + FIND_TW - 1) / FIND_TW, tiles_y = (ncy + FIND_TH - 1) / FIND_TH;
  const long long n_tiles = (long long)tiles_x * tiles_y;
  const long long n_groups = (n_tiles + FIND_WG - 1) / FIND_WG;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (long long g = blockIdx.x; g < n_groups; g += gridDim.x) {
  const long long tile = g * FIND_WG + wv;
  const int ti = (int)(tile % tiles_x), tj = (int)(tile / tiles_x);
  const int ci = ti * FIND_TW + (lane % FIND_TW), cj = tj * FIND_TH + (lane / FIND_TW);
  const bool valid = tile < n_tiles && ci < ncx && cj < ncy;
  const int i = valid ? ci : 0, j = valid ? cj : 0;
  const long long cc = (long long)j * ncx + i;
  const long long v[4] = {(long long)j * F.nx + i, (long long)j * F.nx + i + 1, (long long)(j + 1) * F.nx + i,
                          (long long)(j + 1) * F.nx + i + 1};
  double tx[4], ty[4];
  tx[0] = tx[2] = F.x0 + (i + 0.5) * F.h; tx[1] = tx[3] = F.x0 + (i + 1.5) * F.h;
  ty[0] = ty[1] = F.y0 + (j + 0.5) * F.h; ty[2] = ty[3] = F.y0 + (j + 1.5) * F.h;
  // FP32 copies of the corner deflections for the filters (the FP64 values are read again in
  // the rare case that a source passes them): the bounding-box margin is eps plus a bound on
  // the FP32 rounding (inputs and FMAs, each <= 2^-24 of a magnitude <= R = |theta| +
  // sum w |alpha| + |beta_s|, at most np + 3 of them per coordinate, taken with a factor 4).
  float txf[4], tyf[4], axf[MP][4], ayf[MP][4], amax[MP];
  float tmax = 0.f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    txf[k] = (float)tx[k]; tyf[k] = (float)ty[k];
    tmax = fmaxf(tmax, fmaxf(fabsf(txf[k]), fabsf(tyf[k])));
  }
  for (int p = 0; p < np; ++p) {
    amax[p] = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      axf[p][k] = (float)F.vax[(size_t)F.va_pstride * p + v[k]];
      ayf[p][k] = (float)F.vay[(size_t)F.va_pstride * p + v[k]];
      amax[p] = fmaxf(amax[p], fmaxf(fabsf(axf[p][k]), fabsf(ayf[p][k])));
    }
  }
  const float rel = 4.f * (float)(np + 3) * 5.9604645e-8f;   // 4 (np + 3) 2^-24
  // Coarse test: every mapped corner lies within r_p = h/2 + sum_p |w_p| da_p (in each
  // coordinate) of the mapped centre c - sum_p w_p abar_p, where abar_p is the corners' mean
  // deflection and da_p their largest deviation from it.  The source is kept for the bounding
  // box test below unless it is farther than that plus four times the box's margin from the
  // mapped centre: one margin is the box's own, and the rounding of the centre, the means, the
  // deviations, the radius and the corners adds at most (2 + 7 np) 2^-23 R, within the other
  // three.  So the coarse test keeps a superset of what the box keeps.
  const float cxf = 0.25f * ((txf[0] + txf[1]) + (txf[2] + txf[3]));
  const float cyf = 0.25f * ((tyf[0] + tyf[1]) + (tyf[2] + tyf[3]));
  const float r0 = 0.5f * fmaxf(fabsf(txf[1] - txf[0]), fabsf(tyf[2] - tyf[0]));
  float abx[MP], aby[MP], da[MP];
  for (int p = 0; p < np; ++p) {
    abx[p] = 0.25f * ((axf[p][0] + axf[p][1]) + (axf[p][2] + axf[p][3]));
    aby[p] = 0.25f * ((ayf[p][0] + ayf[p][1]) + (ayf[p][2] + ayf[p][3]));
    da[p] = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) da[p] = fmaxf(da[p], fmaxf(fabsf(axf[p][k] - abx[p]), fabsf(ayf[p][k] - aby[p])));
  }
  // The tile's bounds (invalid lanes take no part); a wave without valid lanes skips the sources.
  const bool any_valid = __any(valid);
  const float INF = __builtin_inff();
  const float Txlo = wave_min(valid ? txf[0] : INF), Txhi = wave_max(valid ? txf[1] : -INF);
  const float Tylo = wave_min(valid ? tyf[0] : INF), Tyhi = wave_max(valid ? tyf[2] : -INF);
  const float Tmax = wave_max(valid ? tmax : 0.f);
  float Axlo[MP], Axhi[MP], Aylo[MP], Ayhi[MP], Amax[MP];
  for (int p = 0; p < np; ++p) {
    const float xl = fminf(fminf(axf[p][0], axf[p][1]), fminf(axf[p][2], axf[p][3]));
    const float xh = fmaxf(fmaxf(axf[p][0], axf[p][1]), fmaxf(axf[p][2], axf[p][3]));
    const float yl = fminf(fminf(ayf[p][0], ayf[p][1]), fminf(ayf[p][2], ayf[p][3]));
    const float yh = fmaxf(fmaxf(ayf[p][0], ayf[p][1]), fmaxf(ayf[p][2], ayf[p][3]));
    Axlo[p] = wave_min(valid ? xl : INF); Axhi[p] = wave_max(valid ? xh : -INF);
    Aylo[p] = wave_min(valid ? yl : INF); Ayhi[p] = wave_max(valid ? yh : -INF);
    Amax[p] = wave_max(valid ? amax[p] : 0.f);
  }
  // The sources are staged in LDS, SCH at a time: read from global memory in the loop, every
  // source would cost each wave a round trip to L2 (the candidate stores keep the compiler
  // from using the scalar cache).
  constexpr int SCH = 256;
  __shared__ double sh_b[2 * SCH], sh_w[SCH * MP];
  for (int s0 = 0; s0 < F.n_src; s0 += SCH) {
    const int ns = min(SCH, F.n_src - s0);
    __syncthreads();
    for (int q = threadIdx.x; q < ns; q += blockDim.x) {
      sh_b[2 * q] = F.beta[2 * (s0 + q)];
      sh_b[2 * q + 1] = F.beta[2 * (s0 + q) + 1];
      for (int p = 0; p < np; ++p) sh_w[q * np + p] = F.w[(s0 + q) * np + p];
    }
    __syncthreads();
    if (!any_valid) continue;
    for (int sb = 0; sb < ns; sb += 64) {
      bool pass = false;
      if (sb + lane < ns) {
        const int q = sb + lane;
        const float sxf = (float)sh_b[2 * q], syf = (float)sh_b[2 * q + 1];
        float lx = Txlo, hx = Txhi, ly = Tylo, hy = Tyhi;
        float R = Tmax + fmaxf(fabsf(sxf), fabsf(syf));
        for (int p = 0; p < np; ++p) {
          const float wf = (float)sh_w[q * np + p];
          const float x1 = wf * Axlo[p], x2 = wf * Axhi[p], y1 = wf * Aylo[p], y2 = wf * Ayhi[p];
          lx -= fmaxf(x1, x2); hx -= fminf(x1, x2);
          ly -= fmaxf(y1, y2); hy -= fminf(y1, y2);
          R = fmaf(fabsf(wf), Amax[p], R);
        }
        const float M = 2.f * ((float)F.eps + rel * R);
        pass = sxf >= lx - M && sxf <= hx + M && syf >= ly - M && syf <= hy + M;
      }
      unsigned long long todo = __ballot(pass);
      while (todo) {
      const int sl = sb + __ffsll((long long)todo) - 1;
      todo &= todo - 1ull;
      const int s = s0 + sl;
      const double* ws = sh_w + sl * np;
      const double sx = sh_b[2 * sl], sy = sh_b[2 * sl + 1];
      {
        const float sxf = (float)sx, syf = (float)sy;
        float R = tmax + fmaxf(fabsf(sxf), fabsf(syf));
        float bcx = cxf, bcy = cyf, rad = r0;
        for (int p = 0; p < np; ++p) {
          const float wf = (float)ws[p];
          R = fmaf(fabsf(wf), amax[p], R);
          bcx = fmaf(-wf, abx[p], bcx);
          bcy = fmaf(-wf, aby[p], bcy);
          rad = fmaf(fabsf(wf), da[p], rad);
        }
        const float lim = rad + 4.f * ((float)F.eps + rel * R);
        if (!__any(valid && fabsf(sxf - bcx) <= lim && fabsf(syf - bcy) <= lim)) continue;
      }
      {
        const float sxf = (float)sx, syf = (float)sy;
        float bxf[4], byf[4];
        float R = tmax + fmaxf(fabsf(sxf), fabsf(syf));
#pragma unroll
        for (int k = 0; k < 4; ++k) { bxf[k] = txf[k]; byf[k] = tyf[k]; }
        for (int p = 0; p < np; ++p) {
          const float wf = (float)ws[p];
          R = fmaf(fabsf(wf), amax[p], R);
#pragma unroll
          for (int k = 0; k < 4; ++k) { bxf[k] = fmaf(-wf, axf[p][k], bxf[k]); byf[k] = fmaf(-wf, ayf[p][k], byf[k]); }
        }
        const float m = (float)F.eps + rel * R;
        const bool in = valid && sxf >= fminf(fminf(bxf[0], bxf[1]), fminf(bxf[2], bxf[3])) - m &&
                        sxf <= fmaxf(fmaxf(bxf[0], bxf[1]), fmaxf(bxf[2], bxf[3])) + m &&
                        syf >= fminf(fminf(byf[0], byf[1]), fminf(byf[2], byf[3])) - m &&
                        syf <= fmaxf(fmaxf(byf[0], byf[1]), fmaxf(byf[2], byf[3])) + m;
        if (!__any(in)) continue;
      }
      double bx[4], by[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) { bx[k] = tx[k]; by[k] = ty[k]; }
      for (int p = 0; p < np; ++p) {
        const double w = ws[p];
        const double* vx = F.vax + (size_t)F.va_pstride * p;
        const double* vy = F.vay + (size_t)F.va_pstride * p;
#pragma unroll
        for (int k = 0; k < 4; ++k) { bx[k] = fma(-w, vx[v[k]], bx[k]); by[k] = fma(-w, vy[v[k]], by[k]); }
      }
      // corners: 0 = v(i,j), 1 = v(i+1,j), 2 = v(i,j+1), 3 = v(i+1,j+1)
      double T0[6] = {bx[0], by[0], bx[1], by[1], bx[3], by[3]};
      double T1[6] = {bx[0], by[0], bx[3], by[3], bx[2], by[2]};
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const bool hit = valid && near_tri(t == 0 ? T0 : T1, sx, sy, F.eps);
        emit_cand<FILL>(F, s, hit, (unsigned long long)(2 * cc + t), lane);
      }
      }
    }
  }
  }
}

// ---------------------------------------------------------------------------------------
// 3. candidates by (source, triangle): per-source segments, each sorted
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_find_reset(const FindArgs F) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < 3) F.n_cand[t] = 0;
  for (int s = t; s < F.n_src; s += gridDim.x * 256) F.src_cnt[s] = 0;
}

// Exclusive prefix sum of the per-source counts (one workgroup; saturating at INT_MAX, where
// nothing fits anyway), the number of candidates kept (all, or those of the sources before
// the first whose segment passes the capacity) and the overflow flag; zeroes the cursors.
__global__ __launch_bounds__(1024) void k_find_scan(const FindArgs F) {
  __shared__ int sh[1024];
  __shared__ long long carry;
  const int tid = threadIdx.x;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int b = 0; b < F.n_src; b += 1024) {
    const int s = b + tid;
    const int v = s < F.n_src ? F.src_cnt[s] : 0;
    sh[tid] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int u = tid >= o ? sh[tid - o] : 0;
      __syncthreads();
      sh[tid] += u;
      __syncthreads();
    }
    const long long excl = carry + sh[tid] - v, incl = excl + v;
    if (s < F.n_src) {
      F.src_off[s] = (int)min(excl, (long long)INT_MAX);
      F.src_cur[s] = 0;
      if (excl <= F.cap && incl > F.cap) F.n_cand[1] = (int)excl;
    }
    __syncthreads();
    if (tid == 1023) carry += sh[1023];
    __syncthreads();
  }
  if (tid == 0) {
    F.src_off[F.n_src] = (int)min(carry, (long long)INT_MAX);
    if (carry <= F.cap) F.n_cand[1] = (int)carry;
    F.n_cand[2] = carry > F.cap ? 1 : 0;
  }
}

// Unordered list -> per-source segments (no overflow; otherwise the second candidate pass
// fills them).
__global__ __launch_bounds__(256) void k_find_scatter(const FindArgs F) {
  if (F.n_cand[2]) return;
  const int n = F.n_cand[0];
  for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) {
    const unsigned long long key = F.cand_raw[k];
    const int s = (int)(key >> 32);
    F.cand[F.src_off[s] + atomicAdd(F.src_cur + s, 1)] = key;
  }
}

// One workgroup per kept source: its segment sorted ascending by a bitonic network in the form
// where every compare-exchange puts the smaller key first (per block of `size`, a mirror step
// then half-cleaners), so a partner past the end is skipped as if it held +infinity and any
// length sorts.  In LDS up to LF_SEG_LDS keys, in place in global memory beyond.
__global__ __launch_bounds__(256) void k_find_segsort(const FindArgs F) {
  __shared__ unsigned long long sk[LF_SEG_LDS];
  const int s = blockIdx.x;
  const int lo = F.src_off[s], hi = F.src_off[s + 1];
  if (hi > F.n_cand[1] || hi - lo < 2) return;
  const int n = hi - lo, tid = threadIdx.x;
  unsigned long long* g = F.cand + lo;
  const bool in_lds = n <= LF_SEG_LDS;
  unsigned long long* a = in_lds ? sk : g;
  if (in_lds)
    for (int k = tid; k < n; k += 256) sk[k] = g[k];
  __syncthreads();
  int m = 1;
  while (m < n) m <<= 1;
  for (int size = 2; size <= m; size <<= 1) {
    for (int k = tid; k < m; k += 256) {
      const int l = k ^ (size - 1);
      if (l > k && l < n) {
        const unsigned long long x = a[k], y = a[l];
        if (y < x) { a[k] = y; a[l] = x; }
      }
    }
    __syncthreads();
    for (int stride = size >> 2; stride > 0; stride >>= 1) {
      for (int k = tid; k < m; k += 256) {
        const int l = k ^ stride;
        if (l > k && l < n) {
          const unsigned long long x = a[k], y = a[l];
          if (y < x) { a[k] = y; a[l] = x; }
        }
      }
      __syncthreads();
    }
  }
  if (in_lds)
    for (int k = tid; k < n; k += 256) g[k] = sk[k];
}

// ---------------------------------------------------------------------------------------
// 4. FP64 containment + Newton polish per candidate
// ---------------------------------------------------------------------------------------
// The first plane of the lens; with CACHE its halo records copied to LDS and read from there.
template <bool CACHE>
__device__ __forceinline__ Plane64 polish_plane(const LensDev& L) {
  Plane64 P = L.pl[0];
  if constexpr (CACHE) {
    __shared__ MainRec sm_main[POL_LDS_MAIN];
    __shared__ MemRec64 sm_mem[POL_LDS_MEM];
    const int nmem = P.seg.off[NSEG];
    for (int i = threadIdx.x; i < P.n_main; i += blockDim.x) sm_main[i] = P.mains[i];
    for (int i = threadIdx.x; i < nmem; i += blockDim.x) sm_mem[i] = P.mem[i];
    __syncthreads();
    P.mains = sm_main;
    P.mem = sm_mem;
  }
  return P;
}

template <bool MULTI, bool ENFW, bool CACHE>
__global__ __launch_bounds__(POL_T) __attribute__((amdgpu_waves_per_eu(2))) void k_find_polish(const FindArgs F, const LensDev L) {
  __shared__ PolRed R;
  const Plane64 P0 = polish_plane<CACHE>(L);
  const int n = F.n_cand[1];
  for (int k = blockIdx.x; k < n; k += gridDim.x) {   // one workgroup per candidate
  unsigned long long key = F.cand[k];
  int s = (int)(key >> 32);
  long long tri = (long long)(key & 0xffffffffull);
  long long cell = tri >> 1;
  int t = (int)(tri & 1);
  int i = (int)(cell % (F.nx - 1)), j = (int)(cell / (F.nx - 1));
  // vertex (i,j), then (i+1,j),(i+1,j+1) for t = 0; (i+1,j+1),(i,j+1) for t = 1
  int vi[3] = {i, t == 0 ? i + 1 : i + 1, t == 0 ? i + 1 : i};
  int vj[3] = {j, t == 0 ? j : j + 1, j + 1};
  const double* w = F.w + (size_t)s * F.n_planes;
  double B[6], T[6], A[4];
  int fl = 0;
  for (int q = 0; q < 3; ++q) {
    T[2 * q] = F.x0 + (vi[q] + 0.5) * F.h;
    T[2 * q + 1] = F.y0 + (vj[q] + 0.5) * F.h;
    lens_eval64<MULTI, ENFW>(L, P0, w, T[2 * q], T[2 * q + 1], B[2 * q], B[2 * q + 1], A, fl, R);
  }
  const double sx = F.beta[2 * s], sy = F.beta[2 * s + 1];
  int status = 4;
  double tx = 0, ty = 0, mu = 0;
  if (d_tri_contains(B, sx, sy)) {
    double area = (B[2] - B[0]) * (B[5] - B[1]) - (B[3] - B[1]) * (B[4] - B[0]);
    double l1 = ((B[4] - B[2]) * (sy - B[3]) - (B[5] - B[3]) * (sx - B[2])) / area;
    double l2 = ((B[0] - B[4]) * (sy - B[5]) - (B[1] - B[5]) * (sx - B[4])) / area;
    double l3 = 1.0 - l1 - l2;
    double tx0 = l1 * T[0] + l2 * T[2] + l3 * T[4], ty0 = l1 * T[1] + l2 * T[3] + l3 * T[5];
    tx = tx0; ty = ty0;
    bool conv = false;
    for (int it = 0; it <= 30; ++it) {
      double ex, ey;
      lens_eval64<MULTI, ENFW>(L, P0, w, tx, ty, ex, ey, A, fl, R);
      double rx = sx - ex, ry = sy - ey;
      if (fabs(rx) < 1e-10 && fabs(ry) < 1e-10) { conv = true; break; }
      if (it == 30) break;
      double det = A[0] * A[3] - A[1] * A[2];
      tx += (A[3] * rx - A[1] * ry) / det;
      ty += (-A[2] * rx + A[0] * ry) / det;
    }
    mu = 1.0 / (A[0] * A[3] - A[1] * A[2]);
    if (!conv) status = 1;
    else if (fabs(tx - tx0) > 2.0 * F.h || fabs(ty - ty0) > 2.0 * F.h) status = 2;
    else status = 0;
  }
  if (threadIdx.x == 0) {
    F.c_status[k] = status;
    F.c_theta[2 * k] = tx;
    F.c_theta[2 * k + 1] = ty;
    F.c_mu[k] = mu;
  }
  }
}

// ---------------------------------------------------------------------------------------
// 5. per source: merge duplicates in candidate order, write outputs
// ---------------------------------------------------------------------------------------
// A source whose candidates were not kept (past the capacity) gets count 0 and FL_OVERFLOW.
// One wave per source.  Up to 64 candidates, lane j holds the source's candidate j: candidate
// k is a duplicate when an earlier candidate that was kept lies within 1e-6"; the candidates
// are settled in order (each by then knows whether the earlier ones were kept, read from their
// lanes), and the kept ones are written in candidate order.  More candidates take the same
// rule in one lane.
__device__ __forceinline__ double lane_f64(double v, int q) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, q), hi = __builtin_amdgcn_readlane((int)(b >> 32), q);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__global__ __launch_bounds__(64) void k_find_final(const FindArgs F) {
  const int s = blockIdx.x, lane = threadIdx.x;
  const int lo = F.src_off[s], hi = F.src_off[s + 1];
  if (hi > F.n_cand[1]) {
    if (lane == 0) {
      F.count_out[s] = 0;
      if (F.flags_out) F.flags_out[s] = FL_OVERFLOW;
    }
    return;
  }
  const int n = hi - lo;
  if (n <= 64) {
    const bool in = lane < n;
    const int k = lo + (in ? lane : 0);
    bool keep = in && F.c_status[k] == 0;
    const double tx = in ? F.c_theta[2 * k] : 0.0, ty = in ? F.c_theta[2 * k + 1] : 0.0;
    bool merged = false;
    for (int q = 0; q < n - 1; ++q) {
      if (!(__ballot(keep) >> q & 1ull)) continue;
      const double qx = lane_f64(tx, q), qy = lane_f64(ty, q);
      const double dx = tx - qx, dy = ty - qy;
      if (keep && lane > q && sqrt(dx * dx + dy * dy) < 1e-6) { keep = false; merged = true; }
    }
    if (merged) F.c_status[k] = 3;
    const unsigned long long km = __ballot(keep);
    const int rank = __popcll(km & ((1ull << lane) - 1ull)), cnt = __popcll(km);
    if (keep && rank < F.max_img) {
      F.theta_out[((size_t)s * F.max_img + rank) * 2] = tx;
      F.theta_out[((size_t)s * F.max_img + rank) * 2 + 1] = ty;
      if (F.mu_out) F.mu_out[(size_t)s * F.max_img + rank] = F.c_mu[k];
    }
    const int fl = (__ballot(merged) ? FL_MERGED : 0) | (cnt > F.max_img ? FL_OVERFLOW : 0);
    if (lane == 0) {
      F.count_out[s] = cnt;
      if (F.flags_out) F.flags_out[s] = fl;
    }
    return;
  }
  if (lane != 0) return;
  int cnt = 0, fl = 0;
  for (int k = lo; k < hi; ++k) {
    if (F.c_status[k] != 0) continue;
    double tx = F.c_theta[2 * k], ty = F.c_theta[2 * k + 1];
    bool dup = false;
    for (int q = lo; q < k; ++q) {
      if (F.c_status[q] != 0) continue;
      double dx = tx - F.c_theta[2 * q], dy = ty - F.c_theta[2 * q + 1];
      if (sqrt(dx * dx + dy * dy) < 1e-6) { dup = true; break; }
    }
    if (dup) { F.c_status[k] = 3; fl |= FL_MERGED; continue; }
    if (cnt < F.max_img) {
      F.theta_out[((size_t)s * F.max_img + cnt) * 2] = tx;
      F.theta_out[((size_t)s * F.max_img + cnt) * 2 + 1] = ty;
      if (F.mu_out) F.mu_out[(size_t)s * F.max_img + cnt] = F.c_mu[k];
    } else {
      fl |= FL_OVERFLOW;
    }
    ++cnt;
  }
  F.count_out[s] = cnt;
  if (F.flags_out) F.flags_out[s] = fl;
}

// The polishing passes' variant for a lens: the LDS copy of the halo records for a small
// single-plane lens.
static bool polish_cache(const LensDev& L) {
  return L.n_planes == 1 && L.pl[0].n_main <= POL_LDS_MAIN && L.pl[0].seg.off[NSEG] <= POL_LDS_MEM;
}
#define LF_POLISH_LAUNCH(KERNEL, ...)                                                                         \
  do {                                                                                                        \
    const bool cache = polish_cache(L);                                                                       \
    const dim3 pgrid((unsigned)min(F.cap, 16 * F.n_cu)), pblock((unsigned)POL_T);                            \
    if (F.n_planes == 1) {                                                                                    \
      if (L.enfw) {                                                                                           \
        if (cache) hipLaunchKernelGGL((KERNEL<false, true, true>), pgrid, pblock, 0, st, __VA_ARGS__);     \
        else hipLaunchKernelGGL((KERNEL<false, true, false>), pgrid, pblock, 0, st, __VA_ARGS__);             \
      } else {                                                                                                \
        if (cache) hipLaunchKernelGGL((KERNEL<false, false, true>), pgrid, pblock, 0, st, __VA_ARGS__);    \
        else hipLaunchKernelGGL((KERNEL<false, false, false>), pgrid, pblock, 0, st, __VA_ARGS__);            \
      }                                                                                                       \
    } else {                                                                                                  \
      if (L.enfw) hipLaunchKernelGGL((KERNEL<true, true, false>), pgrid, pblock, 0, st, __VA_ARGS__);         \
      else hipLaunchKernelGGL((KERNEL<true, false, false>), pgrid, pblock, 0, st, __VA_ARGS__);               \
    }                                                                                                         \
  } while (0)

// prefix sum and, without overflow, the scatter into segments
static void launch_segments(const FindArgs& F, hipStream_t st) {
  hipLaunchKernelGGL(k_find_scan, dim3(1), dim3(1024), 0, st, F);
  hipLaunchKernelGGL(k_find_scatter, dim3((unsigned)max(1, min(4 * F.n_cu, (F.cap + 255) / 256))), dim3(256), 0,
                     st, F);
}

hipError_t launch_find(const FindArgs& F, const LensDev& L, hipStream_t st, void (*mark)(void*, const char*, int),
                       void* ctx) {
  hipLaunchKernelGGL(k_find_reset, dim3((unsigned)min(1024, (F.n_src + 255) / 256 + 1)), dim3(256), 0, st, F);
  mark(ctx, "find_cand", 0);
  const long long n_tiles = (long long)((F.nx - 1 + FIND_TW - 1) / FIND_TW) * ((F.ny - 1 + FIND_TH - 1) / FIND_TH);
  const long long n_groups = (n_tiles + FIND_WG - 1) / FIND_WG;
  const dim3 cgrid((unsigned)(n_groups < (1LL << 30) ? n_groups : (1LL << 30))), fgrid((unsigned)(4 * F.n_cu));
  switch (F.n_planes) {
    case 1: hipLaunchKernelGGL((k_find_cand<1, false>), cgrid, dim3(256), 0, st, F); break;
    case 2: hipLaunchKernelGGL((k_find_cand<2, false>), cgrid, dim3(256), 0, st, F); break;
    case 3: hipLaunchKernelGGL((k_find_cand<3, false>), cgrid, dim3(256), 0, st, F); break;
    case 4: hipLaunchKernelGGL((k_find_cand<4, false>), cgrid, dim3(256), 0, st, F); break;
    default: hipLaunchKernelGGL((k_find_cand<0, false>), cgrid, dim3(256), 0, st, F); break;
  }
  mark(ctx, "find_cand", 1);
  launch_segments(F, st);
  switch (F.n_planes) {
    case 1: hipLaunchKernelGGL((k_find_cand<1, true>), fgrid, dim3(256), 0, st, F); break;
    case 2: hipLaunchKernelGGL((k_find_cand<2, true>), fgrid, dim3(256), 0, st, F); break;
    case 3: hipLaunchKernelGGL((k_find_cand<3, true>), fgrid, dim3(256), 0, st, F); break;
    case 4: hipLaunchKernelGGL((k_find_cand<4, true>), fgrid, dim3(256), 0, st, F); break;
    default: hipLaunchKernelGGL((k_find_cand<0, true>), fgrid, dim3(256), 0, st, F); break;
  }
  hipLaunchKernelGGL(k_find_segsort, dim3((unsigned)F.n_src), dim3(256), 0, st, F);
  mark(ctx, "find_polish", 0);
  LF_POLISH_LAUNCH(k_find_polish, F, L);
  mark(ctx, "find_polish", 1);
  hipLaunchKernelGGL(k_find_final, dim3((unsigned)F.n_src), dim3(64), 0, st, F);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Contour-intersection finder (Sec. 2.3): zero contours of f = beta - theta + a alpha (both
// components) by marching squares, images at the exact intersections of pairs of segments.
// Per cell (corners c0 = (i,j), c1 = (i+1,j), c2 = (i+1,j+1), c3 = (i,j+1); loop edges bottom
// c0-c1, right c1-c2, top c3-c2, left c0-c3; zero counts as positive): two sign changes of a
// component give one segment between the linear-interpolation points, four are paired by the
// asymptotic decider of the bilinear interpolant.  Candidates (source, cell, pair = f1 segment
// * 2 + f2 segment) are sorted like the triangle finder's and take the same final pass.
// ---------------------------------------------------------------------------------------
namespace {
struct MsCell {
  double F1[4], F2[4];
};
// The corners of cell (i, j) in the order of the cell values: positions and deflections.
struct MsCorners {
  double tx[4], ty[4], ax[4], ay[4];
};
__device__ void ms_corners(const FindArgs& F, int i, int j, MsCorners& q) {
#pragma clang fp contract(off)
  const int ci[4] = {i, i + 1, i + 1, i}, cj[4] = {j, j, j + 1, j + 1};
  for (int k = 0; k < 4; ++k) {
    const long long v = (long long)cj[k] * F.nx + ci[k];
    q.tx[k] = F.x0 + (ci[k] + 0.5) * F.h;
    q.ty[k] = F.y0 + (cj[k] + 0.5) * F.h;
    q.ax[k] = F.vax[v];
    q.ay[k] = F.vay[v];
  }
}
// F = beta_s - (theta - a alpha) at the corners, for source (sx, sy) at distance ratio a
__device__ void ms_cell_values(const MsCorners& q, double sx, double sy, double a, MsCell& c) {
#pragma clang fp contract(off)
  for (int k = 0; k < 4; ++k) {
    c.F1[k] = sx - (q.tx[k] - a * q.ax[k]);
    c.F2[k] = sy - (q.ty[k] - a * q.ay[k]);
  }
}
// segments of one component in cell coordinates: seg[k] = (x0, y0, x1, y1); returns 0, 1 or 2
__device__ int ms_segments(const double* Fv, double seg[2][4]) {
#pragma clang fp contract(off)
  const double px[4] = {0.0, 1.0, 1.0, 0.0}, py[4] = {0.0, 0.0, 1.0, 1.0};
  const int ea[4] = {0, 1, 3, 0}, eb[4] = {1, 2, 2, 3};
  double X[4][2];
  bool has[4];
  int n = 0;
  for (int m = 0; m < 4; ++m) {
    const double fa = Fv[ea[m]], fb = Fv[eb[m]];
    has[m] = (fa < 0) != (fb < 0);
    X[m][0] = X[m][1] = 0.0;
    if (has[m]) {
      const double t = fa / (fa - fb);
      X[m][0] = px[ea[m]] + t * (px[eb[m]] - px[ea[m]]);
      X[m][1] = py[ea[m]] + t * (py[eb[m]] - py[ea[m]]);
      ++n;
    }
  }
  auto put = [&](int k, int a, int b) {
    seg[k][0] = X[a][0]; seg[k][1] = X[a][1]; seg[k][2] = X[b][0]; seg[k][3] = X[b][1];
  };
  if (n == 2) {
    int a = -1, b = -1;
    for (int m = 0; m < 4; ++m)
      if (has[m]) { if (a < 0) a = m; else b = m; }
    put(0, a, b);
    return 1;
  }
  if (n == 4) {
    const double D = Fv[0] + Fv[2] - Fv[1] - Fv[3];
    const bool cpos = D == 0.0 ? true : !((Fv[0] * Fv[2] - Fv[1] * Fv[3]) / D < 0);
    if (cpos == !(Fv[0] < 0)) { put(0, 0, 1); put(1, 2, 3); }
    else { put(0, 0, 3); put(1, 1, 2); }
    return 2;
  }
  return 0;
}
// intersection of f1 segment p with f2 segment q; false if they do not cross
__device__ bool ms_cross(const double S1[2][4], int p, const double S2[2][4], int q, double& xi, double& eta) {
#pragma clang fp contract(off)
  const double d1x = S1[p][2] - S1[p][0], d1y = S1[p][3] - S1[p][1];
  const double d2x = S2[q][2] - S2[q][0], d2y = S2[q][3] - S2[q][1];
  const double wx = S2[q][0] - S1[p][0], wy = S2[q][1] - S1[p][1];
  const double den = d1x * d2y - d1y * d2x;
  if (den == 0.0) return false;
  const double tp = (wx * d2y - wy * d2x) / den, tq = (wx * d1y - wy * d1x) / den;
  if (!(tp >= 0 && tp <= 1 && tq >= 0 && tq <= 1)) return false;
  xi = S1[p][0] + tp * d1x;
  eta = S1[p][1] + tp * d1y;
  return true;
}
}  // namespace

template <bool FILL>
__global__ __launch_bounds__(256) void k_ms_cand(const FindArgs F) {
  if (FILL && F.n_cand[2] == 0) return;
  const long long ncell = (long long)(F.nx - 1) * (F.ny - 1);
  for (long long cb = (long long)blockIdx.x * 256; cb < ncell; cb += (long long)gridDim.x * 256) {
  const long long c = cb + threadIdx.x;
  const bool valid = c < ncell;
  const long long cc = valid ? c : 0;
  const int i = (int)(cc % (F.nx - 1)), j = (int)(cc / (F.nx - 1));
  const int lane = threadIdx.x & 63;
  MsCorners cq;
  ms_corners(F, i, j, cq);
  // sources staged in LDS, SCH at a time (see k_find_cand)
  constexpr int SCH = 256;
  __shared__ double sh_s[3 * SCH];
  for (int s0 = 0; s0 < F.n_src; s0 += SCH) {
    const int ns = min(SCH, F.n_src - s0);
    __syncthreads();
    for (int q = threadIdx.x; q < ns; q += blockDim.x) {
      sh_s[3 * q] = F.beta[2 * (s0 + q)];
      sh_s[3 * q + 1] = F.beta[2 * (s0 + q) + 1];
      sh_s[3 * q + 2] = F.w[s0 + q];
    }
    __syncthreads();
    for (int sl = 0; sl < ns; ++sl) {
      const int s = s0 + sl;
      MsCell v;
      ms_cell_values(cq, sh_s[3 * sl], sh_s[3 * sl + 1], sh_s[3 * sl + 2], v);
      int pairs = 0;          // bit p * 2 + q: f1 segment p crosses f2 segment q
      if (valid) {
        double S1[2][4], S2[2][4];
        const int n1 = ms_segments(v.F1, S1);
        if (n1) {
          const int n2 = ms_segments(v.F2, S2);
          for (int p = 0; p < n1; ++p)
            for (int q = 0; q < n2; ++q) {
              double xi, eta;
              if (ms_cross(S1, p, S2, q, xi, eta)) pairs |= 1 << (p * 2 + q);
            }
        }
      }
      if (!__any(pairs != 0)) continue;
      for (int k = 0; k < 4; ++k) emit_cand<FILL>(F, s, (pairs >> k) & 1, (unsigned long long)(cc * 4 + k), lane);
    }
  }
  }
}

// one workgroup per candidate: the intersection, then (polish) FP64 Newton as the triangle finder
template <bool MULTI, bool ENFW, bool CACHE>
__global__ __launch_bounds__(POL_T) __attribute__((amdgpu_waves_per_eu(2))) void k_ms_point(const FindArgs F, const LensDev L, int polish) {
  __shared__ PolRed R;
  const Plane64 P0 = polish_plane<CACHE>(L);
  const int n = F.n_cand[1];
  for (int k = blockIdx.x; k < n; k += gridDim.x) {
  const unsigned long long key = F.cand[k];
  const int s = (int)(key >> 32);
  const long long low = (long long)(key & 0xffffffffull), cell = low >> 2;
  const int pair = (int)(low & 3), p = pair >> 1, q = pair & 1;
  const int i = (int)(cell % (F.nx - 1)), j = (int)(cell / (F.nx - 1));
  MsCorners cq;
  ms_corners(F, i, j, cq);
  MsCell v;
  ms_cell_values(cq, F.beta[2 * s], F.beta[2 * s + 1], F.w[s], v);
  double S1[2][4], S2[2][4], xi = 0.0, eta = 0.0;
  ms_segments(v.F1, S1);
  ms_segments(v.F2, S2);
  ms_cross(S1, p, S2, q, xi, eta);
  double tx, ty;
  {
#pragma clang fp contract(off)
    tx = F.x0 + (i + 0.5) * F.h + F.h * xi;
    ty = F.y0 + (j + 0.5) * F.h + F.h * eta;
  }
  const double* w = F.w + s;
  const double sx = F.beta[2 * s], sy = F.beta[2 * s + 1];
  double A[4], ex, ey;
  int fl = 0, status = 0;
  if (polish) {
    const double tx0 = tx, ty0 = ty;
    bool conv = false;
    for (int it = 0; it <= 30; ++it) {
      lens_eval64<MULTI, ENFW>(L, P0, w, tx, ty, ex, ey, A, fl, R);
      const double rx = sx - ex, ry = sy - ey;
      if (fabs(rx) < 1e-10 && fabs(ry) < 1e-10) { conv = true; break; }
      if (it == 30) break;
      const double det = A[0] * A[3] - A[1] * A[2];
      tx += (A[3] * rx - A[1] * ry) / det;
      ty += (-A[2] * rx + A[0] * ry) / det;
    }
    if (!conv) status = 1;
    else if (fabs(tx - tx0) > 2.0 * F.h || fabs(ty - ty0) > 2.0 * F.h) status = 2;
  } else {
    lens_eval64<MULTI, ENFW>(L, P0, w, tx, ty, ex, ey, A, fl, R);
  }
  if (threadIdx.x == 0) {
    F.c_status[k] = status;
    F.c_theta[2 * k] = tx;
    F.c_theta[2 * k + 1] = ty;
    F.c_mu[k] = 1.0 / (A[0] * A[3] - A[1] * A[2]);
  }
  }
}

hipError_t launch_find_ms(const FindArgs& F, const LensDev& L, int polish, hipStream_t st,
                          void (*mark)(void*, const char*, int), void* ctx) {
  const long long ncell = (long long)(F.nx - 1) * (F.ny - 1);
  hipLaunchKernelGGL(k_find_reset, dim3((unsigned)min(1024, (F.n_src + 255) / 256 + 1)), dim3(256), 0, st, F);
  mark(ctx, "find_ms_cand", 0);
  hipLaunchKernelGGL(k_ms_cand<false>, dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, st, F);
  mark(ctx, "find_ms_cand", 1);
  launch_segments(F, st);
  hipLaunchKernelGGL(k_ms_cand<true>, dim3((unsigned)(4 * F.n_cu)), dim3(256), 0, st, F);
  hipLaunchKernelGGL(k_find_segsort, dim3((unsigned)F.n_src), dim3(256), 0, st, F);
  mark(ctx, "find_ms_point", 0);
  LF_POLISH_LAUNCH(k_ms_point, F, L, polish);
  mark(ctx, "find_ms_point", 1);
  hipLaunchKernelGGL(k_find_final, dim3((unsigned)F.n_src), dim3(64), 0, st, F);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Multi-plane passes: theta_j of every point, and the final recursion (Sec. 2.2).
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mp_theta(const MPArgs M, int j) {
  long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= M.P) return;
  double x, y;
  if (M.grid) {
    long long jj = p / M.nx, ii = p - jj * M.nx;
    x = M.x0 + ((double)ii + 0.5) * M.h;
    y = M.y0 + ((double)jj + 0.5) * M.h;
  } else {
    x = M.px[p];
    y = M.py[p];
  }
  for (int i = 0; i < j; ++i) {
    double w = M.wij[i * LF_MAX_PLANES + j];
    x -= w * M.al[(size_t)(5 * i) * M.P + p];
    y -= w * M.al[(size_t)(5 * i + 1) * M.P + p];
  }
  M.tx[p] = x;
  M.ty[p] = y;
}

// Final pass of the multi-plane trace: per ray, the plane Jacobians A_j (recursion of Sec. 2.2)
// and, per source redshift, beta and A.  NP > 0: the ray's 5 NP plane values are loaded into
// registers once (independent loads, issued together) and reused for every source redshift;
// NP = 0: any number of planes, values read where used.
template <int NP>
__global__ __launch_bounds__(256) void k_mp_final(const MPArgs M) {
  long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= M.P) return;
  double x, y;
  if (M.grid) {
    long long jj = p / M.nx, ii = p - jj * M.nx;
    x = M.x0 + ((double)ii + 0.5) * M.h;
    y = M.y0 + ((double)jj + 0.5) * M.h;
  } else {
    x = M.px[p];
    y = M.py[p];
  }
  constexpr int MP = NP > 0 ? NP : LF_MAX_PLANES;
  const int N = NP > 0 ? NP : M.n_planes;
  const double* __restrict__ al = M.al;
  double v[NP > 0 ? 5 * NP : 1];
  if constexpr (NP > 0) {
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int c = 0; c < 5; ++c) v[5 * j + c] = al[(size_t)(5 * j + c) * M.P + p];
  }
  auto val = [&](int j, int c) -> double {
    if constexpr (NP > 0) return v[5 * j + c];
    else return al[(size_t)(5 * j + c) * M.P + p];
  };
  double Am[4 * MP];
#pragma unroll
  for (int j = 0; j < MP; ++j) {
    if (j >= N) break;
    double A11 = 1, A12 = 0, A21 = 0, A22 = 1;
#pragma unroll
    for (int i = 0; i < MP; ++i) {
      if (i >= j) break;
      const double w = M.wij[i * LF_MAX_PLANES + j];
      const double h11 = val(i, 2), h12 = val(i, 3), h22 = val(i, 4);
      const double* Ai = &Am[4 * i];
      A11 -= w * (h11 * Ai[0] + h12 * Ai[2]); A12 -= w * (h11 * Ai[1] + h12 * Ai[3]);
      A21 -= w * (h12 * Ai[0] + h22 * Ai[2]); A22 -= w * (h12 * Ai[1] + h22 * Ai[3]);
    }
    Am[4 * j] = A11; Am[4 * j + 1] = A12; Am[4 * j + 2] = A21; Am[4 * j + 3] = A22;
  }
  for (int k = 0; k < M.n_zs; ++k) {
    double bx = x, by = y, F11 = 1, F12 = 0, F21 = 0, F22 = 1;
#pragma unroll
    for (int j = 0; j < MP; ++j) {
      if (j >= N) break;
      const double w = M.wjs[(size_t)k * LF_MAX_PLANES + j];
      if (w == 0.0) continue;
      const double ax = val(j, 0), ay = val(j, 1), h11 = val(j, 2), h12 = val(j, 3), h22 = val(j, 4);
      bx -= w * ax; by -= w * ay;
      const double* Aj = &Am[4 * j];
      F11 -= w * (h11 * Aj[0] + h12 * Aj[2]); F12 -= w * (h11 * Aj[1] + h12 * Aj[3]);
      F21 -= w * (h12 * Aj[0] + h22 * Aj[2]); F22 -= w * (h12 * Aj[1] + h22 * Aj[3]);
    }
    size_t o = (size_t)k * M.P + p;
    if (M.beta) { M.beta[2 * o] = bx; M.beta[2 * o + 1] = by; }
    if (M.A) { M.A[4 * o] = F11; M.A[4 * o + 1] = F12; M.A[4 * o + 2] = F21; M.A[4 * o + 3] = F22; }
    if (M.mu) M.mu[o] = 1.0 / (F11 * F22 - F12 * F21);
  }
}

hipError_t launch_mp_theta(const MPArgs& M, int j, hipStream_t st) {
  hipLaunchKernelGGL(k_mp_theta, dim3((unsigned)((M.P + 255) / 256)), dim3(256), 0, st, M, j);
  return hipGetLastError();
}
hipError_t launch_mp_final(const MPArgs& M, hipStream_t st) {
  const dim3 g((unsigned)((M.P + 255) / 256)), b(256);
  switch (M.n_planes) {
    case 1: hipLaunchKernelGGL(k_mp_final<1>, g, b, 0, st, M); break;
    case 2: hipLaunchKernelGGL(k_mp_final<2>, g, b, 0, st, M); break;
    case 3: hipLaunchKernelGGL(k_mp_final<3>, g, b, 0, st, M); break;
    case 4: hipLaunchKernelGGL(k_mp_final<4>, g, b, 0, st, M); break;
    default: hipLaunchKernelGGL(k_mp_final<0>, g, b, 0, st, M); break;
  }
  return hipGetLastError();
}

}  // namespace lf
