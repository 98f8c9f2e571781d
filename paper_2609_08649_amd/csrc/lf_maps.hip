// Halo-table expansion (parametric model -> per-sample halo records) and the halo-sum maps
// kernel (deflection, Hessian, third derivatives and their epilogue fields).
//
// Layout: one lane owns PPL points (strided by the block size so stores coalesce);
// halo records are wave-uniform, so the compiler fetches them through the scalar
// data cache into SGPRs (s_load) and every VALU instruction of the profile maths
// reads them as scalar operands: no LDS staging and no VGPRs spent on halo data.
// Member galaxies are sorted by profile segment; each segment is one branch-free loop.
#include <hip/hip_runtime.h>

#include "lf_device.h"
#include "lf_launch.h"
#include "lf_segs.h"

namespace lf {

static constexpr double C_KMS = 299792.458;
static constexpr double ARCSEC = 206264.80624709636;
static constexpr double PI_D = 3.14159265358979323846;

__device__ double xf_apply(int xf, double raw, const XfConst& k) {
  switch (xf) {
    case 1: { double r = raw / C_KMS; return 4.0 * PI_D * r * r * ARCSEC; }    // sigma -> b
    case 2: return raw * k.arcsec_per_kpc;                                      // kpc -> arcsec
    case 3: return (1.0 - raw) / (1.0 + raw);                                   // eps -> q
    case 4: return raw * (PI_D / 180.0);                                        // deg -> rad
    default: return raw;
  }
}

__device__ double bound_raw(const Bind& b, const double* row, int n_free, int* bad) {
  if (b.kind == 0) return b.value;
  if (b.index < 0 || b.index >= n_free) { *bad = 1; return 0.0; }
  return row[b.index];
}

__global__ void k_expand(const DevModel m, const double* __restrict__ params, int S,
                         MainRec* __restrict__ mains, MulRec* __restrict__ muls,
                         MemRec32* __restrict__ m32, MemRec64* __restrict__ m64) {
  const int s = blockIdx.y;
  const double* row = params ? params + (size_t)s * m.n_free : nullptr;
  // thread t < n_main: main component t; thread == n_main: multipliers; rest: members
  const int per_sample = m.n_main + 1 + ((m32 || m64) ? m.n_mem : 0);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < per_sample; t += gridDim.x * blockDim.x) {
    if (t < m.n_main) {
      const MainDesc& d = m.main[t];
      int bad = 0;
      double f[7];
      int xfs[7];
      for (int k = 0; k < 7; ++k) {
        double raw = bound_raw(d.f[k], row, m.n_free, &bad);
        xfs[k] = d.f[k].xf;
        f[k] = (xfs[k] == 5 || xfs[k] == 6) ? raw : xf_apply(xfs[k], raw, m.xc);
      }
      if (xfs[2] == 5 && xfs[5] == 6) {     // (M200, c200) -> (kappa_s, r_s)
        double m200 = f[2], c = f[5];
        double r200 = cbrt(3.0 * m200 / (4.0 * PI_D * 200.0 * m.xc.rho_c));
        double rs = r200 / c;
        double dc = (200.0 / 3.0) * c * c * c / (log1p(c) - c / (1.0 + c));
        f[2] = dc * m.xc.rho_c * rs / m.xc.sigma_cr;
        f[5] = rs / m.xc.Dd * ARCSEC;
      }
      MainRec r;
      r.type = d.type;
      r.x = f[0]; r.y = f[1]; r.b = f[2]; r.q = f[3]; r.s = f[5]; r.a = f[6];
      double sn, c;
      sincos(f[4], &sn, &c);
      r.c = c; r.sn = sn;
      r.q2 = r.q * r.q;
      r.e = sqrt(fmax(0.0, 1.0 - r.q2));
      r.bqe = r.e > 0 ? r.b * r.q / r.e : 0.0;
      r.pad = 0.0;
      bool ok = !bad;
      for (int k = 0; k < 7; ++k) ok = ok && isfinite(f[k]);
      ok = ok && r.q > 0.0 && r.q <= 1.0 && r.b >= 0.0 && r.s >= 0.0;
      if (d.type == T_PJE) ok = ok && r.a > r.s;
      if (d.type == T_NFW || d.type == T_ENFW) ok = ok && r.s > 0.0;
      r.flags = ok ? 0 : FL_INVALID;
      r.pad0 = r.pad1 = 0;
      mains[(size_t)s * m.n_main + t] = r;
    } else if (t == m.n_main) {
      int bad = 0;
      MulRec u;
      u.b = xf_apply(m.mul[0].xf, bound_raw(m.mul[0], row, m.n_free, &bad), m.xc);
      u.s = xf_apply(m.mul[1].xf, bound_raw(m.mul[1], row, m.n_free, &bad), m.xc);
      u.a = xf_apply(m.mul[2].xf, bound_raw(m.mul[2], row, m.n_free, &bad), m.xc);
      bool ok = !bad && isfinite(u.b) && isfinite(u.s) && isfinite(u.a) && u.b >= 0 && u.s >= 0 && u.a >= 0;
      u.flags = ok ? 0 : FL_INVALID;
      u.pad = 0;
      muls[s] = u;
    } else {
      int i = t - m.n_main - 1;
      // the multipliers are recomputed here (cheap) so that this thread has no dependence
      int bad = 0;
      double bm = xf_apply(m.mul[0].xf, bound_raw(m.mul[0], row, m.n_free, &bad), m.xc);
      double sm = xf_apply(m.mul[1].xf, bound_raw(m.mul[1], row, m.n_free, &bad), m.xc);
      double am = xf_apply(m.mul[2].xf, bound_raw(m.mul[2], row, m.n_free, &bad), m.xc);
      const MemCat& c = m.mem[i];
      double b = bm * c.fb, sc = sm * c.fs, a = am * c.fa;
      double q2 = c.q * c.q, e = sqrt(fmax(0.0, 1.0 - q2));
      double bqe = e > 0 ? b * c.q / e : 0.0;
      const double bd = b * (a - sc), apls = a + sc;
      if (m64) {
        MemRec64 r;
        r.x = c.x; r.y = c.y; r.b = b; r.s = sc; r.a = a; r.s2 = sc * sc; r.a2 = a * a;
        r.c = c.c; r.sn = c.sn; r.q2 = q2; r.e = e; r.bqe = bqe; r.bd = bd; r.apls = apls;
        m64[(size_t)s * m.n_mem + i] = r;
      }
      if (m32) {
        MemRec32 r;
        r.xh = (float)c.x; r.xl = (float)(c.x - (double)r.xh);
        r.yh = (float)c.y; r.yl = (float)(c.y - (double)r.yh);
        r.b = (float)b; r.s = (float)sc; r.a = (float)a;
        r.s2 = (float)(sc * sc); r.a2 = (float)(a * a);
        r.c = (float)c.c; r.sn = (float)c.sn; r.q2 = (float)q2; r.e = (float)e; r.bqe = (float)bqe;
        r.bd = (float)bd; r.apls = (float)apls;
        const double rn = NEAR_K * b / c.q;
        r.rn2 = (float)fmax(rn * rn, 1e-12);
        r.pad0 = r.pad1 = r.pad2 = 0.f;
        // far-field expansion of the circular dPIE b (1/(R_s + s) - 1/(R_a + a)): with t = 1/r,
        // 1/(R_c + c) = t (sqrt(1 + c^2 t^2) - c t) = t (1 - c t + sum_k beta_k (c t)^(2k)),
        // beta_k = binom(1/2, k), so m = b (a - s) t^2 + sum_k b beta_k (s^2k - a^2k) t^(2k+1) and
        // w = 2 dm/d(r^2) = -t^3 dm/dt
        const double beta[6] = {0.0, 0.5, -0.125, 0.0625, -0.0390625, 0.02734375};
        const bool far_ok = a <= FAR_AMAX;
        double sp = 1.0, ap = 1.0;
        for (int k = 0; k < 6; ++k) {
          double mk = 0.0;
          if (k == 0) mk = b * (a - sc);
          else {
            sp *= sc * sc;
            ap *= a * a;
            mk = b * beta[k] * (sp - ap);
          }
          r.fm[k] = far_ok ? (float)mk : 0.f;
          r.fw[k] = far_ok ? (float)(-(2 * k + 1 + (k == 0)) * mk) : 0.f;
        }
        m32[(size_t)s * m.n_mem + i] = r;
        const MemSoA v = mem_soa(m32, S, m.n_mem, s);
        v.x[i] = c.x; v.y[i] = c.y; v.a[i] = a; v.rn2[i] = r.rn2;
        for (int k = 0; k < 6; ++k) v.fm[k * v.pad + i] = r.fm[k];
      }
    }
  }
}

hipError_t launch_expand(const DevModel& m, const double* params, int S, MainRec* mains,
                         MulRec* muls, MemRec32* m32, MemRec64* m64, hipStream_t st) {
  int per = m.n_main + 1 + ((m32 || m64) ? m.n_mem : 0);
  dim3 grid((per + 255) / 256, S);
  hipLaunchKernelGGL(k_expand, grid, dim3(256), 0, st, m, params, S, mains, muls, m32, m64);
  return hipGetLastError();
}

struct MapsArgs {
  DevModel m;
  const MainRec* mains;
  const MemRec32* m32;
  const MemRec64* m64;
  int S;
  PointsSpec pts;
  double a;
  MapsOut out;
  Quad qd;
  double* part;        // partial sums of the heavy pass: [S][NPART][P] (null = none)
};
static constexpr int NPART = 9;

__device__ __forceinline__ void point_of(const PointsSpec& ps, long long p, double& x, double& y) {
  if (ps.grid) {
    long long q = p + ps.p0;
    long long j = q / ps.nx, i = q - j * ps.nx;
    x = ps.x0 + ((double)i + 0.5) * ps.h;
    y = ps.y0 + ((double)j + 0.5) * ps.h;
  } else {
    x = ps.px[p];
    y = ps.py[p];
  }
}

// Fused epilogue (Sec. 2.1; Sec. 6 fields with third derivatives) and the requested planes of
// one point.
template <bool D3>
__device__ __forceinline__ void store_point(const MapsArgs& A, size_t idx, double x, double y, const Acc& acc) {
  const MapsOut& o = A.out;
  Epi e;
  epilogue<D3>(x, y, A.a, acc, e);
  if (o.ax) o.ax[idx] = acc.ax;
  if (o.ay) o.ay[idx] = acc.ay;
  if (o.p11) o.p11[idx] = acc.h11;
  if (o.p12) o.p12[idx] = acc.h12;
  if (o.p22) o.p22[idx] = acc.h22;
  if (o.kappa) o.kappa[idx] = e.kappa;
  if (o.g1) o.g1[idx] = e.g1;
  if (o.g2) o.g2[idx] = e.g2;
  if (o.detA) o.detA[idx] = e.detA;
  if (o.mu) o.mu[idx] = e.mu;
  if (o.bx) o.bx[idx] = e.bx;
  if (o.by) o.by[idx] = e.by;
  if (o.e1) o.e1[idx] = e.e1;
  if (o.e2) o.e2[idx] = e.e2;
  if (D3) {
    if (o.t111) o.t111[idx] = acc.t111;
    if (o.t112) o.t112[idx] = acc.t112;
    if (o.t122) o.t122[idx] = acc.t122;
    if (o.t222) o.t222[idx] = acc.t222;
    if (o.f1) o.f1[idx] = e.f1;
    if (o.f2) o.f2[idx] = e.f2;
  }
  if (o.flags) o.flags[idx] = e.flags;
}

// Heavy pass: main components (FP64) and the rare member segments (elliptical, point,
// NFW) whose closed forms need many registers; writes partial sums per point.
// KIND: 0 = any model; 1 = no elliptical NFW; 2 = main components only (no rare member
// segments) and no elliptical NFW -- variants for the common cluster model, which then needs
// fewer registers (more waves per SIMD hide the FP64 latency).
template <bool MIXED, bool D3, int KIND>
__global__ __launch_bounds__(256) void k_heavy(const MapsArgs A) {
  constexpr bool ENFW = KIND == 0, RARE = KIND < 2;
  const int s = blockIdx.y;
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long P = A.pts.P;
  if (p >= P) return;
  double px[1], py[1];
  Acc acc[1];
  point_of(A.pts, p, px[0], py[0]);
  acc[0].zero();
  const MainRec* mr = A.mains + (size_t)s * A.m.n_main;
  for (int c = 0; c < A.m.n_main; ++c) {
    const MainRec r = mr[c];
    eval_main<D3, ENFW, true>(r, px[0], py[0], A.qd, acc[0]);
    acc[0].flags |= r.flags;
  }
  const SegOff& so = A.m.seg;
  const size_t mo = (size_t)s * A.m.n_mem;
  if (!RARE) {
  } else if (MIXED) {
    seg_loop<SEG_EPJE, D3, 1>(A.m32 + mo, A.m64 + mo, so.off[SEG_EPJE], so.off[SEG_EPJE + 1], px, py, acc, A.qd);
    seg_loop<SEG_ESIE, D3, 1>(A.m32 + mo, A.m64 + mo, so.off[SEG_ESIE], so.off[SEG_ESIE + 1], px, py, acc, A.qd);
    seg_loop<SEG_POINT, D3, 1>(A.m32 + mo, A.m64 + mo, so.off[SEG_POINT], so.off[SEG_POINT + 1], px, py, acc, A.qd);
  } else {
    seg_loop<SEG_EPJE, D3, 1>(A.m64 + mo, nullptr, so.off[SEG_EPJE], so.off[SEG_EPJE + 1], px, py, acc, A.qd);
    seg_loop<SEG_ESIE, D3, 1>(A.m64 + mo, nullptr, so.off[SEG_ESIE], so.off[SEG_ESIE + 1], px, py, acc, A.qd);
    seg_loop<SEG_POINT, D3, 1>(A.m64 + mo, nullptr, so.off[SEG_POINT], so.off[SEG_POINT + 1], px, py, acc, A.qd);
  }
  if constexpr (RARE)
    seg_loop<SEG_NFW, D3, 1>(A.m64 + mo, nullptr, so.off[SEG_NFW], so.off[SEG_NFW + 1], px, py, acc, A.qd);
  if constexpr (ENFW)
    seg_loop<SEG_ENFW, D3, 1>(A.m64 + mo, nullptr, so.off[SEG_ENFW], so.off[SEG_ENFW + 1], px, py, acc, A.qd);
  double* q = A.part + (size_t)s * NPART * P + p;
  q[0] = acc[0].ax; q[P] = acc[0].ay; q[2 * P] = acc[0].h11; q[3 * P] = acc[0].h12; q[4 * P] = acc[0].h22;
  if (D3) { q[5 * P] = acc[0].t111; q[6 * P] = acc[0].t112; q[7 * P] = acc[0].t122; q[8 * P] = acc[0].t222; }
  ((int*)(A.part + (size_t)A.S * NPART * P))[(size_t)s * P + p] = acc[0].flags;
}

// Lean pass: circular cored / dPIE members (the bulk of a cluster) + fused epilogue.
template <bool MIXED, bool D3, int PPL>
__global__ __launch_bounds__(256) void k_maps(const MapsArgs A) {
  const int s = blockIdx.y;
  const long long base = (long long)blockIdx.x * (256 * PPL) + threadIdx.x;
  const long long P = A.pts.P;
  double px[PPL], py[PPL];
  Acc acc[PPL];
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    long long p = base + (long long)k * 256;
    if (p >= P) p = P - 1;            // duplicate the last point; its store is masked below
    point_of(A.pts, p, px[k], py[k]);
    acc[k].zero();
    if (A.part) {
      const double* q = A.part + (size_t)s * NPART * P + p;
      acc[k].ax = q[0]; acc[k].ay = q[P]; acc[k].h11 = q[2 * P]; acc[k].h12 = q[3 * P]; acc[k].h22 = q[4 * P];
      if (D3) { acc[k].t111 = q[5 * P]; acc[k].t112 = q[6 * P]; acc[k].t122 = q[7 * P]; acc[k].t222 = q[8 * P]; }
      acc[k].flags = ((const int*)(A.part + (size_t)A.S * NPART * P))[(size_t)s * P + p];
    }
  }
  const SegOff& so = A.m.seg;
  const size_t mo = (size_t)s * A.m.n_mem;
  if (MIXED) {
    seg_loop<SEG_CPJE, D3, PPL>(A.m32 + mo, A.m64 + mo, so.off[SEG_CPJE], so.off[SEG_CPJE + 1], px, py, acc, A.qd);
    seg_loop<SEG_CSIE, D3, PPL>(A.m32 + mo, A.m64 + mo, so.off[SEG_CSIE], so.off[SEG_CSIE + 1], px, py, acc, A.qd);
  } else {
    seg_loop<SEG_CPJE, D3, PPL>(A.m64 + mo, nullptr, so.off[SEG_CPJE], so.off[SEG_CPJE + 1], px, py, acc, A.qd);
    seg_loop<SEG_CSIE, D3, PPL>(A.m64 + mo, nullptr, so.off[SEG_CSIE], so.off[SEG_CSIE + 1], px, py, acc, A.qd);
  }
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    long long p = base + (long long)k * 256;
    if (p >= P) break;
    store_point<D3>(A, (size_t)s * P + p, px[k], py[k], acc[k]);
  }
}

// Lean pass over a grid in MIXED precision: one wave per TILE_W x (TILE_H TP) block of the
// global grid (seg_loop_tile; a lane holds TP points of one column, TILE_H rows apart), the
// blocks covering the grid rows of the points [p0, p0 + P).  Lanes' points outside those points
// (or past the last column) take part in the member loops but store nothing.
// Without third derivatives four points per lane (16 x 16 blocks) at 3 waves per SIMD: most
// members go through the block's local expansion, whose per-member work is per block, so larger
// blocks amortise it (measured 11% faster than two points per lane at 4 waves, and than four
// points at 4 waves, which spills); with third derivatives two points per lane at 3 waves (each
// LDS record read serves both; faster than one point per lane at 4-7 waves).
template <bool D3>
static constexpr int MAPS_TP = D3 ? 2 : 4;

template <bool D3>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_maps_tile(const MapsArgs A) {
  constexpr int TP = MAPS_TP<D3>, TH = TILE_H * TP;
  __shared__ float dsh[4][64 * TILE_LSTRIDE<SEG_CPJE, D3>];
  const int s = blockIdx.y;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const PointsSpec& ps = A.pts;
  const long long nx = ps.nx, P = ps.P;
  const long long tiles_x = (nx + TILE_W - 1) / TILE_W;
  const long long t = (long long)blockIdx.x * 4 + wave;
  const long long tr = (ps.p0 / nx) / TH + t / tiles_x, tc = t % tiles_x;
  const long long i = tc * TILE_W + lane % TILE_W;
  bool active[TP], any = false;
  long long p[TP];
  TileLane<TP> L;
  L.X = ps.x0 + (double)(tc * TILE_W + TILE_W / 2) * ps.h;
  L.Y = ps.y0 + (double)(tr * TH + TH / 2) * ps.h;
  L.u = (float)(((double)(lane % TILE_W) - 0.5 * (TILE_W - 1)) * ps.h);
  L.hwx = 0.5 * (TILE_W - 1) * ps.h * (1.0 + 1e-6);
  L.hwy = 0.5 * (TH - 1) * ps.h * (1.0 + 1e-6);
  L.px = ps.x0 + ((double)i + 0.5) * ps.h;
  L.dsh = dsh[wave];
#pragma unroll
  for (int k = 0; k < TP; ++k) {
    const long long jr = lane / TILE_W + k * TILE_H, j = tr * TH + jr;
    const long long q = j * nx + i;
    active[k] = i < nx && q >= ps.p0 && q < ps.p0 + P;
    any = any || active[k];
    p[k] = active[k] ? q - ps.p0 : 0;
    L.v[k] = (float)(((double)jr - 0.5 * (TH - 1)) * ps.h);
    L.py[k] = ps.y0 + ((double)j + 0.5) * ps.h;
  }
  if (__ballot(any) == 0) return;           // a whole block outside the call's points
  Acc acc[TP];
#pragma unroll
  for (int k = 0; k < TP; ++k) {
    acc[k].zero();
    if (A.part) {
      const double* pq = A.part + (size_t)s * NPART * P + p[k];
      acc[k].ax = pq[0]; acc[k].ay = pq[P]; acc[k].h11 = pq[2 * P]; acc[k].h12 = pq[3 * P]; acc[k].h22 = pq[4 * P];
      if (D3) { acc[k].t111 = pq[5 * P]; acc[k].t112 = pq[6 * P]; acc[k].t122 = pq[7 * P]; acc[k].t222 = pq[8 * P]; }
      acc[k].flags = ((const int*)(A.part + (size_t)A.S * NPART * P))[(size_t)s * P + p[k]];
    }
  }
  const SegOff& so = A.m.seg;
  const size_t mo = (size_t)s * A.m.n_mem;
  const MemSoA sa = mem_soa(A.m32, A.S, A.m.n_mem, s);
  seg_loop_tile<SEG_CPJE, D3, TP>(A.m32 + mo, A.m64 + mo, sa, so.off[SEG_CPJE], so.off[SEG_CPJE + 1], L, acc, A.qd);
  seg_loop_tile<SEG_CSIE, D3, TP>(A.m32 + mo, A.m64 + mo, sa, so.off[SEG_CSIE], so.off[SEG_CSIE + 1], L, acc, A.qd);
#pragma unroll
  for (int k = 0; k < TP; ++k)
    if (active[k]) store_point<D3>(A, (size_t)s * P + p[k], L.px, L.py[k], acc[k]);
}

template <bool MIXED, bool D3, int PPL>
static void launch_maps_t(const MapsArgs& a, int which, hipStream_t st) {
  if (which == 1) {
    dim3 g1((unsigned)((a.pts.P + 255) / 256), a.S);
    if (a.m.has_enfw) hipLaunchKernelGGL((k_heavy<MIXED, D3, 0>), g1, dim3(256), 0, st, a);
    else if (a.m.has_rare) hipLaunchKernelGGL((k_heavy<MIXED, D3, 1>), g1, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_heavy<MIXED, D3, 2>), g1, dim3(256), 0, st, a);
    return;
  }
  if (MIXED && a.pts.grid) {
    const long long TH = TILE_H * MAPS_TP<D3>;
    const long long nx = a.pts.nx, tiles_x = (nx + TILE_W - 1) / TILE_W;
    const long long tr0 = (a.pts.p0 / nx) / TH, tr1 = ((a.pts.p0 + a.pts.P - 1) / nx) / TH;
    const long long tiles = tiles_x * (tr1 - tr0 + 1);
    dim3 grid((unsigned)((tiles + 3) / 4), a.S);
    hipLaunchKernelGGL((k_maps_tile<D3>), grid, dim3(256), 0, st, a);
    return;
  }
  long long per_block = 256LL * PPL;
  dim3 grid((unsigned)((a.pts.P + per_block - 1) / per_block), a.S);
  hipLaunchKernelGGL((k_maps<MIXED, D3, PPL>), grid, dim3(256), 0, st, a);
}

hipError_t launch_maps(const DevModel& m, const MainRec* mains, const MemRec32* m32,
                       const MemRec64* m64, int S, const PointsSpec& pts, double a_dis,
                       bool mixed, bool d3, const MapsOut& out, const QuadTab& q, int ppl,
                       double* part, int which, hipStream_t st) {
  MapsArgs a;
  a.part = part;
  a.m = m; a.mains = mains; a.m32 = m32; a.m64 = m64; a.S = S; a.pts = pts; a.a = a_dis;
  a.out = out; a.qd.n = q.n; a.qd.u = q.u; a.qd.w = q.w;
#define LF_DISPATCH(MX, D, P)                 \
  if (mixed == MX && d3 == D && ppl == P) {   \
    launch_maps_t<MX, D, P>(a, which, st);    \
    return hipGetLastError();                 \
  }
  LF_DISPATCH(true, false, 1) LF_DISPATCH(false, false, 1) LF_DISPATCH(true, true, 1) LF_DISPATCH(false, true, 1)
#undef LF_DISPATCH
  return hipErrorInvalidValue;
}

}  // namespace lf
