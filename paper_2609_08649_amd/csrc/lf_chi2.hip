// chi^2 per parameter sample (Sec. 3.1 Eq. chi2_src / chi2_img, Sec. 3.5 Newton).
//
// Lanes run over the flattened (image, sample) pairs, sample fastest, so a wave is fully used
// whatever the number of images and mostly holds one image under many samples; member records
// stay wave-uniform (one model per launch) and each lane scales them by its own sample's
// multipliers (b*, s*, a*).  Family and sample reductions run
// one wave per sample: a lane per family sums its images in order, a shuffle tree sums the
// families -- a fixed order, so results are bit-reproducible and independent of batch mates.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lf_chi2.h"
#include "lf_device.h"

namespace lf {

// g indexes the per-(sample, image) buffers sample-major: g = s * n_img + i.
__device__ __forceinline__ void lane_point(const Chi2Args& A, long long g, int& s, int& i, double& x, double& y) {
  s = (int)(g / A.n_img);
  i = (int)(g - (long long)s * A.n_img);
  x = A.th[2 * i];
  y = A.th[2 * i + 1];
}
// Threads run over (image, sample) pairs with the sample fastest: the lanes of a wave hold
// the same observed image under up to 64 parameter samples, so they share the point, the
// member offsets and the near-field decisions (no divergence), and converge alike in Newton.
__device__ __forceinline__ long long lane_slot(const Chi2Args& A, long long t) {
  const long long i = t / A.S, s = t - i * A.S;
  return s * A.n_img + i;
}

// One catalog member scaled by the lane's multipliers, FP64; false on a singular centre.
// D3: third derivatives too.
template <int SEG, bool D3 = false>
__device__ __forceinline__ bool cat_term(const MemCat& c, double dx, double dy, double bm, double sm, double am,
                                         const Quad& qd, Term<double>& t) {
  using T = double;
  T b = bm * c.fb, s = sm * c.fs, a = am * c.fa;
  t.t111 = t.t112 = t.t122 = t.t222 = (T)0;
  if constexpr (SEG == SEG_CPJE || SEG == SEG_CSIE) {
    T r2 = fma(dx, dx, dy * dy);
    if (s == (T)0 && r2 < (T)1e-24) return false;
    T m, w, p = 0;
    if constexpr (SEG == SEG_CPJE) pje_mw<D3>(b, s, a, s * s, a * a, b * (a - s), a + s, r2, m, w, p);
    else cored_mw<D3>(b, s, s * s, r2, m, w, p);
    radial<D3>(dx, dy, m, w, p, t);
  } else if constexpr (SEG == SEG_EPJE || SEG == SEG_ESIE) {
    if (s == (T)0 && dx == (T)0 && dy == (T)0) return false;
    T q2 = c.q * c.q;
    T e = sqrt((T)1 - q2);
    epje<D3>(dx, dy, c.c, c.sn, b * c.q / e, e, q2, s, a, SEG == SEG_EPJE, t);
  } else if constexpr (SEG == SEG_POINT) {
    if (dx == (T)0 && dy == (T)0) return false;
    point_mass<D3>(dx, dy, b, t);
  } else if constexpr (SEG == SEG_NFW) {
    if (dx == (T)0 && dy == (T)0) return false;
    nfw_circ<D3>(dx, dy, b, s, t);
  } else {
    if (dx == (T)0 && dy == (T)0) return false;
    double xp = c.c * dx + c.sn * dy, yp = c.c * dy - c.sn * dx;
    Term<double> pr;
    enfw_prime<D3>(xp, yp, b, s, c.q, qd, pr);
    rotate_back<D3>(c.c, c.sn, pr, t);
  }
  return true;
}

// Potential of one catalog member scaled by the lane's multipliers, FP64 (0 on a singular
// centre).
template <int SEG>
__device__ __forceinline__ double cat_pot(const MemCat& c, double dx, double dy, double bm, double sm, double am,
                                          const Quad& qd) {
  const double b = bm * c.fb, s = sm * c.fs, a = am * c.fa, r2 = fma(dx, dx, dy * dy);
  if constexpr (SEG == SEG_CPJE || SEG == SEG_CSIE || SEG == SEG_EPJE || SEG == SEG_ESIE) {
    if (s == 0.0 && r2 < 1e-24) return 0.0;
  } else {
    if (r2 < 1e-24) return 0.0;
  }
  if constexpr (SEG == SEG_CPJE) return pot_cpje(b, s, a, r2);
  else if constexpr (SEG == SEG_CSIE) return pot_cored(b, s, r2);
  else if constexpr (SEG == SEG_POINT) return b * b * 0.5 * log(r2);
  else if constexpr (SEG == SEG_NFW) return pot_nfw(r2, b, s);
  else {
    const double xp = c.c * dx + c.sn * dy, yp = c.c * dy - c.sn * dx;
    if constexpr (SEG == SEG_ENFW) return pot_enfw(xp, yp, b, s, c.q, qd);
    const double q2 = c.q * c.q, e = sqrt(1.0 - q2), bqe = b * c.q / e;
    double v = pot_esie(xp, yp, bqe, e, q2, s);
    if constexpr (SEG == SEG_EPJE) v -= pot_esie(xp, yp, bqe, e, q2, a);
    return v;
  }
}

// Member segment loop with per-lane multipliers, FP64 (MemCat, every segment).
template <int SEG>
__device__ __forceinline__ void seg_ls(const MemCat* __restrict__ cat, int lo, int hi, double px, double py,
                                       double bm, double sm, double am, Acc& acc, const Quad& qd) {
  for (int h = lo; h < hi; ++h) {
    const MemCat c = cat[h];
    Term<double> t;
    if (cat_term<SEG>(c, px - c.x, py - c.y, bm, sm, am, qd, t)) add<false>(acc, t);
    else acc.flags |= FL_SINGULAR;
  }
}

// The bulk circular segments in FP32 (MemCat32): offsets from FP32 pairs, terms summed in
// FP32 over runs of 16 members and each run added to the FP64 accumulators (the same scheme
// as the maps kernels).  A member closer than its near-field radius (NEAR_K b / q) is
// evaluated from the FP64 catalog instead; its FP32 term is taken at r^2 = 1e24 (dPIE) or 1e30
// (cored isothermal), where it is below 1e-14.
template <int SEG>
__device__ __forceinline__ void seg_ls32(const MemCat32* __restrict__ cat, const MemCat* __restrict__ cat64,
                                         int lo, int hi, double px, double py, const MulRec& u, Acc& acc,
                                         const Quad& qd) {
  static_assert(SEG == SEG_CPJE || SEG == SEG_CSIE, "FP32 catalog path covers the circular segments");
  constexpr int CHUNK = 16;
  const float bm = (float)u.b, sm_ = (float)u.s, am = (float)u.a;
  const float bm2 = bm * bm;
  float xh = (float)px, xl = (float)(px - (double)xh);
  float yh = (float)py, yl = (float)(py - (double)yh);
  for (int h0 = lo; h0 < hi; h0 += CHUNK) {
    const int h1 = min(h0 + CHUNK, hi);
    float sx = 0.f, sy = 0.f, sm = 0.f, s11 = 0.f, s12 = 0.f, s22 = 0.f;
    for (int h = h0; h < h1; ++h) {
      const MemCat32 c = cat[h];
      float dx = (xh - c.xh) + (xl - c.xl), dy = (yh - c.yh) + (yl - c.yl);
      float b = bm * c.fb, s = sm_ * c.fs;
      float r2 = fmaf(dx, dx, dy * dy);
      const bool nr = r2 < fmaxf(bm2 * c.fbk2, 1e-12f);   // also catches r = 0 for b = 0
      if (nr) r2 = SEG == SEG_CPJE ? 1e24f : 1e30f;   // far enough for a term below 1e-14
      float m, w, p = 0.f;
      if constexpr (SEG == SEG_CPJE) {
        float a = am * c.fa;
        pje_mw<false>(b, s, a, s * s, a * a, b * (a - s), a + s, r2, m, w, p);
      } else {
        cored_mw<false>(b, s, s * s, r2, m, w, p);
      }
      // psi_ij = sum(m) delta_ij + sum(w x_i x_j), alpha_i = sum(m x_i)
      sx = fmaf(m, dx, sx); sy = fmaf(m, dy, sy); sm += m;
      float wx = w * dx, wy = w * dy;
      s11 = fmaf(wx, dx, s11); s12 = fmaf(wx, dy, s12); s22 = fmaf(wy, dy, s22);
      if (nr) {
        const MemCat q = cat64[h];
        Term<double> t;
        if (cat_term<SEG>(q, px - q.x, py - q.y, u.b, u.s, u.a, qd, t)) add<false>(acc, t);
        else acc.flags |= FL_SINGULAR;
      }
    }
    const double md = (double)sm;
    acc.ax += (double)sx; acc.ay += (double)sy;
    acc.h11 += md + (double)s11; acc.h12 += (double)s12; acc.h22 += md + (double)s22;
  }
}

__device__ __forceinline__ void rare_members(const Chi2Args& A, double x, double y, const MulRec& u, Acc& acc) {
  const SegOff& so = A.m.seg;
  seg_ls<SEG_EPJE>(A.m.mem, so.off[SEG_EPJE], so.off[SEG_EPJE + 1], x, y, u.b, u.s, u.a, acc, A.qd);
  seg_ls<SEG_ESIE>(A.m.mem, so.off[SEG_ESIE], so.off[SEG_ESIE + 1], x, y, u.b, u.s, u.a, acc, A.qd);
  seg_ls<SEG_POINT>(A.m.mem, so.off[SEG_POINT], so.off[SEG_POINT + 1], x, y, u.b, u.s, u.a, acc, A.qd);
  seg_ls<SEG_NFW>(A.m.mem, so.off[SEG_NFW], so.off[SEG_NFW + 1], x, y, u.b, u.s, u.a, acc, A.qd);
  seg_ls<SEG_ENFW>(A.m.mem, so.off[SEG_ENFW], so.off[SEG_ENFW + 1], x, y, u.b, u.s, u.a, acc, A.qd);
}

// The circular (bulk) segments, or the k-th of K equal member sub-ranges of each of them.
template <bool MIXED>
__device__ __forceinline__ void bulk_members(const Chi2Args& A, double x, double y, const MulRec& u, Acc& acc,
                                             int k = 0, int K = 1) {
  const SegOff& so = A.m.seg;
  auto part = [&](int sg, int& a, int& b) {
    const int lo = so.off[sg], n = so.off[sg + 1] - lo;
    a = lo + (int)((long long)n * k / K);
    b = lo + (int)((long long)n * (k + 1) / K);
  };
  int a0, b0, a1, b1;
  part(SEG_CPJE, a0, b0);
  part(SEG_CSIE, a1, b1);
  if (MIXED) {
    seg_ls32<SEG_CPJE>(A.cat32, A.m.mem, a0, b0, x, y, u, acc, A.qd);
    seg_ls32<SEG_CSIE>(A.cat32, A.m.mem, a1, b1, x, y, u, acc, A.qd);
  } else {
    seg_ls<SEG_CPJE>(A.m.mem, a0, b0, x, y, u.b, u.s, u.a, acc, A.qd);
    seg_ls<SEG_CSIE>(A.m.mem, a1, b1, x, y, u.b, u.s, u.a, acc, A.qd);
  }
}

// Heavy pass: main components (FP64) + rare member segments -> partial sums.
__device__ void chi2_heavy_lane(const Chi2Args& A, long long g) {
  int s, i;
  double x, y;
  lane_point(A, g, s, i, x, y);
  Acc acc;
  acc.zero();
  const MainRec* mr = A.mains + (size_t)s * A.m.n_main;
  for (int c = 0; c < A.m.n_main; ++c) {
    const MainRec r = mr[c];
    eval_main<false, true, true>(r, x, y, A.qd, acc);
    acc.flags |= r.flags;
  }
  const MulRec u = A.muls[s];
  acc.flags |= u.flags;
  rare_members(A, x, y, u, acc);
  double* q = A.part + (size_t)g * 5;
  q[0] = acc.ax; q[1] = acc.ay; q[2] = acc.h11; q[3] = acc.h12; q[4] = acc.h22;
  A.pflags[g] = acc.flags;
}
__global__ __launch_bounds__(256) void k_chi2_heavy(const Chi2Args A) {
  long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= (long long)A.S * A.n_img) return;
  chi2_heavy_lane(A, lane_slot(A, t));
}

// Lean pass: circular members (the bulk), added to the partial sums.  One workgroup takes 64
// (image, sample) threads; each image's members are split into CHI2_SPLIT equal sub-ranges
// per segment and its W waves take sub-ranges k = wave, wave + W, ... (a wave's loop bounds
// stay uniform, so member records remain scalar loads).  At one lane per image the pass is
// latency-bound (a 1024 x 150 batch fills only ~2 waves per SIMD); the split multiplies the
// waves by CHI2_SPLIT.  Sub-range sums meet in LDS and are added to the partial sums in the
// order k = 0, 1, 2, 3 whatever W is, so an image's result never depends on the launch shape,
// tile or batch.
static constexpr int CHI2_SPLIT = 4;

template <bool MIXED>
__device__ void chi2_lean_group(const Chi2Args& A, long long u0, long long u_end) {
  __shared__ double red[CHI2_SPLIT][5][64];
  __shared__ int redf[CHI2_SPLIT][64];
  // wave index made explicitly uniform, so that the member loops' bounds are scalar
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int W = blockDim.x >> 6;
  const long long u = u0 + lane;
  const bool active = u < u_end;
  const long long g = lane_slot(A, active ? u : u_end - 1);
  int s, i;
  double x, y;
  lane_point(A, g, s, i, x, y);
  const MulRec mr = A.muls[s];
  for (int k = wave; k < CHI2_SPLIT; k += W) {
    Acc acc;
    acc.zero();
    bulk_members<MIXED>(A, x, y, mr, acc, k, CHI2_SPLIT);
    red[k][0][lane] = acc.ax; red[k][1][lane] = acc.ay; red[k][2][lane] = acc.h11;
    red[k][3][lane] = acc.h12; red[k][4][lane] = acc.h22; redf[k][lane] = acc.flags;
  }
  __syncthreads();
  if (wave == 0 && active) {
    double* q = A.part + (size_t)g * 5;
    int fl = 0;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      double t = red[0][c][lane];
#pragma unroll
      for (int k = 1; k < CHI2_SPLIT; ++k) t += red[k][c][lane];
      q[c] += t;
    }
#pragma unroll
    for (int k = 0; k < CHI2_SPLIT; ++k) fl |= redf[k][lane];
    A.pflags[g] |= fl;
  }
  __syncthreads();
}
template <bool MIXED>
__global__ __launch_bounds__(256) void k_chi2_lean(const Chi2Args A) {
  chi2_lean_group<MIXED>(A, (long long)blockIdx.x * 64, (long long)A.S * A.n_img);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_or(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v |= __shfl_xor(v, o, 64);
  return v;
}

// Source-plane chi^2: one wave per sample.  Per image: beta_obs = theta - a_f alpha,
// mu = A^-1, W = mu^T S^-1 mu; per family: G = sum W, g = sum W beta_obs, beta_model =
// G^-1 g; chi^2 = sum (beta_obs - beta_model)^T W (beta_obs - beta_model).
// ---------------------------------------------------------------------------------------
// Flux and time-delay terms (Sec. 3.2 Eq. chi2_flux, msrc; Sec. 3.3 Eq. chi2_td, dt0,
// td_approx), FP64 in both precisions.  The observables pass evaluates, per (image, sample),
// the potential, psi_ij and the third derivatives at theta_obs (WHICH = 0) or the potential
// and psi_ij at the accepted image-plane model image (WHICH = 1).  ENFW = false compiles the
// elliptical NFW quadrature out (models without such halos; far fewer registers).
// ---------------------------------------------------------------------------------------
template <bool D3, bool ENFW>
__device__ void obs_sums(const Chi2Args& A, int s, double x, double y, bool want_pot, Acc& acc, double& pot) {
  acc.zero();
  pot = 0.0;
  const MainRec* mr = A.mains + (size_t)s * A.m.n_main;
  for (int c = 0; c < A.m.n_main; ++c) {
    const MainRec r = mr[c];
    eval_main<D3, ENFW>(r, x, y, A.qd, acc);
    if (want_pot) pot += pot_main(r, x, y, A.qd);
  }
  const MulRec u = A.muls[s];
  const SegOff& so = A.m.seg;
  auto seg = [&](auto tag) {
    constexpr int SEG = decltype(tag)::value;
    for (int h = so.off[SEG]; h < so.off[SEG + 1]; ++h) {
      const MemCat c = A.m.mem[h];
      const double dx = x - c.x, dy = y - c.y;
      Term<double> t;
      if (cat_term<SEG, D3>(c, dx, dy, u.b, u.s, u.a, A.qd, t)) add<D3>(acc, t);
      if (want_pot) pot += cat_pot<SEG>(c, dx, dy, u.b, u.s, u.a, A.qd);
    }
  };
  seg(std::integral_constant<int, SEG_CPJE>());
  seg(std::integral_constant<int, SEG_EPJE>());
  seg(std::integral_constant<int, SEG_CSIE>());
  seg(std::integral_constant<int, SEG_ESIE>());
  seg(std::integral_constant<int, SEG_POINT>());
  seg(std::integral_constant<int, SEG_NFW>());
  if constexpr (ENFW) seg(std::integral_constant<int, SEG_ENFW>());
}
template <int WHICH, bool ENFW>
__global__ __launch_bounds__(256) void k_chi2_obs(const Chi2Args A) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= (long long)A.S * A.n_img) return;
  const long long g = lane_slot(A, t);
  int s, i;
  double x, y;
  lane_point(A, g, s, i, x, y);
  const bool want_pot = A.dt != nullptr;
  Acc acc;
  double pot;
  if (WHICH == 0) {
    obs_sums<true, ENFW>(A, s, x, y, want_pot, acc, pot);
    double* e = A.ext + (size_t)g * 8;
    e[0] = pot; e[1] = acc.t111; e[2] = acc.t112; e[3] = acc.t122; e[4] = acc.t222;
    e[5] = acc.h11; e[6] = acc.h12; e[7] = acc.h22;
  } else {
    if (A.iflags[g] != 0) return;              // not accepted: the source-plane expansion is used
    obs_sums<false, ENFW>(A, s, A.tmod[2 * g], A.tmod[2 * g + 1], want_pot, acc, pot);
    double* e = A.extm + (size_t)g * 4;
    e[0] = pot; e[1] = acc.h11; e[2] = acc.h12; e[3] = acc.h22;
  }
}

// Model magnitude term m_i + 2.5 log10 |mu_model| and delay residual dt_obs - dt_model of image
// g (sorted index i, family f).  img: the image-plane solution was accepted (mu and psi at the
// model image); otherwise the source-plane expansions about theta_obs.
__device__ void obs_image(const Chi2Args& A, size_t g, int i, int f, bool img, double& mval, double& tval) {
  const double a = A.afam[f];
  const double bmx = A.bm_ws[(g / A.n_img * A.n_fam + f) * 2], bmy = A.bm_ws[(g / A.n_img * A.n_fam + f) * 2 + 1];
  const double T = A.dt ? A.tsc[f] : 0.0;
  double mu_m, t_m;
  if (img) {
    const double* e = A.extm + g * 4;
    const double B11 = 1.0 - a * e[1], B12 = -a * e[2], B22 = 1.0 - a * e[3];
    mu_m = 1.0 / (B11 * B22 - B12 * B12);
    const double ex = A.tmod[2 * g] - bmx, ey = A.tmod[2 * g + 1] - bmy;
    t_m = T * (0.5 * (ex * ex + ey * ey) - a * e[0]);
  } else {
    const double* e = A.ext + g * 8;
    const double* w = A.wimg + g * 6;
    const double tx = A.th[2 * i], ty = A.th[2 * i + 1], bx = w[3], by = w[4];
    const double A11 = 1.0 - a * e[5], A12 = -a * e[6], A22 = 1.0 - a * e[7];
    const double det = A11 * A22 - A12 * A12, mu = 1.0 / det;
    const double gdx = -a * (e[1] * A22 + A11 * e[3] - 2.0 * A12 * e[2]);
    const double gdy = -a * (e[2] * A22 + A11 * e[4] - 2.0 * A12 * e[3]);
    const double dbx = bmx - bx, dby = bmy - by;
    const double dthx = (A22 * dbx - A12 * dby) / det, dthy = (-A12 * dbx + A11 * dby) / det;
    mu_m = mu - mu * mu * (dthx * gdx + dthy * gdy);
    const double ex = tx - bx, ey = ty - by;
    t_m = T * (0.5 * (ex * ex + ey * ey) - a * e[0]) + T * (dbx * (bx - tx) + dby * (by - ty));
  }
  mval = A.mag ? A.mag[i] + 2.5 * log10(fabs(mu_m)) : 0.0;
  tval = A.dt ? A.dt[i] - t_m : 0.0;
}
// chi^2_f and chi^2_dt of family f of sample s; the nuisance zero points m_src and dt_0 are the
// weighted means of Eq. (msrc) and Eq. (dt0).  img: image-plane mode (accepted images use
// their model image).
__device__ void obs_family(const Chi2Args& A, int s, int f, bool img, double& cf, double& ct) {
  const int i0 = A.fam_start[f], i1 = A.fam_start[f + 1];
  double wf = 0, sf = 0, wt = 0, st = 0;
  for (int pass = 0; pass < 2; ++pass) {
    const double msrc = wf > 0 ? sf / wf : 0.0, dt0 = wt > 0 ? st / wt : 0.0;
    for (int i = i0; i < i1; ++i) {
      const bool hf = A.mag && A.smag[i] > 0, ht = A.dt && A.sdt[i] > 0;
      if (!hf && !ht) continue;
      const size_t g = (size_t)s * A.n_img + i;
      double mv, tv;
      obs_image(A, g, i, f, img && A.iflags[g] == 0, mv, tv);
      if (pass == 0) {
        if (hf) { const double w = 1.0 / (A.smag[i] * A.smag[i]); wf += w; sf += w * mv; }
        if (ht) { const double w = 1.0 / (A.sdt[i] * A.sdt[i]); wt += w; st += w * tv; }
      } else {
        if (hf) { const double d = mv - msrc; cf += d * d / (A.smag[i] * A.smag[i]); }
        if (ht) { const double d = tv - dt0; ct += d * d / (A.sdt[i] * A.sdt[i]); }
      }
    }
  }
}

// obs: add the flux and time-delay terms (source-plane mode with such constraints).
__device__ void chi2_src_sample(const Chi2Args& A, int s, bool obs) {
  const int lane = threadIdx.x & 63;
  double tot = 0.0, cf = 0.0, ct = 0.0;
  int fl = 0;
  for (int f = lane; f < A.n_fam; f += 64) {
    int i0 = A.fam_start[f], i1 = A.fam_start[f + 1];
    double a = A.afam[f];
    double G11 = 0, G12 = 0, G22 = 0, g1 = 0, g2 = 0;
    for (int i = i0; i < i1; ++i) {
      size_t g = (size_t)s * A.n_img + i;
      const double* q = A.part + g * 5;
      fl |= A.pflags[g];
      double bx = A.th[2 * i] - a * q[0], by = A.th[2 * i + 1] - a * q[1];
      double A11 = 1.0 - a * q[2], A12 = -a * q[3], A22 = 1.0 - a * q[4];
      double det = A11 * A22 - A12 * A12;
      double m11 = A22 / det, m12 = -A12 / det, m22 = A11 / det;
      const double* Si = A.sinv + 3 * i;
      double t11 = Si[0] * m11 + Si[1] * m12, t12 = Si[0] * m12 + Si[1] * m22;
      double t21 = Si[1] * m11 + Si[2] * m12, t22 = Si[1] * m12 + Si[2] * m22;
      double W11 = m11 * t11 + m12 * t21, W12 = m11 * t12 + m12 * t22, W22 = m12 * t12 + m22 * t22;
      double* w = A.wimg + g * 6;
      w[0] = W11; w[1] = W12; w[2] = W22; w[3] = bx; w[4] = by; w[5] = det;
      G11 += W11; G12 += W12; G22 += W22;
      g1 += W11 * bx + W12 * by;
      g2 += W12 * bx + W22 * by;
    }
    double bmx = 0, bmy = 0;
    if (i1 > i0) {
      double det = G11 * G22 - G12 * G12, tr = G11 + G22;
      if (!(fabs(det) > 1e-12 * tr * tr)) {
        fl |= FL_GSING;
        double lam = 0.5 * tr + sqrt(0.25 * (G11 - G22) * (G11 - G22) + G12 * G12);
        double vx = G12, vy = lam - G11;
        if (fabs(vx) + fabs(vy) == 0) { vx = 1; vy = 0; }
        double nv = sqrt(vx * vx + vy * vy);
        vx /= nv; vy /= nv;
        double proj = (vx * g1 + vy * g2) / (lam > 0 ? lam : 1.0);
        bmx = proj * vx; bmy = proj * vy;
      } else {
        bmx = (G22 * g1 - G12 * g2) / det;
        bmy = (-G12 * g1 + G11 * g2) / det;
      }
    }
    if (A.bmod) { A.bmod[((size_t)s * A.n_fam + f) * 2] = bmx; A.bmod[((size_t)s * A.n_fam + f) * 2 + 1] = bmy; }
    A.bm_ws[((size_t)s * A.n_fam + f) * 2] = bmx;
    A.bm_ws[((size_t)s * A.n_fam + f) * 2 + 1] = bmy;
    for (int i = i0; i < i1; ++i) {
      size_t g = (size_t)s * A.n_img + i;
      double* w = A.wimg + g * 6;
      double dx = w[3] - bmx, dy = w[4] - bmy;
      // d^T W d = (mu d)^T S^-1 (mu d), evaluated in the second form (non-negative under
      // rounding when mu is huge and W nearly rank one)
      const double* q = A.part + g * 5;
      const double A11 = 1.0 - a * q[2], A12 = -a * q[3], A22 = 1.0 - a * q[4], det = w[5];
      const double m11 = A22 / det, m12 = -A12 / det, m22 = A11 / det;
      const double vx = m11 * dx + m12 * dy, vy = m12 * dx + m22 * dy;
      const double* Si = A.sinv + 3 * i;
      double c = Si[0] * vx * vx + 2.0 * Si[1] * vx * vy + Si[2] * vy * vy;
      A.csrc[g] = c;
      tot += c;
    }
    if (obs) obs_family(A, s, f, false, cf, ct);
  }
  tot = wave_sum(tot);
  fl = wave_or(fl);
  if (obs) { cf = wave_sum(cf); ct = wave_sum(ct); }
  if (lane == 0) {
    A.chi2[s] = (fl & FL_INVALID) ? __builtin_nan("") : tot + cf + ct;
    if (A.flags) A.flags[s] = fl;
    if (A.terms) { A.terms[3 * (size_t)s] = tot; A.terms[3 * (size_t)s + 1] = cf; A.terms[3 * (size_t)s + 2] = ct; }
  }
}
__global__ __launch_bounds__(64) void k_chi2_src(const Chi2Args A, int obs) { chi2_src_sample(A, blockIdx.x, obs != 0); }

// Image-plane chi^2: Newton from theta_obs towards beta_model, full halo sum per step, in
// FP64 for both precisions (the source-plane part that sets beta_model follows the chosen
// precision).  Converged when a step is below newton_tol, at most NEWTON_MAX steps.
//
// Two rounds.  Round 1 runs one lane per image for at most NEWTON_R1 steps.  An image still
// unconverged then is appended to its item's straggler list (indices in pflags, state in
// part: both are free once the source-plane reduction has run) and round 2 continues it with
// a group of NEWTON_G lanes per image, the halo sum split over the group -- so a few slow
// images no longer hold whole waves for 20 steps, and many slow ones still fill the waves
// (64 / NEWTON_G images per wave).  Which round finishes an image, and the group's summation
// order, depend only on that image, so results do not depend on wave mates, tiles or batches.
static constexpr int NEWTON_MAX = 20, NEWTON_R1 = 5, NEWTON_G = 16;

struct NewtonImg {
  int s, i;
  double x0, y0, a, bmx, bmy, det0;
};
__device__ __forceinline__ void newton_img(const Chi2Args& A, long long g, NewtonImg& N) {
  lane_point(A, g, N.s, N.i, N.x0, N.y0);
  const int f = A.fam[N.i];
  N.a = A.afam[f];
  N.bmx = A.bm_ws[((size_t)N.s * A.n_fam + f) * 2];
  N.bmy = A.bm_ws[((size_t)N.s * A.n_fam + f) * 2 + 1];
  N.det0 = A.wimg[(size_t)g * 6 + 5];
}
// One Newton update from the halo sums at (tx, ty); true once a step is below newton_tol.
__device__ __forceinline__ bool newton_update(const Chi2Args& A, const NewtonImg& N, const Acc& acc, double& tx,
                                              double& ty, double& det_last) {
  const double a = N.a;
  double rx = N.bmx - (tx - a * acc.ax), ry = N.bmy - (ty - a * acc.ay);
  double A11 = 1.0 - a * acc.h11, A12 = -a * acc.h12, A22 = 1.0 - a * acc.h22;
  double det = A11 * A22 - A12 * A12;
  det_last = det;
  double dx = (A22 * rx - A12 * ry) / det, dy = (-A12 * rx + A11 * ry) / det;
  tx += dx;
  ty += dy;
  return sqrt(dx * dx + dy * dy) < A.newton_tol;
}
__device__ __forceinline__ void newton_finish(const Chi2Args& A, long long g, const NewtonImg& N, bool conv,
                                              double tx, double ty, double det_last) {
  double ox = N.x0 - tx, oy = N.y0 - ty;
  bool reject = !(sqrt(ox * ox + oy * oy) <= 10.0 * A.sigmax[N.i]) || ((det_last > 0) != (N.det0 > 0));
  int fl = (conv ? 0 : FL_NOCONV) | (reject ? FL_REJECT : 0);
  double c;
  if (!conv || reject) {
    c = A.csrc[g];
  } else {
    const double* Si = A.sinv + 3 * N.i;
    c = ox * (Si[0] * ox + Si[1] * oy) + oy * (Si[1] * ox + Si[2] * oy);
  }
  A.cimg[g] = c;
  A.iflags[g] = fl;
  if (A.tmod) { A.tmod[(size_t)g * 2] = tx; A.tmod[(size_t)g * 2 + 1] = ty; }
}

// Round 1 (every lane of the wave calls it; inactive lanes only take part in the votes).
__device__ void chi2_newton_lane(const Chi2Args& A, long long g, bool active) {
  if (!active) g = (long long)A.S * A.n_img - 1;
  NewtonImg N;
  newton_img(A, g, N);
  const MainRec* mr = A.mains + (size_t)N.s * A.m.n_main;
  const MulRec u = A.muls[N.s];
  double tx = N.x0, ty = N.y0, det_last = N.det0;
  bool conv = false;
  for (int it = 0; it < NEWTON_R1; ++it) {
    Acc acc;
    acc.zero();
    for (int c = 0; c < A.m.n_main; ++c) eval_main<false>(mr[c], tx, ty, A.qd, acc);
    rare_members(A, tx, ty, u, acc);
    bulk_members<false>(A, tx, ty, u, acc);
    if (!conv) conv = newton_update(A, N, acc, tx, ty, det_last);
    if (__all(conv)) break;
  }
  const bool strag = active && !conv;
  const unsigned long long mask = __ballot(strag);
  if (mask) {
    const int lane = threadIdx.x & 63, first = __ffsll((long long)mask) - 1;
    int base = 0;
    if (lane == first) base = atomicAdd(A.strag_n, __popcll(mask));
    base = __shfl(base, first, 64);
    if (strag) {
      A.pflags[base + __popcll(mask & ((1ull << lane) - 1ull))] = (int)g;
      double* st = A.part + (size_t)g * 5;
      st[0] = tx; st[1] = ty; st[2] = det_last;
    }
  }
  if (active && conv) newton_finish(A, g, N, true, tx, ty, det_last);
}
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_chi2_newton(const Chi2Args A) {
  long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  const bool active = t < (long long)A.S * A.n_img;
  chi2_newton_lane(A, active ? lane_slot(A, t) : 0, active);
}

// Full FP64 halo sum of sample s at (x, y) by a group of NEWTON_G adjacent lanes: lane k of the
// group takes halos k, k + G, ...; the partial sums are combined by a butterfly of shuffles
// within the group, after which every lane of the group holds the same bits.
__device__ void chi2_sum_group(const Chi2Args& A, int s, double x, double y, Acc& acc) {
  const int k = threadIdx.x & (NEWTON_G - 1);
  acc.zero();
  const MainRec* mr = A.mains + (size_t)s * A.m.n_main;
  const MulRec u = A.muls[s];
  const int nm = A.m.n_main, H = nm + A.m.n_mem;
  for (int h = k; h < H; h += NEWTON_G) {
    if (h < nm) {
      eval_main<false>(mr[h], x, y, A.qd, acc);
      continue;
    }
    const int m = h - nm;
    int sg = 0;
    while (sg + 1 < NSEG && m >= A.m.seg.off[sg + 1]) ++sg;
    const MemCat c = A.m.mem[m];
    const double dx = x - c.x, dy = y - c.y;
    Term<double> t;
    bool ok;
    switch (sg) {
      case SEG_CPJE: ok = cat_term<SEG_CPJE>(c, dx, dy, u.b, u.s, u.a, A.qd, t); break;
      case SEG_EPJE: ok = cat_term<SEG_EPJE>(c, dx, dy, u.b, u.s, u.a, A.qd, t); break;
      case SEG_CSIE: ok = cat_term<SEG_CSIE>(c, dx, dy, u.b, u.s, u.a, A.qd, t); break;
      case SEG_ESIE: ok = cat_term<SEG_ESIE>(c, dx, dy, u.b, u.s, u.a, A.qd, t); break;
      case SEG_POINT: ok = cat_term<SEG_POINT>(c, dx, dy, u.b, u.s, u.a, A.qd, t); break;
      case SEG_NFW: ok = cat_term<SEG_NFW>(c, dx, dy, u.b, u.s, u.a, A.qd, t); break;
      default: ok = cat_term<SEG_ENFW>(c, dx, dy, u.b, u.s, u.a, A.qd, t); break;
    }
    if (ok) add<false>(acc, t);
  }
#pragma unroll
  for (int o = 1; o < NEWTON_G; o <<= 1) {
    acc.ax += __shfl_xor(acc.ax, o, 64);
    acc.ay += __shfl_xor(acc.ay, o, 64);
    acc.h11 += __shfl_xor(acc.h11, o, 64);
    acc.h12 += __shfl_xor(acc.h12, o, 64);
    acc.h22 += __shfl_xor(acc.h22, o, 64);
  }
}

// Round 2: one group of NEWTON_G lanes per straggler image (g read from the item's list).  The
// lanes of a group always agree (same sums), so a group runs its loop as one; groups of a wave
// may stop at different steps, and their shuffles never leave the group.
__device__ void chi2_newton_group(const Chi2Args& A, long long g) {
  NewtonImg N;
  newton_img(A, g, N);
  const double* st = A.part + (size_t)g * 5;
  double tx = st[0], ty = st[1], det_last = st[2];
  bool conv = false;
  for (int it = NEWTON_R1; it < NEWTON_MAX && !conv; ++it) {
    Acc acc;
    chi2_sum_group(A, N.s, tx, ty, acc);
    conv = newton_update(A, N, acc, tx, ty, det_last);
  }
  if ((threadIdx.x & (NEWTON_G - 1)) == 0) newton_finish(A, g, N, conv, tx, ty, det_last);
}
__device__ __forceinline__ void newton_round2(const Chi2Args& A) {
  const int n = *A.strag_n;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int grp = (int)(t / NEWTON_G), ngrp = (int)((long long)gridDim.x * blockDim.x / NEWTON_G);
  for (int j = grp; j < n; j += ngrp) chi2_newton_group(A, A.pflags[j]);
}
__global__ __launch_bounds__(256) void k_chi2_newton2(const Chi2Args A) { newton_round2(A); }
__global__ void k_chi2_reset(int* p) { *p = 0; }

__device__ void chi2_img_sample(const Chi2Args& A, int s) {
  const int lane = threadIdx.x & 63;
  // per lane: a fixed contiguous block of images, summed in order; then a shuffle tree
  double tot = 0.0, cf = 0.0, ct = 0.0;
  int fl = 0;
  for (int i = lane; i < A.n_img; i += 64) {
    size_t g = (size_t)s * A.n_img + i;
    tot += A.cimg[g];
    fl |= A.iflags[g];
  }
  const bool obs = A.mag || A.dt;
  if (obs)
    for (int f = lane; f < A.n_fam; f += 64) obs_family(A, s, f, true, cf, ct);
  tot = wave_sum(tot);
  fl = wave_or(fl);
  if (obs) { cf = wave_sum(cf); ct = wave_sum(ct); }
  if (lane == 0) {
    int f0 = A.flags ? A.flags[s] : 0;
    A.chi2[s] = (f0 & FL_INVALID) ? __builtin_nan("") : tot + cf + ct;
    if (A.flags) A.flags[s] = f0 | fl;
    if (A.terms) { A.terms[3 * (size_t)s] = tot; A.terms[3 * (size_t)s + 1] = cf; A.terms[3 * (size_t)s + 2] = ct; }
  }
}
__global__ __launch_bounds__(64) void k_chi2_img_sum(const Chi2Args A) { chi2_img_sample(A, blockIdx.x); }

// Model image positions and image flags of every (sample, image) slot, written in the caller's
// constraint order: sorted slot k of sample s goes to constraint order[k].
__global__ __launch_bounds__(256) void k_chi2_images_out(const Chi2Args A, const int* order, double* theta_model,
                                                         int* img_flags) {
  const long long g = (long long)blockIdx.x * 256 + threadIdx.x;
  if (g >= (long long)A.S * A.n_img) return;
  const long long s = g / A.n_img, k = g - s * A.n_img;
  const long long o = s * A.n_img + order[k];
  if (theta_model) {
    theta_model[2 * o] = A.tmod[2 * g];
    theta_model[2 * o + 1] = A.tmod[2 * g + 1];
  }
  if (img_flags) img_flags[o] = A.iflags[g];
}

hipError_t launch_chi2_images_out(const Chi2Args& A, const int* order, double* theta_model, int* img_flags,
                                  hipStream_t st) {
  const long long n = (long long)A.S * A.n_img;
  hipLaunchKernelGGL(k_chi2_images_out, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, A, order, theta_model,
                     img_flags);
  return hipGetLastError();
}

hipError_t launch_chi2(const Chi2Args& A, bool mixed, int mode, hipStream_t st, void (*mark)(void*, const char*, int),
                       void* ctx) {
  long long n = (long long)A.S * A.n_img;
  unsigned blocks = (unsigned)((n + 255) / 256);
  mark(ctx, "chi2_heavy", 0);
  hipLaunchKernelGGL(k_chi2_heavy, dim3(blocks), dim3(256), 0, st, A);
  mark(ctx, "chi2_heavy", 1);
  mark(ctx, "chi2_lean", 0);
  const unsigned lean_blocks = (unsigned)((n + 63) / 64);
  if (mixed) hipLaunchKernelGGL(k_chi2_lean<true>, dim3(lean_blocks), dim3(256), 0, st, A);
  else hipLaunchKernelGGL(k_chi2_lean<false>, dim3(lean_blocks), dim3(256), 0, st, A);
  mark(ctx, "chi2_lean", 1);
  const bool obs = A.mag || A.dt;
  if (obs) {
    mark(ctx, "chi2_obs", 0);
    if (A.m.has_enfw) hipLaunchKernelGGL((k_chi2_obs<0, true>), dim3(blocks), dim3(256), 0, st, A);
    else hipLaunchKernelGGL((k_chi2_obs<0, false>), dim3(blocks), dim3(256), 0, st, A);
    mark(ctx, "chi2_obs", 1);
  }
  mark(ctx, "chi2_src", 0);
  hipLaunchKernelGGL(k_chi2_src, dim3(A.S), dim3(64), 0, st, A, (obs && mode == 0) ? 1 : 0);
  mark(ctx, "chi2_src", 1);
  if (mode == 1) {
    mark(ctx, "chi2_newton", 0);
    hipLaunchKernelGGL(k_chi2_reset, dim3(1), dim3(1), 0, st, A.strag_n);
    hipLaunchKernelGGL(k_chi2_newton, dim3(blocks), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_chi2_newton2, dim3(A.n_cu * 4), dim3(256), 0, st, A);
    mark(ctx, "chi2_newton", 1);
    if (obs && A.m.has_enfw) hipLaunchKernelGGL((k_chi2_obs<1, true>), dim3(blocks), dim3(256), 0, st, A);
    else if (obs) hipLaunchKernelGGL((k_chi2_obs<1, false>), dim3(blocks), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_chi2_img_sum, dim3(A.S), dim3(64), 0, st, A);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Uneven batches (one persistent launch over many items).  Tiles are ordered largest work
// first and taken from an atomic queue by resident workgroups, which stop when the queue is
// empty.  Every lane runs the same per-(sample, image) code as the single-item kernels, so a
// sample's result is bit-identical whichever tile, workgroup or batch it lands in.
// ---------------------------------------------------------------------------------------
__global__ void k_batch_reset(int* counter, const Chi2Args* items, int n_items) {
  if (threadIdx.x < 2) counter[threadIdx.x] = 0;
  for (int i = threadIdx.x; i < n_items; i += blockDim.x) *items[i].strag_n = 0;
}

__global__ __launch_bounds__(256) void k_batch_heavy(const BatchArgs B) {
  for (int t = blockIdx.x; t < B.n_tiles; t += gridDim.x) {
    const BatchTile T = B.tiles[t];
    const Chi2Args& A = B.items[T.item];
    for (long long t = T.g0 + threadIdx.x; t < T.g1; t += blockDim.x) chi2_heavy_lane(A, lane_slot(A, t));
  }
}

__device__ __forceinline__ int next_tile(int* counter) {
  __shared__ int t_sh;
  __syncthreads();
  if (threadIdx.x == 0) t_sh = atomicAdd(counter, 1);
  __syncthreads();
  return t_sh;
}

template <bool MIXED>
__global__ __launch_bounds__(256) void k_batch_lean(const BatchArgs B) {
  for (;;) {
    int t = next_tile(&B.counter[0]);
    if (t >= B.n_tiles) break;
    const BatchTile T = B.tiles[t];
    const Chi2Args& A = B.items[T.item];
    for (long long u0 = T.g0; u0 < T.g1; u0 += 64) chi2_lean_group<MIXED>(A, u0, T.g1);
  }
}

__global__ __launch_bounds__(64) void k_batch_src(const BatchArgs B) {
  int gs = blockIdx.x;
  chi2_src_sample(B.items[B.samp_item[gs]], B.samp_local[gs], false);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_batch_newton(const BatchArgs B) {
  for (;;) {
    int t = next_tile(&B.counter[1]);
    if (t >= B.n_tiles) break;
    const BatchTile T = B.tiles[t];
    const Chi2Args& A = B.items[T.item];
    // uniform trip count so that whole waves take part in the convergence votes
    for (long long base = T.g0; base < T.g1; base += blockDim.x) {
      const long long t = base + threadIdx.x;
      chi2_newton_lane(A, t < T.g1 ? lane_slot(A, t) : 0, t < T.g1);
    }
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_batch_newton2(const BatchArgs B) {
  for (int i = 0; i < B.n_items; ++i) newton_round2(B.items[i]);
}

__global__ __launch_bounds__(64) void k_batch_img(const BatchArgs B) {
  int gs = blockIdx.x;
  chi2_img_sample(B.items[B.samp_item[gs]], B.samp_local[gs]);
}

hipError_t launch_batch_lean_only(const BatchArgs& B, bool mixed, int block, int grid_persist, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, B.counter, B.items, B.n_items);
  if (mixed) hipLaunchKernelGGL(k_batch_lean<true>, dim3(grid_persist), dim3(block), 0, st, B);
  else hipLaunchKernelGGL(k_batch_lean<false>, dim3(grid_persist), dim3(block), 0, st, B);
  return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs& B, bool mixed, int mode, int block, int grid_persist, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, B.counter, B.items, B.n_items);
  hipLaunchKernelGGL(k_batch_heavy, dim3(grid_persist), dim3(block), 0, st, B);
  if (mixed) hipLaunchKernelGGL(k_batch_lean<true>, dim3(grid_persist), dim3(block), 0, st, B);
  else hipLaunchKernelGGL(k_batch_lean<false>, dim3(grid_persist), dim3(block), 0, st, B);
  hipLaunchKernelGGL(k_batch_src, dim3(B.total_S), dim3(64), 0, st, B);
  if (mode == 1) {
    hipLaunchKernelGGL(k_batch_newton, dim3(grid_persist), dim3(block), 0, st, B);
    hipLaunchKernelGGL(k_batch_newton2, dim3(grid_persist), dim3(256), 0, st, B);
    hipLaunchKernelGGL(k_batch_img, dim3(B.total_S), dim3(64), 0, st, B);
  }
  return hipGetLastError();
}

}  // namespace lf
