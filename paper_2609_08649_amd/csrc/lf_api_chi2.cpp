// Constraint tables (positions, fluxes, delays), lf_chi2_batch and lf_chi2_terms.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "lf_api_internal.h"
#include "lf_chi2.h"

void lf_prof_mark(void* c, const char* name, int end_flag) {
  lf_ctx* ctx = (lf_ctx*)c;
  (void)name;
  if (!ctx->prof) return;
  // the stream is carried by the context while a call is in flight
  if (end_flag) ctx->prof_end(ctx->cur_stream);
  else ctx->prof_begin(name, ctx->cur_stream);
}

extern "C" lf_status lf_constraints_upload(lf_ctx* ctx, const double* theta, const int32_t* family,
                                           const double* sig1, const double* sig2, const double* phi,
                                           int32_t n_img, const double* a_fam, int32_t n_fam, lf_cons** out) {
  if (!ctx || !out) return LF_E_INVALID_ARG;
  *out = nullptr;
  if (n_img < 1 || n_fam < 1 || !theta || !family || !sig1 || !sig2 || !phi || !a_fam)
    return ctx->fail(LF_E_INVALID_ARG, "constraints: missing arrays or empty set");
  for (int i = 0; i < n_img; ++i) {
    if (family[i] < 0 || family[i] >= n_fam) return ctx->fail(LF_E_INVALID_ARG, "image %d: family out of range", i);
    if (!(sig1[i] > 0) || !(sig2[i] > 0) || !std::isfinite(sig1[i]) || !std::isfinite(sig2[i]) ||
        !std::isfinite(phi[i]) || !std::isfinite(theta[2 * i]) || !std::isfinite(theta[2 * i + 1]))
      return ctx->fail(LF_E_INVALID_ARG, "image %d: bad position or error ellipse", i);
  }
  for (int f = 0; f < n_fam; ++f)
    if (!(a_fam[f] > 0) || !std::isfinite(a_fam[f])) return ctx->fail(LF_E_INVALID_ARG, "family %d: a_dis must be > 0", f);
  lf_cons* c = new lf_cons();
  c->n_img = n_img;
  c->n_fam = n_fam;
  c->order.resize(n_img);
  std::iota(c->order.begin(), c->order.end(), 0);
  std::stable_sort(c->order.begin(), c->order.end(), [&](int a, int b) { return family[a] < family[b]; });
  c->fam_start.assign(n_fam + 1, 0);
  for (int i = 0; i < n_img; ++i) c->fam_start[family[i] + 1]++;
  for (int f = 0; f < n_fam; ++f) c->fam_start[f + 1] += c->fam_start[f];
  std::vector<double> th(2 * n_img), si(3 * n_img), sm(n_img);
  std::vector<int> fm(n_img);
  for (int k = 0; k < n_img; ++k) {
    int i = c->order[k];
    th[2 * k] = theta[2 * i]; th[2 * k + 1] = theta[2 * i + 1];
    fm[k] = family[i];
    // S^-1 = R^T diag(1/sig1^2, 1/sig2^2) R, R = [[c, s], [-s, c]]  (Sec. 3.1)
    double cs = std::cos(phi[i]), sn = std::sin(phi[i]);
    double i1 = 1.0 / (sig1[i] * sig1[i]), i2 = 1.0 / (sig2[i] * sig2[i]);
    si[3 * k] = cs * cs * i1 + sn * sn * i2;
    si[3 * k + 1] = cs * sn * (i1 - i2);
    si[3 * k + 2] = sn * sn * i1 + cs * cs * i2;
    sm[k] = std::max(sig1[i], sig2[i]);
  }
  size_t bytes = sizeof(double) * (2 * n_img + 3 * n_img + n_img + n_fam) + sizeof(int) * (2 * n_img + n_fam + 1);
  char* base = nullptr;
  lf_status st = ctx->dmalloc((void**)&base, bytes);
  if (st) { delete c; return st; }
  c->bytes = bytes;
  c->d_theta = (double*)base;
  c->d_sinv = c->d_theta + 2 * n_img;
  c->d_sigmax = c->d_sinv + 3 * n_img;
  c->d_afam = c->d_sigmax + n_img;
  c->d_fam = (int*)(c->d_afam + n_fam);
  c->d_fam_start = c->d_fam + n_img;
  c->d_order = c->d_fam_start + n_fam + 1;
  hipMemcpy(c->d_theta, th.data(), sizeof(double) * th.size(), hipMemcpyHostToDevice);
  hipMemcpy(c->d_sinv, si.data(), sizeof(double) * si.size(), hipMemcpyHostToDevice);
  hipMemcpy(c->d_sigmax, sm.data(), sizeof(double) * sm.size(), hipMemcpyHostToDevice);
  hipMemcpy(c->d_afam, a_fam, sizeof(double) * n_fam, hipMemcpyHostToDevice);
  hipMemcpy(c->d_fam, fm.data(), sizeof(int) * n_img, hipMemcpyHostToDevice);
  hipMemcpy(c->d_fam_start, c->fam_start.data(), sizeof(int) * (n_fam + 1), hipMemcpyHostToDevice);
  hipMemcpy(c->d_order, c->order.data(), sizeof(int) * n_img, hipMemcpyHostToDevice);
  *out = c;
  return LF_OK;
}

extern "C" lf_status lf_constraints_observables(lf_ctx* ctx, lf_cons* c, const double* mag, const double* sig_mag,
                                                const double* dt, const double* sig_dt, const double* tscale) {
  if (!ctx || !c) return LF_E_INVALID_ARG;
  if (c->has_obs()) return ctx->fail(LF_E_INVALID_ARG, "constraints: observables already set");
  const bool hf = mag || sig_mag, ht = dt || sig_dt || tscale;
  if (!hf && !ht) return ctx->fail(LF_E_INVALID_ARG, "constraints: no flux or time-delay data");
  if (hf && (!mag || !sig_mag)) return ctx->fail(LF_E_INVALID_ARG, "flux data needs mag and sig_mag");
  if (ht && (!dt || !sig_dt || !tscale)) return ctx->fail(LF_E_INVALID_ARG, "time-delay data needs dt, sig_dt and tscale");
  const int n = c->n_img, nf = c->n_fam;
  for (int i = 0; i < n; ++i) {
    if (hf && (!std::isfinite(sig_mag[i]) || (sig_mag[i] > 0 && !std::isfinite(mag[i]))))
      return ctx->fail(LF_E_INVALID_ARG, "image %d: bad magnitude or error", i);
    if (ht && (!std::isfinite(sig_dt[i]) || (sig_dt[i] > 0 && !std::isfinite(dt[i]))))
      return ctx->fail(LF_E_INVALID_ARG, "image %d: bad delay or error", i);
  }
  if (ht)
    for (int f = 0; f < nf; ++f)
      if (!(tscale[f] > 0) || !std::isfinite(tscale[f])) return ctx->fail(LF_E_INVALID_ARG, "family %d: tscale must be > 0", f);
  std::vector<double> h;
  if (hf) { h.resize(2 * n); for (int k = 0; k < n; ++k) { h[k] = mag[c->order[k]]; h[n + k] = sig_mag[c->order[k]]; } }
  if (ht) {
    size_t o = h.size();
    h.resize(o + 2 * n + nf);
    for (int k = 0; k < n; ++k) { h[o + k] = dt[c->order[k]]; h[o + n + k] = sig_dt[c->order[k]]; }
    for (int f = 0; f < nf; ++f) h[o + 2 * n + f] = tscale[f];
  }
  size_t bytes = sizeof(double) * h.size();
  lf_status st = ctx->dmalloc((void**)&c->d_obs, bytes);
  if (st) return st;
  c->obs_bytes = bytes;
  hipMemcpy(c->d_obs, h.data(), bytes, hipMemcpyHostToDevice);
  double* p = (double*)c->d_obs;
  if (hf) { c->d_mag = p; p += 2 * n; }
  if (ht) { c->d_dt = p; c->d_tsc = p + 2 * n; }
  return LF_OK;
}

extern "C" lf_status lf_constraints_release(lf_ctx* ctx, lf_cons* c) {
  if (!ctx || !c) return LF_E_INVALID_ARG;
  ctx->dfree(c->d_theta, c->bytes);
  if (c->d_obs) ctx->dfree(c->d_obs, c->obs_bytes);
  delete c;
  return LF_OK;
}

lf_status lf_chi2_prepare(lf_ctx* ctx, const lf_model* M, const double* params, int S, const lf_cons* c,
                          hipStream_t st, lf::Chi2Args& A, const char* tag, bool want_tmod) {
  // every workspace buffer is placed before the first launch, so a call that does not fit
  // its workspace fails before anything runs
  lf::MainRec* mains; lf::MulRec* muls; lf::MemRec32* m32; lf::MemRec64* m64;
  lf_status e = lf_expand_alloc(ctx, M, S, false, st, &mains, &muls, &m32, &m64, tag);
  if (e) return e;
  std::string t(tag);
  size_t n = (size_t)S * c->n_img;
  auto wsd = [&](const char* nm, size_t cnt) { return (double*)ctx->ws((t + nm).c_str(), sizeof(double) * std::max<size_t>(1, cnt), st, &e); };
  auto wsi = [&](const char* nm, size_t cnt) { return (int*)ctx->ws((t + nm).c_str(), sizeof(int) * std::max<size_t>(1, cnt), st, &e); };
  A.part = wsd(".part", n * 5); if (e) return e;
  A.pflags = wsi(".pflags", n); if (e) return e;
  A.wimg = wsd(".wimg", n * 6); if (e) return e;
  A.csrc = wsd(".csrc", n); if (e) return e;
  A.cimg = wsd(".cimg", n); if (e) return e;
  A.iflags = wsi(".iflags", n); if (e) return e;
  A.bm_ws = wsd(".bm", (size_t)S * c->n_fam * 2); if (e) return e;
  A.strag_n = wsi(".strag", 1); if (e) return e;
  A.n_cu = ctx->n_cu > 0 ? ctx->n_cu : 256;
  A.mag = A.smag = A.dt = A.sdt = A.tsc = nullptr;
  A.ext = A.extm = A.terms = nullptr;
  if (c->has_obs()) {
    if (c->d_mag) { A.mag = c->d_mag; A.smag = c->d_mag + c->n_img; }
    if (c->d_dt) { A.dt = c->d_dt; A.sdt = c->d_dt + c->n_img; A.tsc = c->d_tsc; }
    A.ext = wsd(".ext", n * 8); if (e) return e;
    A.extm = wsd(".extm", n * 4); if (e) return e;
  }
  A.m = lf_dev_model(M);
  A.mains = mains; A.muls = muls; A.cat32 = M->d_cat32;
  A.S = S; A.n_img = c->n_img; A.n_fam = c->n_fam;
  A.th = c->d_theta; A.fam = c->d_fam; A.fam_start = c->d_fam_start; A.afam = c->d_afam;
  A.sinv = c->d_sinv; A.sigmax = c->d_sigmax;
  lf::QuadTab q = lf_quad(ctx);
  A.qd.n = q.n; A.qd.u = q.u; A.qd.w = q.w;
  A.tmod = nullptr;
  if (c->has_obs() || want_tmod) { A.tmod = wsd(".tmod", n * 2); if (e) return e; }
  return lf_expand_launch(ctx, M, params, S, st, mains, muls, m32, m64);
}

extern "C" lf_status lf_chi2_batch(lf_ctx* ctx, const lf_model* M, const double* params, int32_t S,
                                   const lf_cons* c, int32_t mode, lf_prec prec, double* chi2, int32_t* flags,
                                   double* beta_model, void* stream) {
  return lf_chi2_terms(ctx, M, params, S, c, mode, prec, chi2, flags, beta_model, nullptr, stream);
}

// Argument checks shared by the chi^2 entry points (nothing is launched when they fail).
lf_status lf_chi2_check(lf_ctx* ctx, const lf_model* M, const double* params, int32_t S, const lf_cons* c,
                        int32_t mode, lf_prec prec, const double* chi2) {
  if (!ctx) return LF_E_INVALID_ARG;
  if (!M || !c || !chi2) return ctx->fail(LF_E_INVALID_ARG, "null model/constraints/output");
  if (S < 1) return ctx->fail(LF_E_INVALID_ARG, "S must be >= 1");
  if (M->n_free > 0 && !params) return ctx->fail(LF_E_INVALID_ARG, "model has free fields: params required");
  if (mode != 0 && mode != 1) return ctx->fail(LF_E_INVALID_ARG, "mode must be 0 (source) or 1 (image)");
  if (mode == 1 && (long long)S * c->n_img >= (1LL << 31))
    return ctx->fail(LF_E_INVALID_ARG, "image plane needs S * n_img < 2^31");
  if (prec != LF_PREC_FP64 && prec != LF_PREC_MIXED) return ctx->fail(LF_E_INVALID_ARG, "bad precision");
  return LF_OK;
}

extern "C" lf_status lf_chi2_terms(lf_ctx* ctx, const lf_model* M, const double* params, int32_t S,
                                   const lf_cons* c, int32_t mode, lf_prec prec, double* chi2, int32_t* flags,
                                   double* beta_model, double* terms, void* stream) {
  lf_status ce = lf_chi2_check(ctx, M, params, S, c, mode, prec, chi2);
  if (ce) return ce;
  hipSetDevice(ctx->device);
  hipStream_t st = (hipStream_t)stream;
  lf::Chi2Args A;
  lf_status e = lf_chi2_prepare(ctx, M, params, S, c, st, A, "chi2");
  if (e) return e;
  A.chi2 = chi2; A.flags = flags; A.bmod = beta_model; A.terms = terms;
  bool mixed = prec == LF_PREC_MIXED;
  A.newton_tol = 1e-9;
  ctx->cur_stream = st;
  return ctx->hip(lf::launch_chi2(A, mixed, mode, st, lf_prof_mark, ctx), "chi2 kernels");
}

extern "C" lf_status lf_chi2_images(lf_ctx* ctx, const lf_model* M, const double* params, int32_t S,
                                    const lf_cons* c, lf_prec prec, double* chi2, int32_t* flags,
                                    double* beta_model, double* theta_model, int32_t* img_flags, void* stream) {
  lf_status ce = lf_chi2_check(ctx, M, params, S, c, 1, prec, chi2);
  if (ce) return ce;
  hipSetDevice(ctx->device);
  hipStream_t st = (hipStream_t)stream;
  lf::Chi2Args A;
  lf_status e = lf_chi2_prepare(ctx, M, params, S, c, st, A, "chi2", true);
  if (e) return e;
  A.chi2 = chi2; A.flags = flags; A.bmod = beta_model; A.terms = nullptr;
  A.newton_tol = 1e-9;
  ctx->cur_stream = st;
  e = ctx->hip(lf::launch_chi2(A, prec == LF_PREC_MIXED, 1, st, lf_prof_mark, ctx), "chi2 kernels");
  if (e) return e;
  return ctx->hip(lf::launch_chi2_images_out(A, c->d_order, theta_model, img_flags, st), "chi2 image outputs");
}
