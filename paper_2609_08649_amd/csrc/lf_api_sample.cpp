// lf_aies_run and lf_nelder_mead_run: the inference loops of Sec. 3.5 on the device.  Each
// step enqueues proposal / update kernels around a batched chi^2 evaluation on the caller's
// stream; nothing is copied to the host between steps.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "lf_api_internal.h"
#include "lf_sample.h"

namespace {
lf_status check_common(lf_ctx* ctx, const lf_model* M, const lf_cons* c, int mode, lf_prec prec, const double* lo,
                       const double* hi) {
  if (!M || !c || !lo || !hi) return ctx->fail(LF_E_INVALID_ARG, "null model/constraints/prior box");
  if (M->n_free < 1) return ctx->fail(LF_E_INVALID_ARG, "the model has no free parameter");
  if (mode != 0 && mode != 1) return ctx->fail(LF_E_INVALID_ARG, "mode must be 0 (source) or 1 (image)");
  if (prec != LF_PREC_FP64 && prec != LF_PREC_MIXED) return ctx->fail(LF_E_INVALID_ARG, "bad precision");
  return LF_OK;
}
}  // namespace

extern "C" lf_status lf_aies_run(lf_ctx* ctx, const lf_model* M, const lf_cons* c, int32_t mode, lf_prec prec,
                                 int32_t K, double* X, double* lp, int32_t init_lp, const double* lo,
                                 const double* hi, double a, uint64_t seed, int64_t step0, int32_t n_steps,
                                 double* chain, double* lp_chain, int32_t* n_accept, void* stream) {
  if (!ctx) return LF_E_INVALID_ARG;
  lf_status e = check_common(ctx, M, c, mode, prec, lo, hi);
  if (e) return e;
  if (!X || !lp) return ctx->fail(LF_E_INVALID_ARG, "null walkers");
  if (K < 4 || K % 2) return ctx->fail(LF_E_INVALID_ARG, "K must be even and >= 4");
  if (!(a > 1.0) || !std::isfinite(a)) return ctx->fail(LF_E_INVALID_ARG, "stretch scale a must be > 1");
  if (n_steps < 0 || step0 < 0) return ctx->fail(LF_E_INVALID_ARG, "negative step count");
  hipSetDevice(ctx->device);
  hipStream_t st = (hipStream_t)stream;
  const int D = M->n_free;
  lf::AiesArgs A;
  std::memset(&A, 0, sizeof A);
  A.K = K; A.D = D; A.X = X; A.lp = lp; A.lo = lo; A.hi = hi; A.a = a; A.seed = seed;
  A.acc = n_accept; A.chain = chain; A.lp_chain = lp_chain;
  A.Y = (double*)ctx->ws("aies.Y", sizeof(double) * (size_t)(K / 2) * D, st, &e);
  if (e) return e;
  double* chi2 = (double*)ctx->ws("aies.chi2", sizeof(double) * K, st, &e);
  if (e) return e;
  if (init_lp) {
    e = lf_chi2_terms(ctx, M, X, K, c, mode, prec, chi2, nullptr, nullptr, nullptr, stream);
    if (e) return e;
    if (hipError_t he = lf::launch_aies_lp(A, chi2, st)) return ctx->hip(he, "aies lp");
  }
  for (int s = 0; s < n_steps; ++s) {
    const long long t = step0 + s;
    for (int h = 0; h < 2; ++h) {
      if (hipError_t he = lf::launch_aies_propose(A, t, h, st)) return ctx->hip(he, "aies propose");
      e = lf_chi2_terms(ctx, M, A.Y, K / 2, c, mode, prec, chi2, nullptr, nullptr, nullptr, stream);
      if (e) return e;
      if (hipError_t he = lf::launch_aies_accept(A, t, h, chi2, st)) return ctx->hip(he, "aies accept");
    }
    if (chain || lp_chain)
      if (hipError_t he = lf::launch_aies_record(A, s, st)) return ctx->hip(he, "aies record");
  }
  return LF_OK;
}

extern "C" lf_status lf_nelder_mead_run(lf_ctx* ctx, const lf_model* M, const lf_cons* c, int32_t mode,
                                        lf_prec prec, int32_t R, double* simplex, double* fvals, const double* lo,
                                        const double* hi, int32_t n_rounds, int32_t* n_evals, void* stream) {
  if (!ctx) return LF_E_INVALID_ARG;
  lf_status e = check_common(ctx, M, c, mode, prec, lo, hi);
  if (e) return e;
  if (!simplex || !fvals) return ctx->fail(LF_E_INVALID_ARG, "null simplex/values");
  if (R < 1 || n_rounds < 0) return ctx->fail(LF_E_INVALID_ARG, "R must be >= 1, n_rounds >= 0");
  const int D = M->n_free;
  if ((long long)R * (D + 1) >= (1LL << 31)) return ctx->fail(LF_E_INVALID_ARG, "too many runs");
  if (D > 64) return ctx->fail(LF_E_UNSUPPORTED, "Nelder-Mead runs take at most 64 parameters");
  hipSetDevice(ctx->device);
  hipStream_t st = (hipStream_t)stream;
  lf::NMArgs A;
  std::memset(&A, 0, sizeof A);
  A.R = R; A.D = D; A.x = simplex; A.f = fvals; A.lo = lo; A.hi = hi; A.nev = n_evals;
  A.team = 1;
  while (A.team < D) A.team <<= 1;
  A.xr = (double*)ctx->ws("nm.xr", sizeof(double) * (size_t)R * D, st, &e); if (e) return e;
  A.fr = (double*)ctx->ws("nm.fr", sizeof(double) * R, st, &e); if (e) return e;
  A.state = (int*)ctx->ws("nm.state", sizeof(int) * R, st, &e); if (e) return e;
  A.idx = (int*)ctx->ws("nm.idx", sizeof(int) * R, st, &e); if (e) return e;
  A.pend = (double*)ctx->ws("nm.pend", sizeof(double) * (size_t)R * D, st, &e); if (e) return e;
  double* chi2 = (double*)ctx->ws("nm.chi2", sizeof(double) * (size_t)R * (D + 1), st, &e);
  if (e) return e;
  e = lf_chi2_terms(ctx, M, simplex, R * (D + 1), c, mode, prec, chi2, nullptr, nullptr, nullptr, stream);
  if (e) return e;
  if (hipError_t he = lf::launch_nm_init(A, chi2, st)) return ctx->hip(he, "nm init");
  for (int k = 0; k < n_rounds; ++k) {
    e = lf_chi2_terms(ctx, M, A.pend, R, c, mode, prec, chi2, nullptr, nullptr, nullptr, stream);
    if (e) return e;
    if (hipError_t he = lf::launch_nm_step(A, chi2, st)) return ctx->hip(he, "nm step");
  }
  return LF_OK;
}
