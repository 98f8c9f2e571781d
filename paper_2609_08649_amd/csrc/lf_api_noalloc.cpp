// lf_chi2_batch_noalloc: the chi^2 of lf_chi2_batch for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// Its workspace (expanded halo tables, per-(sample, image) partial sums and terms, the
// per-family source positions and the straggler counter of the image-plane Newton solve) lives
// in `scratch`, a file-scope device array of LF_CHI2_NOALLOC_SCRATCH_BYTES that every GPU the
// library runs on holds until the process ends.  In host code the array's name is a host-side
// stand-in, not a device address: the address of each device's copy is taken once per device
// with hipGetSymbolAddress (lf_noalloc_setup, called by lf_init with that device current) and
// only that address is handed to kernels.  The call launches the same kernels as
// lf_chi2_batch, in the same order, on the same layouts, so its results are bit-identical.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "lf_api_internal.h"
#include "lf_chi2.h"

namespace {

__device__ __align__(256) char scratch[LF_CHI2_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
std::map<int, char*> g_scratch;   // device ordinal -> address of that device's `scratch`

void no_mark(void*, const char*, int) {}

}  // namespace

lf_status lf_noalloc_setup(lf_ctx* ctx) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_scratch.find(ctx->device);
  if (it == g_scratch.end()) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return ctx->hip(e, "hipGetSymbolAddress(scratch)");
    if (!p) return ctx->fail(LF_E_DEVICE, "hipGetSymbolAddress(scratch) returned a null address");
    it = g_scratch.emplace(ctx->device, (char*)p).first;
  }
  ctx->noalloc_scratch = it->second;
  return LF_OK;
}

extern "C" lf_status lf_chi2_batch_noalloc(lf_ctx* ctx, const lf_model* M, const double* params, int32_t S,
                                           const lf_cons* c, int32_t mode, lf_prec prec, double* chi2,
                                           int32_t* flags, double* beta_model, void* stream) {
  lf_status e = lf_chi2_check(ctx, M, params, S, c, mode, prec, chi2);
  if (e) return e;
  if (!ctx->noalloc_scratch) return ctx->fail(LF_E_DEVICE, "lf_chi2_batch_noalloc: no scratch address");
  hipSetDevice(ctx->device);
  hipStream_t st = (hipStream_t)stream;
  // Workspace from the static scratch; kernel timing is off for the call (its events would be
  // created on demand).
  lf_ctx::Arena ar{ctx->noalloc_scratch, (size_t)LF_CHI2_NOALLOC_SCRATCH_BYTES, 0, "lf_chi2_batch_noalloc"};
  const bool prof = ctx->prof;
  ctx->arena = &ar;
  ctx->prof = false;
  lf::Chi2Args A;
  e = lf_chi2_prepare(ctx, M, params, S, c, st, A, "chi2");
  ctx->arena = nullptr;
  ctx->prof = prof;
  if (e) return e;
  A.chi2 = chi2; A.flags = flags; A.bmod = beta_model; A.terms = nullptr;
  A.newton_tol = 1e-9;
  return ctx->hip(lf::launch_chi2(A, prec == LF_PREC_MIXED, mode, st, no_mark, nullptr), "chi2 kernels");
}
