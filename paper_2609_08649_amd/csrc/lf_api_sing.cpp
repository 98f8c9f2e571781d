// lf_singularity_map: vertex fields by the maps kernels (with third derivatives), then the
// extraction kernels of lf_sing.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "lf_api_internal.h"
#include "lf_sing.h"

extern "C" lf_status lf_singularity_map(lf_ctx* ctx, const lf_model* M, const double* params, const lf_grid* grid,
                                        lf_prec prec, int32_t refine, double tol, const lf_sing_out* out,
                                        void* stream) {
  if (!ctx) return LF_E_INVALID_ARG;
  if (!M || !grid || !out) return ctx->fail(LF_E_INVALID_ARG, "null model/grid/output");
  if (M->n_free > 0 && !params) return ctx->fail(LF_E_INVALID_ARG, "model has free fields: params required");
  if (grid->nx < 2 || grid->ny < 2 || !(grid->h > 0) || !std::isfinite(grid->h) || !std::isfinite(grid->x0) ||
      !std::isfinite(grid->y0) || (long long)grid->nx * grid->ny >= (1LL << 31))
    return ctx->fail(LF_E_INVALID_ARG, "grid must have 2..2^31 vertices, 2 or more per side, h > 0");
  if (out->cap < 1) return ctx->fail(LF_E_INVALID_ARG, "cap must be >= 1");
  if (!(tol > 0) || !std::isfinite(tol)) return ctx->fail(LF_E_INVALID_ARG, "tol must be > 0");
  if (!out->cross_pos || !out->cross_k || !out->cross_e || !out->cross_g || !out->cross_flags || !out->seg_a ||
      !out->seg_b || !out->seg_k || !out->umb_pos || !out->umb_kappa || !out->umb_status || !out->swt_pos ||
      !out->swt_k || !out->swt_e || !out->swt_seg || !out->swt_status || !out->counts)
    return ctx->fail(LF_E_INVALID_ARG, "every output list is required");
  if (prec != LF_PREC_FP64 && prec != LF_PREC_MIXED) return ctx->fail(LF_E_INVALID_ARG, "bad precision");
  hipSetDevice(ctx->device);
  hipStream_t st = (hipStream_t)stream;
  const long long P = (long long)grid->nx * grid->ny;
  const int nx = grid->nx, ny = grid->ny, cap = out->cap;
  lf_status e = LF_OK;

  // 1. vertex fields: gamma_1, gamma_2, f_1, f_2, flags
  double* vf = (double*)ctx->ws("sing.vtx", sizeof(double) * 4 * P + sizeof(int) * P, st, &e);
  if (e) return e;
  lf_maps mo;
  std::memset(&mo, 0, sizeof mo);
  mo.gamma1 = vf; mo.gamma2 = vf + P; mo.f1 = vf + 2 * P; mo.f2 = vf + 3 * P;
  mo.flags = (int32_t*)(vf + 4 * P);
  lf_points pts;
  std::memset(&pts, 0, sizeof pts);
  pts.grid = *grid;
  e = lf_lens_maps(ctx, M, params, 1, &pts, 1.0, prec, &mo, stream);
  if (e) return e;

  // 2. FP64 tables for the refinement evaluations
  lf::MainRec* mains; lf::MulRec* muls; lf::MemRec32* m32; lf::MemRec64* m64;
  e = lf_expand_tables(ctx, M, params, 1, true, st, &mains, &muls, &m32, &m64, "sing");
  if (e) return e;
  lf::DevModel dm = lf_dev_model(M);

  lf::SingArgs A;
  std::memset(&A, 0, sizeof A);
  A.x0 = grid->x0; A.y0 = grid->y0; A.h = grid->h; A.nx = nx; A.ny = ny;
  A.g1 = mo.gamma1; A.g2 = mo.gamma2; A.f1 = mo.f1; A.f2 = mo.f2; A.vflags = mo.flags;
  A.pl.mains = mains; A.pl.n_main = dm.n_main; A.pl.mem = m64; A.pl.seg = dm.seg;
  A.enfw = dm.has_enfw;
  lf::QuadTab q = lf_quad(ctx);
  A.qd.n = q.n; A.qd.u = q.u; A.qd.w = q.w;
  A.refine = refine ? 1 : 0;
  A.tol = tol;
  A.cap = cap;
  const int chunks = (cap + 255) / 256;
  auto wsi = [&](const char* nm, size_t cnt) { return (int*)ctx->ws(nm, sizeof(int) * cnt, st, &e); };
  A.xrow_cnt = wsi("sing.xrc", ny); if (e) return e;
  A.xrow_off = wsi("sing.xro", ny + 1); if (e) return e;
  A.srow_cnt = wsi("sing.src", ny); if (e) return e;
  A.srow_off = wsi("sing.sro", ny + 1); if (e) return e;
  A.urow_cnt = wsi("sing.urc", ny); if (e) return e;
  A.urow_off = wsi("sing.uro", ny + 1); if (e) return e;
  A.krow_cnt = wsi("sing.krc", ny); if (e) return e;
  A.krow_off = wsi("sing.kro", ny + 1); if (e) return e;
  A.prow_cnt = wsi("sing.prc", ny); if (e) return e;
  A.prow_off = wsi("sing.pro", ny + 1); if (e) return e;
  A.wch_cnt = wsi("sing.wcc", chunks); if (e) return e;
  A.wch_off = wsi("sing.wco", chunks + 1); if (e) return e;
  A.ucell = wsi("sing.ucell", 2 * (size_t)cap); if (e) return e;
  A.ebits = (unsigned short*)ctx->ws("sing.bits", sizeof(unsigned short) * (size_t)P, st, &e);
  if (e) return e;
  A.xpre = wsi("sing.xpre", 2 * (size_t)P); if (e) return e;
  A.ckey = (long long*)ctx->ws("sing.ckey", sizeof(long long) * cap, st, &e);
  if (e) return e;
  A.cpos = out->cross_pos; A.ck = out->cross_k; A.ce = out->cross_e; A.cg = out->cross_g; A.cfl = out->cross_flags;
  A.sa = out->seg_a; A.sb = out->seg_b; A.sk = out->seg_k;
  A.upos = out->umb_pos; A.ukap = out->umb_kappa; A.ustat = out->umb_status;
  A.wpos = out->swt_pos; A.wk = out->swt_k; A.we = out->swt_e; A.wseg = out->swt_seg; A.wstat = out->swt_status;
  A.counts = out->counts;
  ctx->cur_stream = st;
  return ctx->hip(lf::launch_sing(A, ctx->n_cu > 0 ? ctx->n_cu : 256, st, lf_prof_mark, ctx),
                  "singularity-map kernels");
}
