// lf_find_images (triangle-mapping finder), lf_multiplane_trace (multi-plane recursion),
// lf_find_images_mp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "lf_api_internal.h"
#include "lf_find.h"

namespace {

bool grid_ok(const lf_grid* g) {
  return g && g->nx >= 2 && g->ny >= 2 && g->h > 0 && std::isfinite(g->h) && std::isfinite(g->x0) &&
         std::isfinite(g->y0) && (long long)(g->nx - 1) * (g->ny - 1) * 2 < (1LL << 32);
}

lf::MapsOut alpha_psi_out(double* base, long long P, bool psi) {
  lf::MapsOut o;
  std::memset(&o, 0, sizeof o);
  o.ax = base;
  o.ay = base + P;
  if (psi) { o.p11 = base + 2 * P; o.p12 = base + 3 * P; o.p22 = base + 4 * P; }
  return o;
}

// Deflection (and deformation tensor) of one plane at points; heavy + lean passes.
lf_status plane_sum(lf_ctx* ctx, const lf_model* M, const double* params, const lf::PointsSpec& ps, bool mixed,
                    const lf::MapsOut& o, const char* tag, hipStream_t st, lf::Plane64* keep) {
  lf::MainRec* mains; lf::MulRec* muls; lf::MemRec32* m32; lf::MemRec64* m64;
  lf_status e = lf_expand_tables(ctx, M, params, 1, true, st, &mains, &muls, &m32, &m64, tag);
  if (e) return e;
  lf::DevModel dm = lf_dev_model(M);
  if (keep) { keep->mains = mains; keep->n_main = dm.n_main; keep->mem = m64; keep->seg = dm.seg; }
  double* part = nullptr;
  if (lf::has_heavy(dm)) {
    part = (double*)ctx->ws("plane.part", (size_t)ps.P * (sizeof(double) * 9 + sizeof(int)), st, &e);
    if (e) return e;
    ctx->prof_begin("maps_heavy", st);
    hipError_t he = lf::launch_maps(dm, mains, m32, m64, 1, ps, 1.0, mixed, false, o, lf_quad(ctx), 1, part, 1, st);
    ctx->prof_end(st);
    if (he != hipSuccess) return ctx->hip(he, "plane heavy pass");
  }
  ctx->prof_begin("maps_lean", st);
  hipError_t he = lf::launch_maps(dm, mains, m32, m64, 1, ps, 1.0, mixed, false, o, lf_quad(ctx),
                                  ctx->maps_ppl(mixed, false), part, 2, st);
  ctx->prof_end(st);
  return ctx->hip(he, "plane lean pass");
}

// Candidate capacity: max(LF_FIND_CAP_MIN, LF_FIND_CAP_PER_SRC n_src), or the context's
// (LF_FIND_CAND_CAP at lf_init), at most 2^28.  F.n_src must be set.
lf_status finder_buffers(lf_ctx* ctx, hipStream_t st, lf::FindArgs& F) {
  lf_status e = LF_OK;
  long long cap = ctx->find_cap > 0 ? ctx->find_cap
                                    : std::max<long long>(LF_FIND_CAP_MIN, (long long)LF_FIND_CAP_PER_SRC * F.n_src);
  F.cap = (int)std::min<long long>(cap, 1LL << 28);
  F.n_cu = ctx->n_cu > 0 ? ctx->n_cu : 256;
  F.cand_raw = (unsigned long long*)ctx->ws("find.craw", sizeof(unsigned long long) * F.cap, st, &e); if (e) return e;
  F.cand = (unsigned long long*)ctx->ws("find.cand", sizeof(unsigned long long) * F.cap, st, &e); if (e) return e;
  F.n_cand = (int*)ctx->ws("find.ncand", 64, st, &e); if (e) return e;
  F.src_cnt = (int*)ctx->ws("find.scnt", sizeof(int) * F.n_src, st, &e); if (e) return e;
  F.src_off = (int*)ctx->ws("find.soff", sizeof(int) * (F.n_src + 1), st, &e); if (e) return e;
  F.src_cur = (int*)ctx->ws("find.scur", sizeof(int) * F.n_src, st, &e); if (e) return e;
  F.c_status = (int*)ctx->ws("find.status", sizeof(int) * F.cap, st, &e); if (e) return e;
  F.c_theta = (double*)ctx->ws("find.theta", sizeof(double) * 2 * F.cap, st, &e); if (e) return e;
  F.c_mu = (double*)ctx->ws("find.mu", sizeof(double) * F.cap, st, &e); if (e) return e;
  return LF_OK;
}

bool planes_ok(lf_ctx* ctx, const lf_model* const* planes, const double* zp, int n, const lf_cosmo* cosmo) {
  if (!planes || !zp || n < 1 || n > LF_MAX_PLANES || !cosmo) return false;
  for (int j = 0; j < n; ++j) {
    if (!planes[j] || planes[j]->n_free != 0 || !(zp[j] > 0) || !std::isfinite(zp[j])) return false;
    if (j > 0 && !(zp[j] >= zp[j - 1])) return false;
  }
  (void)ctx;
  return true;
}

void plane_ratios(const lf_cosmo* c, const double* zp, int N, double* wij) {
  for (int k = 0; k < LF_MAX_PLANES * LF_MAX_PLANES; ++k) wij[k] = 0.0;
  for (int j = 0; j < N; ++j) {
    double Dj;
    lf_cosmo_dist(c, 0.0, zp[j], &Dj);
    for (int i = 0; i < j; ++i) {
      double Dij = 0.0;
      if (zp[j] > zp[i]) lf_cosmo_dist(c, zp[i], zp[j], &Dij);
      wij[i * LF_MAX_PLANES + j] = Dij / Dj;
    }
  }
}
void source_ratios(const lf_cosmo* c, const double* zp, int N, double zs, double* w) {
  double Ds;
  lf_cosmo_dist(c, 0.0, zs, &Ds);
  for (int j = 0; j < LF_MAX_PLANES; ++j) w[j] = 0.0;
  for (int j = 0; j < N; ++j) {
    if (!(zp[j] < zs)) continue;
    double Djs;
    lf_cosmo_dist(c, zp[j], zs, &Djs);
    w[j] = Djs / Ds;
  }
}

// Trace all planes at the points: per-plane alpha, psi at theta_j into M.al (and tables).
lf_status trace_planes(lf_ctx* ctx, const lf_model* const* planes, int N, const lf::PointsSpec& ps, bool mixed,
                       hipStream_t st, lf::MPArgs& M, lf::LensDev* L) {
  lf_status e = LF_OK;
  long long P = ps.P;
  M.P = P;
  M.grid = ps.grid; M.x0 = ps.x0; M.y0 = ps.y0; M.h = ps.h; M.nx = ps.nx; M.px = ps.px; M.py = ps.py;
  M.n_planes = N;
  M.al = (double*)ctx->ws("mp.al", sizeof(double) * 5 * (size_t)N * P, st, &e); if (e) return e;
  M.tx = (double*)ctx->ws("mp.tx", sizeof(double) * (size_t)P, st, &e); if (e) return e;
  M.ty = (double*)ctx->ws("mp.ty", sizeof(double) * (size_t)P, st, &e); if (e) return e;
  for (int j = 0; j < N; ++j) {
    hipError_t he = lf::launch_mp_theta(M, j, st);
    if (he != hipSuccess) return ctx->hip(he, "multi-plane theta_j");
    lf::PointsSpec pj;
    pj.grid = 0; pj.px = M.tx; pj.py = M.ty; pj.P = P; pj.p0 = 0; pj.x0 = pj.y0 = pj.h = 0; pj.nx = pj.ny = 0;
    std::string tag = "mp" + std::to_string(j);
    lf::Plane64 keep;
    e = plane_sum(ctx, planes[j], nullptr, pj, mixed, alpha_psi_out(M.al + (size_t)5 * j * P, P, true), tag.c_str(),
                  st, &keep);
    if (e) return e;
    if (L) L->pl[j] = keep;
  }
  return LF_OK;
}

}  // namespace

extern "C" lf_status lf_find_images(lf_ctx* ctx, const lf_model* M, const double* params, const double* beta,
                                    const double* a_src, int32_t n_src, const lf_grid* grid, int32_t max_img,
                                    lf_prec prec, double* theta_out, double* mu_out, int32_t* count_out,
                                    int32_t* flags, void* stream) {
  if (!ctx) return LF_E_INVALID_ARG;
  if (!M || !beta || !a_src || !theta_out || !count_out) return ctx->fail(LF_E_INVALID_ARG, "null argument");
  if (n_src < 1 || max_img < 1) return ctx->fail(LF_E_INVALID_ARG, "n_src and max_img must be >= 1");
  if (!grid_ok(grid)) return ctx->fail(LF_E_INVALID_ARG, "bad grid (need nx, ny >= 2, h > 0)");
  if (M->n_free > 0 && !params) return ctx->fail(LF_E_INVALID_ARG, "model has free fields: params required");
  if (prec != LF_PREC_FP64 && prec != LF_PREC_MIXED) return ctx->fail(LF_E_INVALID_ARG, "bad precision");
  hipSetDevice(ctx->device);
  hipStream_t st = (hipStream_t)stream;
  bool mixed = prec == LF_PREC_MIXED;
  lf::PointsSpec ps;
  lf_points pts;
  pts.grid = *grid; pts.px = pts.py = nullptr; pts.n = 0;
  lf_points_spec(&pts, ps);
  lf_status e = LF_OK;
  double* va = (double*)ctx->ws("find.va", sizeof(double) * 2 * (size_t)ps.P, st, &e);
  if (e) return e;
  lf::LensDev L;
  std::memset(&L, 0, sizeof L);
  L.n_planes = 1;
  L.enfw = lf_model_has_enfw(M) ? 1 : 0;
  e = plane_sum(ctx, M, params, ps, mixed, alpha_psi_out(va, ps.P, false), "find", st, &L.pl[0]);
  if (e) return e;
  lf::QuadTab q = lf_quad(ctx);
  L.qd.n = q.n; L.qd.u = q.u; L.qd.w = q.w;
  lf::FindArgs F;
  F.x0 = grid->x0; F.y0 = grid->y0; F.h = grid->h; F.nx = grid->nx; F.ny = grid->ny;
  F.n_planes = 1; F.va_pstride = 0; F.vax = va; F.vay = va + ps.P;
  F.n_src = n_src; F.beta = beta; F.w = a_src;
  F.eps = mixed ? 5e-5 : 1e-9;
  F.max_img = max_img; F.theta_out = theta_out; F.mu_out = mu_out; F.count_out = count_out; F.flags_out = flags;
  e = finder_buffers(ctx, st, F);
  if (e) return e;
  ctx->cur_stream = st;
  return ctx->hip(lf::launch_find(F, L, st, lf_prof_mark, ctx), "finder kernels");
}

extern "C" lf_status lf_find_images_alpha(lf_ctx* ctx, const lf_model* M, const double* params,
                                          const double* alpha_x, const double* alpha_y, const double* beta,
                                          const double* a_src, int32_t n_src, const lf_grid* grid, int32_t max_img,
                                          lf_prec prec, double* theta_out, double* mu_out, int32_t* count_out,
                                          int32_t* flags, void* stream) {
  if (!ctx) return LF_E_INVALID_ARG;
  if (!M || !alpha_x || !alpha_y || !beta || !a_src || !theta_out || !count_out)
    return ctx->fail(LF_E_INVALID_ARG, "null argument");
  if (n_src < 1 || max_img < 1) return ctx->fail(LF_E_INVALID_ARG, "n_src and max_img must be >= 1");
  if (!grid_ok(grid)) return ctx->fail(LF_E_INVALID_ARG, "bad grid (need nx, ny >= 2, h > 0)");
  if (M->n_free > 0 && !params) return ctx->fail(LF_E_INVALID_ARG, "model has free fields: params required");
  if (prec != LF_PREC_FP64 && prec != LF_PREC_MIXED) return ctx->fail(LF_E_INVALID_ARG, "bad precision");
  hipSetDevice(ctx->device);
  hipStream_t st = (hipStream_t)stream;
  // the FP64 tables of the sample for containment and polishing; the vertex deflections are the
  // caller's map
  lf::MainRec* mains; lf::MulRec* muls; lf::MemRec32* m32; lf::MemRec64* m64;
  lf_status e = lf_expand_tables(ctx, M, params, 1, true, st, &mains, &muls, &m32, &m64, "find");
  if (e) return e;
  lf::DevModel dm = lf_dev_model(M);
  lf::LensDev L;
  std::memset(&L, 0, sizeof L);
  L.n_planes = 1;
  L.enfw = lf_model_has_enfw(M) ? 1 : 0;
  L.pl[0].mains = mains; L.pl[0].n_main = dm.n_main; L.pl[0].mem = m64; L.pl[0].seg = dm.seg;
  lf::QuadTab q = lf_quad(ctx);
  L.qd.n = q.n; L.qd.u = q.u; L.qd.w = q.w;
  lf::FindArgs F;
  F.x0 = grid->x0; F.y0 = grid->y0; F.h = grid->h; F.nx = grid->nx; F.ny = grid->ny;
  F.n_planes = 1; F.va_pstride = 0; F.vax = alpha_x; F.vay = alpha_y;
  F.n_src = n_src; F.beta = beta; F.w = a_src;
  F.eps = prec == LF_PREC_MIXED ? 5e-5 : 1e-9;
  F.max_img = max_img; F.theta_out = theta_out; F.mu_out = mu_out; F.count_out = count_out; F.flags_out = flags;
  e = finder_buffers(ctx, st, F);
  if (e) return e;
  ctx->cur_stream = st;
  return ctx->hip(lf::launch_find(F, L, st, lf_prof_mark, ctx), "finder kernels");
}

extern "C" lf_status lf_find_images_ms(lf_ctx* ctx, const lf_model* M, const double* params, const double* beta,
                                       const double* a_src, int32_t n_src, const lf_grid* grid, int32_t max_img,
                                       lf_prec prec, int32_t polish, double* theta_out, double* mu_out,
                                       int32_t* count_out, int32_t* flags, void* stream) {
  if (!ctx) return LF_E_INVALID_ARG;
  if (!M || !beta || !a_src || !theta_out || !count_out) return ctx->fail(LF_E_INVALID_ARG, "null argument");
  if (n_src < 1 || max_img < 1) return ctx->fail(LF_E_INVALID_ARG, "n_src and max_img must be >= 1");
  if (!grid_ok(grid) || (long long)(grid->nx - 1) * (grid->ny - 1) * 4 >= (1LL << 32))
    return ctx->fail(LF_E_INVALID_ARG, "bad grid (need nx, ny >= 2, h > 0, fewer than 2^30 cells)");
  if (M->n_free > 0 && !params) return ctx->fail(LF_E_INVALID_ARG, "model has free fields: params required");
  if (prec != LF_PREC_FP64 && prec != LF_PREC_MIXED) return ctx->fail(LF_E_INVALID_ARG, "bad precision");
  hipSetDevice(ctx->device);
  hipStream_t st = (hipStream_t)stream;
  lf::PointsSpec ps;
  lf_points pts;
  pts.grid = *grid; pts.px = pts.py = nullptr; pts.n = 0;
  lf_points_spec(&pts, ps);
  lf_status e = LF_OK;
  double* va = (double*)ctx->ws("find.va", sizeof(double) * 2 * (size_t)ps.P, st, &e);
  if (e) return e;
  lf::LensDev L;
  std::memset(&L, 0, sizeof L);
  L.n_planes = 1;
  L.enfw = lf_model_has_enfw(M) ? 1 : 0;
  e = plane_sum(ctx, M, params, ps, prec == LF_PREC_MIXED, alpha_psi_out(va, ps.P, false), "find", st, &L.pl[0]);
  if (e) return e;
  lf::QuadTab q = lf_quad(ctx);
  L.qd.n = q.n; L.qd.u = q.u; L.qd.w = q.w;
  lf::FindArgs F;
  std::memset(&F, 0, sizeof F);
  F.x0 = grid->x0; F.y0 = grid->y0; F.h = grid->h; F.nx = grid->nx; F.ny = grid->ny;
  F.n_planes = 1; F.va_pstride = 0; F.vax = va; F.vay = va + ps.P;
  F.n_src = n_src; F.beta = beta; F.w = a_src;
  F.max_img = max_img; F.theta_out = theta_out; F.mu_out = mu_out; F.count_out = count_out; F.flags_out = flags;
  e = finder_buffers(ctx, st, F);
  if (e) return e;
  ctx->cur_stream = st;
  return ctx->hip(lf::launch_find_ms(F, L, polish ? 1 : 0, st, lf_prof_mark, ctx), "contour finder kernels");
}

extern "C" lf_status lf_multiplane_trace(lf_ctx* ctx, const lf_model* const* planes, const double* z_planes,
                                         int32_t n_planes, const lf_cosmo* cosmo, const double* z_src, int32_t n_zs,
                                         const lf_points* pts, lf_prec prec, double* beta_out, double* A_out,
                                         double* mu_out, void* stream) {
  if (!ctx) return LF_E_INVALID_ARG;
  if (!planes_ok(ctx, planes, z_planes, n_planes, cosmo))
    return ctx->fail(LF_E_INVALID_ARG, "planes: 1..%d models without free fields, sorted by z > 0", LF_MAX_PLANES);
  if (n_zs < 1 || !z_src) return ctx->fail(LF_E_INVALID_ARG, "need at least one source redshift");
  for (int k = 0; k < n_zs; ++k)
    if (!(z_src[k] > 0) || !std::isfinite(z_src[k])) return ctx->fail(LF_E_INVALID_ARG, "bad source redshift");
  if (!beta_out && !A_out && !mu_out) return ctx->fail(LF_E_INVALID_ARG, "no output requested");
  if (prec != LF_PREC_FP64 && prec != LF_PREC_MIXED) return ctx->fail(LF_E_INVALID_ARG, "bad precision");
  lf::PointsSpec ps;
  if (!lf_points_spec(pts, ps)) return ctx->fail(LF_E_INVALID_ARG, "bad points");
  hipSetDevice(ctx->device);
  hipStream_t st = (hipStream_t)stream;
  lf::MPArgs M;
  std::memset(&M, 0, sizeof M);
  plane_ratios(cosmo, z_planes, n_planes, M.wij);
  std::vector<double> wjs((size_t)n_zs * LF_MAX_PLANES);
  for (int k = 0; k < n_zs; ++k) source_ratios(cosmo, z_planes, n_planes, z_src[k], &wjs[(size_t)k * LF_MAX_PLANES]);
  lf_status e = LF_OK;
  double* d_wjs = (double*)ctx->ws("mp.wjs", sizeof(double) * wjs.size(), st, &e);
  if (e) return e;
  hipMemcpyAsync(d_wjs, wjs.data(), sizeof(double) * wjs.size(), hipMemcpyHostToDevice, st);
  e = trace_planes(ctx, planes, n_planes, ps, prec == LF_PREC_MIXED, st, M, nullptr);
  if (e) return e;
  M.n_zs = n_zs; M.wjs = d_wjs; M.beta = beta_out; M.A = A_out; M.mu = mu_out;
  ctx->prof_begin("mp_final", st);
  hipError_t he = lf::launch_mp_final(M, st);
  ctx->prof_end(st);
  hipError_t se = hipStreamSynchronize(st);   // the weight table above is host memory
  if (he != hipSuccess) return ctx->hip(he, "multi-plane final pass");
  return ctx->hip(se, "multi-plane sync");
}

extern "C" lf_status lf_find_images_mp(lf_ctx* ctx, const lf_model* const* planes, const double* z_planes,
                                       int32_t n_planes, const lf_cosmo* cosmo, const double* beta,
                                       const double* z_src, int32_t n_src, const lf_grid* grid, int32_t max_img,
                                       lf_prec prec, double* theta_out, double* mu_out, int32_t* count_out,
                                       int32_t* flags, void* stream) {
  if (!ctx) return LF_E_INVALID_ARG;
  if (!planes_ok(ctx, planes, z_planes, n_planes, cosmo))
    return ctx->fail(LF_E_INVALID_ARG, "planes: 1..%d models without free fields, sorted by z > 0", LF_MAX_PLANES);
  if (!beta || !z_src || !theta_out || !count_out) return ctx->fail(LF_E_INVALID_ARG, "null argument");
  if (n_src < 1 || max_img < 1) return ctx->fail(LF_E_INVALID_ARG, "n_src and max_img must be >= 1");
  if (!grid_ok(grid)) return ctx->fail(LF_E_INVALID_ARG, "bad grid (need nx, ny >= 2, h > 0)");
  for (int s = 0; s < n_src; ++s)
    if (!(z_src[s] > 0) || !std::isfinite(z_src[s])) return ctx->fail(LF_E_INVALID_ARG, "bad source redshift");
  if (prec != LF_PREC_FP64 && prec != LF_PREC_MIXED) return ctx->fail(LF_E_INVALID_ARG, "bad precision");
  hipSetDevice(ctx->device);
  hipStream_t st = (hipStream_t)stream;
  bool mixed = prec == LF_PREC_MIXED;
  lf::PointsSpec ps;
  lf_points pts;
  pts.grid = *grid; pts.px = pts.py = nullptr; pts.n = 0;
  lf_points_spec(&pts, ps);
  lf::MPArgs M;
  std::memset(&M, 0, sizeof M);
  plane_ratios(cosmo, z_planes, n_planes, M.wij);
  lf::LensDev L;
  std::memset(&L, 0, sizeof L);
  L.n_planes = n_planes;
  for (int j = 0; j < n_planes; ++j) L.enfw |= lf_model_has_enfw(planes[j]) ? 1 : 0;
  std::memcpy(L.wij, M.wij, sizeof L.wij);
  lf::QuadTab q = lf_quad(ctx);
  L.qd.n = q.n; L.qd.u = q.u; L.qd.w = q.w;
  lf_status e = trace_planes(ctx, planes, n_planes, ps, mixed, st, M, &L);
  if (e) return e;
  std::vector<double> w((size_t)n_src * n_planes);
  for (int s = 0; s < n_src; ++s) {
    double ws[LF_MAX_PLANES];
    source_ratios(cosmo, z_planes, n_planes, z_src[s], ws);
    for (int j = 0; j < n_planes; ++j) w[(size_t)s * n_planes + j] = ws[j];
  }
  double* d_w = (double*)ctx->ws("findmp.w", sizeof(double) * w.size(), st, &e);
  if (e) return e;
  hipMemcpyAsync(d_w, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice, st);
  lf::FindArgs F;
  F.x0 = grid->x0; F.y0 = grid->y0; F.h = grid->h; F.nx = grid->nx; F.ny = grid->ny;
  F.n_planes = n_planes; F.va_pstride = 5 * M.P; F.vax = M.al; F.vay = M.al + M.P;
  F.n_src = n_src; F.beta = beta; F.w = d_w;
  F.eps = mixed ? 5e-5 : 1e-9;
  F.max_img = max_img; F.theta_out = theta_out; F.mu_out = mu_out; F.count_out = count_out; F.flags_out = flags;
  e = finder_buffers(ctx, st, F);
  if (e) return e;
  ctx->cur_stream = st;
  hipError_t he = lf::launch_find(F, L, st, lf_prof_mark, ctx);
  hipError_t se = hipStreamSynchronize(st);   // the weight table above is host memory
  if (he != hipSuccess) return ctx->hip(he, "finder kernels");
  return ctx->hip(se, "finder sync");
}
