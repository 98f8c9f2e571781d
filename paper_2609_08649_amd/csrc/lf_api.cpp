// Host runtime and C ABI of the lensfield library (see include/lensfield.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lensfield.h"
#include "lf_api_internal.h"

using namespace lf;

// ------------------------------------------------------------------------------ errors
lf_status lf_ctx::fail(lf_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  last_error = buf;
  return st;
}
lf_status lf_ctx::hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return LF_OK;
  return fail(LF_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ------------------------------------------------------------------------------ workspace
void* lf_ctx::ws(const char* name, size_t bytes, hipStream_t st, lf_status* err) {
  if (arena) {
    // allocation-free call: consecutive 256-byte aligned slices of the caller-held scratch
    const size_t at = (arena->used + 255) & ~(size_t)255;
    if (at + bytes > arena->cap) {
      *err = fail(LF_E_OUT_OF_BUDGET, "%s: workspace %s does not fit the static scratch (needs %zu bytes from "
                  "offset %zu; the scratch holds %zu)", arena->who, name, bytes, at, arena->cap);
      return nullptr;
    }
    arena->used = at + bytes;
    return arena->base + at;
  }
  Buf& b = bufs[name];
  if (b.bytes >= bytes && b.ptr) return b.ptr;
  size_t want = std::max(bytes, b.bytes + b.bytes / 2);
  if (b.ptr) {
    hipStreamSynchronize(st);
    hipFree(b.ptr);
    dev_bytes -= b.bytes;
    b.ptr = nullptr;
    b.bytes = 0;
  }
  if (dev_bytes + want > budget) want = bytes;
  if (dev_bytes + want > budget) {
    *err = fail(LF_E_OUT_OF_BUDGET, "workspace %s needs %zu bytes; budget %zu, in use %zu", name, want,
                budget, dev_bytes);
    return nullptr;
  }
  hipError_t e = hipMalloc(&b.ptr, want);
  if (e != hipSuccess) {
    b.ptr = nullptr;
    *err = hip(e, "hipMalloc(workspace)");
    return nullptr;
  }
  b.bytes = want;
  dev_bytes += want;
  return b.ptr;
}

lf_status lf_ctx::dmalloc(void** p, size_t bytes) {
  if (dev_bytes + bytes > budget)
    return fail(LF_E_OUT_OF_BUDGET, "allocation of %zu bytes exceeds budget %zu (in use %zu)", bytes,
                budget, dev_bytes);
  hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 16));
  if (e != hipSuccess) return hip(e, "hipMalloc");
  dev_bytes += bytes;
  return LF_OK;
}
void lf_ctx::dfree(void* p, size_t bytes) {
  if (p) { hipFree(p); dev_bytes -= bytes; }
}

// ------------------------------------------------------------------------------ kernel timing
hipEvent_t lf_ctx::prof_ev() {
  if (!ev_pool.empty()) { hipEvent_t e = ev_pool.back(); ev_pool.pop_back(); return e; }
  hipEvent_t e;
  hipEventCreate(&e);
  return e;
}
void lf_ctx::prof_begin(const char* name, hipStream_t st) {
  if (!prof) return;
  prof_skip = !prof_only.empty() && prof_only != name;
  if (prof_skip) return;
  Rec r;
  r.name = name; r.a = prof_ev(); r.b = nullptr;
  hipEventRecord(r.a, st);
  prof_pending.push_back(r);
}
void lf_ctx::prof_end(hipStream_t st) {
  if (prof_skip) { prof_skip = false; return; }
  if (!prof || prof_pending.empty() || prof_pending.back().b) return;
  prof_pending.back().b = prof_ev();
  hipEventRecord(prof_pending.back().b, st);
}
void lf_ctx::prof_flush() {
  for (auto& r : prof_pending) {
    if (r.b) {
      hipEventSynchronize(r.b);
      float ms = 0.f;
      hipEventElapsedTime(&ms, r.a, r.b);
      auto& t = prof_tally[r.name];
      t.first += ms;
      t.second += 1;
      ev_pool.push_back(r.b);
    }
    ev_pool.push_back(r.a);
  }
  prof_pending.clear();
}
extern "C" lf_status lf_profile_enable(lf_ctx* ctx, int32_t on) {
  if (!ctx) return LF_E_INVALID_ARG;
  ctx->prof_flush();
  ctx->prof = on != 0;
  return LF_OK;
}
extern "C" lf_status lf_profile_only(lf_ctx* ctx, const char* kernel) {
  if (!ctx) return LF_E_INVALID_ARG;
  ctx->prof_only = kernel ? kernel : "";
  return LF_OK;
}
extern "C" lf_status lf_profile_read(lf_ctx* ctx, const char* kernel, double* total_ms, int64_t* launches) {
  if (!ctx || !kernel || !total_ms || !launches) return LF_E_INVALID_ARG;
  ctx->prof_flush();
  auto it = ctx->prof_tally.find(kernel);
  *total_ms = it == ctx->prof_tally.end() ? 0.0 : it->second.first;
  *launches = it == ctx->prof_tally.end() ? 0 : it->second.second;
  return LF_OK;
}
extern "C" lf_status lf_profile_reset(lf_ctx* ctx) {
  if (!ctx) return LF_E_INVALID_ARG;
  ctx->prof_flush();
  ctx->prof_tally.clear();
  return LF_OK;
}

// ------------------------------------------------------------------------------ cosmology
// Flat LCDM distances by adaptive Simpson quadrature of 1/E(z).
namespace {
const double C_KMS = 299792.458;
const double G_MPC = 4.30091727e-9;
const double ARCSEC = 206264.80624709636;
const double PI_D = 3.14159265358979323846;

double invE(double z, double Om) { double a = 1 + z; return 1.0 / std::sqrt(Om * a * a * a + (1 - Om)); }
double simpson(double a, double b, double fa, double fm, double fb, double whole, double tol, int depth,
               double Om) {
  double m = 0.5 * (a + b), lm = 0.5 * (a + m), rm = 0.5 * (m + b);
  double flm = invE(lm, Om), frm = invE(rm, Om);
  double left = (m - a) / 6 * (fa + 4 * flm + fm), right = (b - m) / 6 * (fm + 4 * frm + fb);
  double diff = left + right - whole;
  if (depth > 45 || std::fabs(diff) <= 15 * tol) return left + right + diff / 15;
  return simpson(a, m, fa, flm, fm, left, 0.5 * tol, depth + 1, Om) +
         simpson(m, b, fm, frm, fb, right, 0.5 * tol, depth + 1, Om);
}
double comoving_mpc(double z1, double z2, double H0, double Om) {
  if (z1 == z2) return 0.0;
  double fa = invE(z1, Om), fb = invE(z2, Om), fm = invE(0.5 * (z1 + z2), Om);
  double whole = (z2 - z1) / 6 * (fa + 4 * fm + fb);
  return C_KMS / H0 * simpson(z1, z2, fa, fm, fb, whole, 1e-14 * std::fabs(z2 - z1), 0, Om);
}
double dist_mpc(double z1, double z2, double H0, double Om) { return comoving_mpc(z1, z2, H0, Om) / (1 + z2); }
bool cosmo_ok(const lf_cosmo* c) {
  return c && std::isfinite(c->H0) && c->H0 > 0 && std::isfinite(c->Om) && c->Om >= 0 && c->Om <= 1;
}

// Gauss-Legendre nodes on [-1, 1] by Newton iteration on the three-term recurrence.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n); w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(PI_D * (i + 0.75) / (n + 0.5)), dp = 0;
    for (int it = 0; it < 60; ++it) {
      double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) { double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k; p0 = p1; p1 = p2; }
      dp = n * (z * p1 - p0) / (z * z - 1);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z; w[i] = 2.0 / ((1 - z * z) * dp * dp);
  }
}
}  // namespace

// ------------------------------------------------------------------------------ context
extern "C" lf_status lf_init(lf_ctx** out, int32_t device, size_t hbm_budget_bytes) {
  if (!out) return LF_E_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return LF_E_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return LF_E_DEVICE;
  lf_ctx* c = new lf_ctx();
  c->device = device;
  size_t fr = 0, tot = 0;
  hipMemGetInfo(&fr, &tot);
  c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)fr);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    c->n_cu = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
  }
  if (const char* fc = std::getenv("LF_FIND_CAND_CAP")) c->find_cap = std::max(1LL, std::atoll(fc));
  // eNFW quadrature: Gauss-Legendre in t on [0, 1] with u = t^6 (weights carry du/dt)
  std::vector<double> x, w;
  gauss_legendre(LF_ENFW_NODES, x, w);
  std::vector<double> hu(LF_ENFW_NODES), hw(LF_ENFW_NODES);
  for (int i = 0; i < LF_ENFW_NODES; ++i) {
    double t = 0.5 * (x[i] + 1.0), wt = 0.5 * w[i];
    hu[i] = std::pow(t, 6);
    hw[i] = wt * 6.0 * std::pow(t, 5);
  }
  if (c->dmalloc((void**)&c->quad_u, sizeof(double) * LF_ENFW_NODES) != LF_OK ||
      c->dmalloc((void**)&c->quad_w, sizeof(double) * LF_ENFW_NODES) != LF_OK) {
    delete c;
    return LF_E_DEVICE;
  }
  hipMemcpy(c->quad_u, hu.data(), sizeof(double) * LF_ENFW_NODES, hipMemcpyHostToDevice);
  hipMemcpy(c->quad_w, hw.data(), sizeof(double) * LF_ENFW_NODES, hipMemcpyHostToDevice);
  // address of this device's static scratch (allocation-free entry point), with the device current
  if (lf_noalloc_setup(c) != LF_OK) {
    lf_shutdown(c);
    return LF_E_DEVICE;
  }
  *out = c;
  return LF_OK;
}

extern "C" lf_status lf_shutdown(lf_ctx* ctx) {
  if (!ctx) return LF_E_INVALID_ARG;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  ctx->prof_flush();
  for (auto e : ctx->ev_pool) hipEventDestroy(e);
  for (auto& kv : ctx->bufs) if (kv.second.ptr) hipFree(kv.second.ptr);
  if (ctx->quad_u) hipFree(ctx->quad_u);
  if (ctx->quad_w) hipFree(ctx->quad_w);
  delete ctx;
  return LF_OK;
}

extern "C" const char* lf_last_error(const lf_ctx* ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }
extern "C" size_t lf_device_bytes(const lf_ctx* ctx) { return ctx ? ctx->dev_bytes : 0; }

// ------------------------------------------------------------------------------ cosmology ABI
extern "C" lf_status lf_cosmo_dist(const lf_cosmo* c, double z1, double z2, double* out) {
  if (!cosmo_ok(c) || !out || !(z1 >= 0) || !(z2 >= z1) || !std::isfinite(z2)) return LF_E_INVALID_ARG;
  *out = dist_mpc(z1, z2, c->H0, c->Om);
  return LF_OK;
}
extern "C" lf_status lf_cosmo_adis(const lf_cosmo* c, double zd, double zs, double* out) {
  if (!cosmo_ok(c) || !out || !(zd >= 0) || !(zs > zd) || !std::isfinite(zs)) return LF_E_INVALID_ARG;
  *out = dist_mpc(zd, zs, c->H0, c->Om) / dist_mpc(0, zs, c->H0, c->Om);
  return LF_OK;
}
extern "C" lf_status lf_cosmo_tdscale(const lf_cosmo* c, double zd, double zs, double* out) {
  if (!cosmo_ok(c) || !out || !(zd > 0) || !(zs > zd) || !std::isfinite(zs)) return LF_E_INVALID_ARG;
  const double MPC_M = 3.0856775814913673e22, C_MS = C_KMS * 1e3, DAY = 86400.0, th0 = 1.0 / ARCSEC;
  const double Dd = dist_mpc(0, zd, c->H0, c->Om), Ds = dist_mpc(0, zs, c->H0, c->Om);
  const double Dds = dist_mpc(zd, zs, c->H0, c->Om);
  *out = (1.0 + zd) / C_MS * (Dd * Ds / Dds) * MPC_M * th0 * th0 / DAY;
  return LF_OK;
}
extern "C" lf_status lf_nfw_params(const lf_cosmo* c, double zd, double m200, double c200, double* ks,
                                   double* rs_arcsec) {
  if (!cosmo_ok(c) || !(zd > 0) || !(m200 > 0) || !(c200 > 0) || !ks || !rs_arcsec) return LF_E_INVALID_ARG;
  lf::XfConst xc = lf_xf_const(c, zd);
  double r200 = std::cbrt(3.0 * m200 / (4.0 * PI_D * 200.0 * xc.rho_c));
  double rs = r200 / c200;
  double dc = (200.0 / 3.0) * c200 * c200 * c200 / (std::log1p(c200) - c200 / (1.0 + c200));
  *ks = dc * xc.rho_c * rs / xc.sigma_cr;
  *rs_arcsec = rs / xc.Dd * ARCSEC;
  return LF_OK;
}

lf::XfConst lf_xf_const(const lf_cosmo* c, double zd) {
  lf::XfConst x;
  x.Dd = dist_mpc(0, zd, c->H0, c->Om);
  x.arcsec_per_kpc = 1e-3 / x.Dd * ARCSEC;
  double Hz = c->H0 * std::sqrt(c->Om * std::pow(1 + zd, 3) + 1 - c->Om);
  x.rho_c = 3 * Hz * Hz / (8 * PI_D * G_MPC);
  x.sigma_cr = C_KMS * C_KMS / (4 * PI_D * G_MPC * x.Dd);
  return x;
}

// ------------------------------------------------------------------------------ models
static bool bind_ok(const lf_binding& b, int n_free) {
  if (b.kind == LF_FIXED) return std::isfinite(b.value) && b.xform >= 0 && b.xform <= 6;
  if (b.kind == LF_FREE) return b.index >= 0 && b.index < n_free && b.xform >= 0 && b.xform <= 6;
  return false;
}
static lf::Bind to_bind(const lf_binding& b) {
  lf::Bind r;
  r.kind = b.kind; r.index = b.index; r.xf = b.xform; r.pad = 0; r.value = b.value;
  return r;
}

extern "C" lf_status lf_model_upload(lf_ctx* ctx, const lf_component* mainc, int32_t n_main,
                                     const lf_members* mem, double z_d, const lf_cosmo* cosmo,
                                     int32_t n_free, lf_model** out) {
  if (!ctx || !out) return LF_E_INVALID_ARG;
  *out = nullptr;
  if (n_main < 0 || (n_main > 0 && !mainc) || n_free < 0) return ctx->fail(LF_E_INVALID_ARG, "bad main components");
  if (!cosmo_ok(cosmo) || !(z_d > 0) || !std::isfinite(z_d)) return ctx->fail(LF_E_INVALID_ARG, "bad cosmology / z_d");
  int n_mem = mem ? mem->n : 0;
  if (n_mem < 0) return ctx->fail(LF_E_INVALID_ARG, "negative member count");
  for (int m = 0; m < n_main; ++m) {
    if (mainc[m].type < LF_POINT || mainc[m].type > LF_MPOLE3) return ctx->fail(LF_E_INVALID_ARG, "main %d: bad profile", m);
    for (int k = 0; k < 7; ++k)
      if (!bind_ok(mainc[m].f[k], n_free)) return ctx->fail(LF_E_INVALID_ARG, "main %d field %d: bad binding", m, k);
    bool m200 = mainc[m].f[2].xform == LF_XF_M200, c200 = mainc[m].f[5].xform == LF_XF_C200;
    if (m200 != c200) return ctx->fail(LF_E_INVALID_ARG, "main %d: M200 and C200 transforms come in pairs", m);
    if (m200 && mainc[m].type != LF_NFW && mainc[m].type != LF_ENFW)
      return ctx->fail(LF_E_INVALID_ARG, "main %d: M200/C200 only for NFW profiles", m);
  }
  lf_model* M = new lf_model();
  M->n_free = n_free;
  M->z_d = z_d;
  M->cosmo = *cosmo;
  M->xc = lf_xf_const(cosmo, z_d);
  for (int m = 0; m < n_main; ++m) {
    lf::MainDesc d;
    d.type = mainc[m].type; d.pad = 0;
    for (int k = 0; k < 7; ++k) d.f[k] = to_bind(mainc[m].f[k]);
    M->main.push_back(d);
  }
  lf::Bind unit = {LF_FIXED, 0, LF_XF_NONE, 0, 1.0};
  M->mul[0] = M->mul[1] = M->mul[2] = unit;
  std::vector<std::pair<int, lf::MemCat>> cat;
  if (n_mem > 0) {
    if (!mem->type || !mem->x || !mem->y || (!mem->lum && (!mem->b0 || !mem->s0 || !mem->a0))) {
      delete M;
      return ctx->fail(LF_E_INVALID_ARG, "members: missing arrays");
    }
    if (!bind_ok(mem->bmul, n_free) || !bind_ok(mem->smul, n_free) || !bind_ok(mem->amul, n_free)) {
      delete M;
      return ctx->fail(LF_E_INVALID_ARG, "members: bad multiplier binding");
    }
    M->mul[0] = to_bind(mem->bmul); M->mul[1] = to_bind(mem->smul); M->mul[2] = to_bind(mem->amul);
    for (int i = 0; i < n_mem; ++i) {
      lf::MemCat c;
      c.x = mem->x[i]; c.y = mem->y[i];
      c.q = mem->q ? mem->q[i] : 1.0;
      double pa = mem->pa ? mem->pa[i] : 0.0;
      c.c = std::cos(pa); c.sn = std::sin(pa);
      if (mem->lum) {
        double L = mem->lum[i];
        if (!(L > 0) || !std::isfinite(L)) { delete M; return ctx->fail(LF_E_INVALID_ARG, "member %d: bad luminosity", i); }
        c.fb = std::pow(L, 2 * mem->lam); c.fs = std::pow(L, mem->bet); c.fa = std::pow(L, mem->alp);
      } else {
        c.fb = mem->b0[i]; c.fs = mem->s0[i]; c.fa = mem->a0[i];
      }
      int t = mem->type[i];
      bool circ = c.q >= 1.0;
      if (!(c.q > 0 && c.q <= 1) || !std::isfinite(c.x) || !std::isfinite(c.y) || !(c.fb >= 0) || !(c.fs >= 0) ||
          !(c.fa >= 0) || !std::isfinite(pa)) {
        delete M;
        return ctx->fail(LF_E_INVALID_ARG, "member %d: field out of range", i);
      }
      int seg;
      switch (t) {
        case LF_PJE: seg = circ ? SEG_CPJE : SEG_EPJE; break;
        case LF_SIE: seg = circ ? SEG_CSIE : SEG_ESIE; break;
        case LF_SIS: seg = SEG_CSIE; c.fs = 0.0; c.q = 1.0; break;
        case LF_POINT: seg = SEG_POINT; break;
        case LF_NFW: seg = SEG_NFW; break;
        case LF_ENFW: seg = circ ? SEG_NFW : SEG_ENFW; break;
        default: delete M; return ctx->fail(LF_E_INVALID_ARG, "member %d: bad profile", i);
      }
      cat.push_back({seg, c});
    }
    std::stable_sort(cat.begin(), cat.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
  }
  for (int k = 0; k <= NSEG; ++k) M->seg.off[k] = 0;
  for (auto& e : cat) M->seg.off[e.first + 1]++;
  for (int k = 0; k < NSEG; ++k) M->seg.off[k + 1] += M->seg.off[k];
  for (auto& e : cat) M->mem.push_back(e.second);
  // device copies
  size_t bm = sizeof(lf::MainDesc) * std::max<size_t>(1, M->main.size());
  size_t bc = sizeof(lf::MemCat) * std::max<size_t>(1, M->mem.size());
  size_t b32 = sizeof(lf::MemCat32) * std::max<size_t>(1, M->mem.size());
  lf_status st = ctx->dmalloc((void**)&M->d_main, bm);
  if (st == LF_OK) { M->d_main_bytes = bm; st = ctx->dmalloc((void**)&M->d_mem, bc); }
  if (st == LF_OK) { M->d_mem_bytes = bc; st = ctx->dmalloc((void**)&M->d_cat32, b32); }
  if (st != LF_OK) { lf_model_release(ctx, M); return st; }
  M->d_cat32_bytes = b32;
  {
    std::vector<lf::MemCat32> c32(M->mem.size());
    for (size_t i = 0; i < M->mem.size(); ++i) {
      const lf::MemCat& c = M->mem[i];
      c32[i].xh = (float)c.x; c32[i].xl = (float)(c.x - (double)c32[i].xh);
      c32[i].yh = (float)c.y; c32[i].yl = (float)(c.y - (double)c32[i].yh);
      c32[i].fb = (float)c.fb; c32[i].fs = (float)c.fs; c32[i].fa = (float)c.fa;
      c32[i].q = (float)c.q; c32[i].c = (float)c.c; c32[i].sn = (float)c.sn;
      const double fk = lf::NEAR_K * c.fb / c.q;
      c32[i].fbk2 = (float)(fk * fk);
      c32[i].pad1 = 0.f;
    }
    if (!c32.empty()) hipMemcpy(M->d_cat32, c32.data(), sizeof(lf::MemCat32) * c32.size(), hipMemcpyHostToDevice);
  }
  if (!M->main.empty()) hipMemcpy(M->d_main, M->main.data(), sizeof(lf::MainDesc) * M->main.size(), hipMemcpyHostToDevice);
  if (!M->mem.empty()) hipMemcpy(M->d_mem, M->mem.data(), sizeof(lf::MemCat) * M->mem.size(), hipMemcpyHostToDevice);
  // a model whose fields are all fixed is validated now (expanded on the host side of the ABI)
  *out = M;
  return LF_OK;
}

extern "C" lf_status lf_model_release(lf_ctx* ctx, lf_model* m) {
  if (!ctx || !m) return LF_E_INVALID_ARG;
  ctx->dfree(m->d_main, m->d_main_bytes);
  ctx->dfree(m->d_mem, m->d_mem_bytes);
  ctx->dfree(m->d_cat32, m->d_cat32_bytes);
  delete m;
  return LF_OK;
}
extern "C" int32_t lf_model_n_halos(const lf_model* m) { return m ? (int32_t)(m->main.size() + m->mem.size()) : -1; }

lf::DevModel lf_dev_model(const lf_model* M) {
  lf::DevModel d;
  d.main = M->d_main; d.n_main = (int)M->main.size();
  d.mem = M->d_mem; d.n_mem = (int)M->mem.size();
  d.seg = M->seg;
  for (int k = 0; k < 3; ++k) d.mul[k] = M->mul[k];
  d.xc = M->xc;
  d.n_free = M->n_free;
  d.has_enfw = lf_model_has_enfw(M) ? 1 : 0;
  d.has_rare = 0;
  for (int k : {lf::SEG_EPJE, lf::SEG_ESIE, lf::SEG_POINT, lf::SEG_NFW, lf::SEG_ENFW})
    if (M->seg.off[k + 1] > M->seg.off[k]) d.has_rare = 1;
  return d;
}

lf::QuadTab lf_quad(const lf_ctx* ctx) {
  lf::QuadTab q;
  q.n = LF_ENFW_NODES; q.u = ctx->quad_u; q.w = ctx->quad_w;
  return q;
}

bool lf_model_has_enfw(const lf_model* M) {
  for (auto& d : M->main) if (d.type == LF_ENFW) return true;
  return M->seg.off[SEG_ENFW + 1] > M->seg.off[SEG_ENFW];
}

bool lf_points_spec(const lf_points* p, lf::PointsSpec& s) {
  if (!p) return false;
  if (p->px) {
    if (!p->py || p->n <= 0) return false;
    s.grid = 0; s.px = p->px; s.py = p->py; s.P = p->n; s.p0 = 0;
    s.x0 = s.y0 = s.h = 0; s.nx = s.ny = 0;
  } else {
    const lf_grid& g = p->grid;
    if (!(g.h > 0) || !std::isfinite(g.h) || !std::isfinite(g.x0) || !std::isfinite(g.y0) || g.nx <= 0 || g.ny <= 0)
      return false;
    s.grid = 1; s.x0 = g.x0; s.y0 = g.y0; s.h = g.h; s.nx = g.nx; s.ny = g.ny;
    s.px = s.py = nullptr; s.P = (long long)g.nx * g.ny; s.p0 = 0;
  }
  return true;
}

// Workspace tables for S expanded samples of a model (nothing is launched).
lf_status lf_expand_alloc(lf_ctx* ctx, const lf_model* M, int S, bool need_mem, hipStream_t st,
                          lf::MainRec** mains, lf::MulRec** muls, lf::MemRec32** m32, lf::MemRec64** m64,
                          const char* tag) {
  lf_status err = LF_OK;
  std::string t(tag);
  int nm = (int)M->main.size(), nb = (int)M->mem.size();
  *mains = (lf::MainRec*)ctx->ws((t + ".mains").c_str(), sizeof(lf::MainRec) * std::max(1, S * nm), st, &err);
  if (err) return err;
  *muls = (lf::MulRec*)ctx->ws((t + ".muls").c_str(), sizeof(lf::MulRec) * std::max(1, S), st, &err);
  if (err) return err;
  *m32 = nullptr; *m64 = nullptr;
  if (need_mem) {
    *m32 = (lf::MemRec32*)ctx->ws((t + ".m32").c_str(), std::max(sizeof(lf::MemRec32), lf::mem32_bytes(S, nb)), st, &err);
    if (err) return err;
    *m64 = (lf::MemRec64*)ctx->ws((t + ".m64").c_str(), sizeof(lf::MemRec64) * std::max<size_t>(1, (size_t)S * nb), st, &err);
    if (err) return err;
  }
  return LF_OK;
}

// Expand S samples of a model into tables placed by lf_expand_alloc.
lf_status lf_expand_launch(lf_ctx* ctx, const lf_model* M, const double* params, int S, hipStream_t st,
                           lf::MainRec* mains, lf::MulRec* muls, lf::MemRec32* m32, lf::MemRec64* m64) {
  ctx->prof_begin("expand", st);
  hipError_t he = lf::launch_expand(lf_dev_model(M), params, S, mains, muls, m32, m64, st);
  ctx->prof_end(st);
  return ctx->hip(he, "expand");
}

// Expand S samples of a model into workspace tables; returns device pointers.
lf_status lf_expand_tables(lf_ctx* ctx, const lf_model* M, const double* params, int S, bool need_mem,
                           hipStream_t st, lf::MainRec** mains, lf::MulRec** muls, lf::MemRec32** m32,
                           lf::MemRec64** m64, const char* tag) {
  lf_status err = lf_expand_alloc(ctx, M, S, need_mem, st, mains, muls, m32, m64, tag);
  if (err) return err;
  return lf_expand_launch(ctx, M, params, S, st, *mains, *muls, *m32, *m64);
}

// Points per lane of the lean maps kernel: one (two and four points per lane, sharing a member
// record between points, measured 7-17% slower on gfx950: occupancy wins).
int lf_ctx::maps_ppl(bool, bool) { return 1; }

// ------------------------------------------------------------------------------ lens maps
extern "C" lf_status lf_lens_maps(lf_ctx* ctx, const lf_model* M, const double* params, int32_t S,
                                  const lf_points* pts, double a_dis, lf_prec prec, const lf_maps* out,
                                  void* stream) {
  if (!ctx) return LF_E_INVALID_ARG;
  if (!M || !out) return ctx->fail(LF_E_INVALID_ARG, "null model/output");
  if (S < 1) return ctx->fail(LF_E_INVALID_ARG, "S must be >= 1");
  if (M->n_free > 0 && !params) return ctx->fail(LF_E_INVALID_ARG, "model has free fields: params required");
  if (!(a_dis > 0) || !std::isfinite(a_dis)) return ctx->fail(LF_E_INVALID_ARG, "a_dis must be > 0");
  if (prec != LF_PREC_FP64 && prec != LF_PREC_MIXED) return ctx->fail(LF_E_INVALID_ARG, "bad precision");
  lf::PointsSpec ps;
  if (!lf_points_spec(pts, ps)) return ctx->fail(LF_E_INVALID_ARG, "bad points");
  bool d3 = out->psi111 || out->psi112 || out->psi122 || out->psi222 || out->f1 || out->f2;
  bool any = d3 || out->alpha_x || out->alpha_y || out->psi11 || out->psi12 || out->psi22 || out->kappa ||
             out->gamma1 || out->gamma2 || out->detA || out->mu || out->beta_x || out->beta_y || out->e1 ||
             out->e2 || out->flags;
  if (!any) return ctx->fail(LF_E_INVALID_ARG, "no output requested");
  if ((long long)S * ps.P > (1LL << 40)) return ctx->fail(LF_E_INVALID_ARG, "S * P too large");
  hipSetDevice(ctx->device);
  hipStream_t st = (hipStream_t)stream;
  lf::MainRec* mains; lf::MulRec* muls; lf::MemRec32* m32; lf::MemRec64* m64;
  lf_status e = lf_expand_tables(ctx, M, params, S, true, st, &mains, &muls, &m32, &m64, "maps");
  if (e) return e;
  lf::MapsOut o;
  o.ax = out->alpha_x; o.ay = out->alpha_y; o.p11 = out->psi11; o.p12 = out->psi12; o.p22 = out->psi22;
  o.kappa = out->kappa; o.g1 = out->gamma1; o.g2 = out->gamma2; o.detA = out->detA; o.mu = out->mu;
  o.bx = out->beta_x; o.by = out->beta_y; o.t111 = out->psi111; o.t112 = out->psi112; o.t122 = out->psi122;
  o.t222 = out->psi222; o.e1 = out->e1; o.e2 = out->e2; o.f1 = out->f1; o.f2 = out->f2; o.flags = out->flags;
  bool mixed = prec == LF_PREC_MIXED;
  int ppl = ctx->maps_ppl(mixed, d3);
  lf::DevModel dm = lf_dev_model(M);
  double* part = nullptr;
  if (lf::has_heavy(dm)) {
    size_t bytes = (size_t)S * ps.P * (sizeof(double) * 9 + sizeof(int));
    part = (double*)ctx->ws("maps.part", bytes, st, &e);
    if (e) return e;
  }
  if (part) {
    ctx->prof_begin("maps_heavy", st);
    hipError_t he = lf::launch_maps(dm, mains, m32, m64, S, ps, a_dis, mixed, d3, o, lf_quad(ctx), ppl, part, 1, st);
    ctx->prof_end(st);
    if (he != hipSuccess) return ctx->hip(he, "maps heavy kernel");
  }
  ctx->prof_begin("maps_lean", st);
  hipError_t he = lf::launch_maps(dm, mains, m32, m64, S, ps, a_dis, mixed, d3, o, lf_quad(ctx), ppl, part, 2, st);
  ctx->prof_end(st);
  return ctx->hip(he, "maps kernel");
}
