// Host-side internal state of the lensfield library (contexts, resident tables).
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/lensfield.h"
#include "lf_internal.h"
#include "lf_launch.h"

#define LF_ENFW_NODES 24

struct lf_ctx {
  int device = 0;
  size_t budget = 0, dev_bytes = 0;
  int n_cu = 256;
  long long find_cap = 0;       // finder candidate capacity (0: sized from the source count)
  std::string arch;
  std::string last_error;
  struct Buf {
    void* ptr = nullptr;
    size_t bytes = 0;
  };
  std::map<std::string, Buf> bufs;
  double* quad_u = nullptr;
  double* quad_w = nullptr;
  // kernel timing (HIP events on the launching stream)
  bool prof = false;
  std::string prof_only;      // time only this kernel name (empty: every kernel)
  bool prof_skip = false;     // the open bracket was not recorded
  hipStream_t cur_stream = nullptr;
  struct Rec { std::string name; hipEvent_t a, b; };
  std::vector<Rec> prof_pending;
  std::vector<hipEvent_t> ev_pool;
  std::map<std::string, std::pair<double, long long>> prof_tally;
  hipEvent_t prof_ev();
  void prof_begin(const char* name, hipStream_t st);
  void prof_end(hipStream_t st);
  void prof_flush();
  lf_status fail(lf_status st, const char* fmt, ...);
  lf_status hip(hipError_t e, const char* what);
  void* ws(const char* name, size_t bytes, hipStream_t st, lf_status* err);
  lf_status dmalloc(void** p, size_t bytes);
  void dfree(void* p, size_t bytes);
  int maps_ppl(bool mixed, bool d3);   // points per lane of the lean maps kernel
  // Allocation-free calls: while `arena` is set, ws() hands out slices of it and never
  // allocates.  noalloc_scratch is this device's static scratch array (lf_api_noalloc.cpp).
  struct Arena {
    char* base;
    size_t cap, used;
    const char* who;
  };
  Arena* arena = nullptr;
  char* noalloc_scratch = nullptr;
};

struct lf_model {
  int n_free = 0;
  double z_d = 0;
  lf_cosmo cosmo{70.0, 0.3};
  lf::XfConst xc{};
  std::vector<lf::MainDesc> main;
  std::vector<lf::MemCat> mem;
  lf::SegOff seg{};
  lf::Bind mul[3];
  lf::MainDesc* d_main = nullptr;
  lf::MemCat* d_mem = nullptr;
  lf::MemCat32* d_cat32 = nullptr;
  size_t d_main_bytes = 0, d_mem_bytes = 0, d_cat32_bytes = 0;
};

struct lf_cons {
  int n_img = 0, n_fam = 0;
  std::vector<int> order;        // host: constraint index of each sorted image
  std::vector<int> fam_start;    // host: [n_fam + 1] offsets of families in sorted order
  double* d_theta = nullptr;     // [n_img*2] sorted by family
  double* d_sinv = nullptr;      // [n_img*3] S^-1 (xx, xy, yy)
  double* d_sigmax = nullptr;    // [n_img] max(sig1, sig2)
  int* d_fam = nullptr;          // [n_img] family of each sorted image
  int* d_fam_start = nullptr;    // [n_fam + 1]
  int* d_order = nullptr;        // [n_img] constraint index of each sorted image (as order)
  double* d_afam = nullptr;      // [n_fam]
  size_t bytes = 0;
  // flux and time-delay data (Sec. 3.2, 3.3), sorted like the images; null when absent
  double* d_mag = nullptr;       // [n_img] magnitudes and [n_img] errors (d_mag + n_img)
  double* d_dt = nullptr;        // [n_img] delays and [n_img] errors (d_dt + n_img)
  double* d_tsc = nullptr;       // [n_fam] time-delay scales [days / arcsec^2]
  size_t obs_bytes = 0;
  char* d_obs = nullptr;
  bool has_obs() const { return d_mag || d_dt; }
};

lf::XfConst lf_xf_const(const lf_cosmo* c, double zd);
lf::DevModel lf_dev_model(const lf_model* M);
lf::QuadTab lf_quad(const lf_ctx* ctx);
bool lf_model_has_enfw(const lf_model* M);
bool lf_points_spec(const lf_points* p, lf::PointsSpec& s);
lf_status lf_expand_alloc(lf_ctx* ctx, const lf_model* M, int S, bool need_mem, hipStream_t st,
                          lf::MainRec** mains, lf::MulRec** muls, lf::MemRec32** m32, lf::MemRec64** m64,
                          const char* tag);
lf_status lf_expand_launch(lf_ctx* ctx, const lf_model* M, const double* params, int S, hipStream_t st,
                           lf::MainRec* mains, lf::MulRec* muls, lf::MemRec32* m32, lf::MemRec64* m64);
lf_status lf_noalloc_setup(lf_ctx* ctx);
lf_status lf_expand_tables(lf_ctx* ctx, const lf_model* M, const double* params, int S, bool need_mem,
                           hipStream_t st, lf::MainRec** mains, lf::MulRec** muls, lf::MemRec32** m32,
                           lf::MemRec64** m64, const char* tag);
void lf_prof_mark(void* ctx, const char* name, int end_flag);
namespace lf { struct Chi2Args; }
// Set-up shared by the chi^2 entry points: argument checks (nothing is launched when they fail);
// workspace placement and the parameter expansion (want_tmod keeps the model image positions
// of an image-plane launch).
lf_status lf_chi2_check(lf_ctx* ctx, const lf_model* M, const double* params, int32_t S, const lf_cons* c,
                        int32_t mode, lf_prec prec, const double* chi2);
lf_status lf_chi2_prepare(lf_ctx* ctx, const lf_model* M, const double* params, int S, const lf_cons* c,
                          hipStream_t st, lf::Chi2Args& A, const char* tag, bool want_tmod = false);
