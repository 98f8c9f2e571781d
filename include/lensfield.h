/*
 * lensfield — MI355X (gfx950) implementation of the lens-equation hot path of
 * parametric strong-lens modeling (arXiv 2609.08649, "LensFactory.jl").
 *
 * Plain C ABI.  Every call returns an lf_status (0 = LF_OK, negative = error);
 * lf_last_error() returns a message for the last failing call on a context.
 * No exception crosses the boundary.
 *
 * Conventions (paper Sec. 2.1):
 *   - Angles are in arcsec (the angular scale theta_0 is 1").
 *   - The lensing potential psi, the deflection alpha = grad psi, the deformation
 *     tensor psi_ij, kappa and gamma are defined WITHOUT the distance ratio
 *     a_dis = D_ds / D_s; a_dis enters only the lens equation
 *     beta = theta - a_dis alpha (Eq. lens_eq) and the Jacobian
 *     A_ij = delta_ij - a_dis psi_ij (Eq. jac).
 *   - Position angles are counter-clockwise from +x; PA = 0 puts the major axis
 *     of an elliptical profile on +x.
 *
 * Memory and ownership:
 *   - "device" pointers are HIP device allocations owned by the caller (for example
 *     the data_ptr of a torch CUDA/ROCm tensor); "host" pointers are ordinary host
 *     memory owned by the caller.  The library never frees caller memory.
 *   - Models and constraint sets are copied into library-owned device tables at
 *     upload and stay resident until released.
 *   - Compute calls are asynchronous on the caller's stream (a hipStream_t passed
 *     as void*; NULL = the default stream); outputs are valid once that stream has
 *     synchronised.  Calls that share an lf_ctx share its scratch workspace: issue
 *     them from one host thread on one stream, or use one context per stream.
 *   - All per-point / per-sample outputs are structure-of-arrays in FP64, sample
 *     major: element (s, p) of a plane lives at plane[s * P + p].
 *
 * Precision (lf_prec):
 *   LF_PREC_FP64  every step in IEEE double precision.
 *   LF_PREC_MIXED member-galaxy halo terms in FP32 (runs of 16 summed in FP32, then
 *                 accumulated in FP64; a member closer than 3 b/q to the point in
 *                 FP64); main halos, beta, det A, mu, chi^2, triangle containment,
 *                 Newton solves and polishing and the final multi-plane source
 *                 positions in FP64.
 */
#ifndef LENSFIELD_H
#define LENSFIELD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lf_status;
enum {
  LF_OK = 0,
  LF_E_INVALID_ARG = -1,   /* bad argument; nothing was launched                       */
  LF_E_UNSUPPORTED = -2,   /* valid request the library does not implement              */
  LF_E_OUT_OF_BUDGET = -3, /* request exceeds the context's HBM budget                   */
  LF_E_DEVICE = -4,        /* HIP runtime error; the context should be shut down         */
  LF_E_OVERFLOW = -5,      /* an output capacity was exceeded (see per-item flags)       */
  LF_E_NOT_READY = -6      /* serving: ticket not complete yet                           */
};

typedef enum { LF_PREC_FP64 = 0, LF_PREC_MIXED = 1 } lf_prec;

/* Halo profiles.  Field meaning per profile (all a_dis-free, arcsec; SHEAR and MPOLE3 only as
 * main components):
 *   LF_POINT  b = Einstein radius (alpha = b^2 r / |r|^2)
 *   LF_SIS    b = isothermal strength (|alpha| = b)
 *   LF_SIE    cored isothermal ellipsoid, kappa = (b/2) / sqrt(s^2 + x'^2 + y'^2/q^2)
 *   LF_PJE    pseudo-Jaffe / dPIE = SIE(b, q, s) - SIE(b, q, a), 0 <= s < a (Sec. 3.4)
 *   LF_NFW    circular NFW: b = kappa_s, s = r_s
 *   LF_ENFW   elliptical NFW: kappa(xi), xi^2 = x'^2 + y'^2/q^2; b = kappa_s, s = r_s
 *   LF_SHEAR  external shear (Sec. 4): psi = (b/2) [(x^2 - y^2) cos 2pa + 2 x y sin 2pa] about
 *             (x, y); b = amplitude, pa = angle; q, s, a unused
 *   LF_MPOLE3 m = 3 multipole with psi ~ r^2 (Sec. 4): psi = (b/3) r^2 cos 3(phi - pa) about
 *             (x, y); b = amplitude, pa = angle; q, s, a unused */
typedef enum { LF_POINT = 0, LF_SIS = 1, LF_SIE = 2, LF_PJE = 3, LF_NFW = 4, LF_ENFW = 5, LF_SHEAR = 6,
               LF_MPOLE3 = 7 } lf_profile;

/* How a raw value becomes a lensing-unit field. */
typedef enum {
  LF_XF_NONE = 0,       /* value already in lensing units                                  */
  LF_XF_SIGMA_TO_B = 1, /* velocity dispersion [km/s] -> b = 4 pi (sigma/c)^2 [arcsec]      */
  LF_XF_KPC = 2,        /* proper length at the lens redshift [kpc] -> arcsec              */
  LF_XF_EPS_TO_Q = 3,   /* ellipticity (1-q)/(1+q) -> q (Sec. 2.1)                         */
  LF_XF_DEG = 4,        /* degrees -> radians                                              */
  LF_XF_M200 = 5,       /* NFW virial mass M200 [Msun] in the b slot (pairs with C200)      */
  LF_XF_C200 = 6        /* NFW concentration c200 in the s slot                            */
} lf_xform;

typedef enum { LF_FIXED = 0, LF_FREE = 1 } lf_bind_kind;

/* A model field: a fixed value, or column `index` of a parameter sample row. */
typedef struct {
  int32_t kind;   /* lf_bind_kind */
  int32_t index;  /* column of the sample row when kind == LF_FREE          */
  int32_t xform;  /* lf_xform                                               */
  int32_t pad;
  double value;   /* raw value when kind == LF_FIXED                       */
} lf_binding;

/* Main component (cluster halo, individually modelled galaxy).  Fields in order
 * x, y, b, q, pa, s, a. */
typedef struct {
  int32_t type;   /* lf_profile */
  int32_t pad;
  lf_binding f[7];
} lf_component;

/* Member galaxies on the scaling relations of Sec. 3.4, Eq. (scaling):
 * v_d = v* (L/L*)^lam, theta_core = theta*_core (L/L*)^bet, theta_cut = theta*_cut (L/L*)^alp.
 * Per member: b = bmul * lum^(2 lam), s = smul * lum^bet, a = amul * lum^alp when lum != NULL,
 * else b = bmul * b0, s = smul * s0, a = amul * a0.  bmul/smul/amul are bindings
 * (bmul usually v* with LF_XF_SIGMA_TO_B).  All arrays are host pointers of length n;
 * q and pa may be NULL (circular members). */
typedef struct {
  int32_t n;
  int32_t pad;
  const int32_t* type;
  const double *x, *y, *q, *pa;
  const double* lum;
  double lam, bet, alp;
  const double *b0, *s0, *a0;
  lf_binding bmul, smul, amul;
} lf_members;

/* Flat LCDM (Omega_r = 0, w = -1; the paper's defaults are H0 = 70, Om = 0.3). */
typedef struct { double H0, Om; } lf_cosmo;

/* Regular grid of pixel centres: point (i, j) = (x0 + (i + 1/2) h, y0 + (j + 1/2) h),
 * flattened p = j * nx + i. */
typedef struct { double x0, y0, h; int32_t nx, ny; } lf_grid;

/* Evaluation points: the grid when px == NULL, else explicit device arrays px, py of length n. */
typedef struct {
  lf_grid grid;
  const double* px;
  const double* py;
  int64_t n;
} lf_points;

/* Caller-owned device output planes, each [S][P] FP64 (flags int32).  NULL = not requested.
 * psi1xx planes are third potential derivatives (singularity maps, Sec. 6); e1 = kappa + |gamma|,
 * e2 = kappa - |gamma|; f1, f2 = v_k . grad e_k (A3-line fields, zero where |gamma| ~ 0). */
typedef struct {
  double *alpha_x, *alpha_y;
  double *psi11, *psi12, *psi22;
  double *kappa, *gamma1, *gamma2;
  double *detA, *mu;
  double *beta_x, *beta_y;
  double *psi111, *psi112, *psi122, *psi222;
  double *e1, *e2, *f1, *f2;
  int32_t* flags;
} lf_maps;

/* Per-item flag bits (maps: per point; chi^2: per sample; finder: per source). */
enum {
  LF_F_SINGULAR = 1,   /* a point sits on a singular halo centre (its term is zero) */
  LF_F_GSING = 2,      /* singular family matrix G; pseudo-inverse used             */
  LF_F_NOCONV = 4,     /* Newton did not converge                                   */
  LF_F_REJECT = 8,     /* image-plane solution rejected (moved > 10 sigma / parity)  */
  LF_F_MERGED = 16,    /* finder merged duplicate candidates                        */
  LF_F_OVERFLOW = 32,  /* more images / candidates than the output capacity         */
  LF_F_UMBILIC = 64,   /* |gamma| ~ 0: singularity fields not evaluated             */
  LF_F_INVALID = 128   /* sampled parameters out of range (result is NaN)          */
};

typedef struct lf_ctx lf_ctx;
typedef struct lf_model lf_model;
typedef struct lf_cons lf_cons;

/* ---------------------------------------------------------------- context */
/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the library's own
 * device allocations (0 = 90% of free memory).  The environment variable LF_FIND_CAND_CAP,
 * when set, fixes the image finders' candidate capacity per call (otherwise
 * max(65536, 64 n_src)).  Errors: LF_E_INVALID_ARG, LF_E_DEVICE. */
lf_status lf_init(lf_ctx** out, int32_t device, size_t hbm_budget_bytes);
lf_status lf_shutdown(lf_ctx* ctx);
const char* lf_last_error(const lf_ctx* ctx);
/* Library-owned device bytes currently allocated by this context. */
size_t lf_device_bytes(const lf_ctx* ctx);

/* Kernel timing: when enabled, every kernel the library launches is bracketed by HIP events
 * recorded on the launching stream.  lf_profile_read synchronises those events and returns the
 * summed duration [ms] and launch count of one kernel name ("maps_lean", "maps_heavy",
 * "expand", "chi2_halo", ...); lf_profile_reset clears the tallies. */
lf_status lf_profile_enable(lf_ctx* ctx, int32_t on);
lf_status lf_profile_read(lf_ctx* ctx, const char* kernel, double* total_ms, int64_t* launches);
lf_status lf_profile_reset(lf_ctx* ctx);
/* Restrict kernel timing to one kernel name (host string, copied), so that the events of the
 * other launches stay off the streams; NULL or "" times every kernel again.  Returns
 * LF_E_INVALID_ARG for a null context. */
lf_status lf_profile_only(lf_ctx* ctx, const char* kernel);

/* ---------------------------------------------------------------- cosmology helpers (host) */
/* Angular-diameter distance D(z1, z2) [Mpc] in flat LCDM (Sec. 2.1, 2.2). */
lf_status lf_cosmo_dist(const lf_cosmo* c, double z1, double z2, double* out);
/* Distance ratio a_dis = D(z_d, z_s) / D(0, z_s) of Eq. (lens_eq). */
lf_status lf_cosmo_adis(const lf_cosmo* c, double z_d, double z_s, double* out);
/* NFW (kappa_s, r_s[arcsec]) from (M200 [Msun], c200) at lens redshift z_d; kappa_s is
 * relative to the a_dis-free critical density c^2 / (4 pi G D_d). */
lf_status lf_nfw_params(const lf_cosmo* c, double z_d, double m200, double c200,
                        double* kappa_s, double* r_s);
/* Time-delay scale (1 + z_d)/c D_d D_s / D_ds theta_0^2 of Eq. (time_delay) with
 * theta_0 = 1", in days per arcsec^2 (multiplies the Fermat potential in arcsec^2). */
lf_status lf_cosmo_tdscale(const lf_cosmo* c, double z_d, double z_s, double* out);

/* ---------------------------------------------------------------- resident model tables */
/* Upload a parametric model (main components with field bindings + members on
 * the scaling relations, Sec. 3.4).  `n_free` is the width of a parameter sample row.
 * All pointers are host pointers; the library copies them.  Errors: LF_E_INVALID_ARG
 * (bad profile code, binding index >= n_free, a fixed field out of range). */
lf_status lf_model_upload(lf_ctx* ctx, const lf_component* main, int32_t n_main,
                          const lf_members* members, double z_d, const lf_cosmo* cosmo,
                          int32_t n_free, lf_model** out);
lf_status lf_model_release(lf_ctx* ctx, lf_model* m);
int32_t lf_model_n_halos(const lf_model* m);

/* Upload image-position constraints (Sec. 3.1): observed positions theta [n_img*2],
 * family id [n_img] in 0..n_fam-1, error-ellipse semi-axes sig1, sig2 and angle phi
 * [n_img] (S_i = R^T diag(sig1^2, sig2^2) R; circular errors: sig1 = sig2, phi = 0), and
 * the distance ratio of each family a_fam [n_fam].  Host pointers, copied. */
lf_status lf_constraints_upload(lf_ctx* ctx, const double* theta, const int32_t* family,
                                const double* sig1, const double* sig2, const double* phi,
                                int32_t n_img, const double* a_fam, int32_t n_fam, lf_cons** out);
lf_status lf_constraints_release(lf_ctx* ctx, lf_cons* c);
/* Attach flux (Sec. 3.2) and/or time-delay (Sec. 3.3) measurements to a constraint set, in
 * the image order of lf_constraints_upload: magnitudes mag and errors sig_mag [n_img]
 * (both NULL: no flux data), delays dt [days] and errors sig_dt [n_img] with the time-delay
 * scale of each family tscale [n_fam] (lf_cosmo_tdscale; all three NULL: no delays).  An
 * image enters a term only where its error is > 0.  Host pointers, copied; at most once per
 * set.  Errors: LF_E_INVALID_ARG (incomplete or non-finite data, tscale <= 0). */
lf_status lf_constraints_observables(lf_ctx* ctx, lf_cons* c, const double* mag, const double* sig_mag,
                                     const double* dt, const double* sig_dt, const double* tscale);

/* ---------------------------------------------------------------- hot-path calls */
/* Halo-sum maps: for each of S parameter samples (device params [S * n_free], or
 * NULL with S = 1 when the model has no free field) and each point, the halo sum of
 * alpha and psi_ij (Sec. 2.1) and, when any of psi111..f2 is requested, the third
 * derivatives psi_ijk and the A3-line fields of Sec. 6.  a_dis > 0 sets beta, det A, mu.
 * Errors: LF_E_INVALID_ARG (no output requested, S < 1, bad points). */
lf_status lf_lens_maps(lf_ctx* ctx, const lf_model* m, const double* params, int32_t S,
                       const lf_points* pts, double a_dis, lf_prec prec, const lf_maps* out,
                       void* stream);

/* chi^2 per parameter sample (Sec. 3.1).  mode 0 = source plane, Eq. (chi2_src)
 * with the full magnification tensor mu_i = A^-1(theta_obs) and beta_model = G^-1 g;
 * mode 1 = image plane, Eq. (chi2_img), with each model image found by Newton-Raphson
 * from its observed position towards beta_model (Sec. 3.5; FP64 steps in both precisions,
 * MIXED affecting only the source-plane fit that sets beta_model; converged when a step is
 * below 1e-9", at most 20 steps; an image that does not converge, moves > 10 sigma or
 * changes parity keeps its source-plane term and is flagged).
 * params: device [S * n_free]; chi2: device [S]; flags: device [S] (or NULL).
 * beta_model: device [S * n_fam * 2] or NULL. */
lf_status lf_chi2_batch(lf_ctx* ctx, const lf_model* m, const double* params, int32_t S,
                        const lf_cons* c, int32_t mode, lf_prec prec, double* chi2,
                        int32_t* flags, double* beta_model, void* stream);

/* chi^2 with flux and time-delay terms: the total chi^2 = chi2_pos + chi2_f + chi2_dt of Sec. 3.2
 * and 3.3 when the constraint set carries flux or delay data (lf_constraints_observables),
 * with the per-term values in terms [S * 3] (position, flux, delay; device, or NULL).  Per
 * family, the source magnitude (Eq. msrc) and the delay zero point (Eq. dt0) are the
 * weighted means; magnitudes use 2.5 log10 |mu|.  mode 0: mu_model and dt_model from the
 * linear expansions about theta_obs (mu + A^-1 (beta_model - beta_obs) . grad mu, with
 * grad mu from the third derivatives; Eq. td_approx); mode 1: mu and the Fermat potential at
 * the accepted model image (Eq. time_delay), the expansions for images the Newton solve did
 * not accept.  These terms are evaluated in FP64 in both precisions.  Without such data the
 * call equals lf_chi2_batch.  Errors: those of lf_chi2_batch. */
lf_status lf_chi2_terms(lf_ctx* ctx, const lf_model* m, const double* params, int32_t S,
                        const lf_cons* c, int32_t mode, lf_prec prec, double* chi2,
                        int32_t* flags, double* beta_model, double* terms, void* stream);

/* Image-plane chi^2 (Sec. 3.1 Eq. chi2_img, solved as in Sec. 3.5) with its per-image results:
 * the same launch and chi2 / flags / beta_model as lf_chi2_batch in mode 1, and per observed
 * image theta_model [S * n_img * 2], the model image that image's Newton solve reached (its
 * last iterate when the solve did not converge), and img_flags [S * n_img], that image's
 * LF_F_NOCONV / LF_F_REJECT bits.  Both are device arrays in the constraint order given to
 * lf_constraints_upload (sample-major), and either may be NULL.  Errors: those of
 * lf_chi2_batch. */
lf_status lf_chi2_images(lf_ctx* ctx, const lf_model* m, const double* params, int32_t S,
                         const lf_cons* c, lf_prec prec, double* chi2, int32_t* flags,
                         double* beta_model, double* theta_model, int32_t* img_flags, void* stream);

/* Allocation-free lf_chi2_batch, for the callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, kernels and results (bit-identical) as lf_chi2_batch, but the call allocates
 * nothing: its workspace is a static device array of LF_CHI2_NOALLOC_SCRATCH_BYTES that every
 * GPU the library runs on holds until the process ends (lf_init takes its address once per
 * device).  Workspace (bytes): S * (112 n_main + 32 + 16 n_fam) + 112 S n_img, plus
 * 112 S n_img with flux or delay data, plus up to 256 per slice for alignment (the
 * 1024-sample, 150-image, 60-family cluster case needs 18.5 MB).  Every call on a GPU shares
 * that GPU's array and leaves its contents behind: calls that overlap on one GPU (from any
 * context or stream) race, so the caller serialises them.  Kernel timing (lf_profile_enable)
 * does not cover this call.  Errors: those of lf_chi2_batch; LF_E_OUT_OF_BUDGET when the
 * workspace exceeds the array (nothing is launched). */
#define LF_CHI2_NOALLOC_SCRATCH_BYTES (32u << 20)
lf_status lf_chi2_batch_noalloc(lf_ctx* ctx, const lf_model* m, const double* params, int32_t S,
                                const lf_cons* c, int32_t mode, lf_prec prec, double* chi2,
                                int32_t* flags, double* beta_model, void* stream);

/* Image finder by triangle mapping (replacing the marching-squares contours of
 * Sec. 2.3).  Grid vertices are pixel centres; cell (i, j) splits along its
 * (i,j)-(i+1,j+1) diagonal.  A source is inside a mapped triangle by exact orientation
 * signs (ties broken by edge direction so shared edges are watertight); each candidate is
 * polished by FP64 Newton (<= 30 steps to |d beta| < 1e-10"), accepted if it stays within
 * 2h of its start, and merged with an earlier image closer than 1e-6".
 * params: device row [n_free] or NULL; beta: device [n_src*2]; a_src: device [n_src].
 * Outputs (device): theta_out [n_src*max_img*2], mu_out [n_src*max_img], count_out [n_src]
 * (true count even when it exceeds max_img), flags [n_src] or NULL.  Candidate triangles are
 * kept per source in source order up to the call's candidate capacity; a source whose
 * candidates do not all fit, and every source after it, gets count 0 and LF_F_OVERFLOW
 * (the same sources on every run). */
lf_status lf_find_images(lf_ctx* ctx, const lf_model* m, const double* params,
                         const double* beta, const double* a_src, int32_t n_src,
                         const lf_grid* grid, int32_t max_img, lf_prec prec, double* theta_out,
                         double* mu_out, int32_t* count_out, int32_t* flags, void* stream);

/* lf_find_images on a deflection map the caller already has: alpha_x, alpha_y (device, [ny][nx],
 * a_dis-free, at the grid's vertices) replace the finder's own vertex halo sum, so a pipeline
 * that computes maps and then images of the same sample (Sec. 2.1, 2.3) sums the halos on the
 * grid once.  With the maps of lf_lens_maps for the same model, sample, grid and precision the
 * results are those of lf_find_images bit for bit; the FP64 containment tests and the Newton
 * polish use the model as there.  Other arguments, outputs and errors as lf_find_images. */
lf_status lf_find_images_alpha(lf_ctx* ctx, const lf_model* m, const double* params,
                               const double* alpha_x, const double* alpha_y, const double* beta,
                               const double* a_src, int32_t n_src, const lf_grid* grid, int32_t max_img,
                               lf_prec prec, double* theta_out, double* mu_out, int32_t* count_out,
                               int32_t* flags, void* stream);

/* Image finder of Sec. 2.3, kept as a cross-check on triangle mapping: zero contours of both
 * components of f = beta - theta + a alpha on the grid vertices (marching squares: linear
 * interpolation on cell edges, the asymptotic decider in cells crossed four times), images at
 * the exact intersections of pairs of contour segments (accuracy O(h^2); a singular centre,
 * where alpha jumps, can give a spurious intersection).  polish != 0: each intersection is
 * refined by FP64 Newton (<= 30 steps to |d beta| < 1e-10") and kept if it converged within
 * 2h of it.  Images closer than 1e-6" to an earlier one are merged.  Arguments, outputs and
 * errors as lf_find_images (single plane); the grid has fewer than 2^30 cells. */
lf_status lf_find_images_ms(lf_ctx* ctx, const lf_model* m, const double* params, const double* beta,
                            const double* a_src, int32_t n_src, const lf_grid* grid, int32_t max_img,
                            lf_prec prec, int32_t polish, double* theta_out, double* mu_out,
                            int32_t* count_out, int32_t* flags, void* stream);

/* Multi-plane ray trace (Sec. 2.2).  planes sorted by z_planes (increasing),
 * each a model without free fields.  For each point and each source redshift z_src[k]:
 * beta [n_zs][P][2], Jacobian A [n_zs][P][4] (A11 A12 A21 A22; not symmetric), mu [n_zs][P].
 * Planes at or behind a source do not deflect it.  Any output may be NULL. */
lf_status lf_multiplane_trace(lf_ctx* ctx, const lf_model* const* planes, const double* z_planes,
                              int32_t n_planes, const lf_cosmo* cosmo, const double* z_src,
                              int32_t n_zs, const lf_points* pts, lf_prec prec, double* beta_out,
                              double* A_out, double* mu_out, void* stream);

/* Multi-plane image finder: as lf_find_images, each source at its own redshift
 * z_src [n_src] (host pointer; device beta). */
lf_status lf_find_images_mp(lf_ctx* ctx, const lf_model* const* planes, const double* z_planes,
                            int32_t n_planes, const lf_cosmo* cosmo, const double* beta,
                            const double* z_src, int32_t n_src, const lf_grid* grid,
                            int32_t max_img, lf_prec prec, double* theta_out, double* mu_out,
                            int32_t* count_out, int32_t* flags, void* stream);

/* ---------------------------------------------------------------- singularity-map extraction */
/* Output lists of lf_singularity_map (all device pointers, each list holding at most cap
 * entries; counts holds the true counts). */
typedef struct {
  int32_t cap;
  double* cross_pos;     /* [cap*2] A3 crossings on grid edges                              */
  int32_t* cross_k;      /* [cap] family: 1 (e_1 = kappa + |gamma|) or 2 (e_2)              */
  double* cross_e;       /* [cap] e_k there: the cusp forms for distance ratio 1 / e_k       */
  double* cross_g;       /* [cap] g_k = v_k . grad f_k there                                */
  int32_t* cross_flags;  /* [cap] 1 umbilic-flagged evaluation, 2 no convergence, 4 a jump  */
  int32_t* seg_a;        /* [cap] segment ends: crossing index, or -(umbilic index) - 1     */
  int32_t* seg_b;
  int32_t* seg_k;        /* [cap] family                                                    */
  double* umb_pos;       /* [cap*2] umbilics (D4)                                           */
  double* umb_kappa;     /* [cap] kappa there: the umbilic forms for distance ratio 1/kappa */
  int32_t* umb_status;   /* [cap] 0 ok, 1 no convergence, 2 outside its cell, +4 unjoined   */
  double* swt_pos;       /* [cap*2] swallowtails (A4)                                       */
  int32_t* swt_k;        /* [cap] family                                                    */
  double* swt_e;         /* [cap] e_k there                                                 */
  int32_t* swt_seg;      /* [cap] segment it lies on                                        */
  int32_t* swt_status;   /* [cap] 0 ok, 1 no convergence, 2 moved > h, +8 umbilic-flagged  */
  int32_t* counts;       /* [6] crossings, segments, umbilics, swallowtails, cells skipped  */
                         /*     next to umbilic-flagged vertices, cells left unpaired       */
} lf_sing_out;

/* Singularity map of a single-plane lens (Sec. 6): the A3 lines, where the eigenvector v_k
 * of the deformation tensor is tangent to the critical curve of e_k (f_k = v_k . grad e_k =
 * 0), umbilics (D4, gamma = 0, where the two families meet) and swallowtails (A4, where v_k is
 * tangent to the A3 line: g_k = v_k . grad f_k = 0), with the refinement the paper plans.
 * The fields are evaluated at the grid vertices x0 + (i + 1/2) h (FP64, or MIXED for the
 * vertex pass only); f_k is compared along each grid edge after aligning the eigenvectors
 * (line fields); crossings come in the order row j, horizontal edges by i, vertical edges by
 * i, k = 1, 2.  refine != 0: each crossing is the root of f_k on its edge to a bracket below
 * tol arcsec (Illinois regula falsi, FP64, <= 100 steps), swallowtails are polished by Newton
 * on (f_k, g_k) = 0 (<= 20 steps, stopping below 1e-10"; accepted when the last step is below
 * 1e-8"); refine = 0: linear interpolation.  Segments
 * join the crossings of a cell (marching squares, the asymptotic decider in saddle cells);
 * cells whose eigenvector loop has orientation product -1 hold an umbilic, found by Newton
 * on (gamma_1, gamma_2) = 0 from the cell centre (<= 30 steps to 1e-10"), and an odd number
 * of lines of each family ends there.  Next to singular centres and where the eigenvectors
 * turn fast within a cell, spurious entries are flagged by their status.  When counts[0] >
 * cap no segment, umbilic or swallowtail is produced.  params: device row [n_free] or NULL.
 * Errors: LF_E_INVALID_ARG (grid smaller than 2 x 2 or above 2^31 vertices, cap < 1, tol <=
 * 0, a NULL output). */
lf_status lf_singularity_map(lf_ctx* ctx, const lf_model* m, const double* params, const lf_grid* grid,
                             lf_prec prec, int32_t refine, double tol, const lf_sing_out* out, void* stream);

/* ---------------------------------------------------------------- inference on the device */
/* Affine-invariant ensemble sampler (Sec. 3.5; the stretch move of Goodman & Weare): n_steps
 * steps of K walkers (K even, >= 4) in the n_free parameters of the model, walkers and
 * log-probabilities staying on the device.  log p = -chi^2 / 2 (lf_chi2_terms in the given mode
 * and precision, flux and delay terms included when the constraints carry them) inside the
 * prior box lo <= x <= hi, -inf outside it or where chi^2 is undefined.  Each step updates
 * the two halves of the ensemble in turn, each against the other: walker k of the moving
 * half proposes Y = X_j + z (X_k - X_j) (j drawn from the other half, z = ((a-1) u + 1)^2 / a)
 * and takes it when log u' < (D-1) log z + log p(Y) - log p(X_k).  u = the top 53 bits of
 * output n of SplitMix64 seeded with seed, n = ((t * 2 + half) * K + k) * 3 + d for step t
 * (step0 + s), walker k and draw d (0 partner, 1 stretch, 2 acceptance): a run continued with
 * step0 = the steps done so far reproduces an uninterrupted one.
 * Device pointers: X [K * D] and lp [K] in/out (init_lp != 0: lp computed from X first);
 * lo, hi [D]; chain [n_steps * K * D] and lp_chain [n_steps * K] (state after each step; NULL:
 * not recorded); n_accept [K] accumulated (NULL: not counted).  Errors: LF_E_INVALID_ARG (no
 * free parameter, K odd or < 4, a <= 1, bad mode/precision), those of lf_chi2_terms. */
lf_status lf_aies_run(lf_ctx* ctx, const lf_model* m, const lf_cons* c, int32_t mode, lf_prec prec, int32_t K,
                      double* X, double* lp, int32_t init_lp, const double* lo, const double* hi, double a,
                      uint64_t seed, int64_t step0, int32_t n_steps, double* chain, double* lp_chain,
                      int32_t* n_accept, void* stream);

/* Nelder-Mead downhill simplex (Sec. 3.5) for R independent runs in lockstep: the R initial
 * simplices [R][D+1][D] (device, in/out) are evaluated, then n_rounds rounds each evaluate
 * one pending point per run (reflection; expansion or contraction; shrink vertices one per
 * round).  f = chi^2 (as in lf_aies_run), +inf outside the prior box or where undefined.
 * Coefficients 1, 2, 1/2, 1/2 and the rules of Lagarias et al. (1998): reflection accepted
 * when f_0 <= f_r < f_{D-1}; expansion when f_r < f_0 (the better of the two kept); outside
 * contraction when f_{D-1} <= f_r < f_D (kept if <= f_r), inside when f_r >= f_D (kept if <
 * f_D); otherwise shrink towards the best vertex.  On return the simplices are sorted by f
 * (fvals [R][D+1], ties in insertion order) and n_evals [R] (or NULL) counts evaluations.
 * Errors: LF_E_INVALID_ARG (no free parameter, R < 1, bad mode/precision), LF_E_UNSUPPORTED
 * (more than 64 free parameters: a run is handled by one wave, a lane per parameter), those of
 * lf_chi2_terms. */
lf_status lf_nelder_mead_run(lf_ctx* ctx, const lf_model* m, const lf_cons* c, int32_t mode, lf_prec prec,
                             int32_t R, double* simplex, double* fvals, const double* lo, const double* hi,
                             int32_t n_rounds, int32_t* n_evals, void* stream);

/* ---------------------------------------------------------------- uneven batched chi^2 */
/* One chi^2 problem of an uneven batch: a model, its constraints and S parameter samples. */
typedef struct {
  const lf_model* model;
  const lf_cons* cons;
  const double* params;  /* device [S * n_free] (NULL when the model has no free field)  */
  int32_t S;
  double* chi2;          /* device [S] output                                             */
  int32_t* flags;        /* device [S] output or NULL                                     */
} lf_batch_item;

typedef struct lf_batch lf_batch;

/* Plan a batch of chi^2 problems of different sizes (models with different halo counts,
 * constraint sets of different lengths) to run as one persistent launch: per-item expansion,
 * the halo sums of all items from one queue of tiles ordered largest work first, then the
 * per-sample reductions (and, mode 1, the image-plane Newton solves), all captured in a
 * hipGraph.  autotune != 0 times candidate tile shapes (workgroup size, tile length, resident
 * workgroups per CU) and keeps the fastest, caching the choice on disk (file named by the
 * environment variable LF_AUTOTUNE_CACHE, else $HOME/.cache/lensfield/autotune.txt).
 * The plan owns its workspace; the item pointers must stay valid until lf_batch_release.
 * Results are bit-identical to lf_chi2_batch on each item.  Errors: LF_E_INVALID_ARG,
 * LF_E_OUT_OF_BUDGET, LF_E_DEVICE. */
lf_status lf_batch_create(lf_ctx* ctx, const lf_batch_item* items, int32_t n_items, int32_t mode,
                          lf_prec prec, int32_t autotune, lf_batch** out);
/* Replay the plan's graph on `stream` (reads the current contents of each item's params). */
lf_status lf_batch_run(lf_batch* b, void* stream);
/* Chosen tile shape: workgroup size, resident workgroups, lanes per tile, number of tiles. */
lf_status lf_batch_info(const lf_batch* b, int32_t* block, int32_t* grid, int32_t* tile_lanes,
                        int32_t* n_tiles);
lf_status lf_batch_release(lf_batch* b);

/* ---------------------------------------------------------------- serving */
typedef struct lf_server lf_server;

typedef struct {
  size_t hbm_budget;         /* device bytes the server may hold for admitted requests      */
  int32_t n_streams;         /* >= 2: one for chi^2 batches, the rest for map chunks         */
  int32_t max_batch_samples; /* cap on the samples of one continuous chi^2 batch (0 = 65536) */
  int32_t map_chunk_rows;    /* grid rows per map chunk (0 = 256): preemption granularity   */
} lf_serve_config;

enum { LF_REQ_CHI2 = 0, LF_REQ_MU_MAP = 1, LF_REQ_SING_MAP = 2 };

/* A request.  chi^2: model, cons, host params [S * n_free] (copied at submit), S, mode, prec;
 * output out_host [S] (and flags_host [S] or NULL).  LF_REQ_MU_MAP: model (+ host params row or
 * NULL), grid, a_dis, prec; out_host [P] = mu.  LF_REQ_SING_MAP: out_host [6][P] = kappa,
 * det A, e1, e2, f1, f2 (Sec. 6).  Outputs are written by asynchronous copies: pass pinned host
 * memory (pageable memory works but stalls the scheduler while it copies).  Maps may instead
 * keep their result on the device: out_device (caller-owned device memory of the same layout,
 * and flags_device [P] or NULL) replaces out_host, which is then NULL; nothing is copied to the
 * host, the output planes are not counted in the request's footprint, and the result is
 * complete once the ticket is done. */
typedef struct {
  int32_t kind;
  int32_t S;
  const lf_model* model;
  const lf_cons* cons;
  const double* params;
  int32_t mode;
  int32_t prec;
  lf_grid grid;
  double a_dis;
  double* out_host;
  int32_t* flags_host;
  double* out_device;
  int32_t* flags_device;
} lf_request;

/* Start a server on a context: a scheduler thread admits requests in arrival order whenever
 * their device footprint fits the budget (a later, smaller request may pass one that does not
 * fit yet), merges all admitted chi^2 requests of one (mode, precision) into one persistent
 * batch launch while the previous batch runs (continuous batching), and runs maps in row
 * chunks on the other streams so that their work overlaps with the chi^2 batches.  A request
 * larger than the whole budget fails with LF_E_OUT_OF_BUDGET; a failing request does not
 * affect the others.  Each result is bit-identical to the same request served alone. */
lf_status lf_serve_start(lf_ctx* ctx, const lf_serve_config* cfg, lf_server** out);
/* Thread-safe.  Returns a ticket (> 0) or an error for a malformed request. */
lf_status lf_serve_submit(lf_server* s, const lf_request* req, int64_t* ticket);
/* status: 0 pending, 1 done, < 0 the request's error; latency_ms = completion - submission. */
lf_status lf_serve_poll(lf_server* s, int64_t ticket, int32_t* status, double* latency_ms);
lf_status lf_serve_wait(lf_server* s, int64_t ticket, int32_t* status, double* latency_ms);
/* Latency statistics of completed requests of one kind (-1 = all): count, p50, p99, mean [ms]. */
lf_status lf_serve_stats(lf_server* s, int32_t kind, int64_t* count, double* p50_ms, double* p99_ms,
                         double* mean_ms);
/* Waits for admitted work, fails queued requests with LF_E_NOT_READY, frees the arena. */
lf_status lf_serve_stop(lf_server* s);

#ifdef __cplusplus
}
#endif
#endif /* LENSFIELD_H */
