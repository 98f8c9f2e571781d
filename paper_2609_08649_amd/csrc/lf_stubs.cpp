// Entry points not yet implemented report LF_E_UNSUPPORTED.
#include "lf_api_internal.h"

int lf_ctx::maps_ppl(bool mixed, bool d3) { return (mixed && !d3) ? 2 : 1; }
void lf_release_extras(lf_ctx*) {}

extern "C" lf_status lf_find_images(lf_ctx*, const lf_model*, const double*, const double*, const double*, int32_t,
                                    const lf_grid*, int32_t, lf_prec, double*, double*, int32_t*, int32_t*, void*) {
  return LF_E_UNSUPPORTED;
}
extern "C" lf_status lf_multiplane_trace(lf_ctx*, const lf_model* const*, const double*, int32_t, const lf_cosmo*,
                                         const double*, int32_t, const lf_points*, lf_prec, double*, double*, double*,
                                         void*) { return LF_E_UNSUPPORTED; }
extern "C" lf_status lf_find_images_mp(lf_ctx*, const lf_model* const*, const double*, int32_t, const lf_cosmo*,
                                       const double*, const double*, int32_t, const lf_grid*, int32_t, lf_prec,
                                       double*, double*, int32_t*, int32_t*, void*) { return LF_E_UNSUPPORTED; }
