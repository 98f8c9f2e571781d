// Entry points not yet implemented report LF_E_UNSUPPORTED.
#include "lf_api_internal.h"

int lf_ctx::maps_ppl(bool mixed, bool d3) { return (mixed && !d3) ? 2 : 1; }
void lf_release_extras(lf_ctx*) {}

