// Heterodyned (relative-binning) likelihood: set-up and evaluation.
#include "gw_ctx.h"

struct gw_het_state {};
struct gw_graph_cache {};

namespace gw {

void het_free(gw_ctx* ctx) { ctx->het = nullptr; }
void graphs_free(gw_ctx* ctx) { ctx->graphs = nullptr; }

gw_status loglike_het(gw_ctx* ctx, const double* theta, int64_t n, int marg, int prec, double* logl,
                      hipStream_t st) {
  (void)theta; (void)n; (void)marg; (void)prec; (void)logl; (void)st;
  if (!ctx->het) return set_error(GW_ESTATE, "loglike_batch: heterodyne_setup has not been called");
  return GW_OK;
}

}  // namespace gw
