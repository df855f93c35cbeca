// asg_build_components: adaptive cut-HDMR build with device hierarchisation.
#include "hdmr_internal.h"

using namespace hdmr;

extern "C" int asg_build_components(const asg_build_params *params, hdmr_fn f, void *user, hdmr_model **out) {
  (void)params; (void)f; (void)user; (void)out;
  return fail(HDMR_EUNSUPPORTED, "asg_build_components not built yet");
}
