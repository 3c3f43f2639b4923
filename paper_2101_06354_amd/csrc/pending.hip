// Entry points whose kernels are not in this build yet: they validate
// nothing and report SSIMX_ENOTSUP.
#include "host_common.hpp"

using namespace ssimx;

extern "C" {
ssimx_status ssimx_plan_create(const ssimx_pair*, int, void*, ssimx_plan**) { return SSIMX_ENOTSUP; }
ssimx_status ssimx_plan_run(ssimx_plan*, float*, void*) { return SSIMX_ENOTSUP; }
ssimx_status ssimx_plan_run_unbatched(ssimx_plan*, float*, void*) { return SSIMX_ENOTSUP; }
ssimx_status ssimx_plan_destroy(ssimx_plan*) { return SSIMX_ENOTSUP; }
ssimx_status ssimx_plan_info(const ssimx_plan*, int*, int*) { return SSIMX_ENOTSUP; }
}
