// Many uneven images in one persistent launch (placeholder until the
// persistent kernel lands: the entry points report UNSUPPORTED).
#include "plan.h"

namespace fbc {
void destroy_batched(Plan* p) { (void)p; }
std::string batched_describe(const Plan* p) { (void)p; return "batched"; }
}  // namespace fbc

using namespace fbc;

extern "C" fbcorr_status fbcorr_plan_batched(int32_t count, const fbcorr_desc* descs, int device, fbcorr_plan_t* out) {
    (void)count; (void)descs; (void)device; (void)out;
    set_error(FBCORR_ERR_UNSUPPORTED, "batched plans are not available in this build");
    return FBCORR_ERR_UNSUPPORTED;
}

extern "C" fbcorr_status fbcorr_forward_batched(fbcorr_plan_t plan, const float* const* xs, const float* const* ws_,
                                                float* const* ys, void* workspace, size_t workspace_bytes,
                                                void* stream, int use_graph) {
    (void)plan; (void)xs; (void)ws_; (void)ys; (void)workspace; (void)workspace_bytes; (void)stream; (void)use_graph;
    set_error(FBCORR_ERR_UNSUPPORTED, "batched plans are not available in this build");
    return FBCORR_ERR_UNSUPPORTED;
}
