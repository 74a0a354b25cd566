// The allocation-free forward entry point and its device scratch array.
//
// fbcorr_forward_noalloc runs a plan's forward role exactly as
// fbcorr_forward does, with the role's workspace (the packed filter bank of
// the matrix-core kernels, or the tap-major filter copy of the direct
// kernel's scalar-weight variant) taken from a file-scope device array
// instead of a caller buffer, so that it calls no allocator at any point.
// Each device the library runs on holds its own copy of the array until the
// process ends; its address on a device is looked up once, with that device
// current, and kept.  In host code the array's name is only a stand-in for
// the symbol: every use below goes through the looked-up device address.
#include <hip/hip_runtime.h>

#include "plan.h"

namespace fbc {

// 16 MiB: room for the packed bank of any filter bank up to about eight
// million weights.
constexpr size_t kNoAllocScratchBytes = 16u << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}

// The device address of `scratch` on `device` (the caller has made it the
// current device); looked up on the first call per device.
static fbcorr_status scratch_address(int device, void** out) {
    FBC_RETURN_IF(device < 0 || device >= kMaxDevices, FBCORR_ERR_INVALID_ARGUMENT, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        FBC_RETURN_IF(e != hipSuccess || !ptr, FBCORR_ERR_LAUNCH,
                      std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return FBCORR_OK;
}

}  // namespace fbc

using namespace fbc;

extern "C" {

fbcorr_status fbcorr_forward_noalloc(fbcorr_plan_t plan, const float* x, const float* w, float* y, void* stream) {
    FBC_API_BEGIN
    clear_error();
    Plan* p = reinterpret_cast<Plan*>(plan);
    FBC_RETURN_IF(!p, FBCORR_ERR_INVALID_ARGUMENT, "plan is NULL");
    FBC_RETURN_IF(p->batched, FBCORR_ERR_INVALID_ARGUMENT, "batched plan: use fbcorr_forward_batched");
    fbcorr_status st;
    if ((st = check_ptr(x, "x")) || (st = check_ptr(w, "w")) || (st = check_ptr(y, "y"))) return st;
    const RoleExec& ex = p->role[FBCORR_ROLE_FORWARD];
    const size_t need = ex.build.ws_bytes;
    FBC_RETURN_IF(need > kNoAllocScratchBytes, FBCORR_ERR_WORKSPACE,
                  "the forward role needs " + std::to_string(need) + " B of scratch; the static scratch holds " +
                      std::to_string(kNoAllocScratchBytes) + " B");
    DeviceGuard g(p->device);
    void* ws = nullptr;
    if (need > 0 && (st = scratch_address(p->device, &ws))) return st;
    return run_forward(p, ex, x, w, y, ws, (hipStream_t)stream);
    FBC_API_END
}

}  // extern "C"
