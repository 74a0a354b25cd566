// The plan object behind fbcorr_plan_t.
#pragma once

#include "geometry.h"

#include <atomic>

namespace fbc {

struct RoleExec {
    RoleBuild build;
    Kernel main;
    std::vector<Kernel> aux;
};

struct BatchedState;   // batched.cpp

// Timing events kept per role before the oldest are folded into the totals.
constexpr size_t kMaxPendingEvents = 1024;

struct Plan {
    fbcorr_desc desc{};
    int device = 0;
    DeviceInfo dev;
    RoleExec role[FBCORR_ROLE_COUNT];
    // have[r]: role r is compiled and installed.  Set (release) only after
    // role[r] is complete; the first use of a role compiles it under
    // compile_mu, and ensure_role never replaces an installed role, so a
    // caller that saw have[r] may use role[r] while other threads call in.
    std::atomic<bool> have[FBCORR_ROLE_COUNT] = {{false}, {false}, {false}};
    std::mutex compile_mu;
    std::mutex mu;
    // kernel timing
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[FBCORR_ROLE_COUNT];
    double acc_ms[FBCORR_ROLE_COUNT] = {0, 0, 0};
    int64_t acc_calls[FBCORR_ROLE_COUNT] = {0, 0, 0};
    // fused forward epilogue (empty: none)
    std::string epilogue;
    // backward: dW runs on a side stream forked from and joined back into
    // the caller's stream, concurrently with dX
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    std::mutex side_mu;      // one fork/launch/join sequence at a time
    // many uneven images
    bool batched = false;
    size_t batch_ws = 0;
    BatchedState* bstate = nullptr;
};

class DeviceGuard {
public:
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
private:
    int prev_ = 0;
    bool changed_ = false;
};

fbcorr_status validate_desc(const fbcorr_desc* d);
fbcorr_status compile_role(Plan* p, int role, const Config& c);
fbcorr_status ensure_role(Plan* p, int role);
fbcorr_status launch(const Kernel& k, const LaunchGeom& g, hipStream_t s, void** args);
fbcorr_status check_ptr(const void* p, const char* what);
fbcorr_status check_ws(void* ws, size_t have, size_t need);
fbcorr_status run_forward(Plan* p, const RoleExec& ex, const float* x, const float* w, float* y, void* ws,
                          hipStream_t s);
fbcorr_status run_backward_x(Plan* p, const RoleExec& ex, const float* w, const float* dy, float* dx, void* ws,
                             hipStream_t s);
fbcorr_status run_backward_w(Plan* p, const RoleExec& ex, const float* x, const float* dy, float* dw, void* ws,
                             hipStream_t s);
size_t backward_ws(const Plan* p, size_t* off_w);
void timing_begin(Plan* p, int role, hipStream_t s, hipEvent_t& a);
void timing_end(Plan* p, int role, hipStream_t s, hipEvent_t a);

// tune.cpp
size_t tune_workspace(Plan* p);
fbcorr_status tune_plan(Plan* p, const float* x, const float* w, float* y, void* workspace, size_t workspace_bytes,
                        hipStream_t s, const fbcorr_tune_opts* opts, bool four_waves, bool install,
                        fbcorr_tune_report* report, Config* chosen_out);
// batched.cpp
fbcorr_status tune_batched(Plan* p, void* workspace, size_t workspace_bytes, hipStream_t s,
                           const fbcorr_tune_opts* opts, fbcorr_tune_report* report);
size_t batched_tune_workspace(const Plan* p);
// batched.cpp
void destroy_batched(Plan* p);
std::string batched_describe(const Plan* p);

}  // namespace fbc
