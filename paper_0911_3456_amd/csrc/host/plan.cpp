// Plans and the C ABI entry points for single problems.
#include "plan.h"

#include <algorithm>
#include <cstring>

namespace fbc {

DeviceGuard::DeviceGuard(int dev) {
    hipGetDevice(&prev_);
    if (prev_ != dev) { hipSetDevice(dev); changed_ = true; }
}
DeviceGuard::~DeviceGuard() {
    if (changed_) hipSetDevice(prev_);
}

fbcorr_status validate_desc(const fbcorr_desc* d) {
    FBC_RETURN_IF(!d, FBCORR_ERR_INVALID_ARGUMENT, "descriptor is NULL");
    FBC_RETURN_IF(d->batch <= 0 || d->H <= 0 || d->W <= 0 || d->D <= 0 || d->N <= 0 || d->fh <= 0 || d->fw <= 0,
                  FBCORR_ERR_INVALID_ARGUMENT, "every dimension must be >= 1");
    FBC_RETURN_IF(d->fh > d->H || d->fw > d->W, FBCORR_ERR_SHAPE,
                  "filter " + std::to_string(d->fh) + "x" + std::to_string(d->fw) + " larger than input " +
                      std::to_string(d->H) + "x" + std::to_string(d->W));
    FBC_RETURN_IF(d->precision < FBCORR_FP32 || d->precision > FBCORR_FP16, FBCORR_ERR_INVALID_ARGUMENT,
                  "unknown precision");
    FBC_RETURN_IF(d->algo < FBCORR_ALGO_AUTO || d->algo > FBCORR_ALGO_IGEMM, FBCORR_ERR_INVALID_ARGUMENT,
                  "unknown algorithm");
    FBC_RETURN_IF(d->algo == FBCORR_ALGO_DIRECT && d->precision != FBCORR_FP32, FBCORR_ERR_UNSUPPORTED,
                  "the direct kernel computes in fp32 only");
    FBC_RETURN_IF((d->flags & ~FBCORR_FLAG_OVERLAP_BACKWARD) != 0, FBCORR_ERR_INVALID_ARGUMENT,
                  "unknown bits in flags");
    const double elems_x = (double)d->batch * d->H * d->W * d->D;
    const double elems_y = (double)d->batch * (d->H - d->fh + 1) * (d->W - d->fw + 1) * d->N;
    FBC_RETURN_IF(elems_x > 2.0e9 || elems_y > 2.0e9, FBCORR_ERR_UNSUPPORTED, "tensor larger than 2^31 elements");
    return FBCORR_OK;
}

fbcorr_status compile_role(Plan* p, int role, const Config& c) {
    RoleBuild rb;
    std::string err;
    if (!build_role(p->desc, role, c, p->dev, rb, err)) {
        set_error(FBCORR_ERR_UNSUPPORTED, err);
        return FBCORR_ERR_UNSUPPORTED;
    }
    if (role == FBCORR_ROLE_FORWARD && !p->epilogue.empty())
        rb.main.options.push_back("-DFB_EPILOGUE(v,c)=(" + p->epilogue + ")");
    RoleExec ex;
    fbcorr_status st = load_kernel(rb.main, p->device, ex.main);
    if (st != FBCORR_OK) return st;
    FBC_RETURN_IF(ex.main.lds_bytes > p->dev.lds_per_block, FBCORR_ERR_UNSUPPORTED, "kernel LDS exceeds the device");
    for (auto& a : rb.aux) {
        Kernel k;
        st = load_kernel(a, p->device, k);
        if (st != FBCORR_OK) return st;
        ex.aux.push_back(k);
    }
    ex.build = rb;
    std::lock_guard<std::mutex> lk(p->mu);
    p->role[role] = std::move(ex);
    p->have[role].store(true, std::memory_order_release);
    return FBCORR_OK;
}

fbcorr_status launch(const Kernel& k, const LaunchGeom& g, hipStream_t s, void** args) {
    hipError_t e = hipModuleLaunchKernel(k.fn, g.grid_x, g.grid_y, 1, g.threads, 1, 1, 0, s, args, nullptr);
    FBC_RETURN_IF(e != hipSuccess, FBCORR_ERR_LAUNCH, std::string("hipModuleLaunchKernel: ") + hipGetErrorString(e));
    return FBCORR_OK;
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

fbcorr_status check_ptr(const void* p, const char* what) {
    FBC_RETURN_IF(!p, FBCORR_ERR_INVALID_ARGUMENT, std::string(what) + " is NULL");
    FBC_RETURN_IF(!aligned16(p), FBCORR_ERR_INVALID_ARGUMENT, std::string(what) + " is not 16-byte aligned");
    return FBCORR_OK;
}

fbcorr_status check_ws(void* ws, size_t have, size_t need) {
    if (need == 0) return FBCORR_OK;
    FBC_RETURN_IF(have < need, FBCORR_ERR_WORKSPACE,
                  "workspace " + std::to_string(have) + " B < required " + std::to_string(need) + " B");
    return check_ptr(ws, "workspace");
}

// Timing: events around every kernel a role launches (filter preparation,
// the main kernel and the partial sum), on the stream they are launched on.
void timing_begin(Plan* p, int role, hipStream_t s, hipEvent_t& a) {
    a = nullptr;
    if (!p->timing) return;
    hipEventCreate(&a);
    hipEventRecord(a, s);
}
void timing_end(Plan* p, int role, hipStream_t s, hipEvent_t a) {
    if (!a) return;
    hipEvent_t b = nullptr;
    hipEventCreate(&b);
    hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(p->mu);
    auto& pend = p->pending[role];
    pend.push_back({a, b});
    // Keep the number of live events bounded when the totals are not read:
    // fold the completed half into the running totals.
    if (pend.size() > kMaxPendingEvents) {
        const size_t half = pend.size() / 2;
        for (size_t i = 0; i < half; ++i) {
            hipEventSynchronize(pend[i].second);
            float t = 0.f;
            if (hipEventElapsedTime(&t, pend[i].first, pend[i].second) == hipSuccess) {
                p->acc_ms[role] += t;
                p->acc_calls[role] += 1;
            }
            hipEventDestroy(pend[i].first);
            hipEventDestroy(pend[i].second);
        }
        pend.erase(pend.begin(), pend.begin() + half);
    }
}

fbcorr_status run_forward(Plan* p, const RoleExec& ex, const float* x, const float* w, float* y, void* ws,
                          hipStream_t s) {
    const RoleBuild& rb = ex.build;
    const void* wt = w;
    const float* unscale = nullptr;
    fbcorr_status st;
    hipEvent_t ev;
    timing_begin(p, FBCORR_ROLE_FORWARD, s, ev);
    if (!ex.aux.empty() && rb.cfg.algo == "direct") {
        // scalar-weight direct kernel: tap-major copy of the filters
        float* wtt = (float*)ws;
        void* args[] = {(void*)&w, &wtt};
        st = launch(ex.aux[0], rb.aux_geom[0], s, args);
        if (st != FBCORR_OK) { timing_end(p, FBCORR_ROLE_FORWARD, s, ev); return st; }
        w = wtt;
    } else if (!ex.aux.empty()) {
        // low precision: scale, round and pack the filters into the workspace
        char* base = (char*)ws;
        void* wq = base + rb.ws_lowp_w;
        float* us = (float*)(base + rb.ws_unscale);
        void* args[] = {(void*)&w, &wq, &us};
        st = launch(ex.aux[0], rb.aux_geom[0], s, args);
        if (st != FBCORR_OK) { timing_end(p, FBCORR_ROLE_FORWARD, s, ev); return st; }
        wt = wq;
        unscale = us;
        if (rb.nxp > 0) {
            // fp16: partial maxima of |x| for the per-tensor input scale
            const fbcorr_desc& d = p->desc;
            long n = (long)d.batch * d.H * d.W * d.D;
            float* part = (float*)(base + rb.ws_xmax);
            void* a1[] = {(void*)&x, &n, &part};
            st = launch(ex.aux[1], rb.aux_geom[1], s, a1);
            if (st != FBCORR_OK) { timing_end(p, FBCORR_ROLE_FORWARD, s, ev); return st; }
        }
    }
    if (rb.cfg.algo == "direct") {
        void* args[] = {(void*)&x, (void*)&w, (void*)&y};
        st = launch(ex.main, rb.main_geom, s, args);
    } else {
        void* args[] = {(void*)&x, (void*)&wt, (void*)&unscale, (void*)&y};
        st = launch(ex.main, rb.main_geom, s, args);
    }
    timing_end(p, FBCORR_ROLE_FORWARD, s, ev);
    return st;
}

fbcorr_status run_backward_x(Plan* p, const RoleExec& ex, const float* w, const float* dy, float* dx, void* ws,
                             hipStream_t s) {
    const RoleBuild& rb = ex.build;
    const float* wfc = w;                   // fused flip: the kernel reads w itself
    hipEvent_t ev;
    timing_begin(p, FBCORR_ROLE_BACKWARD_X, s, ev);
    if (!ex.aux.empty()) {
        // flipped copy of the filters (fbcorr_flip_filters), or the
        // fragment-ordered flipped bank (fbcorr_pack_frag, no scales)
        float* wf = (float*)ws;
        float* no_scale = nullptr;
        void* a0[] = {(void*)&w, (void*)&wf, (void*)&no_scale};
        fbcorr_status st = launch(ex.aux[0], rb.aux_geom[0], s, a0);
        if (st != FBCORR_OK) { timing_end(p, FBCORR_ROLE_BACKWARD_X, s, ev); return st; }
        wfc = wf;
    }
    fbcorr_status st;
    const float* unscale = nullptr;
    void* a1[] = {(void*)&dy, (void*)&wfc, (void*)&unscale, (void*)&dx};
    st = launch(ex.main, rb.main_geom, s, a1);
    timing_end(p, FBCORR_ROLE_BACKWARD_X, s, ev);
    return st;
}

fbcorr_status run_backward_w(Plan* p, const RoleExec& ex, const float* x, const float* dy, float* dw, void* ws,
                             hipStream_t s) {
    const RoleBuild& rb = ex.build;
    float* part = (float*)ws;
    hipEvent_t ev;
    timing_begin(p, FBCORR_ROLE_BACKWARD_W, s, ev);
    void* a0[] = {(void*)&x, (void*)&dy, (void*)&part};
    fbcorr_status st = launch(ex.main, rb.main_geom, s, a0);
    if (st == FBCORR_OK) {
        const float* pc = part;
        void* a1[] = {(void*)&pc, (void*)&dw};
        st = launch(ex.aux[0], rb.aux_geom[0], s, a1);
    }
    timing_end(p, FBCORR_ROLE_BACKWARD_W, s, ev);
    return st;
}

size_t backward_ws(const Plan* p, size_t* off_w) {
    size_t a = p->have[FBCORR_ROLE_BACKWARD_X] ? p->role[FBCORR_ROLE_BACKWARD_X].build.ws_bytes : 0;
    size_t b = p->have[FBCORR_ROLE_BACKWARD_W] ? p->role[FBCORR_ROLE_BACKWARD_W].build.ws_bytes : 0;
    if (off_w) *off_w = a;
    return a + b;
}

fbcorr_status ensure_role(Plan* p, int role) {
    if (p->have[role].load(std::memory_order_acquire)) return FBCORR_OK;
    // First use: one thread compiles, the others wait for it and then find
    // the role installed (an installed role is never replaced from here).
    std::lock_guard<std::mutex> lk(p->compile_mu);
    if (p->have[role].load(std::memory_order_acquire)) return FBCORR_OK;
    return compile_role(p, role, default_config(p->desc, role, p->dev));
}

}  // namespace fbc

using namespace fbc;

// ====================================================================== C ABI


extern "C" {

int fbcorr_version(void) { return 100; }

const char* fbcorr_status_string(fbcorr_status s) {
    switch (s) {
    case FBCORR_OK: return "FBCORR_OK";
    case FBCORR_ERR_INVALID_ARGUMENT: return "FBCORR_ERR_INVALID_ARGUMENT";
    case FBCORR_ERR_SHAPE: return "FBCORR_ERR_SHAPE";
    case FBCORR_ERR_UNSUPPORTED: return "FBCORR_ERR_UNSUPPORTED";
    case FBCORR_ERR_COMPILE: return "FBCORR_ERR_COMPILE";
    case FBCORR_ERR_LAUNCH: return "FBCORR_ERR_LAUNCH";
    case FBCORR_ERR_WORKSPACE: return "FBCORR_ERR_WORKSPACE";
    case FBCORR_ERR_NO_DEVICE: return "FBCORR_ERR_NO_DEVICE";
    case FBCORR_ERR_INTERNAL: return "FBCORR_ERR_INTERNAL";
    }
    return "FBCORR_ERR_UNKNOWN";
}

fbcorr_status fbcorr_plan(const fbcorr_desc* desc, int device, fbcorr_plan_t* out) {
    FBC_API_BEGIN
    clear_error();
    FBC_RETURN_IF(!out, FBCORR_ERR_INVALID_ARGUMENT, "output handle pointer is NULL");
    fbcorr_status st = validate_desc(desc);
    if (st != FBCORR_OK) return st;
    std::unique_ptr<Plan> p(new Plan());
    p->desc = *desc;
    p->device = device;
    st = device_info(device, p->dev);
    if (st != FBCORR_OK) return st;
    DeviceGuard g(device);
    st = compile_role(p.get(), FBCORR_ROLE_FORWARD, default_config(*desc, FBCORR_ROLE_FORWARD, p->dev));
    if (st != FBCORR_OK) return st;
    *out = reinterpret_cast<fbcorr_plan_t>(p.release());
    return FBCORR_OK;
    FBC_API_END
}

fbcorr_status fbcorr_plan_destroy(fbcorr_plan_t plan) {
    FBC_API_BEGIN
    clear_error();
    Plan* p = reinterpret_cast<Plan*>(plan);
    if (!p) return FBCORR_OK;
    for (auto& v : p->pending)
        for (auto& e : v) { hipEventDestroy(e.first); hipEventDestroy(e.second); }
    if (p->side) {
        DeviceGuard g(p->device);
        hipStreamSynchronize(p->side);
        hipEventDestroy(p->fork);
        hipEventDestroy(p->join);
        hipStreamDestroy(p->side);
    }
    destroy_batched(p);
    delete p;
    return FBCORR_OK;
    FBC_API_END
}

fbcorr_status fbcorr_workspace_size(fbcorr_plan_t plan, int pass, size_t* bytes) {
    FBC_API_BEGIN
    clear_error();
    Plan* p = reinterpret_cast<Plan*>(plan);
    FBC_RETURN_IF(!p || !bytes, FBCORR_ERR_INVALID_ARGUMENT, "NULL argument");
    if (p->batched) {
        *bytes = pass == 2 ? batched_tune_workspace(p) : p->batch_ws;
        return FBCORR_OK;
    }
    DeviceGuard g(p->device);
    if (pass == 0) {
        *bytes = p->role[FBCORR_ROLE_FORWARD].build.ws_bytes;
        return FBCORR_OK;
    }
    if (pass == 1) {
        fbcorr_status st = ensure_role(p, FBCORR_ROLE_BACKWARD_X);
        if (st == FBCORR_OK) st = ensure_role(p, FBCORR_ROLE_BACKWARD_W);
        if (st != FBCORR_OK) return st;
        *bytes = backward_ws(p, nullptr);
        return FBCORR_OK;
    }
    if (pass == 2) {
        *bytes = tune_workspace(p);
        return FBCORR_OK;
    }
    set_error(FBCORR_ERR_INVALID_ARGUMENT, "pass must be 0 (forward), 1 (backward) or 2 (tune)");
    return FBCORR_ERR_INVALID_ARGUMENT;
    FBC_API_END
}

fbcorr_status fbcorr_forward(fbcorr_plan_t plan, const float* x, const float* w, float* y, void* workspace,
                             size_t workspace_bytes, void* stream) {
    FBC_API_BEGIN
    clear_error();
    Plan* p = reinterpret_cast<Plan*>(plan);
    FBC_RETURN_IF(!p, FBCORR_ERR_INVALID_ARGUMENT, "plan is NULL");
    FBC_RETURN_IF(p->batched, FBCORR_ERR_INVALID_ARGUMENT, "batched plan: use fbcorr_forward_batched");
    fbcorr_status st;
    if ((st = check_ptr(x, "x")) || (st = check_ptr(w, "w")) || (st = check_ptr(y, "y"))) return st;
    const RoleExec& ex = p->role[FBCORR_ROLE_FORWARD];
    if ((st = check_ws(workspace, workspace_bytes, ex.build.ws_bytes))) return st;
    DeviceGuard g(p->device);
    return run_forward(p, ex, x, w, y, workspace, (hipStream_t)stream);
    FBC_API_END
}

fbcorr_status fbcorr_backward(fbcorr_plan_t plan, const float* x, const float* w, const float* dy, float* dx,
                              float* dw, void* workspace, size_t workspace_bytes, void* stream) {
    FBC_API_BEGIN
    clear_error();
    Plan* p = reinterpret_cast<Plan*>(plan);
    FBC_RETURN_IF(!p, FBCORR_ERR_INVALID_ARGUMENT, "plan is NULL");
    FBC_RETURN_IF(p->batched, FBCORR_ERR_UNSUPPORTED, "batched plans have no backward pass");
    fbcorr_status st;
    if ((st = check_ptr(dy, "dy"))) return st;
    if (dx && ((st = check_ptr(w, "w")) || (st = check_ptr(dx, "dx")))) return st;
    if (dw && ((st = check_ptr(x, "x")) || (st = check_ptr(dw, "dw")))) return st;
    if (!dx && !dw) return FBCORR_OK;
    FBC_RETURN_IF(!p->epilogue.empty(), FBCORR_ERR_UNSUPPORTED,
                  "the backward pass of a plan with a fused epilogue is not provided");
    DeviceGuard g(p->device);
    if ((st = ensure_role(p, FBCORR_ROLE_BACKWARD_X)) || (st = ensure_role(p, FBCORR_ROLE_BACKWARD_W))) return st;
    size_t off_w = 0;
    const size_t need = backward_ws(p, &off_w);
    if ((st = check_ws(workspace, workspace_bytes, need))) return st;
    hipStream_t s = (hipStream_t)stream;
    if (dx && dw && (p->desc.flags & FBCORR_FLAG_OVERLAP_BACKWARD)) {
        // The two gradients are independent: dW goes to a side stream forked
        // from the caller's stream and joined back, so the two kernels
        // overlap.  (Default-priority stream; the event pair also works under
        // graph capture.)  Calls from several threads enqueue their
        // fork/join sequences one at a time.
        std::lock_guard<std::mutex> side_lock(p->side_mu);
        if (!p->side) {
            hipError_t e = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join, hipEventDisableTiming);
            FBC_RETURN_IF(e != hipSuccess, FBCORR_ERR_LAUNCH, std::string("side stream: ") + hipGetErrorString(e));
        }
        hipError_t e = hipEventRecord(p->fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(p->side, p->fork, 0);
        FBC_RETURN_IF(e != hipSuccess, FBCORR_ERR_LAUNCH, std::string("fork: ") + hipGetErrorString(e));
        st = run_backward_w(p, p->role[FBCORR_ROLE_BACKWARD_W], x, dy, dw, (char*)workspace + off_w, p->side);
        fbcorr_status st2 = run_backward_x(p, p->role[FBCORR_ROLE_BACKWARD_X], w, dy, dx, workspace, s);
        e = hipEventRecord(p->join, p->side);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, p->join, 0);
        if (st != FBCORR_OK) return st;
        if (st2 != FBCORR_OK) return st2;
        FBC_RETURN_IF(e != hipSuccess, FBCORR_ERR_LAUNCH, std::string("join: ") + hipGetErrorString(e));
        return FBCORR_OK;
    }
    if (dx) {
        st = run_backward_x(p, p->role[FBCORR_ROLE_BACKWARD_X], w, dy, dx, workspace, s);
        if (st != FBCORR_OK) return st;
    }
    if (dw) {
        st = run_backward_w(p, p->role[FBCORR_ROLE_BACKWARD_W], x, dy, dw, (char*)workspace + off_w, s);
        if (st != FBCORR_OK) return st;
    }
    return FBCORR_OK;
    FBC_API_END
}

fbcorr_status fbcorr_plan_get_config(fbcorr_plan_t plan, int role, char* buf, size_t len) {
    FBC_API_BEGIN
    clear_error();
    Plan* p = reinterpret_cast<Plan*>(plan);
    FBC_RETURN_IF(!p || !buf || len == 0, FBCORR_ERR_INVALID_ARGUMENT, "NULL argument");
    FBC_RETURN_IF(role < 0 || role >= FBCORR_ROLE_COUNT, FBCORR_ERR_INVALID_ARGUMENT, "unknown role");
    std::string s;
    if (p->batched) {
        s = batched_describe(p);
    } else {
        DeviceGuard g(p->device);
        fbcorr_status st = ensure_role(p, role);
        if (st != FBCORR_OK) return st;
        s = p->role[role].build.cfg.str();
        if (role == FBCORR_ROLE_BACKWARD_W) s += " (partials=" + std::to_string(p->role[role].build.np) + ")";
    }
    FBC_RETURN_IF(s.size() + 1 > len, FBCORR_ERR_INVALID_ARGUMENT, "buffer too small");
    memcpy(buf, s.c_str(), s.size() + 1);
    return FBCORR_OK;
    FBC_API_END
}

fbcorr_status fbcorr_plan_set_config(fbcorr_plan_t plan, int role, const char* cfg) {
    FBC_API_BEGIN
    clear_error();
    Plan* p = reinterpret_cast<Plan*>(plan);
    FBC_RETURN_IF(!p || !cfg, FBCORR_ERR_INVALID_ARGUMENT, "NULL argument");
    FBC_RETURN_IF(p->batched, FBCORR_ERR_UNSUPPORTED, "batched plans are configured at plan time");
    FBC_RETURN_IF(role < 0 || role >= FBCORR_ROLE_COUNT, FBCORR_ERR_INVALID_ARGUMENT, "unknown role");
    DeviceGuard g(p->device);
    Config c;
    std::string err;
    if (!config_from_text(p->desc, role, p->dev, cfg, true, c, err)) {
        set_error(FBCORR_ERR_INVALID_ARGUMENT, err);
        return FBCORR_ERR_INVALID_ARGUMENT;
    }
    return compile_role(p, role, c);
    FBC_API_END
}

fbcorr_status fbcorr_plan_set_epilogue(fbcorr_plan_t plan, const char* expr) {
    FBC_API_BEGIN
    clear_error();
    Plan* p = reinterpret_cast<Plan*>(plan);
    FBC_RETURN_IF(!p, FBCORR_ERR_INVALID_ARGUMENT, "plan is NULL");
    FBC_RETURN_IF(p->batched, FBCORR_ERR_UNSUPPORTED, "batched plans have no epilogue");
    const std::string e = expr ? expr : "";
    FBC_RETURN_IF(e.size() > 1024, FBCORR_ERR_INVALID_ARGUMENT, "epilogue longer than 1024 characters");
    for (char ch : e)
        FBC_RETURN_IF(ch == '\n' || ch == '\r' || ch == '#' || ch == '\\', FBCORR_ERR_INVALID_ARGUMENT,
                      "epilogue must be a single-line expression (no '#', '\\' or line breaks)");
    DeviceGuard g(p->device);
    const std::string prev = p->epilogue;
    p->epilogue = e;
    fbcorr_status st = compile_role(p, FBCORR_ROLE_FORWARD, p->role[FBCORR_ROLE_FORWARD].build.cfg);
    if (st != FBCORR_OK) {
        p->epilogue = prev;     // the previous kernel stays installed
        return st;
    }
    return FBCORR_OK;
    FBC_API_END
}

fbcorr_status fbcorr_plan_enable_timing(fbcorr_plan_t plan, int enable) {
    FBC_API_BEGIN
    clear_error();
    Plan* p = reinterpret_cast<Plan*>(plan);
    FBC_RETURN_IF(!p, FBCORR_ERR_INVALID_ARGUMENT, "plan is NULL");
    p->timing = enable != 0;
    return FBCORR_OK;
    FBC_API_END
}

fbcorr_status fbcorr_plan_read_timing(fbcorr_plan_t plan, double* ms, int64_t* calls, int reset) {
    FBC_API_BEGIN
    clear_error();
    Plan* p = reinterpret_cast<Plan*>(plan);
    FBC_RETURN_IF(!p, FBCORR_ERR_INVALID_ARGUMENT, "plan is NULL");
    DeviceGuard g(p->device);
    std::lock_guard<std::mutex> lk(p->mu);
    for (int r = 0; r < FBCORR_ROLE_COUNT; ++r) {
        for (auto& e : p->pending[r]) {
            hipEventSynchronize(e.second);
            float t = 0.f;
            if (hipEventElapsedTime(&t, e.first, e.second) == hipSuccess) {
                p->acc_ms[r] += t;
                p->acc_calls[r] += 1;
            }
            hipEventDestroy(e.first);
            hipEventDestroy(e.second);
        }
        p->pending[r].clear();
        if (ms) ms[r] = p->acc_ms[r];
        if (calls) calls[r] = p->acc_calls[r];
        if (reset) { p->acc_ms[r] = 0; p->acc_calls[r] = 0; }
    }
    return FBCORR_OK;
    FBC_API_END
}

static DeviceInfo offline_device(const char* arch) {
    DeviceInfo di;
    di.arch = arch ? arch : "gfx950";
    di.cus = 256;
    di.lds_per_block = 160 * 1024;
    di.max_threads = 1024;
    return di;
}

static fbcorr_status offline_build(const fbcorr_desc* desc, int role, const char* cfg, const char* arch,
                                   RoleBuild& rb) {
    fbcorr_status st = validate_desc(desc);
    if (st != FBCORR_OK) return st;
    FBC_RETURN_IF(role < 0 || role >= FBCORR_ROLE_COUNT, FBCORR_ERR_INVALID_ARGUMENT, "unknown role");
    DeviceInfo di = offline_device(arch);
    Config c = default_config(*desc, role, di);
    std::string err;
    if (cfg) {
        if (!config_from_text(*desc, role, di, cfg, false, c, err)) {
            set_error(FBCORR_ERR_INVALID_ARGUMENT, err);
            return FBCORR_ERR_INVALID_ARGUMENT;
        }
    }
    if (!build_role(*desc, role, c, di, rb, err)) {
        set_error(FBCORR_ERR_UNSUPPORTED, err);
        return FBCORR_ERR_UNSUPPORTED;
    }
    return FBCORR_OK;
}

fbcorr_status fbcorr_codegen(const fbcorr_desc* desc, int role, const char* cfg, char* source, size_t* source_len,
                             char* options, size_t* options_len) {
    FBC_API_BEGIN
    clear_error();
    FBC_RETURN_IF(!source_len || !options_len, FBCORR_ERR_INVALID_ARGUMENT, "length pointers are NULL");
    RoleBuild rb;
    fbcorr_status st = offline_build(desc, role, cfg, nullptr, rb);
    if (st != FBCORR_OK) return st;
    std::string o;
    for (auto& s : rb.main.options) o += s + " ";
    const size_t need_s = rb.main.source.size() + 1, need_o = o.size() + 1;
    const bool fits = source && options && *source_len >= need_s && *options_len >= need_o;
    *source_len = need_s;
    *options_len = need_o;
    if (!source || !options) return FBCORR_OK;     // size query
    FBC_RETURN_IF(!fits, FBCORR_ERR_INVALID_ARGUMENT, "buffers too small");
    memcpy(source, rb.main.source.c_str(), need_s);
    memcpy(options, o.c_str(), need_o);
    return FBCORR_OK;
    FBC_API_END
}

fbcorr_status fbcorr_compile_check(const fbcorr_desc* desc, int role, const char* cfg, const char* arch,
                                   size_t* code_bytes) {
    FBC_API_BEGIN
    clear_error();
    RoleBuild rb;
    fbcorr_status st = offline_build(desc, role, cfg, arch, rb);
    if (st != FBCORR_OK) return st;
    const std::string a = arch ? arch : "gfx950";
    std::shared_ptr<const std::vector<char>> code;
    size_t total = 0;
    st = compile_cached(rb.main, a, code);
    if (st != FBCORR_OK) return st;
    total += code->size();
    for (auto& k : rb.aux) {
        st = compile_cached(k, a, code);
        if (st != FBCORR_OK) return st;
        total += code->size();
    }
    if (code_bytes) *code_bytes = total;
    return FBCORR_OK;
    FBC_API_END
}

fbcorr_status fbcorr_cache_stats(int64_t* hits, int64_t* misses, int64_t* entries, int64_t* disk_hits) {
    FBC_API_BEGIN
    clear_error();
    int64_t h, m, e, d;
    cache_stats(h, m, e, d);
    if (hits) *hits = h;
    if (misses) *misses = m;
    if (entries) *entries = e;
    if (disk_hits) *disk_hits = d;
    return FBCORR_OK;
    FBC_API_END
}

fbcorr_status fbcorr_cache_clear(void) {
    FBC_API_BEGIN
    clear_error();
    cache_clear_memory();
    tuning_db_reload();
    return FBCORR_OK;
    FBC_API_END
}

}  // extern "C"
