// Internal declarations of the fbcorr host library (C++17).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <array>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "fbcorr.h"

namespace fbc {

// ---------------------------------------------------------------- errors
// Status plus a thread-local message (the C ABI's fbcorr_last_error()).
struct Error {
    fbcorr_status status;
    std::string msg;
};
void set_error(fbcorr_status s, const std::string& msg);
void clear_error();
#define FBC_RETURN_IF(cond, status, msg)          \
    do {                                          \
        if (cond) {                               \
            ::fbc::set_error((status), (msg));    \
            return (status);                      \
        }                                         \
    } while (0)

// C ABI entry points turn exceptions into FBCORR_ERR_INTERNAL.
#define FBC_API_BEGIN try {
#define FBC_API_END                                                            \
    }                                                                          \
    catch (const std::exception& e) {                                          \
        ::fbc::set_error(FBCORR_ERR_INTERNAL, std::string("exception: ") + e.what()); \
        return FBCORR_ERR_INTERNAL;                                            \
    }                                                                          \
    catch (...) {                                                              \
        ::fbc::set_error(FBCORR_ERR_INTERNAL, "unknown exception");            \
        return FBCORR_ERR_INTERNAL;                                            \
    }

// --------------------------------------------------------------- configs
// A kernel configuration: ordered key -> integer map plus the algorithm.
// Text form: "algo=igemm kc=8 s=1 ...".
struct Config {
    std::string algo;                 // "igemm", "direct", "dw", "nn"
    std::map<std::string, int> v;
    int get(const char* k) const;
    std::string str() const;
};
bool parse_config(const std::string& text, Config& base, std::string& err);

// ------------------------------------------------------------- kernels
// One compiled kernel: module function plus the resources it needs.
struct Kernel {
    hipFunction_t fn = nullptr;
    int threads = 0;        // workgroup size
    int lds_bytes = 0;      // static LDS
    int vgprs = 0;
    std::string key;
};

// Generated source (embedded template) + -D options for one kernel.
struct KernelSource {
    std::string name;       // kernel symbol
    std::string file;       // template name
    std::string source;
    std::vector<std::string> options;
};

const std::string& template_source(const std::string& file);

// hiprtc compile through the in-process cache; returns code object bytes.
fbcorr_status compile_cached(const KernelSource& ks, const std::string& arch,
                             std::shared_ptr<const std::vector<char>>& code);
// Load (cached per device + key) and fetch the function.
fbcorr_status load_kernel(const KernelSource& ks, int device, Kernel& out);
std::string hiprtc_version_string();
void cache_stats(int64_t& hits, int64_t& misses, int64_t& entries, int64_t& disk_hits);
void cache_clear_memory();
std::string disk_cache_dir();

// FBCORR_TUNE_PROGRESS=1: the tuners print a progress line to stderr as
// candidates compile and are timed (long sweeps otherwise run silently).
bool tune_progress_on();
void tune_progress(const char* fmt, ...) __attribute__((format(printf, 1, 2)));

// Device facts used for validation and launch shapes.
struct DeviceInfo {
    std::string arch;       // e.g. "gfx950"
    int cus = 0;
    int lds_per_block = 0;
    int max_threads = 1024;
};
fbcorr_status device_info(int device, DeviceInfo& out);

}  // namespace fbc
