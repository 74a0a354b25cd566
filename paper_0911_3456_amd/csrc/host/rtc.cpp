// Run-time code generation core: hiprtc compilation behind an in-process
// cache, module loading, device facts, errors.
//
// The paper's compile path (Sec. 5, Fig. 2): source string -> cache lookup
// keyed by the source and the hardware/software environment -> compile on a
// miss -> load -> fetch the function.  Here the key is a hash of the
// generated source, every compile option, the target architecture and the
// hiprtc version; the cache lives for the process.
#include "internal.h"

#include <dlfcn.h>
#include <sys/stat.h>
#include <unistd.h>

#include <cstdarg>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <unordered_map>

#include "kernels_embed.h"   // generated: embedded kernel templates

namespace fbc {

// ---------------------------------------------------------------- errors
namespace {
thread_local std::string t_last_error;
}

void set_error(fbcorr_status s, const std::string& msg) {
    t_last_error = std::string(fbcorr_status_string(s)) + ": " + msg;
}
void clear_error() { t_last_error.clear(); }

// ------------------------------------------------------------ templates
const std::string& template_source(const std::string& file) {
    static std::map<std::string, std::string> table = [] {
        std::map<std::string, std::string> t;
        for (size_t i = 0; i < kEmbeddedCount; ++i) t[kEmbedded[i].name] = kEmbedded[i].text;
        return t;
    }();
    static const std::string empty;
    auto it = table.find(file);
    return it == table.end() ? empty : it->second;
}

// ---------------------------------------------------------------- hashing
static uint64_t fnv1a(const std::string& s, uint64_t h = 1469598103934665603ull) {
    for (unsigned char c : s) { h ^= c; h *= 1099511628211ull; }
    return h;
}

std::string hiprtc_version_string() {
    int major = 0, minor = 0;
    hiprtcVersion(&major, &minor);
    return std::to_string(major) + "." + std::to_string(minor);
}

// ------------------------------------------------------------ compile cache
namespace {
std::mutex g_cache_mu;
std::unordered_map<std::string, std::shared_ptr<const std::vector<char>>> g_code;
int64_t g_hits = 0, g_misses = 0, g_disk_hits = 0;

struct LoadedKey {
    int device;
    std::string key;
    bool operator==(const LoadedKey& o) const { return device == o.device && key == o.key; }
};
struct LoadedKeyHash {
    size_t operator()(const LoadedKey& k) const { return std::hash<std::string>()(k.key) ^ (size_t)k.device; }
};
std::unordered_map<LoadedKey, hipModule_t, LoadedKeyHash> g_modules;
}  // namespace

static std::string cache_key(const KernelSource& ks, const std::string& arch) {
    std::string all = ks.source;
    all += '\x1f';
    for (auto& o : ks.options) { all += o; all += '\x1f'; }
    all += arch;
    all += '\x1f';
    all += hiprtc_version_string();
    char buf[40];
    snprintf(buf, sizeof buf, "%016llx-%016llx", (unsigned long long)fnv1a(all),
             (unsigned long long)fnv1a(all, 0x84222325cbf29ce4ull));
    // Named after the template, not the kernel: every kernel of one code
    // object (e.g. a dispatch kernel and its reset kernel) shares the entry.
    return ks.file + "-" + buf;
}

// Semi-permanent on-disk cache (Fig. 2: compiled code survives the process
// and is reused while source and environment are unchanged).  The file name
// is the cache key, which already hashes the source, the options, the
// architecture and the compiler version.  Entries carry a checksum; a
// damaged entry is ignored and rewritten.
std::string disk_cache_dir() {
    const char* off = getenv("FBCORR_CACHE");
    if (off && std::string(off) == "0") return "";
    const char* env = getenv("FBCORR_CACHE_DIR");
    if (env && *env) return env;
    Dl_info info;
    if (dladdr((void*)&disk_cache_dir, &info) && info.dli_fname) {
        std::string so = info.dli_fname;
        auto slash = so.rfind('/');
        return (slash == std::string::npos ? std::string(".") : so.substr(0, slash)) + "/_rtc_cache";
    }
    return "";
}

static const char kMagic[8] = {'F', 'B', 'C', 'C', 'O', 'D', 'E', '1'};

static bool disk_load(const std::string& key, std::vector<char>& code) {
    const std::string dir = disk_cache_dir();
    if (dir.empty()) return false;
    std::ifstream in(dir + "/" + key + ".co", std::ios::binary);
    if (!in) return false;
    char magic[8];
    uint64_t size = 0, sum = 0;
    if (!in.read(magic, 8) || memcmp(magic, kMagic, 8) != 0) return false;
    if (!in.read((char*)&size, 8) || !in.read((char*)&sum, 8) || size == 0 || size > (1ull << 30)) return false;
    code.resize(size);
    if (!in.read(code.data(), (std::streamsize)size)) return false;
    return fnv1a(std::string(code.data(), code.size())) == sum;
}

static void disk_store(const std::string& key, const std::vector<char>& code) {
    const std::string dir = disk_cache_dir();
    if (dir.empty()) return;
    mkdir(dir.c_str(), 0755);
    const std::string path = dir + "/" + key + ".co";
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    {
        std::ofstream out(tmp, std::ios::binary);
        if (!out) return;
        const uint64_t size = code.size(), sum = fnv1a(std::string(code.data(), code.size()));
        out.write(kMagic, 8);
        out.write((const char*)&size, 8);
        out.write((const char*)&sum, 8);
        out.write(code.data(), (std::streamsize)size);
        if (!out) { out.close(); unlink(tmp.c_str()); return; }
    }
    if (rename(tmp.c_str(), path.c_str()) != 0) unlink(tmp.c_str());
}

static bool supported_arch(const std::string& a) {
    // The kernels use CDNA3/CDNA4 matrix instructions; gfx950 is the target.
    return a == "gfx950";
}

bool tune_progress_on() {
    static const bool on = [] {
        const char* e = getenv("FBCORR_TUNE_PROGRESS");
        return e && *e && strcmp(e, "0") != 0;
    }();
    return on;
}

void tune_progress(const char* fmt, ...) {
    if (!tune_progress_on()) return;
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    va_list ap;
    va_start(ap, fmt);
    fputs("fbcorr tune: ", stderr);
    vfprintf(stderr, fmt, ap);
    fputc('\n', stderr);
    fflush(stderr);
    va_end(ap);
}

// FBCORR_CACHE_TRACE=1 prints one line per lookup to stderr: where the code
// object came from (memory, disk, compile) and its key.
static void trace_lookup(const char* where, const std::string& key) {
    static const bool on = [] {
        const char* e = getenv("FBCORR_CACHE_TRACE");
        return e && *e && strcmp(e, "0") != 0;
    }();
    if (on) fprintf(stderr, "fbcorr cache: %-7s %s\n", where, key.c_str());
}

// FBCORR_KEEP_SOURCE=<dir> writes every generated source that is compiled
// (not served from a cache) to <dir>/<key>.hip, with its compiler options in
// a leading comment, so a kernel can be inspected or rebuilt offline.
static void keep_source(const KernelSource& ks, const std::string& key) {
    const char* dir = getenv("FBCORR_KEEP_SOURCE");
    if (!dir || !*dir) return;
    FILE* f = fopen((std::string(dir) + "/" + key + ".hip").c_str(), "w");
    if (!f) return;
    fputs("// options:", f);
    for (auto& o : ks.options) fprintf(f, " %s", o.c_str());
    fputs("\n", f);
    fwrite(ks.source.data(), 1, ks.source.size(), f);
    fclose(f);
}

fbcorr_status compile_cached(const KernelSource& ks, const std::string& arch,
                             std::shared_ptr<const std::vector<char>>& code) {
    FBC_RETURN_IF(!supported_arch(arch), FBCORR_ERR_UNSUPPORTED, "architecture '" + arch + "' is not supported");
    const std::string key = cache_key(ks, arch);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_code.find(key);
        if (it != g_code.end()) {
            ++g_hits;
            code = it->second;
            trace_lookup("memory", key);
            return FBCORR_OK;
        }
    }
    {
        auto buf = std::make_shared<std::vector<char>>();
        if (disk_load(key, *buf)) {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            ++g_disk_hits;
            g_code[key] = buf;
            code = buf;
            trace_lookup("disk", key);
            return FBCORR_OK;
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        ++g_misses;
    }
    trace_lookup("compile", key);
    keep_source(ks, key);
    hiprtcProgram prog;
    hiprtcResult r = hiprtcCreateProgram(&prog, ks.source.c_str(), (ks.file + ".hip").c_str(), 0, nullptr, nullptr);
    FBC_RETURN_IF(r != HIPRTC_SUCCESS, FBCORR_ERR_COMPILE, std::string("hiprtcCreateProgram: ") + hiprtcGetErrorString(r));
    std::vector<std::string> opts;
    opts.push_back("--offload-arch=" + arch);
    opts.push_back("-O3");
    // Packed fp32 instructions are kept out of every kernel.
    opts.push_back("-Xclang"); opts.push_back("-target-feature");
    opts.push_back("-Xclang"); opts.push_back("-packed-fp32-ops");
    for (auto& o : ks.options) opts.push_back(o);
    std::vector<const char*> cop;
    for (auto& o : opts) cop.push_back(o.c_str());
    r = hiprtcCompileProgram(prog, (int)cop.size(), cop.data());
    if (r != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls, '\0');
        if (ls) hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        std::string optstr;
        for (auto& o : ks.options) optstr += o + " ";
        set_error(FBCORR_ERR_COMPILE, ks.name + " [" + optstr + "]: " + log);
        return FBCORR_ERR_COMPILE;
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    auto buf = std::make_shared<std::vector<char>>(cs);
    hiprtcGetCode(prog, buf->data());
    hiprtcDestroyProgram(&prog);
    disk_store(key, *buf);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        g_code[key] = buf;
    }
    code = buf;
    return FBCORR_OK;
}

void cache_stats(int64_t& hits, int64_t& misses, int64_t& entries, int64_t& disk_hits) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    hits = g_hits; misses = g_misses; entries = (int64_t)g_code.size(); disk_hits = g_disk_hits;
}

void cache_clear_memory() {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_code.clear();
}

fbcorr_status device_info(int device, DeviceInfo& out) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    FBC_RETURN_IF(e != hipSuccess || count <= 0, FBCORR_ERR_NO_DEVICE, "no HIP device available");
    FBC_RETURN_IF(device < 0 || device >= count, FBCORR_ERR_NO_DEVICE,
                  "device index " + std::to_string(device) + " out of range");
    hipDeviceProp_t p;
    e = hipGetDeviceProperties(&p, device);
    FBC_RETURN_IF(e != hipSuccess, FBCORR_ERR_NO_DEVICE, std::string("hipGetDeviceProperties: ") + hipGetErrorString(e));
    std::string arch = p.gcnArchName;
    auto colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    out.arch = arch;
    out.cus = p.multiProcessorCount;
    out.lds_per_block = (int)p.sharedMemPerBlock;
    out.max_threads = p.maxThreadsPerBlock;
    return FBCORR_OK;
}

fbcorr_status load_kernel(const KernelSource& ks, int device, Kernel& out) {
    DeviceInfo di;
    fbcorr_status st = device_info(device, di);
    if (st != FBCORR_OK) return st;
    const std::string key = cache_key(ks, di.arch);
    hipModule_t mod = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_modules.find(LoadedKey{device, key});
        if (it != g_modules.end()) mod = it->second;
    }
    if (!mod) {
        std::shared_ptr<const std::vector<char>> code;
        st = compile_cached(ks, di.arch, code);
        if (st != FBCORR_OK) return st;
        int prev = 0;
        hipGetDevice(&prev);
        hipSetDevice(device);
        hipError_t e = hipModuleLoadData(&mod, code->data());
        hipSetDevice(prev);
        FBC_RETURN_IF(e != hipSuccess, FBCORR_ERR_LAUNCH, std::string("hipModuleLoadData: ") + hipGetErrorString(e));
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto ins = g_modules.emplace(LoadedKey{device, key}, mod);
        if (!ins.second) {               // another thread won the race
            hipModuleUnload(mod);
            mod = ins.first->second;
        }
    }
    hipFunction_t fn = nullptr;
    hipError_t e = hipModuleGetFunction(&fn, mod, ks.name.c_str());
    FBC_RETURN_IF(e != hipSuccess, FBCORR_ERR_LAUNCH, std::string("hipModuleGetFunction(") + ks.name + "): " + hipGetErrorString(e));
    int regs = 0, lds = 0;
    hipFuncGetAttribute(&regs, HIP_FUNC_ATTRIBUTE_NUM_REGS, fn);
    hipFuncGetAttribute(&lds, HIP_FUNC_ATTRIBUTE_SHARED_SIZE_BYTES, fn);
    out.fn = fn;
    out.vgprs = regs;
    out.lds_bytes = lds;
    out.key = key;
    return FBCORR_OK;
}

}  // namespace fbc

extern "C" const char* fbcorr_last_error(void) { return fbc::t_last_error.c_str(); }
