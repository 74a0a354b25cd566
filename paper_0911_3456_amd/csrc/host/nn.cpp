// Exact nearest-neighbour search (Sec. 6.4) behind the fbnn_* entry points:
// plans, run-time specialised kernels, launches, timing and tuning.
//
// A search is five kernels from nn.hip: the neighbour norms with per-block
// counts of even norms, their prefix sums, the stable partition of the
// neighbours by norm parity (index and half-norm score term per position),
// the int8 matrix-core scan that keeps, per target and chunk, the best exact
// score and the first tile group reaching it, and the final selection that
// merges the chunks and re-measures that group's rows exactly.
#include "plan.h"
#include "fbnn.h"

#include <algorithm>
#include <atomic>
#include <cstring>
#include <set>
#include <thread>

namespace fbc {

namespace {

constexpr int kScoreTargets = 2048;   // workgroups the default chunking aims for

struct NNGeom {
    int nt = 0, wv = 0, ch = 0, fw = 0, tg = 0, bt = 0, split = 0;
    long tpg = 0, tb = 0, mts = 0, nblk = 0, nchk = 0;
    LaunchGeom norms, offsets, scatter, scan, fin;
    size_t off_hdr = 0, off_nn = 0, off_cnt = 0, off_perm = 0, off_cneg = 0, off_part = 0, ws_bytes = 0;
};

// The five kernels of a search, in launch order.
enum { K_NORMS, K_OFFSETS, K_SCATTER, K_SCAN, K_FINAL, K_COUNT };

struct NNBuild {
    Config cfg;
    NNGeom g;
    KernelSource ks[K_COUNT];
};

struct NNPlan {
    fbnn_desc desc{};
    int device = 0;
    DeviceInfo dev;
    NNBuild build;
    Kernel k[K_COUNT];
    std::mutex mu;
    bool timing = false;
    std::vector<std::array<hipEvent_t, 4>> pending;
    double acc_ms[3] = {0, 0, 0};
    int64_t acc_calls[3] = {0, 0, 0};
};

long cdiv(long a, long b) { return (a + b - 1) / b; }
size_t align256(size_t x) { return (x + 255) / 256 * 256; }

fbcorr_status validate(const fbnn_desc* d) {
    FBC_RETURN_IF(!d, FBCORR_ERR_INVALID_ARGUMENT, "descriptor is NULL");
    FBC_RETURN_IF(d->flags != 0, FBCORR_ERR_INVALID_ARGUMENT, "flags must be 0");
    FBC_RETURN_IF(d->n_targets < 0, FBCORR_ERR_INVALID_ARGUMENT, "n_targets < 0");
    FBC_RETURN_IF(d->n_neighbors < 1, FBCORR_ERR_INVALID_ARGUMENT, "the neighbour set is empty");
    FBC_RETURN_IF(d->n_neighbors + 16 >= (int64_t)1 << 31 || d->n_targets >= (int64_t)1 << 31,
                  FBCORR_ERR_UNSUPPORTED, "more than 2^31 - 16 rows");
    FBC_RETURN_IF(d->dim < 16 || d->dim > 512 || d->dim % 16 != 0, FBCORR_ERR_INVALID_ARGUMENT,
                  "dim must be a multiple of 16 in [16, 512]");
    return FBCORR_OK;
}

std::string db_key(const std::string& arch, const fbnn_desc& d) {
    return arch + " nearest u8 " + std::to_string(d.n_targets) + " " + std::to_string(d.n_neighbors) + " " +
           std::to_string(d.dim);
}

// Chunk length (neighbour tiles) that gives about `wgs` scan workgroups.
int chunk_for(const fbnn_desc& d, int nt, int wv, long wgs) {
    const long tb = std::max(1L, cdiv(std::max<int64_t>(d.n_targets, 1), (long)nt * wv * 16));
    const long mt = cdiv(d.n_neighbors, 16);
    const long chunks = std::max(1L, wgs / tb);
    return (int)std::max(1L, cdiv(mt, chunks));
}

Config heuristic(const fbnn_desc& d) {
    Config c;
    const int kb = (d.dim + 63) / 64;
    const int nt = std::max(1, std::min(8, 16 / kb));   // target fragments stay <= 64 VGPRs
    c.algo = "nn";
    c.v["nt"] = nt;
    c.v["wv"] = 4;
    c.v["bt"] = 4;
    c.v["tg"] = 2;
    // the parity partition costs three small kernels; it pays off once the
    // scan is long enough
    c.v["split"] = d.n_neighbors >= 65536 ? 1 : 0;
    c.v["xcd"] = 1;
    c.v["fw"] = 4;
    c.v["ch"] = chunk_for(d, nt, 4, kScoreTargets);
    return c;
}

bool make_build(const fbnn_desc& d, const Config& c, const DeviceInfo& di, NNBuild& b, std::string& err);

// The tuning database's entry when there is one and it still builds (an
// entry written for another version of the kernels is ignored), else the
// heuristic.
Config default_cfg(const fbnn_desc& d, const DeviceInfo& di) {
    Config c = heuristic(d);
    std::string text, err;
    if (tuning_db_lookup_key(db_key(di.arch, d), text)) {
        Config t = c;
        NNBuild probe;
        if (parse_config(text, t, err) && make_build(d, t, di, probe, err)) c = t;
    }
    return c;
}

void opt(std::vector<std::string>& o, const char* k, long v) {
    o.push_back(std::string("-DFB_") + k + "=" + std::to_string(v));
}

bool make_build(const fbnn_desc& d, const Config& c, const DeviceInfo& di, NNBuild& b, std::string& err) {
    static const std::set<std::string> known = {"nt", "wv", "ch", "bt", "tg", "split", "xcd", "fw",
                                                "inject_error"};
    if (c.algo != "nn") { err = "algo must be nn"; return false; }
    for (auto& kv : c.v)
        if (!known.count(kv.first)) { err = "unknown key '" + kv.first + "' for algo=nn"; return false; }
    NNGeom& g = b.g;
    g.nt = c.get("nt");
    g.wv = c.get("wv");
    g.ch = c.get("ch");
    g.fw = c.get("fw");
    g.tg = c.get("tg");
    g.bt = c.get("bt");
    g.split = c.get("split");
    const int xcd = c.get("xcd");
    const int kb = (d.dim + 63) / 64;
    if (g.nt < 1 || g.nt > 8) { err = "nt must be in [1, 8]"; return false; }
    if (g.nt * kb > 16) { err = "nt * ceil(dim/64) > 16 (target fragments would not fit in registers)"; return false; }
    if (g.wv < 1 || g.wv * 64 > di.max_threads) { err = "wv out of range"; return false; }
    if (g.fw != 1 && g.fw != 2 && g.fw != 4 && g.fw != 8 && g.fw != 16) {
        err = "fw must be 1, 2, 4, 8 or 16";
        return false;
    }
    if (g.ch < 1) { err = "ch must be >= 1"; return false; }
    if (g.bt != 1 && g.bt != 2 && g.bt != 4 && g.bt != 8 && g.bt != 16) { err = "bt must be 1, 2, 4, 8 or 16"; return false; }
    if (g.tg != 1 && g.tg != 2 && g.tg != 4) { err = "tg must be 1, 2 or 4"; return false; }
    if (g.bt % g.tg != 0) { err = "tg must divide bt"; return false; }
    if (g.split < 0 || g.split > 1 || xcd < 0 || xcd > 1) { err = "split and xcd are 0 or 1"; return false; }
    const long lds = 2L * g.bt * 16 * (d.dim + 16) + 2L * g.bt * 16 * 4;
    if (lds > di.lds_per_block) { err = "LDS batch exceeds the device limit"; return false; }
    const long T = d.n_targets;
    g.tpg = (long)g.wv * g.nt * 16;
    g.tb = std::max(1L, cdiv(T, g.tpg));
    g.mts = cdiv(d.n_neighbors, 16) + g.split;   // with the partition: two classes padded to whole tiles
    g.nblk = cdiv(d.n_neighbors, 64);
    g.ch = (int)std::min<long>(g.ch, g.mts);
    g.nchk = cdiv(g.mts, g.ch);
    if (g.tb * g.nchk >= (1L << 31)) { err = "too many scan workgroups"; return false; }
    g.norms = LaunchGeom{(int)cdiv(g.nblk, 4), 1, 256, 0};   // four 64-row blocks per workgroup
    g.offsets = LaunchGeom{1, 1, 1024, 0};
    g.scatter = LaunchGeom{(int)g.nblk, 1, 64, 0};
    g.scan = LaunchGeom{(int)(g.tb * g.nchk), 1, g.wv * 64, 0};
    g.fin = LaunchGeom{(int)std::max(1L, cdiv(T, 16)), 1, g.fw * 64, 0};
    size_t off = 0;
    g.off_hdr = off;  off += 256;
    if (g.split) {
        g.off_nn = off;   off += align256((size_t)d.n_neighbors * 4);
        g.off_cnt = off;  off += align256((size_t)g.nblk * 4);
        g.off_perm = off; off += align256((size_t)g.mts * 16 * 4);
    }
    g.off_cneg = off; off += align256((size_t)g.mts * 16 * 4);
    g.off_part = off; off += align256((size_t)g.nchk * (size_t)std::max(T, 1L) * 8);
    g.ws_bytes = off;
    b.cfg = c;
    b.cfg.v["ch"] = g.ch;

    auto base = [&](KernelSource& ks, const char* name, const char* section) {
        ks = KernelSource();
        ks.name = name;
        ks.file = "nn";
        ks.source = template_source("nn");
        ks.options.push_back(std::string("-DFB_") + section);
        opt(ks.options, "T", std::max(T, 1L));
        opt(ks.options, "M", d.n_neighbors);
        opt(ks.options, "D", d.dim);
        opt(ks.options, "SPLIT", g.split);
        if (c.get("inject_error")) ks.options.push_back("-DFB_INJECT_ERROR");
    };
    for (auto& ks : b.ks) ks = KernelSource();
    base(b.ks[K_NORMS], "fbnn_norms", "NN_NORMS");
    if (g.split) {
        base(b.ks[K_OFFSETS], "fbnn_offsets", "NN_OFFSETS");
        base(b.ks[K_SCATTER], "fbnn_scatter", "NN_SCATTER");
    }
    base(b.ks[K_SCAN], "fbnn_scan", "NN_SCAN");
    auto& sc = b.ks[K_SCAN].options;
    opt(sc, "NT", g.nt);
    opt(sc, "WV", g.wv);
    opt(sc, "CH", g.ch);
    opt(sc, "BT", g.bt);
    opt(sc, "TG", g.tg);
    opt(sc, "XCDMAP", xcd);
    base(b.ks[K_FINAL], "fbnn_final", "NN_FINAL");
    opt(b.ks[K_FINAL].options, "FW", g.fw);
    opt(b.ks[K_FINAL].options, "TG", g.tg);
    opt(b.ks[K_FINAL].options, "NCHK", g.nchk);
    return true;
}

fbcorr_status load_build(NNPlan* p, const NNBuild& b, Kernel* k) {
    for (int i = 0; i < K_COUNT; ++i) {
        if (b.ks[i].name.empty()) continue;      // not part of this configuration
        fbcorr_status st = load_kernel(b.ks[i], p->device, k[i]);
        if (st != FBCORR_OK) return st;
    }
    return FBCORR_OK;
}

fbcorr_status install(NNPlan* p, const Config& c) {
    NNBuild b;
    std::string err;
    FBC_RETURN_IF(!make_build(p->desc, c, p->dev, b, err), FBCORR_ERR_UNSUPPORTED, err);
    Kernel k[K_COUNT];
    fbcorr_status st = load_build(p, b, k);
    if (st != FBCORR_OK) return st;
    std::lock_guard<std::mutex> lk(p->mu);
    p->build = b;
    for (int i = 0; i < K_COUNT; ++i) p->k[i] = k[i];
    return FBCORR_OK;
}

// Enqueue the five kernels of one search.  With events: ev[0] before the
// neighbour preparation, ev[1] before the scan, ev[2] before the final
// selection, ev[3] after it.
fbcorr_status run(const NNBuild& b, const Kernel* k, const uint8_t* tg, const uint8_t* nb, int32_t* idx,
                  int32_t* dist, void* ws, hipStream_t s, hipEvent_t* ev) {
    char* base = (char*)ws;
    int* hdr = (int*)(base + b.g.off_hdr);
    int* nn = (int*)(base + b.g.off_nn);
    int* cnt = (int*)(base + b.g.off_cnt);
    int* perm = (int*)(base + b.g.off_perm);
    int* cneg = (int*)(base + b.g.off_cneg);
    unsigned long long* part = (unsigned long long*)(base + b.g.off_part);
    fbcorr_status st;
    if (ev) hipEventRecord(ev[0], s);
    if (b.g.split) {
        {
            void* args[] = {&nb, &nn, &cnt};
            if ((st = launch(k[K_NORMS], b.g.norms, s, args))) return st;
        }
        {
            void* args[] = {&cnt, &hdr, &perm, &cneg};
            if ((st = launch(k[K_OFFSETS], b.g.offsets, s, args))) return st;
        }
        {
            void* args[] = {&nn, &cnt, &hdr, &perm, &cneg};
            if ((st = launch(k[K_SCATTER], b.g.scatter, s, args))) return st;
        }
    } else {
        int* unused = nullptr;
        void* args[] = {&nb, &cneg, &unused};       // start values -|n|^2 straight into cneg
        if ((st = launch(k[K_NORMS], b.g.norms, s, args))) return st;
    }
    if (ev) hipEventRecord(ev[1], s);
    {
        void* args[] = {&tg, &nb, &perm, &cneg, &hdr, &part};
        if ((st = launch(k[K_SCAN], b.g.scan, s, args))) return st;
    }
    if (ev) hipEventRecord(ev[2], s);
    {
        void* args[] = {&tg, &nb, &perm, &part, &idx, &dist};
        if ((st = launch(k[K_FINAL], b.g.fin, s, args))) return st;
    }
    if (ev) hipEventRecord(ev[3], s);
    return FBCORR_OK;
}

DeviceInfo offline(const char* arch) {
    DeviceInfo di;
    di.arch = arch ? arch : "gfx950";
    di.cus = 256;
    di.lds_per_block = 160 * 1024;
    di.max_threads = 1024;
    return di;
}

// Candidate configurations for the tuner: targets per wave, waves per
// workgroup, about how many scan workgroups (which sets the chunk length),
// load-ahead.  Duplicates (after clamping the chunk) are dropped.
std::vector<Config> candidates(const fbnn_desc& d) {
    std::vector<Config> out;
    std::set<std::string> seen;
    const int kb = (d.dim + 63) / 64;
    static const int btg[][2] = {{2, 1}, {4, 2}, {8, 2}, {8, 4}};
    for (int split : {0, 1})
        for (int nt : {2, 4, 8})
            for (int wv : {2, 4, 8})
                for (long wgs : {512L, 1024L, 2048L, 4096L})
                    for (auto& bg : btg) {
                        if (nt * kb > 16) continue;
                        Config c;
                        c.algo = "nn";
                        c.v["nt"] = nt;
                        c.v["wv"] = wv;
                        c.v["bt"] = bg[0];
                        c.v["tg"] = bg[1];
                        c.v["split"] = split;
                        c.v["xcd"] = 1;
                        c.v["fw"] = 4;
                        c.v["ch"] = chunk_for(d, nt, wv, wgs);
                        if (seen.insert(c.str()).second) out.push_back(c);
                    }
    return out;
}

size_t tune_ws(const NNPlan* p) {
    size_t need = 0;
    std::string err;
    for (auto& c : candidates(p->desc)) {
        NNBuild b;
        if (make_build(p->desc, c, p->dev, b, err)) need = std::max(need, b.g.ws_bytes);
    }
    need = std::max(need, p->build.g.ws_bytes);
    const size_t out = align256((size_t)std::max<int64_t>(p->desc.n_targets, 1) * 4);
    return need + 4 * out;      // reference idx/dist + candidate idx/dist
}

}  // namespace

}  // namespace fbc

using namespace fbc;

struct fbnn_plan_s {};   // opaque handle type; the object is an fbc::NNPlan

static NNPlan* as_plan(fbnn_plan_t h) { return reinterpret_cast<NNPlan*>(h); }

extern "C" {

fbcorr_status fbnn_plan(const fbnn_desc* desc, int device, fbnn_plan_t* out) {
    FBC_API_BEGIN
    clear_error();
    FBC_RETURN_IF(!out, FBCORR_ERR_INVALID_ARGUMENT, "output handle pointer is NULL");
    fbcorr_status st = validate(desc);
    if (st != FBCORR_OK) return st;
    std::unique_ptr<NNPlan> p(new NNPlan());
    p->desc = *desc;
    p->device = device;
    st = device_info(device, p->dev);
    if (st != FBCORR_OK) return st;
    DeviceGuard g(device);
    st = install(p.get(), default_cfg(*desc, p->dev));
    if (st != FBCORR_OK) return st;
    *out = reinterpret_cast<fbnn_plan_t>(p.release());
    return FBCORR_OK;
    FBC_API_END
}

fbcorr_status fbnn_plan_destroy(fbnn_plan_t plan) {
    FBC_API_BEGIN
    clear_error();
    NNPlan* p = as_plan(plan);
    if (!p) return FBCORR_OK;
    DeviceGuard g(p->device);
    for (auto& e : p->pending)
        for (auto ev : e) hipEventDestroy(ev);
    delete p;
    return FBCORR_OK;
    FBC_API_END
}

fbcorr_status fbnn_workspace_size(fbnn_plan_t plan, int pass, size_t* bytes) {
    FBC_API_BEGIN
    clear_error();
    NNPlan* p = as_plan(plan);
    FBC_RETURN_IF(!p || !bytes, FBCORR_ERR_INVALID_ARGUMENT, "NULL argument");
    FBC_RETURN_IF(pass != 0 && pass != 1, FBCORR_ERR_INVALID_ARGUMENT, "pass must be 0 (search) or 1 (tune)");
    std::lock_guard<std::mutex> lk(p->mu);
    *bytes = pass == 0 ? p->build.g.ws_bytes : tune_ws(p);
    return FBCORR_OK;
    FBC_API_END
}

fbcorr_status fbnn_search(fbnn_plan_t plan, const uint8_t* targets, const uint8_t* neighbors, int32_t* idx,
                          int32_t* dist, void* workspace, size_t workspace_bytes, void* stream) {
    FBC_API_BEGIN
    clear_error();
    NNPlan* p = as_plan(plan);
    FBC_RETURN_IF(!p, FBCORR_ERR_INVALID_ARGUMENT, "plan is NULL");
    if (p->desc.n_targets == 0) return FBCORR_OK;
    fbcorr_status st;
    if ((st = check_ptr(targets, "targets")) || (st = check_ptr(neighbors, "neighbors")) ||
        (st = check_ptr(idx, "idx")) || (st = check_ptr(dist, "dist")))
        return st;
    NNBuild b;
    Kernel k[K_COUNT];
    bool timing;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        b = p->build;
        for (int i = 0; i < K_COUNT; ++i) k[i] = p->k[i];
        timing = p->timing;
    }
    if ((st = check_ws(workspace, workspace_bytes, b.g.ws_bytes))) return st;
    DeviceGuard g(p->device);
    hipStream_t s = (hipStream_t)stream;
    std::array<hipEvent_t, 4> ev{};
    if (timing)
        for (auto& e : ev) hipEventCreate(&e);
    st = run(b, k, targets, neighbors, idx, dist, workspace, s, timing ? ev.data() : nullptr);
    if (timing) {
        std::lock_guard<std::mutex> lk(p->mu);
        p->pending.push_back(ev);
        if (p->pending.size() > kMaxPendingEvents) {    // fold the oldest half into the totals
            const size_t half = p->pending.size() / 2;
            for (size_t i = 0; i < half; ++i) {
                auto& e = p->pending[i];
                hipEventSynchronize(e[3]);
                for (int q = 0; q < 3; ++q) {
                    float t = 0.f;
                    if (hipEventElapsedTime(&t, e[q], e[q + 1]) == hipSuccess) {
                        p->acc_ms[q] += t;
                        p->acc_calls[q] += 1;
                    }
                }
                for (auto x : e) hipEventDestroy(x);
            }
            p->pending.erase(p->pending.begin(), p->pending.begin() + half);
        }
    }
    return st;
    FBC_API_END
}

fbcorr_status fbnn_plan_get_config(fbnn_plan_t plan, char* buf, size_t len) {
    FBC_API_BEGIN
    clear_error();
    NNPlan* p = as_plan(plan);
    FBC_RETURN_IF(!p || !buf || len == 0, FBCORR_ERR_INVALID_ARGUMENT, "NULL argument");
    std::string s;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        s = p->build.cfg.str();
    }
    FBC_RETURN_IF(s.size() + 1 > len, FBCORR_ERR_INVALID_ARGUMENT, "buffer too small");
    memcpy(buf, s.c_str(), s.size() + 1);
    return FBCORR_OK;
    FBC_API_END
}

fbcorr_status fbnn_plan_set_config(fbnn_plan_t plan, const char* cfg) {
    FBC_API_BEGIN
    clear_error();
    NNPlan* p = as_plan(plan);
    FBC_RETURN_IF(!p || !cfg, FBCORR_ERR_INVALID_ARGUMENT, "NULL argument");
    Config c;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        c = p->build.cfg;
    }
    std::string err;
    FBC_RETURN_IF(!parse_config(cfg, c, err), FBCORR_ERR_INVALID_ARGUMENT, err);
    DeviceGuard g(p->device);
    return install(p, c);
    FBC_API_END
}

fbcorr_status fbnn_plan_enable_timing(fbnn_plan_t plan, int enable) {
    FBC_API_BEGIN
    clear_error();
    NNPlan* p = as_plan(plan);
    FBC_RETURN_IF(!p, FBCORR_ERR_INVALID_ARGUMENT, "plan is NULL");
    std::lock_guard<std::mutex> lk(p->mu);
    p->timing = enable != 0;
    return FBCORR_OK;
    FBC_API_END
}

fbcorr_status fbnn_plan_read_timing(fbnn_plan_t plan, double* ms, int64_t* calls, int reset) {
    FBC_API_BEGIN
    clear_error();
    NNPlan* p = as_plan(plan);
    FBC_RETURN_IF(!p, FBCORR_ERR_INVALID_ARGUMENT, "plan is NULL");
    DeviceGuard g(p->device);
    std::lock_guard<std::mutex> lk(p->mu);
    for (auto& e : p->pending) {
        hipEventSynchronize(e[3]);
        for (int k = 0; k < 3; ++k) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, e[k], e[k + 1]) == hipSuccess) {
                p->acc_ms[k] += t;
                p->acc_calls[k] += 1;
            }
        }
        for (auto ev : e) hipEventDestroy(ev);
    }
    p->pending.clear();
    for (int k = 0; k < 3; ++k) {
        if (ms) ms[k] = p->acc_ms[k];
        if (calls) calls[k] = p->acc_calls[k];
        if (reset) {
            p->acc_ms[k] = 0;
            p->acc_calls[k] = 0;
        }
    }
    return FBCORR_OK;
    FBC_API_END
}

fbcorr_status fbnn_compile_check(const fbnn_desc* desc, const char* cfg, const char* arch, size_t* code_bytes) {
    FBC_API_BEGIN
    clear_error();
    fbcorr_status st = validate(desc);
    if (st != FBCORR_OK) return st;
    const DeviceInfo di = offline(arch);
    Config c = default_cfg(*desc, di);
    std::string err;
    FBC_RETURN_IF(cfg && !parse_config(cfg, c, err), FBCORR_ERR_INVALID_ARGUMENT, err);
    NNBuild b;
    FBC_RETURN_IF(!make_build(*desc, c, di, b, err), FBCORR_ERR_UNSUPPORTED, err);
    size_t total = 0;
    for (const KernelSource& ks : b.ks) {
        if (ks.name.empty()) continue;
        std::shared_ptr<const std::vector<char>> code;
        st = compile_cached(ks, di.arch, code);
        if (st != FBCORR_OK) return st;
        total += code->size();
    }
    if (code_bytes) *code_bytes = total;
    return FBCORR_OK;
    FBC_API_END
}

fbcorr_status fbnn_tune(fbnn_plan_t plan, const uint8_t* targets, const uint8_t* neighbors, void* workspace,
                        size_t workspace_bytes, void* stream, const fbcorr_tune_opts* opts,
                        fbcorr_tune_report* report) {
    FBC_API_BEGIN
    clear_error();
    NNPlan* p = as_plan(plan);
    FBC_RETURN_IF(!p, FBCORR_ERR_INVALID_ARGUMENT, "plan is NULL");
    FBC_RETURN_IF(p->desc.n_targets == 0, FBCORR_ERR_INVALID_ARGUMENT, "nothing to tune: no targets");
    fbcorr_status st;
    if ((st = check_ptr(targets, "targets")) || (st = check_ptr(neighbors, "neighbors"))) return st;
    const size_t need = tune_ws(p);
    if ((st = check_ws(workspace, workspace_bytes, need))) return st;
    const int warmup = opts ? std::max(0, opts->warmup) : 2;
    const int reps = opts ? std::max(1, opts->reps) : 10;
    const int max_cand = opts ? opts->max_candidates : 0;
    const bool record = opts && (opts->flags & 2);
    DeviceGuard g(p->device);
    hipStream_t s = (hipStream_t)stream;

    const long T = p->desc.n_targets;
    const size_t out = align256((size_t)T * 4);
    char* base = (char*)workspace;
    const size_t role_ws = need - 4 * out;
    int32_t* ref_i = (int32_t*)(base + role_ws);
    int32_t* ref_d = (int32_t*)(base + role_ws + out);
    int32_t* cand_i = (int32_t*)(base + role_ws + 2 * out);
    int32_t* cand_d = (int32_t*)(base + role_ws + 3 * out);

    fbcorr_tune_report rep;
    memset(&rep, 0, sizeof rep);

    auto time_it = [&](const NNBuild& b, const Kernel* k, int32_t* oi,
                       int32_t* od, double& ms) -> fbcorr_status {
        fbcorr_status r = FBCORR_OK;
        for (int i = 0; i < warmup && r == FBCORR_OK; ++i)
            r = run(b, k, targets, neighbors, oi, od, workspace, s, nullptr);
        std::vector<hipEvent_t> ev(reps + 1);
        for (auto& e : ev) hipEventCreate(&e);
        hipEventRecord(ev[0], s);
        for (int i = 0; i < reps && r == FBCORR_OK; ++i) {
            r = run(b, k, targets, neighbors, oi, od, workspace, s, nullptr);
            hipEventRecord(ev[i + 1], s);
        }
        hipError_t he = hipStreamSynchronize(s);
        std::vector<double> t;
        for (int i = 0; i < reps && r == FBCORR_OK; ++i) {
            float f = 0;
            hipEventElapsedTime(&f, ev[i], ev[i + 1]);
            t.push_back(f);
        }
        for (auto& e : ev) hipEventDestroy(e);
        if (r != FBCORR_OK) return r;
        FBC_RETURN_IF(he != hipSuccess, FBCORR_ERR_LAUNCH, std::string("stream: ") + hipGetErrorString(he));
        std::sort(t.begin(), t.end());
        ms = t[t.size() / 2];
        return FBCORR_OK;
    };

    // Reference: the heuristic default.
    NNBuild db;
    std::string err;
    const Config dcfg = heuristic(p->desc);
    FBC_RETURN_IF(!make_build(p->desc, dcfg, p->dev, db, err), FBCORR_ERR_INTERNAL, "default: " + err);
    Kernel dk[K_COUNT];
    if ((st = load_build(p, db, dk))) return st;
    double dms = 0;
    if ((st = time_it(db, dk, ref_i, ref_d, dms))) return st;
    std::vector<int32_t> hi(T), hd(T), ci(T), cd(T);
    hipError_t he = hipMemcpyDtoH(hi.data(), (hipDeviceptr_t)ref_i, T * 4);
    if (he == hipSuccess) he = hipMemcpyDtoH(hd.data(), (hipDeviceptr_t)ref_d, T * 4);
    FBC_RETURN_IF(he != hipSuccess, FBCORR_ERR_LAUNCH, std::string("copy: ") + hipGetErrorString(he));
    rep.default_ms = dms;
    snprintf(rep.default_cfg, sizeof rep.default_cfg, "%s", dcfg.str().c_str());

    // Candidates: build descriptions, deterministic subsample, parallel compile.
    std::vector<Config> cands = candidates(p->desc);
    if (max_cand > 0 && (int)cands.size() > max_cand) {
        std::vector<Config> pick;
        const double step = (double)cands.size() / max_cand;
        for (int i = 0; i < max_cand; ++i) pick.push_back(cands[(size_t)(i * step)]);
        cands.swap(pick);
    }
    std::vector<NNBuild> builds;
    for (auto& c : cands) {
        NNBuild b;
        ++rep.n_tried;
        if (!make_build(p->desc, c, p->dev, b, err)) {
            ++rep.n_rejected_resources;
            continue;
        }
        builds.push_back(b);
    }
    {
        std::vector<fbcorr_status> res(builds.size(), FBCORR_OK);
        std::atomic<size_t> next{0};
        std::atomic<size_t> done{0};
        auto worker = [&]() {
            for (size_t i; (i = next.fetch_add(1)) < builds.size();) {
                std::shared_ptr<const std::vector<char>> code;
                for (const KernelSource& ks : builds[i].ks) {
                    if (ks.name.empty()) continue;
                    res[i] = compile_cached(ks, p->dev.arch, code);
                    if (res[i] != FBCORR_OK) break;
                }
                const size_t n = ++done;
                if (n % 25 == 0 || n == builds.size())
                    tune_progress("nearest: compiled %zu of %zu candidates", n, builds.size());
            }
        };
        const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> pool;
        for (unsigned i = 0; i < nth; ++i) pool.emplace_back(worker);
        for (auto& th : pool) th.join();
        clear_error();
        std::vector<NNBuild> ok;
        for (size_t i = 0; i < builds.size(); ++i) {
            if (res[i] == FBCORR_OK) ok.push_back(builds[i]);
            else ++rep.n_failed;
        }
        builds.swap(ok);
    }

    double best = dms;
    NNBuild win = db;
    for (auto& b : builds) {
        Kernel k[K_COUNT];
        if (load_build(p, b, k) != FBCORR_OK) {
            ++rep.n_failed;
            clear_error();
            continue;
        }
        ++rep.n_compiled;
        double ms = 0;
        if ((st = time_it(b, k, cand_i, cand_d, ms))) return st;
        he = hipMemcpyDtoH(ci.data(), (hipDeviceptr_t)cand_i, T * 4);
        if (he == hipSuccess) he = hipMemcpyDtoH(cd.data(), (hipDeviceptr_t)cand_d, T * 4);
        FBC_RETURN_IF(he != hipSuccess, FBCORR_ERR_LAUNCH, std::string("copy: ") + hipGetErrorString(he));
        if (ci != hi || cd != hd) {       // an exact search must agree bit for bit
            ++rep.n_rejected_parity;
            continue;
        }
        if (ms < best) {
            best = ms;
            win = b;
        }
        tune_progress("nearest: timed %d, best %.4f ms (default %.4f ms)", rep.n_compiled, best, dms);
    }
    rep.best_ms = best;
    snprintf(rep.best_cfg, sizeof rep.best_cfg, "%s", win.cfg.str().c_str());
    if ((st = install(p, win.cfg))) return st;
    if (record) {
        FBC_RETURN_IF(!tuning_db_record_key(db_key(p->dev.arch, p->desc), win.cfg.str(), err),
                      FBCORR_ERR_INTERNAL, err);
    }
    if (report) *report = rep;
    return FBCORR_OK;
    FBC_API_END
}

}  // extern "C"
