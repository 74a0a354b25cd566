// Many uneven images in one persistent launch.
//
// Every distinct problem key (fh, fw, D, N) of the batch gets one tile
// configuration, and the generator emits one kernel holding exactly those
// variants (Sec. 4.2: generate code for exactly one purpose): the
// implicit-GEMM body section is pasted once per key with that key's constants
// substituted and the image extents left run-time, followed by a dispatch
// loop.  Each body stays a function of its own (not inlined into the loop),
// so registers are allocated per variant.  At plan time the host builds a work table of (variant, image, tile)
// items sorted by cost, largest first; at run time each persistent
// workgroup takes the next item from an integer counter until the table is
// exhausted.  The launch (a counter-reset kernel plus the persistent kernel)
// can be captured once into a HIP graph per stream and replayed.
#include "plan.h"

#include <algorithm>
#include <cstring>
#include <numeric>
#include <set>
#include <sstream>

namespace fbc {

struct BVariant {
    int fh, fw, D, N;
    Config cfg;
    int th, two, cb;       // tile geometry: output rows, columns, channels
    int lds;
    // the -DFB_<name>[=<value>] options build_role generated for this key's
    // standalone kernel (clamped and completed exactly as that kernel was)
    std::vector<std::string> opts;
};

struct BatchedState {
    std::vector<fbcorr_desc> descs;
    std::vector<BVariant> vars;
    std::vector<int> img_var;
    std::vector<int32_t> items;     // 4 ints per item: variant, image, tile, 0
    std::vector<int32_t> imgs;      // 4 ints per image: H, W, Ho, Wo
    Kernel kernel, reset;
    int grid = 0, threads = 256, per_cu = 1;
    size_t off_counter = 0, off_items = 0, off_imgs = 0, ws_bytes = 0;
    int64_t nitems = 0;
    double flops = 0;
    std::string source_desc;
    // uploads and graphs
    std::set<void*> uploaded;
    struct GraphKey {
        hipStream_t s;
        void* ws;
        const void *xs, *wts, *ys;
        bool operator<(const GraphKey& o) const {
            return std::tie(s, ws, xs, wts, ys) < std::tie(o.s, o.ws, o.xs, o.wts, o.ys);
        }
    };
    std::map<GraphKey, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
    std::mutex mu;           // uploads and graphs are shared by calling threads
};

static int cdiv(int a, int b) { return (a + b - 1) / b; }
static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Four waves per workgroup for every variant (one block size for the launch).
static Config batched_variant_config(int D, int N) {
    Config c = default_igemm(D, N, false);
    const int s = c.get("s");
    const int tiles = std::min(4, std::max(1, cdiv(N * s, 32)));
    int nt = 1, wn = 1;
    if (tiles >= 4) { nt = 2; wn = 2; }
    else if (tiles >= 2) { nt = 2; wn = 1; }
    const int wm = 4 / wn;
    c.v["nt"] = nt;
    c.v["wn"] = wn;
    c.v["wm"] = wm;
    c.v["ks"] = 1;
    c.v["mt"] = 1;
    c.v["mr"] = 2;
    c.v["ustage"] = 1;
    c.v["kc"] = D <= 16 ? D : 16;
    c.v["mf"] = 32;
    return c;
}

static std::vector<std::string> body_macros(const std::string& body) {
    std::vector<std::string> names;
    std::istringstream is(body);
    std::string line;
    while (std::getline(is, line)) {
        size_t p = line.find_first_not_of(" \t");
        if (p == std::string::npos || line.compare(p, 7, "#define") != 0) continue;
        std::istringstream ls(line.substr(p + 7));
        std::string name;
        ls >> name;
        auto paren = name.find('(');
        if (paren != std::string::npos) name = name.substr(0, paren);
        if (!name.empty()) names.push_back(name);
    }
    return names;
}

static bool generate(BatchedState& st, const DeviceInfo& di, KernelSource& ks, std::string& err) {
    const std::string& tpl = template_source("igemm");
    const auto b0 = tpl.find("//@@BODY-BEGIN"), b1 = tpl.find("//@@BODY-END");
    if (b0 == std::string::npos || b1 == std::string::npos) { err = "igemm template lacks body markers"; return false; }
    const std::string header = tpl.substr(0, b0);
    const std::string body = tpl.substr(b0, b1 - b0);
    const std::vector<std::string> macros = body_macros(body);
    std::ostringstream src;
    src << "// Generated persistent batched filter-bank correlation: " << st.vars.size() << " variant(s).\n";
    src << "#define FB_BATCHED 1\n" << header;
    int maxlds = 16;
    // Options of the standalone kernel that do not apply inside the
    // persistent kernel: its name, the batch, the image extents (run-time
    // arguments here) and the workgroup order (set by the dispatch loop).
    static const std::set<std::string> skip = {"FB_KNAME", "FB_BATCH", "FB_HI", "FB_WI", "FB_HO", "FB_WO",
                                               "FB_XCDMAP"};
    for (size_t v = 0; v < st.vars.size(); ++v) {
        const BVariant& bv = st.vars[v];
        src << "\n// ---- variant " << v << ": fh=" << bv.fh << " fw=" << bv.fw << " D=" << bv.D << " N=" << bv.N
            << "  [" << bv.cfg.str() << "]\n";
        src << "#undef FB_TAG\n#define FB_TAG v" << v << "\n";
        // The variant's constants are exactly those its standalone kernel
        // was built (and tuned) with: clamped values, unrolling switches and
        // all.
        std::vector<std::string> defined;
        for (const std::string& o : bv.opts) {
            if (o.compare(0, 2, "-D") != 0) continue;
            const auto eq = o.find('=');
            const std::string name = o.substr(2, eq == std::string::npos ? std::string::npos : eq - 2);
            if (skip.count(name) || name.find('(') != std::string::npos) continue;
            src << "#define " << name << " " << (eq == std::string::npos ? std::string("1") : o.substr(eq + 1))
                << "\n";
            defined.push_back(name);
        }
        src << body << "\n";
        for (auto& m : macros) src << "#undef " << m << "\n";
        for (auto& d : defined) src << "#undef " << d << "\n";
        maxlds = std::max(maxlds, bv.lds);
    }
    src << "\n#define MAXLDS " << ((maxlds + 15) / 16 * 16) << "\n";
    src << R"KSRC(
// Dispatch: each workgroup takes (variant, image, tile) items from the
// counter until the table is exhausted; every workgroup then exits.  Two
// waves per SIMD (registers within 256; every variant's LDS within half a
// CU): two workgroups per CU.
extern "C" __global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
fbcorr_batched(const int4* __restrict__ items, const int nitems, const int4* __restrict__ imgs,
               const float* const* __restrict__ xs, const float* const* __restrict__ wts,
               float* const* __restrict__ ys, int* __restrict__ counter)
{
    __shared__ __attribute__((aligned(16))) unsigned char lds_raw[MAXLDS];
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int it = next;
        __syncthreads();
        if (it >= nitems) break;
        const int4 w = items[it];
        const int4 im = imgs[w.y];
        const float* x = xs[w.y];
        const float* wt = wts[w.y];
        float* y = ys[w.y];
        switch (w.x) {
)KSRC";
    for (size_t v = 0; v < st.vars.size(); ++v) {
        const BVariant& bv = st.vars[v];
        src << "        case " << v << ": {\n"
            << "            const int ntx = (im.w + " << bv.two - 1 << ") / " << bv.two << ";\n"
            << "            const int nty = (im.z + " << bv.th - 1 << ") / " << bv.th << ";\n"
            << "            const int tx = w.z % ntx, ty = (w.z / ntx) % nty, cb = w.z / (ntx * nty);\n"
            << "            igemm_body_v" << v << "(x, wt, nullptr, y, im.x, im.y, im.z, im.w, ty * " << bv.th
            << ", tx * " << bv.two << ", cb * " << bv.cb << ", lds_raw);\n"
            << "        } break;\n";
    }
    src << R"KSRC(        default: break;
        }
    }
}

extern "C" __global__ void __launch_bounds__(64) fbcorr_batched_reset(int* __restrict__ counter)
{
    if (threadIdx.x == 0) *counter = 0;
}
)KSRC";
    ks.name = "fbcorr_batched";
    ks.file = "batched";
    ks.source = src.str();
    ks.options.clear();
    (void)di;
    return true;
}

void destroy_batched(Plan* p) {
    if (!p->bstate) return;
    for (auto& g : p->bstate->graphs) {
        hipGraphExecDestroy(g.second.second);
        hipGraphDestroy(g.second.first);
    }
    delete p->bstate;
    p->bstate = nullptr;
}

std::string batched_describe(const Plan* p) {
    if (!p->bstate) return "batched";
    std::ostringstream os;
    os << "batched images=" << p->bstate->descs.size() << " variants=" << p->bstate->vars.size()
       << " items=" << p->bstate->nitems << " grid=" << p->bstate->grid << " per_cu=" << p->bstate->per_cu;
    for (size_t v = 0; v < p->bstate->vars.size(); ++v) {
        const BVariant& b = p->bstate->vars[v];
        os << " | v" << v << " fh=" << b.fh << " fw=" << b.fw << " D=" << b.D << " N=" << b.N << " " << b.cfg.str();
    }
    return os.str();
}

// Plan-time work shared by the device and the offline paths: variants, the
// work table, the workspace layout and the generated source.
using KeyT = std::tuple<int, int, int, int>;

// The tuning-database key of a batched variant: role "batched", extents 0.
static fbcorr_desc variant_key_desc(int fh, int fw, int D, int N) {
    fbcorr_desc k{};
    k.batch = 1; k.H = 0; k.W = 0; k.D = D; k.N = N; k.fh = fh; k.fw = fw;
    k.precision = FBCORR_FP32; k.algo = FBCORR_ALGO_AUTO; k.flags = 0;
    return k;
}
static const int kRoleBatched = 3;

static bool four_waves(const Config& c) {
    return c.algo == "igemm" && c.get("wm") * c.get("wn") * c.get("ks") == 4;
}

static fbcorr_status prepare_batched(const DeviceInfo& dev, int32_t count, const fbcorr_desc* descs,
                                     BatchedState* st, KernelSource& ks,
                                     const std::map<KeyT, Config>* overrides = nullptr) {
    std::map<KeyT, int> keyidx;
    for (int32_t i = 0; i < count; ++i) {
        fbcorr_desc d = descs[i];
        fbcorr_status s0 = validate_desc(&d);
        if (s0 != FBCORR_OK) return s0;
        FBC_RETURN_IF(d.batch != 1, FBCORR_ERR_INVALID_ARGUMENT, "batched descriptors must have batch = 1");
        FBC_RETURN_IF(d.precision != FBCORR_FP32, FBCORR_ERR_UNSUPPORTED, "batched plans compute in fp32");
        st->descs.push_back(d);
        auto key = std::make_tuple(d.fh, d.fw, d.D, d.N);
        auto it = keyidx.find(key);
        if (it == keyidx.end()) {
            BVariant bv{d.fh, d.fw, d.D, d.N, batched_variant_config(d.D, d.N), 0, 0, 0, 0};
            RoleBuild rb;
            std::string err;
            bool ok = false;
            // a tuned configuration for this key: from the caller, else the database
            Config tuned;
            bool have = false;
            if (overrides) {
                auto o = overrides->find(key);
                if (o != overrides->end()) { tuned = o->second; have = true; }
            }
            std::string text;
            if (!have && tuning_db_lookup(dev.arch, kRoleBatched, variant_key_desc(d.fh, d.fw, d.D, d.N), text)) {
                tuned = bv.cfg;
                have = parse_config(text, tuned, err);
            }
            if (have && four_waves(tuned) && build_role(d, FBCORR_ROLE_FORWARD, tuned, dev, rb, err) &&
                rb.main_geom.lds <= dev.lds_per_block / 2 - 256) {
                bv.cfg = tuned;
                ok = true;
            }
            // otherwise the heuristic, shrunk until it fits half a CU's LDS
            // (the launch's occupancy is set by its largest variant: two
            // workgroups per CU need every variant within half)
            for (int attempt = 0; attempt < 8 && !ok; ++attempt) {
                ok = build_role(d, FBCORR_ROLE_FORWARD, bv.cfg, dev, rb, err) &&
                     rb.main_geom.lds <= dev.lds_per_block / 2 - 256;
                if (!ok) {
                    if (bv.cfg.v["kc"] > 4) bv.cfg.v["kc"] /= 2;
                    else if (bv.cfg.v["mr"] > 1) bv.cfg.v["mr"] /= 2;
                    else if (bv.cfg.v["nt"] > 1) bv.cfg.v["nt"] /= 2;
                    else break;
                }
            }
            // the smallest configuration if even that does not fit half
            if (!ok) ok = build_role(d, FBCORR_ROLE_FORWARD, bv.cfg, dev, rb, err);
            FBC_RETURN_IF(!ok, FBCORR_ERR_UNSUPPORTED, "no batched variant fits for key: " + err);
            const int s = bv.cfg.get("s");
            bv.th = bv.cfg.get("wm") * bv.cfg.get("mt") * bv.cfg.get("mr");
            const int mf = bv.cfg.get("mf");
            bv.two = s * (mf / bv.cfg.get("mr"));
            bv.cb = bv.cfg.get("wn") * bv.cfg.get("nt") * mf / s;
            bv.lds = rb.main_geom.lds;
            bv.opts = rb.main.options;
            it = keyidx.emplace(key, (int)st->vars.size()).first;
            st->vars.push_back(bv);
        }
        st->img_var.push_back(it->second);
    }
    // work table, largest tiles first (stable: image, then tile order)
    struct Item { double cost; int v, img, tile; };
    std::vector<Item> items;
    for (int32_t i = 0; i < count; ++i) {
        const fbcorr_desc& d = st->descs[i];
        const BVariant& bv = st->vars[st->img_var[i]];
        const int ho = d.H - d.fh + 1, wo = d.W - d.fw + 1;
        const int nt = cdiv(wo, bv.two) * cdiv(ho, bv.th) * cdiv(d.N, bv.cb);
        const double cost = (double)bv.th * bv.two * bv.cb * d.fh * d.fw * d.D;
        for (int t = 0; t < nt; ++t) items.push_back({cost, st->img_var[i], i, t});
        st->imgs.insert(st->imgs.end(), {d.H, d.W, ho, wo});
        st->flops += 2.0 * ho * wo * d.N * d.fh * d.fw * d.D;
    }
    std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.cost > b.cost; });
    for (auto& it : items) st->items.insert(st->items.end(), {it.v, it.img, it.tile, 0});
    st->nitems = (int64_t)items.size();
    FBC_RETURN_IF(st->nitems > 0x7fffffff, FBCORR_ERR_UNSUPPORTED, "too many tiles");
    // workspace: counter | items | image table
    st->off_counter = 0;
    st->off_items = 256;
    st->off_imgs = st->off_items + align256(st->items.size() * 4);
    st->ws_bytes = st->off_imgs + align256(st->imgs.size() * 4);
    std::string err;
    FBC_RETURN_IF(!generate(*st, dev, ks, err), FBCORR_ERR_INTERNAL, err);
    return FBCORR_OK;
}

static fbcorr_status build_batched(Plan* p, int32_t count, const fbcorr_desc* descs) {
    std::unique_ptr<BatchedState> st(new BatchedState());
    KernelSource ks;
    fbcorr_status s = prepare_batched(p->dev, count, descs, st.get(), ks);
    if (s != FBCORR_OK) return s;
    s = load_kernel(ks, p->device, st->kernel);
    if (s != FBCORR_OK) return s;
    KernelSource rs = ks;
    rs.name = "fbcorr_batched_reset";
    s = load_kernel(rs, p->device, st->reset);
    if (s != FBCORR_OK) return s;
    int per_cu = 0;
    hipError_t e = hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, st->kernel.fn, 256, 0);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    st->per_cu = per_cu;
    st->grid = (int)std::min<int64_t>(st->nitems, (int64_t)p->dev.cus * per_cu);
    st->grid = std::max(st->grid, 1);
    p->batch_ws = st->ws_bytes;
    p->bstate = st.release();
    return FBCORR_OK;
}

static fbcorr_status launch_batched(Plan* p, const float* const* xs, const float* const* wts, float* const* ys,
                                    void* ws, hipStream_t s) {
    BatchedState* st = p->bstate;
    char* base = (char*)ws;
    int* counter = (int*)(base + st->off_counter);
    const void* items = base + st->off_items;
    const void* imgs = base + st->off_imgs;
    int nitems = (int)st->nitems;
    void* a0[] = {&counter};
    fbcorr_status r = launch(st->reset, LaunchGeom{1, 1, 64, 0}, s, a0);
    if (r != FBCORR_OK) return r;
    void* a1[] = {(void*)&items, &nitems, (void*)&imgs, (void*)&xs, (void*)&wts, (void*)&ys, &counter};
    hipEvent_t ev;
    timing_begin(p, FBCORR_ROLE_FORWARD, s, ev);
    r = launch(st->kernel, LaunchGeom{st->grid, 1, 256, 0}, s, a1);
    timing_end(p, FBCORR_ROLE_FORWARD, s, ev);
    return r;
}

// Representative problem of a variant: its largest image.
static fbcorr_desc variant_rep(const BatchedState* st, size_t v) {
    const BVariant& bv = st->vars[v];
    fbcorr_desc best{};
    double bf = -1;
    for (size_t i = 0; i < st->descs.size(); ++i) {
        if (st->img_var[i] != (int)v) continue;
        const fbcorr_desc& d = st->descs[i];
        const double f = (double)(d.H - d.fh + 1) * (d.W - d.fw + 1);
        if (f > bf) { bf = f; best = d; }
    }
    (void)bv;
    return best;
}

size_t batched_tune_workspace(const Plan* p) {
    size_t need = 0;
    if (!p->bstate) return 0;
    for (size_t v = 0; v < p->bstate->vars.size(); ++v) {
        Plan tmp;
        tmp.desc = variant_rep(p->bstate, v);
        tmp.device = p->device;
        tmp.dev = p->dev;
        need = std::max(need, tune_workspace(&tmp));
    }
    return need;
}

// Per-key tuning of a batched plan (Sec. 6.2: the best variant differs per
// input): each variant is tuned on its largest image among four-wave
// implicit-GEMM candidates, then the persistent kernel is regenerated.
fbcorr_status tune_batched(Plan* p, void* workspace, size_t workspace_bytes, hipStream_t s,
                           const fbcorr_tune_opts* opts, fbcorr_tune_report* report) {
    BatchedState* st = p->bstate;
    FBC_RETURN_IF(!st, FBCORR_ERR_INVALID_ARGUMENT, "not a batched plan");
    fbcorr_tune_opts o{};
    if (opts) o = *opts;
    o.role = FBCORR_ROLE_FORWARD;
    o.flags &= ~(1u | 4u);      // no direct variants in the persistent kernel
    const bool record = opts && (opts->flags & 2u);
    fbcorr_tune_report total;
    memset(&total, 0, sizeof total);
    std::map<KeyT, Config> chosen;
    for (size_t v = 0; v < st->vars.size(); ++v) {
        const BVariant& bv = st->vars[v];
        Plan tmp;
        tmp.desc = variant_rep(st, v);
        tmp.device = p->device;
        tmp.dev = p->dev;
        fbcorr_tune_report r;
        Config best;
        fbcorr_status e = tune_plan(&tmp, nullptr, nullptr, nullptr, workspace, workspace_bytes, s, &o, true, false,
                                    &r, &best);
        if (e != FBCORR_OK) return e;
        total.n_tried += r.n_tried;
        total.n_compiled += r.n_compiled;
        total.n_rejected_resources += r.n_rejected_resources;
        total.n_rejected_parity += r.n_rejected_parity;
        total.n_failed += r.n_failed;
        total.best_ms += r.best_ms;
        total.default_ms += r.default_ms;
        const KeyT key = std::make_tuple(bv.fh, bv.fw, bv.D, bv.N);
        if (four_waves(best)) {
            chosen[key] = best;
            if (record) {
                std::string err;
                FBC_RETURN_IF(!tuning_db_record(p->dev.arch, kRoleBatched, variant_key_desc(bv.fh, bv.fw, bv.D, bv.N),
                                                best.str(), err),
                              FBCORR_ERR_INTERNAL, err);
            }
        }
    }
    // regenerate the persistent kernel with the chosen variants
    std::unique_ptr<BatchedState> ns(new BatchedState());
    KernelSource ks;
    fbcorr_status e = prepare_batched(p->dev, (int32_t)st->descs.size(), st->descs.data(), ns.get(), ks, &chosen);
    if (e != FBCORR_OK) return e;
    e = load_kernel(ks, p->device, ns->kernel);
    if (e != FBCORR_OK) return e;
    KernelSource rs = ks;
    rs.name = "fbcorr_batched_reset";
    e = load_kernel(rs, p->device, ns->reset);
    if (e != FBCORR_OK) return e;
    int per_cu = 0;
    if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ns->kernel.fn, 256, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    ns->per_cu = per_cu;
    ns->grid = (int)std::max<int64_t>(1, std::min<int64_t>(ns->nitems, (int64_t)p->dev.cus * per_cu));
    destroy_batched(p);
    p->batch_ws = ns->ws_bytes;
    p->bstate = ns.release();
    snprintf(total.best_cfg, sizeof total.best_cfg, "%zu variants tuned", chosen.size());
    snprintf(total.default_cfg, sizeof total.default_cfg, "per-key heuristics");
    if (report) *report = total;
    return FBCORR_OK;
}

}  // namespace fbc

using namespace fbc;

extern "C" fbcorr_status fbcorr_plan_batched(int32_t count, const fbcorr_desc* descs, int device, fbcorr_plan_t* out) {
    try {
        clear_error();
        FBC_RETURN_IF(!out || !descs, FBCORR_ERR_INVALID_ARGUMENT, "NULL argument");
        FBC_RETURN_IF(count <= 0, FBCORR_ERR_INVALID_ARGUMENT, "count must be >= 1");
        std::unique_ptr<Plan> p(new Plan());
        p->desc = descs[0];
        p->device = device;
        p->batched = true;
        fbcorr_status st = device_info(device, p->dev);
        if (st != FBCORR_OK) return st;
        DeviceGuard g(device);
        st = build_batched(p.get(), count, descs);
        if (st != FBCORR_OK) return st;
        *out = reinterpret_cast<fbcorr_plan_t>(p.release());
        return FBCORR_OK;
    } catch (const std::exception& e) {
        set_error(FBCORR_ERR_INTERNAL, std::string("exception: ") + e.what());
        return FBCORR_ERR_INTERNAL;
    }
}

extern "C" fbcorr_status fbcorr_forward_batched(fbcorr_plan_t plan, const float* const* xs, const float* const* ws_,
                                                float* const* ys, void* workspace, size_t workspace_bytes,
                                                void* stream, int use_graph) {
    try {
        clear_error();
        Plan* p = reinterpret_cast<Plan*>(plan);
        FBC_RETURN_IF(!p || !p->batched || !p->bstate, FBCORR_ERR_INVALID_ARGUMENT, "not a batched plan");
        FBC_RETURN_IF(!xs || !ws_ || !ys, FBCORR_ERR_INVALID_ARGUMENT, "pointer arrays must not be NULL");
        BatchedState* st = p->bstate;
        fbcorr_status r = check_ws(workspace, workspace_bytes, st->ws_bytes);
        if (r != FBCORR_OK) return r;
        DeviceGuard g(p->device);
        hipStream_t s = (hipStream_t)stream;
        std::lock_guard<std::mutex> lock(st->mu);
        if (!st->uploaded.count(workspace)) {
            // the work table and image table live in the caller's workspace
            char* base = (char*)workspace;
            hipError_t e = hipMemcpyAsync(base + st->off_items, st->items.data(), st->items.size() * 4,
                                          hipMemcpyHostToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(base + st->off_imgs, st->imgs.data(), st->imgs.size() * 4,
                                   hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            FBC_RETURN_IF(e != hipSuccess, FBCORR_ERR_LAUNCH, std::string("table upload: ") + hipGetErrorString(e));
            st->uploaded.insert(workspace);
        }
        if (!use_graph) return launch_batched(p, xs, ws_, ys, workspace, s);
        FBC_RETURN_IF(s == nullptr, FBCORR_ERR_INVALID_ARGUMENT,
                      "graph capture needs a created stream, not the null stream");
        BatchedState::GraphKey key{s, workspace, xs, ws_, ys};
        auto it = st->graphs.find(key);
        if (it == st->graphs.end()) {
            hipGraph_t graph = nullptr;
            hipGraphExec_t exec = nullptr;
            hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            FBC_RETURN_IF(e != hipSuccess, FBCORR_ERR_LAUNCH, std::string("begin capture: ") + hipGetErrorString(e));
            const bool was = p->timing;
            p->timing = false;             // no event records inside the graph
            r = launch_batched(p, xs, ws_, ys, workspace, s);
            p->timing = was;
            e = hipStreamEndCapture(s, &graph);
            FBC_RETURN_IF(r != FBCORR_OK, r, fbcorr_last_error());
            FBC_RETURN_IF(e != hipSuccess, FBCORR_ERR_LAUNCH, std::string("end capture: ") + hipGetErrorString(e));
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                hipGraphDestroy(graph);
                set_error(FBCORR_ERR_LAUNCH, std::string("graph instantiate: ") + hipGetErrorString(e));
                return FBCORR_ERR_LAUNCH;
            }
            it = st->graphs.emplace(key, std::make_pair(graph, exec)).first;
        }
        hipEvent_t ev;
        timing_begin(p, FBCORR_ROLE_FORWARD, s, ev);
        hipError_t e = hipGraphLaunch(it->second.second, s);
        timing_end(p, FBCORR_ROLE_FORWARD, s, ev);
        FBC_RETURN_IF(e != hipSuccess, FBCORR_ERR_LAUNCH, std::string("graph launch: ") + hipGetErrorString(e));
        return FBCORR_OK;
    } catch (const std::exception& e) {
        set_error(FBCORR_ERR_INTERNAL, std::string("exception: ") + e.what());
        return FBCORR_ERR_INTERNAL;
    }
}

extern "C" fbcorr_status fbcorr_compile_check_batched(int32_t count, const fbcorr_desc* descs, const char* arch,
                                                     size_t* code_bytes) {
    try {
        clear_error();
        FBC_RETURN_IF(!descs || count <= 0, FBCORR_ERR_INVALID_ARGUMENT, "need at least one descriptor");
        DeviceInfo di;
        di.arch = arch ? arch : "gfx950";
        di.cus = 256;
        di.lds_per_block = 160 * 1024;
        di.max_threads = 1024;
        BatchedState st;
        KernelSource ks;
        fbcorr_status s = prepare_batched(di, count, descs, &st, ks);
        if (s != FBCORR_OK) return s;
        std::shared_ptr<const std::vector<char>> code;
        s = compile_cached(ks, di.arch, code);
        if (s != FBCORR_OK) return s;
        if (code_bytes) *code_bytes = code->size();
        return FBCORR_OK;
    } catch (const std::exception& e) {
        set_error(FBCORR_ERR_INTERNAL, std::string("exception: ") + e.what());
        return FBCORR_ERR_INTERNAL;
    }
}
