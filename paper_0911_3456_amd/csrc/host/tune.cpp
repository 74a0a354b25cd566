// Automated tuning (Sec. 4.1; Sec. 6.2's "coarse grid search" over code
// variants).  Variants are generated from a grid of knobs, pruned by
// resources before anything runs (Sec. 6.1's early rejection of poor
// variants), compiled in parallel, gated for exactness against the default
// variant on integer-valued data, timed with HIP events, and the fastest is
// installed in the plan.
#include "plan.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <set>
#include <thread>

namespace fbc {

static int cdiv(long a, long b) { return (int)((a + b - 1) / b); }
static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct TuneLayout {
    size_t xi = 0, wi = 0, gi = 0, ref = 0, cand = 0, role_ws = 0, total = 0;
    size_t nx = 0, nw = 0, ny = 0, nout = 0;
};

static const size_t kMaxPartialsForTuning = 1024;

static TuneLayout tune_layout(const Plan* p) {
    const fbcorr_desc& d = p->desc;
    TuneLayout t;
    t.nx = (size_t)d.batch * d.H * d.W * d.D;
    t.nw = (size_t)d.N * d.fh * d.fw * d.D;
    t.ny = (size_t)d.batch * (d.H - d.fh + 1) * (d.W - d.fw + 1) * d.N;
    t.nout = std::max(t.nx, std::max(t.nw, t.ny));
    size_t off = 0;
    t.xi = off; off += align256(t.nx * 4);
    t.wi = off; off += align256(t.nw * 4);
    t.gi = off; off += align256(t.ny * 4);
    t.ref = off; off += align256(t.nout * 4);
    t.cand = off; off += align256(t.nout * 4);
    t.role_ws = off;
    // largest role workspace any candidate may ask for
    size_t rw = std::max(align256(t.nw * 2) + align256((size_t)d.N * 4 + 2048), align256(t.nw * 4));
    rw = std::max(rw, align256(kMaxPartialsForTuning * t.nw * 4));
    // the fragment-ordered bank of the register-streamed forward kernel:
    // columns padded to at most 256, chunks of at least 4 channels, steps of
    // at least 8 values (one padded step per filter row and chunk) and 8
    // ring steps per chunk, at most 64 bytes per column and step
    // (forward: columns N over D channels; input gradient: D over N)
    for (int r = 0; r < 2; ++r) {
        const int co = r == 0 ? d.N : d.D, ci = r == 0 ? d.D : d.N;
        const size_t cols = (size_t)(co + 255) / 256 * 256;
        const size_t chunks = (size_t)(ci + 3) / 4;
        const size_t steps = (size_t)d.fh * d.fw * (ci + 63) / 8 + chunks * d.fh + chunks * 8;
        rw = std::max(rw, align256(cols * steps * 64) + align256(cols * 4 + 2048));
    }
    off += rw;
    t.total = off;
    return t;
}

size_t tune_workspace(Plan* p) { return tune_layout(p).total; }

// ------------------------------------------------------------ candidate grids

static void add(std::vector<Config>& out, std::set<std::string>& seen, const Config& c) {
    if (seen.insert(c.str()).second) out.push_back(c);
}

std::vector<Config> tune_candidates(const fbcorr_desc& d, int role, bool with_direct, bool direct_only) {
    std::vector<Config> out;
    std::set<std::string> seen;
    const bool lowp = d.precision != FBCORR_FP32;
    if (role == FBCORR_ROLE_FORWARD || role == FBCORR_ROLE_BACKWARD_X) {
        const int cin = role == FBCORR_ROLE_FORWARD ? d.D : d.N;
        const int cout = role == FBCORR_ROLE_FORWARD ? d.N : d.D;
        const Config base = default_igemm(cin, cout, lowp && role == FBCORR_ROLE_FORWARD);
        const bool lp = lowp && role == FBCORR_ROLE_FORWARD;
        std::vector<int> kcs = {base.get("kc")};
        for (int kc : {4, 8, 16, 32})
            if (kc <= cin && (cin % kc == 0 || kc == 8) && (!lp || kc % 8 == 0) && kc != base.get("kc"))
                kcs.push_back(kc);
        std::vector<int> ss = {base.get("s")};
        if (base.get("s") > 1) ss.push_back(base.get("s") / 2);
        // (mt, nt, wm, wn): per-wave tiles and waves per contraction group
        const int shapes[][4] = {{1, 1, 4, 1}, {1, 2, 4, 1}, {2, 1, 2, 2}, {2, 2, 2, 1}, {1, 2, 2, 2},
                                 {2, 2, 4, 1}, {1, 4, 4, 1}, {2, 2, 2, 2}, {4, 2, 1, 1}, {1, 1, 8, 1},
                                 {1, 1, 1, 1}, {2, 1, 1, 1}, {1, 2, 1, 1}, {2, 2, 1, 1}, {1, 1, 2, 1},
                                 {2, 4, 2, 1}, {4, 2, 2, 1}, {4, 4, 1, 1}, {4, 4, 2, 1}, {2, 4, 4, 1},
                                 // 512-pixel workgroups: each staged filter slice serves twice the
                                 // products (16-bit operands, where the filter staging dominates)
                                 {2, 2, 8, 1}, {4, 1, 4, 1}, {1, 2, 16, 1}};
        std::vector<Config> grid;
        for (int kc : kcs)
            for (int s : ss)
              for (int mf : {32, 16})
                for (int mr : {1, 2, 4, 8})
                    for (auto& sh : shapes)
                        for (int ksp : {1, 2, 4})
                            for (int us : {1, 3})
                                for (int pad : {0, 1, 2, 3, 4}) {
                                    Config c = base;
                                    c.v["mf"] = mf;
                                    c.v["kc"] = kc;
                                    c.v["s"] = mf == 16 ? std::max(1, s / 2) : s;
                                    c.v["mr"] = mr;
                                    c.v["mt"] = sh[0]; c.v["nt"] = sh[1]; c.v["wm"] = sh[2]; c.v["wn"] = sh[3];
                                    c.v["ks"] = ksp;
                                    // skip tiles whose columns exceed what the channels can fill
                                    const int cs = c.v["s"];
                                    if (sh[1] * sh[3] * mf > std::max(mf, ((cout * cs + mf - 1) / mf) * mf)) continue;
                                    if (sh[0] * sh[1] * sh[2] * sh[3] * ksp > 32) continue;
                                    if (sh[0] * sh[1] > 8 && !lp) continue;   // big wave tiles pay off for 16-bit
                                    c.v["ustage"] = us;
                                    // LDS row padding (bank-conflict avoidance), in whole vectors
                                    const int unit = lp ? 8 : 4;
                                    const int xp[] = {0, 1, 2, 3, 3}, wp[] = {0, 1, 0, 3, 1};
                                    c.v["xpad"] = xp[pad] * unit;
                                    c.v["wpad"] = wp[pad] * unit;
                                    grid.push_back(c);
                                    if (role == FBCORR_ROLE_BACKWARD_X) {
                                        c.v["flip"] = 1;    // flip fused into the staging
                                        grid.push_back(c);
                                    }
                                    if (us > 1 && !lp) {
                                        c.v["uunr"] = 1;    // filter rows of a stage unrolled
                                        grid.push_back(c);
                                    }
                                    if (lp && kc == 16 && (s * kc) % 8 == 0) {
                                        Config z = c;
                                        z.v["swz"] = 1;     // swizzled 16-bit tile
                                        grid.push_back(z);
                                    }
                                }
        // a coarse, deterministic subsample of the full grid (Fisher-Yates
        // with a fixed LCG), the default first
        uint64_t st = 0x9E3779B97F4A7C15ull;
        for (size_t i = grid.size(); i > 1; --i) {
            st = st * 6364136223846793005ull + 1442695040888963407ull;
            std::swap(grid[i - 1], grid[(st >> 33) % i]);
        }
        // Filter fragments streamed into registers: tile size, chunk width,
        // tile rows, per-wave tiles and waves, ring depth, row padding,
        // register budget.  Interleaved with the staged-filter
        // grid so that any candidate budget samples both.
        std::vector<Config> rgrid;
        {
            const Config rb = default_rgemm(cin, cout, lp);
            const int pe = lp ? 8 : 4;
            std::vector<int> rkcs = {pe};
            for (int k : {2 * pe, 4 * pe, 8 * pe})
                if (k <= std::max(cin, 2 * pe) && (cin % pe == 0)) rkcs.push_back(k);
            const int rshapes[][4] = {{4, 2, 2, 2}, {4, 2, 1, 2}, {4, 2, 4, 1}, {2, 2, 2, 2}, {2, 2, 4, 2},
                                      {4, 1, 2, 4}, {4, 1, 4, 2}, {8, 1, 2, 2}, {2, 4, 2, 1}, {4, 2, 2, 1},
                                      {2, 2, 4, 1}, {4, 1, 4, 1}, {4, 4, 1, 2}, {2, 1, 4, 2}, {8, 1, 1, 4},
                                      // 16 tiles per wave: one wave per SIMD (wpe=1), half the
                                      // fragment loads per product of the 8-tile shapes
                                      {4, 4, 2, 1}, {4, 4, 4, 1}, {8, 2, 1, 2}, {8, 2, 2, 2}};
            // column shifts for banks narrower than a tile
            std::vector<int> rss = {1};
            for (int sv : {2, 4})
                if (cout * sv <= 32) rss.push_back(sv);
            for (int kc : rkcs)
              for (int mf : {32, 16})
               for (int sv : rss)
                for (int mr : {1, 2, 4})
                    for (auto& sh : rshapes)
                        for (int pf : {2, 3, 4, 6})
                            for (int xp : {0, 1})
                                for (int wpe : {1, 2})
                                  for (int nts : {0, 1})
                                   for (int ste : {0, 1}) {
                                    Config c = rb;
                                    c.v["nts"] = nts;
                                    if (ste && (sv != 1 || cout % 4)) continue;
                                    c.v["ste"] = ste;
                                    if (sh[1] * sh[3] * mf > std::max(mf, ((cout * sv + mf - 1) / mf) * mf)) continue;
                                    if (mf == 16 && cout > 64) continue;
                                    if (sv > 1 && (sh[1] * sh[3] * mf) % sv) continue;
                                    c.v["mf"] = mf;
                                    c.v["s"] = sv;
                                    c.v["kc"] = kc; c.v["mr"] = mr;
                                    c.v["mt"] = sh[0]; c.v["nt"] = sh[1]; c.v["wm"] = sh[2]; c.v["wn"] = sh[3];
                                    c.v["pf"] = pf; c.v["xpadc"] = xp; c.v["wpe"] = wpe;
                                    rgrid.push_back(c);
                                }
            uint64_t st2 = 0xD1B54A32D192ED03ull;
            for (size_t i = rgrid.size(); i > 1; --i) {
                st2 = st2 * 6364136223846793005ull + 1442695040888963407ull;
                std::swap(rgrid[i - 1], rgrid[(st2 >> 33) % i]);
            }
        }
        add(out, seen, base);
        if (!rgrid.empty()) add(out, seen, default_rgemm(cin, cout, lp));
        for (size_t i = 0; i < std::max(grid.size(), rgrid.size()); ++i) {
            if (i < rgrid.size()) add(out, seen, rgrid[i]);
            if (i < grid.size()) add(out, seen, grid[i]);
        }
        if (direct_only) out.clear();
        if ((with_direct || direct_only) && role == FBCORR_ROLE_FORWARD && !lowp) {
            const Config db = default_direct(d);
            for (int th : {4, 8, 16})
                for (int tw : {16, 32, 64})
                    for (int p : {2, 4, 8})
                        for (int q : {8, 16})
                            for (int nb : {32, 64})
                                for (int layout : {0, 1})
                                    for (int ds : {1, 2}) {
                                        Config c = db;
                                        c.v["th"] = th; c.v["tw"] = tw; c.v["p"] = p; c.v["q"] = q;
                                        c.v["nb"] = std::min(nb, ((d.N + q - 1) / q) * q);
                                        c.v["layout"] = layout;
                                        c.v["ds"] = (d.D % ds == 0) ? ds : 1;
                                        const int thr = th * (tw / p) * (c.v["nb"] / q) * c.v["ds"];
                                        if (thr < 64 || thr > 1024 || thr % 64) continue;
                                        add(out, seen, c);
                                        if (c.v["ds"] == 1 && (th * (tw / p)) % 64 == 0) {
                                            c.v["fsrc"] = 1;           // weights by scalar loads
                                            add(out, seen, c);
                                        }
                                    }
        }
    } else {
        const Config base = default_config(d, role, DeviceInfo{"gfx950", 256, 160 * 1024, 1024});
        const int tiles = ((d.N + 31) / 32) * ((d.fh * d.fw * d.D + 31) / 32);
        std::vector<Config> grid;
        // chunk widths: powers of two, and the widths that cut the output
        // width into k nearly equal chunks (exactly when k divides it), so
        // the last chunk column carries little or no padding
        std::vector<int> rws = {32, 64};
        const int wo = d.W - d.fw + 1;
        for (int k = 1; k <= 16; ++k) {
            const int rw = (wo + k - 1) / k;
            if (rw >= 16 && rw <= 128 && k * rw - wo < k &&
                std::find(rws.begin(), rws.end(), rw) == rws.end())
                rws.push_back(rw);
        }
        const int ho = d.H - d.fh + 1;
        for (int rh : {1, 2, 4})
            for (int rw : rws) {
                if ((rh * rw) % 2) continue;
                // partial counts: fixed fractions of the chip, and those that
                // give every workgroup the same number of chunks
                const long nchunks = (long)d.batch * cdiv(ho, rh) * cdiv(wo, rw);
                std::vector<int> nps = {32, 64, 128, 256};
                for (int k = 1; k <= 8; ++k)
                    if (nchunks % k == 0 && nchunks / k >= 32 && nchunks / k <= 512 &&
                        std::find(nps.begin(), nps.end(), (int)(nchunks / k)) == nps.end())
                        nps.push_back((int)(nchunks / k));
                for (int nw : {2, 4, 6, 8, 12, 14, 16})
                    for (int split : {1, 2, 3, 4, 6})
                        for (int np : nps)
                            for (int pf : {0, 1, 2})
                                for (int bal : {0, 1})
                                    for (int unr : {0, 4})
                                      for (int pad : {0, 4}) {
                                        Config c = base;
                                        c.v["rh"] = rh; c.v["rw"] = rw; c.v["nw"] = nw;
                                        c.v["tpb"] = (tiles + split - 1) / split;
                                        c.v["np"] = np; c.v["pf"] = pf; c.v["bal"] = bal; c.v["unr"] = unr;
                                        // row padding of the staged dy and input tiles (0: each
                                        // tile is one contiguous run in LDS)
                                        c.v["gpad"] = pad; c.v["xpad"] = pad;
                                        // round-robin deals: empty last slots skipped
                                        c.v["skipe"] = bal ? 0 : 1;
                                        grid.push_back(c);
                                    }
            }
        uint64_t st = 0x2545F4914F6CDD1Dull;
        for (size_t i = grid.size(); i > 1; --i) {
            st = st * 6364136223846793005ull + 1442695040888963407ull;
            std::swap(grid[i - 1], grid[(st >> 33) % i]);
        }
        add(out, seen, base);
        for (auto& c : grid) add(out, seen, c);
    }
    return out;
}

// ------------------------------------------------------------ running

struct TuneBuffers {
    const float *x, *w, *g;     // inputs for the role
    float* out;
    void* ws;
};

static fbcorr_status run_role(Plan* p, int role, const RoleExec& ex, const TuneBuffers& b, hipStream_t s) {
    if (role == FBCORR_ROLE_FORWARD) return run_forward(p, ex, b.x, b.w, b.out, b.ws, s);
    if (role == FBCORR_ROLE_BACKWARD_X) return run_backward_x(p, ex, b.w, b.g, b.out, b.ws, s);
    return run_backward_w(p, ex, b.x, b.g, b.out, b.ws, s);
}

static size_t out_elems(const TuneLayout& t, int role) {
    return role == FBCORR_ROLE_FORWARD ? t.ny : (role == FBCORR_ROLE_BACKWARD_X ? t.nx : t.nw);
}

static fbcorr_status fill_int(Plan* p, float* dst, size_t n, unsigned seed, int R, hipStream_t s) {
    KernelSource ks;
    ks.name = "fbcorr_fill_int";
    ks.file = "util";
    ks.source = template_source("util");
    ks.options.push_back("-DFB_FILL_INT");
    Kernel k;
    fbcorr_status st = load_kernel(ks, p->device, k);
    if (st != FBCORR_OK) return st;
    long nn = (long)n;
    void* args[] = {&dst, &nn, &seed, &R};
    LaunchGeom g{cdiv(nn, 256), 1, 256, 0};
    return launch(k, g, s, args);
}

static fbcorr_status time_role(Plan* p, int role, const RoleExec& ex, const TuneBuffers& b, hipStream_t s,
                               int warmup, int reps, double& ms) {
    const bool was = p->timing;
    p->timing = false;
    fbcorr_status st = FBCORR_OK;
    for (int i = 0; i < warmup && st == FBCORR_OK; ++i) st = run_role(p, role, ex, b, s);
    std::vector<hipEvent_t> ev(reps + 1);
    for (auto& e : ev) hipEventCreate(&e);
    hipEventRecord(ev[0], s);
    for (int i = 0; i < reps && st == FBCORR_OK; ++i) {
        st = run_role(p, role, ex, b, s);
        hipEventRecord(ev[i + 1], s);
    }
    hipError_t he = hipStreamSynchronize(s);
    std::vector<double> t;
    for (int i = 0; i < reps && st == FBCORR_OK; ++i) {
        float f = 0;
        hipEventElapsedTime(&f, ev[i], ev[i + 1]);
        t.push_back(f);
    }
    for (auto& e : ev) hipEventDestroy(e);
    p->timing = was;
    if (st != FBCORR_OK) return st;
    FBC_RETURN_IF(he != hipSuccess, FBCORR_ERR_LAUNCH, std::string("stream: ") + hipGetErrorString(he));
    std::sort(t.begin(), t.end());
    ms = t.empty() ? 1e30 : t[t.size() / 2];
    return FBCORR_OK;
}

static fbcorr_status make_exec(Plan* p, int role, const RoleBuild& rb, RoleExec& ex) {
    ex = RoleExec();
    ex.build = rb;
    fbcorr_status st = load_kernel(rb.main, p->device, ex.main);
    if (st != FBCORR_OK) return st;
    for (auto& a : rb.aux) {
        Kernel k;
        st = load_kernel(a, p->device, k);
        if (st != FBCORR_OK) return st;
        ex.aux.push_back(k);
    }
    return FBCORR_OK;
}

}  // namespace fbc

using namespace fbc;

namespace fbc {

// The tuning loop for one plan and role.  x, w, y may be NULL: then the
// timing runs on the integer gate data as well.  With four_waves only
// implicit-GEMM variants of exactly four waves are tried (the block size of
// the persistent batched kernel).  install: put the winner into the plan.
fbcorr_status tune_plan(Plan* p, const float* x, const float* w, float* y, void* workspace,
                        size_t workspace_bytes, hipStream_t s, const fbcorr_tune_opts* opts, bool four_waves,
                        bool install, fbcorr_tune_report* report, Config* chosen_out) {
    {
        const int role = opts ? opts->role : FBCORR_ROLE_FORWARD;
        FBC_RETURN_IF(role < 0 || role >= FBCORR_ROLE_COUNT, FBCORR_ERR_INVALID_ARGUMENT, "unknown role");
        const int warmup = (opts && opts->warmup > 0) ? opts->warmup : 2;
        const int reps = (opts && opts->reps > 0) ? opts->reps : 10;
        const int maxc = (opts && opts->max_candidates > 0) ? opts->max_candidates : 1 << 30;
        const bool with_direct = opts && (opts->flags & 1u);
        const bool direct_only = opts && (opts->flags & 4u);
        FBC_RETURN_IF(direct_only && (role != FBCORR_ROLE_FORWARD || p->desc.precision != FBCORR_FP32),
                      FBCORR_ERR_UNSUPPORTED, "the direct algorithm exists for the fp32 forward role only");
        fbcorr_status st;
        const bool own_data = !x && !w && !y;
        if (!own_data) {
            if ((st = check_ptr(y, "y"))) return st;
            if (role != FBCORR_ROLE_BACKWARD_X && (st = check_ptr(x, "x"))) return st;
            if (role != FBCORR_ROLE_BACKWARD_W && (st = check_ptr(w, "w"))) return st;
        }
        const TuneLayout t = tune_layout(p);
        if ((st = check_ws(workspace, workspace_bytes, t.total))) return st;
        char* base = (char*)workspace;
        const fbcorr_desc& d = p->desc;

        // Integer-valued gate data: every partial sum stays exact in fp32.
        long kdepth = role == FBCORR_ROLE_FORWARD ? (long)d.fh * d.fw * d.D
                      : role == FBCORR_ROLE_BACKWARD_X ? (long)d.fh * d.fw * d.N
                                                       : (long)d.batch * (d.H - d.fh + 1) * (d.W - d.fw + 1);
        int R = (int)std::floor(std::sqrt((double)(1 << 24) / (double)kdepth));
        R = std::max(1, std::min(8, R));
        const bool exact = (double)R * R * kdepth < (double)(1 << 24);
        float* xi = (float*)(base + t.xi);
        float* wi = (float*)(base + t.wi);
        float* gi = (float*)(base + t.gi);
        float* ref = (float*)(base + t.ref);
        float* cand = (float*)(base + t.cand);
        void* rws = base + t.role_ws;
        if ((st = fill_int(p, xi, t.nx, 11u, R, s)) || (st = fill_int(p, wi, t.nw, 23u, R, s)) ||
            (st = fill_int(p, gi, t.ny, 37u, R, s)))
            return st;
        const TuneBuffers gate{xi, wi, gi, nullptr, rws};
        const TuneBuffers timed = own_data ? TuneBuffers{xi, wi, gi, nullptr, rws} : TuneBuffers{x, w, y, nullptr, rws};
        const size_t nout = out_elems(t, role);

        fbcorr_tune_report rep;
        memset(&rep, 0, sizeof rep);

        // Default variant: the reference for the gate and the "default" time.
        Config dcfg = heuristic_default(d, role, p->dev);
        if (direct_only) dcfg = default_direct(d);
        RoleBuild drb;
        std::string err;
        FBC_RETURN_IF(!build_role(d, role, dcfg, p->dev, drb, err), FBCORR_ERR_UNSUPPORTED, "default: " + err);
        RoleExec dex;
        if ((st = make_exec(p, role, drb, dex))) return st;
        TuneBuffers g1 = gate;
        g1.out = ref;
        if ((st = run_role(p, role, dex, g1, s))) return st;
        std::vector<float> href(nout), hc(nout);
        hipError_t he = hipMemcpyDtoHAsync(href.data(), (hipDeviceptr_t)ref, nout * 4, s);
        if (he == hipSuccess) he = hipStreamSynchronize(s);
        FBC_RETURN_IF(he != hipSuccess, FBCORR_ERR_LAUNCH, std::string("gate copy: ") + hipGetErrorString(he));
        float refmax = 0.f;
        for (float v : href) refmax = std::max(refmax, std::fabs(v));
        TuneBuffers t1 = timed;
        t1.out = (role == FBCORR_ROLE_FORWARD && !own_data) ? y : cand;
        double dms = 0;
        if ((st = time_role(p, role, dex, t1, s, warmup, reps, dms))) return st;
        rep.default_ms = dms;
        snprintf(rep.default_cfg, sizeof rep.default_cfg, "%s", dcfg.str().c_str());

        // Candidates: resource pruning, then parallel compilation.
        std::vector<Config> cands = tune_candidates(d, role, with_direct, direct_only);
        std::vector<RoleBuild> builds;
        for (auto& c : cands) {
            if ((int)builds.size() >= maxc) break;
            if (four_waves && (c.algo != "igemm" || c.get("wm") * c.get("wn") * c.get("ks") != 4)) continue;
            RoleBuild rb;
            rep.n_tried++;
            if (!build_role(d, role, c, p->dev, rb, err)) { rep.n_rejected_resources++; continue; }
            // batched variants share one kernel: keep two workgroups per CU
            if (four_waves && rb.main_geom.lds > p->dev.lds_per_block / 2) { rep.n_rejected_resources++; continue; }
            if (rb.ws_bytes > workspace_bytes - t.role_ws) { rep.n_rejected_resources++; continue; }
            builds.push_back(rb);
        }
        std::vector<int> ok(builds.size(), 0);
        {
            std::atomic<size_t> next{0};
            unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
            std::vector<std::thread> pool;
            std::atomic<size_t> done{0};
            for (unsigned i = 0; i < nth; ++i)
                pool.emplace_back([&] {
                    for (size_t j; (j = next++) < builds.size();) {
                        std::shared_ptr<const std::vector<char>> code;
                        bool good = compile_cached(builds[j].main, p->dev.arch, code) == FBCORR_OK;
                        for (auto& a : builds[j].aux)
                            good = good && compile_cached(a, p->dev.arch, code) == FBCORR_OK;
                        ok[j] = good ? 1 : 0;
                        const size_t n = ++done;
                        if (n % 25 == 0 || n == builds.size())
                            tune_progress("role %d: compiled %zu of %zu candidates", role, n, builds.size());
                    }
                });
            for (auto& th : pool) th.join();
        }
        double best = dms;
        int best_i = -1;
        for (size_t j = 0; j < builds.size(); ++j) {
            if (!ok[j]) { rep.n_failed++; continue; }
            rep.n_compiled++;
            RoleExec ex;
            if (make_exec(p, role, builds[j], ex) != FBCORR_OK) { rep.n_failed++; continue; }
            if (ex.main.lds_bytes > p->dev.lds_per_block) { rep.n_rejected_resources++; continue; }
            TuneBuffers g2 = gate;
            g2.out = cand;
            if (run_role(p, role, ex, g2, s) != FBCORR_OK) { rep.n_failed++; continue; }
            he = hipMemcpyDtoHAsync(hc.data(), (hipDeviceptr_t)cand, nout * 4, s);
            if (he == hipSuccess) he = hipStreamSynchronize(s);
            FBC_RETURN_IF(he != hipSuccess, FBCORR_ERR_LAUNCH, std::string("gate copy: ") + hipGetErrorString(he));
            bool same;
            if (exact) {
                same = memcmp(hc.data(), href.data(), nout * 4) == 0;
            } else {
                same = true;
                for (size_t i = 0; i < nout && same; ++i) same = std::fabs(hc[i] - href[i]) <= 1e-5f * refmax;
            }
            if (!same) { rep.n_rejected_parity++; continue; }
            TuneBuffers t2 = timed;
            t2.out = (role == FBCORR_ROLE_FORWARD && !own_data) ? y : cand;
            double ms = 0;
            if (time_role(p, role, ex, t2, s, warmup, reps, ms) != FBCORR_OK) { rep.n_failed++; continue; }
            if (ms < best) { best = ms; best_i = (int)j; }
            if ((j + 1) % 25 == 0 || j + 1 == builds.size())
                tune_progress("role %d: timed %zu of %zu, best %.4f ms (default %.4f ms)", role, j + 1,
                              builds.size(), best, dms);
        }
        const Config& chosen = best_i >= 0 ? builds[best_i].cfg : dcfg;
        rep.best_ms = best;
        snprintf(rep.best_cfg, sizeof rep.best_cfg, "%s", chosen.str().c_str());
        if (chosen_out) *chosen_out = chosen;
        if (install) {
            st = compile_role(p, role, chosen);
            if (st != FBCORR_OK) return st;
            if (opts && (opts->flags & 2u)) {
                std::string e2;
                FBC_RETURN_IF(!tuning_db_record(p->dev.arch, role, d, chosen.str(), e2), FBCORR_ERR_INTERNAL, e2);
            }
        }
        if (report) *report = rep;
        return FBCORR_OK;
    }
}

}  // namespace fbc

extern "C" fbcorr_status fbcorr_tune(fbcorr_plan_t plan, const float* x, const float* w, float* y, void* workspace,
                                     size_t workspace_bytes, void* stream, const fbcorr_tune_opts* opts,
                                     fbcorr_tune_report* report) {
    try {
        clear_error();
        Plan* p = reinterpret_cast<Plan*>(plan);
        FBC_RETURN_IF(!p, FBCORR_ERR_INVALID_ARGUMENT, "plan is NULL");
        DeviceGuard guard(p->device);
        if (p->batched) return tune_batched(p, workspace, workspace_bytes, (hipStream_t)stream, opts, report);
        FBC_RETURN_IF(!x && !w && !y, FBCORR_ERR_INVALID_ARGUMENT, "x, w and y are NULL");
        return tune_plan(p, x, w, y, workspace, workspace_bytes, (hipStream_t)stream, opts, false, true, report,
                         nullptr);
    } catch (const std::exception& e) {
        set_error(FBCORR_ERR_INTERNAL, std::string("exception: ") + e.what());
        return FBCORR_ERR_INTERNAL;
    } catch (...) {
        set_error(FBCORR_ERR_INTERNAL, "unknown exception");
        return FBCORR_ERR_INTERNAL;
    }
}
