// Kernel configurations: defaults, validation, geometry and source generation.
//
// A configuration is the set of code-variant knobs the paper's vision
// application tunes over (Sec. 6.2: loop unrolling depth, block/grid
// dimensions, thread work size, shared-memory padding), extended by the
// matrix-core tiling.  Each knob becomes a -D constant of the kernel source
// (Sec. 5.3, keyword substitution), so every variant is compiled for exactly
// one problem (Sec. 4.2).
#include "geometry.h"

#include <algorithm>
#include <cstdio>
#include <sstream>

namespace fbc {

int Config::get(const char* k) const {
    auto it = v.find(k);
    return it == v.end() ? 0 : it->second;
}

std::string Config::str() const {
    std::string s = "algo=" + algo;
    for (auto& kv : v) s += " " + kv.first + "=" + std::to_string(kv.second);
    return s;
}

bool parse_config(const std::string& text, Config& base, std::string& err) {
    std::istringstream is(text);
    std::string tok;
    Config c = base;
    while (is >> tok) {
        auto eq = tok.find('=');
        if (eq == std::string::npos || eq == 0) { err = "bad token '" + tok + "'"; return false; }
        std::string k = tok.substr(0, eq), val = tok.substr(eq + 1);
        if (k == "algo") {
            if (val != "igemm" && val != "direct" && val != "dw" && val != "nn" && val != "rgemm") {
                err = "unknown algo '" + val + "'";
                return false;
            }
            if (val != c.algo) {
                c.algo = val;
                c.v.clear();          // keys of another algorithm do not carry over
            }
            continue;
        }
        char* end = nullptr;
        long x = strtol(val.c_str(), &end, 10);
        if (!end || *end || val.empty()) { err = "bad value in '" + tok + "'"; return false; }
        c.v[k] = (int)x;
    }
    base = c;
    return true;
}

static int round_up(int a, int m) { return (a + m - 1) / m * m; }
static int cdiv(int a, int b) { return (a + b - 1) / b; }
static int cdivl(long a, long b) { return (int)((a + b - 1) / b); }

// ------------------------------------------------------------ defaults

static int pick_kc(int cin, bool lowp) {
    if (lowp) {
        if (cin % 16 == 0) return 16;
        if (cin % 8 == 0) return 8;
        return cin <= 16 ? cin : 8;
    }
    if (cin <= 16) return cin;
    if (cin % 16 == 0) return 16;
    if (cin % 8 == 0) return 8;
    return 8;
}

static int pick_shift(int cout) {
    if (cout >= 32) return 1;
    if (cout >= 16) return 2;
    if (cout >= 8) return 4;
    return 8;
}

Config default_igemm(int cin, int cout, bool lowp) {
    Config c;
    c.algo = "igemm";
    const int s = pick_shift(cout);
    const int cols = cout * s;
    const int nt = cols >= 64 ? 2 : 1;
    const int kc = pick_kc(cin, lowp);
    const int nchunk = (cin + kc - 1) / kc;
    c.v = {{"mf", 32}, {"kc", kc}, {"s", s}, {"mr", s >= 2 ? 4 : 1}, {"mt", 1}, {"nt", nt}, {"wm", s >= 2 ? 1 : 4},
           {"wn", 1}, {"ks", s >= 2 ? std::min(4, nchunk) : 1}, {"xpad", lowp ? 8 : 4},
           {"wpad", lowp ? 8 : 4}, {"ustage", 1}, {"xcd", 1}};
    return c;
}

// Filter fragments streamed into registers (rgemm.hip): 2 x 2 waves of
// 4 x 2 tiles (256 pixels x 128 filters per workgroup), whole channel
// chunks of up to 16 (fp32) or 32 (16-bit) channels, three steps in flight;
// for at most 16 output channels four waves of eight 16x16 tiles.
Config default_rgemm(int cin, int cout, bool lowp) {
    Config c;
    c.algo = "rgemm";
    const int pe = lowp ? 8 : 4;
    int kc = pe;
    for (int k : {4 * pe, 2 * pe})
        if (cin % k == 0 || cin > k) { kc = k; break; }
    if (cin % pe) kc = pe;
    if (cout <= 16) {
        // 16x16 tiles: a 32-wide tile would leave half its columns empty
        c.v = {{"mf", 16}, {"kc", kc}, {"mr", 1}, {"mt", 8}, {"nt", 1}, {"wm", 4}, {"wn", 1}, {"pf", 3},
               {"xpadc", 0}, {"wpe", 2}, {"xcd", 1}};
        return c;
    }
    const int nt = cout > 32 ? 2 : 1;
    const int wn = cout > 64 ? 2 : 1;
    c.v = {{"mf", 32}, {"kc", kc}, {"mr", 2}, {"mt", 4}, {"nt", nt}, {"wm", 2}, {"wn", wn}, {"pf", 3},
           {"xpadc", 0}, {"wpe", 2}, {"xcd", 1}};
    return c;
}

// Variants of a default that use fewer resources, tried in order until one
// fits the device.
static std::vector<Config> shrink_sequence(const Config& base) {
    std::vector<Config> out{base};
    Config c = base;
    for (int step = 0; step < 16; ++step) {
        if (c.algo == "igemm") {
            if (c.v["ks"] > 1) c.v["ks"] /= 2;
            else if (c.v["kc"] > 4 && c.v["kc"] % 2 == 0) c.v["kc"] /= 2;
            else if (c.v["nt"] > 1) c.v["nt"] /= 2;
            else if (c.v["wm"] > 1) c.v["wm"] /= 2;
            else if (c.v["mr"] > 1) c.v["mr"] /= 2;
            else if (c.v["kc"] > 1) c.v["kc"] = (c.v["kc"] + 1) / 2;
            else break;
        } else if (c.algo == "direct") {
            if (c.v["th"] > 1) c.v["th"] /= 2;
            else break;
        } else {
            if (c.v["pf"]) c.v["pf"] = 0;
            else if (c.v["rh"] > 1) c.v["rh"] /= 2;
            else if (c.v["rw"] > 8) c.v["rw"] /= 2;
            else if (c.v["nw"] < 16) c.v["nw"] *= 2;
            else break;
        }
        out.push_back(c);
    }
    return out;
}

Config default_direct(const fbcorr_desc& d) {
    Config c;
    c.algo = "direct";
    int q = 16;
    while (q > 4 && q > round_up(d.N, 4)) q /= 2;
    int nb = std::min(64, round_up(d.N, q));
    c.v = {{"th", 8}, {"tw", 32}, {"p", 4}, {"q", q}, {"nb", nb}, {"ds", 1}, {"layout", 1},
           {"xpad", 1}, {"wpad", 4}, {"ud", 1}, {"xcd", 1}};
    // keep the workgroup within 1024 threads
    while ((c.v["th"] * (c.v["tw"] / c.v["p"]) * (nb / q)) > 1024 && c.v["th"] > 1) c.v["th"] /= 2;
    return c;
}

static int dw_tiles(const fbcorr_desc& d) {
    return cdiv(d.N, 32) * cdiv(d.fh * d.fw * d.D, 32);
}

Config default_dw(const fbcorr_desc& d, int cus) {
    Config c;
    c.algo = "dw";
    const int tiles = dw_tiles(d);
    const int tpb = cdiv(tiles, 2);
    const int ho = d.H - d.fh + 1, wo = d.W - d.fw + 1;
    const long nchunks = (long)d.batch * cdiv(ho, 2) * cdiv(wo, 32);
    const int np = (int)std::max<long>(1, std::min<long>(nchunks, std::max(1, cus) / 2));
    c.v = {{"rh", 2}, {"rw", 32}, {"nw", 8}, {"tpb", tpb}, {"np", np}, {"gpad", 0}, {"xpad", 0}, {"pf", 1},
           {"bal", 0}, {"unr", 4}};
    return c;
}

static Config heuristic_config(const fbcorr_desc& d, int role, int cus) {
    const bool lowp = d.precision != FBCORR_FP32;
    switch (role) {
    case FBCORR_ROLE_FORWARD:
        if (d.algo == FBCORR_ALGO_DIRECT && !lowp) return default_direct(d);
        return default_igemm(d.D, d.N, lowp);
    case FBCORR_ROLE_BACKWARD_X:
        return default_igemm(d.N, d.D, false);
    default:
        return default_dw(d, cus);
    }
}

// ---------------------------------------------------------- geometry

static void opt(std::vector<std::string>& o, const char* k, long v) {
    // Every constant is passed as FB_<name>: hiprtc's implicit runtime header
    // sees -D macros too, and short names such as N would collide with it.
    o.push_back(std::string("-DFB_") + k + "=" + std::to_string(v));
}

// igemm: valid correlation over a virtually padded input (see igemm.hip).
static bool geom_igemm(const char* kname, const Config& c, int batch, int hi, int wi, int cin, int cout,
                       int fh, int fw, int padh, int padw, int dt, const DeviceInfo& di, LaunchGeom& g,
                       KernelSource& ks, std::string& err) {
    const int kc = c.get("kc"), s = c.get("s"), mt = c.get("mt"), nt = c.get("nt");
    const int wm = c.get("wm"), wn = c.get("wn"), xpad = c.get("xpad"), wpad = c.get("wpad");
    const int ustage = std::min(c.get("ustage"), fh), xcd = c.get("xcd");
    const int mr = c.get("mr"), ksp = c.get("ks");
    const int mf = c.v.count("mf") ? c.get("mf") : 32;
    if (kc < 1 || s < 1 || mt < 1 || nt < 1 || wm < 1 || wn < 1 || xpad < 0 || wpad < 0 || ustage < 1 ||
        mr < 1 || ksp < 1) {
        err = "igemm: every knob must be positive"; return false;
    }
    if (mf != 32 && mf != 16) { err = "igemm: mf must be 32 or 16"; return false; }
    if (s != 1 && s != 2 && s != 4 && s != 8) { err = "igemm: s must be 1, 2, 4 or 8"; return false; }
    if (mf % mr) { err = "igemm: mr must divide mf"; return false; }
    const int threads = wm * wn * ksp * 64;
    if (threads > std::min(1024, di.max_threads)) { err = "igemm: too many threads"; return false; }
    const int nreg = mf * mf / 64;
    // accumulators live in the AGPR half of the register file: at most 256
    if (mt * nt * nreg > 256) { err = "igemm: more than 256 accumulator registers per lane"; return false; }
    const int ncol = wn * nt * mf;
    if (ncol % s) { err = "igemm: columns must split evenly into shifts"; return false; }
    const int cb = ncol / s;
    const int mc = mf / mr;
    const int ho = hi + 2 * padh - fh + 1, wo = wi + 2 * padw - fw + 1;
    const int esz = dt == 0 ? 4 : 2;
    const int runit = (64 / mf) * (dt == 0 ? 4 : 8);
    const int krraw = (fw + s - 1) * kc;
    const int kr = round_up(krraw, runit);
    const int rowe = (mc - 1) * s * kc + kr;
    const int rows = rowe + xpad;
    const int wrs = (s - 1) * kc + kr + wpad;
    int av, bv;
    if (dt == 0) {
        av = ((s * kc) % 4 == 0) ? 4 : (((s * kc) % 2 == 0) ? 2 : 1);
        bv = (s == 1 || kc % 4 == 0) ? 4 : ((kc % 2 == 0) ? 2 : 1);
    } else {
        av = ((s * kc) % 8 == 0) ? 8 : (((s * kc) % 4 == 0) ? 4 : (((s * kc) % 2 == 0) ? 2 : 1));
        bv = (s == 1 || kc % 8 == 0) ? 8 : ((kc % 4 == 0) ? 4 : ((kc % 2 == 0) ? 2 : 1));
    }
    if (rows % av) { err = "igemm: xpad breaks A-read alignment"; return false; }
    if (wrs % bv) { err = "igemm: wpad breaks B-read alignment"; return false; }
    const int th = wm * mt * mr;
    const int tr = th + fh - 1;
    const long tile = round_up(tr * rows, 8);
    const long wsl = (long)ustage * cb * wrs;
    const long group = (tile + 2 * wsl + 7) / 8 * 8;
    const long red = (long)(ksp - 1) * wm * wn * mt * nt * nreg * 64 * 4;
    const long lds = std::max(ksp * group * esz, red);
    if (lds > di.lds_per_block) { err = "igemm: LDS " + std::to_string(lds) + " B exceeds the device limit"; return false; }
    const long grid = (long)cdiv(wo, s * mc) * cdiv(ho, th) * cdiv(cout, cb) * batch;
    if (grid <= 0 || grid > 0x7fffffffL) { err = "igemm: grid out of range"; return false; }
    g.grid_x = (int)grid;
    g.grid_y = 1;
    g.threads = threads;
    g.lds = (int)lds;
    ks.name = kname;
    ks.file = "igemm";
    ks.source = template_source("igemm");
    ks.options.clear();
    ks.options.push_back(std::string("-DFB_KNAME=") + kname);
    opt(ks.options, "BATCH", batch); opt(ks.options, "FH", fh); opt(ks.options, "FW", fw);
    opt(ks.options, "CIN", cin); opt(ks.options, "COUT", cout);
    opt(ks.options, "HI", hi); opt(ks.options, "WI", wi); opt(ks.options, "HO", ho); opt(ks.options, "WO", wo);
    opt(ks.options, "PADH", padh); opt(ks.options, "PADW", padw);
    opt(ks.options, "MF", mf); opt(ks.options, "KC", kc); opt(ks.options, "S", s); opt(ks.options, "MR", mr);
    opt(ks.options, "MT", mt); opt(ks.options, "NT", nt);
    opt(ks.options, "WM", wm); opt(ks.options, "WN", wn); opt(ks.options, "KS", ksp); opt(ks.options, "DT", dt);
    opt(ks.options, "XPAD", xpad); opt(ks.options, "WPAD", wpad);
    opt(ks.options, "USTAGE", ustage); opt(ks.options, "XCDMAP", xcd ? 1 : 0);
    if (c.get("uunr")) opt(ks.options, "UUNR", 1);
    if (c.get("swz")) {
        if (dt == 0 || kc != 16) { err = "igemm: swz needs 16-bit operands and kc=16"; return false; }
        opt(ks.options, "SWZ", 1);
    }
    return true;
}

// rgemm: implicit GEMM with the filter fragments streamed into registers
// (see rgemm.hip).  Returns the packed bank's size in bytes in bank_bytes.
static bool geom_rgemm(const char* kname, const Config& c, int batch, int hi, int wi, int cin, int cout,
                       int fh, int fw, int padh, int padw, int dt, const DeviceInfo& di, LaunchGeom& g,
                       KernelSource& ks, KernelSource& pack, LaunchGeom& pack_geom, size_t& bank_bytes,
                       std::string& err) {
    const int kc = c.get("kc"), mr = c.get("mr"), mt = c.get("mt"), nt = c.get("nt");
    const int wm = c.get("wm"), wn = c.get("wn"), pf = c.get("pf"), xpadc = c.get("xpadc");
    const int wpe = c.v.count("wpe") ? c.get("wpe") : 2, xcd = c.get("xcd"), unr = c.get("unr");
    const int mf = c.v.count("mf") ? c.get("mf") : 32;
    const int sh = c.v.count("s") ? c.get("s") : 1;
    if (kc < 1 || mr < 1 || mt < 1 || nt < 1 || wm < 1 || wn < 1 || pf < 1 || xpadc < 0) {
        err = "rgemm: every knob must be positive"; return false;
    }
    if (sh != 1 && sh != 2 && sh != 4 && sh != 8) { err = "rgemm: s must be 1, 2, 4 or 8"; return false; }
    if ((wn * nt * mf) % sh) { err = "rgemm: the columns must split evenly into shifts"; return false; }
    if (mf != 32 && mf != 16) { err = "rgemm: mf must be 32 or 16"; return false; }
    if (pf > 8) { err = "rgemm: pf is at most 8"; return false; }
    if (wpe < 1 || wpe > 8) { err = "rgemm: wpe must be 1..8"; return false; }
    if (mf % mr) { err = "rgemm: mr must divide mf"; return false; }
    const int pe = dt == 0 ? 4 : 8, e = (64 / mf) * pe;
    const int npl = kc / pe;
    if (kc % pe || (npl & (npl - 1))) {
        err = "rgemm: kc must be " + std::to_string(pe) + " times a power of two"; return false;
    }
    if (kc > 64) { err = "rgemm: kc is at most 64"; return false; }
    if (cin % pe && kc != pe) { err = "rgemm: channels not a multiple of the cell width need kc=" + std::to_string(pe); return false; }
    const int threads = wm * wn * 64;
    if (threads > std::min(1024, di.max_threads)) { err = "rgemm: too many threads"; return false; }
    // accumulators, the fragment ring and two sets of A fragments must fit
    // the per-lane register budget of wpe waves per SIMD (512 / wpe)
    const int regs = mt * nt * (mf * mf / 64) + pf * nt * 4 + 2 * mt * 4 + 24;
    if (regs > 512 / wpe) {
        err = "rgemm: needs about " + std::to_string(regs) + " registers per lane, more than wpe allows"; return false;
    }
    const int nstep = ((fw + sh - 1) * kc + e - 1) / e;
    const int ntaps = nstep * e / kc;
    const int nchunk = (cin + kc - 1) / kc;
    const int ksteps2 = fh * nstep + pf;
    const int mc = mf / mr;
    const int ncolw = wn * nt * mf, cb = ncolw / sh;
    const int th = wm * mt * mr, two = sh * mc;
    const int tr = th + fh - 1, tc = sh * (mc - 1) + ntaps, tcp = tc + xpadc;
    const int ste = c.get("ste");
    if (ste && (sh != 1 || cout % 4)) { err = "rgemm: ste needs s=1 and a multiple of 4 output channels"; return false; }
    long lds = (long)npl * tr * tcp * 16;
    if (ste) lds = std::max(lds, (long)wm * wn * mf * (nt * mf + 8) * 4);
    if (lds > di.lds_per_block) { err = "rgemm: LDS " + std::to_string(lds) + " B exceeds the device limit"; return false; }
    const int ho = hi + 2 * padh - fh + 1, wo = wi + 2 * padw - fw + 1;
    const long grid = (long)cdiv(wo, two) * cdiv(ho, th) * cdiv(cout, cb) * batch;
    if (grid <= 0 || grid > 0x7fffffffL) { err = "rgemm: grid out of range"; return false; }
    // the packed bank covers whole column blocks of the correlation kernel
    // (NCOLW columns of shifted filters each): one kilobyte per column tile,
    // chunk and step
    const int ncols = cdiv(cout, cb) * ncolw;
    bank_bytes = (size_t)(ncols / mf) * nchunk * ksteps2 * 1024;
    g.grid_x = (int)grid;
    g.grid_y = 1;
    g.threads = threads;
    g.lds = (int)lds;
    ks.name = kname;
    ks.file = "rgemm";
    ks.source = template_source("rgemm");
    ks.options.clear();
    ks.options.push_back(std::string("-DFB_KNAME=") + kname);
    opt(ks.options, "BATCH", batch); opt(ks.options, "FH", fh); opt(ks.options, "FW", fw);
    opt(ks.options, "CIN", cin); opt(ks.options, "COUT", cout);
    opt(ks.options, "HI", hi); opt(ks.options, "WI", wi); opt(ks.options, "HO", ho); opt(ks.options, "WO", wo);
    opt(ks.options, "PADH", padh); opt(ks.options, "PADW", padw); opt(ks.options, "DT", dt);
    opt(ks.options, "MF", mf); opt(ks.options, "KC", kc); opt(ks.options, "MR", mr);
    opt(ks.options, "MT", mt); opt(ks.options, "NT", nt); opt(ks.options, "S", sh);
    opt(ks.options, "WM", wm); opt(ks.options, "WN", wn); opt(ks.options, "PF", pf);
    opt(ks.options, "XPADC", xpadc); opt(ks.options, "WPE", wpe); opt(ks.options, "XCDMAP", xcd ? 1 : 0);
    if (unr) opt(ks.options, "UNR", 1);
    if (c.get("nts")) opt(ks.options, "NTS", 1);
    if (ste) opt(ks.options, "STE", 1);
    pack = KernelSource();
    pack.name = "fbcorr_pack_frag";
    pack.file = "rgemm";
    pack.source = template_source("rgemm");
    pack.options.push_back("-DFB_PACK_FRAG");
    opt(pack.options, "FH", fh); opt(pack.options, "FW", fw); opt(pack.options, "CIN", cin);
    opt(pack.options, "COUT", cout); opt(pack.options, "DT", dt); opt(pack.options, "MF", mf);
    opt(pack.options, "KC", kc); opt(pack.options, "PF", pf); opt(pack.options, "S", sh);
    opt(pack.options, "NCOLW", ncolw);
    pack_geom = LaunchGeom{ncols, 1, 256, 0};
    return true;
}

static bool geom_direct(const Config& c, const fbcorr_desc& d, const DeviceInfo& di, LaunchGeom& g,
                        KernelSource& ks, std::string& err) {
    const int th = c.get("th"), tw = c.get("tw"), p = c.get("p"), q = c.get("q"), nb = c.get("nb");
    const int ds = c.get("ds"), layout = c.get("layout"), xpad = c.get("xpad"), wpad = c.get("wpad");
    const int ud = c.get("ud"), xcd = c.get("xcd"), fsrc = c.get("fsrc"), sb = c.get("sb");
    if (th < 1 || tw < 1 || p < 1 || q < 1 || nb < 1 || ds < 1 || xpad < 0 || wpad < 0 || ud < 1) {
        err = "direct: every knob must be positive"; return false;
    }
    if (fsrc != 0 && fsrc != 1) { err = "direct: fsrc is 0 or 1"; return false; }
    if (sb != 0 && sb != 1) { err = "direct: sb is 0 or 1"; return false; }
    if (fsrc && (ds != 1 || (th * (tw / p)) % 64 != 0)) {
        err = "direct: scalar weights (fsrc=1) need ds=1 and th*tw/p a multiple of 64"; return false;
    }
    if (tw % p) { err = "direct: p must divide tw"; return false; }
    if (nb % q) { err = "direct: q must divide nb"; return false; }
    if (q % 4) { err = "direct: q must be a multiple of 4"; return false; }
    if ((ds & (ds - 1)) || ds > 64 || d.D % ds) { err = "direct: ds must be a power of two dividing D"; return false; }
    if ((nb + wpad) % 4) { err = "direct: nb + wpad must be a multiple of 4"; return false; }
    if (layout != 0 && layout != 1) { err = "direct: layout is 0 or 1"; return false; }
    const int threads = th * (tw / p) * (nb / q) * ds;
    if (threads > std::min(1024, di.max_threads) || threads < 64 || threads % 64) {
        err = "direct: workgroup must be 64..1024 threads in whole waves"; return false;
    }
    const int ho = d.H - d.fh + 1, wo = d.W - d.fw + 1;
    const int trr = th + d.fh - 1, tcc = tw + d.fw - 1;
    const long tile = layout == 0 ? (long)trr * (tcc * d.D + xpad) : (long)d.D * trr * (tcc + xpad);
    const long lds = (tile + (fsrc ? 0L : (long)d.fw * d.D * (nb + wpad))) * 4;
    if (lds > di.lds_per_block) { err = "direct: LDS " + std::to_string(lds) + " B exceeds the device limit"; return false; }
    const long grid = (long)cdiv(wo, tw) * cdiv(ho, th) * cdiv(d.N, nb) * d.batch;
    if (grid <= 0 || grid > 0x7fffffffL) { err = "direct: grid out of range"; return false; }
    g.grid_x = (int)grid;
    g.grid_y = 1;
    g.threads = threads;
    g.lds = (int)lds;
    ks.name = "fbcorr_direct";
    ks.file = "direct";
    ks.source = template_source("direct");
    ks.options.clear();
    opt(ks.options, "BATCH", d.batch); opt(ks.options, "FH", d.fh); opt(ks.options, "FW", d.fw);
    opt(ks.options, "D", d.D); opt(ks.options, "N", d.N); opt(ks.options, "H", d.H); opt(ks.options, "W", d.W);
    opt(ks.options, "HO", ho); opt(ks.options, "WO", wo);
    opt(ks.options, "TH", th); opt(ks.options, "TW", tw); opt(ks.options, "P", p); opt(ks.options, "Q", q);
    opt(ks.options, "NB", nb); opt(ks.options, "DS", ds); opt(ks.options, "LAYOUT", layout);
    opt(ks.options, "XPAD", xpad); opt(ks.options, "WPAD", wpad); opt(ks.options, "UD", ud);
    opt(ks.options, "XCDMAP", xcd ? 1 : 0);
    if (sb) opt(ks.options, "SB", 1);
    if (fsrc) {
        opt(ks.options, "FSRC", 1);
        opt(ks.options, "NPAD", cdiv(d.N, nb) * nb);
    }
    return true;
}

static bool geom_dw(const Config& c, const fbcorr_desc& d, const DeviceInfo& di, LaunchGeom& g,
                    KernelSource& ks, int& np_out, std::string& err) {
    const int rh = c.get("rh"), rw = c.get("rw"), nw = c.get("nw"), tpb = c.get("tpb");
    const int gpad = c.get("gpad"), xpad = c.get("xpad"), pf = c.get("pf"), bal = c.get("bal");
    const int unr = c.v.count("unr") ? c.get("unr") : 4;
    int np = c.get("np");
    if (rh < 1 || rw < 1 || nw < 1 || tpb < 1 || gpad < 0 || xpad < 0 || np < 1) {
        err = "dw: every knob must be positive"; return false;
    }
    if ((rh * rw) % 2) { err = "dw: rh*rw must be even"; return false; }
    const int tiles = dw_tiles(d);
    const int tpb_eff = std::min(tpb, tiles);
    if (bal < 0 || bal > 1) { err = "dw: bal must be 0 or 1"; return false; }
    if (unr < 0 || unr > 64) { err = "dw: unr must be 0 (complete) or 1..64"; return false; }
    // accumulator slots per wave: round-robin tiles, or full rounds + two
    // slots for the left-over tiles split by pixels
    const int slots = bal ? tpb_eff / nw + 2 : cdiv(tpb_eff, nw);
    if (slots > 8) { err = "dw: more than 8 accumulator tiles per wave"; return false; }
    const int threads = nw * 64;
    if (threads > std::min(1024, di.max_threads)) { err = "dw: too many threads"; return false; }
    const int ho = d.H - d.fh + 1, wo = d.W - d.fw + 1;
    const int npad = cdiv(d.N, 32) * 32;
    const int pc = rh * rw;
    if (pf < 0 || pf > 2) { err = "dw: pf must be 0, 1 or 2"; return false; }
    const long stage = (pf == 2 ? 2 : 1) *
                       ((long)pc * (npad + gpad) + (long)(rh + d.fh - 1) * ((rw + d.fw - 1) * d.D + xpad)) * 4;
    // with bal the staging memory is reused for the left-over slots (two
    // 32x32 fp32 tiles per wave)
    const long lds = std::max(stage, bal ? (long)nw * 2 * 1024 * 4 : 0L);
    if (lds > di.lds_per_block) { err = "dw: LDS " + std::to_string(lds) + " B exceeds the device limit"; return false; }
    const long prefetch_regs = pf ? (cdivl((long)pc * npad, threads) + cdivl((long)(rh + d.fh - 1) * (rw + d.fw - 1) * d.D, threads)) : 0;
    if (prefetch_regs > 96) { err = "dw: prefetch needs too many registers"; return false; }
    const long nchunks = (long)d.batch * cdiv(ho, rh) * cdiv(wo, rw);
    if (np > nchunks) np = (int)nchunks;
    if (np > 65535) { err = "dw: partial count out of range"; return false; }
    g.grid_x = np;
    g.grid_y = cdiv(tiles, tpb_eff);
    g.threads = threads;
    g.lds = (int)lds;
    np_out = np;
    ks.name = "fbcorr_dw_partial";
    ks.file = "dw";
    ks.source = template_source("dw");
    ks.options.clear();
    opt(ks.options, "BATCH", d.batch); opt(ks.options, "FH", d.fh); opt(ks.options, "FW", d.fw);
    opt(ks.options, "D", d.D); opt(ks.options, "N", d.N); opt(ks.options, "H", d.H); opt(ks.options, "W", d.W);
    opt(ks.options, "HO", ho); opt(ks.options, "WO", wo);
    opt(ks.options, "RH", rh); opt(ks.options, "RW", rw); opt(ks.options, "NW", nw); opt(ks.options, "TPB", tpb_eff);
    opt(ks.options, "NP", np); opt(ks.options, "GPAD", gpad); opt(ks.options, "XPAD", xpad);
    opt(ks.options, "PF", pf);
    if (bal) opt(ks.options, "BAL", bal);
    if (c.get("skipe")) opt(ks.options, "SKIPE", 1);
    opt(ks.options, "UNR", unr);
    return true;
}

static KernelSource util_source(const char* name, const char* define) {
    KernelSource ks;
    ks.name = name;
    ks.file = "util";
    ks.source = template_source("util");
    ks.options.push_back(std::string("-DFB_") + define);
    return ks;
}

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// fp16 forward: the per-tensor input scale (reading c-10).  256 partial
// maxima of |x| from fbcorr_absmax, written after `ucount` unscale floats,
// are combined by the correlation kernel (option FB_XMOFF).  Returns the
// bytes of the unscale + partials region.
static const int kInputMaxParts = 256;
static size_t add_input_scale(const fbcorr_desc& d, int dt, size_t ucount, RoleBuild& rb) {
    if (dt != 2) return align256(ucount * 4);
    const size_t xmoff = (ucount + 63) / 64 * 64;
    rb.main.options.push_back("-DFB_XMOFF=" + std::to_string(xmoff));
    KernelSource ks = util_source("fbcorr_absmax", "ABSMAX");
    rb.aux.push_back(ks);
    rb.aux_geom.push_back(LaunchGeom{kInputMaxParts, 1, 256, 0});
    rb.ws_xmax = rb.ws_unscale + xmoff * 4;
    rb.nxp = kInputMaxParts;
    (void)d;
    return align256((xmoff + kInputMaxParts) * 4);
}

static bool build_role_impl(const fbcorr_desc& d, int role, const Config& c, const DeviceInfo& di,
                            RoleBuild& rb, std::string& err);

bool build_role(const fbcorr_desc& d, int role, const Config& c, const DeviceInfo& di,
                RoleBuild& rb, std::string& err) {
    if (!build_role_impl(d, role, c, di, rb, err)) return false;
    // Test hook: "inject_error=1" makes the generated source fail to compile.
    if (c.get("inject_error")) rb.main.options.push_back("-DFB_INJECT_ERROR");
    return true;
}

static bool known_keys(const Config& c, std::string& err) {
    static const std::map<std::string, std::vector<std::string>> keys = {
        {"igemm", {"mf", "kc", "s", "mr", "mt", "nt", "wm", "wn", "ks", "xpad", "wpad", "ustage", "xcd", "flip",
                   "uunr", "swz"}},
        {"direct", {"th", "tw", "p", "q", "nb", "ds", "layout", "xpad", "wpad", "ud", "xcd", "fsrc", "sb"}},
        {"dw", {"rh", "rw", "nw", "tpb", "np", "gpad", "xpad", "pf", "bal", "unr", "skipe"}},
        {"rgemm", {"mf", "kc", "s", "mr", "mt", "nt", "wm", "wn", "pf", "xpadc", "wpe", "unr", "xcd", "flip", "nts",
                   "ste"}},
    };
    auto it = keys.find(c.algo);
    if (it == keys.end()) { err = "unknown algorithm '" + c.algo + "'"; return false; }
    for (auto& kv : c.v) {
        if (kv.first == "inject_error") continue;
        if (std::find(it->second.begin(), it->second.end(), kv.first) == it->second.end()) {
            err = "unknown key '" + kv.first + "' for algo=" + c.algo;
            return false;
        }
    }
    return true;
}

static bool build_role_impl(const fbcorr_desc& d, int role, const Config& c, const DeviceInfo& di,
                            RoleBuild& rb, std::string& err) {
    rb = RoleBuild();
    rb.cfg = c;
    if (!known_keys(c, err)) return false;
    const int ho = d.H - d.fh + 1, wo = d.W - d.fw + 1;
    const long K = (long)d.fh * d.fw * d.D;
    if (role == FBCORR_ROLE_FORWARD) {
        const int dt = d.precision == FBCORR_BF16 ? 1 : (d.precision == FBCORR_FP16 ? 2 : 0);
        if (c.algo == "direct") {
            if (dt != 0) { err = "the direct kernel is fp32 only"; return false; }
            if (!geom_direct(c, d, di, rb.main_geom, rb.main, err)) return false;
            if (c.get("fsrc")) {
                // tap-major copy of the filters for the scalar loads
                const int npad = cdiv(d.N, c.get("nb")) * c.get("nb");
                KernelSource ks = util_source("fbcorr_transpose_filters", "TRANSPOSE_FILTERS");
                opt(ks.options, "N", d.N); opt(ks.options, "FH", d.fh); opt(ks.options, "FW", d.fw);
                opt(ks.options, "D", d.D); opt(ks.options, "NPAD", npad);
                rb.aux.push_back(ks);
                rb.aux_geom.push_back(LaunchGeom{cdivl(K * npad, 256), 1, 256, 0});
                rb.ws_lowp_w = 0;
                rb.ws_bytes = align256((size_t)K * npad * 4);
            }
        } else if (c.algo == "igemm") {
            if (c.get("flip")) { err = "flip applies to the input-gradient role only"; return false; }
            if (!geom_igemm("fbcorr_fwd_igemm", c, d.batch, d.H, d.W, d.D, d.N, d.fh, d.fw, 0, 0, dt, di,
                            rb.main_geom, rb.main, err))
                return false;
        } else if (c.algo == "rgemm") {
            if (c.get("flip")) { err = "flip applies to the input-gradient role only"; return false; }
            // the filters are always repacked (fragment order; scaled and
            // rounded for 16-bit operands)
            KernelSource pk;
            LaunchGeom pg;
            size_t bank = 0;
            if (!geom_rgemm("fbcorr_fwd_rgemm", c, d.batch, d.H, d.W, d.D, d.N, d.fh, d.fw, 0, 0, dt, di,
                            rb.main_geom, rb.main, pk, pg, bank, err))
                return false;
            rb.aux.push_back(pk);
            rb.aux_geom.push_back(pg);
            rb.ws_lowp_w = 0;
            rb.ws_unscale = align256(bank);
            rb.ws_bytes = rb.ws_unscale + add_input_scale(d, dt, (size_t)pg.grid_x, rb);
            return true;
        } else {
            err = "forward role needs algo=igemm, algo=rgemm or algo=direct";
            return false;
        }
        if (dt != 0) {
            KernelSource ks = util_source("fbcorr_pack_lowp", "PACK_LOWP");
            opt(ks.options, "N", d.N); opt(ks.options, "FH", d.fh); opt(ks.options, "FW", d.fw);
            opt(ks.options, "D", d.D); opt(ks.options, "LOWP", dt);
            rb.aux.push_back(ks);
            rb.aux_geom.push_back(LaunchGeom{d.N, 1, 256, 0});
            rb.ws_lowp_w = 0;
            rb.ws_unscale = align256((size_t)d.N * K * 2);
            rb.ws_bytes = rb.ws_unscale + add_input_scale(d, dt, (size_t)d.N, rb);
        }
        return true;
    }
    if (role == FBCORR_ROLE_BACKWARD_X && c.algo == "rgemm") {
        // dx = valid correlation of dy (padded by fh-1, fw-1) with the
        // flipped, transposed filters, which the pack reads straight from
        // the forward bank (the flip is part of the repacking)
        KernelSource pk;
        LaunchGeom pg;
        size_t bank = 0;
        if (!geom_rgemm("fbcorr_dx_rgemm", c, d.batch, ho, wo, d.N, d.D, d.fh, d.fw, d.fh - 1, d.fw - 1, 0, di,
                        rb.main_geom, rb.main, pk, pg, bank, err))
            return false;
        pk.options.push_back("-DFB_FLIP");
        rb.aux.push_back(pk);
        rb.aux_geom.push_back(pg);
        rb.ws_bytes = align256(bank);
        return true;
    }
    if (role == FBCORR_ROLE_BACKWARD_X) {
        if (c.algo != "igemm") { err = "input-gradient role needs algo=igemm or algo=rgemm"; return false; }
        // dx = valid correlation of dy (padded by fh-1, fw-1) with flipped,
        // transposed filters: CIN = N, COUT = D, input extent Ho x Wo.
        if (!geom_igemm("fbcorr_dx_igemm", c, d.batch, ho, wo, d.N, d.D, d.fh, d.fw, d.fh - 1, d.fw - 1, 0, di,
                        rb.main_geom, rb.main, err))
            return false;
        if (c.get("flip")) {
            // the flip happens while staging: the kernel reads the forward bank
            rb.main.options.push_back("-DFB_FLIPW");
            return true;
        }
        KernelSource ks = util_source("fbcorr_flip_filters", "FLIP_FILTERS");
        opt(ks.options, "N", d.N); opt(ks.options, "FH", d.fh); opt(ks.options, "FW", d.fw); opt(ks.options, "D", d.D);
        rb.aux.push_back(ks);
        rb.aux_geom.push_back(LaunchGeom{cdivl((long)d.N * K, 256), 1, 256, 0});
        rb.ws_bytes = align256((size_t)d.N * K * 4);
        return true;
    }
    if (role == FBCORR_ROLE_BACKWARD_W) {
        if (c.algo != "dw") { err = "filter-gradient role needs algo=dw"; return false; }
        int np = 0;
        if (!geom_dw(c, d, di, rb.main_geom, rb.main, np, err)) return false;
        rb.np = np;
        const long L = (long)d.N * K;
        // 16 slices x 16 lanes per workgroup: several hundred workgroups for
        // a few hundred kilobytes of output, each thread with NP/16 loads
        const int rs = 16, lanes = 16;
        const int sv = (L % 4 == 0) ? 4 : 1;    // outputs per thread (16-byte loads when possible)
        KernelSource ks = util_source("fbcorr_sum_partials", "SUM_PARTIALS");
        opt(ks.options, "L", L); opt(ks.options, "NP", np); opt(ks.options, "RS", rs);
        opt(ks.options, "LANES", lanes);
        rb.aux.push_back(ks);
        rb.aux_geom.push_back(LaunchGeom{cdivl(L / sv, lanes), 1, lanes * rs, 0});
        rb.ws_bytes = align256((size_t)np * L * 4);
        return true;
    }
    err = "unknown role";
    return false;
}

Config default_config(const fbcorr_desc& d, int role, const DeviceInfo& di) {
    std::string text;
    if (tuning_db_lookup(di.arch, role, d, text)) {
        Config c = heuristic_config(d, role, di.cus);
        std::string err;
        Config probe;
        probe.algo = c.algo;
        if (parse_config(text, probe, err)) {
            // start from the chosen algorithm's heuristic and apply the entry
            const int cin = role == FBCORR_ROLE_BACKWARD_X ? d.N : d.D;
            const int cout = role == FBCORR_ROLE_BACKWARD_X ? d.D : d.N;
            const bool lp = d.precision != FBCORR_FP32 && role == FBCORR_ROLE_FORWARD;
            Config base = probe.algo == c.algo ? c
                          : (probe.algo == "direct" ? default_direct(d)
                             : probe.algo == "rgemm" ? default_rgemm(cin, cout, lp)
                                                     : default_igemm(cin, cout, d.precision != FBCORR_FP32));
            RoleBuild rb;
            if (parse_config(text, base, err) && build_role(d, role, base, di, rb, err)) return base;
        }
    }
    return heuristic_default(d, role, di);
}

bool config_from_text(const fbcorr_desc& d, int role, const DeviceInfo& di, const std::string& text,
                      bool reset_named, Config& out, std::string& err) {
    // A text that names another algorithm than the role's default starts
    // from that algorithm's hand-written defaults ("algo=direct" alone is a
    // complete configuration); with reset_named a forward-role text that
    // names an algorithm always does.  Otherwise unnamed knobs keep the
    // role's default.
    Config c = default_config(d, role, di);
    const int cin = role == FBCORR_ROLE_BACKWARD_X ? d.N : d.D;
    const int cout = role == FBCORR_ROLE_BACKWARD_X ? d.D : d.N;
    const bool lp = d.precision != FBCORR_FP32 && role == FBCORR_ROLE_FORWARD;
    if (role == FBCORR_ROLE_FORWARD) {
        if (text.find("algo=direct") != std::string::npos) c = default_direct(d);
        if (text.find("algo=igemm") != std::string::npos && (reset_named || c.algo != "igemm"))
            c = default_igemm(cin, cout, lp);
        if (text.find("algo=rgemm") != std::string::npos && (reset_named || c.algo != "rgemm"))
            c = default_rgemm(cin, cout, lp);
    } else if (role == FBCORR_ROLE_BACKWARD_X) {
        if (text.find("algo=igemm") != std::string::npos && c.algo != "igemm") c = default_igemm(cin, cout, false);
        if (text.find("algo=rgemm") != std::string::npos && c.algo != "rgemm") c = default_rgemm(cin, cout, false);
    }
    if (!parse_config(text, c, err)) return false;
    out = c;
    return true;
}

Config heuristic_default(const fbcorr_desc& d, int role, const DeviceInfo& di) {
    const Config h = heuristic_config(d, role, di.cus);
    for (const Config& c : shrink_sequence(h)) {
        RoleBuild rb;
        std::string err;
        if (build_role(d, role, c, di, rb, err)) return c;
    }
    return h;   // nothing fits: the caller reports the heuristic's error
}

}  // namespace fbc
