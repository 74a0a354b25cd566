// Tuning database: tuned configurations keyed by hardware and problem.
//
// The paper's vision application notes that the best variant differs per
// input and per GPU, and that an application can either tune in situ or ship
// a database of configurations for the platforms it runs on (Sec. 6.2).
// This is that database.  One entry per line:
//
//   <arch> <role> <precision> <batch> <H> <W> <D> <N> <fh> <fw> : <config text>
//   <arch> nearest u8 <T> <M> <D> : <config text>      (nearest-neighbour search)
//
// A batched plan's variants use role "batched" with H = W = 0: one entry per
// key (fh, fw, D, N), whatever the image sizes.
//
// '#' starts a comment.  The file is tuning_db.txt next to libfbcorr.so, or
// the path in FBCORR_TUNING_DB.  fbcorr_tune can record its winner here.
#include "plan.h"

#include <dlfcn.h>
#include <unistd.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>

namespace fbc {

namespace {
std::mutex g_db_mu;
bool g_db_loaded = false;
std::map<std::string, std::string> g_db;
}  // namespace

static const char* kRoleNames[] = {"forward", "backward_x", "backward_w", "batched"};
static const char* kPrecNames[] = {"fp32", "bf16", "fp16"};

std::string tuning_db_path() {
    const char* env = getenv("FBCORR_TUNING_DB");
    if (env && *env) return env;
    Dl_info info;
    if (dladdr((void*)&tuning_db_path, &info) && info.dli_fname) {
        std::string so = info.dli_fname;
        auto slash = so.rfind('/');
        return (slash == std::string::npos ? std::string(".") : so.substr(0, slash)) + "/tuning_db.txt";
    }
    return "tuning_db.txt";
}

static std::string db_key(const std::string& arch, int role, const fbcorr_desc& d) {
    std::ostringstream os;
    os << arch << ' ' << kRoleNames[role] << ' ' << kPrecNames[d.precision] << ' ' << d.batch << ' ' << d.H << ' '
       << d.W << ' ' << d.D << ' ' << d.N << ' ' << d.fh << ' ' << d.fw;
    // the forward role also depends on the requested algorithm
    if (role == FBCORR_ROLE_FORWARD && d.algo == FBCORR_ALGO_DIRECT) os << " direct";
    return os.str();
}

static void load_locked() {
    if (g_db_loaded) return;
    g_db_loaded = true;
    std::ifstream in(tuning_db_path());
    std::string line;
    while (std::getline(in, line)) {
        auto hash = line.find('#');
        if (hash != std::string::npos) line = line.substr(0, hash);
        auto colon = line.find(':');
        if (colon == std::string::npos) continue;
        std::string key = line.substr(0, colon), cfg = line.substr(colon + 1);
        // normalise whitespace of the key
        std::istringstream ks(key);
        std::string tok, norm;
        while (ks >> tok) norm += (norm.empty() ? "" : " ") + tok;
        while (!cfg.empty() && (cfg[0] == ' ' || cfg[0] == '\t')) cfg.erase(0, 1);
        while (!cfg.empty() && (cfg.back() == ' ' || cfg.back() == '\r' || cfg.back() == '\t')) cfg.pop_back();
        if (!norm.empty() && !cfg.empty()) g_db[norm] = cfg;
    }
}

bool tuning_db_lookup_key(const std::string& key, std::string& cfg) {
    std::lock_guard<std::mutex> lk(g_db_mu);
    load_locked();
    auto it = g_db.find(key);
    if (it == g_db.end()) return false;
    cfg = it->second;
    return true;
}

bool tuning_db_lookup(const std::string& arch, int role, const fbcorr_desc& d, std::string& cfg) {
    return tuning_db_lookup_key(db_key(arch, role, d), cfg);
}

bool tuning_db_record(const std::string& arch, int role, const fbcorr_desc& d, const std::string& cfg,
                      std::string& err) {
    return tuning_db_record_key(db_key(arch, role, d), cfg, err);
}

bool tuning_db_record_key(const std::string& key, const std::string& cfg, std::string& err) {
    std::lock_guard<std::mutex> lk(g_db_mu);
    load_locked();
    g_db[key] = cfg;
    const std::string path = tuning_db_path();
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    {
        std::ofstream out(tmp);
        if (!out) { err = "cannot write " + tmp; return false; }
        out << "# fbcorr tuning database: <arch> <role> <precision> <batch> <H> <W> <D> <N> <fh> <fw> : <config>\n"
               "#                          <arch> nearest u8 <T> <M> <D> : <config>\n";
        for (auto& kv : g_db) out << kv.first << " : " << kv.second << "\n";
    }
    if (rename(tmp.c_str(), path.c_str()) != 0) { err = "cannot replace " + path; return false; }
    return true;
}

void tuning_db_reload() {
    std::lock_guard<std::mutex> lk(g_db_mu);
    g_db.clear();
    g_db_loaded = false;
}

}  // namespace fbc
