// Launch geometry and per-role build descriptions.
#pragma once

#include "internal.h"

namespace fbc {

struct LaunchGeom {
    int grid_x = 0, grid_y = 1;
    int threads = 0;
    int lds = 0;
};

// Everything needed to run one role: the main kernel, helper kernels (run
// before the main kernel for the forward/input-gradient roles, after it for
// the filter-gradient role), their launch shapes, and workspace use.
struct RoleBuild {
    Config cfg;
    KernelSource main;
    LaunchGeom main_geom;
    std::vector<KernelSource> aux;
    std::vector<LaunchGeom> aux_geom;
    size_t ws_bytes = 0;
    size_t ws_lowp_w = 0, ws_unscale = 0;   // forward low-precision layout
    size_t ws_xmax = 0;                     // fp16: partial maxima of |x| (aux[1])
    int nxp = 0;                            //   their count (0: no input scale)
    int np = 0;                             // filter-gradient partial count
};

// Default configuration of a role: the tuning database's entry for this
// hardware and problem if there is one, else the hand-written heuristic
// (shrunk until it fits the device).
Config default_config(const fbcorr_desc& d, int role, const DeviceInfo& di);
Config heuristic_default(const fbcorr_desc& d, int role, const DeviceInfo& di);

// tuning_db.cpp
std::string tuning_db_path();
bool tuning_db_lookup(const std::string& arch, int role, const fbcorr_desc& d, std::string& cfg);
bool tuning_db_record(const std::string& arch, int role, const fbcorr_desc& d, const std::string& cfg,
                      std::string& err);
void tuning_db_reload();
bool tuning_db_lookup_key(const std::string& key, std::string& cfg);
bool tuning_db_record_key(const std::string& key, const std::string& cfg, std::string& err);
Config default_igemm(int cin, int cout, bool lowp);
Config default_rgemm(int cin, int cout, bool lowp);
Config default_direct(const fbcorr_desc& d);
// The configuration a text such as "algo=rgemm mt=2" describes for a role:
// unnamed knobs come from the role's default, or from the named algorithm's
// hand-written defaults when it differs from the default's (always, on the
// forward role, with reset_named).
bool config_from_text(const fbcorr_desc& d, int role, const DeviceInfo& di, const std::string& text,
                      bool reset_named, Config& out, std::string& err);
bool build_role(const fbcorr_desc& d, int role, const Config& c, const DeviceInfo& di,
                RoleBuild& rb, std::string& err);

// Tuning grids (tune.cpp).
std::vector<Config> tune_candidates(const fbcorr_desc& d, int role, bool with_direct, bool direct_only);

}  // namespace fbc
