// Autotune cache of the solver's launch shapes: a JSON object file mapping a
// configuration key to the shapes chosen for it (host code only).
//
//   { "<key>": {"block": 256, "zb": 4, "zb_down": [16, 4, 1], "zb_up": [16, 4, 1],
//               "dn_region": [0, 0, 512], "step_ms": 12.1, "default_step_ms": 12.9}, ... }
//
// Array entry l belongs to multigrid level l (the pass from level l down to
// l + 1, and the up pass on level l); dn_region 0 = automatic.
#pragma once

#include <map>
#include <string>
#include <vector>

namespace hh {

struct TuneEntry {
    int block = 256;            // lanes of the flat Krylov kernels
    int zb = 4;                 // z-planes per workgroup of the operator apply
    std::vector<int> zb_down;   // per level: coarse planes per workgroup of the down pass
    std::vector<int> zb_up;     // per level: fine planes per workgroup of the up pass
    std::vector<int> dn_region; // per level: region of a one-plane down pass (0 = automatic)
    double step_ms = 0.0;       // measured time of one step with these shapes
    double default_step_ms = 0.0;  // and with the built-in rule
};

// Reads `path` into `out`.  A missing file is an empty cache (true).  Returns
// false with a message in `err` when the file exists but is not a JSON object
// of such entries.
bool tune_cache_read(const char* path, std::map<std::string, TuneEntry>& out, std::string& err);

// Writes every entry of `m` to "<path>.tmp" and renames it to `path`.
bool tune_cache_write(const char* path, const std::map<std::string, TuneEntry>& m, std::string& err);

}  // namespace hh
