// Persistent kernel-tuning choices.
//
// The autotuners of contexts and batches time their candidate kernels once
// per process and configuration.  When the environment variable
// OTM_TUNE_CACHE names a file, a choice is also looked up there before any
// timing and appended there after it, so later processes (and other
// machines of the same architecture, if the file is shipped with them) reuse
// it instead of re-timing candidates whose times differ by noise.
//
// File format: plain text, one choice per line,
//   <device architecture> <key> <value> <value> ...
// with whitespace-free architecture and key strings; '#' starts a comment
// line.  The last line for an (architecture, key) pair wins, so appending a
// newer choice overrides an older one.  A line that does not parse is
// ignored.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "otm_internal.h"

namespace otm {
namespace {
std::mutex g_file_mu;

const char* cache_path() {
    const char* p = std::getenv("OTM_TUNE_CACHE");
    return (p && p[0]) ? p : nullptr;
}
}  // namespace

std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string a = prop.gcnArchName;
    for (char& ch : a)
        if (ch == ' ' || ch == '\t') ch = '_';
    return a.empty() ? "unknown" : a;
}

bool tune_cache_lookup(const std::string& key, std::vector<double>& vals) {
    const char* path = cache_path();
    if (!path) return false;
    const std::string arch = device_arch();
    std::lock_guard<std::mutex> lock(g_file_mu);
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    bool found = false;
    char line[1024];
    while (std::fgets(line, sizeof(line), f)) {
        if (line[0] == '#') continue;
        std::istringstream in(line);
        std::string a, k;
        if (!(in >> a >> k) || a != arch || k != key) continue;
        std::vector<double> v;
        double x;
        while (in >> x) v.push_back(x);
        if (v.size() == vals.size()) {
            vals = v;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void tune_cache_store(const std::string& key, const std::vector<double>& vals) {
    const char* path = cache_path();
    if (!path) return;
    std::ostringstream out;
    out << device_arch() << ' ' << key;
    for (double v : vals) out << ' ' << v;
    out << '\n';
    const std::string s = out.str();
    std::lock_guard<std::mutex> lock(g_file_mu);
    FILE* f = std::fopen(path, "a");
    if (!f) return;  // an unwritable cache only costs re-timing
    (void)std::fwrite(s.data(), 1, s.size(), f);
    std::fclose(f);
}

}  // namespace otm
