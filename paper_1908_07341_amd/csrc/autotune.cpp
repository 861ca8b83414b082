// Autotuner cache and selection helpers.
#include "sd_autotune.hpp"

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>

namespace sd {
namespace {

std::map<std::string, long> read_cache(const char* path) {
    std::map<std::string, long> out;
    std::ifstream f(path);
    if (!f)
        return out;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t i = 0;
    while (true) {
        size_t k0 = s.find('"', i);
        if (k0 == std::string::npos)
            break;
        size_t k1 = s.find('"', k0 + 1);
        if (k1 == std::string::npos)
            break;
        size_t colon = s.find(':', k1);
        if (colon == std::string::npos)
            break;
        const char* start = s.c_str() + colon + 1;
        char* end = nullptr;
        long v = std::strtol(start, &end, 10);
        if (end != start)
            out[s.substr(k0 + 1, k1 - k0 - 1)] = v;
        i = (size_t)(end - s.c_str());
        if (end == start)
            i = colon + 1;
    }
    return out;
}

}  // namespace

long tune_cache_get(const char* path, const std::string& key) {
    if (!path || !*path)
        return -1;
    auto m = read_cache(path);
    auto it = m.find(key);
    return it == m.end() ? -1 : it->second;
}

bool tune_cache_put(const char* path, const std::string& key, long value) {
    if (!path || !*path)
        return false;
    auto m = read_cache(path);
    m[key] = value;
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f)
            return false;
        f << "{\n";
        size_t n = 0;
        for (auto& kv : m)
            f << "  \"" << kv.first << "\": " << kv.second << (++n < m.size() ? ",\n" : "\n");
        f << "}\n";
        if (!f)
            return false;
    }
    return std::rename(tmp.c_str(), path) == 0;
}

std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string a = prop.gcnArchName;
    size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

long tune_pick(const std::vector<long>& candidates, const std::function<double(long)>& measure) {
    long best = -1;
    double best_t = 0.0;
    for (long c : candidates) {
        const double t = measure(c);
        if (t > 0.0 && (best < 0 || t < best_t)) {
            best = c;
            best_t = t;
        }
    }
    return best;
}

}  // namespace sd
