// Launch-shape autotuner: measures candidate shapes with HIP events and keeps
// the winners in a small JSON file (a flat object of "key": integer pairs).
#pragma once

#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

struct sd_batch_plan;

namespace sd {

// Value cached under `key` in the JSON file at `path`, or -1.
long tune_cache_get(const char* path, const std::string& key);
// Store `value` under `key` (the rest of the file is kept).  Returns false on I/O error.
bool tune_cache_put(const char* path, const std::string& key, long value);

// Name of the current device's architecture ("gfx950" style), for cache keys.
std::string device_arch();

// Pick the candidate with the smallest measured time (seconds, < 0 = failed).
long tune_pick(const std::vector<long>& candidates, const std::function<double(long)>& measure);

// Block size of the batched kernel for chains of size L (see batch.cpp).
uint32_t autotune_batch_threads(const char* cache_path, uint32_t L, uint32_t paired, uint32_t n_chains,
                                sd_batch_plan* plan);

}  // namespace sd
