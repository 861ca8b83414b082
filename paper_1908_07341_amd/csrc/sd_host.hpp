// Host helpers shared by the C-ABI translation units.
#pragma once

#include <stdint.h>

#include <mutex>

#include "shaken.h"
#include "sd_kernels.hpp"

namespace sd {

sd_status fail(sd_status s, const char* fmt, ...);
sd_status hip_fail(hipError_t e, const char* what);
bool layout_supported(int32_t L, int32_t layout);
size_t lattice_bytes(int32_t L, int32_t layout);
Geom make_geom(int32_t L, int klay);
int kernel_layout(int32_t L, int32_t layout, const void* p);
int packed_rows_layout(int32_t L);
uint32_t threshold(double h);
void threshold_table(double J, double q, uint32_t T[6]);
DrawParams dynamics_params(double J, double q, uint64_t seed, uint32_t stream, uint32_t t, uint32_t flags);

// Device scratch of kPartialsWords int64 for per-workgroup partial sums, one
// per (device, stream), allocated on first use and kept for the process.
// Null when it does not exist yet and cannot be made now (the stream is
// being captured, or the allocation failed); callers then use atomics.  A
// call holds mu while it enqueues the launches that write and read p, so
// that calls from several host threads on one stream do not interleave
// their use of the slots.
constexpr size_t kPartialsWords = 65536;
struct Workspace {
    int64_t* p = nullptr;
    std::mutex mu;
};
Workspace* partials_workspace(hipStream_t st);

}  // namespace sd
