// Host helpers shared by the C-ABI translation units.
#pragma once

#include <stdint.h>

#include "shaken.h"
#include "sd_kernels.hpp"

namespace sd {

sd_status fail(sd_status s, const char* fmt, ...);
sd_status hip_fail(hipError_t e, const char* what);
bool layout_supported(int32_t L, int32_t layout);
size_t lattice_bytes(int32_t L, int32_t layout);
Geom make_geom(int32_t L, int klay);
uint32_t threshold(double h);
void threshold_table(double J, double q, uint32_t T[6]);
DrawParams dynamics_params(double J, double q, uint64_t seed, uint32_t stream, uint32_t t, uint32_t flags);

}  // namespace sd
