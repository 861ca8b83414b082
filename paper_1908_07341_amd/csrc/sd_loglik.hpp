// Internal interface of the log-likelihood kernels.
#pragma once

#include "sd_kernels.hpp"

namespace sd {

// out: the 12 counts, or (paired) the 6 paired statistics.
// partials: device scratch of partials_words int64 for the workgroup sums
// (null, or too small for the grid: the workgroups add with atomics).
hipError_t launch_loglik_counts(const void* traj, uint32_t n_traj, uint32_t n_lat, uint32_t L, int64_t* out,
                                bool paired, hipStream_t st, int64_t* partials = nullptr, size_t partials_words = 0);
hipError_t launch_loglik_fwd(const int64_t* stats, bool paired, const float* Jq, float* ll, hipStream_t st);
hipError_t launch_loglik_bwd(const int64_t* stats, bool paired, const float* Jq, const float* g_out, float* grad,
                             hipStream_t st);

}  // namespace sd
