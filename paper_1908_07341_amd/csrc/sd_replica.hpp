// Internal interface of the replica-coded kernels (multi-spin coding across
// chains that share one stream).
#pragma once

#include "sd_kernels.hpp"

namespace sd {

constexpr uint32_t kReplicas = 64;

// Per-replica threshold data, passed by value to the kernels.
struct ReplicaParams {
    uint64_t S[8][3];             // bit r: bit (31 - m) of T_r[k], leader classes k = 0, 1, 2
    uint32_t T24[6][kReplicas];   // paired_tail(T_r, idx)
};

ReplicaParams replica_params(const double* J, const double* q);

// One half-step of all replicas: which = 0 draws tau from sigma (down/left
// field), 1 draws sigma from tau (up/right).  L % 8 == 0; dp carries seed,
// stream and half-step index (its thresholds are not used).
hipError_t launch_replica_half(int which, const uint64_t* src, uint64_t* dst, uint32_t L, const DrawParams& dp,
                               const ReplicaParams& rp, hipStream_t st);
// out[3 r + {0, 1, 2}] = (M, A, B) of replica r's pair (sigma, tau).
hipError_t launch_replica_observe(const uint64_t* sigma, const uint64_t* tau, uint32_t L, int64_t* out,
                                  hipStream_t st);

}  // namespace sd
