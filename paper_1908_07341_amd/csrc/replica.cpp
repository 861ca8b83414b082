// Host side of the replica-coded chains: per-replica threshold data and the
// C-ABI entry points.
#include <cmath>
#include <cstring>

#include "sd_host.hpp"
#include "sd_replica.hpp"

namespace sd {

ReplicaParams replica_params(const double* J, const double* q) {
    ReplicaParams rp;
    std::memset(&rp, 0, sizeof rp);
    for (uint32_t r = 0; r < kReplicas; ++r) {
        uint32_t T[6];
        threshold_table(J[r], q[r], T);
        for (int m = 0; m < 8; ++m)
            for (int k = 0; k < 3; ++k)
                rp.S[m][k] |= (uint64_t)((T[k] >> (31 - m)) & 1u) << r;
        for (int idx = 0; idx < 6; ++idx)
            rp.T24[idx][r] = paired_tail(T, idx);
    }
    return rp;
}

}  // namespace sd

using namespace sd;

namespace {

sd_status check_replica_lattice(const void* p, int32_t L, const char* what) {
    if (!p)
        return fail(SD_EINVAL, "%s: null lattice", what);
    if (L < 8 || L > 32768 || L % 8 != 0)
        return fail(SD_EINVAL, "%s: L must be a multiple of 8 in [8, 32768]", what);
    if (reinterpret_cast<uintptr_t>(p) & 7u)
        return fail(SD_EINVAL, "%s: replica lattices must be 8-byte aligned", what);
    return SD_OK;
}

}  // namespace

extern "C" {

size_t sd_replica_lattice_bytes(int32_t L) {
    if (L < 8 || L > 32768 || L % 8 != 0)
        return 0;
    return (size_t)L * (size_t)L * sizeof(uint64_t);
}

sd_status sd_replica_run(void* sigma, void* tau, int32_t L, const double* J, const double* q, uint64_t seed,
                         uint32_t stream, uint64_t step0, uint32_t k_steps, void* hip_stream) {
    sd_status s = check_replica_lattice(sigma, L, "sd_replica_run(sigma)");
    if (s == SD_OK)
        s = check_replica_lattice(tau, L, "sd_replica_run(tau)");
    if (s != SD_OK)
        return s;
    if (!J || !q)
        return fail(SD_EINVAL, "sd_replica_run: null parameter arrays");
    for (uint32_t r = 0; r < kReplicas; ++r)
        if (!std::isfinite(J[r]) || !std::isfinite(q[r]))
            return fail(SD_EINVAL, "sd_replica_run: J and q of replica %u must be finite", r);
    if (step0 + (uint64_t)k_steps > (1ull << 29))
        return fail(SD_EINVAL, "sd_replica_run: step indices must stay below 2^29");
    const size_t bytes = sd_replica_lattice_bytes(L);
    const uintptr_t a = reinterpret_cast<uintptr_t>(sigma), b = reinterpret_cast<uintptr_t>(tau);
    if (a < b + bytes && b < a + bytes)
        return fail(SD_EINVAL, "sd_replica_run: sigma and tau overlap");
    const ReplicaParams rp = replica_params(J, q);
    const hipStream_t st = static_cast<hipStream_t>(hip_stream);
    uint64_t* sg = static_cast<uint64_t*>(sigma);
    uint64_t* tu = static_cast<uint64_t*>(tau);
    hipError_t e = hipSuccess;
    for (uint32_t m = 0; m < k_steps && e == hipSuccess; ++m) {
        const uint64_t n = step0 + m;
        DrawParams dp = dynamics_params(0.0, 0.0, seed, stream, (uint32_t)(2 * n), 0);
        e = launch_replica_half(0, sg, tu, (uint32_t)L, dp, rp, st);
        if (e == hipSuccess) {
            dp.t = (uint32_t)(2 * n + 1);
            e = launch_replica_half(1, tu, sg, (uint32_t)L, dp, rp, st);
        }
    }
    return e == hipSuccess ? SD_OK : hip_fail(e, "sd_replica_run");
}

sd_status sd_replica_observe(const void* sigma, const void* tau, int32_t L, int64_t* out, void* hip_stream) {
    sd_status s = check_replica_lattice(sigma, L, "sd_replica_observe(sigma)");
    if (s == SD_OK)
        s = check_replica_lattice(tau, L, "sd_replica_observe(tau)");
    if (s != SD_OK)
        return s;
    if (!out)
        return fail(SD_EINVAL, "sd_replica_observe: null output");
    hipError_t e = launch_replica_observe(static_cast<const uint64_t*>(sigma), static_cast<const uint64_t*>(tau),
                                          (uint32_t)L, out, static_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? SD_OK : hip_fail(e, "sd_replica_observe");
}

}  // extern "C"
