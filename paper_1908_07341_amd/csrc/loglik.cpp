// Host side of the trajectory generator and the log-likelihood entry points.
#include <cmath>

#include "sd_batch.hpp"
#include "sd_host.hpp"
#include "sd_loglik.hpp"

using namespace sd;

extern "C" {

sd_status sd_trajectory(const void* sigma0, void* traj, int32_t L, int32_t layout, double J, double q, uint64_t seed,
                        uint32_t stream, uint64_t step0, uint32_t k_steps, void* hip_stream) {
    if (layout != SD_P64 && layout != SD_P32)
        return fail(SD_EUNSUPPORTED, "sd_trajectory: trajectories are stored packed (SD_P64 or SD_P32)");
    if (!layout_supported(L, layout) || !sigma0 || !traj)
        return fail(SD_EINVAL, "sd_trajectory: bad lattice size or null pointer");
    if (!std::isfinite(J) || !std::isfinite(q))
        return fail(SD_EINVAL, "sd_trajectory: J and q must be finite");
    if (step0 + (uint64_t)k_steps > (1ull << 29))
        return fail(SD_EINVAL, "sd_trajectory: step indices must stay below 2^29");
    const uintptr_t align = layout == SD_P64 ? 8u : 4u;
    if ((reinterpret_cast<uintptr_t>(sigma0) | reinterpret_cast<uintptr_t>(traj)) & (align - 1))
        return fail(SD_EINVAL, "sd_trajectory: pointers not aligned to the word size");
    const size_t bytes = lattice_bytes(L, layout);
    const uintptr_t s0 = reinterpret_cast<uintptr_t>(sigma0), t0 = reinterpret_cast<uintptr_t>(traj);
    if (s0 < t0 + bytes * (2 * (size_t)k_steps + 1) && t0 < s0 + bytes && s0 != t0)
        return fail(SD_EINVAL, "sd_trajectory: sigma0 overlaps the trajectory (other than as its first lattice)");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    uint8_t* base = static_cast<uint8_t*>(traj);
    hipError_t e = hipSuccess;
    if (sigma0 != traj)
        e = hipMemcpyAsync(base, sigma0, bytes, hipMemcpyDeviceToDevice, st);
    const int klay = kernel_layout(L, layout, traj);
    const Geom G = make_geom(L, klay);
    for (uint32_t m = 0; m < k_steps && e == hipSuccess; ++m) {
        const uint64_t n = step0 + m;
        uint8_t* x = base + (2 * (size_t)m) * bytes;
        DrawParams dp = dynamics_params(J, q, seed, stream, (uint32_t)(2 * n), 0);
        e = launch_half_step(klay, 0, x, x + bytes, G, dp, nullptr, st);
        if (e == hipSuccess) {
            dp.t = (uint32_t)(2 * n + 1);
            e = launch_half_step(klay, 1, x + bytes, x + 2 * bytes, G, dp, nullptr, st);
        }
    }
    return e == hipSuccess ? SD_OK : hip_fail(e, "sd_trajectory");
}

sd_status sd_trajectories(const void* sigma0, void* traj, int32_t n_traj, int32_t L, int32_t layout, double J,
                          double q, uint64_t seed, uint32_t stream0, uint64_t step0, uint32_t k_steps,
                          void* hip_stream) {
    if (layout != SD_P64 && layout != SD_P32)
        return fail(SD_EUNSUPPORTED, "sd_trajectories: trajectories are stored packed (SD_P64 or SD_P32)");
    if (n_traj < 0 || !layout_supported(L, layout) || (n_traj > 0 && (!sigma0 || !traj)))
        return fail(SD_EINVAL, "sd_trajectories: bad count, lattice size or null pointer");
    if (!std::isfinite(J) || !std::isfinite(q))
        return fail(SD_EINVAL, "sd_trajectories: J and q must be finite");
    if (step0 + (uint64_t)k_steps > (1ull << 29))
        return fail(SD_EINVAL, "sd_trajectories: step indices must stay below 2^29");
    if ((uint64_t)stream0 + (uint64_t)n_traj > (1ull << 32))
        return fail(SD_EINVAL, "sd_trajectories: stream ids must stay below 2^32");
    if ((reinterpret_cast<uintptr_t>(sigma0) | reinterpret_cast<uintptr_t>(traj)) & 7u)
        return fail(SD_EINVAL, "sd_trajectories: pointers must be 8-byte aligned");
    if (n_traj == 0)
        return SD_OK;
    const size_t bytes = lattice_bytes(L, layout);
    const size_t per = bytes * (2 * (size_t)k_steps + 1);
    const uintptr_t s0 = reinterpret_cast<uintptr_t>(sigma0), t0 = reinterpret_cast<uintptr_t>(traj);
    if (s0 < t0 + per * (size_t)n_traj && t0 < s0 + bytes * (size_t)n_traj)
        return fail(SD_EINVAL, "sd_trajectories: the start lattices overlap the trajectories");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const uint32_t n_words = (uint32_t)(((uint64_t)L * (uint64_t)L) / 64u);
    int dev = 0, max_lds = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess)
        return hip_fail(e, "sd_trajectories");
    // 512 threads from 1024 words up: 256 trajectories of 256^2 (one workgroup each) leave
    // the CUs short of waves at 256 threads
    const uint32_t threads = n_words >= 1024u ? 512u : 256u;
    if (L % 8 == 0 && batch_lds_bytes(n_words, threads) <= (size_t)max_lds) {
        e = launch_trajectories_lds(sigma0, traj, (uint32_t)n_traj, L, J, q, seed, stream0, step0, k_steps, threads,
                                    st);
        return e == hipSuccess ? SD_OK : hip_fail(e, "sd_trajectories");
    }
    for (int32_t a = 0; a < n_traj; ++a) {
        const sd_status r = sd_trajectory(static_cast<const uint8_t*>(sigma0) + (size_t)a * bytes,
                                          static_cast<uint8_t*>(traj) + (size_t)a * per, L, layout, J, q, seed,
                                          stream0 + (uint32_t)a, step0, k_steps, hip_stream);
        if (r != SD_OK)
            return r;
    }
    return SD_OK;
}

}  // extern "C"

namespace {

sd_status loglik_sums(const char* name, const void* traj, int32_t n_traj, int32_t n_lat, int32_t L, int64_t* out,
                      bool paired, void* hip_stream) {
    if (!traj || !out)
        return fail(SD_EINVAL, "%s: null pointer", name);
    if (n_traj < 0 || n_lat < 1 || L < 64 || L > 65535 || L % 64 != 0)
        return fail(SD_EINVAL, "%s: need n_traj >= 0, n_lat >= 1 and L a multiple of 64", name);
    if (reinterpret_cast<uintptr_t>(traj) & 7u)
        return fail(SD_EINVAL, "%s: trajectories must be 8-byte aligned", name);
    const hipStream_t st = static_cast<hipStream_t>(hip_stream);
    Workspace* ws = partials_workspace(st);
    std::unique_lock<std::mutex> hold;   // keeps this call's use of the workspace contiguous on the stream
    if (ws)
        hold = std::unique_lock<std::mutex>(ws->mu);
    hipError_t e = launch_loglik_counts(traj, (uint32_t)n_traj, (uint32_t)n_lat, (uint32_t)L, out, paired, st,
                                        ws ? ws->p : nullptr, kPartialsWords);
    return e == hipSuccess ? SD_OK : hip_fail(e, name);
}

sd_status loglik_fwd(const char* name, const int64_t* stats, bool paired, const float* Jq, float* ll,
                     void* hip_stream) {
    if (!stats || !Jq || !ll)
        return fail(SD_EINVAL, "%s: null pointer", name);
    hipError_t e = launch_loglik_fwd(stats, paired, Jq, ll, static_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? SD_OK : hip_fail(e, name);
}

sd_status loglik_bwd(const char* name, const int64_t* stats, bool paired, const float* Jq, const float* g_out,
                     float* grad, void* hip_stream) {
    if (!stats || !Jq || !grad)
        return fail(SD_EINVAL, "%s: null pointer", name);
    hipError_t e = launch_loglik_bwd(stats, paired, Jq, g_out, grad, static_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? SD_OK : hip_fail(e, name);
}

}  // namespace

extern "C" {

sd_status sd_loglik_counts(const void* traj, int32_t n_traj, int32_t n_lat, int32_t L, int64_t* counts12,
                           void* hip_stream) {
    return loglik_sums("sd_loglik_counts", traj, n_traj, n_lat, L, counts12, false, hip_stream);
}

sd_status sd_loglik_fwd(const int64_t* counts12, const float* Jq, float* ll, void* hip_stream) {
    return loglik_fwd("sd_loglik_fwd", counts12, false, Jq, ll, hip_stream);
}

sd_status sd_loglik_bwd(const int64_t* counts12, const float* Jq, const float* g_out, float* grad,
                        void* hip_stream) {
    return loglik_bwd("sd_loglik_bwd", counts12, false, Jq, g_out, grad, hip_stream);
}

sd_status sd_loglik_stats(const void* traj, int32_t n_traj, int32_t n_lat, int32_t L, int64_t* stats6,
                          void* hip_stream) {
    return loglik_sums("sd_loglik_stats", traj, n_traj, n_lat, L, stats6, true, hip_stream);
}

sd_status sd_loglik_fwd_stats(const int64_t* stats6, const float* Jq, float* ll, void* hip_stream) {
    return loglik_fwd("sd_loglik_fwd_stats", stats6, true, Jq, ll, hip_stream);
}

sd_status sd_loglik_bwd_stats(const int64_t* stats6, const float* Jq, const float* g_out, float* grad,
                              void* hip_stream) {
    return loglik_bwd("sd_loglik_bwd_stats", stats6, true, Jq, g_out, grad, hip_stream);
}

}  // extern "C"
