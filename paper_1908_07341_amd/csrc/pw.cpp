// Host side of coupling from the past (Propp-Wilson) on the monotone coupling
// of section 3.2.  Each round runs every pair still open, from all +1 and
// all -1 at time -T, through the batched chain kernel (the two chains of a
// pair are two queue entries with the same stream), then compares the pairs
// on the device and reads one flag per pair back; T doubles between rounds.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "sd_batch.hpp"
#include "sd_host.hpp"

using namespace sd;

namespace {

// Device scratch of one sd_propp_wilson call, freed when it returns.
struct PwScratch {
    ChainDesc* descs = nullptr;
    uint32_t* order = nullptr;
    uint32_t* pairs = nullptr;
    uint32_t* equal = nullptr;
    uint32_t* counter = nullptr;
    ~PwScratch() {
        (void)hipFree(descs);
        (void)hipFree(order);
        (void)hipFree(pairs);
        (void)hipFree(equal);
        (void)hipFree(counter);
    }
    hipError_t alloc(uint32_t n) {
        hipError_t e = hipMalloc(&descs, sizeof(ChainDesc) * 2 * (size_t)n);
        if (e == hipSuccess) e = hipMalloc(&order, sizeof(uint32_t) * 2 * (size_t)n);
        if (e == hipSuccess) e = hipMalloc(&pairs, sizeof(uint32_t) * (size_t)n);
        if (e == hipSuccess) e = hipMalloc(&equal, sizeof(uint32_t) * (size_t)n);
        if (e == hipSuccess) e = hipMalloc(&counter, sizeof(uint32_t));
        return e;
    }
};

uint32_t chain_threads(uint32_t words) { return words <= 64u ? 64u : words <= 256u ? 128u : 256u; }

}  // namespace

extern "C" {

sd_status sd_propp_wilson(void* samples, void* work, int32_t n_samples, int32_t L, double J, double q,
                          uint64_t seed, uint32_t stream0, uint64_t step_end, uint32_t T0, uint32_t T_max,
                          int64_t* T_used, void* hip_stream) {
    if (!samples || !work || !T_used || n_samples < 0)
        return fail(SD_EINVAL, "sd_propp_wilson: null pointer or negative sample count");
    if (L < 8 || L > 65535 || L % 8 != 0)
        return fail(SD_EINVAL, "sd_propp_wilson: L must be a multiple of 8");
    if (!(J >= 0.0) || !(q >= 0.0) || !std::isfinite(J) || !std::isfinite(q))
        return fail(SD_EINVAL, "sd_propp_wilson: the coupling is monotone only for finite J, q >= 0");
    if (T0 < 1 || T_max < T0 || step_end < T_max || step_end > (1ull << 29))
        return fail(SD_EINVAL, "sd_propp_wilson: need 1 <= T0 <= T_max <= step_end <= 2^29");
    if ((reinterpret_cast<uintptr_t>(samples) | reinterpret_cast<uintptr_t>(work)) & 7u)
        return fail(SD_EINVAL, "sd_propp_wilson: buffers must be 8-byte aligned");
    if ((uint64_t)stream0 + (uint64_t)n_samples > (1ull << 32))
        return fail(SD_EINVAL, "sd_propp_wilson: stream ids past 2^32");
    const uint32_t n = (uint32_t)n_samples;
    const uint32_t words = lattice_words((uint32_t)L);
    const size_t nb = (size_t)words * sizeof(uint64_t);
    const uint8_t* s0 = static_cast<const uint8_t*>(samples);
    const uint8_t* w0 = static_cast<const uint8_t*>(work);
    if (n && s0 < w0 + 4 * nb * n && w0 < s0 + nb * n)
        return fail(SD_EINVAL, "sd_propp_wilson: samples and work overlap");
    for (uint32_t p = 0; p < n; ++p)
        T_used[p] = 0;
    if (n == 0)
        return SD_OK;

    int device = 0, max_lds = 0, n_cu = 1;
    hipError_t e = hipGetDevice(&device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess)
        return hip_fail(e, "sd_propp_wilson");
    const uint32_t threads = chain_threads(words);
    const size_t lds = batch_lds_bytes(words, threads);
    if (lds > (size_t)max_lds)
        return fail(SD_EUNSUPPORTED, "sd_propp_wilson: an L = %d lattice pair does not fit one workgroup's LDS", L);

    ChainDesc proto;
    std::memset(&proto, 0, sizeof proto);
    threshold_table(J, q, proto.T);
    proto.paired = thresholds_paired(proto.T) ? 1u : 0u;
    proto.L = (uint32_t)L;
    set_divisors(proto, (uint32_t)L);
    int per_cu = 0;
    e = batch_kernel_attributes(lds);
    if (e == hipSuccess) e = batch_occupancy(threads, lds, proto.paired != 0, L % 64 != 0, &per_cu);
    if (e != hipSuccess)
        return hip_fail(e, "sd_propp_wilson");
    PwScratch sc;
    e = sc.alloc(n);
    if (e != hipSuccess)
        return hip_fail(e, "sd_propp_wilson: scratch");

    const hipStream_t st = static_cast<hipStream_t>(hip_stream);
    uint8_t* lat = static_cast<uint8_t*>(work);
    std::vector<uint32_t> open(n);
    for (uint32_t p = 0; p < n; ++p)
        open[p] = p;
    std::vector<ChainDesc> descs;
    std::vector<uint32_t> order, equal;
    for (uint64_t T = T0; T <= T_max && !open.empty(); T *= 2) {
        const uint32_t R = (uint32_t)open.size();
        descs.assign(2 * (size_t)R, proto);
        order.resize(2 * (size_t)R);
        for (uint32_t i = 0; i < R; ++i) {
            const uint32_t p = open[i];
            for (uint32_t b = 0; b < 2; ++b) {   // b = 0: top chain, 1: bottom chain
                ChainDesc& d = descs[2 * i + b];
                d.stream = stream0 + p;
                d.sig_offset = (4 * (uint64_t)p + 2 * b) * nb;
                d.tau_offset = d.sig_offset + nb;
                order[2 * i + b] = 2 * i + b;
            }
        }
        e = hipMemcpyAsync(sc.descs, descs.data(), sizeof(ChainDesc) * descs.size(), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(sc.order, order.data(), sizeof(uint32_t) * order.size(), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(sc.pairs, open.data(), sizeof(uint32_t) * R, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = launch_pw_reset(lat, sc.pairs, R, words, st);
        if (e == hipSuccess) e = launch_zero_u32(sc.counter, 1, st);
        if (e == hipSuccess) {
            BatchArgs a;
            std::memset(&a, 0, sizeof a);
            a.chains = sc.descs;
            a.order = sc.order;
            a.n_chains = 2 * R;
            a.counter = sc.counter;
            a.lattices = lat;
            a.key0 = (uint32_t)(seed & 0xFFFFFFFFu);
            a.key1 = (uint32_t)(seed >> 32);
            a.step0 = (uint32_t)(step_end - T);
            a.k_steps = (uint32_t)T;
            a.obs_every = 1;
            a.max_words = words;
            a.bits = L % 64 != 0 ? 1u : 0u;
            a.paired = proto.paired;
            const uint32_t blocks =
                std::max<uint32_t>(1, std::min<uint64_t>(2 * (uint64_t)R, (uint64_t)per_cu * (uint64_t)n_cu));
            e = launch_batch_chains(a, blocks, threads, st);
        }
        if (e == hipSuccess)
            e = launch_pw_finish(lat, sc.pairs, R, words, static_cast<uint8_t*>(samples), sc.equal, st);
        equal.resize(R);
        if (e == hipSuccess)
            e = hipMemcpyAsync(equal.data(), sc.equal, sizeof(uint32_t) * R, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess)
            return hip_fail(e, "sd_propp_wilson");
        std::vector<uint32_t> still;
        for (uint32_t i = 0; i < R; ++i) {
            if (equal[i])
                T_used[open[i]] = (int64_t)T;
            else
                still.push_back(open[i]);
        }
        open.swap(still);
    }
    return SD_OK;
}

}  // extern "C"
