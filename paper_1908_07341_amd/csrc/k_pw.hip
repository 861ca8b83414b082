// Coupling from the past (Propp-Wilson) on the monotone coupling of section
// 3.2: the pair bookkeeping around the batched chain kernel.  Each pair of
// chains (started from all +1 and all -1, sharing a stream) owns four
// consecutive lattices of its work slot: top sigma, top tau, bottom sigma,
// bottom tau.  One workgroup per listed pair.
#include "sd_batch.hpp"

namespace sd {

namespace {

__global__ __launch_bounds__(256) void k_pw_reset(uint64_t* __restrict__ work, const uint32_t* __restrict__ pairs,
                                                  uint32_t words) {
    uint64_t* slot = work + (size_t)4 * words * pairs[blockIdx.x];
    for (uint32_t g = threadIdx.x; g < words; g += blockDim.x) {
        slot[g] = ~0ull;              // top sigma: all +1
        slot[2u * words + g] = 0ull;  // bottom sigma: all -1
    }
}

__global__ __launch_bounds__(256) void k_pw_finish(const uint64_t* __restrict__ work,
                                                   const uint32_t* __restrict__ pairs, uint32_t words,
                                                   uint64_t* __restrict__ samples, uint32_t* __restrict__ equal) {
    const uint32_t p = pairs[blockIdx.x];
    const uint64_t* slot = work + (size_t)4 * words * p;
    uint64_t* out = samples + (size_t)words * p;
    uint64_t diff = 0;
    for (uint32_t g = threadIdx.x; g < words; g += blockDim.x) {
        const uint64_t top = slot[g];
        diff |= top ^ slot[2u * words + g];
        out[g] = top;
    }
    const int any = __syncthreads_or(diff != 0 ? 1 : 0);
    if (threadIdx.x == 0)
        equal[blockIdx.x] = any ? 0u : 1u;
}

uint32_t pw_threads(uint32_t words) { return words <= 64u ? 64u : words <= 128u ? 128u : 256u; }

}  // namespace

hipError_t launch_pw_reset(uint8_t* work, const uint32_t* pairs, uint32_t n, uint32_t words, hipStream_t st) {
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_pw_reset, dim3(n), dim3(pw_threads(words)), 0, st, reinterpret_cast<uint64_t*>(work), pairs,
                       words);
    return hipGetLastError();
}

hipError_t launch_pw_finish(const uint8_t* work, const uint32_t* pairs, uint32_t n, uint32_t words, uint8_t* samples,
                            uint32_t* equal, hipStream_t st) {
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_pw_finish, dim3(n), dim3(pw_threads(words)), 0, st, reinterpret_cast<const uint64_t*>(work),
                       pairs, words, reinterpret_cast<uint64_t*>(samples), equal);
    return hipGetLastError();
}

}  // namespace sd
