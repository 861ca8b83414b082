// Batched shaken dynamics: many independent chains, each with its own (J, q),
// lattice size L and stream id, in one persistent launch.
//
// The paper's parameter scan runs one chain per CPU thread (section 4, the
// Julia implementation with 80 threads over (q, J) pairs).  Here one workgroup
// owns one chain at a time with both packed lattices resident in LDS: it pops a
// chain index from a global work queue (chains are ordered longest first on the
// host), loads sigma, runs all steps with barriers between half-steps, records
// (M, A, B) of every obs_every-th step into the chain's trace, writes sigma and
// tau back and pops the next chain.  HBM is touched only for the initial and
// final lattices and the traces.
//
// Undecided sites (top byte of the uniform equal to the threshold's, about one
// site in 256) are appended to an LDS list during the half-step, the decided
// bits are written straight to the LDS lattice, and after one barrier the list
// is resolved by the whole workgroup with LDS atomic ORs into the lattice.  A
// lane whose entries would overflow the list resolves them itself before the
// barrier.
#include "sd_batch.hpp"

namespace sd {

namespace {

struct HalfCtx {
    const uint64_t* src;
    uint64_t* dst;
    uint32_t L, W, n_words;
    FastDiv divW;
};

template <int WHICH>
__device__ __forceinline__ void gather_lds(const HalfCtx& h, uint32_t g, uint64_t& c, uint64_t& n1, uint64_t& n2) {
    const uint32_t j = fdiv(g, h.divW);
    const uint32_t w = g - j * h.W;
    const uint32_t row = j * h.W;
    c = h.src[g];
    if constexpr (WHICH == 0) {
        n1 = h.src[(j == 0 ? h.L - 1 : j - 1) * h.W + w];
        const uint64_t prev = h.src[row + (w == 0 ? h.W - 1 : w - 1)];
        n2 = (c << 1) | (prev >> 63);
    } else {
        n1 = h.src[(j == h.L - 1 ? 0 : j + 1) * h.W + w];
        const uint64_t next = h.src[row + (w == h.W - 1 ? 0 : w + 1)];
        n2 = (c >> 1) | (next << 63);
    }
}

struct TailList {
    uint32_t* site;
    uint32_t cap;
    uint32_t* count;   // two counters, used alternately by consecutive half-steps
    const uint32_t* T; // the chain's thresholds, in LDS
};

// Exclusive prefix sum of v across the wavefront and the wavefront total.
__device__ __forceinline__ uint32_t wave_exclusive_sum(uint32_t v, uint32_t& total) {
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t incl = v;
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(incl, d, 64);
        if (lane >= d)
            incl += t;
    }
    total = __shfl(incl, 63, 64);
    return incl - v;
}

constexpr uint32_t kBatchWords = 4;   // words per thread between two slot reservations

// One half-step of the workgroup's chain, src -> dst in LDS.  Each thread
// handles its words kBatchWords at a time: draws and compares them, writes the
// decided bits to dst and keeps the undecided masks; then the batch's
// undecided sites get list slots (one LDS atomic per wavefront).  After a
// barrier the list is resolved by the whole workgroup (the class of an entry
// is read back from src) and decisions are or-ed into dst.
template <int WHICH, bool PAIRED, bool COMPLEMENT>
__device__ __forceinline__ void lds_half_step(const HalfCtx& h, const DrawParams& dp, const PlaneMasks& pm,
                                              TailList& tl, uint32_t parity) {
    uint32_t* cnt = tl.count + parity;
    const uint32_t span = kBatchWords * blockDim.x;
    for (uint32_t base = 0; base < h.n_words; base += span) {
        uint64_t und[kBatchWords];
        uint32_t chain = 0;
#pragma unroll
        for (uint32_t k = 0; k < kBatchWords; ++k) {
            uint32_t g = base + threadIdx.x + k * blockDim.x;
            // one word at a time (see k_half_step): g depends on the previous word
            asm volatile("" : "+v"(g) : "v"(chain));
            und[k] = 0;
            if (g < h.n_words) {
                uint64_t c, n1, n2;
                gather_lds<WHICH>(h, g, c, n1, n2);
                uint64_t P[8];
                draw_planes(dp, g, P);
                const WordDraw wd = compare_planes<PAIRED, COMPLEMENT>(P, c, n1, n2, pm);
                h.dst[g] = wd.lt;
                und[k] = wd.und;
                chain = (uint32_t)wd.lt;
            }
        }
        uint32_t n = 0;
#pragma unroll
        for (uint32_t k = 0; k < kBatchWords; ++k)
            n += (uint32_t)__popcll(und[k]);
        uint32_t wave_total = 0;
        const uint32_t offset = wave_exclusive_sum(n, wave_total);
        uint32_t first = 0;
        if ((threadIdx.x & 63u) == 63u && wave_total)
            first = atomicAdd(cnt, wave_total);
        first = __shfl(first, 63, 64);
        if (n) {
            uint32_t slot = first + offset;
#pragma unroll
            for (uint32_t k = 0; k < kBatchWords; ++k) {
                const uint32_t g = base + threadIdx.x + k * blockDim.x;
                uint64_t u = und[k];
                while (u) {
                    const int b = __ffsll((unsigned long long)u) - 1;
                    u &= u - 1;
                    if (slot < tl.cap) {
                        tl.site[slot] = 64u * g + (uint32_t)b;
                    } else {
                        uint64_t c, n1, n2;
                        gather_lds<WHICH>(h, g, c, n1, n2);
                        if (decide_tail_thr(dp, 64u * g + (uint32_t)b, tl.T[class_at(c, n1, n2, b)]))
                            h.dst[g] |= 1ull << b;   // only this thread writes word g before the barrier
                    }
                    ++slot;
                }
            }
        }
    }
    __syncthreads();
    const uint32_t total = *cnt < tl.cap ? *cnt : tl.cap;
    for (uint32_t e = threadIdx.x; e < total; e += blockDim.x) {
        const uint32_t s = tl.site[e];
        const uint32_t g = s >> 6, b = s & 63u;
        uint64_t c, n1, n2;
        gather_lds<WHICH>(h, g, c, n1, n2);
        if (decide_tail_thr(dp, s, tl.T[class_at(c, n1, n2, (int)b)]))
            atomicOr(reinterpret_cast<unsigned long long*>(h.dst + g), 1ull << b);
    }
    if (threadIdx.x == 0)
        tl.count[parity ^ 1u] = 0;
    __syncthreads();
}

__device__ __forceinline__ void lds_observe(const uint64_t* sig, const uint64_t* tau, const HalfCtx& h,
                                            int64_t* out3, int64_t* red) {
    int64_t pc = 0, dpair = 0, dself = 0;
    for (uint32_t g = threadIdx.x; g < h.n_words; g += blockDim.x) {
        const uint32_t j = fdiv(g, h.divW);
        const uint32_t w = g - j * h.W;
        const uint64_t s = sig[g], t = tau[g];
        const uint64_t up = tau[(j == h.L - 1 ? 0 : j + 1) * h.W + w];
        const uint64_t next = tau[j * h.W + (w == h.W - 1 ? 0 : w + 1)];
        const uint64_t right = (t >> 1) | (next << 63);
        pc += __popcll(s);
        dpair += __popcll(s ^ up) + __popcll(s ^ right);
        dself += __popcll(s ^ t);
    }
    int64_t v[3] = {pc, dpair, dself};
    block_sum_i64<3>(v, red);
    if (threadIdx.x == 0) {
        const int64_t n = (int64_t)h.n_words * 64;
        out3[0] = 2 * v[0] - n;
        out3[1] = 2 * n - 2 * v[1];
        out3[2] = n - 2 * v[2];
    }
}

__device__ __forceinline__ uint32_t lds_bytes_to_bits4(uint32_t x) {
    uint32_t y = (~x >> 7) & 0x01010101u;
    return (y * 0x10204080u) >> 28;
}

__device__ __forceinline__ uint32_t lds_bits4_to_bytes(uint32_t n) {
    uint32_t z = (n * 0x00204081u) & 0x01010101u;
    uint32_t w = z ^ 0x01010101u;
    return z | ((w << 8) - w);
}

template <bool PAIRED, bool COMPLEMENT>
__device__ __forceinline__ void run_steps(const BatchArgs& a, const HalfCtx& hA, const HalfCtx& hB, DrawParams dp,
                                          TailList& tl, int64_t* trace, int64_t* red) {
    const PlaneMasks pm = make_plane_masks<PAIRED>(dp);
    uint32_t parity = 0;
    for (uint32_t m = 0; m < a.k_steps; ++m) {
        const uint32_t n = a.step0 + m;
        dp.t = 2u * n;
        lds_half_step<0, PAIRED, COMPLEMENT>(hA, dp, pm, tl, parity);
        parity ^= 1u;
        dp.t = 2u * n + 1u;
        lds_half_step<1, PAIRED, COMPLEMENT>(hB, dp, pm, tl, parity);
        parity ^= 1u;
        if (trace && (m + 1) % a.obs_every == 0)
            lds_observe(hB.dst, hA.dst, hA, trace + 3u * (size_t)((m + 1) / a.obs_every - 1), red);
    }
}

template <bool COMPLEMENT>
__global__ __launch_bounds__(512) void k_batch_chains(BatchArgs a) {
    extern __shared__ uint64_t smem[];
    __shared__ uint32_t s_chain;
    __shared__ uint32_t s_count[2];
    __shared__ uint32_t s_T[6];
    __shared__ int64_t red[3 * 8];
    uint64_t* sig = smem;
    uint64_t* tau = smem + a.max_words;
    TailList tl;
    tl.site = reinterpret_cast<uint32_t*>(tau + a.max_words);
    tl.cap = a.tail_cap;
    tl.count = s_count;
    tl.T = s_T;

    for (uint32_t iter = 0;; ++iter) {
        ChainDesc cd;
        if (a.counter) {
            if (threadIdx.x == 0)
                s_chain = atomicAdd(a.counter, 1u);
            __syncthreads();
            const uint32_t qi = s_chain;
            if (qi >= a.n_chains)
                break;
            cd = a.chains[a.order[qi]];
        } else {
            if (iter > 0 || blockIdx.x != 0)
                break;
            cd = a.single;
        }
        HalfCtx hA, hB;
        hA.L = hB.L = cd.L;
        hA.W = hB.W = cd.L / 64u;
        hA.n_words = hB.n_words = cd.L * (cd.L / 64u);
        hA.divW = hB.divW = cd.divW;
        hA.src = sig; hA.dst = tau;
        hB.src = tau; hB.dst = sig;
        const uint32_t n_words = hA.n_words;

        // load sigma (packed words, or int8 bytes converted to bits)
        if (a.int8_io) {
            const int8_t* src8 = reinterpret_cast<const int8_t*>(a.counter ? a.lattices + cd.sig_offset : a.single_sig);
            for (uint32_t g = threadIdx.x; g < n_words; g += blockDim.x) {
                const uint4* v = reinterpret_cast<const uint4*>(src8 + (size_t)64u * g);
                uint64_t bits = 0;
#pragma unroll
                for (int qd = 0; qd < 4; ++qd) {
                    uint4 x = v[qd];
                    uint32_t b16 = lds_bytes_to_bits4(x.x) | (lds_bytes_to_bits4(x.y) << 4) |
                                   (lds_bytes_to_bits4(x.z) << 8) | (lds_bytes_to_bits4(x.w) << 12);
                    bits |= (uint64_t)b16 << (16 * qd);
                }
                sig[g] = bits;
            }
        } else {
            const uint64_t* src = reinterpret_cast<const uint64_t*>(a.counter ? a.lattices + cd.sig_offset : a.single_sig);
            for (uint32_t g = threadIdx.x; g < n_words; g += blockDim.x)
                sig[g] = src[g];
        }
        if (threadIdx.x == 0) {
            s_count[0] = 0;
            s_count[1] = 0;
        }
        if (threadIdx.x == 0) {
#pragma unroll
            for (int i = 0; i < 6; ++i)
                s_T[i] = cd.T[i];
        }
        __syncthreads();

        DrawParams dp;
#pragma unroll
        for (int i = 0; i < 6; ++i)
            dp.T[i] = cd.T[i];
        dp.key0 = a.key0;
        dp.key1 = a.key1;
        dp.stream = cd.stream;
        dp.tag2 = 0;
        dp.rng_xor = COMPLEMENT ? 0xFFFFFFFFu : 0u;
        int64_t* trace = a.traces ? a.traces + cd.trace_offset : nullptr;

        if (cd.paired)
            run_steps<true, COMPLEMENT>(a, hA, hB, dp, tl, trace, red);
        else
            run_steps<false, COMPLEMENT>(a, hA, hB, dp, tl, trace, red);

        // write sigma and tau back
        if (a.int8_io) {
            int8_t* dst8 = reinterpret_cast<int8_t*>(a.counter ? a.lattices + cd.sig_offset : a.single_sig);
            int8_t* dst8t = reinterpret_cast<int8_t*>(a.counter ? a.lattices + cd.tau_offset : a.single_tau);
            for (uint32_t g = threadIdx.x; g < (a.k_steps ? 2u : 1u) * n_words; g += blockDim.x) {
                const bool is_tau = g >= n_words;
                const uint32_t gg = is_tau ? g - n_words : g;
                const uint64_t bits = is_tau ? tau[gg] : sig[gg];
                uint4* v = reinterpret_cast<uint4*>((is_tau ? dst8t : dst8) + (size_t)64u * gg);
#pragma unroll
                for (int qd = 0; qd < 4; ++qd) {
                    uint32_t b16 = (uint32_t)(bits >> (16 * qd)) & 0xFFFFu;
                    uint4 x;
                    x.x = lds_bits4_to_bytes(b16 & 0xF);
                    x.y = lds_bits4_to_bytes((b16 >> 4) & 0xF);
                    x.z = lds_bits4_to_bytes((b16 >> 8) & 0xF);
                    x.w = lds_bits4_to_bytes((b16 >> 12) & 0xF);
                    v[qd] = x;
                }
            }
        } else {
            uint64_t* dsig = reinterpret_cast<uint64_t*>(a.counter ? a.lattices + cd.sig_offset : a.single_sig);
            uint64_t* dtau = reinterpret_cast<uint64_t*>(a.counter ? a.lattices + cd.tau_offset : a.single_tau);
            for (uint32_t g = threadIdx.x; g < n_words; g += blockDim.x) {
                dsig[g] = sig[g];
                if (a.k_steps)
                    dtau[g] = tau[g];
            }
        }
        __syncthreads();
    }
}

__global__ void k_zero_u32(uint32_t* p, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = 0;
}

}  // namespace

size_t batch_lds_bytes(uint32_t max_words, uint32_t tail_cap) {
    return (size_t)2 * max_words * sizeof(uint64_t) + (size_t)tail_cap * sizeof(uint32_t);
}

hipError_t launch_batch_chains(const BatchArgs& a, uint32_t blocks, uint32_t threads, hipStream_t st) {
    const size_t lds = batch_lds_bytes(a.max_words, a.tail_cap);
    if (a.rng_xor)
        hipLaunchKernelGGL(k_batch_chains<true>, dim3(blocks), dim3(threads), lds, st, a);
    else
        hipLaunchKernelGGL(k_batch_chains<false>, dim3(blocks), dim3(threads), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* p, uint32_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, p, n);
    return hipGetLastError();
}

hipError_t batch_kernel_attributes(size_t max_dynamic_lds) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_chains<false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_dynamic_lds);
    if (e != hipSuccess)
        return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_chains<true>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_dynamic_lds);
}

hipError_t batch_occupancy(uint32_t threads, size_t lds, int* blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batch_chains<false>, (int)threads, lds);
}

}  // namespace sd
