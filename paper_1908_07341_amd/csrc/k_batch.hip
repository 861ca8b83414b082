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
// Within a half-step each wavefront takes 64-word tiles of the lattice in
// turn (one word per lane).  Decided bits go straight to the LDS lattice; the
// undecided sites (top byte of the uniform equal to the threshold's, about
// one site in 256) are listed in the wavefront's LDS list, one per lane and
// round of ballots.  Whenever 64 or more sites are listed, and once at the
// end of the half-step, the wavefront resolves its list (one site per lane:
// one tail draw each) and ors the decided bits into the lattice words with
// LDS atomics (several sites may share a word; no other wavefront touches
// it).  So a half-step needs a single workgroup barrier, before the next one
// reads the lattice.  On recorded steps half-step B also accumulates M, A, B:
// the owner counts the decided sites of its word, the resolver the rest.
#include "sd_batch.hpp"

namespace sd {

namespace {

// BITS: rows need not start on a word (L % 64 != 0, L % 8 == 0); neighbours
// are windows of the lattice's bit string.
template <bool BITS>
struct HalfCtx {
    const uint64_t* src;
    uint64_t* dst;
    uint32_t L, W, n_words;
    FastDiv divW;   // division by W = L / 64 (rows of whole words)
    FastDiv divL;   // division by L (bit strings)
};

// Rows of whole words: word g = j * W + w (row j, column word w) and its
// neighbours; every index is g plus or minus W or 1.
template <int WHICH, bool BITS>
__device__ __forceinline__ void gather_lds_g(const HalfCtx<BITS>& h, uint32_t g, uint32_t j, uint32_t w,
                                             uint64_t& c, uint64_t& n1, uint64_t& n2) {
    c = h.src[g];
    const uint32_t c_lo = (uint32_t)c, c_hi = (uint32_t)(c >> 32);
    if constexpr (WHICH == 0) {
        n1 = h.src[j == 0 ? g + h.n_words - h.W : g - h.W];
        const uint32_t prev_hi = (uint32_t)(h.src[w == 0 ? g + h.W - 1u : g - 1u] >> 32);
        n2 = (uint64_t)__builtin_amdgcn_alignbit(c_lo, prev_hi, 31) |
             ((uint64_t)__builtin_amdgcn_alignbit(c_hi, c_lo, 31) << 32);
    } else {
        n1 = h.src[j == h.L - 1 ? g + h.W - h.n_words : g + h.W];
        const uint32_t next_lo = (uint32_t)h.src[w == h.W - 1 ? g + 1u - h.W : g + 1u];
        n2 = (uint64_t)__builtin_amdgcn_alignbit(c_hi, c_lo, 1) |
             ((uint64_t)__builtin_amdgcn_alignbit(next_lo, c_hi, 1) << 32);
    }
}

template <int WHICH, bool BITS>
__device__ __forceinline__ void gather_lds(const HalfCtx<BITS>& h, uint32_t g, uint64_t& c, uint64_t& n1,
                                           uint64_t& n2) {
    if constexpr (BITS) {
        gather_bits<WHICH>(h.src, h.L, h.n_words, h.divL, g, c, n1, n2);
    } else {
        const uint32_t j = fdiv(g, h.divW);
        gather_lds_g<WHICH>(h, g, j, g - j * h.W, c, n1, n2);
    }
}

// Per-wavefront list of undecided sites (64 * word + bit).  A round of
// ballots adds at most 64 entries and the list is resolved as soon as it
// holds 64, so it never holds more than 127.
constexpr uint32_t kWListCap = 128;

struct WaveWordList {
    uint32_t site[kWListCap];
};

// The chain's per-launch constants in LDS.
struct ChainShared {
    uint32_t T24[6];   // tail thresholds of the classes (paired_tail in the paired form)
};

// A thread's counts of one half-step: at most 2 per site of the lattice
// (10240 words of 64 sites at most in LDS), so 32 bits hold them and every
// popcount adds in one instruction.
struct ObsSums {
    uint32_t pc = 0, dpair = 0, dself = 0;   // #+1, #differences to up+right, to the partner
};

// Resolves the first n sites of the wavefront's list into the lattice.
template <int WHICH, bool OBS, bool BITS>
__device__ __forceinline__ void resolve_list(const HalfCtx<BITS>& h, const DrawParams& dp, const uint32_t* T24,
                                             WaveWordList& wl, uint32_t n, ObsSums& acc) {
    for (uint32_t e = threadIdx.x & 63u; e < n; e += 64u) {
        const uint32_t v = wl.site[e];
        const uint32_t g = v >> 6, b = v & 63u;
        uint64_t c, n1, n2;
        gather_lds<WHICH>(h, g, c, n1, n2);
        const uint32_t bit = draw_tail24(dp, v) < T24[class_at(c, n1, n2, (int)b)] ? 1u : 0u;
        if (bit)
            atomicOr(reinterpret_cast<unsigned long long*>(&h.dst[g]), 1ull << b);
        if constexpr (OBS) {
            acc.pc += bit;
            acc.dpair += (bit ^ (uint32_t)((n1 >> b) & 1u)) + (bit ^ (uint32_t)((n2 >> b) & 1u));
            acc.dself += bit ^ (uint32_t)((c >> b) & 1u);
        }
    }
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Adds the wavefront's observable sums to obs_sum[0 .. 2] (LDS), one atomic
// per quantity.  A wavefront's counts of one half-step stay far below 2^32
// (at most 2 per site of the lattice).
__device__ __forceinline__ void add_wave_obs(const ObsSums& acc, unsigned long long* obs_sum) {
    const uint32_t v0 = wave_sum_dpp(acc.pc);
    const uint32_t v1 = wave_sum_dpp(acc.dpair);
    const uint32_t v2 = wave_sum_dpp(acc.dself);
    if ((threadIdx.x & 63u) == 0) {
        atomicAdd(&obs_sum[0], (unsigned long long)v0);
        atomicAdd(&obs_sum[1], (unsigned long long)v1);
        atomicAdd(&obs_sum[2], (unsigned long long)v2);
    }
}

// One half-step of the workgroup's chain, src -> dst in LDS, ending with a
// workgroup barrier.  OBS (half-step B of a recorded step): accumulate the
// observables of the new pair (dst, src) in acc and add the wavefront's sums
// to obs_sum[0 .. 2] (LDS) before the closing barrier.
template <int WHICH, bool PAIRED, bool COMPLEMENT, bool OBS, bool BITS>
__device__ __forceinline__ void lds_half_step(const HalfCtx<BITS>& h, const DrawParams& dp, const PlaneMasks& pm,
                                              const uint32_t* T24, WaveWordList& wl, ObsSums& acc,
                                              unsigned long long* obs_sum) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t n_waves = blockDim.x >> 6;
    const uint32_t n_tiles = (h.n_words + 63u) / 64u;
    uint32_t listed = 0;   // wavefront-uniform
    // rows of whole words: (row, column word) of the lane's word, stepped by
    // the 64 * n_waves words between a wavefront's tiles
    uint32_t j = 0, w = 0, step_rows = 0, step_cols = 0;
    if constexpr (!BITS) {
        const uint32_t g0 = 64u * (threadIdx.x >> 6) + lane;
        j = fdiv(g0, h.divW);
        w = g0 - j * h.W;
        const uint32_t step = 64u * n_waves;
        step_rows = step / h.W;
        step_cols = step - step_rows * h.W;
    }
    for (uint32_t tile = threadIdx.x >> 6; tile < n_tiles; tile += n_waves) {
        const uint32_t g = 64u * tile + lane;
        // rows of whole words hold L * L / 64 = 64 * L * (L / 64) words: every
        // tile is full
        const bool active = !BITS || g < h.n_words;
        uint64_t c = 0, n1 = 0, n2 = 0;
        if (active) {
            if constexpr (BITS)
                gather_lds<WHICH>(h, g, c, n1, n2);
            else
                gather_lds_g<WHICH>(h, g, j, w, c, n1, n2);
        }
        if constexpr (!BITS) {
            w += step_cols;
            j += step_rows;
            if (w >= h.W) {
                w -= h.W;
                ++j;
            }
        }
        uint64_t P[8];
        draw_planes(dp, active ? g : 0u, P);
        const WordDraw wd = compare_planes<PAIRED, COMPLEMENT>(P, c, n1, n2, pm);
        uint64_t und = active ? wd.und : 0ull;
        if (active) {
            h.dst[g] = wd.lt;
            if constexpr (OBS) {
                acc.pc += __popcll(wd.lt);
                acc.dpair += __popcll((wd.lt ^ n1) & ~und) + __popcll((wd.lt ^ n2) & ~und);
                acc.dself += __popcll((wd.lt ^ c) & ~und);
            }
        }
        for (;;) {
            const uint64_t m = __ballot(und != 0);
            if (m == 0)
                break;
            if (und != 0) {
                const uint32_t e = listed + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                wl.site[e] = 64u * g + (uint32_t)__builtin_ctzll(und);
                und &= und - 1;
            }
            listed += (uint32_t)__popcll(m);
            if (listed >= 64u) {
                wave_sync_lds();
                resolve_list<WHICH, OBS>(h, dp, T24, wl, listed, acc);
                wave_sync_lds();
                listed = 0;
            }
        }
    }
    if (listed) {
        wave_sync_lds();
        resolve_list<WHICH, OBS>(h, dp, T24, wl, listed, acc);
    }
    if constexpr (OBS)
        add_wave_obs(acc, obs_sum);
    __syncthreads();
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

// Observables of the pair (sig, tau) as sums over the workgroup's threads
// (a separate pass, used for chains with the general compare).
template <bool BITS>
__device__ __forceinline__ ObsSums lds_observe(const uint64_t* sig, const uint64_t* tau, const HalfCtx<BITS>& h) {
    ObsSums acc;
    if constexpr (BITS) {
        for (uint32_t g = threadIdx.x; g < h.n_words; g += blockDim.x) {
            uint64_t t, up, right;
            gather_bits<1>(tau, h.L, h.n_words, h.divL, g, t, up, right);
            const uint64_t sg = sig[g];
            acc.pc += __popcll(sg);
            acc.dpair += __popcll(sg ^ up) + __popcll(sg ^ right);
            acc.dself += __popcll(sg ^ t);
        }
        return acc;
    }
    for (uint32_t g = threadIdx.x; g < h.n_words; g += blockDim.x) {
        const uint32_t j = fdiv(g, h.divW);
        const uint32_t w = g - j * h.W;
        const uint64_t s = sig[g], t = tau[g];
        const uint64_t up = tau[(j == h.L - 1 ? 0 : j + 1) * h.W + w];
        const uint64_t next = tau[j * h.W + (w == h.W - 1 ? 0 : w + 1)];
        const uint64_t right = (t >> 1) | (next << 63);
        acc.pc += __popcll(s);
        acc.dpair += __popcll(s ^ up) + __popcll(s ^ right);
        acc.dself += __popcll(s ^ t);
    }
    return acc;
}

// Steps of one chain.  Paired chains fold the observables into half-step B;
// the general compare (rare: some field is exactly zero) leaves them to a
// separate pass so that its register count stays low.
// Copy of an LDS lattice to global memory (the workgroup's threads).
__device__ __forceinline__ void store_lattice(uint64_t* out, const uint64_t* lat, uint32_t n_words) {
    for (uint32_t g = threadIdx.x; g < n_words; g += blockDim.x)
        out[g] = lat[g];
}

// mom (used by thread 0 only): the chain's running sums in moments mode.
template <bool PAIRED, bool COMPLEMENT, bool BITS>
__device__ __forceinline__ void run_steps(const BatchArgs& a, const HalfCtx<BITS>& hA, const HalfCtx<BITS>& hB,
                                          DrawParams dp,
                                          const uint32_t* T24, WaveWordList& wl, int64_t* trace,
                                          unsigned long long* obs_sum, uint64_t* traj,
                                          int64_t (&mom)[kMomentWords]) {
    const PlaneMasks pm = make_plane_masks<PAIRED>(dp);
    for (uint32_t m = 0; m < a.k_steps; ++m) {
        const uint32_t n = a.step0 + m;
        ObsSums acc;
        dp.t = 2u * n;
        lds_half_step<0, PAIRED, COMPLEMENT, false>(hA, dp, pm, T24, wl, acc, obs_sum);
        // (each half-step ends with a barrier, so a copy made here is complete
        // before the lattice is next overwritten, two half-steps later)
        if (traj)
            store_lattice(traj + (size_t)(2u * m + 1u) * hA.n_words, hA.dst, hA.n_words);
        dp.t = 2u * n + 1u;
        if (trace && (m + 1) % a.obs_every == 0) {
            if constexpr (PAIRED) {
                lds_half_step<1, PAIRED, COMPLEMENT, true>(hB, dp, pm, T24, wl, acc, obs_sum);
            } else {
                lds_half_step<1, PAIRED, COMPLEMENT, false>(hB, dp, pm, T24, wl, acc, obs_sum);
                acc = lds_observe(hB.dst, hA.dst, hA);
                add_wave_obs(acc, obs_sum);
                __syncthreads();
            }
            // every wavefront added its sums before the last barrier; the
            // next recorded step adds again only after half-step A's barrier
            if (threadIdx.x == 0) {
                const int64_t v[3] = {(int64_t)obs_sum[0], (int64_t)obs_sum[1], (int64_t)obs_sum[2]};
                obs_sum[0] = obs_sum[1] = obs_sum[2] = 0;
                const int64_t sites = (int64_t)hA.n_words * 64;
                const int64_t M = 2 * v[0] - sites, A = 2 * sites - 2 * v[1], B = sites - 2 * v[2];
                if (a.moments) {
                    mom[0] += M;
                    mom[1] += M * M;
                    mom[2] += M < 0 ? -M : M;
                    mom[3] += A;
                    mom[4] += B;
                } else {
                    int64_t* out3 = trace + 3u * (size_t)((m + 1) / a.obs_every - 1);
                    out3[0] = M;
                    out3[1] = A;
                    out3[2] = B;
                }
            }
        } else {
            lds_half_step<1, PAIRED, COMPLEMENT, false>(hB, dp, pm, T24, wl, acc, obs_sum);
        }
        if (traj)
            store_lattice(traj + (size_t)(2u * m + 2u) * hB.n_words, hB.dst, hB.n_words);
    }
}

// PAIRED: every chain of the launch has a paired threshold table.  BITS: the
// chains' L are multiples of 8 but not of 64 (bit-string neighbours).
template <bool COMPLEMENT, bool PAIRED, bool BITS>
__device__ __forceinline__ void batch_chains_body(const BatchArgs& a) {
    extern __shared__ uint64_t smem[];
    __shared__ uint32_t s_chain;
    __shared__ uint32_t s_queue;   // the queue this workgroup takes chains from (0: its own)
    __shared__ ChainShared s_ch;
    __shared__ unsigned long long s_obs[3];   // a recorded step's sums, added by every wavefront
    uint64_t* sig = smem;
    uint64_t* tau = smem + a.max_words;
    WaveWordList& wl = reinterpret_cast<WaveWordList*>(tau + a.max_words)[threadIdx.x >> 6];

    if (threadIdx.x == 0) {
        s_queue = 0;
        s_obs[0] = s_obs[1] = s_obs[2] = 0;
        if (a.t_start)
            atomicMin(a.t_start, (unsigned long long)wall_clock64());
    }
    for (uint32_t iter = 0;; ++iter) {
        ChainDesc cd;
        if (a.counter) {
            // the next chain of this launch's queue, then of the later queues
            // in turn once it is empty (every queue is exhausted at most once
            // per workgroup: s_queue only moves forward)
            if (threadIdx.x == 0) {
                uint32_t chain = ~0u;
                while (s_queue <= a.n_steal) {
                    const uint32_t q = s_queue;
                    uint32_t* ctr = q == 0 ? a.counter : a.steal_counter[q - 1];
                    const uint32_t cnt = q == 0 ? a.n_chains : a.steal_count[q - 1];
                    const uint32_t i = atomicAdd(ctr, 1u);
                    if (i < cnt) {
                        chain = q == 0 ? a.order[i] : a.steal_order[q - 1][i];
                        break;
                    }
                    s_queue = q + 1;
                }
                s_chain = chain;
            }
            __syncthreads();
            // a workgroup-uniform index, so that the descriptor is read with
            // scalar loads into scalar registers
            const uint32_t ci = __builtin_amdgcn_readfirstlane(s_chain);
            if (ci == ~0u)
                break;
            cd = a.chains[ci];
        } else if (a.n_uniform) {
            if (iter > 0 || blockIdx.x >= a.n_uniform)
                break;
            cd = a.single;
            cd.stream += blockIdx.x;
        } else {
            if (iter > 0 || blockIdx.x != 0)
                break;
            cd = a.single;
        }
        // the chain's geometry is the same for the whole workgroup: keep it in
        // scalar registers
        auto uni = [](uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane(v); };
        auto uni_div = [&](const FastDiv& f) {
            FastDiv u;
            u.d = uni(f.d);
            u.mul = uni(f.mul);
            u.shift = uni(f.shift);
            u.add = uni(f.add);
            return u;
        };
        cd.L = uni(cd.L);
        cd.stream = uni(cd.stream);
        HalfCtx<BITS> hA, hB;
        hA.L = hB.L = cd.L;
        hA.W = hB.W = cd.L / 64u;
        hA.n_words = hB.n_words = (uint32_t)(((uint64_t)cd.L * cd.L) / 64u);
        hA.divW = hB.divW = uni_div(cd.divW);
        hA.divL = hB.divL = uni_div(cd.divL);
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
            const uint64_t* src =
                a.counter ? reinterpret_cast<const uint64_t*>(a.lattices + cd.sig_offset)
                          : reinterpret_cast<const uint64_t*>(a.single_sig) + (size_t)(a.n_uniform ? blockIdx.x : 0u) * n_words;
            for (uint32_t g = threadIdx.x; g < n_words; g += blockDim.x)
                sig[g] = src[g];
        }
        if (threadIdx.x == 0) {
#pragma unroll
            for (int i = 0; i < 6; ++i)
                s_ch.T24[i] = PAIRED ? paired_tail(cd.T, i) : cd.T[i] & 0xFFFFFFu;
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
        uint64_t* traj = a.traj ? reinterpret_cast<uint64_t*>(a.traj + (size_t)blockIdx.x * a.traj_chain_bytes) : nullptr;
        if (traj)
            store_lattice(traj, sig, n_words);

        int64_t mom[kMomentWords] = {0, 0, 0, 0, 0};
        run_steps<PAIRED, COMPLEMENT, BITS>(a, hA, hB, dp, s_ch.T24, wl, trace, s_obs, traj, mom);
        if (a.moments && trace && threadIdx.x == 0) {
#pragma unroll
            for (uint32_t i = 0; i < kMomentWords; ++i)
                trace[i] = mom[i];
        }
        if (traj) {
            __syncthreads();
            continue;
        }

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
    if (a.t_end && threadIdx.x == 0)
        atomicMax(a.t_end, (unsigned long long)wall_clock64());
}

// The paired compare (every threshold table by default) in workgroups of up
// to 640 threads held to 96 VGPRs, so that two workgroups of ten wavefronts
// share a CU with the largest (512^2) chains in LDS; the six-class compare
// keeps the compiler's register count and at most 512 threads.
template <bool COMPLEMENT, bool BITS>
__global__ __launch_bounds__(kBatchMaxThreads) __attribute__((amdgpu_waves_per_eu(5))) void k_batch_chains(
    BatchArgs a) {
    batch_chains_body<COMPLEMENT, true, BITS>(a);
}

template <bool COMPLEMENT, bool BITS>
__global__ __launch_bounds__(512) void k_batch_chains_general(BatchArgs a) {
    batch_chains_body<COMPLEMENT, false, BITS>(a);
}

__global__ void k_zero_u32(uint32_t* p, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = 0;
}

}  // namespace

size_t batch_lds_bytes(uint32_t max_words, uint32_t threads) {
    return (size_t)2 * max_words * sizeof(uint64_t) + (size_t)((threads + 63u) / 64u) * sizeof(WaveWordList);
}

template <bool BITS>
void launch_batch_chains_t(const BatchArgs& a, uint32_t blocks, uint32_t threads, size_t lds, hipStream_t st) {
    if (a.rng_xor && a.paired)
        hipLaunchKernelGGL((k_batch_chains<true, BITS>), dim3(blocks), dim3(threads), lds, st, a);
    else if (a.rng_xor)
        hipLaunchKernelGGL((k_batch_chains_general<true, BITS>), dim3(blocks), dim3(threads), lds, st, a);
    else if (a.paired)
        hipLaunchKernelGGL((k_batch_chains<false, BITS>), dim3(blocks), dim3(threads), lds, st, a);
    else
        hipLaunchKernelGGL((k_batch_chains_general<false, BITS>), dim3(blocks), dim3(threads), lds, st, a);
}

hipError_t launch_batch_chains(const BatchArgs& a, uint32_t blocks, uint32_t threads, hipStream_t st) {
    const size_t lds = batch_lds_bytes(a.max_words, threads);
    if (a.bits)
        launch_batch_chains_t<true>(a, blocks, threads, lds, st);
    else
        launch_batch_chains_t<false>(a, blocks, threads, lds, st);
    return hipGetLastError();
}

__global__ void k_times_reset(unsigned long long* starts, unsigned long long* ends, uint32_t n) {
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        starts[i] = ~0ull;
        ends[i] = 0ull;
    }
}

hipError_t launch_times_reset(unsigned long long* starts, unsigned long long* ends, uint32_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_times_reset, dim3(1), dim3(64), 0, st, starts, ends, n);
    return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* p, uint32_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, p, n);
    return hipGetLastError();
}

hipError_t batch_kernel_attributes(size_t max_dynamic_lds) {
    const void* kernels[8] = {reinterpret_cast<const void*>(&k_batch_chains_general<false, false>),
                              reinterpret_cast<const void*>(&k_batch_chains<false, false>),
                              reinterpret_cast<const void*>(&k_batch_chains_general<true, false>),
                              reinterpret_cast<const void*>(&k_batch_chains<true, false>),
                              reinterpret_cast<const void*>(&k_batch_chains_general<false, true>),
                              reinterpret_cast<const void*>(&k_batch_chains<false, true>),
                              reinterpret_cast<const void*>(&k_batch_chains_general<true, true>),
                              reinterpret_cast<const void*>(&k_batch_chains<true, true>)};
    for (const void* k : kernels) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_dynamic_lds);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t batch_occupancy(uint32_t threads, size_t lds, bool paired, bool bits, int* blocks_per_cu) {
    const void* k = bits ? (paired ? reinterpret_cast<const void*>(&k_batch_chains<false, true>)
                                   : reinterpret_cast<const void*>(&k_batch_chains_general<false, true>))
                         : (paired ? reinterpret_cast<const void*>(&k_batch_chains<false, false>)
                                   : reinterpret_cast<const void*>(&k_batch_chains_general<false, false>));
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, (int)threads, lds);
}

}  // namespace sd
