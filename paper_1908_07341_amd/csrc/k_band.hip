// Whole steps of several chains of one size, several steps per launch
// (sd_run_many on lattices of a few thousand words).
//
// A full step of the shaken dynamics is half-step A (eq. (15): every tau_x
// from sigma at x, below and left) followed by half-step B (eq. (16): every
// sigma'_x from tau at x, above and right).  So sigma' on a row depends on
// tau on that row and the one above, and that tau on sigma on the same two
// rows and the one below: a step widens the dependence of a row by one row
// on each side, and n steps of rows [a, a + R) depend only on sigma on rows
// [a - n, a + R + n).  Workgroup (chain, band) loads those R + 2n rows into
// LDS and runs the n steps there, each half-step on the rows whose
// dependence is still inside the loaded ones (one row fewer at the bottom
// after each half-step A and at the top after each half-step B); the rows
// outside [a, a + R) are drawn by the neighbouring bands too, from the same
// counter-based uniforms of the same sites, so they get the same bits.  The
// last sigma of the band's own rows goes to the other lattice of the pair
// (every band reads the previous sigma while others write theirs), so the
// launches alternate the two lattices of each chain, and nothing but sigma
// crosses global memory.  tau itself is not written: the caller runs the last
// step (or two) with the half-step kernels, which leave tau in place.
//
// Within each half-step a wavefront takes 64-word tiles (one word per lane);
// words with undecided sites are listed through a ballot and resolved by the
// wavefront at the end of the half-step (one tail draw per undecided site),
// the resolver or-ing the decided bits into the LDS word.  On recorded steps
// half-step B also counts M, A, B of the band's own rows: the owner counts
// its decided sites, the resolver the rest.
#include "sd_kernels.hpp"


namespace sd {

namespace {

constexpr uint32_t kBandWaves = kBandMaxThreads / 64;
constexpr uint32_t kBandListCap = 128;   // sites listed by a wavefront before it resolves them

struct BandShared {
    uint64_t sig[kBandMaxRowsWords];         // sigma, rows a - n .. a + R + n - 1
    uint64_t tau[kBandMaxRowsWords];         // tau, the same rows
    uint32_t site[kBandWaves][kBandListCap]; // undecided sites of each wavefront: 64 * LDS word + bit
    unsigned long long obs[3];               // a recorded step's sums, added by every wavefront
    uint32_t T24[6];
};

// A thread's counts of one half-step (at most 2 per site of a band of at
// most 1280 words): 32 bits hold them.
struct BandSums {
    uint32_t pc = 0, dpair = 0, dself = 0;
};

__device__ __forceinline__ void band_sync_wave() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Partner and neighbour words of LDS word u = i * W + w (row i, word w) of a
// half-step (both lattices use the same row numbering): A (WHICH 0) from
// sigma rows i (the site's own) and i - 1 (below); B (WHICH 1) from tau rows
// i and i + 1 (above).  The rows in LDS need no wrap-around; the words of a
// row do.
template <int WHICH>
__device__ __forceinline__ void band_gather(const uint64_t* src, uint32_t u, uint32_t w, uint32_t W, uint64_t& c,
                                            uint64_t& n1, uint64_t& n2) {
    c = src[u];
    if constexpr (WHICH == 0) {
        n1 = src[u - W];
        const uint32_t prev_hi = (uint32_t)(src[w == 0 ? u + W - 1u : u - 1u] >> 32);
        n2 = (uint64_t)__builtin_amdgcn_alignbit((uint32_t)c, prev_hi, 31) |
             ((uint64_t)__builtin_amdgcn_alignbit((uint32_t)(c >> 32), (uint32_t)c, 31) << 32);
    } else {
        n1 = src[u + W];
        const uint32_t next_lo = (uint32_t)src[w == W - 1u ? u + 1u - W : u + 1u];
        n2 = (uint64_t)__builtin_amdgcn_alignbit((uint32_t)(c >> 32), (uint32_t)c, 1) |
             ((uint64_t)__builtin_amdgcn_alignbit(next_lo, (uint32_t)(c >> 32), 1) << 32);
    }
}

// Decision of undecided site b of LDS word u of a half-step (tail uniform
// below the threshold's low 24 bits), with its word and neighbour words.
template <int WHICH>
__device__ __forceinline__ uint32_t band_tail(const uint64_t* src, uint32_t u, uint32_t b, uint32_t base, uint32_t L,
                                              uint32_t W, uint32_t shW, const DrawParams& dp,
                                              const uint32_t* T24, uint32_t& i, uint64_t& c, uint64_t& n1,
                                              uint64_t& n2) {
    i = u >> shW;
    const uint32_t w = u & (W - 1u);
    band_gather<WHICH>(src, u, w, W, c, n1, n2);
    uint32_t row = base + i;
    row = row >= L ? row - L : row;
    row = row >= L ? row - L : row;
    return draw_tail24(dp, 64u * ((row << shW) + w) + b) < T24[class_at(c, n1, n2, (int)b)] ? 1u : 0u;
}

template <bool OBS>
__device__ __forceinline__ void band_count_site(uint32_t bit, uint64_t c, uint64_t n1, uint64_t n2, uint32_t b,
                                                BandSums& acc) {
    if constexpr (OBS) {
        acc.pc += bit;
        acc.dpair += (bit ^ (uint32_t)((n1 >> b) & 1u)) + (bit ^ (uint32_t)((n2 >> b) & 1u));
        acc.dself += bit ^ (uint32_t)((c >> b) & 1u);
    }
}

// Resolve the first k sites of a wavefront's list, one per lane, or-ing the
// decided bits into dst (several sites may share a word).
template <int WHICH, bool OBS>
__device__ __forceinline__ void band_resolve(const uint64_t* src, uint64_t* dst, const uint32_t* list, uint32_t k,
                                             uint32_t o0, uint32_t o1, uint32_t base, uint32_t L, uint32_t W,
                                             uint32_t shW, const DrawParams& dp, const uint32_t* T24,
                                             BandSums& acc) {
    band_sync_wave();
    for (uint32_t e = threadIdx.x & 63u; e < k; e += 64u) {
        const uint32_t v = list[e];
        const uint32_t u = v >> 6, b = v & 63u;
        uint32_t i;
        uint64_t c, n1, n2;
        const uint32_t bit = band_tail<WHICH>(src, u, b, base, L, W, shW, dp, T24, i, c, n1, n2);
        if (bit)
            atomicOr(reinterpret_cast<unsigned long long*>(&dst[u]), 1ull << b);
        if (OBS && i >= o0 && i < o1)
            band_count_site<OBS>(bit, c, n1, n2, b, acc);
    }
    band_sync_wave();
}

// One half-step of the band on LDS rows [r0, r1) of dst, from src (both LDS,
// the same row numbering; B writes sigma in place, which it does not read).
// LDS row i is lattice row (base + i) mod L, so its word w is stream group
// ((base + i) mod L) * W + w.  OBS: count the new pair on rows [o0, o1).
// Must be called by every thread of the workgroup; ends with a barrier, after
// which dst holds the half-step's result.
//
// Wavefronts take 64-word tiles (one word per lane) and write the decided
// bits; each wavefront lists its undecided sites (one per lane and round of
// ballots) and resolves them one site per lane whenever 64 are listed and at
// the end.
template <int WHICH, bool PAIRED, bool COMPLEMENT, bool OBS>
__device__ __forceinline__ void band_half(const uint64_t* src, uint64_t* dst, uint32_t r0, uint32_t r1, uint32_t o0,
                                          uint32_t o1, uint32_t base, uint32_t L, uint32_t W, uint32_t shW,
                                          const DrawParams& dp, const PlaneMasks& pm, BandShared& sh,
                                          BandSums& acc) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t n_waves = blockDim.x >> 6;
    const uint32_t n_out = (r1 - r0) * W;
    const uint32_t n_tiles = (n_out + 63u) / 64u;
    uint32_t* list = sh.site[wave];
    uint32_t listed = 0;
    for (uint32_t tile = wave; tile < n_tiles; tile += n_waves) {
        const uint32_t uo = 64u * tile + lane;
        const bool active = uo < n_out;
        const uint32_t i = r0 + (uo >> shW);
        const uint32_t w = uo & (W - 1u);
        const uint32_t u = (r0 << shW) + uo;
        uint64_t c = 0, n1 = 0, n2 = 0;
        if (active)
            band_gather<WHICH>(src, u, w, W, c, n1, n2);
        uint32_t row = base + i;
        row = row >= L ? row - L : row;
        row = row >= L ? row - L : row;
        uint64_t P[8];
        draw_planes(dp, active ? (row << shW) + w : 0u, P);
        const WordDraw wd = compare_planes<PAIRED, COMPLEMENT>(P, c, n1, n2, pm);
        uint64_t und = active ? wd.und : 0ull;
        if (active) {
            dst[u] = wd.lt;
            if (OBS && i >= o0 && i < o1) {
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
                list[e] = 64u * u + (uint32_t)__builtin_ctzll(und);
                und &= und - 1;
            }
            listed += (uint32_t)__popcll(m);
            if (listed >= 64u) {
                band_resolve<WHICH, OBS>(src, dst, list, listed, o0, o1, base, L, W, shW, dp, sh.T24, acc);
                listed = 0;
            }
        }
    }
    if (listed)
        band_resolve<WHICH, OBS>(src, dst, list, listed, o0, o1, base, L, W, shW, dp, sh.T24, acc);
    if constexpr (OBS) {
        const uint32_t v[3] = {wave_sum_dpp(acc.pc), wave_sum_dpp(acc.dpair), wave_sum_dpp(acc.dself)};
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 3; ++k)
                atomicAdd(&sh.obs[k], (unsigned long long)v[k]);
        }
    }
    __syncthreads();
}

// ba.steps whole steps of band (chain, band) from step index ba.t0 / 2.
// INT8: lattices in global memory are int8 (16-byte aligned rows), else
// 64-bit words.  OBS: for every step s (from 0) with bit s of ba.rec_mask, the
// workgroup's (#+1, #differences to up + right, #to the partner, #sites) of
// its own rows go to partials + k * ba.rec_stride + 4 * blockIdx.x, k the
// number of recorded steps before s in this launch.
template <bool INT8, bool PAIRED, bool COMPLEMENT, bool OBS>
__global__ __launch_bounds__(kBandMaxThreads) void k_band_step(BandArgs ba, int64_t* __restrict__ partials) {
    __shared__ BandShared sh;
    const uint32_t chain = blockIdx.x / ba.bands;
    const uint32_t band = blockIdx.x - chain * ba.bands;
    const uint32_t L = ba.L, W = ba.W, R = ba.R, n = ba.steps;
    const uint32_t a = band * R;
    const uint32_t H = R + 2u * n;                        // LDS rows: lattice rows a - n .. a + R + n - 1
    const uint32_t base = a + (n / L + 1u) * L - n;       // lattice row of LDS row 0, plus a multiple of L
    const uint32_t base_mod = base % L;
    for (uint32_t q = threadIdx.x; q < H * W; q += blockDim.x) {
        const uint32_t i = q >> ba.shW;
        const uint32_t w = q & (W - 1u);
        const uint32_t row = (base_mod + i) % L;
        if constexpr (INT8)
            sh.sig[q] = load_bits64_i8(static_cast<const int8_t*>(ba.src[chain]) + (size_t)row * L + 64u * w);
        else
            sh.sig[q] = static_cast<const uint64_t*>(ba.src[chain])[(size_t)row * W + w];
    }
    if (threadIdx.x < 6)
        sh.T24[threadIdx.x] = PAIRED ? paired_tail(ba.T[chain], threadIdx.x) : ba.T[chain][threadIdx.x] & 0xFFFFFFu;
    if (threadIdx.x < 3)
        sh.obs[threadIdx.x] = 0;
    __syncthreads();
    DrawParams dp;
#pragma unroll
    for (int i = 0; i < 6; ++i)
        dp.T[i] = ba.T[chain][i];
    dp.key0 = ba.key0;
    dp.key1 = ba.key1;
    dp.stream = ba.stream[chain];
    dp.tag2 = 2u * kTagDynamics;
    dp.rng_xor = COMPLEMENT ? 0xFFFFFFFFu : 0u;
    const PlaneMasks pm = make_plane_masks<PAIRED>(dp);
    uint32_t rec = 0;
    for (uint32_t s = 1; s <= n; ++s) {
        BandSums acc;
        dp.t = ba.t0 + 2u * (s - 1u);
        // tau on rows s .. H - s (its sigma rows below are valid from s - 1)
        band_half<0, PAIRED, COMPLEMENT, false>(sh.sig, sh.tau, s, H - s + 1u, 0, 0, base_mod, L, W, ba.shW, dp,
                                                pm, sh, acc);
        dp.t += 1u;
        const bool recorded = OBS && ((ba.rec_mask >> (s - 1u)) & 1u);
        if (recorded) {
            band_half<1, PAIRED, COMPLEMENT, true>(sh.tau, sh.sig, s, H - s, n, n + R, base_mod, L, W, ba.shW, dp,
                                                   pm, sh, acc);
        } else {
            band_half<1, PAIRED, COMPLEMENT, false>(sh.tau, sh.sig, s, H - s, 0, 0, base_mod, L, W, ba.shW, dp, pm,
                                                    sh, acc);
        }
        if constexpr (OBS) {
            // every wavefront has added its sums before the half-step's
            // barrier; the next recorded half-step adds again only after
            // the next half-step A's barrier, so the reset cannot race
            if (recorded) {
                if (threadIdx.x == 0) {
                    int64_t* p = partials + (size_t)rec * ba.rec_stride + 4u * (size_t)blockIdx.x;
                    p[0] = (int64_t)sh.obs[0];
                    p[1] = (int64_t)sh.obs[1];
                    p[2] = (int64_t)sh.obs[2];
                    p[3] = (int64_t)R * L;
                    sh.obs[0] = sh.obs[1] = sh.obs[2] = 0;
                }
                ++rec;
            }
        }
    }
    // the band's own rows (LDS rows n .. n + R - 1) to the other lattice
    const uint64_t* own = sh.sig + n * W;
    for (uint32_t u = threadIdx.x; u < R * W; u += blockDim.x) {
        if constexpr (INT8)
            store_bits64_i8(static_cast<int8_t*>(ba.dst[chain]) + (size_t)a * L + 64u * u, own[u]);
        else
            static_cast<uint64_t*>(ba.dst[chain])[(size_t)a * W + u] = own[u];
    }
}

template <bool INT8, bool OBS>
void launch_band_t(const BandArgs& ba, bool paired, bool complement, int64_t* partials, hipStream_t st) {
    const dim3 grid(ba.n_chains * ba.bands), block(ba.threads);
    if (paired && !complement)
        hipLaunchKernelGGL((k_band_step<INT8, true, false, OBS>), grid, block, 0, st, ba, partials);
    else if (paired)
        hipLaunchKernelGGL((k_band_step<INT8, true, true, OBS>), grid, block, 0, st, ba, partials);
    else if (!complement)
        hipLaunchKernelGGL((k_band_step<INT8, false, false, OBS>), grid, block, 0, st, ba, partials);
    else
        hipLaunchKernelGGL((k_band_step<INT8, false, true, OBS>), grid, block, 0, st, ba, partials);
}

}  // namespace

// Rows per band and steps per launch, measured on five chains with records
// every step: the small lattices leave most of the device idle, so they take
// narrow bands and many steps per launch (latency bound: the redundant halo
// rows cost nothing); the larger ones are issue bound, and the halo's share
// of the work, (2 steps - 1) / (2 R) of a step, decides.
uint32_t band_rows(int32_t L) {
    if (L < 64 || L % 64 != 0)
        return 0;
    const uint32_t W = (uint32_t)L / 64u;
    switch (W) {
        case 1:
        case 2:
        case 4:
            return 32u / W;   // half a tile of own words
        case 8:
            return 16u;       // two tiles
        case 16:
            return 16u;       // four tiles
        case 32:
            return 8u;
        case 64:
            return 4u;
        default:
            return 0;         // rows of more than 64 words, or not dividing 256
    }
}

uint32_t band_depth(int32_t L) {
    const uint32_t W = (uint32_t)L / 64u;
    return W <= 16u ? 8u : W == 32u ? 4u : 1u;
}

uint32_t band_threads(uint32_t R, uint32_t W, uint32_t steps) {
    // the widest half-step is the first A: rows 1 .. R + 2 steps - 1
    const uint32_t tiles = ((R + 2u * steps - 1u) * W + 63u) / 64u;
    const uint32_t t = 64u * tiles;
    return t < kBandMaxThreads ? t : kBandMaxThreads;
}

hipError_t launch_band_step(const BandArgs& ba, bool int8, bool paired, bool complement, int64_t* partials,
                            hipStream_t st) {
    if (int8) {
        if (partials)
            launch_band_t<true, true>(ba, paired, complement, partials, st);
        else
            launch_band_t<true, false>(ba, paired, complement, partials, st);
    } else {
        if (partials)
            launch_band_t<false, true>(ba, paired, complement, partials, st);
        else
            launch_band_t<false, false>(ba, paired, complement, partials, st);
    }
    return hipGetLastError();
}

}  // namespace sd
