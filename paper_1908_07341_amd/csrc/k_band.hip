// Whole steps of several chains of one size in one launch each (sd_run_many
// on lattices of a few thousand words).
//
// A full step of the shaken dynamics is half-step A (eq. (15): every tau_x
// from sigma at x, below and left) followed by half-step B (eq. (16): every
// sigma'_x from tau at x, above and right).  So sigma' on rows [a, a + R)
// depends on tau on rows [a, a + R], and that tau on sigma on rows
// [a - 1, a + R]: a band of R rows can take a whole step from R + 2 rows of
// sigma with no other band's help.  Workgroup (chain, band) loads those rows
// into LDS, draws tau on its R rows and on the row above the band (the next
// band draws that row too, from the same counter-based uniforms, so both get
// the same bits), then sigma' on its R rows, and writes sigma' to the other
// buffer of the pair: every band reads the previous sigma while others write
// the new one, so the launch alternates the two lattices of each chain.  One
// launch per step instead of two, and nothing but sigma goes through global
// memory.  tau itself is not written: the caller runs the last step (or two)
// with the half-step kernels, which leave tau of the last step in place.
//
// Within each half-step a wavefront takes 64-word tiles (one word per lane);
// words with undecided sites are listed through a ballot and resolved by the
// wavefront at the end of the half-step (one tail draw per undecided site),
// the resolver or-ing the decided bits into the LDS word.  On recorded steps
// half-step B also counts M, A, B of the new pair: the owner counts its
// decided sites, the resolver the rest.
#include "sd_kernels.hpp"

namespace sd {

namespace {

constexpr uint32_t kBandWaves = 5;
constexpr uint32_t kBandListCap = 128;   // a half-step lists at most 64 words per tile before resolving

struct BandList {
    uint64_t und[kBandListCap];
    uint32_t u[kBandListCap];
};

struct BandShared {
    uint64_t sig[kBandMaxWords + 2 * 64];   // sigma rows a - 1 .. a + R
    uint64_t tau[kBandMaxWords + 64];       // tau rows a .. a + R
    uint64_t out[kBandMaxWords];            // sigma' rows a .. a + R - 1
    BandList list[kBandWaves];
    uint32_t T24[6];
};

struct BandSums {
    int64_t pc = 0, dpair = 0, dself = 0;
};

__device__ __forceinline__ void band_sync_wave() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Partner and neighbour words of output word u = t * W + w of a half-step:
// A (WHICH 0): tau row t from sigma rows t + 1 (the same lattice row) and t
// (the row below); B (WHICH 1): sigma' row t from tau rows t and t + 1 (above).
template <int WHICH>
__device__ __forceinline__ void band_gather(const uint64_t* src, uint32_t t, uint32_t w, uint32_t W, uint64_t& c,
                                            uint64_t& n1, uint64_t& n2) {
    if constexpr (WHICH == 0) {
        const uint64_t* row = src + (t + 1) * W;
        c = row[w];
        n1 = src[t * W + w];
        const uint32_t prev_hi = (uint32_t)(row[w == 0 ? W - 1 : w - 1] >> 32);
        n2 = (uint64_t)__builtin_amdgcn_alignbit((uint32_t)c, prev_hi, 31) |
             ((uint64_t)__builtin_amdgcn_alignbit((uint32_t)(c >> 32), (uint32_t)c, 31) << 32);
    } else {
        const uint64_t* row = src + t * W;
        c = row[w];
        n1 = src[(t + 1) * W + w];
        const uint32_t next_lo = (uint32_t)row[w == W - 1 ? 0 : w + 1];
        n2 = (uint64_t)__builtin_amdgcn_alignbit((uint32_t)(c >> 32), (uint32_t)c, 1) |
             ((uint64_t)__builtin_amdgcn_alignbit(next_lo, (uint32_t)(c >> 32), 1) << 32);
    }
}

// One half-step of the band: n_out words of dst from src (both LDS).  Output
// row t is lattice row (a + t) mod L, so its word w is stream group
// ((a + t) mod L) * W + w.
template <int WHICH, bool PAIRED, bool COMPLEMENT, bool OBS>
__device__ __forceinline__ void band_half(const uint64_t* src, uint64_t* dst, uint32_t n_out, uint32_t a, uint32_t L,
                                          uint32_t W, const FastDiv& divW, const DrawParams& dp, const PlaneMasks& pm,
                                          const uint32_t* T24, BandList& wl, BandSums& acc) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t n_tiles = (n_out + 63u) / 64u;
    uint32_t listed = 0;
    for (uint32_t tile = wave; tile < n_tiles; tile += kBandWaves) {
        const uint32_t u = 64u * tile + lane;
        const bool active = u < n_out;
        const uint32_t t = fdiv(u, divW);
        const uint32_t w = u - t * W;
        uint64_t c = 0, n1 = 0, n2 = 0;
        if (active)
            band_gather<WHICH>(src, t, w, W, c, n1, n2);
        const uint32_t row = a + t >= L ? a + t - L : a + t;
        uint64_t P[8];
        draw_planes(dp, active ? row * W + w : 0u, P);
        const WordDraw wd = compare_planes<PAIRED, COMPLEMENT>(P, c, n1, n2, pm);
        const uint64_t und = active ? wd.und : 0ull;
        if (active) {
            dst[u] = wd.lt;
            if constexpr (OBS) {
                acc.pc += __popcll(wd.lt);
                acc.dpair += __popcll((wd.lt ^ n1) & ~und) + __popcll((wd.lt ^ n2) & ~und);
                acc.dself += __popcll((wd.lt ^ c) & ~und);
            }
        }
        const uint64_t need = __ballot(und != 0);
        if (und != 0) {
            const uint32_t e = listed + __builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
            wl.und[e] = und;
            wl.u[e] = u;
        }
        listed += (uint32_t)__popcll(need);
        if (listed >= 64u || tile + kBandWaves >= n_tiles) {
            band_sync_wave();
            for (uint32_t e = lane; e < listed; e += 64u) {
                const uint32_t uu = wl.u[e];
                const uint64_t ud = wl.und[e];
                const uint32_t tt = fdiv(uu, divW);
                const uint32_t ww = uu - tt * W;
                uint64_t cc, a1, a2;
                band_gather<WHICH>(src, tt, ww, W, cc, a1, a2);
                const uint32_t rr = a + tt >= L ? a + tt - L : a + tt;
                const uint32_t site0 = 64u * (rr * W + ww);
                uint64_t r = 0, rem = ud;
                while (rem) {
                    const int b = __ffsll((unsigned long long)rem) - 1;
                    rem &= rem - 1;
                    if (draw_tail24(dp, site0 + (uint32_t)b) < T24[class_at(cc, a1, a2, b)])
                        r |= 1ull << b;
                }
                dst[uu] |= r;   // this lane is the only writer of word uu in this half-step
                if constexpr (OBS) {
                    acc.pc += __popcll(r);
                    acc.dpair += __popcll((r ^ a1) & ud) + __popcll((r ^ a2) & ud);
                    acc.dself += __popcll((r ^ cc) & ud);
                }
            }
            band_sync_wave();
            listed = 0;
        }
    }
}

// INT8: lattices in global memory are int8 (16-byte aligned rows), else
// 64-bit words.  OBS: the workgroup's (#+1, #differences to up + right, #to
// the partner, #sites) go to partials[4 * blockIdx.x ...].
template <bool INT8, bool PAIRED, bool COMPLEMENT, bool OBS>
__global__ __launch_bounds__(64 * kBandWaves) void k_band_step(BandArgs ba, int64_t* __restrict__ partials) {
    __shared__ BandShared sh;
    __shared__ int64_t red[3 * kBandWaves];
    const uint32_t chain = blockIdx.x / ba.bands;
    const uint32_t band = blockIdx.x - chain * ba.bands;
    const uint32_t L = ba.L, W = ba.W, R = ba.R;
    const uint32_t a = band * R;
    // sigma rows a - 1 .. a + R into LDS
    const uint32_t n_in = (R + 2) * W;
    for (uint32_t q = threadIdx.x; q < n_in; q += blockDim.x) {
        const uint32_t t = fdiv(q, ba.divW);
        const uint32_t w = q - t * W;
        uint32_t row = a + t;   // lattice row a - 1 + t, kept non-negative
        row = row == 0 ? L - 1 : row - 1;
        row = row >= L ? row - L : row;
        if constexpr (INT8)
            sh.sig[q] = load_bits64_i8(static_cast<const int8_t*>(ba.src[chain]) + (size_t)row * L + 64u * w);
        else
            sh.sig[q] = static_cast<const uint64_t*>(ba.src[chain])[(size_t)row * W + w];
    }
    if (threadIdx.x < 6)
        sh.T24[threadIdx.x] = PAIRED ? paired_tail(ba.T[chain], threadIdx.x) : ba.T[chain][threadIdx.x] & 0xFFFFFFu;
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
    BandList& wl = sh.list[threadIdx.x >> 6];
    BandSums acc;
    dp.t = ba.t0;
    band_half<0, PAIRED, COMPLEMENT, false>(sh.sig, sh.tau, (R + 1) * W, a, L, W, ba.divW, dp, pm, sh.T24, wl, acc);
    __syncthreads();
    dp.t = ba.t0 + 1u;
    band_half<1, PAIRED, COMPLEMENT, OBS>(sh.tau, sh.out, R * W, a, L, W, ba.divW, dp, pm, sh.T24, wl, acc);
    __syncthreads();
    // sigma' rows a .. a + R - 1 to the other lattice of the pair
    const uint32_t n_out = R * W;
    for (uint32_t u = threadIdx.x; u < n_out; u += blockDim.x) {
        if constexpr (INT8)
            store_bits64_i8(static_cast<int8_t*>(ba.dst[chain]) + (size_t)a * L + 64u * u, sh.out[u]);
        else
            static_cast<uint64_t*>(ba.dst[chain])[(size_t)a * W + u] = sh.out[u];
    }
    if constexpr (OBS) {
        int64_t v[3] = {acc.pc, acc.dpair, acc.dself};
        block_sum_i64<3>(v, red);
        if (threadIdx.x == 0) {
            int64_t* p = partials + 4u * (size_t)blockIdx.x;
            p[0] = v[0];
            p[1] = v[1];
            p[2] = v[2];
            p[3] = (int64_t)n_out * 64;
        }
    }
}

template <bool INT8, bool OBS>
void launch_band_t(const BandArgs& ba, bool paired, bool complement, int64_t* partials, hipStream_t st) {
    const dim3 grid(ba.n_chains * ba.bands), block(64 * kBandWaves);
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

uint32_t band_rows(int32_t L) {
    if (L < 64 || L % 64 != 0)
        return 0;
    const uint32_t W = (uint32_t)L / 64u;
    if (W > 64u || 256u % W != 0)
        return 0;
    const uint32_t R = 256u / W;   // four 64-word tiles of output rows per band
    return R < (uint32_t)L ? R : (uint32_t)L;
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
