// Replica-coded shaken dynamics: multi-spin coding across chains.  Word s of a
// replica lattice holds site s (row-major, s = j L + i) of 64 replicas, bit r
// for replica r (1 = spin +1).  The replicas share the seed and the stream, so
// each site's uniform r_s -- the eight bit-planes of its 64-site group and its
// 24-bit tail, exactly as a single chain draws them -- serves all 64, and
// replica r compares it with its own thresholds T_r (its own J_r, q_r).
// Replica r therefore follows, bit for bit, the single chain at (J_r, q_r) with
// that seed and stream, while the uniforms are drawn once per site instead of
// once per site and chain.
//
// A wavefront takes batches of 16 groups (1024 sites).  Its 64 lanes first
// evaluate the batch's 64 plane calls (lane 4 g + p: call p of group g) and its
// 256 tail calls (four evaluations, tails kept in LDS), then walk the groups
// one lane per site: the plane words of the group are read from LDS, where
// the lanes that drew them left them, each lane takes its site's bit as an
// all-ones or all-zeros mask, and the 64 replicas of the site are compared bit-sliced in
// the paired form (per-replica threshold bits S[m][k] as uniform words).
// Replicas left undecided after the eight planes (top byte of r_s equal to
// their scan byte) compare the site's tail with their tail threshold.
// Replicas whose thresholds share a top byte (strongly ordered classes: 0x00
// or 0xFF) are undecided together at a site whose top byte matches; such a
// site is resolved by the whole wavefront, one replica per lane, the others
// (at most two undecided replicas) in their own lane.
#include "sd_replica.hpp"

namespace sd {

namespace {

constexpr uint32_t kBatch = 16;   // groups per batch: 16 groups x 4 plane calls = one call per lane

// Immediates of V_BITOP3: the function applied bitwise to the operand patterns
// 0xF0, 0xCC, 0xAA.
constexpr uint32_t kTA = 0xF0u, kTB = 0xCCu, kTC = 0xAAu;
constexpr uint32_t tt3(uint32_t f) { return f & 0xFFu; }
constexpr uint32_t kAllEqual = tt3(~((kTA ^ kTB) | (kTA ^ kTC)));
constexpr uint32_t kMajority = tt3((kTA & kTB) | (kTA & kTC) | (kTB & kTC));
constexpr uint32_t kNor = tt3(~(kTA | kTB));
constexpr uint32_t kSelect = tt3((kTA & kTB) | (~kTA & kTC));       // a ? b : c
constexpr uint32_t kSelectNot = tt3((kTA & ~kTB) | (~kTA & kTC));   // a ? ~b : c
constexpr uint32_t kAndNotXor = tt3(kTA & ~(kTB ^ kTC));            // a & ~(b ^ c)

template <uint32_t TT>
__device__ __forceinline__ uint32_t op3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, TT);
}

__device__ __forceinline__ void lds_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr uint32_t kWaves = 4;   // wavefronts per workgroup

// Lane h's 64-bit value (h wavefront-uniform).  The builtin returns a signed
// 32-bit value: each half is taken as unsigned before widening.
__device__ __forceinline__ uint64_t lane_word(uint64_t x, uint32_t h) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((uint32_t)x, h);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((uint32_t)(x >> 32), h);
    return ((uint64_t)hi << 32) | lo;
}

template <int WHICH>
__global__ __launch_bounds__(64 * kWaves) void k_replica_half(const uint64_t* __restrict__ src,
                                                             uint64_t* __restrict__ dst, uint32_t L, FastDiv divL,
                                                             uint32_t n_groups, DrawParams dp, ReplicaParams rp) {
    __shared__ uint32_t tail_thr[6][kReplicas];
    __shared__ uint32_t tails[kWaves][kBatch * 64];
    __shared__ uint32_t planes[kWaves][64][4];   // lane 4 g + p: the four words of plane call p of group g
    for (uint32_t e = threadIdx.x; e < 6 * kReplicas; e += blockDim.x)
        tail_thr[e / kReplicas][e % kReplicas] = rp.T24[e / kReplicas][e % kReplicas];
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: loop bounds stay scalar
    const uint32_t waves_total = gridDim.x * kWaves;
    uint32_t* my_tails = tails[wave];
    for (uint32_t b0 = (blockIdx.x * kWaves + wave) * kBatch; b0 < n_groups; b0 += waves_total * kBatch) {
        // plane call (lane & 3) of group b0 + (lane >> 2)
        {
            const U4 pl = philox10_uuuv(dp.stream, dp.t | ((lane & 3u) << 30), dp.tag2, b0 + (lane >> 2), dp.key0,
                                        dp.key1);
            planes[wave][lane][0] = pl.x0;
            planes[wave][lane][1] = pl.x1;
            planes[wave][lane][2] = pl.x2;
            planes[wave][lane][3] = pl.x3;
        }
        // tails of the batch's 1024 sites: quad 16 b0 + 64 e + lane holds sites 4 quad .. 4 quad + 3
#pragma unroll
        for (uint32_t e = 0; e < 4; ++e) {
            const U4 y = philox10_uuuv(dp.stream, dp.t, dp.tag2 + 1u, 16u * b0 + 64u * e + lane, dp.key0, dp.key1);
            uint32_t* t4 = my_tails + 4u * (64u * e + lane);
            t4[0] = y.x0 >> 8;
            t4[1] = y.x1 >> 8;
            t4[2] = y.x2 >> 8;
            t4[3] = y.x3 >> 8;
        }
        lds_wave_sync();
        const uint32_t nb = n_groups - b0 < kBatch ? n_groups - b0 : kBatch;
        // the words of a group are loaded one group ahead of their use
        auto load = [&](uint32_t g, uint64_t& c, uint64_t& n1, uint64_t& n2) __attribute__((always_inline)) {
            const uint32_t s = 64u * g + lane;
            const uint32_t j = fdiv(s, divL);
            const uint32_t i = s - j * L;
            c = src[s];
            if (WHICH == 0) {
                n1 = src[(j == 0 ? L - 1 : j - 1) * L + i];
                n2 = src[j * L + (i == 0 ? L - 1 : i - 1)];
            } else {
                n1 = src[(j == L - 1 ? 0 : j + 1) * L + i];
                n2 = src[j * L + (i == L - 1 ? 0 : i + 1)];
            }
        };
        uint64_t nc, nn1, nn2;
        load(b0, nc, nn1, nn2);
        for (uint32_t gi = 0; gi < nb; ++gi) {
            const uint32_t s = 64u * (b0 + gi) + lane;
            const uint64_t c = nc, n1 = nn1, n2 = nn2;
            if (gi + 1 < nb)
                load(b0 + gi + 1, nc, nn1, nn2);
            uint32_t q0[2], w1[2], q2[2], nl[2], und[2], v[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const uint32_t a = (uint32_t)(n1 >> (32 * h)), b = (uint32_t)(n2 >> (32 * h)),
                               cc = (uint32_t)(c >> (32 * h));
                q0[h] = op3<kAllEqual>(a, b, cc);
                q2[h] = a ^ b;
                w1[h] = op3<kNor>(q0[h], q2[h], 0u);
                nl[h] = op3<kMajority>(a, b, cc);
                und[h] = ~0u;
                v[h] = 0u;
            }
            // plane m of this group: word (m & 1) * 2 + (lane >= 32) of call m / 2;
            // this lane's site is its bit lane % 32
            const uint32_t* pg = &planes[wave][4u * gi][lane >> 5];
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const uint32_t word = pg[4 * (m >> 1) + 2 * (m & 1)];
                const uint32_t rm = (uint32_t)__builtin_amdgcn_sbfe(word, lane & 31u, 1u);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const uint32_t S0 = (uint32_t)(rp.S[m][0] >> (32 * h));
                    const uint32_t S1 = (uint32_t)(rp.S[m][1] >> (32 * h));
                    const uint32_t S2 = (uint32_t)(rp.S[m][2] >> (32 * h));
                    const uint32_t tb = op3<kSelect>(q0[h], S0, op3<kSelect>(w1[h], S1, S2));
                    v[h] = op3<kSelectNot>(und[h], rm, v[h]);
                    und[h] = op3<kAndNotXor>(und[h], rm ^ nl[h], tb);
                }
            }
            uint64_t lt = ((uint64_t)(v[0] & ~und[0])) | ((uint64_t)(v[1] & ~und[1]) << 32);
            uint64_t u = (uint64_t)und[0] | ((uint64_t)und[1] << 32);
            const uint32_t t24 = my_tails[64u * gi + lane];
            // Sites with at most kFewTails undecided chains resolve them in
            // their own lane; a site with more (chains whose thresholds share
            // the site's top byte) is resolved by the whole wavefront, one
            // chain per lane, so that one lane's many compares do not hold up
            // the others.
            constexpr int kFewTails = 3;
            const bool many = __popcll(u) > kFewTails;
#pragma unroll
            for (int it = 0; it < kFewTails; ++it) {
                if (!many && u) {
                    const int r = __ffsll((unsigned long long)u) - 1;
                    u &= u - 1;
                    const uint32_t idx = 2u * ((uint32_t)((n1 >> r) & 1u) + (uint32_t)((n2 >> r) & 1u)) +
                                         (uint32_t)((c >> r) & 1u);
                    if (t24 < tail_thr[idx][r])
                        lt |= 1ull << r;
                }
            }
            uint64_t heavy = __ballot(many);
            while (heavy) {   // wavefront-uniform
                const uint32_t h = (uint32_t)__ffsll((unsigned long long)heavy) - 1u;
                heavy &= heavy - 1;
                const uint64_t uh = lane_word(u, h), ch = lane_word(c, h), ah = lane_word(n1, h),
                               bh = lane_word(n2, h);
                const uint32_t th = (uint32_t)__builtin_amdgcn_readlane(t24, h);
                // lane l decides chain l of site h
                const uint32_t idx = 2u * ((uint32_t)((ah >> lane) & 1u) + (uint32_t)((bh >> lane) & 1u)) +
                                     (uint32_t)((ch >> lane) & 1u);
                const bool plus = ((uh >> lane) & 1u) && th < tail_thr[idx][lane];
                const uint64_t res = __ballot(plus);
                if (lane == h)
                    lt |= res;
            }
            dst[s] = lt;
        }
        lds_wave_sync();
    }
}

// Sites per lane of k_replica_observe: the bit-sliced counters have eight
// planes, so every count stays below 256.
constexpr uint32_t kObsWordsPerLane = 128;
constexpr uint32_t kWavesObs = 4;   // 256 threads
constexpr uint32_t kObsRow = 33;   // padded row of the transposition buffer (32 replicas)

__device__ __forceinline__ void ripple_add(uint64_t (&P)[8], uint64_t w) {
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const uint64_t carry = P[b] & w;
        P[b] ^= w;
        w = carry;
    }
}

// All 64 replicas' (M, A, B) in one pass over the sites.  Lane t of the
// workgroup reads site words s0 + 256 k + t and adds, per quantity (+1
// spins, sigma != tau_up, sigma != tau_right, sigma != tau), the word's bits
// into eight bit-sliced counter planes, one count per replica bit.  Each lane
// then decodes its counts per quantity, 32 replicas at a time, into a padded
// LDS row (33 words, so that rows and columns are read and written without
// bank conflicts); lane l sums column l mod 32 over half of the wavefront's
// rows and adds it to the workgroup's count of that replica.  One lane per
// replica adds the workgroup's contributions to out[3 r ...] (zeroed before
// the launch).
__global__ __launch_bounds__(256) void k_replica_observe(const uint64_t* __restrict__ sig,
                                                         const uint64_t* __restrict__ tau, uint32_t L, FastDiv divL,
                                                         int64_t* __restrict__ out) {
    __shared__ uint32_t rows[kWavesObs][64 * kObsRow];
    __shared__ uint32_t blk[4][64];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    blk[threadIdx.x >> 6][threadIdx.x & 63u] = 0u;
    __syncthreads();
    const uint32_t n = L * L;
    const uint32_t s0 = blockIdx.x * (256u * kObsWordsPerLane);
    uint64_t P[4][8];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 8; ++b)
            P[q][b] = 0ull;
    for (uint32_t k = 0; k < kObsWordsPerLane; ++k) {
        const uint32_t s = s0 + 256u * k + threadIdx.x;
        if (s >= n)
            break;
        const uint32_t j = fdiv(s, divL);
        const uint32_t i = s - j * L;
        const uint64_t x = sig[s];
        ripple_add(P[0], x);
        ripple_add(P[1], x ^ tau[(j == L - 1 ? 0 : j + 1) * L + i]);
        ripple_add(P[2], x ^ tau[j * L + (i == L - 1 ? 0 : i + 1)]);
        ripple_add(P[3], x ^ tau[s]);
    }
    uint32_t* row = rows[wave];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int r = 0; r < 32; ++r) {
                uint32_t c = 0;
#pragma unroll
                for (int b = 0; b < 8; ++b)
                    c |= (uint32_t)((P[q][b] >> (32 * h + r)) & 1ull) << b;
                row[lane * kObsRow + r] = c;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const uint32_t col = lane & 31u, first = (lane >> 5) * 32u;
            uint32_t sum = 0;
            for (uint32_t l = 0; l < 32u; ++l)
                sum += row[(first + l) * kObsRow + col];
            atomicAdd(&blk[q][32u * h + col], sum);
            // every lane's reads of the rows precede the next writes
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    __syncthreads();
    if (threadIdx.x < 64u) {
        const uint32_t r = threadIdx.x;
        const uint32_t e = s0 + 256u * kObsWordsPerLane < n ? s0 + 256u * kObsWordsPerLane : n;
        const int64_t N = e > s0 ? (int64_t)(e - s0) : 0;
        unsigned long long* o = reinterpret_cast<unsigned long long*>(out + 3 * r);
        atomicAdd(o, (unsigned long long)(2 * (int64_t)blk[0][r] - N));
        atomicAdd(o + 1, (unsigned long long)(2 * N - 2 * ((int64_t)blk[1][r] + (int64_t)blk[2][r])));
        atomicAdd(o + 2, (unsigned long long)(N - 2 * (int64_t)blk[3][r]));
    }
}

}  // namespace

hipError_t launch_replica_half(int which, const uint64_t* src, uint64_t* dst, uint32_t L, const DrawParams& dp,
                               const ReplicaParams& rp, hipStream_t st) {
    const uint32_t n_groups = (uint32_t)(((uint64_t)L * L) / 64u);
    const uint32_t batches = (n_groups + kBatch - 1) / kBatch;
    uint32_t blocks = (batches + kWaves - 1) / kWaves;
    if (blocks > 8192u)
        blocks = 8192u;
    const FastDiv divL = make_fastdiv(L);
    if (which == 0)
        hipLaunchKernelGGL(k_replica_half<0>, dim3(blocks), dim3(64 * kWaves), 0, st, src, dst, L, divL, n_groups, dp,
                           rp);
    else
        hipLaunchKernelGGL(k_replica_half<1>, dim3(blocks), dim3(64 * kWaves), 0, st, src, dst, L, divL, n_groups, dp,
                           rp);
    return hipGetLastError();
}

hipError_t launch_replica_observe(const uint64_t* sigma, const uint64_t* tau, uint32_t L, int64_t* out,
                                  hipStream_t st) {
    hipError_t e = launch_fill_i64(out, 3 * kReplicas, 0, st);
    if (e != hipSuccess)
        return e;
    const uint32_t n = L * L;
    const uint32_t per_block = 256u * kObsWordsPerLane;
    hipLaunchKernelGGL(k_replica_observe, dim3((n + per_block - 1) / per_block), dim3(256), 0, st, sigma, tau, L,
                       make_fastdiv(L), out);
    return hipGetLastError();
}

}  // namespace sd
