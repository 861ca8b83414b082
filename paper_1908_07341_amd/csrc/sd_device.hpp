// Device building blocks of the shaken-dynamics kernels (gfx950, wave64).
//
// The heat-bath draw of Algorithm 3 ("+1 if rand() < p") is realised as
// r_s < T[class] with r_s a 32-bit uniform and T a uint32 threshold table.  The
// uniform of site s at half-step index t is defined by the stream contract:
//   * sites are grouped 64 at a time in linear order (group g = s / 64,
//     bit b = s % 64);
//   * four Philox4x32-10 calls X = Philox(ctr = (stream, t | p<<30, 2*tag, g))
//     give eight 64-bit planes (plane 2p = X0 | X1<<32, plane 2p+1 = X2 | X3<<32);
//     bit (31 - m) of r_s is bit b of plane m;
//   * the low 24 bits of r_s are Y[s % 4] >> 8 with
//     Y = Philox(ctr = (stream, t, 2*tag + 1, s / 4)).
// A site is decided by the most significant bit where r_s and T differ, so the
// kernels compare the eight planes bit-sliced against the thresholds (one lane
// per 64-site word) and draw the low bits only for the ~1/256 sites whose top
// byte equals the threshold's.  The result is identical to comparing the full
// 32-bit r_s.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sd {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

constexpr uint32_t kTagDynamics = 0;
constexpr uint32_t kTagInit = 1;

// Per-launch constants of one draw (one half-step or one random initialisation).
struct DrawParams {
    uint32_t T[6];      // thresholds by class idx = 2k + [c = +1]
    uint32_t key0;      // seed mod 2^32
    uint32_t key1;      // seed div 2^32
    uint32_t stream;    // chain id
    uint32_t t;         // half-step index (< 2^30)
    uint32_t tag2;      // 2 * tag
    uint32_t rng_xor;   // 0, or ~0 to replace every uniform r by 2^32 - 1 - r
};

__device__ __forceinline__ uint32_t hi32(uint64_t x) { return (uint32_t)(x >> 32); }
__device__ __forceinline__ uint32_t lo32(uint64_t x) { return (uint32_t)x; }

// Three-way XOR in one VALU op (gfx950 V_BITOP3_B32, truth table 0x96 is
// symmetric in its operands).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

struct U4 { uint32_t x0, x1, x2, x3; };

// The full 64-bit product a * m in one v_mad_u64_u32.  Left to itself the
// compiler splits some of the last round's products into v_mul_hi_u32 and
// v_mul_lo_u32, two instructions for one product.
__device__ __forceinline__ uint64_t mul_wide(uint32_t a, uint32_t m) {
    uint64_t r, carry;
    asm("v_mad_u64_u32 %0, %1, %2, %3, 0" : "=v"(r), "=s"(carry) : "v"(a), "s"(m));
    return r;
}

// One Philox round whose counter words are all lane-varying.
__device__ __forceinline__ U4 philox_round(U4 c, uint32_t k0, uint32_t k1) {
    uint64_t p0 = mul_wide(c.x0, kPhiloxM0);
    uint64_t p1 = mul_wide(c.x2, kPhiloxM1);
    U4 n;
    n.x0 = xor3(hi32(p1), c.x1, k0);
    n.x1 = lo32(p1);
    n.x2 = xor3(hi32(p0), c.x3, k1);
    n.x3 = lo32(p0);
    return n;
}

// Philox4x32-10 for a counter (u0, u1, u2, v3) whose first three words are
// wavefront-uniform and whose last word v3 varies per lane.  Rounds 1-3 are
// written out so the uniform parts stay on the scalar unit.
__device__ __forceinline__ U4 philox10_uuuv(uint32_t u0, uint32_t u1, uint32_t u2, uint32_t v3,
                                            uint32_t k0, uint32_t k1) {
    // round 1: both products uniform
    uint64_t a0 = (uint64_t)kPhiloxM0 * u0;
    uint64_t a1 = (uint64_t)kPhiloxM1 * u2;
    uint32_t c0 = hi32(a1) ^ u1 ^ k0;           // uniform
    uint32_t c1 = lo32(a1);                     // uniform
    uint32_t c2 = (hi32(a0) ^ k1) ^ v3;         // lane-varying
    uint32_t c3 = lo32(a0);                     // uniform
    k0 += kPhiloxW0; k1 += kPhiloxW1;
    // round 2: product of c0 uniform, of c2 varying
    uint64_t b0 = (uint64_t)kPhiloxM0 * c0;
    uint64_t b1 = (uint64_t)kPhiloxM1 * c2;
    uint32_t d0 = hi32(b1) ^ (c1 ^ k0);
    uint32_t d1 = lo32(b1);
    uint32_t d2 = hi32(b0) ^ c3 ^ k1;          // uniform
    uint32_t d3 = lo32(b0);                    // uniform
    k0 += kPhiloxW0; k1 += kPhiloxW1;
    // round 3: product of d0 varying, of d2 uniform
    uint64_t e0 = (uint64_t)kPhiloxM0 * d0;
    uint64_t e1 = (uint64_t)kPhiloxM1 * d2;
    U4 c;
    c.x0 = d1 ^ (hi32(e1) ^ k0);
    c.x1 = lo32(e1);                           // uniform
    c.x2 = hi32(e0) ^ (d3 ^ k1);
    c.x3 = lo32(e0);
    k0 += kPhiloxW0; k1 += kPhiloxW1;
    // round 4: x1 is still uniform
    {
        uint64_t p0 = (uint64_t)kPhiloxM0 * c.x0;
        uint64_t p1 = (uint64_t)kPhiloxM1 * c.x2;
        U4 n;
        n.x0 = hi32(p1) ^ (c.x1 ^ k0);
        n.x1 = lo32(p1);
        n.x2 = xor3(hi32(p0), c.x3, k1);
        n.x3 = lo32(p0);
        c = n;
    }
#pragma unroll
    for (int r = 4; r < 10; ++r) {
        k0 += kPhiloxW0; k1 += kPhiloxW1;
        c = philox_round(c, k0, k1);
    }
    return c;
}

// The eight random planes of group g.  The four calls differ only in counter
// word 1 (t | p<<30), which is uniform, so the compiler shares the
// lane-varying products of rounds 2 and 3 between them.
__device__ __forceinline__ void draw_planes(const DrawParams& dp, uint32_t g, uint64_t P[8]) {
#pragma unroll
    for (uint32_t p = 0; p < 4; ++p) {
        U4 x = philox10_uuuv(dp.stream, dp.t | (p << 30), dp.tag2, g, dp.key0, dp.key1);
        P[2 * p] = ((uint64_t)x.x0 | ((uint64_t)x.x1 << 32));
        P[2 * p + 1] = ((uint64_t)x.x2 | ((uint64_t)x.x3 << 32));
    }
}

// Low 24 bits of r_s (already complemented when rng_xor is set).
__device__ __forceinline__ uint32_t draw_tail24(const DrawParams& dp, uint32_t s) {
    U4 y = philox10_uuuv(dp.stream, dp.t, dp.tag2 + 1u, s >> 2, dp.key0, dp.key1);
    uint32_t w = (s & 3u) == 0 ? y.x0 : (s & 3u) == 1 ? y.x1 : (s & 3u) == 2 ? y.x2 : y.x3;
    return (w ^ dp.rng_xor) >> 8;
}

__device__ __forceinline__ uint32_t threshold_of(const DrawParams& dp, uint32_t idx) {
    uint32_t v = dp.T[0];
    v = idx == 1 ? dp.T[1] : v;
    v = idx == 2 ? dp.T[2] : v;
    v = idx == 3 ? dp.T[3] : v;
    v = idx == 4 ? dp.T[4] : v;
    v = idx == 5 ? dp.T[5] : v;
    return v;
}

// Copy of a wavefront-uniform value held in a vector register.  Loop-invariant
// uniforms of the inner loops (threshold bit masks) are kept this way so that
// they do not crowd the scalar register file.
__device__ __forceinline__ uint32_t in_vgpr(uint32_t x) {
    uint32_t v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "v"(x));
    return v;
}

// Threshold bits of the eight planes as all-ones / all-zeros masks, one per
// (plane m, class idx): S[m][idx] = ~0 iff bit (31 - m) of T[idx] is set.
// Classes idx and 5 - idx have opposite fields (k -> 2 - k, c -> -c), so
// T[5 - idx] = 2^32 - T[idx]: the top bytes of a pair are bitwise complements
// unless both thresholds are multiples of 2^24, and the scan needs only the
// three "leader" classes 0, 1, 2 (paired form, see compare_planes_paired and
// paired_tail for the exception).
struct PlaneMasks {
    uint32_t S[8][6];   // general form: all ones where bit (31 - m) of T[i] is set
    uint32_t code;      // paired form: bits 3m..3m+2 = bit (31 - m) of T[0], T[1], T[2]
};

// With PAIRED only the wave-uniform plane codes are formed; otherwise the
// masks of all six classes are materialised in VGPRs.
template <bool PAIRED>
__device__ __forceinline__ PlaneMasks make_plane_masks(const DrawParams& dp) {
    PlaneMasks pm;
    pm.code = 0;
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const uint32_t bit = (dp.T[i] >> (31 - m)) & 1u;
            if (PAIRED) {
                pm.S[m][i] = 0u;
                if (i < 3)
                    pm.code |= bit << (3 * m + i);
            } else {
                pm.S[m][i] = in_vgpr(0u - bit);
            }
        }
    if (PAIRED)
        pm.code = __builtin_amdgcn_readfirstlane(pm.code);
    return pm;
}

// True when every class pair satisfies T[idx] + T[5 - idx] = 2^32, the
// condition of the paired compare.  The threshold table always meets it
// (the classes of a pair have opposite fields and T(h) + T(-h) = 2^32), so
// the general form remains only as a checked fallback.
inline bool thresholds_paired(const uint32_t T[6]) {
    for (int i = 0; i < 3; ++i)
        if ((uint32_t)(T[i] + T[5 - i]) != 0u)
            return false;
    return true;
}

// The tail threshold of class idx in the paired compare.  The scan compares
// the top byte of r with the top byte of T[idx] for idx < 3 and with the
// complement of the top byte of T[5 - idx] for idx >= 3; a site left
// undecided has r's top byte equal to that scan byte B, so r < T[idx] iff its
// low 24 bits are below T[idx] - B * 2^24.  That is T[idx] mod 2^24 when B is
// T[idx]'s own top byte, and 2^24 (every tail) when the pair's thresholds are
// multiples of 2^24 (T[5 - idx] = B' 2^24 makes T[idx] = (256 - B') 2^24 while
// the scan byte is 255 - B').
__host__ __device__ inline uint32_t paired_tail(const uint32_t T[6], int idx) {
    if (idx < 3)
        return T[idx] & 0xFFFFFFu;
    const uint32_t scan_byte = 255u - (T[5 - idx] >> 24);
    return T[idx] - (scan_byte << 24);
}

// Bit-sliced comparison of the top 8 bits of every r_s in a 32-site half word
// against the per-site thresholds.  n1, n2 are the two J-neighbour bits and c
// the partner bit of each site (bit 1 = spin +1).  Returns in lt the sites
// already known to satisfy r < T and in und those whose top byte equals the
// threshold's top byte.  COMPLEMENT replaces every r by its complement.
//
// Paired form: with Q0 = (n1 == n2 == c) (classes 0 and 5), Q2 = n1 ^ n2
// (classes 2 and 3), W1 = the rest (classes 1 and 4), and nl =
// majority(n1, n2, c) marking the classes 3, 4, 5, the threshold bit of plane m
// is nl ^ (Q0 & S[m][0] | W1 & S[m][1] | Q2 & S[m][2]).  The S are uniform, so
// that word is one of eight per-site candidates, picked by the 3-bit plane code.
// The scan keeps und (top bits equal so far) and v, the complement of r at the
// last plane where the site was still undecided: for a decided site that is
// the first differing plane, where r < T iff r's bit is 0.  Each plane costs
// the pick and two three-input ops.
// General form: the union of the class masks whose threshold bit is set.
struct HalfWord {
    uint32_t lt, und;
};

template <bool COMPLEMENT>
__device__ __forceinline__ HalfWord compare_planes_32(const uint32_t P[8], uint32_t c, uint32_t n1, uint32_t n2,
                                                      const PlaneMasks& pm) {
    uint32_t lt = 0, und = ~0u;
    {
        const uint32_t k2 = n1 & n2;
        const uint32_t k1 = n1 ^ n2;
        const uint32_t k0 = ~(n1 | n2);
        const uint32_t m0 = k0 & ~c, m1 = k0 & c;
        const uint32_t m2 = k1 & ~c, m3 = k1 & c;
        const uint32_t m4 = k2 & ~c, m5 = k2 & c;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const uint32_t tb = (m0 & pm.S[m][0]) | (m1 & pm.S[m][1]) | (m2 & pm.S[m][2]) |
                                (m3 & pm.S[m][3]) | (m4 & pm.S[m][4]) | (m5 & pm.S[m][5]);
            const uint32_t r = COMPLEMENT ? ~P[m] : P[m];
            lt |= und & tb & ~r;
            und &= ~(r ^ tb);
        }
    }
    return {lt, und};
}

struct WordDraw {
    uint64_t lt, und;
};

typedef uint32_t u32x16 __attribute__((ext_vector_type(16)));

// Truth tables of V_BITOP3_B32 from the operand patterns a = 0xF0, b = 0xCC,
// c = 0xAA.  kScanV(und, r, v): ~r where und, else v; kScanUnd(r, tb, und):
// und where r equals tb.  The C forms compare the complemented stream ~r.
constexpr uint32_t kBopA = 0xF0u, kBopB = 0xCCu, kBopC = 0xAAu;
constexpr uint32_t kScanV = ((kBopA & ~kBopB) | (~kBopA & kBopC)) & 0xFFu;
constexpr uint32_t kScanVC = ((kBopA & kBopB) | (~kBopA & kBopC)) & 0xFFu;
constexpr uint32_t kScanUnd = (~(kBopA ^ kBopB) & kBopC) & 0xFFu;
constexpr uint32_t kScanUndC = ((kBopA ^ kBopB) & kBopC) & 0xFFu;
static_assert(kScanV == 0x3Au && kScanVC == 0xCAu && kScanUnd == 0x82u && kScanUndC == 0x28u, "scan tables");

// Paired form on a 64-site word.  The candidates of both 32-bit halves sit in
// one 16-entry vector so that the uniform pick is an indexed VGPR move.
template <bool COMPLEMENT>
__device__ __forceinline__ WordDraw compare_planes_paired(const uint64_t P[8], uint64_t c64, uint64_t n164,
                                                          uint64_t n264, uint32_t code) {
    u32x16 cand;
    uint32_t und[2], v[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t c = (uint32_t)(c64 >> (32 * h)), n1 = (uint32_t)(n164 >> (32 * h)),
                       n2 = (uint32_t)(n264 >> (32 * h));
        const uint32_t q0 = ~((n1 ^ c) | (n2 ^ c));
        const uint32_t q2 = n1 ^ n2;
        const uint32_t nl = (n1 & n2) | (c & (n1 | n2));
        cand[8 * h + 0] = nl;
        cand[8 * h + 1] = nl ^ q0;
        cand[8 * h + 2] = ~(nl ^ (q0 | q2));
        cand[8 * h + 4] = nl ^ q2;
        cand[8 * h + 7] = ~nl;
        cand[8 * h + 6] = ~(nl ^ q0);
        cand[8 * h + 5] = nl ^ (q0 | q2);
        cand[8 * h + 3] = ~(nl ^ q2);
        und[h] = ~0u;
        v[h] = 0u;
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const uint32_t idx = (code >> (3 * m)) & 7u;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t tb = cand[idx + 8u * h];
            const uint32_t r = (uint32_t)(P[m] >> (32 * h));
            v[h] = __builtin_amdgcn_bitop3_b32(und[h], r, v[h], COMPLEMENT ? kScanVC : kScanV);
            und[h] = __builtin_amdgcn_bitop3_b32(r, tb, und[h], COMPLEMENT ? kScanUndC : kScanUnd);
        }
    }
    const uint64_t u = (uint64_t)und[0] | ((uint64_t)und[1] << 32);
    const uint64_t vv = (uint64_t)v[0] | ((uint64_t)v[1] << 32);
    return {vv & ~u, u};
}

template <bool PAIRED, bool COMPLEMENT>
__device__ __forceinline__ WordDraw compare_planes(const uint64_t P[8], uint64_t c, uint64_t n1, uint64_t n2,
                                                   const PlaneMasks& pm) {
    if constexpr (PAIRED)
        return compare_planes_paired<COMPLEMENT>(P, c, n1, n2, pm.code);
    uint32_t Plo[8], Phi[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        Plo[m] = (uint32_t)P[m];
        Phi[m] = (uint32_t)(P[m] >> 32);
    }
    HalfWord lo = compare_planes_32<COMPLEMENT>(Plo, (uint32_t)c, (uint32_t)n1, (uint32_t)n2, pm);
    HalfWord hi = compare_planes_32<COMPLEMENT>(Phi, (uint32_t)(c >> 32), (uint32_t)(n1 >> 32),
                                                (uint32_t)(n2 >> 32), pm);
    return {(uint64_t)lo.lt | ((uint64_t)hi.lt << 32), (uint64_t)lo.und | ((uint64_t)hi.und << 32)};
}

__device__ __forceinline__ uint32_t class_at(uint64_t c, uint64_t n1, uint64_t n2, int b) {
    uint32_t k = (uint32_t)((n1 >> b) & 1u) + (uint32_t)((n2 >> b) & 1u);
    return 2u * k + (uint32_t)((c >> b) & 1u);
}

// Decision of one undecided site with threshold thr: its top byte equals the
// threshold's, so r < thr iff the low 24 bits compare below.
__device__ __forceinline__ bool decide_tail_thr(const DrawParams& dp, uint32_t s, uint32_t thr) {
    return draw_tail24(dp, s) < (thr & 0xFFFFFFu);
}

__device__ __forceinline__ bool decide_tail(const DrawParams& dp, uint32_t s, uint32_t idx) {
    return decide_tail_thr(dp, s, threshold_of(dp, idx));
}

// Workgroup-shared scratch for resolving undecided sites cooperatively.
template <int CAP>
struct TailScratch {
    uint32_t count;
    uint32_t site[CAP];
    uint8_t info[CAP];   // class idx on entry, decision (0/1) on exit
};

// Resolve the undecided sites of every lane of the workgroup.  Must be called
// by all threads of the block (it contains barriers).  `und` marks undecided
// bits of the word whose bit 0 is site `site0`; the decided +1 bits are or-ed
// into `lt`.  Entries are handed out with one LDS atomic per lane that has
// undecided bits, resolved one per thread, and read back by their owners in
// the order they were written.  If more than CAP sites are undecided (never
// observed: the mean is 0.25 per word) each lane resolves its own bits.
template <int CAP>
__device__ __forceinline__ void resolve_tails(uint64_t& lt, uint64_t und, uint64_t c, uint64_t n1, uint64_t n2,
                                              uint32_t site0, const DrawParams& dp, TailScratch<CAP>& sh) {
    const uint32_t tid = threadIdx.x;
    if (tid == 0)
        sh.count = 0;
    __syncthreads();
    const uint32_t cnt = (uint32_t)__popcll(und);
    uint32_t base = 0;
    if (cnt)
        base = atomicAdd(&sh.count, cnt);
    __syncthreads();
    const uint32_t total = sh.count;
    if (total <= (uint32_t)CAP) {
        if (cnt) {
            uint64_t u = und;
            uint32_t e = base;
            while (u) {
                int b = __ffsll((unsigned long long)u) - 1;
                u &= u - 1;
                sh.site[e] = site0 + (uint32_t)b;
                sh.info[e] = (uint8_t)class_at(c, n1, n2, b);
                ++e;
            }
        }
        __syncthreads();
        for (uint32_t e = tid; e < total; e += blockDim.x)
            sh.info[e] = decide_tail(dp, sh.site[e], sh.info[e]) ? 1 : 0;
        __syncthreads();
        if (cnt) {
            uint64_t u = und;
            uint32_t e = base;
            while (u) {
                int b = __ffsll((unsigned long long)u) - 1;
                u &= u - 1;
                if (sh.info[e])
                    lt |= 1ull << b;
                ++e;
            }
        }
    } else if (cnt) {
        uint64_t u = und;
        while (u) {
            int b = __ffsll((unsigned long long)u) - 1;
            u &= u - 1;
            if (decide_tail(dp, site0 + (uint32_t)b, class_at(c, n1, n2, b)))
                lt |= 1ull << b;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// Sum of v over a wavefront whose 64 lanes are all active, returned in every
// lane: prefix sums within each row of 16 lanes by DPP row shifts (lanes
// shifted in from outside the row read 0), then lane 15 of rows 0 and 2 added
// into rows 1 and 3 and lane 31 into rows 2 and 3, which leaves the total in
// lane 63.  All in-lane adds, no LDS round trip.
__device__ __forceinline__ uint32_t wave_sum_dpp(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);   // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Block-wide sum of N int64 values, result valid in thread 0.  `red` must hold
// N * (blockDim.x / 64) entries.
template <int N>
__device__ __forceinline__ void block_sum_i64(int64_t (&v)[N], int64_t* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < N; ++i)
        v[i] = wave_sum_i64(v[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i)
            red[i * nw + wave] = v[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            int64_t s = 0;
            for (int w = 0; w < nw; ++w)
                s += red[i * nw + w];
            v[i] = s;
        }
    }
    __syncthreads();
}

// Fast division by a launch-constant divisor d >= 1 (n < 2^32):
// q = (umulhi(n, mul) + n) >> shift, the sum taken in 64 bits.  (add is
// always 1 for the constants make_fastdiv produces.)
struct FastDiv {
    uint32_t d, mul, shift, add;
};

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
    const uint32_t hi = __umulhi(n, f.mul);
    return (uint32_t)(((uint64_t)hi + n) >> f.shift);
}

// ---------------------------------------------------------------------------
// int8 lattices (+1 -> 0x01, -1 -> 0xFF) and 64-site bit words
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t bytes_to_bits4(uint32_t x) {
    // byte k of x is 0x01 (+1) or 0xFF (-1); bit k of the result is 1 for +1
    uint32_t y = (~x >> 7) & 0x01010101u;
    return (y * 0x10204080u) >> 28;
}

__device__ __forceinline__ uint32_t bits4_to_bytes(uint32_t n) {
    uint32_t z = (n * 0x00204081u) & 0x01010101u;   // byte k = bit k of n
    uint32_t w = z ^ 0x01010101u;                    // 1 where the spin is -1
    return z | ((w << 8) - w);
}

// The 64 sites at p (16-byte aligned) as one word, bit b = site b.
__device__ __forceinline__ uint64_t load_bits64_i8(const int8_t* p) {
    const uint4* v = reinterpret_cast<const uint4*>(p);
    uint64_t bits = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint4 x = v[q];
        uint32_t b16 = bytes_to_bits4(x.x) | (bytes_to_bits4(x.y) << 4) | (bytes_to_bits4(x.z) << 8) |
                       (bytes_to_bits4(x.w) << 12);
        bits |= (uint64_t)b16 << (16 * q);
    }
    return bits;
}

__device__ __forceinline__ void store_bits64_i8(int8_t* p, uint64_t bits) {
    uint4* v = reinterpret_cast<uint4*>(p);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t b16 = (uint32_t)(bits >> (16 * q)) & 0xFFFFu;
        uint4 x;
        x.x = bits4_to_bytes(b16 & 0xF);
        x.y = bits4_to_bytes((b16 >> 4) & 0xF);
        x.z = bits4_to_bytes((b16 >> 8) & 0xF);
        x.w = bits4_to_bytes((b16 >> 12) & 0xF);
        v[q] = x;
    }
}

// ---------------------------------------------------------------------------
// Packed lattices as one bit string: site s = j*L + i is bit s % 64 of word
// s / 64 whatever L is.  With L % 8 == 0 the N = L*L sites fill whole words,
// so every word is a full 64-site group of the stream and the neighbours of a
// word are 64-bit windows of the string (rows need not start on a word).
// ---------------------------------------------------------------------------

// Bits 64 g + off .. 64 g + off + 63 of the string (indices mod N = 64
// n_words) for g < n_words and off < N.  Since 64 g is a whole number of
// words, the window starts off >> 6 words after g, at bit off & 63.
__device__ __forceinline__ uint64_t bit_window(const uint64_t* lat, uint32_t n_words, uint32_t g, uint32_t off) {
    uint32_t q = g + (off >> 6);
    q = q >= n_words ? q - n_words : q;
    const uint32_t sh = off & 63u;
    const uint64_t w0 = lat[q];
    const uint64_t w1 = lat[q + 1u == n_words ? 0u : q + 1u];
    return sh ? ((w0 >> sh) | (w1 << (64u - sh))) : w0;
}

// Bits b of word g whose site is in column r of its row ((64 g + b) % L == r).
__device__ __forceinline__ uint64_t column_mask(uint32_t g, uint32_t L, const FastDiv& divL, uint32_t r) {
    const uint32_t s0 = 64u * g;
    const uint32_t m = s0 - fdiv(s0, divL) * L;   // column of bit 0
    uint32_t b = r >= m ? r - m : r + L - m;
    if (L >= 64u)   // at most one site of the word lies in column r
        return b < 64u ? (1ull << b) : 0ull;
    uint64_t mask = 0;
    for (; b < 64u; b += L)
        mask |= 1ull << b;
    return mask;
}

// Partner word c and neighbour words n1, n2 of word g (L % 8 == 0).
// WHICH 0 (half-step A): n1 = down (s - L), n2 = left (s - 1, or s + L - 1 in
// column 0).  WHICH 1 (half-step B): n1 = up (s + L), n2 = right (s + 1, or
// s - L + 1 in column L - 1).
template <int WHICH>
__device__ __forceinline__ void gather_bits(const uint64_t* lat, uint32_t L, uint32_t n_words, const FastDiv& divL,
                                            uint32_t g, uint64_t& c, uint64_t& n1, uint64_t& n2) {
    const uint32_t N = 64u * n_words;
    c = lat[g];
    if constexpr (WHICH == 0) {
        n1 = bit_window(lat, n_words, g, N - L);
        const uint64_t prev = lat[g == 0 ? n_words - 1u : g - 1u];
        const uint64_t base = (c << 1) | (prev >> 63);
        const uint64_t wrap = bit_window(lat, n_words, g, L - 1u);
        const uint64_t col0 = column_mask(g, L, divL, 0u);
        n2 = (base & ~col0) | (wrap & col0);
    } else {
        n1 = bit_window(lat, n_words, g, L);
        const uint64_t next = lat[g + 1u == n_words ? 0u : g + 1u];
        const uint64_t base = (c >> 1) | (next << 63);
        const uint64_t wrap = bit_window(lat, n_words, g, N + 1u - L);
        const uint64_t last = column_mask(g, L, divL, L - 1u);
        n2 = (base & ~last) | (wrap & last);
    }
}

}  // namespace sd
