// Trajectory log-likelihood of the shaken dynamics and its gradient.
//
// By the product form of the half-step transition probabilities (section 2,
// eqs. (15)-(16)) a trajectory X_0 = sigma_0, X_1 = tau_1, X_2 = sigma_1, ...
// has log-probability  sum over transitions and sites of h_x s_x - log 2cosh h_x,
// with s_x the drawn spin and h_x its field (down/left neighbours of X_m for
// even m, up/right for odd m).  h takes six values, so the 12 counts
//   n[2*idx + [s = +1]],  idx = 2k + [c = +1]
// are sufficient statistics: LL = sum n (h s - log 2cosh h),
// dLL/dJ = sum n (2k-2)(s - tanh h),  dLL/dq = sum n c (s - tanh h).
//
// The classes idx and 5 - idx have opposite fields, and log 2cosh is even and
// tanh odd, so LL and its gradient need only the six paired statistics
//   S_j = sites of the pair (j, 5 - j),
//   Z_j = sites of class j drawn +1 plus sites of class 5 - j drawn -1,
// j = 0, 1, 2 (class j is the pair's leader, with field h_j).  Pair 0 holds the
// sites whose two neighbours agree with the spin, pair 1 those whose neighbours
// agree with each other but not with the spin, pair 2 those whose neighbours
// differ; in every pair the drawn spin counts towards Z_j when it differs from
// the majority of (n1, n2, c).  Five popcounts per word instead of twelve.
//
// k_loglik_counts streams the packed trajectories once (HBM-bound) and
// accumulates the counts (or the paired statistics) exactly in integers.  The forward and backward
// kernels combine them with binary32 arithmetic only; every value is carried
// as an unevaluated sum of two floats (about 48 significant bits) because near
// the maximum of the likelihood the per-class terms (size ~N) cancel down to a
// gradient of size ~sqrt(N).
#include "sd_loglik.hpp"

namespace sd {

namespace {

// ---------------------------------------------------------------------------
// Counts
// ---------------------------------------------------------------------------
__device__ __forceinline__ void count_transition(uint64_t c, uint64_t n1, uint64_t n2, uint64_t y, int64_t (&acc)[12]) {
    const uint64_t k2 = n1 & n2, k1 = n1 ^ n2, k0 = ~(n1 | n2);
    const uint64_t cls[6] = {k0 & ~c, k0 & c, k1 & ~c, k1 & c, k2 & ~c, k2 & c};
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const int64_t plus = __popcll(cls[i] & y);
        acc[2 * i + 1] += plus;
        acc[2 * i] += __popcll(cls[i]) - plus;
    }
}

// Immediates of the three-input logic instruction (V_BITOP3): the function
// applied bitwise to the operand patterns 0xF0, 0xCC, 0xAA.
constexpr uint32_t kTA = 0xF0u, kTB = 0xCCu, kTC = 0xAAu;
constexpr uint32_t tt(uint32_t f) { return f & 0xFFu; }
constexpr uint32_t kAllEqual = tt(~((kTA ^ kTB) | (kTA ^ kTC)));      // a = b = c
constexpr uint32_t kMajority = tt((kTA & kTB) | (kTA & kTC) | (kTB & kTC));
constexpr uint32_t kXorAnd = tt((kTA ^ kTB) & kTC);                   // (a ^ b) & c

template <uint32_t TT>
__device__ __forceinline__ uint32_t lop3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, TT);
}

// acc + popcount(x) as one accumulating v_bcnt.  Written as an instruction so
// that the compiler does not regroup a chain of them into three-way adds of
// separate popcounts (one more instruction per pair).
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t acc) {
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}

// The popcounts of one 32-site half of a word-transition that fix its 12
// counts, only the sites of `live`.  With k0 = sites whose two J-neighbours
// are both -1 and k2 = both +1 (class idx = 2k + [c = +1]):
//   base = {c, n1 | n2, k0 & c, k2 & c}, ybase = {y, c, k0, k2, k0 & c, k2 & c}
//   each and-ed with y.
// The totals of k0 and k2 come from the one popcount of n1 | n2: k0 is its
// complement, and since each neighbour word of a whole lattice is a
// permutation of the lattice's bits, the +1 neighbours n1 and n2 each sum to
// the source's +1 sites, so #k2 = #n1 + #n2 - #(n1 | n2) = 2 #c - #(n1 | n2)
// over a workgroup that covers every word (the counts are linear in these
// sums, so one thread's share need not satisfy it).  Ten accumulating v_bcnt
// per half minus the source's (below) and eight logic ops, instead of counting
// the six class masks and their +1 sites one by one; count_totals turns the
// sums into the 12 counts.  A thread adds at most 32 per half-word and
// transition, so 2^27 word-transitions per thread stay exact.  base[0] (the
// source's +1 sites) is left out: over consecutive transitions each lattice
// is the target of one and the source of the next, so its sum is ybase[0]'s
// plus the first source's and minus the last target's +1 sites.
constexpr uint32_t kNeither = tt(~kTA & ~kTB & kTC), kBoth = tt(kTA & kTB & kTC);   // (a, b, mask)
constexpr uint32_t kEither = tt((kTA | kTB) & kTC);

__device__ __forceinline__ void count_half(uint32_t c, uint32_t n1, uint32_t n2, uint32_t y, uint32_t live,
                                           uint32_t (&base)[4], uint32_t (&ybase)[6]) {
    const uint32_t cl = c & live, yl = y & live;
    const uint32_t k0c = lop3<kNeither>(n1, n2, cl);
    const uint32_t k2c = lop3<kBoth>(n1, n2, cl);
    base[1] = bcnt_acc(lop3<kEither>(n1, n2, live), base[1]);
    base[2] = bcnt_acc(k0c, base[2]);
    base[3] = bcnt_acc(k2c, base[3]);
    ybase[0] = bcnt_acc(yl, ybase[0]);
    ybase[1] = bcnt_acc(cl & y, ybase[1]);
    ybase[2] = bcnt_acc(lop3<kNeither>(n1, n2, yl), ybase[2]);
    ybase[3] = bcnt_acc(lop3<kBoth>(n1, n2, yl), ybase[3]);
    ybase[4] = bcnt_acc(k0c & y, ybase[4]);
    ybase[5] = bcnt_acc(k2c & y, ybase[5]);
}

// The 12 counts (class idx: drawn -1 at 2 idx, drawn +1 at 2 idx + 1) from
// the sums of count_half over n_sites sites.  Class 1 is k0 & c, class 0 the
// rest of k0, classes 5 and 4 likewise from k2, class 3 the c = +1 sites
// of neither, class 2 what remains.
__device__ __forceinline__ void count_totals(const int64_t (&B)[5], const int64_t (&Y)[6], int64_t n_sites,
                                             int64_t (&acc)[12]) {
    const int64_t t3 = B[0] - B[3] - B[4], p3 = Y[1] - Y[4] - Y[5];
    const int64_t t[6] = {B[1] - B[3], B[3], n_sites - B[1] - B[2] - t3, t3, B[2] - B[4], B[4]};
    const int64_t p[6] = {Y[2] - Y[4], Y[4], Y[0] - Y[2] - Y[3] - p3, p3, Y[3] - Y[5], Y[5]};
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        acc[2 * i] = t[i] - p[i];
        acc[2 * i + 1] = p[i];
    }
}

// The paired sums of one word-transition: acc gets popc(Q0), popc(Q2),
// popc(Q0 & z), popc(Q2 & z) and popc(z), with Q0 = sites whose neighbours
// both equal the spin, Q2 = sites whose neighbours differ (W1 = the rest) and
// z = y ^ majority(n1, n2, c), the sites that drew the opposite of the
// majority; Z_1 = popc(z) - Z_0 - Z_2 and S_1 follows from the number of
// sites.  Only the sites of `live` count.
__device__ __forceinline__ void pair_half(uint32_t c, uint32_t n1, uint32_t n2, uint32_t y, uint32_t live,
                                          uint32_t (&acc)[5]) {
    const uint32_t q2 = lop3<kXorAnd>(n1, n2, live);
    const uint32_t q0 = lop3<kAllEqual>(n1, n2, c) & live;
    const uint32_t z = lop3<kXorAnd>(y, lop3<kMajority>(n1, n2, c), live);
    acc[0] += __popc(q0);
    acc[1] += __popc(q2);
    acc[2] += __popc(q0 & z);
    acc[3] += __popc(q2 & z);
    acc[4] += __popc(z);
}

template <typename T>
__device__ __forceinline__ void pair_transition(uint64_t c, uint64_t n1, uint64_t n2, uint64_t y, T (&acc)[5]) {
    const uint64_t q2 = n1 ^ n2;
    const uint64_t q0 = ~((n1 ^ c) | q2);
    const uint64_t z = y ^ ((q2 & c) | (~q2 & n1));
    const uint64_t v[5] = {q0, q2, q0 & z, q2 & z, z};
#pragma unroll
    for (int i = 0; i < 5; ++i)
        acc[i] += __popcll(v[i]);
}

// (S_0, S_1, S_2, Z_0, Z_1, Z_2) from the five paired sums over n_words
// word-transitions.
template <typename T>
__device__ __forceinline__ void pair_stats(const T (&acc)[5], int64_t n_words, int64_t (&out)[6]) {
    out[0] = (int64_t)acc[0];
    out[2] = (int64_t)acc[1];
    out[1] = 64 * n_words - out[0] - out[2];
    out[3] = (int64_t)acc[2];
    out[5] = (int64_t)acc[3];
    out[4] = (int64_t)acc[4] - out[3] - out[5];
}

// Workgroup sums of the 12 counts (or the 6 paired statistics): into partials[12 * block ...] when
// partials is non-null (k_counts_finish adds them up), else into counts
// through 64-bit atomics.
template <int N>
__device__ __forceinline__ void flush_counts(int64_t (&acc)[N], int64_t* red, unsigned long long* counts,
                                             int64_t* partials, uint32_t block) {
    block_sum_i64<N>(acc, red);
    if (threadIdx.x == 0) {
        if (partials) {
#pragma unroll
            for (int i = 0; i < N; ++i)
                partials[(size_t)N * block + i] = acc[i];
        } else {
#pragma unroll
            for (int i = 0; i < N; ++i)
                if (acc[i])
                    atomicAdd(counts + i, (unsigned long long)acc[i]);
        }
    }
}

template <int N>
__global__ __launch_bounds__(1024) void k_counts_finish(const int64_t* __restrict__ partials, uint32_t n_blocks,
                                                        int64_t* __restrict__ counts) {
    __shared__ int64_t red[N * 16];
    int64_t v[N];
#pragma unroll
    for (int i = 0; i < N; ++i)
        v[i] = 0;
    for (uint32_t b = threadIdx.x; b < n_blocks; b += blockDim.x)
#pragma unroll
        for (int i = 0; i < N; ++i)
            v[i] += partials[(uint32_t)N * b + i];
    block_sum_i64<N>(v, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < N; ++i)
            counts[i] = v[i];
}

// Lattices of at most kStageWords words: one workgroup walks a chunk of
// kChunk consecutive transitions of one trajectory.  Every lattice is read
// from HBM exactly once (coalesced, each of the THREADS threads owning the
// words tid, tid + THREADS, ...), DEPTH lattices ahead of use; the source lattice of each
// transition is staged in LDS (double-buffered) so that the neighbour words
// come from LDS.  One barrier per transition.  The loads are unconditional
// (lanes without a word read word 0, lattices past the chunk are clamped to
// its last one) so that the code between barriers has no divergent branch
// and each load is waited for only when its lattice is used; FULL = every
// lane owns WPT words.  Chunks start at even transitions and DEPTH is even,
// so the parity of a transition (half-step A or B) is that of its slot in
// the unrolled ring.
constexpr uint32_t kStageWords = 4096;   // L <= 512
constexpr uint32_t kChunk = 256;

// The full-tile count kernels of up to 256 threads are held to five waves
// per SIMD (94 VGPRs instead of 115): the fifth wave hides more of the HBM
// latency and the counts run 5-7% faster.
template <uint32_t THREADS, bool PAIRED, bool FULL>
constexpr int counts_min_waves() {
    return (THREADS <= 256u && FULL && !PAIRED) ? 5 : 1;
}

template <uint32_t THREADS, uint32_t WPT, uint32_t DEPTH, bool PAIRED, bool FULL>
__global__ __launch_bounds__(THREADS, (counts_min_waves<THREADS, PAIRED, FULL>())) void k_loglik_counts_lds(
    const uint64_t* __restrict__ traj, uint32_t n_lat, uint32_t L, FastDiv divW,
    unsigned long long* __restrict__ counts, int64_t* __restrict__ partials) {
    static_assert(DEPTH % 2 == 0 && kChunk % DEPTH == 0, "transition parity must follow the ring slot");
    __shared__ uint64_t buf[2][THREADS * WPT];
    __shared__ int64_t red[12 * (THREADS / 64)];
    const uint32_t W = L / 64u;
    const uint32_t n_words = L * W;
    const uint32_t a = blockIdx.x;
    const uint32_t m0 = blockIdx.y * kChunk;
    const uint32_t n_trans = n_lat - 1;
    const uint32_t m1 = m0 + kChunk < n_trans ? m0 + kChunk : n_trans;
    const uint64_t* X = traj + (size_t)a * n_lat * n_words;
    // per 32-site half: [0] low, [1] high
    uint32_t base[2][4], ybase[2][6], pst[2][5];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int i = 0; i < 6; ++i)
            ybase[h][i] = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            base[h][i] = 0;
#pragma unroll
        for (int i = 0; i < 5; ++i)
            pst[h][i] = 0;
    }
    uint32_t n_mine = 0;
    uint32_t gi[WPT], i_down[WPT], i_up[WPT], i_prev[WPT], i_next[WPT];
    uint32_t live[WPT];
#pragma unroll
    for (uint32_t k = 0; k < WPT; ++k) {
        const uint32_t g = threadIdx.x + THREADS * k;
        const bool mine = FULL || g < n_words;
        n_mine += mine ? 1u : 0u;
        live[k] = mine ? ~0u : 0u;
        const uint32_t gg = mine ? g : 0u;
        const uint32_t j = fdiv(gg, divW);
        const uint32_t w = gg - j * W;
        gi[k] = gg;
        i_down[k] = (j == 0 ? L - 1 : j - 1) * W + w;
        i_up[k] = (j == L - 1 ? 0 : j + 1) * W + w;
        i_prev[k] = j * W + (w == 0 ? W - 1 : w - 1);
        i_next[k] = j * W + (w == W - 1 ? 0 : w + 1);
    }
    // ring[d] holds lattice m + 1 + d while transition m is processed
    uint64_t cur[WPT], ring[DEPTH][WPT];
    {
        const uint64_t* X0 = X + (size_t)m0 * n_words;
#pragma unroll
        for (uint32_t k = 0; k < WPT; ++k)
            cur[k] = X0[gi[k]];
    }
    // +1 sites of the chunk's first lattice (the counts' source sum, see count_half)
    if (!PAIRED) {
#pragma unroll
        for (uint32_t k = 0; k < WPT; ++k) {
            const uint32_t lv = FULL ? ~0u : live[k];
            base[0][0] = bcnt_acc(lo32(cur[k]) & lv, base[0][0]);
            base[1][0] = bcnt_acc(hi32(cur[k]) & lv, base[1][0]);
        }
    }
#pragma unroll
    for (uint32_t d = 0; d < DEPTH; ++d) {
        const uint32_t mf = m0 + 1 + d <= m1 ? m0 + 1 + d : m1;
        const uint64_t* Xf = X + (size_t)mf * n_words;
#pragma unroll
        for (uint32_t k = 0; k < WPT; ++k)
            ring[d][k] = Xf[gi[k]];
    }
    auto transition = [&](uint32_t m, uint32_t d) __attribute__((always_inline)) {
        uint64_t* S = buf[d & 1u];
#pragma unroll
        for (uint32_t k = 0; k < WPT; ++k)
            S[threadIdx.x + THREADS * k] = cur[k];
        __syncthreads();
        const uint32_t mf = m + 1 + DEPTH <= m1 ? m + 1 + DEPTH : m1;
        const uint64_t* Xf = X + (size_t)mf * n_words;
        // all neighbour words first: the LDS reads overlap instead of each
        // waiting for the previous one
        uint64_t nv[WPT], nh[WPT];
#pragma unroll
        for (uint32_t k = 0; k < WPT; ++k) {
            nv[k] = S[(d & 1u) == 0 ? i_down[k] : i_up[k]];
            nh[k] = S[(d & 1u) == 0 ? i_prev[k] : i_next[k]];
        }
#pragma unroll
        for (uint32_t k = 0; k < WPT; ++k) {
            const uint32_t c0 = lo32(cur[k]), c1 = hi32(cur[k]);
            // the second neighbour: the word shifted by one site, the missing
            // bit from the adjacent word (funnel shifts of the halves)
            uint32_t m0, m1;
            if ((d & 1u) == 0) {
                m0 = __builtin_amdgcn_alignbit(c0, hi32(nh[k]), 31);
                m1 = __builtin_amdgcn_alignbit(c1, c0, 31);
            } else {
                m0 = __builtin_amdgcn_alignbit(c1, c0, 1);
                m1 = __builtin_amdgcn_alignbit(lo32(nh[k]), c1, 1);
            }
            const uint32_t lv = FULL ? ~0u : live[k];
            const uint64_t y = ring[d][k];
            if (PAIRED) {
                pair_half(c0, lo32(nv[k]), m0, lo32(y), lv, pst[0]);
                pair_half(c1, hi32(nv[k]), m1, hi32(y), lv, pst[1]);
            } else {
                count_half(c0, lo32(nv[k]), m0, lo32(y), lv, base[0], ybase[0]);
                count_half(c1, hi32(nv[k]), m1, hi32(y), lv, base[1], ybase[1]);
            }
            cur[k] = y;
            ring[d][k] = Xf[gi[k]];
        }
    };
    uint32_t mb = m0;
    for (; mb + DEPTH <= m1; mb += DEPTH) {
#pragma unroll
        for (uint32_t d = 0; d < DEPTH; ++d)
            transition(mb + d, d);
    }
#pragma unroll
    for (uint32_t d = 0; d < DEPTH; ++d)
        if (mb + d < m1)
            transition(mb + d, d);
    if (PAIRED) {
        int64_t sums[5], acc[6];
#pragma unroll
        for (int i = 0; i < 5; ++i)
            sums[i] = (int64_t)pst[0][i] + (int64_t)pst[1][i];
        pair_stats(sums, (int64_t)n_mine * (m1 - m0), acc);
        flush_counts<6>(acc, red, counts, partials, blockIdx.y * gridDim.x + blockIdx.x);
    } else {
        // sources' +1 sites = targets' + first lattice's - last lattice's (cur)
        uint32_t last[2] = {0, 0};
#pragma unroll
        for (uint32_t k = 0; k < WPT; ++k) {
            const uint32_t lv = FULL ? ~0u : live[k];
            last[0] = bcnt_acc(lo32(cur[k]) & lv, last[0]);
            last[1] = bcnt_acc(hi32(cur[k]) & lv, last[1]);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
            base[h][0] = base[h][0] + ybase[h][0] - last[h];
        int64_t S[4], Y[6], acc[12];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            S[i] = (int64_t)base[0][i] + (int64_t)base[1][i];
#pragma unroll
        for (int i = 0; i < 6; ++i)
            Y[i] = (int64_t)ybase[0][i] + (int64_t)ybase[1][i];
        // sites seen by this thread; #k0 and #k2 from #(n1 | n2) (count_half)
        const int64_t n_sites = 64 * (int64_t)n_mine * (m1 - m0);
        const int64_t B[5] = {S[0], n_sites - S[1], 2 * S[0] - S[1], S[2], S[3]};
        count_totals(B, Y, n_sites, acc);
        flush_counts<12>(acc, red, counts, partials, blockIdx.y * gridDim.x + blockIdx.x);
    }
}

// Any L % 64 == 0: one lane per word of one trajectory, walking all its
// transitions; neighbour words from the caches.
template <bool PAIRED>
__global__ __launch_bounds__(256) void k_loglik_counts(const uint64_t* __restrict__ traj, uint32_t n_traj,
                                                        uint32_t n_lat, uint32_t L, FastDiv divW,
                                                        unsigned long long* __restrict__ counts,
                                                        int64_t* __restrict__ partials) {
    __shared__ int64_t red[12 * 4];
    const uint32_t W = L / 64u;
    const uint32_t n_words = L * W;
    const uint32_t blocks_per_traj = (n_words + blockDim.x - 1) / blockDim.x;
    const uint32_t a = blockIdx.x / blocks_per_traj;
    const uint32_t g = (blockIdx.x % blocks_per_traj) * blockDim.x + threadIdx.x;
    int64_t acc[12], pst[5];
#pragma unroll
    for (int i = 0; i < 12; ++i)
        acc[i] = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i)
        pst[i] = 0;
    const bool live = a < n_traj && g < n_words;
    if (live) {
        const uint32_t j = fdiv(g, divW);
        const uint32_t w = g - j * W;
        const uint32_t down = (j == 0 ? L - 1 : j - 1) * W + w;
        const uint32_t up = (j == L - 1 ? 0 : j + 1) * W + w;
        const uint32_t prev = j * W + (w == 0 ? W - 1 : w - 1);
        const uint32_t next = j * W + (w == W - 1 ? 0 : w + 1);
        const uint64_t* X = traj + (size_t)a * n_lat * n_words;
        uint64_t c = X[g];
        for (uint32_t m = 0; m + 1 < n_lat; ++m) {
            const uint64_t* Xm = X + (size_t)m * n_words;
            const uint64_t y = Xm[n_words + g];
            const bool even = (m & 1u) == 0;
            const uint64_t n1 = Xm[even ? down : up];
            const uint64_t w2 = Xm[even ? prev : next];
            const uint64_t n2 = even ? ((c << 1) | (w2 >> 63)) : ((c >> 1) | (w2 << 63));
            if (PAIRED)
                pair_transition(c, n1, n2, y, pst);
            else
                count_transition(c, n1, n2, y, acc);
            c = y;
        }
    }
    if (PAIRED) {
        int64_t out[6];
        pair_stats(pst, live ? (int64_t)(n_lat - 1) : 0, out);
        flush_counts<6>(out, red, counts, partials, blockIdx.x);
    } else {
        flush_counts<12>(acc, red, counts, partials, blockIdx.x);
    }
}

// ---------------------------------------------------------------------------
// Float-float arithmetic (pairs of binary32, error-free transformations).
// ---------------------------------------------------------------------------
struct ff {
    float hi, lo;
};

__device__ __forceinline__ ff two_sum(float a, float b) {
    const float s = a + b;
    const float bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}

__device__ __forceinline__ ff quick_two_sum(float a, float b) {
    const float s = a + b;
    return {s, b - (s - a)};
}

__device__ __forceinline__ ff two_prod(float a, float b) {
    const float p = a * b;
    return {p, __builtin_fmaf(a, b, -p)};
}

__device__ __forceinline__ ff ff_add(ff x, ff y) {
    ff s = two_sum(x.hi, y.hi);
    ff t = two_sum(x.lo, y.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ ff ff_neg(ff x) { return {-x.hi, -x.lo}; }

__device__ __forceinline__ ff ff_sub(ff x, ff y) { return ff_add(x, ff_neg(y)); }

__device__ __forceinline__ ff ff_mul(ff x, ff y) {
    ff p = two_prod(x.hi, y.hi);
    p.lo += x.hi * y.lo + x.lo * y.hi;
    return quick_two_sum(p.hi, p.lo);
}

__device__ __forceinline__ ff ff_mul_f(ff x, float y) {
    ff p = two_prod(x.hi, y);
    p.lo += x.lo * y;
    return quick_two_sum(p.hi, p.lo);
}

__device__ __forceinline__ ff ff_div(ff x, ff y) {
    const float q1 = x.hi / y.hi;
    ff r = ff_sub(x, ff_mul_f(y, q1));
    const float q2 = r.hi / y.hi;
    r = ff_sub(r, ff_mul_f(y, q2));
    const float q3 = r.hi / y.hi;
    ff q = quick_two_sum(q1, q2);
    return ff_add(q, ff{q3, 0.0f});
}

__device__ __forceinline__ ff ff_from_i64(int64_t v) {
    const float hi = (float)v;
    const float lo = (float)(v - (int64_t)hi);
    return {hi, lo};
}

__device__ __forceinline__ ff ff_ldexp(ff x, int k) { return {ldexpf(x.hi, k), ldexpf(x.lo, k)}; }

// ln 2 = 0.6931471805599453094...: binary32 head and the remainder.
constexpr float kLn2Hi = 0.693147182464599609375f;
constexpr float kLn2Lo = -1.904654323148236e-09f;

// e^x for x <= 0 (x given as float-float): x = k ln2 + r with |r| <= ln2/2,
// e^r by its Taylor series to degree 13 (truncation below 2e-16), then 2^k.
__device__ ff ff_exp_nonpos(ff x) {
    const float k = rintf(x.hi / kLn2Hi);
    ff r = ff_sub(x, two_prod(k, kLn2Hi));
    r = ff_sub(r, ff_mul_f(ff{kLn2Lo, 0.0f}, k));
    // Horner with coefficients 1/i!
    ff inv_fact[14];
    inv_fact[0] = {1.0f, 0.0f};
    for (int i = 1; i < 14; ++i)
        inv_fact[i] = ff_div(inv_fact[i - 1], ff{(float)i, 0.0f});
    ff p = inv_fact[13];
    for (int i = 12; i >= 0; --i)
        p = ff_add(ff_mul(p, r), inv_fact[i]);
    return ff_ldexp(p, (int)k);
}

// log(1 + y) for 0 <= y <= 1: 2 atanh(z), z = y / (2 + y) <= 1/3, by the odd
// series of atanh to 20 terms (truncation below 1e-19).
__device__ ff ff_log1p_unit(ff y) {
    const ff z = ff_div(y, ff_add(ff{2.0f, 0.0f}, y));
    const ff z2 = ff_mul(z, z);
    ff s = ff_div(ff{1.0f, 0.0f}, ff{41.0f, 0.0f});
    for (int i = 19; i >= 0; --i)
        s = ff_add(ff_mul(s, z2), ff_div(ff{1.0f, 0.0f}, ff{(float)(2 * i + 1), 0.0f}));
    return ff_mul_f(ff_mul(z, s), 2.0f);
}

struct ClassTerms {
    ff h;        // field of the class
    ff log2ch;   // log 2cosh h
    ff tanh_h;
    float a, c;  // dh/dJ, dh/dq
};

__device__ ClassTerms class_terms(int idx, float J, float q) {
    const int k = idx >> 1;
    ClassTerms t;
    t.a = (float)(2 * k - 2);
    t.c = (idx & 1) ? 1.0f : -1.0f;
    t.h = two_sum(J * t.a, q * t.c);   // both products are exact
    const ff absh = t.h.hi < 0.0f ? ff_neg(t.h) : t.h;
    const ff y = ff_exp_nonpos(ff_mul_f(absh, -2.0f));   // e^{-2|h|}
    t.log2ch = ff_add(absh, ff_log1p_unit(y));
    ff th = ff_div(ff_sub(ff{1.0f, 0.0f}, y), ff_add(ff{1.0f, 0.0f}, y));
    t.tanh_h = t.h.hi < 0.0f ? ff_neg(th) : th;
    return t;
}

// Class idx's site count N and signed sum D = (drawn +1) - (drawn -1): from
// the 12 counts, or (PAIRED, idx < 3) from the pair statistics, where the pair
// acts as its leader class with N = S_j and D = 2 Z_j - S_j.
template <bool PAIRED>
__device__ __forceinline__ void class_sums(const int64_t* __restrict__ v, int idx, int64_t& D, int64_t& N) {
    if (PAIRED) {
        N = v[idx];
        D = 2 * v[3 + idx] - v[idx];
    } else {
        N = v[2 * idx + 1] + v[2 * idx];
        D = v[2 * idx + 1] - v[2 * idx];
    }
}

template <bool PAIRED>
__global__ void k_loglik_fwd(const int64_t* __restrict__ counts, const float* __restrict__ Jq,
                             float* __restrict__ ll) {
    if (blockIdx.x != 0 || threadIdx.x != 0)
        return;
    const float J = Jq[0], q = Jq[1];
    ff acc = {0.0f, 0.0f};
    for (int idx = 0; idx < (PAIRED ? 3 : 6); ++idx) {
        const ClassTerms t = class_terms(idx, J, q);
        int64_t Di, Ni;
        class_sums<PAIRED>(counts, idx, Di, Ni);
        const ff d = ff_from_i64(Di), N = ff_from_i64(Ni);
        acc = ff_add(acc, ff_sub(ff_mul(d, t.h), ff_mul(N, t.log2ch)));
    }
    ll[0] = acc.hi + acc.lo;
}

template <bool PAIRED>
__global__ void k_loglik_bwd(const int64_t* __restrict__ counts, const float* __restrict__ Jq,
                             const float* __restrict__ g_out, float* __restrict__ grad) {
    if (blockIdx.x != 0 || threadIdx.x != 0)
        return;
    const float J = Jq[0], q = Jq[1];
    ff gJ = {0.0f, 0.0f}, gq = {0.0f, 0.0f};
    for (int idx = 0; idx < (PAIRED ? 3 : 6); ++idx) {
        const ClassTerms t = class_terms(idx, J, q);
        int64_t Di, Ni;
        class_sums<PAIRED>(counts, idx, Di, Ni);
        const ff resid = ff_sub(ff_from_i64(Di), ff_mul(ff_from_i64(Ni), t.tanh_h));
        gJ = ff_add(gJ, ff_mul_f(resid, t.a));
        gq = ff_add(gq, ff_mul_f(resid, t.c));
    }
    const float go = g_out ? g_out[0] : 1.0f;
    const ff rJ = ff_mul_f(gJ, go), rq = ff_mul_f(gq, go);
    grad[0] = rJ.hi + rJ.lo;
    grad[1] = rq.hi + rq.lo;
}

}  // namespace

hipError_t launch_loglik_counts(const void* traj, uint32_t n_traj, uint32_t n_lat, uint32_t L, int64_t* out,
                                bool paired, hipStream_t st, int64_t* partials, size_t partials_words) {
    const uint32_t n_out = paired ? 6u : 12u;
    hipError_t e = launch_fill_i64(out, n_out, 0, st);
    if (e != hipSuccess)
        return e;
    const uint32_t n_words = L * (L / 64u);
    if (n_traj == 0 || n_lat < 2)
        return hipSuccess;
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(out);
    const uint32_t chunks = (n_lat - 1 + kChunk - 1) / kChunk;
    if (n_words <= kStageWords && chunks > 65535u)
        return hipErrorInvalidValue;
    uint64_t blocks;
    if (n_words <= kStageWords)
        blocks = (uint64_t)n_traj * chunks;
    else
        blocks = (uint64_t)((n_words + 255u) / 256u) * n_traj;
    if (blocks > 0x7FFFFFFFull)
        return hipErrorInvalidValue;
    int64_t* part = (partials && n_out * blocks <= partials_words) ? partials : nullptr;
    const uint64_t* X = static_cast<const uint64_t*>(traj);
    const FastDiv divW = make_fastdiv(L / 64u);
    const dim3 grid(n_traj, chunks);
#define SD_LL_LDS(THREADS, WPT, DEPTH_PAIRED, DEPTH_COUNTS)                                                          \
    do {                                                                                                               \
        const bool full = n_words == (THREADS) * (WPT);                                                                \
        if (paired && full)                                                                                            \
            hipLaunchKernelGGL((k_loglik_counts_lds<THREADS, WPT, DEPTH_PAIRED, true, true>), grid, dim3(THREADS), 0, \
                               st, X, n_lat, L, divW, acc, part);                                                      \
        else if (paired)                                                                                               \
            hipLaunchKernelGGL((k_loglik_counts_lds<THREADS, WPT, DEPTH_PAIRED, true, false>), grid, dim3(THREADS),   \
                               0, st, X, n_lat, L, divW, acc, part);                                                   \
        else if (full)                                                                                                 \
            hipLaunchKernelGGL((k_loglik_counts_lds<THREADS, WPT, DEPTH_COUNTS, false, true>), grid, dim3(THREADS),   \
                               0, st, X, n_lat, L, divW, acc, part);                                                   \
        else                                                                                                           \
            hipLaunchKernelGGL((k_loglik_counts_lds<THREADS, WPT, DEPTH_COUNTS, false, false>), grid, dim3(THREADS),  \
                               0, st, X, n_lat, L, divW, acc, part);                                                   \
    } while (0)
    // a lattice of n_words words is spread over THREADS x WPT slots; the ring
    // depth keeps each variant within the registers of its occupancy
    if (n_words <= 64u) {
        SD_LL_LDS(64, 1, 16, 16);
    } else if (n_words <= 256u) {
        SD_LL_LDS(256, 1, 16, 16);
    } else if (n_words <= 1024u) {
        SD_LL_LDS(256, 4, 2, 2);
    } else if (n_words <= kStageWords) {
        SD_LL_LDS(1024, 4, 2, 2);
#undef SD_LL_LDS
    } else {
        if (paired)
            hipLaunchKernelGGL(k_loglik_counts<true>, dim3((uint32_t)blocks), dim3(256), 0, st, X, n_traj, n_lat, L,
                               divW, acc, part);
        else
            hipLaunchKernelGGL(k_loglik_counts<false>, dim3((uint32_t)blocks), dim3(256), 0, st, X, n_traj, n_lat, L,
                               divW, acc, part);
    }
    if (part) {
        if (paired)
            hipLaunchKernelGGL(k_counts_finish<6>, dim3(1), dim3(1024), 0, st, part, (uint32_t)blocks, out);
        else
            hipLaunchKernelGGL(k_counts_finish<12>, dim3(1), dim3(1024), 0, st, part, (uint32_t)blocks, out);
    }
    return hipGetLastError();
}

hipError_t launch_loglik_fwd(const int64_t* stats, bool paired, const float* Jq, float* ll, hipStream_t st) {
    if (paired)
        hipLaunchKernelGGL(k_loglik_fwd<true>, dim3(1), dim3(64), 0, st, stats, Jq, ll);
    else
        hipLaunchKernelGGL(k_loglik_fwd<false>, dim3(1), dim3(64), 0, st, stats, Jq, ll);
    return hipGetLastError();
}

hipError_t launch_loglik_bwd(const int64_t* stats, bool paired, const float* Jq, const float* g_out, float* grad,
                             hipStream_t st) {
    if (paired)
        hipLaunchKernelGGL(k_loglik_bwd<true>, dim3(1), dim3(64), 0, st, stats, Jq, g_out, grad);
    else
        hipLaunchKernelGGL(k_loglik_bwd<false>, dim3(1), dim3(64), 0, st, stats, Jq, g_out, grad);
    return hipGetLastError();
}

}  // namespace sd
