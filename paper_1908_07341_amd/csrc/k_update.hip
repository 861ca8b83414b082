// Half-step kernels of the shaken dynamics and the random initial lattice.
//
// Half-step A (section 2, eq. (15) and the per-site sampling after it): every
// tau_x is drawn at once from the field J(sigma_down + sigma_left) + q sigma_x.
// Half-step B (eq. (16)): every sigma'_x from J(tau_up + tau_right) + q tau_x.
// One lane owns one 64-site group (64 consecutive sites in row-major order):
// it gathers the partner bits c and the two J-neighbour bits n1, n2 of its 64
// sites, draws the eight random planes of the group, compares them bit-sliced
// against the threshold table and resolves the rare undecided sites together
// with the rest of the workgroup.  Half-step B can also fold the observables
// M, A, B of the new pair (sigma', tau) into the same pass, since it already
// holds tau_x, tau_up and tau_right of every site it writes.
#include "sd_kernels.hpp"

namespace sd {

namespace {

constexpr int kTailCap = 1024;

// The 64-bit-word layout when every row is a whole number of 64-word chunks
// (L % 4096 == 0): the 64 words a wavefront handles at once then lie in one
// row, so the row and its neighbour rows are wavefront-uniform addresses
// and the word before (after) a lane's word is the next lower (higher)
// lane's word.  Same bytes as kLayP64; only the half-step kernel tells the
// two apart.
constexpr int kLayP64Rows = 16;

// Partner bits c and neighbour bits n1, n2 of group g (all 64 bits valid for
// every layout except the generic int8 one, which reports its valid mask).
template <int LAYOUT, int WHICH>
__device__ __forceinline__ void gather(const void* src, const Geom& G, uint32_t g, uint64_t& c, uint64_t& n1,
                                       uint64_t& n2, uint64_t& valid) {
    valid = ~0ull;
    if constexpr (LAYOUT == kLayP64 || LAYOUT == kLayP64Rows) {
        const uint64_t* s = static_cast<const uint64_t*>(src);
        const uint32_t W = G.words_row;
        const uint32_t j = fdiv(g, G.div_row);
        const uint32_t w = g - j * W;
        const uint32_t row = j * W;
        c = s[g];
        if constexpr (WHICH == 0) {
            n1 = s[(j == 0 ? G.L - 1 : j - 1) * W + w];                       // down
            uint64_t prev = s[row + (w == 0 ? W - 1 : w - 1)];
            n2 = (c << 1) | (prev >> 63);                                     // left
        } else {
            n1 = s[(j == G.L - 1 ? 0 : j + 1) * W + w];                       // up
            uint64_t next = s[row + (w == W - 1 ? 0 : w + 1)];
            n2 = (c >> 1) | (next << 63);                                     // right
        }
    } else if constexpr (LAYOUT == kLayP32) {
        const uint32_t* s = static_cast<const uint32_t*>(src);
        const uint32_t W = G.words_row;   // 32-bit words per row
        uint32_t cc[2], a[2], b[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t u = 2 * g + h;
            const uint32_t j = fdiv(u, G.div_row);
            const uint32_t w = u - j * W;
            const uint32_t row = j * W;
            const uint32_t x = s[u];
            cc[h] = x;
            if constexpr (WHICH == 0) {
                a[h] = s[(j == 0 ? G.L - 1 : j - 1) * W + w];
                uint32_t prev = s[row + (w == 0 ? W - 1 : w - 1)];
                b[h] = (x << 1) | (prev >> 31);
            } else {
                a[h] = s[(j == G.L - 1 ? 0 : j + 1) * W + w];
                uint32_t next = s[row + (w == W - 1 ? 0 : w + 1)];
                b[h] = (x >> 1) | (next << 31);
            }
        }
        c = (uint64_t)cc[0] | ((uint64_t)cc[1] << 32);
        n1 = (uint64_t)a[0] | ((uint64_t)a[1] << 32);
        n2 = (uint64_t)b[0] | ((uint64_t)b[1] << 32);
    } else if constexpr (LAYOUT == kLayI8Row) {
        const int8_t* s = static_cast<const int8_t*>(src);
        const uint32_t W = G.words_row;   // 64-site groups per row
        const uint32_t j = fdiv(g, G.div_row);
        const uint32_t w = g - j * W;
        const size_t row = (size_t)j * G.L;
        const size_t s0 = row + 64u * w;
        c = load_bits64_i8(s + s0);
        if constexpr (WHICH == 0) {
            const size_t nrow = (size_t)(j == 0 ? G.L - 1 : j - 1) * G.L;
            n1 = load_bits64_i8(s + nrow + 64u * w);
            const int8_t edge = s[row + (w == 0 ? G.L - 1 : 64u * w - 1)];
            n2 = (c << 1) | (edge > 0 ? 1ull : 0ull);
        } else {
            const size_t nrow = (size_t)(j == G.L - 1 ? 0 : j + 1) * G.L;
            n1 = load_bits64_i8(s + nrow + 64u * w);
            const int8_t edge = s[row + (w == W - 1 ? 0 : 64u * w + 64u)];
            n2 = (c >> 1) | (edge > 0 ? (1ull << 63) : 0ull);
        }
    } else if constexpr (LAYOUT == kLayBits) {
        gather_bits<WHICH>(static_cast<const uint64_t*>(src), G.L, G.n_groups, G.div_L, g, c, n1, n2);
    } else {  // kLayI8Any: per-site gather, any L >= 2
        const int8_t* s = static_cast<const int8_t*>(src);
        const uint32_t s0 = 64u * g;
        const uint32_t nv = G.n_sites - s0 < 64u ? G.n_sites - s0 : 64u;
        uint32_t j = fdiv(s0, G.div_L);
        uint32_t i = s0 - j * G.L;
        c = 0; n1 = 0; n2 = 0;
        for (uint32_t b = 0; b < nv; ++b) {
            const size_t row = (size_t)j * G.L;
            const uint64_t bit = 1ull << b;
            if (s[row + i] > 0) c |= bit;
            if constexpr (WHICH == 0) {
                if (s[(size_t)(j == 0 ? G.L - 1 : j - 1) * G.L + i] > 0) n1 |= bit;
                if (s[row + (i == 0 ? G.L - 1 : i - 1)] > 0) n2 |= bit;
            } else {
                if (s[(size_t)(j == G.L - 1 ? 0 : j + 1) * G.L + i] > 0) n1 |= bit;
                if (s[row + (i == G.L - 1 ? 0 : i + 1)] > 0) n2 |= bit;
            }
            if (++i == G.L) { i = 0; ++j; }
        }
        valid = nv == 64u ? ~0ull : ((1ull << nv) - 1ull);
    }
}

template <int LAYOUT>
__device__ __forceinline__ void scatter(void* dst, const Geom& /*G*/, uint32_t g, uint64_t bits, uint64_t valid) {
    if constexpr (LAYOUT == kLayP64 || LAYOUT == kLayP64Rows || LAYOUT == kLayBits) {
        static_cast<uint64_t*>(dst)[g] = bits;
    } else if constexpr (LAYOUT == kLayP32) {
        uint32_t* d = static_cast<uint32_t*>(dst);
        d[2 * g] = (uint32_t)bits;
        d[2 * g + 1] = (uint32_t)(bits >> 32);
    } else if constexpr (LAYOUT == kLayI8Row) {
        store_bits64_i8(static_cast<int8_t*>(dst) + (size_t)64u * g, bits);
    } else {
        int8_t* d = static_cast<int8_t*>(dst) + (size_t)64u * g;
        for (int b = 0; b < 64; ++b)
            if ((valid >> b) & 1ull)
                d[b] = ((bits >> b) & 1ull) ? 1 : -1;
    }
}

// Partner and neighbour bits of the 64-bit-word layouts (P64, I8Row) for the
// word at row j, column word w of the row.
template <int LAYOUT, int WHICH>
__device__ __forceinline__ void gather_row(const void* src, const Geom& G, uint32_t j, uint32_t w, uint64_t& c,
                                           uint64_t& n1, uint64_t& n2) {
    const uint32_t W = G.words_row;
    if constexpr (LAYOUT == kLayP64) {
        const uint64_t* s = static_cast<const uint64_t*>(src);
        const uint32_t row = j * W;
        c = s[row + w];
        const uint32_t c_lo = (uint32_t)c, c_hi = (uint32_t)(c >> 32);
        if constexpr (WHICH == 0) {
            n1 = s[(j == 0 ? G.L - 1 : j - 1) * W + w];                                  // down
            const uint32_t prev_hi =
                reinterpret_cast<const uint32_t*>(s + row + (w == 0 ? W - 1 : w - 1))[1];
            n2 = (uint64_t)__builtin_amdgcn_alignbit(c_lo, prev_hi, 31) |                 // left
                 ((uint64_t)__builtin_amdgcn_alignbit(c_hi, c_lo, 31) << 32);
        } else {
            n1 = s[(j == G.L - 1 ? 0 : j + 1) * W + w];                                  // up
            const uint32_t next_lo = reinterpret_cast<const uint32_t*>(s + row + (w == W - 1 ? 0 : w + 1))[0];
            n2 = (uint64_t)__builtin_amdgcn_alignbit(c_hi, c_lo, 1) |                     // right
                 ((uint64_t)__builtin_amdgcn_alignbit(next_lo, c_hi, 1) << 32);
        }
    } else {
        static_assert(LAYOUT == kLayI8Row, "row walk needs 64-site words");
        const int8_t* s = static_cast<const int8_t*>(src);
        const size_t row = (size_t)j * G.L;
        c = load_bits64_i8(s + row + 64u * w);
        if constexpr (WHICH == 0) {
            n1 = load_bits64_i8(s + (size_t)(j == 0 ? G.L - 1 : j - 1) * G.L + 64u * w);
            const int8_t edge = s[row + (w == 0 ? G.L - 1 : 64u * w - 1)];
            n2 = (c << 1) | (edge > 0 ? 1ull : 0ull);
        } else {
            n1 = load_bits64_i8(s + (size_t)(j == G.L - 1 ? 0 : j + 1) * G.L + 64u * w);
            const int8_t edge = s[row + (w == W - 1 ? 0 : 64u * w + 64u)];
            n2 = (c >> 1) | (edge > 0 ? (1ull << 63) : 0ull);
        }
    }
}

// 64-bit word at a wavefront-uniform base plus a 32-bit byte offset, the
// form the global load and store instructions take directly (scalar base,
// vector offset), with no 64-bit address arithmetic per lane.
__device__ __forceinline__ uint64_t load_at(const uint64_t* base, uint32_t byte_off) {
    return *reinterpret_cast<const uint64_t*>(reinterpret_cast<const char*>(base) + byte_off);
}

__device__ __forceinline__ void store_at(uint64_t* base, uint32_t byte_off, uint64_t v) {
    *reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

// One half-step.  Each wavefront walks tiles of kWaveTile consecutive words;
// lane l owns words l, l + 64, ... of its tile (coalesced loads and stores).
// For every word it draws the eight planes and compares them (decided sites
// in lt, undecided ones in und).  A word with undecided sites (about 22% of
// them at 1/256 per site) claims a slot of the wavefront's LDS list through a
// ballot and stores und and its tile index there; the list has room for every
// word of the tile.  Then lane e resolves list entries e, e + 64, ...: it
// reloads the word's partner and neighbour bits (cache hits), draws one tail
// per undecided site and leaves the decided +1 sites in the slot, which the
// owner ors into its word before the store.  All of this is local to the
// wavefront, so the tile loop has no workgroup barrier.
// obs (half-step B only, may be null) receives the observable contributions
// of the written pair through 64-bit atomics; it must hold zeros (or earlier
// partial sums of the same record) before the launch.
// Words per lane and tile: 4 for the paired compare on bit-packed layouts,
// 2 where the general compare or the int8 loads need more registers.
constexpr int words_per_lane(int layout, bool paired) {
    return (paired && (layout == kLayP64 || layout == kLayP64Rows || layout == kLayP32 || layout == kLayBits)) ? 4
                                                                                                             : 2;
}
constexpr int kMaxWordsPerLane = 4;
constexpr uint32_t kMaxWaveTile = 64u * kMaxWordsPerLane;
constexpr int kWavesPerBlock = 4;

struct WaveList {
    uint64_t und[kMaxWaveTile + 1];   // undecided sites on entry, decided +1 sites on exit;
                                      // entry kMaxWaveTile stays zero (slot of unlisted words)
    uint16_t local[kMaxWaveTile];     // tile index of the listed word
};

// Words whose second and later undecided sites wait for the workgroup's
// last pass (64-bit word layouts, whole tiles).
constexpr uint32_t kPoolCap = 256;
struct TailPool {
    uint32_t count;
    uint32_t g[kPoolCap];
    uint64_t und[kPoolCap];
};

struct HalfStepScratch {
    WaveList list[kWavesPerBlock];
    uint32_t T24[6];               // tail thresholds of the classes (paired_tail in the paired form)
    TailPool pool;
};

// Layouts whose words are the lattice's 64-bit words: a decided +1 site can be
// or-ed into a stored word later.
constexpr bool pooled_layout(int layout) { return layout == kLayP64 || layout == kLayP64Rows || layout == kLayBits; }

struct ObsAcc {
    int64_t pc = 0, d_up = 0, d_right = 0, d_self = 0, nsites = 0;
};

// Decided +1 sites among the undecided sites u of the word starting at site0.
__device__ __forceinline__ uint64_t resolve_word(const DrawParams& dp, const uint32_t* T24, uint64_t u, uint64_t c,
                                                 uint64_t n1, uint64_t n2, uint32_t site0) {
    uint64_t r = 0;
    while (u) {
        const int b = __ffsll((unsigned long long)u) - 1;
        u &= u - 1;
        if (draw_tail24(dp, site0 + (uint32_t)b) < T24[class_at(c, n1, n2, b)])
            r |= 1ull << b;
    }
    return r;
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One tile of 64 * WPL words.  FULL: every word of the tile holds 64 sites
// of the lattice (no bounds checks).
template <int LAYOUT, int WHICH, bool PAIRED, bool COMPLEMENT, bool OBS, bool FULL, int WPL>
__device__ __forceinline__ void half_step_tile(const void* __restrict__ src, void* __restrict__ dst, const Geom& G,
                                               const DrawParams& dp, const PlaneMasks& pm, const uint32_t* T24,
                                               WaveList& wl, uint32_t tile0, uint32_t lane, ObsAcc& acc,
                                               TailPool& pool) {
    constexpr int kWordsPerLane = WPL;
    constexpr bool kRowWalk = LAYOUT == kLayP64 || LAYOUT == kLayI8Row;
    uint64_t lt[kWordsPerLane], c[kWordsPerLane], n1[kWordsPerLane], n2[kWordsPerLane], valid[kWordsPerLane];
    uint32_t slot[kWordsPerLane];
    // all loads of the tile first, so that their latency overlaps the Philox
    // work of the first words
    if constexpr (LAYOUT == kLayP64Rows) {
        static_assert(FULL, "row-chunk tiles are whole");
        // tile0 is wavefront-uniform: chunk k of the tile is words w0 .. w0 + 63
        // of row j, loaded as one uniform row address plus the lane offset
        const uint64_t* s = static_cast<const uint64_t*>(src);
        const uint32_t W = G.words_row;
#pragma unroll
        for (int k = 0; k < kWordsPerLane; ++k) {
            const uint32_t g0 = tile0 + 64u * k;
            const uint32_t j = fdiv(g0, G.div_row);
            const uint32_t w0 = g0 - j * W;
            const uint64_t* row = s + (size_t)j * W;
            const uint32_t off = 8u * (w0 + lane);
            c[k] = load_at(row, off);
            const uint32_t c_lo = (uint32_t)c[k], c_hi = (uint32_t)(c[k] >> 32);
            if constexpr (WHICH == 0) {
                const uint64_t* nrow = s + (size_t)(j == 0 ? G.L - 1 : j - 1) * W;
                n1[k] = load_at(nrow, off);                                                // down
                // high half of the word before: the lower lane's, the row's
                // wrap-around word for lane 0
                const uint32_t edge = reinterpret_cast<const uint32_t*>(row + (w0 == 0 ? W - 1 : w0 - 1))[1];
                const uint32_t prev_hi = (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)c_hi, 0x138, 0xF,
                                                                               0xF, false);   // wave_shr:1
                n2[k] = (uint64_t)__builtin_amdgcn_alignbit(c_lo, prev_hi, 31) |            // left
                        ((uint64_t)__builtin_amdgcn_alignbit(c_hi, c_lo, 31) << 32);
            } else {
                const uint64_t* nrow = s + (size_t)(j == G.L - 1 ? 0 : j + 1) * W;
                n1[k] = load_at(nrow, off);                                                // up
                // low half of the word after: the higher lane's, the row's
                // wrap-around word for lane 63
                const uint32_t edge = reinterpret_cast<const uint32_t*>(row + (w0 + 64u == W ? 0 : w0 + 64u))[0];
                const uint32_t next_lo = (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)c_lo, 0x130, 0xF,
                                                                               0xF, false);   // wave_shl:1
                n2[k] = (uint64_t)__builtin_amdgcn_alignbit(c_hi, c_lo, 1) |                // right
                        ((uint64_t)__builtin_amdgcn_alignbit(next_lo, c_hi, 1) << 32);
            }
            valid[k] = ~0ull;
        }
    } else if constexpr (kRowWalk) {
        const uint32_t g0 = tile0 + lane;
        uint32_t j = fdiv(g0, G.div_row);
        uint32_t w = g0 - j * G.words_row;
#pragma unroll
        for (int k = 0; k < kWordsPerLane; ++k) {
            const uint32_t g = g0 + 64u * k;
            if (FULL || g < G.n_groups) {
                gather_row<LAYOUT, WHICH>(src, G, j, w, c[k], n1[k], n2[k]);
                valid[k] = ~0ull;
            } else {
                c[k] = n1[k] = n2[k] = valid[k] = 0;
            }
            w += G.step_cols;
            j += G.step_rows;
            if (w >= G.words_row) {
                w -= G.words_row;
                ++j;
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < kWordsPerLane; ++k) {
            const uint32_t g = tile0 + lane + 64u * k;
            c[k] = n1[k] = n2[k] = valid[k] = 0;
            if (FULL || g < G.n_groups)
                gather<LAYOUT, WHICH>(src, G, g, c[k], n1[k], n2[k], valid[k]);
            if (FULL)
                valid[k] = ~0ull;
        }
    }
    uint32_t listed = 0;   // wavefront-uniform list length
    uint32_t chain = 0;    // orders the words' Philox work, see below
#pragma unroll
    for (int k = 0; k < kWordsPerLane; ++k) {
        uint32_t g = tile0 + lane + 64u * k;
        // The words of a tile are independent; left alone the compiler
        // interleaves all their Philox evaluations and needs far more VGPRs.
        // An empty asm making g depend on the previous word's result keeps
        // them one after the other.
        asm volatile("" : "+v"(g) : "v"(chain));
        uint64_t P[8];
        draw_planes(dp, (FULL || g < G.n_groups) ? g : 0u, P);
        const WordDraw wd = compare_planes<PAIRED, COMPLEMENT>(P, c[k], n1[k], n2[k], pm);
        lt[k] = wd.lt;
        chain = (uint32_t)wd.lt;
        const uint64_t und = FULL ? wd.und : (wd.und & valid[k]);
        const uint64_t need = __ballot(und != 0);
        slot[k] = kMaxWaveTile;   // the zero entry
        if (und != 0) {
            const uint32_t e = listed + __builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
            slot[k] = e;
            wl.und[e] = und;
            wl.local[e] = (uint16_t)(lane + 64u * k);
        }
        listed += (uint32_t)__popcll(need);
    }
    wave_sync_lds();
    // Every listed word has one undecided site or more (two or more in about
    // one word of eight).  Resolving all of a word's sites here would run as
    // many tail passes as the most crowded word has sites; on whole tiles of
    // the 64-bit word layouts only the first site is resolved here, and the
    // rest of the word goes to the workgroup's pool, resolved once at the end
    // of the launch and or-ed into the stored word.
    constexpr bool kPool = FULL && pooled_layout(LAYOUT);
    for (uint32_t e = lane; e < listed; e += 64u) {
        const uint32_t g = tile0 + wl.local[e];
        uint64_t cc, a1, a2, v;
        gather<LAYOUT, WHICH>(src, G, g, cc, a1, a2, v);
        const uint64_t u = wl.und[e];
        if constexpr (kPool) {
            const uint64_t first = u & (0ull - u);
            const uint64_t rest = u ^ first;
            uint64_t r = resolve_word(dp, T24, first, cc, a1, a2, 64u * g);
            if (rest) {
                const uint32_t slot = atomicAdd(&pool.count, 1u);
                if (slot < kPoolCap) {
                    pool.g[slot] = g;
                    pool.und[slot] = rest;
                } else {
                    r |= resolve_word(dp, T24, rest, cc, a1, a2, 64u * g);
                }
            }
            wl.und[e] = r;
        } else {
            wl.und[e] = resolve_word(dp, T24, u, cc, a1, a2, 64u * g);
        }
    }
    wave_sync_lds();
#pragma unroll
    for (int k = 0; k < kWordsPerLane; ++k) {
        const uint32_t g = tile0 + lane + 64u * k;
        const uint64_t bits = FULL ? (lt[k] | wl.und[slot[k]]) : ((lt[k] | wl.und[slot[k]]) & valid[k]);
        if (FULL || g < G.n_groups) {
            if constexpr (LAYOUT == kLayP64Rows)
                store_at(static_cast<uint64_t*>(dst) + (tile0 + 64u * k), 8u * lane, bits);
            else
                scatter<LAYOUT>(dst, G, g, bits, valid[k]);
            if constexpr (OBS) {
                acc.pc += __popcll(bits);
                acc.d_up += __popcll((bits ^ n1[k]) & valid[k]);
                acc.d_right += __popcll((bits ^ n2[k]) & valid[k]);
                acc.d_self += __popcll((bits ^ c[k]) & valid[k]);
                acc.nsites += __popcll(valid[k]);
            }
        }
    }
    // the owners' reads above precede, in this wavefront's program order, the
    // next tile's list writes
    wave_sync_lds();
}

// One half-step of one chain by the workgroups block = 0 .. n_blocks - 1 of
// a launch, each wavefront walking tiles of 64 * WPL words.
// OBS (half-step B only): the workgroup sums of (#+1, #differences to the
// up and right neighbours, #differences to the partner, #sites) go to
// partials[4 * block ...] when partials is non-null (a finishing launch turns
// them into M, A, B), else straight into obs through 64-bit atomics.
template <int LAYOUT, int WHICH, bool PAIRED, bool COMPLEMENT, bool OBS, int WPL>
__device__ __forceinline__ void half_step_body(const void* __restrict__ src, void* __restrict__ dst, const Geom& G,
                                               const DrawParams& dp, int64_t* __restrict__ obs,
                                               int64_t* __restrict__ partials, uint32_t block, uint32_t n_blocks,
                                               HalfStepScratch& sh, int64_t* red) {
    static_assert(!OBS || WHICH == 1, "observables are folded into half-step B");
    constexpr uint32_t kWaveTile = 64u * WPL;
    ObsAcc acc;
    const PlaneMasks pm = make_plane_masks<PAIRED>(dp);
    const uint32_t lane = threadIdx.x & 63u;
    WaveList& wl = sh.list[threadIdx.x >> 6];
    if (lane == 0)
        wl.und[kMaxWaveTile] = 0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < 6; ++i)
            sh.T24[i] = PAIRED ? paired_tail(dp.T, i) : dp.T[i] & 0xFFFFFFu;
        sh.pool.count = 0;
    }
    __syncthreads();
    const uint32_t n_tiles = (G.n_groups + kWaveTile - 1) / kWaveTile;
    // tiles whose every word holds 64 lattice sites
    const uint32_t n_full = (uint32_t)((uint64_t)G.n_sites / (64ull * kWaveTile));
    // the wavefront's index in the workgroup, as a uniform value (tile
    // origins then stay in scalar registers)
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr int kPartLayout = LAYOUT == kLayP64Rows ? kLayP64 : LAYOUT;
    for (uint32_t tile = block * kWavesPerBlock + wave; tile < n_tiles; tile += n_blocks * kWavesPerBlock) {
        if (tile < n_full) {
            half_step_tile<LAYOUT, WHICH, PAIRED, COMPLEMENT, OBS, true, WPL>(src, dst, G, dp, pm, sh.T24, wl,
                                                                              tile * kWaveTile, lane, acc, sh.pool);
        } else {
            // the last, partial tile: 64 words at a time, with bounds checks
            for (uint32_t sub = tile * kWaveTile; sub < (tile + 1) * kWaveTile; sub += 64u)
                half_step_tile<kPartLayout, WHICH, PAIRED, COMPLEMENT, OBS, false, 1>(src, dst, G, dp, pm, sh.T24,
                                                                                       wl, sub, lane, acc, sh.pool);
        }
    }
    if constexpr (pooled_layout(LAYOUT)) {
        // the pool's sites: every word of the workgroup is stored (each
        // wavefront waits for its stores before the barrier), so the decided
        // +1 sites are or-ed into the words in memory; with observables, the
        // owner counted those sites as -1 and the resolver adds the difference
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (wave == 0) {
            const uint32_t n_pool = sh.pool.count < kPoolCap ? sh.pool.count : kPoolCap;
            uint64_t* d = static_cast<uint64_t*>(dst);
            for (uint32_t e = lane; e < n_pool; e += 64u) {
                const uint32_t g = sh.pool.g[e];
                uint64_t cc, a1, a2, v;
                gather<kPartLayout, WHICH>(src, G, g, cc, a1, a2, v);
                const uint64_t r = resolve_word(dp, sh.T24, sh.pool.und[e], cc, a1, a2, 64u * g);
                if (r) {
                    atomicOr(reinterpret_cast<unsigned long long*>(d + g), (unsigned long long)r);
                    if constexpr (OBS) {
                        const int64_t n = __popcll(r);
                        acc.pc += n;
                        acc.d_up += n - 2 * __popcll(r & a1);
                        acc.d_right += n - 2 * __popcll(r & a2);
                        acc.d_self += n - 2 * __popcll(r & cc);
                    }
                }
            }
        }
    }
    if constexpr (OBS) {
        int64_t v[4] = {acc.pc, acc.d_up + acc.d_right, acc.d_self, acc.nsites};
        block_sum_i64<4>(v, red);
        if (threadIdx.x == 0 && partials) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                partials[4u * block + i] = v[i];
        } else if (threadIdx.x == 0) {
            const int64_t n = v[3];
            atomicAdd(reinterpret_cast<unsigned long long*>(obs + 0), (unsigned long long)(2 * v[0] - n));
            atomicAdd(reinterpret_cast<unsigned long long*>(obs + 1), (unsigned long long)(2 * n - 2 * v[1]));
            atomicAdd(reinterpret_cast<unsigned long long*>(obs + 2), (unsigned long long)(n - 2 * v[2]));
        }
    }
}

// The half-step kernel, held to six wavefronts per SIMD (80 VGPRs) where that
// costs no scratch spills (the plain half-steps on 64- and 32-bit words with
// the paired compare), and left to the compiler's register count otherwise.
template <int LAYOUT, int WHICH, bool PAIRED, bool COMPLEMENT, bool OBS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_half_step(
    const void* __restrict__ src, void* __restrict__ dst, Geom G, DrawParams dp, int64_t* __restrict__ obs,
    int64_t* __restrict__ partials) {
    __shared__ HalfStepScratch sh;
    __shared__ int64_t red[4 * 4];
    half_step_body<LAYOUT, WHICH, PAIRED, COMPLEMENT, OBS, words_per_lane(LAYOUT, PAIRED)>(
        src, dst, G, dp, obs, partials, blockIdx.x, gridDim.x, sh, red);
}

template <int LAYOUT, int WHICH, bool PAIRED, bool COMPLEMENT, bool OBS>
__global__ __launch_bounds__(256) void k_half_step_free(const void* __restrict__ src, void* __restrict__ dst, Geom G,
                                                        DrawParams dp, int64_t* __restrict__ obs,
                                                        int64_t* __restrict__ partials) {
    __shared__ HalfStepScratch sh;
    __shared__ int64_t red[4 * 4];
    half_step_body<LAYOUT, WHICH, PAIRED, COMPLEMENT, OBS, words_per_lane(LAYOUT, PAIRED)>(
        src, dst, G, dp, obs, partials, blockIdx.x, gridDim.x, sh, red);
}

constexpr bool six_waves(int layout, bool paired, bool obs) {
    return paired && !obs && (layout == kLayP64 || layout == kLayP64Rows || layout == kLayP32);
}

// Several chains of one size advanced together: workgroups
// chain * blocks_per_chain .. (chain + 1) * blocks_per_chain - 1 take the
// half-step of chain `chain`, with its own lattices, threshold table and
// stream id (the per-chain values are wavefront-uniform kernel arguments).
// Tiles of 64 words (one word per lane) give lattices of a few thousand
// words enough wavefronts.  Partial sums of recorded steps go to
// partials[4 * workgroup ...], chain-major.
template <int LAYOUT, int WHICH, bool PAIRED, bool COMPLEMENT, bool OBS>
__global__ __launch_bounds__(256) void k_half_step_many(ManyChains mc, Geom G, DrawParams base,
                                                        int64_t* __restrict__ partials) {
    __shared__ HalfStepScratch sh;
    __shared__ int64_t red[4 * 4];
    const uint32_t chain = blockIdx.x / mc.blocks_per_chain;
    const uint32_t block = blockIdx.x - chain * mc.blocks_per_chain;
    DrawParams dp = base;
#pragma unroll
    for (int i = 0; i < 6; ++i)
        dp.T[i] = mc.T[chain][i];
    dp.stream = mc.stream[chain];
    half_step_body<LAYOUT, WHICH, PAIRED, COMPLEMENT, OBS, 1>(
        WHICH == 0 ? mc.sigma[chain] : mc.tau[chain], WHICH == 0 ? mc.tau[chain] : mc.sigma[chain], G, dp, nullptr,
        partials + 4u * (size_t)chain * mc.blocks_per_chain, block, mc.blocks_per_chain, sh, red);
}

// Random initial lattice: site s is +1 iff r_s(t = 0, tag 1) < P, the same
// threshold for every site (all six table entries equal P).
template <int LAYOUT>
__global__ __launch_bounds__(256) void k_init_random(void* __restrict__ dst, Geom G, DrawParams dp) {
    __shared__ TailScratch<kTailCap> tails;
    const PlaneMasks pm = make_plane_masks<false>(dp);
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = blockIdx.x * blockDim.x; base < G.n_groups; base += stride) {
        const uint32_t g = base + threadIdx.x;
        const bool active = g < G.n_groups;
        uint64_t valid = 0;
        if (active) {
            const uint32_t s0 = 64u * g;
            const uint32_t nv = G.n_sites - s0 < 64u ? G.n_sites - s0 : 64u;
            valid = nv == 64u ? ~0ull : ((1ull << nv) - 1ull);
        }
        uint64_t P[8];
        draw_planes(dp, active ? g : 0u, P);
        WordDraw wd = compare_planes<false, false>(P, 0, 0, 0, pm);
        uint64_t lt = wd.lt;
        resolve_tails<kTailCap>(lt, wd.und & valid, 0, 0, 0, 64u * g, dp, tails);
        if (active)
            scatter<LAYOUT>(dst, G, g, lt & valid, valid);
    }
}

template <int LAYOUT>
__global__ __launch_bounds__(256) void k_init_const(void* __restrict__ dst, Geom G, uint32_t up) {
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint64_t bits = up ? ~0ull : 0ull;
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < G.n_groups; g += stride) {
        const uint32_t s0 = 64u * g;
        const uint32_t nv = G.n_sites - s0 < 64u ? G.n_sites - s0 : 64u;
        const uint64_t valid = nv == 64u ? ~0ull : ((1ull << nv) - 1ull);
        scatter<LAYOUT>(dst, G, g, bits & valid, valid);
    }
}

// Sums the per-workgroup partials of observables launches into records of
// obs (M, A, B): workgroup r adds the n_blocks partials at partials + r * stride
// into record r.
__global__ __launch_bounds__(1024) void k_obs_finish(const int64_t* __restrict__ partials, uint32_t n_blocks,
                                                     uint32_t stride, int64_t* __restrict__ obs) {
    __shared__ int64_t red[4 * 16];
    const int64_t* p = partials + (size_t)blockIdx.x * stride;
    int64_t* o = obs + 3u * blockIdx.x;
    int64_t v[4] = {0, 0, 0, 0};
    for (uint32_t b = threadIdx.x; b < n_blocks; b += blockDim.x)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            v[i] += p[4u * b + i];
    block_sum_i64<4>(v, red);
    if (threadIdx.x == 0) {
        const int64_t n = v[3];
        o[0] += 2 * v[0] - n;
        o[1] += 2 * n - 2 * v[1];
        o[2] += n - 2 * v[2];
    }
}

// Records of several chains: workgroup (r, a) = (blockIdx.x / n_chains,
// blockIdx.x % n_chains) adds the n_blocks partials at
// partials + r * stride + 4 * a * n_blocks into record r of chain a,
// obs[a * obs_chain + 3 * (rec0 + r) ...].
__global__ __launch_bounds__(256) void k_obs_finish_many(const int64_t* __restrict__ partials, uint32_t n_blocks,
                                                         uint32_t n_chains, uint32_t stride, int64_t* __restrict__ obs,
                                                         uint64_t obs_chain, uint32_t rec0) {
    __shared__ int64_t red[4 * 4];
    const uint32_t r = blockIdx.x / n_chains, a = blockIdx.x - r * n_chains;
    const int64_t* p = partials + (size_t)r * stride + 4u * (size_t)a * n_blocks;
    int64_t v[4] = {0, 0, 0, 0};
    for (uint32_t b = threadIdx.x; b < n_blocks; b += blockDim.x)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            v[i] += p[4u * b + i];
    block_sum_i64<4>(v, red);
    if (threadIdx.x == 0) {
        int64_t* o = obs + a * obs_chain + 3u * (size_t)(rec0 + r);
        const int64_t n = v[3];
        o[0] = 2 * v[0] - n;
        o[1] = 2 * n - 2 * v[1];
        o[2] = n - 2 * v[2];
    }
}

__global__ void k_fill_i64(int64_t* __restrict__ p, size_t n, int64_t v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

uint32_t grid_for(uint32_t n_groups) {
    uint32_t blocks = (n_groups + 255u) / 256u;
    return blocks < kMaxBlocks ? (blocks ? blocks : 1u) : kMaxBlocks;
}

}  // namespace

template <int LAY, int WHICH, bool PAIRED, bool COMPLEMENT, bool OBS>
void launch_half_step_kernel(dim3 grid, dim3 block, hipStream_t st, const void* src, void* dst, const Geom& G,
                             const DrawParams& dp, int64_t* obs, int64_t* partials) {
    if constexpr (six_waves(LAY, PAIRED, OBS))
        hipLaunchKernelGGL((k_half_step<LAY, WHICH, PAIRED, COMPLEMENT, OBS>), grid, block, 0, st, src, dst, G, dp,
                           obs, partials);
    else
        hipLaunchKernelGGL((k_half_step_free<LAY, WHICH, PAIRED, COMPLEMENT, OBS>), grid, block, 0, st, src, dst,
                           G, dp, obs, partials);
}

template <int LAY, int WHICH, bool OBS>
void launch_half_step_mode(bool paired, bool complement, dim3 grid, dim3 block, hipStream_t st, const void* src,
                           void* dst, const Geom& G, const DrawParams& dp, int64_t* obs, int64_t* partials) {
    if (paired && !complement)
        launch_half_step_kernel<LAY, WHICH, true, false, OBS>(grid, block, st, src, dst, G, dp, obs, partials);
    else if (paired)
        launch_half_step_kernel<LAY, WHICH, true, true, OBS>(grid, block, st, src, dst, G, dp, obs, partials);
    else if (!complement)
        launch_half_step_kernel<LAY, WHICH, false, false, OBS>(grid, block, st, src, dst, G, dp, obs, partials);
    else
        launch_half_step_kernel<LAY, WHICH, false, true, OBS>(grid, block, st, src, dst, G, dp, obs, partials);
}

uint32_t half_step_blocks(int layout, const Geom& G, bool paired, uint32_t max_blocks) {
    // one workgroup per four wavefront tiles; at most kMaxBlocks by default,
    // at most max_blocks when the caller gives a cap
    const uint32_t wave_tile = 64u * words_per_lane(layout, paired);
    const uint32_t tiles = (G.n_groups + wave_tile - 1) / wave_tile;
    uint32_t blocks = (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    blocks = blocks ? blocks : 1u;
    const uint32_t cap = max_blocks ? max_blocks : kMaxBlocks;
    return blocks > cap ? cap : blocks;
}

hipError_t launch_obs_finish(const int64_t* partials, uint32_t n_blocks, uint32_t n_rec, uint32_t stride,
                             int64_t* obs, hipStream_t st) {
    hipLaunchKernelGGL(k_obs_finish, dim3(n_rec), dim3(1024), 0, st, partials, n_blocks, stride, obs);
    return hipGetLastError();
}

hipError_t launch_half_step(int layout, int which, const void* src, void* dst, const Geom& G, const DrawParams& dp,
                            int64_t* obs, hipStream_t st, uint32_t max_blocks, int64_t* partials, bool general,
                            bool finish) {
    const bool paired = !general && thresholds_paired(dp.T);
    const uint32_t blocks = half_step_blocks(layout, G, paired, max_blocks);
    const dim3 grid(blocks), block(256);
    const bool complement = dp.rng_xor != 0;
#define SD_HALF(LAY)                                                                                       \
    case LAY:                                                                                              \
        if (which == 0)                                                                                    \
            launch_half_step_mode<LAY, 0, false>(paired, complement, grid, block, st, src, dst, G, dp,      \
                                                 nullptr, nullptr);                                        \
        else if (obs == nullptr)                                                                           \
            launch_half_step_mode<LAY, 1, false>(paired, complement, grid, block, st, src, dst, G, dp,      \
                                                 nullptr, nullptr);                                        \
        else                                                                                               \
            launch_half_step_mode<LAY, 1, true>(paired, complement, grid, block, st, src, dst, G, dp, obs,  \
                                                partials);                                                 \
        break;
    const int klay = (layout == kLayP64 && G.words_row % 64u == 0) ? kLayP64Rows : layout;
    switch (klay) {
        SD_HALF(kLayP64Rows)
        SD_HALF(kLayP64)
        SD_HALF(kLayP32)
        SD_HALF(kLayI8Row)
        SD_HALF(kLayI8Any)
        SD_HALF(kLayBits)
        default:
            return hipErrorInvalidValue;
    }
#undef SD_HALF
    if (which == 1 && obs != nullptr && partials != nullptr && finish)
        hipLaunchKernelGGL(k_obs_finish, dim3(1), dim3(1024), 0, st, partials, blocks, 0u, obs);
    return hipGetLastError();
}

template <int LAY, int WHICH, bool OBS>
void launch_many_mode(bool paired, bool complement, dim3 grid, hipStream_t st, const ManyChains& mc, const Geom& G,
                      const DrawParams& dp, int64_t* partials) {
    if (paired && !complement)
        hipLaunchKernelGGL((k_half_step_many<LAY, WHICH, true, false, OBS>), grid, dim3(256), 0, st, mc, G, dp,
                           partials);
    else if (paired)
        hipLaunchKernelGGL((k_half_step_many<LAY, WHICH, true, true, OBS>), grid, dim3(256), 0, st, mc, G, dp,
                           partials);
    else if (!complement)
        hipLaunchKernelGGL((k_half_step_many<LAY, WHICH, false, false, OBS>), grid, dim3(256), 0, st, mc, G, dp,
                           partials);
    else
        hipLaunchKernelGGL((k_half_step_many<LAY, WHICH, false, true, OBS>), grid, dim3(256), 0, st, mc, G, dp,
                           partials);
}

uint32_t many_blocks_per_chain(const Geom& G) {
    const uint32_t tiles = (G.n_groups + 63u) / 64u;
    const uint32_t blocks = (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    return blocks < kMaxBlocks ? (blocks ? blocks : 1u) : kMaxBlocks;
}

hipError_t launch_half_step_many(int layout, int which, const ManyChains& mc, const Geom& G, const DrawParams& base,
                                 bool paired, int64_t* partials, hipStream_t st) {
    const dim3 grid(mc.n_chains * mc.blocks_per_chain);
    const bool complement = base.rng_xor != 0;
    const int klay = (layout == kLayP64 && G.words_row % 64u == 0) ? kLayP64Rows : layout;
#define SD_MANY(LAY)                                                                                       \
    case LAY:                                                                                              \
        if (which == 0)                                                                                    \
            launch_many_mode<LAY, 0, false>(paired, complement, grid, st, mc, G, base, nullptr);          \
        else if (partials == nullptr)                                                                      \
            launch_many_mode<LAY, 1, false>(paired, complement, grid, st, mc, G, base, nullptr);          \
        else                                                                                               \
            launch_many_mode<LAY, 1, true>(paired, complement, grid, st, mc, G, base, partials);          \
        break;
    switch (klay) {
        SD_MANY(kLayP64Rows)
        SD_MANY(kLayP64)
        SD_MANY(kLayP32)
        SD_MANY(kLayI8Row)
        SD_MANY(kLayI8Any)
        SD_MANY(kLayBits)
        default:
            return hipErrorInvalidValue;
    }
#undef SD_MANY
    return hipGetLastError();
}

hipError_t launch_obs_finish_many(const int64_t* partials, uint32_t n_blocks, uint32_t n_chains, uint32_t n_rec,
                                  uint32_t stride, int64_t* obs, uint64_t obs_chain, uint32_t rec0, hipStream_t st) {
    hipLaunchKernelGGL(k_obs_finish_many, dim3(n_rec * n_chains), dim3(256), 0, st, partials, n_blocks, n_chains,
                       stride, obs, obs_chain, rec0);
    return hipGetLastError();
}

hipError_t launch_init(int layout, void* dst, const Geom& G, int kind_const_up, bool random, const DrawParams& dp,
                       hipStream_t st) {
    const dim3 grid(grid_for(G.n_groups)), block(256);
#define SD_INIT(LAY)                                                                                    \
    case LAY:                                                                                           \
        if (random)                                                                                     \
            hipLaunchKernelGGL((k_init_random<LAY>), grid, block, 0, st, dst, G, dp);                   \
        else                                                                                            \
            hipLaunchKernelGGL((k_init_const<LAY>), grid, block, 0, st, dst, G, (uint32_t)kind_const_up); \
        break;
    switch (layout) {
        SD_INIT(kLayP64)
        SD_INIT(kLayP32)
        SD_INIT(kLayI8Row)
        SD_INIT(kLayI8Any)
        SD_INIT(kLayBits)
        default:
            return hipErrorInvalidValue;
    }
#undef SD_INIT
    return hipGetLastError();
}

hipError_t launch_fill_i64(int64_t* p, size_t n, int64_t v, hipStream_t st) {
    if (n == 0)
        return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 1024)
        blocks = 1024;
    hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace sd
