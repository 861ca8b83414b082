// Internal interface between the C-ABI host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "sd_device.hpp"

namespace sd {

// Kernel-side lattice layouts.  P64, P32 and Bits are the same bytes (bit s of
// the lattice is bit s % 64 of 64-bit word s / 64).  P64 and P32 work in
// 64- or 32-bit words with rows starting on a word (L % 64 == 0, L % 32 == 0);
// Bits takes neighbours as windows of the bit string (any L % 8 == 0).  I8Row
// is the int8 layout when every row is a whole number of 64-site groups
// (L % 64 == 0); I8Any handles any L >= 2.
enum KernelLayout : int { kLayP64 = 0, kLayP32 = 1, kLayI8Row = 2, kLayI8Any = 3, kLayBits = 4 };

constexpr uint32_t kMaxBlocks = 2048;

struct Geom {
    uint32_t L;
    uint32_t n_sites;     // L * L
    uint32_t n_groups;    // ceil(n_sites / 64)
    uint32_t words_row;   // P64: L/64; P32: L/32; I8Row: L/64; I8Any: unused
    FastDiv div_row;      // division by words_row
    FastDiv div_L;        // division by L
    uint32_t step_rows;   // 64 = step_rows * words_row + step_cols: moving 64
    uint32_t step_cols;   // words on in row-major order
};

// Granlund-Montgomery constants for division by d (1 <= d < 2^32).
inline FastDiv make_fastdiv(uint32_t d) {
    FastDiv f;
    uint32_t l = 0;
    while (l < 32 && (1ull << l) < d)
        ++l;
    uint64_t m = (((1ull << 32) * ((1ull << l) - d)) / d) + 1ull;
    f.d = d;
    f.mul = (uint32_t)m;
    f.shift = l;
    f.add = 1;
    return f;
}

inline uint32_t fdiv_host(uint32_t n, const FastDiv& f) {
    uint32_t hi = (uint32_t)(((uint64_t)n * f.mul) >> 32);
    return (uint32_t)(((uint64_t)hi + n) >> f.shift);
}

// max_blocks = 0: the default grid (four wavefront tiles per workgroup, at
// most kMaxBlocks workgroups); otherwise at most max_blocks workgroups (and
// never more than one per four tiles) walk the tiles.  With obs (half-step B
// only) and partials (device scratch of 4 int64 per workgroup), the
// workgroups' partial sums go to partials and a one-workgroup kernel adds
// M, A, B into obs; without partials every workgroup adds into obs with
// atomics.
// general: use the six-class compare even when the table is paired.
// finish = false leaves the partial sums in partials for a later
// launch_obs_finish that handles several records at once.
hipError_t launch_half_step(int layout, int which, const void* src, void* dst, const Geom& G, const DrawParams& dp,
                            int64_t* obs, hipStream_t st, uint32_t max_blocks = 0, int64_t* partials = nullptr,
                            bool general = false, bool finish = true);
// Workgroups of a half-step launch (the partial sums it leaves per record:
// four per workgroup).
uint32_t half_step_blocks(int layout, const Geom& G, bool paired, uint32_t max_blocks);
// Adds n_rec records into obs[3 * r ...]: record r from the n_blocks partial
// sums at partials + r * stride.
hipError_t launch_obs_finish(const int64_t* partials, uint32_t n_blocks, uint32_t n_rec, uint32_t stride,
                             int64_t* obs, hipStream_t st);
// Several chains of one size and layout advanced together (sd_run_many):
// per-chain lattices, threshold tables and stream ids; every chain's
// half-step is done by blocks_per_chain workgroups of one launch.
constexpr uint32_t kManyMax = 16;
struct ManyChains {
    void* sigma[kManyMax];
    void* tau[kManyMax];
    uint32_t T[kManyMax][6];
    uint32_t stream[kManyMax];
    uint32_t n_chains;
    uint32_t blocks_per_chain;
};
// Workgroups per chain of a multi-chain half-step (64-word tiles, four per
// workgroup, at most kMaxBlocks).
uint32_t many_blocks_per_chain(const Geom& G);
// which = 0: tau_a <- sigma_a, which = 1: sigma_a <- tau_a for every chain a;
// with partials (which = 1 only) the workgroups of chain a leave their
// partial sums at partials + 4 * (a * blocks_per_chain + block).
hipError_t launch_half_step_many(int layout, int which, const ManyChains& mc, const Geom& G, const DrawParams& base,
                                 bool paired, int64_t* partials, hipStream_t st);
// Writes records rec0 .. rec0 + n_rec - 1 of every chain: record r of chain a
// from the partials at partials + r * stride + 4 * a * n_blocks, into
// obs + a * obs_chain + 3 * (rec0 + r).
hipError_t launch_obs_finish_many(const int64_t* partials, uint32_t n_blocks, uint32_t n_chains, uint32_t n_rec,
                                  uint32_t stride, int64_t* obs, uint64_t obs_chain, uint32_t rec0, hipStream_t st);
// Whole steps of several chains, several per launch (lattices whose rows are
// at most 64 words, L = 64 * W with W dividing 256): workgroup (chain, band)
// runs `steps` steps of R = band_rows(L) rows (R * W at most 256) from sigma
// in src, with `steps` rows of halo on each side, writing the last sigma of
// its rows to dst (the other lattice of the pair).  src, dst, t0, steps and
// rec_mask change from launch to launch.
constexpr uint32_t kBandMaxSteps = 8;
constexpr uint32_t kBandMaxRowsWords = 256 + 2 * kBandMaxSteps * 64;   // (R + 2 steps) * W
constexpr uint32_t kBandMaxThreads = 768;
struct BandArgs {
    const void* src[kManyMax];
    void* dst[kManyMax];
    uint32_t T[kManyMax][6];
    uint32_t stream[kManyMax];
    uint32_t n_chains;
    uint32_t bands;      // L / R per chain
    uint32_t L, W, R;
    uint32_t shW;        // log2 W (W divides 256)
    uint32_t key0, key1;
    uint32_t t0;         // half-step index of the launch's first half-step A
    uint32_t steps;      // 1 .. kBandMaxSteps
    uint32_t threads;    // workgroup size: 64 per tile of the widest half-step
    uint32_t rec_mask;   // bit s: record step s of the launch
    uint32_t rec_stride; // int64 between the partial sums of consecutive records
};
// Rows per band for L, or 0 when L does not take the whole-step kernel.
uint32_t band_rows(int32_t L);
// Steps per launch of the whole-step kernel for lattices of side L.
uint32_t band_depth(int32_t L);
// Workgroup size for `steps` steps of bands of R rows of W words.
uint32_t band_threads(uint32_t R, uint32_t W, uint32_t steps);
// partials (non-null when rec_mask is not zero): the sums of recorded step k
// of the launch at partials + k * rec_stride + 4 b for workgroup b.
hipError_t launch_band_step(const BandArgs& ba, bool int8, bool paired, bool complement, int64_t* partials,
                            hipStream_t st);
hipError_t launch_init(int layout, void* dst, const Geom& G, int const_up, bool random, const DrawParams& dp,
                       hipStream_t st);
hipError_t launch_fill_i64(int64_t* p, size_t n, int64_t v, hipStream_t st);

// Observables of a pair and the row correlation, for any layout.
hipError_t launch_observe(int layout, const void* sigma, const void* tau, const Geom& G, int64_t* out3,
                          hipStream_t st);
hipError_t launch_corr_row(int layout, const void* sigma, const Geom& G, int32_t rmax, int64_t* out,
                           hipStream_t st);
// D(r) of n (1 .. kManyMax) lattices of one size and layout: lattice a's sums
// at out + a (rmax + 1); one launch for rows of whole 64-bit words (P64,
// I8Row), one per lattice otherwise.
struct CorrLattices {
    const void* p[kManyMax];
};
hipError_t launch_corr_row_many(int layout, const void* const* sigma, uint32_t n, const Geom& G, int32_t rmax,
                                int64_t* out, hipStream_t st);
hipError_t launch_corr_diag(int layout, const void* sigma, const Geom& G, int32_t lmax, int64_t* out,
                            hipStream_t st);

}  // namespace sd
