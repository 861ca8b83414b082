// Internal interface of the batched (many-chain) persistent kernel.
#pragma once

#include "sd_kernels.hpp"

namespace sd {

// One chain of a batch (device array, built on the host).
struct ChainDesc {
    uint32_t T[6];          // threshold table of this chain's (J, q)
    uint32_t L;             // lattice size, L % 64 == 0
    uint32_t stream;        // stream id of the chain's randomness
    uint32_t paired;        // thresholds_paired(T): the compare may use the paired form
    FastDiv divW;           // division by L / 64
    FastDiv divL;           // division by L
    uint64_t sig_offset;    // sigma, in bytes from the lattices base
    uint64_t tau_offset;    // tau, in bytes from the lattices base
    uint64_t trace_offset;  // first int64 of the chain's trace
};

// Queues of later buckets a launch may take chains from once its own is
// empty (buckets of smaller lattices with the same kernel form).
constexpr uint32_t kMaxSteal = 3;

struct BatchArgs {
    const ChainDesc* chains;
    const uint32_t* order;   // queue position -> chain index (longest first)
    uint32_t n_chains;       // chains in this launch's queue
    uint32_t* counter;       // queue head, zero before the launch; null: run `single` in block 0
    uint32_t n_steal;        // further queues, taken in order after this one
    const uint32_t* steal_order[kMaxSteal];
    uint32_t steal_count[kMaxSteal];
    uint32_t* steal_counter[kMaxSteal];
    ChainDesc single;        // the chain of a single-chain launch (offsets unused)
    uint8_t* single_sig;     // its sigma
    uint8_t* single_tau;     // its tau
    uint8_t* lattices;       // base of all lattices
    int64_t* traces;         // may be null
    uint32_t key0, key1;
    uint32_t step0;          // first step index
    uint32_t k_steps;
    uint32_t obs_every;
    uint32_t rng_xor;
    uint32_t max_words;      // capacity (64-bit words) of each LDS lattice buffer
    uint32_t int8_io;        // lattices in global memory are int8 (L % 64 == 0)
    uint32_t paired;         // every chain of the launch has a paired threshold table
    uint32_t bits;           // the chains' L % 64 != 0 (L % 8 == 0): bit-string neighbours
    uint32_t moments;        // traces hold, per chain, sum M, sum M^2, sum |M|, sum A, sum B over the
                             // recorded steps (kMomentWords int64) instead of the records
    uint32_t n_uniform;      // counter null and n_uniform > 0: workgroup b runs `single` with stream
                             // single.stream + b from packed sigma single_sig + b * lattice bytes
    uint8_t* traj;           // non-null: workgroup b writes lattice x of its trajectory (x = 0 the
                             // start, 2m+1 after half-step A of step m, 2m+2 after B) to
                             // traj + b * traj_chain_bytes + x * lattice bytes, and skips the write-back
    uint64_t traj_chain_bytes;
    unsigned long long* t_start;   // non-null: the launch's first start and last end on the device
    unsigned long long* t_end;     // wall clock (atomic min / max by thread 0 of every workgroup)
};

// Largest workgroup of the batched kernel (the paired compare; the six-class
// compare takes at most 512 threads).
constexpr uint32_t kBatchMaxThreads = 640;

// Dynamic LDS of a launch: the two lattice buffers and one list of undecided
// words per wavefront of a threads-sized workgroup.
constexpr uint32_t kMomentWords = 5;

// 64-site words of an L x L lattice (L % 8 == 0).
uint32_t lattice_words(uint32_t L);
// Division constants of a chain: by the words per row (rows of whole words
// only; 1 otherwise) and by L.
void set_divisors(ChainDesc& d, uint32_t L);

size_t batch_lds_bytes(uint32_t max_words, uint32_t threads);
hipError_t launch_batch_chains(const BatchArgs& a, uint32_t blocks, uint32_t threads, hipStream_t st);
hipError_t launch_zero_u32(uint32_t* p, uint32_t n, hipStream_t st);
// starts[0 .. n) = all ones and ends[0 .. n) = 0, before the launches that time themselves.
hipError_t launch_times_reset(unsigned long long* starts, unsigned long long* ends, uint32_t n, hipStream_t st);
hipError_t batch_kernel_attributes(size_t max_dynamic_lds);
hipError_t batch_occupancy(uint32_t threads, size_t lds, bool paired, bool bits, int* blocks_per_cu);

// Coupling from the past: pair p of `pairs` owns four lattices of `words`
// words at work + 4 p words*8 bytes (top sigma, top tau, bottom sigma, bottom
// tau).  reset: top sigma all +1, bottom sigma all -1.  finish: equal[i] =
// (top sigma == bottom sigma) of pair pairs[i], and its top sigma is copied
// to samples + pairs[i] * words * 8 bytes.
hipError_t launch_pw_reset(uint8_t* work, const uint32_t* pairs, uint32_t n, uint32_t words, hipStream_t st);
hipError_t launch_pw_finish(const uint8_t* work, const uint32_t* pairs, uint32_t n, uint32_t words, uint8_t* samples,
                            uint32_t* equal, hipStream_t st);

// Lattices with at most this many 64-site words run in one workgroup with
// LDS-resident lattices when sd_run is called without SD_FLAG_GLOBAL_KERNELS.
constexpr uint32_t kSingleLdsMaxWords = 1024;

// n_traj packed trajectories of one (J, q) with streams stream0 + a in one
// launch (workgroup a runs trajectory a); L * L / 64 words must fit in LDS.
hipError_t launch_trajectories_lds(const void* sigma0, void* traj, uint32_t n_traj, int32_t L, double J, double q,
                                   uint64_t seed, uint32_t stream0, uint64_t step0, uint32_t k_steps,
                                   uint32_t threads, hipStream_t st);

hipError_t launch_single_chain_lds(void* sigma, void* tau, int32_t L, bool int8_io, double J, double q,
                                   uint64_t seed, uint32_t stream, uint64_t step0, uint32_t k_steps, int64_t* obs,
                                   uint32_t obs_every, uint32_t flags, uint32_t threads, hipStream_t st);

}  // namespace sd
