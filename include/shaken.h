/*
 * libshaken — C ABI of the MI355X (gfx950) shaken-dynamics library.
 *
 * The shaken dynamics (D'Autilia, Andrianaivo and Troiani, "Parallel
 * simulation of two-dimensional Ising models using Probabilistic Cellular
 * Automata", arXiv:1908.07341, section 2) is a probabilistic cellular
 * automaton on a pair of L x L tori (sigma, tau).  One step is two half-steps:
 *   A: every tau_x is drawn independently from the field
 *      J (sigma_down + sigma_left) + q sigma_x                (eq. (15))
 *   B: every sigma'_x is drawn independently from the field
 *      J (tau_up + tau_right) + q tau_x                        (eq. (16))
 * with P(new spin = +1) = e^h / (2 cosh h).
 *
 * Conventions shared by every entry point:
 *   - site x = (i, j), i = column (east), j = row (north), linear index
 *     s = j*L + i; up = (i, j+1), right = (i+1, j), down = (i, j-1),
 *     left = (i-1, j), all mod L (eq. (4));
 *   - layouts: SD_I8 = one int8 per site, +1 -> 0x01, -1 -> 0xFF;
 *     SD_P64 / SD_P32 = one bit per site (1 = +1), bit s of the lattice is
 *     bit s%64 of 64-bit word s/64 (the same bytes for both; P64 needs
 *     L % 8 == 0, so that L*L fills whole words, and 8-byte alignment; rows
 *     start on a word only when L % 64 == 0.  P32 needs L % 32 == 0 and
 *     4-byte alignment);
 *   - randomness: the counter-based stream keyed by (seed, stream, half-step
 *     index t, site s): step n of a chain uses t = 2n (A) and t = 2n+1 (B); the
 *     result is a pure function of the arguments, so run(k1) followed by
 *     run(step0 + k1, k2) equals run(k1 + k2);
 *   - pointers named "device" must be device memory (hipMalloc or torch CUDA
 *     tensors); the library never frees, keeps or reallocates caller memory;
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream); work is
 *     enqueued asynchronously on it, except where a function says otherwise;
 *   - every function validates its arguments before enqueuing anything and
 *     returns SD_EINVAL (or SD_EUNSUPPORTED) without side effects on bad
 *     arguments; SD_EHIP reports a HIP runtime error (asynchronous errors of
 *     earlier work may surface here); sd_last_error() gives a message for the
 *     last non-OK status of the calling thread.  Limits: 2 <= L <= 65535;
 *     step indices below 2^29.
 */
#ifndef SHAKEN_H
#define SHAKEN_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define SD_API __attribute__((visibility("default")))
#else
#define SD_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SD_OK = 0,
    SD_EINVAL = -1,
    SD_EUNSUPPORTED = -2,
    SD_EHIP = -3,
    SD_ENOSPACE = -4
} sd_status;

typedef enum { SD_I8 = 0, SD_P32 = 1, SD_P64 = 2 } sd_layout;

typedef enum { SD_INIT_UP = 0, SD_INIT_DOWN = 1, SD_INIT_RANDOM = 2 } sd_init_kind;

/* Flags of sd_half_step / sd_run. */
#define SD_FLAG_COMPLEMENT_RNG 1u /* replace every uniform r by 2^32-1-r (global spin-flip check) */
#define SD_FLAG_MOMENTS 4u        /* batch plans: keep per-chain sums of the records instead of traces */
#define SD_FLAG_GLOBAL_KERNELS 2u /* sd_run: always use one grid-wide launch per half-step, never the
                                     single-workgroup LDS-resident kernel used for small lattices */
#define SD_FLAG_GENERAL_COMPARE 8u /* sd_half_step, sd_run, batch plans: decide the sites with the
                                      six-class bit-sliced compare instead of the paired one (same
                                      results, slower; a cross-check of the two forms) */

#define SD_ABI_VERSION 1

SD_API int32_t sd_abi_version(void);

/* Message of the last non-OK status returned to the calling thread. */
SD_API const char* sd_last_error(void);

/* Bytes of one lattice, or 0 if (L, layout) is not supported. */
SD_API size_t sd_lattice_bytes(int32_t L, int32_t layout);

/*
 * Heat-bath thresholds of Algorithm 3's draw "+1 if rand() < e^h/(2cosh h)".
 * out_host[idx], idx = 2k + [c = +1] (k = number of +1 among the two
 * J-neighbours, c = partner spin), for h = J(2k-2) + q(2c-1):
 *   U = max(1, round-half-even(2^32 / (1 + exp(2|h|)))),
 *   T = 2^32 - U (h > 0), U (h < 0), 2^31 (h = 0);
 * a new spin is +1 iff its 32-bit uniform is < T.  Host memory, synchronous.
 * EINVAL: non-finite J or q, null out_host.
 */
SD_API sd_status sd_threshold_table(double J, double q, uint32_t out_host[6]);

/*
 * Fill a lattice (device, sd_lattice_bytes(L, layout) bytes): all +1, all -1,
 * or i.i.d. +1 with probability p_up (RANDOM: site s is +1 iff its uniform at
 * t = 0 of the initialisation stream is < round-half-even(p_up * 2^32)).
 * The paper's runs start from all -1 (section 3.1).
 * EINVAL: bad L/layout/kind, p_up outside [0, 1] for RANDOM, null lattice.
 */
SD_API sd_status sd_init(void* lattice, int32_t L, int32_t layout, int32_t kind, double p_up, uint64_t seed,
                  uint32_t stream, void* hip_stream);

/*
 * One half-step: which = 0 draws tau (dst) from sigma (src) with the
 * down/left field (eq. (15)); which = 1 draws sigma' (dst) from tau (src) with
 * the up/right field (eq. (16)).  t is the half-step index (< 2^30).  src and
 * dst are device lattices of the same layout and must not overlap.  flags:
 * SD_FLAG_COMPLEMENT_RNG, SD_FLAG_GENERAL_COMPARE.
 */
SD_API sd_status sd_half_step(const void* src, void* dst, int32_t L, int32_t layout, int32_t which, double J, double q,
                       uint64_t seed, uint32_t stream, uint32_t t, uint32_t flags, void* hip_stream);

/*
 * k_steps full steps of one chain, steps step0 .. step0+k_steps-1, in place:
 * (lattices of at most 65536 sites with L % 64 == 0 run in one workgroup with
 * both lattices held in LDS, one launch for all steps; larger ones use two
 * grid-wide launches per step and, with obs, one more launch per chunk of
 * records, whose partial sums wait in a 512 KiB device buffer the library
 * allocates once per (device, stream) and keeps; the result is the same bit
 * for bit)
 * sigma (device) is updated, tau (device, same size) receives the last
 * half-step-A lattice (its input content is ignored).  If obs (device) is not
 * NULL it receives, after every obs_every-th step, the int64 triple
 * (M, A, B) = (sum sigma, sum sigma_x (tau_up + tau_right), sum sigma_x tau_x)
 * of the pair (sigma_n, tau_n) — the new sigma and the tau it was drawn from —
 * so that m = M / L^2 and H(sigma, tau) = -(J A + q B) (section 3.1, eq. (5)):
 * obs[3 * r + {0, 1, 2}] for record r = 0 .. k_steps/obs_every - 1.
 * flags: SD_FLAG_COMPLEMENT_RNG, SD_FLAG_GLOBAL_KERNELS, SD_FLAG_GENERAL_COMPARE.
 * EINVAL: bad sizes, obs without obs_every, step0 + k_steps >= 2^29.
 */
SD_API sd_status sd_run(void* sigma, void* tau, int32_t L, int32_t layout, double J, double q, uint64_t seed,
                 uint32_t stream, uint64_t step0, uint32_t k_steps, int64_t* obs, uint32_t obs_every,
                 uint32_t flags, void* hip_stream);

/*
 * sd_run for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same
 * arguments, the same results bit for bit, and no allocation, ever.  Where
 * sd_run keeps per-workgroup partial sums of recorded steps in a buffer it
 * allocates once per (device, stream), this call uses a fixed array of
 * 65536 int64 (512 KiB) that the library holds in device memory per device
 * from load until the process ends; its device address is looked up once per
 * device, on the first call.  That array is shared by every call on the
 * device and keeps the last call's contents (each recorded half-step writes
 * every slot it later reads), so calls that overlap on one device — on
 * different streams or from different host threads — race and must not be
 * made.  EINVAL: as sd_run, and a grid whose per-record partial sums (4 per
 * workgroup) would not fit the array.
 */
SD_API sd_status sd_run_noalloc(void* sigma, void* tau, int32_t L, int32_t layout, double J, double q, uint64_t seed,
                                uint32_t stream, uint64_t step0, uint32_t k_steps, int64_t* obs, uint32_t obs_every,
                                uint32_t flags, void* hip_stream);

/*
 * n_chains (1..16) chains of one size and layout advanced together: chain a
 * is exactly sd_run(sigma[a], tau[a], L, layout, J[a], q[a], seed,
 * streams[a], step0, k_steps, ...), but every launch covers all the chains,
 * so that lattices of a few thousand words, which alone fill a small part of
 * the device, run together at the launch rate of one.  Lattices whose rows
 * are whole 64-bit words, at most 64 of them (L = 64 W with W dividing 256;
 * packed, or int8 with 16-byte aligned lattices), run all but the last step
 * as whole steps, up to eight per launch: each workgroup takes a band of rows
 * plus one halo row per step on each side into LDS and recomputes the halo
 * from the same counter-based uniforms (sections 2 and 4: eqs. (15)-(16)
 * drawn site by site), so results do not change; tau's memory holds sigma
 * between launches and the last step, as two half-step launches, leaves tau
 * as sd_run does.  Other lattices take one launch per half-step for all the
 * chains (the chains' words split into 64-word tiles, a share of the
 * workgroups per chain).  sigma, tau: host arrays of n_chains device lattice pointers (no two of
 * the 2 n_chains lattices may overlap); J, q, streams: host arrays of
 * n_chains.  obs (device) NULL, or n_chains x (k_steps / obs_every) records
 * of (M, A, B), chain-major: obs[3 * (a * (k_steps / obs_every) + r) + {0,1,2}]
 * is sd_run's record r of chain a.  Records go through the same per-(device,
 * stream) partial-sum buffer as sd_run (allocated on first use and kept), so
 * a first call with records cannot be made under stream capture.  flags:
 * SD_FLAG_COMPLEMENT_RNG, SD_FLAG_GENERAL_COMPARE.  EINVAL: bad sizes or
 * pointers, overlapping lattices, obs without obs_every, step0 + k_steps
 * above 2^29.
 */
SD_API sd_status sd_run_many(void* const* sigma, void* const* tau, int32_t n_chains, int32_t L, int32_t layout,
                             const double* J, const double* q, uint64_t seed, const uint32_t* streams, uint64_t step0,
                             uint32_t k_steps, int64_t* obs, uint32_t obs_every, uint32_t flags, void* hip_stream);

/*
 * Measure and fix how sd_run executes chains of this (L, layout) on the
 * current device: the single-workgroup LDS-resident kernel (workgroup size
 * 128/256/512, lattices up to the device's LDS) or one grid-wide launch per
 * half-step (64- or 32-bit word kernels when L % 64 == 0 — the same bytes —
 * and the number of workgroups).  Each candidate runs a few steps on scratch
 * lattices (allocated and freed here) with HIP events; the fastest is used by
 * every later sd_run of this process with these (L, layout) and stored under
 * a "run:<arch>:L=..:layout=.." key in the JSON file tune_cache_path (NULL:
 * not stored); a later sd_tune finding the key there takes it without
 * measuring.  Synchronises the stream.  Results of sd_run do not depend on
 * the choice.
 */
SD_API sd_status sd_tune(int32_t L, int32_t layout, const char* tune_cache_path, void* hip_stream);

/* The choice sd_run currently uses for (L, layout): mode 0 = built-in rule,
 * 1 = LDS kernel, 2 = grid kernels; word width; the workgroups of each
 * half-step launch when sd_run takes the grid kernels; the LDS kernel's
 * workgroup size. */
SD_API sd_status sd_tuned_choice(int32_t L, int32_t layout, int32_t* mode, int32_t* width, int32_t* blocks,
                                 int32_t* threads);

/* (M, A, B) of an arbitrary pair of device lattices into out3 (device, 3 int64). */
SD_API sd_status sd_observe(const void* sigma, const void* tau, int32_t L, int32_t layout, int64_t* out3,
                     void* hip_stream);

/*
 * Row-wise correlation sums D(r) = sum_x sigma_(i,j) sigma_(i+r mod L, j),
 * r = 0 .. rmax (0 <= rmax < L), into out (device, rmax+1 int64).  The
 * normalised C(r) = D(r) / L^2 and the connected form are left to the caller
 * (the paper's Table 1 reports diagonal correlations of this kind).
 */
SD_API sd_status sd_corr_row(const void* sigma, int32_t L, int32_t layout, int32_t rmax, int64_t* out,
                      void* hip_stream);

/*
 * sd_corr_row for n (1..16) lattices of one size and layout in one pass:
 * sigma is a host array of n device lattice pointers, out (device) receives
 * n x (rmax + 1) int64, lattice a's D(r) at out[a * (rmax + 1) + r], each
 * exactly what sd_corr_row returns for it.  Lattices whose rows are whole
 * 64-bit words (packed with L % 64 == 0, or int8 with 16-byte aligned
 * lattices) share one launch; other lattices take one launch each.  The
 * sums are those of section 3.3's correlations, row by row, as for
 * sd_corr_row.  EINVAL: n outside [1, 16], a null host array, output or
 * lattice pointer, a packed lattice not aligned to its word size, an
 * unsupported (L, layout), rmax outside [0, L).
 */
SD_API sd_status sd_corr_row_many(const void* const* sigma, int32_t n, int32_t L, int32_t layout, int32_t rmax,
                                  int64_t* out, void* hip_stream);

/*
 * Diagonal correlation sums of section 3.3 (Table 1) for l = 0 .. lmax
 * (0 <= lmax < L): out[l] = sum_x sigma_(i,j) sigma_(i+l, j+l) (SW-NE) and
 * out[lmax + 1 + l] = sum_x sigma_(i,j) sigma_(i+l, j-l) (NW-SE), coordinates
 * mod L, exact int64 (device, 2 * (lmax + 1) entries).  C = sum / L^2.
 */
SD_API sd_status sd_corr_diag(const void* sigma, int32_t L, int32_t layout, int32_t lmax, int64_t* out,
                              void* hip_stream);

/* ------------------------------------------------------------------------- */
/* Trajectories and their log-likelihood (differentiation with respect to     */
/* (J, q)).                                                                   */
/* ------------------------------------------------------------------------- */

/*
 * Record a trajectory: traj (device) receives the 2*k_steps + 1 lattices
 * X_0 = sigma0, X_1 = tau_1, X_2 = sigma_1, ..., X_{2k} = sigma_k of the chain
 * started from sigma0 at step step0, back to back, each sd_lattice_bytes(L,
 * layout) bytes (layout SD_P64 or SD_P32).  sigma0 may be traj itself (then it
 * is not copied) but must not otherwise overlap it.  The lattices are
 * bit-identical to those of sd_run.
 */
SD_API sd_status sd_trajectory(const void* sigma0, void* traj, int32_t L, int32_t layout, double J, double q,
                               uint64_t seed, uint32_t stream, uint64_t step0, uint32_t k_steps, void* hip_stream);

/*
 * n_traj trajectories of one (J, q) at once: trajectory a starts from the
 * packed lattice sigma0 + a * sd_lattice_bytes(L, layout) (device) with
 * stream id stream0 + a, and its 2*k_steps + 1 lattices go to
 * traj + a * (2*k_steps + 1) * sd_lattice_bytes(L, layout), laid out as
 * sd_trajectory writes them; the result is that of n_traj calls of
 * sd_trajectory.  When L is a multiple of 8 and a lattice pair fits in LDS
 * (L <= 512 on gfx950) every trajectory runs in one workgroup of a single
 * launch with its lattices in LDS; otherwise the trajectories are recorded
 * one after the other.  The start lattices must not overlap the
 * trajectories; pointers 8-byte aligned; stream0 + n_traj <= 2^32.
 */
SD_API sd_status sd_trajectories(const void* sigma0, void* traj, int32_t n_traj, int32_t L, int32_t layout, double J,
                                 double q, uint64_t seed, uint32_t stream0, uint64_t step0, uint32_t k_steps,
                                 void* hip_stream);

/*
 * Sufficient statistics of the log-likelihood of n_traj packed (SD_P64)
 * trajectories of n_lat lattices each (traj[a][m][L][L/64], device, as written
 * by sd_trajectory): counts12[2*idx + [s = +1]] (device, 12 int64) counts the
 * sites drawn to s with field class idx = 2k + [c = +1] over every transition
 * X_m -> X_{m+1} (half-step A for even m, B for odd m) of every trajectory.
 * By the product form of eqs. (15)-(16) the log-likelihood of the trajectories
 * is  LL(J, q) = sum over the counts of n * (h s - log 2cosh h),
 * h = J(2k-2) + q(2c-1).  L must be a multiple of 64.
 */
SD_API sd_status sd_loglik_counts(const void* traj, int32_t n_traj, int32_t n_lat, int32_t L, int64_t* counts12,
                                  void* hip_stream);

/*
 * ll[0] (device float) = LL(J, q) from the counts, Jq (device) = {J, q} in
 * FP32.  Evaluated with binary32 operations only (values carried as pairs of
 * floats), rounded to FP32 at the end.
 */
SD_API sd_status sd_loglik_fwd(const int64_t* counts12, const float* Jq, float* ll, void* hip_stream);

/*
 * grad[0..1] (device floats) = g_out[0] * (dLL/dJ, dLL/dq), with
 * dLL/dJ = sum n (2k-2)(s - tanh h), dLL/dq = sum n (2c-1)(s - tanh h);
 * g_out (device float) may be NULL for 1.  Same arithmetic as sd_loglik_fwd.
 */
SD_API sd_status sd_loglik_bwd(const int64_t* counts12, const float* Jq, const float* g_out, float* grad,
                               void* hip_stream);

/*
 * Paired sufficient statistics of the same log-likelihood (same trajectories,
 * layout and L as sd_loglik_counts).  The classes idx and 5 - idx have
 * opposite fields h, and log 2cosh is even and tanh odd, so LL and its
 * gradient depend on each pair (j, 5 - j), j = 0, 1, 2, only through
 *   stats6[j]     = S_j = sites of class j or 5 - j,
 *   stats6[3 + j] = Z_j = sites of class j drawn +1 plus sites of class 5 - j
 *                         drawn -1
 * (device, 6 int64, over every transition of every trajectory).  In terms of
 * the 12 counts: S_j = n[2j] + n[2j+1] + n[2(5-j)] + n[2(5-j)+1],
 * Z_j = n[2j+1] + n[2(5-j)].  Exact integers; five popcounts per word and
 * transition where the counts take twelve.
 */
SD_API sd_status sd_loglik_stats(const void* traj, int32_t n_traj, int32_t n_lat, int32_t L, int64_t* stats6,
                                 void* hip_stream);

/*
 * ll[0] (device float) = LL(J, q) = sum_j h_j (2 Z_j - S_j) - S_j log 2cosh h_j
 * from the paired statistics, h_j the field of class j (h_j = J(2k-2) + q(2c-1)
 * with j = 2k + [c = +1]).  Same arithmetic as sd_loglik_fwd.
 */
SD_API sd_status sd_loglik_fwd_stats(const int64_t* stats6, const float* Jq, float* ll, void* hip_stream);

/*
 * grad[0..1] (device floats) = g_out[0] * (dLL/dJ, dLL/dq) from the paired
 * statistics: dLL/dJ = sum_j (2k-2)(2 Z_j - S_j - S_j tanh h_j), dLL/dq the
 * same with (2c-1).  g_out may be NULL for 1.  Same arithmetic as sd_loglik_bwd.
 */
SD_API sd_status sd_loglik_bwd_stats(const int64_t* stats6, const float* Jq, const float* g_out, float* grad,
                                     void* hip_stream);

/*
 * Exact samples from the stationary law of the shaken dynamics by coupling
 * from the past (Propp-Wilson), the sampler that section 3.2 builds on the
 * coupling of two copies driven by the same randomness.  For J, q >= 0 a full
 * step is monotone (sigma <= sigma' site by site stays so under shared
 * uniforms), so the chains from all +1 and all -1 bound every other chain.
 * Sample p (0 <= p < n_samples) uses stream stream0 + p; time -t (t >= 1)
 * draws the uniforms of step index step_end - t.  T runs through T0, 2 T0,
 * 4 T0, ... while T <= T_max; the two chains are started at time -T and run
 * to time 0, and the sample is their common lattice at the first T at which
 * they agree.
 *   samples: device, n_samples lattices of sd_lattice_bytes(L, SD_P64) bytes
 *            (SD_P64 layout), written.
 *   work:    device scratch of 4 * n_samples * sd_lattice_bytes(L, SD_P64)
 *            bytes, owned by the caller, contents overwritten; must not
 *            overlap samples.
 *   T_used:  host, n_samples int64: the T that coalesced, or 0 if none up to
 *            T_max (that sample is then the top chain's lattice at time 0 from
 *            the largest T tried).
 * Needs finite J, q >= 0, L a multiple of 8 whose lattice pair fits one
 * workgroup's LDS, 1 <= T0 <= T_max <= step_end <= 2^29, 8-byte aligned
 * buffers.  Synchronises hip_stream once per T (to read the pairs' flags) and
 * allocates a few bytes of device scratch per sample for the call.
 */
SD_API sd_status sd_propp_wilson(void* samples, void* work, int32_t n_samples, int32_t L, double J, double q,
                                 uint64_t seed, uint32_t stream0, uint64_t step_end, uint32_t T0, uint32_t T_max,
                                 int64_t* T_used, void* hip_stream);

/* ------------------------------------------------------------------------- */
/* Replica-coded chains: 64 chains that share one stream, one bit each.        */
/* ------------------------------------------------------------------------- */

/*
 * Bytes of a replica lattice: L * L 64-bit words, word s = j L + i holding
 * site (i, j) of 64 replicas, bit r for replica r (1 = spin +1).  0 unless L
 * is a multiple of 8 in [8, 32768].
 */
SD_API size_t sd_replica_lattice_bytes(int32_t L);

/*
 * k_steps full steps (steps step0 .. step0+k_steps-1) of 64 chains at once,
 * chain r at (J[r], q[r]) (host arrays of 64), all with the same seed and
 * stream: every site's uniform (eqs. (15)-(16) draw each spin independently,
 * so one uniform per site and half-step) is drawn once and compared with the
 * 64 chains' own thresholds.  Replica r's lattices equal, bit for bit, those
 * of sd_run at (J[r], q[r], seed, stream) from the same start; the chains are
 * not independent of each other (they share their randomness, which is what
 * makes them a monotone coupling when their (J, q) agree), but each is an
 * exact chain of its own (J, q).  sigma (device) is updated in place; tau
 * (device, same size) receives the last half-step-A lattice.  Layout as
 * sd_replica_lattice_bytes; 8-byte aligned, non-overlapping.  EINVAL: bad L,
 * null or non-finite parameters, step0 + k_steps > 2^29.
 */
SD_API sd_status sd_replica_run(void* sigma, void* tau, int32_t L, const double* J, const double* q, uint64_t seed,
                                uint32_t stream, uint64_t step0, uint32_t k_steps, void* hip_stream);

/*
 * out (device, 192 int64): out[3 r + {0, 1, 2}] = (M, A, B) of replica r's
 * pair (sigma, tau), as sd_observe computes them for one chain.
 */
SD_API sd_status sd_replica_observe(const void* sigma, const void* tau, int32_t L, int64_t* out, void* hip_stream);

/* ------------------------------------------------------------------------- */
/* Batched scan: many independent chains in one persistent launch.            */
/* ------------------------------------------------------------------------- */

/* One chain of a batch: its couplings, lattice size (a multiple of 8) and
 * stream id (the chain's randomness is exactly that of sd_run with the same
 * seed and stream). */
typedef struct {
    double J;
    double q;
    int32_t L;
    uint32_t stream;
} sd_chain_desc;

typedef struct sd_batch_plan sd_batch_plan;

/*
 * Plan a batch of n_chains chains (the paper's (q, J) scan of section 3.1 runs
 * one chain per parameter pair).  Host-side setup, synchronous: computes every
 * chain's threshold table, lays out one lattice buffer holding sigma and tau of
 * every chain (sd_batch_lattice_bytes, offsets from sd_batch_chain_offset) and a
 * trace buffer of sd_batch_trace_len int64 = n_chains x (k_steps / obs_every)
 * records x (M, A, B), groups the chains by lattice size (largest first) and
 * picks each group's workgroup size: measured and cached in the JSON file
 * tune_cache_path if that is not NULL (measuring allocates scratch device
 * memory for the duration of the call), 256 otherwise.  layout is SD_P64 or
 * SD_I8.  flags: SD_FLAG_COMPLEMENT_RNG, SD_FLAG_GENERAL_COMPARE, and SD_FLAG_MOMENTS (needs
 * obs_every > 0), under which the trace buffer holds instead, per chain, the
 * 5 int64 sums over the run's recorded steps of M, M^2, |M|, A and B (the
 * mean and variance of the magnetisation that section 3.1 scans; each
 * sd_batch_run overwrites them).  The plan owns small device tables, side
 * streams and a hipGraph; free it with sd_batch_plan_destroy.  EUNSUPPORTED: a
 * chain whose two lattices do not fit in one workgroup's LDS.
 */
SD_API sd_status sd_batch_plan_create(sd_batch_plan** plan, const sd_chain_desc* chains_host, int32_t n_chains,
                                      int32_t layout, uint64_t seed, uint32_t k_steps, uint32_t obs_every,
                                      uint32_t flags, const char* tune_cache_path);

/* Size in bytes of the lattice buffer of a plan (0 for NULL). */
SD_API size_t sd_batch_lattice_bytes(const sd_batch_plan* plan);

/* Number of int64 in the trace buffer of a plan (0 for NULL). */
SD_API size_t sd_batch_trace_len(const sd_batch_plan* plan);

/* Byte offset of chain's sigma (which = 0) or tau (which = 1) in the lattice
 * buffer, or -1 for a bad argument. */
SD_API int64_t sd_batch_chain_offset(const sd_batch_plan* plan, int32_t chain, int32_t which);

/* Launch shape chosen for size group `bucket` (0 = largest L); outputs may be NULL. */
SD_API sd_status sd_batch_launch_shape(const sd_batch_plan* plan, int32_t bucket, int32_t* L, int32_t* n_chains,
                                       int32_t* threads, int32_t* blocks);

/* Initialise every chain's sigma as sd_init would with the chain's own stream. */
SD_API sd_status sd_batch_init(sd_batch_plan* plan, void* lattices, int32_t kind, double p_up, void* hip_stream);

/*
 * Run every chain for the plan's k_steps steps from step index step0, in
 * place, as one graph launch: a kernel zeroes the work-queue counters, then one
 * persistent kernel per size group (on forked streams) pops chains from its
 * queue.  Chain c ends bit-identical to sd_run on the same sigma with the same
 * seed, stream, step0 and k_steps, and its trace rows equal sd_run's obs rows.
 * lattices (device, 16-byte aligned) and traces (device, or NULL when the plan
 * records nothing) follow the plan's layout.  The graph is captured on the
 * first call and reused while (lattices, traces, step0) stay the same.
 */
SD_API sd_status sd_batch_run(sd_batch_plan* plan, void* lattices, int64_t* traces, uint64_t step0,
                              void* hip_stream);

/* The same work as sd_batch_run, enqueued as plain kernel launches (no graph). */
SD_API sd_status sd_batch_run_direct(sd_batch_plan* plan, void* lattices, int64_t* traces, uint64_t step0,
                                     void* hip_stream);

/*
 * Times of bucket `bucket` (the order of sd_batch_launch_shape) in the last
 * run of the plan (sd_batch_run or sd_batch_run_direct), in ms from the
 * earliest start among that run's launches: when the bucket's persistent
 * launch started (its first workgroup) and when it ended (its last
 * workgroup), taken on the device with its constant-rate wall clock.  A
 * launch takes chains of its own size first, then of the later (smaller)
 * buckets of the same kernel form, so that no bucket's workgroups wait while
 * another's queue still holds chains.  Synchronises the device.  EINVAL: no
 * such bucket, null outputs, or no run yet; EHIP: a HIP error, or no time
 * stamps (the run failed).
 */
SD_API sd_status sd_batch_bucket_times(sd_batch_plan* plan, int32_t bucket, float* start_ms, float* end_ms);

/* Free a plan (NULL is ignored).  Synchronises with nothing; the caller must
 * not destroy a plan whose graph is still executing. */
SD_API void sd_batch_plan_destroy(sd_batch_plan* plan);

/*
 * Diagnostics.  sd_debug_fastdiv returns n / d (d >= 1) computed with the
 * multiply-shift division the kernels use for row and column indices; 0 for
 * d == 0.  Host only, synchronous.
 */
SD_API uint32_t sd_debug_fastdiv(uint32_t n, uint32_t d);

#ifdef __cplusplus
}
#endif

#endif /* SHAKEN_H */
