/*
 * Shaken-dynamics CPU oracle.  TEST INFRASTRUCTURE ONLY.
 *
 * Plain, single-threaded, deliberately unoptimised implementation of the two
 * half-step probabilistic cellular automaton of D'Autilia, Andrianaivo and
 * Troiani, "Parallel simulation of two-dimensional Ising models using
 * Probabilistic Cellular Automata" (arXiv:1908.07341).  It exists to check the
 * GPU library: only the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code with the GPU
 * library; every convention below is written out again from the paper and
 * from the frozen stream contract described in the repository design notes.
 *
 * Lattice: an L x L torus, site x = (i, j) with i the column (east) and j the
 * row (north), linear index s = j*L + i, one int8 per site holding +1 or -1.
 * Neighbours (section 2, the four unit-distance points): up = (i, j+1),
 * right = (i+1, j), down = (i, j-1), left = (i-1, j), all taken mod L.
 *
 * Dynamics (section 2, transition probabilities eqs. (15)-(16), and the
 * per-site independent sampling that follows them):
 *   half-step A: every tau_x is drawn with field  J (sigma_down + sigma_left) + q sigma_x
 *   half-step B: every sigma'_x is drawn with field J (tau_up + tau_right) + q tau_x
 *   P(new spin = +1) = e^h / (2 cosh h).
 * Step n (counted from 0) draws half-step A with half-step index t = 2n and
 * half-step B with t = 2n + 1.  Both half-steps read only the previous
 * lattice: that is what makes the automaton parallel (introduction, eq. (1)).
 *
 * Reading of the paper's ambiguities (each listed in the design notes):
 *   - the arrows on the two field symbols are not used; the neighbour sets of
 *     the two forms of the pair Hamiltonian (eq. (5)) decide which field drives
 *     which half-step;
 *   - the half-step order is the one of section 2 (down-left field first), not
 *     the mirror order of Algorithm 3 (equal in law, not pathwise);
 *   - "rand() < p" of Algorithm 3 becomes r < T with r a 32-bit uniform and T a
 *     32-bit threshold, see or_threshold().
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel Random Numbers: As  */
/* Easy as 1, 2, 3", SC'11).  Ten rounds of the Philox S-box on a 128-bit       */
/* counter, with the 64-bit key bumped by the Weyl constants between rounds.    */
/* ------------------------------------------------------------------------- */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u;
static const uint32_t PHILOX_W1 = 0xBB67AE85u;

OR_EXPORT void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t prod0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------- */
/* The per-site 32-bit uniform r_s(t) of the frozen stream contract.            */
/*                                                                              */
/* key = (seed mod 2^32, seed div 2^32).  Sites are grouped 64 at a time in     */
/* linear order: group g = s div 64, bit b = s mod 64.                          */
/*   plane calls, p = 0..3:  X = Philox(ctr = (stream, t | p<<30, 2*tag, g))    */
/*     plane 2p   = X0 | X1<<32,   plane 2p+1 = X2 | X3<<32                     */
/*     bit (31 - m) of r_s = bit b of plane m,  m = 0..7                        */
/*   tail call:  Y = Philox(ctr = (stream, t, 2*tag + 1, s div 4))              */
/*     bits 23..0 of r_s = (Y[s mod 4]) >> 8                                    */
/* tag 0 draws the dynamics, tag 1 the random initial lattice.                  */
/* ------------------------------------------------------------------------- */
enum { OR_TAG_DYNAMICS = 0, OR_TAG_INIT = 1 };

typedef struct {
    uint64_t seed;
    uint32_t stream, t, tag;
    uint64_t cached_group;  /* group whose planes are in plane[] (UINT64_MAX: none) */
    uint64_t plane[8];
    uint64_t cached_quad;   /* s div 4 whose tail call is in tail[] */
    uint32_t tail[4];
} or_uniform_source;

static void or_source_begin(or_uniform_source* src, uint64_t seed, uint32_t stream, uint32_t t, uint32_t tag)
{
    src->seed = seed;
    src->stream = stream;
    src->t = t;
    src->tag = tag;
    src->cached_group = UINT64_MAX;
    src->cached_quad = UINT64_MAX;
}

static uint32_t or_source_uniform(or_uniform_source* src, uint64_t s)
{
    const uint32_t key[2] = {(uint32_t)(src->seed & 0xFFFFFFFFu), (uint32_t)(src->seed >> 32)};
    const uint64_t g = s >> 6;
    const unsigned b = (unsigned)(s & 63u);
    if (g != src->cached_group) {
        for (uint32_t p = 0; p < 4; ++p) {
            uint32_t ctr[4] = {src->stream, src->t | (p << 30), 2u * src->tag, (uint32_t)g};
            uint32_t x[4];
            or_philox4x32_10(ctr, key, x);
            src->plane[2 * p] = (uint64_t)x[0] | ((uint64_t)x[1] << 32);
            src->plane[2 * p + 1] = (uint64_t)x[2] | ((uint64_t)x[3] << 32);
        }
        src->cached_group = g;
    }
    const uint64_t quad = s >> 2;
    if (quad != src->cached_quad) {
        uint32_t ctr[4] = {src->stream, src->t, 2u * src->tag + 1u, (uint32_t)quad};
        or_philox4x32_10(ctr, key, src->tail);
        src->cached_quad = quad;
    }
    uint32_t top = 0;
    for (int m = 0; m < 8; ++m)
        top = (top << 1) | (uint32_t)((src->plane[m] >> b) & 1u);
    return (top << 24) | (src->tail[s & 3u] >> 8);
}

/* Debug switch for the global spin-flip pin: when set, every uniform r is
 * replaced by 2^32 - 1 - r.  Not thread-safe; tests only. */
static int or_complement_randoms = 0;

OR_EXPORT void or_set_complement(int on) { or_complement_randoms = on ? 1 : 0; }

OR_EXPORT uint32_t or_site_uniform(uint64_t seed, uint32_t stream, uint32_t t, uint32_t tag, uint64_t s)
{
    or_uniform_source src;
    or_source_begin(&src, seed, stream, t, tag);
    uint32_t r = or_source_uniform(&src, s);
    return or_complement_randoms ? ~r : r;
}

/* ------------------------------------------------------------------------- */
/* Heat-bath threshold (Algorithm 3: draw +1 when rand() < e^h / (2 cosh h)).  */
/* With r uniform on [0, 2^32), +1 is drawn when r < T(h), where               */
/*   U = max(1, round-half-even(2^32 / (1 + exp(2|h|))))                       */
/*   T = 2^32 - U for h > 0,   T = U for h < 0,   T = 2^31 for h = 0.          */
/* T/2^32 differs from e^h/(2 cosh h) by at most 2^-33 whenever |h| < 11, and  */
/* T(-h) = 2^32 - T(h) holds exactly.                                          */
/* ------------------------------------------------------------------------- */
OR_EXPORT uint32_t or_threshold(double h)
{
    if (h == 0.0)
        return 0x80000000u;
    double a = fabs(h);
    double u = 4294967296.0 / (1.0 + exp(2.0 * a));
    double rounded = nearbyint(u);
    uint64_t U = (rounded < 1.0) ? 1u : (uint64_t)rounded;
    if (h > 0.0)
        return (uint32_t)(4294967296ull - U);
    return (uint32_t)U;
}

/* Local field of a site from its two J-neighbours n1, n2 and its partner c
 * (all +-1): h = J (n1 + n2) + q c  (section 2, eq. (14)). */
static double or_field(double J, double q, int n1, int n2, int c)
{
    return J * (double)(n1 + n2) + q * (double)c;
}

/* The six possible thresholds, indexed by idx = 2k + [c = +1], k = number of
 * +1 among the two J-neighbours. */
OR_EXPORT void or_threshold_table(double J, double q, uint32_t T[6])
{
    for (int k = 0; k <= 2; ++k) {
        for (int cplus = 0; cplus <= 1; ++cplus) {
            int n1 = (k >= 1) ? 1 : -1;
            int n2 = (k >= 2) ? 1 : -1;
            int c = cplus ? 1 : -1;
            T[2 * k + cplus] = or_threshold(or_field(J, q, n1, n2, c));
        }
    }
}

static int or_class_index(int n1, int n2, int c)
{
    int k = (n1 > 0) + (n2 > 0);
    return 2 * k + (c > 0);
}

static size_t or_site(int L, int i, int j)
{
    i = ((i % L) + L) % L;
    j = ((j % L) + L) % L;
    return (size_t)j * (size_t)L + (size_t)i;
}

/* ------------------------------------------------------------------------- */
/* Initial lattices (section 3.1 starts from all -1; the workloads also use     */
/* all +1 and i.i.d. +1 with probability p).                                    */
/* ------------------------------------------------------------------------- */
enum { OR_INIT_UP = 0, OR_INIT_DOWN = 1, OR_INIT_RANDOM = 2 };

OR_EXPORT int or_init(int8_t* sigma, int L, int kind, double p_up, uint64_t seed, uint32_t stream)
{
    size_t N = (size_t)L * (size_t)L;
    if (kind == OR_INIT_UP || kind == OR_INIT_DOWN) {
        for (size_t s = 0; s < N; ++s)
            sigma[s] = (kind == OR_INIT_UP) ? 1 : -1;
        return 0;
    }
    if (kind != OR_INIT_RANDOM || !(p_up >= 0.0 && p_up <= 1.0))
        return -1;
    /* +1 with probability P / 2^32, P = round-half-even(p * 2^32); P = 2^32 is all +1. */
    uint64_t P = (uint64_t)nearbyint(p_up * 4294967296.0);
    or_uniform_source src;
    or_source_begin(&src, seed, stream, 0u, OR_TAG_INIT);
    for (size_t s = 0; s < N; ++s) {
        uint32_t r = or_source_uniform(&src, s);
        if (or_complement_randoms)
            r = ~r;
        sigma[s] = ((uint64_t)r < P) ? 1 : -1;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Half-steps.                                                                  */
/* ------------------------------------------------------------------------- */

/* Per-site thresholds of one row j for one half-step, in the same order as the
 * sites of that row.  which = 0: half-step A, field J(src_down + src_left) +
 * q src_x; which = 1: half-step B, field J(src_up + src_right) + q src_x. */
OR_EXPORT void or_row_thresholds(const int8_t* src, int L, double J, double q, int which, int j, uint32_t* T_row)
{
    uint32_t T[6];
    or_threshold_table(J, q, T);
    for (int i = 0; i < L; ++i) {
        int n1, n2;
        if (which == 0) {
            n1 = src[or_site(L, i, j - 1)]; /* down */
            n2 = src[or_site(L, i - 1, j)]; /* left */
        } else {
            n1 = src[or_site(L, i, j + 1)]; /* up */
            n2 = src[or_site(L, i + 1, j)]; /* right */
        }
        T_row[i] = T[or_class_index(n1, n2, src[or_site(L, i, j)])];
    }
}

/* One half-step: every site of dst is drawn independently from src,
 * dst_x = +1 iff r_x(t) < T_x. */
static void or_half_step(const int8_t* src, int8_t* dst, int L, double J, double q, int which,
                         uint64_t seed, uint32_t stream, uint32_t t)
{
    uint32_t* T_row = (uint32_t*)malloc((size_t)L * sizeof(uint32_t));
    or_uniform_source rng;
    or_source_begin(&rng, seed, stream, t, OR_TAG_DYNAMICS);
    for (int j = 0; j < L; ++j) {
        or_row_thresholds(src, L, J, q, which, j, T_row);
        for (int i = 0; i < L; ++i) {
            size_t s = or_site(L, i, j);
            uint32_t r = or_source_uniform(&rng, s);
            if (or_complement_randoms)
                r = ~r;
            dst[s] = (r < T_row[i]) ? 1 : -1;
        }
    }
    free(T_row);
}

/* Half-step A: tau_x ~ field J(sigma_down + sigma_left) + q sigma_x. */
OR_EXPORT void or_half_step_A(const int8_t* sigma, int8_t* tau, int L, double J, double q,
                              uint64_t seed, uint32_t stream, uint32_t t)
{
    or_half_step(sigma, tau, L, J, q, 0, seed, stream, t);
}

/* Half-step B: sigma'_x ~ field J(tau_up + tau_right) + q tau_x. */
OR_EXPORT void or_half_step_B(const int8_t* tau, int8_t* sigma_out, int L, double J, double q,
                              uint64_t seed, uint32_t stream, uint32_t t)
{
    or_half_step(tau, sigma_out, L, J, q, 1, seed, stream, t);
}

/* ------------------------------------------------------------------------- */
/* Observables on the pair (sigma, tau) (section 3.1 magnetisation; section 2  */
/* pair Hamiltonian eq. (5)):                                                   */
/*   M = sum_x sigma_x,  A = sum_x sigma_x (tau_up + tau_right),                */
/*   B = sum_x sigma_x tau_x,  so that H(sigma, tau) = -(J A + q B).            */
/* ------------------------------------------------------------------------- */
OR_EXPORT void or_observe(const int8_t* sigma, const int8_t* tau, int L, int64_t out[3])
{
    int64_t M = 0, A = 0, B = 0;
    for (int j = 0; j < L; ++j) {
        for (int i = 0; i < L; ++i) {
            int sx = sigma[or_site(L, i, j)];
            M += sx;
            A += (int64_t)sx * (tau[or_site(L, i, j + 1)] + tau[or_site(L, i + 1, j)]);
            B += (int64_t)sx * tau[or_site(L, i, j)];
        }
    }
    out[0] = M;
    out[1] = A;
    out[2] = B;
}

/* Row-wise spin-spin correlation sums D(r) = sum_x sigma_(i,j) sigma_(i+r,j),
 * r = 0..rmax (the connected / normalised forms are taken on the host). */
OR_EXPORT int or_corr_row(const int8_t* sigma, int L, int rmax, int64_t* out)
{
    if (rmax < 0 || rmax >= L)
        return -1;
    for (int r = 0; r <= rmax; ++r) {
        int64_t D = 0;
        for (int j = 0; j < L; ++j)
            for (int i = 0; i < L; ++i)
                D += (int64_t)sigma[or_site(L, i, j)] * sigma[or_site(L, i + r, j)];
        out[r] = D;
    }
    return 0;
}

/* Diagonal correlation sums of section 3.3 (Table 1), brute force:           */
/* out[l] = sum_x sigma(i,j) sigma(i+l, j+l)            (SW-NE direction),      */
/* out[lmax+1+l] = sum_x sigma(i,j) sigma(i+l, j-l)     (NW-SE direction),      */
/* l = 0 .. lmax, coordinates mod L.                                             */
OR_EXPORT int or_corr_diag(const int8_t* sigma, int L, int lmax, int64_t* out)
{
    if (lmax < 0 || lmax >= L)
        return -1;
    for (int l = 0; l <= lmax; ++l) {
        int64_t up = 0, down = 0;
        for (int j = 0; j < L; ++j)
            for (int i = 0; i < L; ++i) {
                const int64_t s = sigma[or_site(L, i, j)];
                up += s * sigma[or_site(L, i + l, j + l)];
                down += s * sigma[or_site(L, i + l, j - l)];
            }
        out[l] = up;
        out[lmax + 1 + l] = down;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Chain driver: k full steps from step index step0, recording (M, A, B) on the */
/* pair (sigma_n, tau_n) after every obs_every-th step (obs may be NULL).       */
/* sigma is updated in place; tau receives the last half-step-A lattice.        */
/* ------------------------------------------------------------------------- */
OR_EXPORT int or_run(int8_t* sigma, int8_t* tau, int L, double J, double q, uint64_t seed,
                     uint32_t stream, uint64_t step0, uint32_t k, int64_t* obs, uint32_t obs_every)
{
    if (L < 2 || (obs && obs_every == 0))
        return -1;
    if (step0 + (uint64_t)k > (1ull << 29))
        return -1;
    for (uint32_t m = 0; m < k; ++m) {
        uint64_t n = step0 + m;
        or_half_step_A(sigma, tau, L, J, q, seed, stream, (uint32_t)(2 * n));
        or_half_step_B(tau, sigma, L, J, q, seed, stream, (uint32_t)(2 * n + 1));
        if (obs && ((m + 1) % obs_every) == 0)
            or_observe(sigma, tau, L, obs + 3 * (size_t)((m + 1) / obs_every - 1));
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Coupling from the past (Propp and Wilson), the exact sampler that section   */
/* 3.2 builds on the coupling.  For J, q >= 0 one full step is monotone: with   */
/* the same uniforms, sigma <= sigma' site by site stays so after the step.     */
/* The uniforms of time -t (t = 1, 2, ...) are those of step index             */
/* step_end - t.  T runs through T0, 2 T0, 4 T0, ... while T <= T_max; the      */
/* chains started from all +1 and all -1 at time -T are run to time 0, and at   */
/* the first T where they agree their common lattice is the sample (every      */
/* chain started at -T lies between them).  Returns that T; 0 if no T up to    */
/* T_max coalesced (sample: the top chain at time 0 from the largest T tried); */
/* -1 on bad arguments.                                                         */
/* ------------------------------------------------------------------------- */
OR_EXPORT int64_t or_propp_wilson(int8_t* sample, int L, double J, double q, uint64_t seed, uint32_t stream,
                                  uint64_t step_end, uint32_t T0, uint32_t T_max)
{
    if (L < 2 || T0 < 1 || T_max < T0 || !(J >= 0.0) || !(q >= 0.0) || step_end < T_max ||
        step_end > (1ull << 29))
        return -1;
    size_t N = (size_t)L * (size_t)L;
    int8_t* top = (int8_t*)malloc(N);
    int8_t* bot = (int8_t*)malloc(N);
    int8_t* tau = (int8_t*)malloc(N);
    if (!top || !bot || !tau) {
        free(top);
        free(bot);
        free(tau);
        return -1;
    }
    int64_t found = 0;
    for (uint64_t T = T0; T <= T_max; T *= 2) {
        or_init(top, L, OR_INIT_UP, 0.5, seed, stream);
        or_init(bot, L, OR_INIT_DOWN, 0.5, seed, stream);
        or_run(top, tau, L, J, q, seed, stream, step_end - T, (uint32_t)T, NULL, 0);
        or_run(bot, tau, L, J, q, seed, stream, step_end - T, (uint32_t)T, NULL, 0);
        memcpy(sample, top, N);
        if (memcmp(top, bot, N) == 0) {
            found = (int64_t)T;
            break;
        }
    }
    free(top);
    free(bot);
    free(tau);
    return found;
}

/* ------------------------------------------------------------------------- */
/* Trajectory log-likelihood.  A trajectory is X_0 = sigma_0, X_1 = tau_1,      */
/* X_2 = sigma_1, ...; the transition X_m -> X_(m+1) is a half-step A draw for  */
/* even m and a half-step B draw for odd m.  By the product form of eqs.        */
/* (15)-(16) its log-probability is sum_x [h_x s_x - log 2cosh h_x], s_x being  */
/* the drawn spin.  The sufficient statistics are the 12 counts                 */
/*   counts[2*idx + [s = +1]],  idx = 2k + [c = +1]                             */
/* over all sites of all transitions of all trajectories.                      */
/* traj holds n_traj trajectories of n_lat lattices of L*L int8 each.           */
/* ------------------------------------------------------------------------- */
OR_EXPORT int or_loglik_counts(const int8_t* traj, int n_traj, int n_lat, int L, int64_t counts[12])
{
    if (n_traj < 0 || n_lat < 1 || L < 2)
        return -1;
    memset(counts, 0, 12 * sizeof(int64_t));
    size_t N = (size_t)L * (size_t)L;
    for (int a = 0; a < n_traj; ++a) {
        for (int m = 0; m + 1 < n_lat; ++m) {
            const int8_t* X = traj + ((size_t)a * (size_t)n_lat + (size_t)m) * N;
            const int8_t* Y = X + N;
            for (int j = 0; j < L; ++j) {
                for (int i = 0; i < L; ++i) {
                    int n1, n2;
                    if ((m & 1) == 0) { /* half-step A: down and left neighbours */
                        n1 = X[or_site(L, i, j - 1)];
                        n2 = X[or_site(L, i - 1, j)];
                    } else { /* half-step B: up and right neighbours */
                        n1 = X[or_site(L, i, j + 1)];
                        n2 = X[or_site(L, i + 1, j)];
                    }
                    int c = X[or_site(L, i, j)];
                    int s = Y[or_site(L, i, j)];
                    counts[2 * or_class_index(n1, n2, c) + (s > 0)] += 1;
                }
            }
        }
    }
    return 0;
}

/* Paired sufficient statistics.  Classes idx and 5 - idx have opposite fields
 * (h -> -h); log 2cosh is even and tanh odd, so the log-likelihood and its
 * gradient depend on each pair j = (j, 5 - j), j = 0, 1, 2, only through
 *   S_j = number of sites of the pair,
 *   Z_j = sites of class j drawn +1 plus sites of class 5 - j drawn -1,
 * by a site loop over every transition as in or_loglik_counts.
 * stats[0..2] = S_0..S_2, stats[3..5] = Z_0..Z_2. */
OR_EXPORT int or_loglik_stats(const int8_t* traj, int n_traj, int n_lat, int L, int64_t stats[6])
{
    if (n_traj < 0 || n_lat < 1 || L < 2)
        return -1;
    memset(stats, 0, 6 * sizeof(int64_t));
    size_t N = (size_t)L * (size_t)L;
    for (int a = 0; a < n_traj; ++a) {
        for (int m = 0; m + 1 < n_lat; ++m) {
            const int8_t* X = traj + ((size_t)a * (size_t)n_lat + (size_t)m) * N;
            const int8_t* Y = X + N;
            for (int j = 0; j < L; ++j) {
                for (int i = 0; i < L; ++i) {
                    int n1, n2;
                    if ((m & 1) == 0) {
                        n1 = X[or_site(L, i, j - 1)];
                        n2 = X[or_site(L, i - 1, j)];
                    } else {
                        n1 = X[or_site(L, i, j + 1)];
                        n2 = X[or_site(L, i + 1, j)];
                    }
                    int idx = or_class_index(n1, n2, X[or_site(L, i, j)]);
                    int s = Y[or_site(L, i, j)];
                    int leader = idx < 3;
                    int pair = leader ? idx : 5 - idx;
                    stats[pair] += 1;
                    stats[3 + pair] += leader ? (s > 0) : (s < 0);
                }
            }
        }
    }
    return 0;
}

/* LL and its gradient from the paired statistics, in FP64: the leader class j
 * has h_j = J (2k - 2) + q c, and the pair contributes
 * h_j (2 Z_j - S_j) - S_j log 2cosh h_j, resp. (a_j, c_j) (2 Z_j - S_j - S_j tanh h_j). */
static double or_log2cosh(double h);

OR_EXPORT double or_loglik_from_stats(const int64_t stats[6], double J, double q, double grad[2])
{
    double ll = 0.0, gJ = 0.0, gq = 0.0;
    for (int j = 0; j < 3; ++j) {
        int k = j >> 1, cplus = j & 1;
        double a = (double)(2 * k - 2), c = (double)(2 * cplus - 1);
        double h = J * a + q * c;
        double S = (double)stats[j], D = 2.0 * (double)stats[3 + j] - (double)stats[j];
        ll += h * D - S * or_log2cosh(h);
        gJ += a * (D - S * tanh(h));
        gq += c * (D - S * tanh(h));
    }
    if (grad) {
        grad[0] = gJ;
        grad[1] = gq;
    }
    return ll;
}

/* log(2 cosh h) without overflow: |h| + log1p(exp(-2|h|)). */
static double or_log2cosh(double h)
{
    double a = fabs(h);
    return a + log1p(exp(-2.0 * a));
}

/* LL(J, q) = sum over the 12 counts of n * (h s - log 2cosh h), in FP64. */
OR_EXPORT double or_loglik(const int64_t counts[12], double J, double q)
{
    double ll = 0.0;
    for (int k = 0; k <= 2; ++k) {
        for (int cplus = 0; cplus <= 1; ++cplus) {
            double h = J * (double)(2 * k - 2) + q * (double)(2 * cplus - 1);
            for (int splus = 0; splus <= 1; ++splus) {
                double s = splus ? 1.0 : -1.0;
                double n = (double)counts[2 * (2 * k + cplus) + splus];
                ll += n * (h * s - or_log2cosh(h));
            }
        }
    }
    return ll;
}

/* Gradient of LL: dh/dJ = 2k - 2, dh/dq = c, and
 * d/dh [h s - log 2cosh h] = s - tanh h. */
OR_EXPORT void or_loglik_grad(const int64_t counts[12], double J, double q, double grad[2])
{
    double gJ = 0.0, gq = 0.0;
    for (int k = 0; k <= 2; ++k) {
        for (int cplus = 0; cplus <= 1; ++cplus) {
            double a = (double)(2 * k - 2);
            double c = (double)(2 * cplus - 1);
            double h = J * a + q * c;
            for (int splus = 0; splus <= 1; ++splus) {
                double s = splus ? 1.0 : -1.0;
                double n = (double)counts[2 * (2 * k + cplus) + splus];
                gJ += n * a * (s - tanh(h));
                gq += n * c * (s - tanh(h));
            }
        }
    }
    grad[0] = gJ;
    grad[1] = gq;
}
