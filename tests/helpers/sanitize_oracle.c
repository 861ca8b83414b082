/*
 * Driver for the sanitizer test: every exported oracle function on small and
 * edge-sized inputs (L = 2, 3, 5, 17, 64; step indices just below 2^29; both
 * half-steps; records; correlations at rmax = L - 1; log-likelihood counts
 * and statistics; coupling from the past), built with AddressSanitizer and
 * UndefinedBehaviorSanitizer so that any out-of-bounds access, overflow or
 * other undefined behaviour aborts the run.  Prints a checksum of the
 * results so that nothing is optimised away.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]);
void or_set_complement(int on);
uint32_t or_site_uniform(uint64_t seed, uint32_t stream, uint32_t t, uint32_t tag, uint64_t s);
uint32_t or_threshold(double h);
void or_threshold_table(double J, double q, uint32_t T[6]);
int or_init(int8_t* sigma, int L, int kind, double p_up, uint64_t seed, uint32_t stream);
void or_row_thresholds(const int8_t* src, int L, double J, double q, int which, int j, uint32_t* T_row);
void or_half_step_A(const int8_t* sigma, int8_t* tau, int L, double J, double q, uint64_t seed, uint32_t stream,
                    uint32_t t);
void or_half_step_B(const int8_t* tau, int8_t* sigma_out, int L, double J, double q, uint64_t seed, uint32_t stream,
                    uint32_t t);
void or_observe(const int8_t* sigma, const int8_t* tau, int L, int64_t out[3]);
int or_corr_row(const int8_t* sigma, int L, int rmax, int64_t* out);
int or_corr_diag(const int8_t* sigma, int L, int lmax, int64_t* out);
int or_run(int8_t* sigma, int8_t* tau, int L, double J, double q, uint64_t seed, uint32_t stream, uint64_t step0,
           uint32_t k, int64_t* obs, uint32_t obs_every);
int64_t or_propp_wilson(int8_t* sample, int L, double J, double q, uint64_t seed, uint32_t stream, uint64_t step_end,
                        uint32_t T0, uint32_t T_max);
int or_loglik_counts(const int8_t* traj, int n_traj, int n_lat, int L, int64_t counts[12]);
int or_loglik_stats(const int8_t* traj, int n_traj, int n_lat, int L, int64_t stats[6]);
double or_loglik_from_stats(const int64_t stats[6], double J, double q, double grad[2]);
double or_loglik(const int64_t counts[12], double J, double q);
void or_loglik_grad(const int64_t counts[12], double J, double q, double grad[2]);

static uint64_t mix(uint64_t h, int64_t v) { return (h ^ (uint64_t)v) * 0x100000001B3ull; }

int main(void) {
    uint64_t h = 0xCBF29CE484222325ull;
    const int sizes[] = {2, 3, 5, 17, 64};
    uint32_t ctr[4] = {0xFFFFFFFFu, 0, 0xFFFFFFFFu, 7}, key[2] = {0xFFFFFFFFu, 0xFFFFFFFFu}, out4[4];
    or_philox4x32_10(ctr, key, out4);
    for (int i = 0; i < 4; ++i) h = mix(h, out4[i]);
    for (double x = -12.0; x <= 12.0; x += 0.37) h = mix(h, or_threshold(x));
    for (size_t si = 0; si < sizeof sizes / sizeof sizes[0]; ++si) {
        const int L = sizes[si];
        const size_t n = (size_t)L * L;
        int8_t* s = malloc(n);
        int8_t* t = malloc(n);
        int64_t* obs = malloc(sizeof(int64_t) * 3 * 6);
        int64_t* corr = malloc(sizeof(int64_t) * 2 * L);
        uint32_t* row = malloc(sizeof(uint32_t) * L);
        if (!s || !t || !obs || !corr || !row) return 2;
        for (int kind = 0; kind < 3; ++kind) {
            if (or_init(s, L, kind, 0.37, 0xDEADBEEFCAFEull, 3) != 0) return 3;
            h = mix(h, s[n - 1]);
        }
        for (int cmp = 0; cmp < 2; ++cmp) {
            or_set_complement(cmp);
            /* step indices just below the 2^29 limit, then from zero */
            if (or_run(s, t, L, 0.45, 0.7, 1, 9, (1ull << 29) - 6, 6, obs, 1) != 0) return 4;
            for (int i = 0; i < 18; ++i) h = mix(h, obs[i]);
            if (or_run(s, t, L, -0.3, 1.2, 1, 9, 0, 5, obs, 2) != 0) return 5;
        }
        or_set_complement(0);
        or_half_step_A(s, t, L, 0.0, 0.0, 2, 1, (1u << 30) - 2);
        or_half_step_B(t, s, L, 1.5, 2.0, 2, 1, (1u << 30) - 1);
        for (int j = 0; j < L; ++j) {
            or_row_thresholds(s, L, 0.4, 0.6, j & 1, j, row);
            h = mix(h, row[L - 1]);
        }
        int64_t o3[3];
        or_observe(s, t, L, o3);
        h = mix(h, o3[0] + o3[1] + o3[2]);
        if (or_corr_row(s, L, L - 1, corr) != 0) return 6;
        h = mix(h, corr[L - 1]);
        if (or_corr_diag(s, L, L - 1, corr) != 0) return 7;
        h = mix(h, corr[2 * L - 1]);
        h = mix(h, or_site_uniform(~0ull, 0xFFFFFFFFu, (1u << 30) - 1, 1, n - 1));
        /* a two-trajectory set of three lattices each */
        int8_t* traj = malloc(2 * 3 * n);
        if (!traj) return 8;
        for (int a = 0; a < 2; ++a) {
            or_init(traj + a * 3 * n, L, 2, 0.5, 5, a);
            or_half_step_A(traj + a * 3 * n, traj + a * 3 * n + n, L, 0.45, 0.7, 5, a, 0);
            or_half_step_B(traj + a * 3 * n + n, traj + a * 3 * n + 2 * n, L, 0.45, 0.7, 5, a, 1);
        }
        int64_t c12[12], s6[6];
        double g[2];
        if (or_loglik_counts(traj, 2, 3, L, c12) != 0) return 9;
        if (or_loglik_stats(traj, 2, 3, L, s6) != 0) return 10;
        h = mix(h, (int64_t)(1e3 * or_loglik(c12, 0.45, 0.7)));
        or_loglik_grad(c12, 0.2, 0.2, g);
        h = mix(h, (int64_t)(1e3 * g[0]));
        h = mix(h, (int64_t)(1e3 * or_loglik_from_stats(s6, 0.45, 0.7, g)));
        if (L <= 17) {
            int64_t T = or_propp_wilson(s, L, 0.3, 0.5, 3, 4, 1u << 20, 4, 1u << 12);
            if (T < 0) return 11;
            h = mix(h, T);
        }
        free(traj);
        free(s);
        free(t);
        free(obs);
        free(corr);
        free(row);
    }
    printf("sanitized oracle run ok %016llx\n", (unsigned long long)h);
    return 0;
}
