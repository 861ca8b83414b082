/*
 * Driver for the sanitizer test of the library's host code: the pure host
 * functions (lattice sizes, threshold tables, the fast division) over their
 * whole argument ranges, and every entry point with invalid arguments, which
 * must come back as SD_EINVAL / SD_EUNSUPPORTED with a message and touch
 * nothing.  Built, with the library's host code, under AddressSanitizer and
 * UndefinedBehaviorSanitizer.  Runs without a GPU: no call here gets past its
 * argument checks (device pointers are never dereferenced on the host).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "shaken.h"

static int failures = 0;

static void expect_err(sd_status s, const char* what) {
    if (s != SD_EINVAL && s != SD_EUNSUPPORTED) {
        printf("FAIL %s: status %d\n", what, (int)s);
        ++failures;
    } else if (strlen(sd_last_error()) == 0) {
        printf("FAIL %s: empty message\n", what);
        ++failures;
    }
}

int main(void) {
    void* p = (void*)(uintptr_t)0x100000;   /* aligned, never dereferenced */
    void* p2 = (void*)(uintptr_t)0x200000;
    int64_t* o = (int64_t*)(uintptr_t)0x300000;
    uint32_t T[6];
    if (sd_abi_version() != SD_ABI_VERSION) ++failures;
    for (int32_t L = -3; L < 300; ++L)
        for (int32_t lay = -1; lay < 4; ++lay)
            (void)sd_lattice_bytes(L, lay);
    if (sd_lattice_bytes(65535, SD_I8) != 65535ull * 65535ull) ++failures;
    (void)sd_lattice_bytes(65536, SD_P64);
    (void)sd_lattice_bytes(INT32_MAX, SD_P32);
    for (double J = -40.0; J <= 40.0; J += 0.73)
        for (double q = -40.0; q <= 40.0; q += 1.31)
            if (sd_threshold_table(J, q, T) != SD_OK) ++failures;
    expect_err(sd_threshold_table(NAN, 0.5, T), "table NaN");
    expect_err(sd_threshold_table(0.5, INFINITY, T), "table inf");
    expect_err(sd_threshold_table(0.5, 0.5, NULL), "table null");
    for (uint32_t d = 1; d < 70000; d += 7)
        for (uint32_t n = 0; n < 4000000000u; n += 99991u)
            if (sd_debug_fastdiv(n, d) != n / d) { ++failures; break; }
    (void)sd_debug_fastdiv(5, 0);

    expect_err(sd_init(NULL, 64, SD_P64, SD_INIT_UP, 0.5, 1, 0, NULL), "init null");
    expect_err(sd_init(p, 1, SD_I8, SD_INIT_UP, 0.5, 1, 0, NULL), "init L=1");
    expect_err(sd_init(p, 65536, SD_I8, SD_INIT_UP, 0.5, 1, 0, NULL), "init L too large");
    expect_err(sd_init(p, 60, SD_P32, SD_INIT_UP, 0.5, 1, 0, NULL), "init P32 L");
    expect_err(sd_init(p, 64, SD_P64, 7, 0.5, 1, 0, NULL), "init kind");
    expect_err(sd_init(p, 64, SD_P64, SD_INIT_RANDOM, 1.5, 1, 0, NULL), "init p");
    expect_err(sd_init(p, 64, SD_P64, SD_INIT_RANDOM, NAN, 1, 0, NULL), "init p NaN");
    expect_err(sd_init((char*)p + 4, 64, SD_P64, SD_INIT_UP, 0.5, 1, 0, NULL), "init misaligned");
    expect_err(sd_half_step(p, p, 64, SD_P64, 0, 0.5, 0.5, 1, 0, 0, 0, NULL), "half overlap");
    expect_err(sd_half_step(p, p2, 64, SD_P64, 2, 0.5, 0.5, 1, 0, 0, 0, NULL), "half which");
    expect_err(sd_half_step(p, p2, 64, SD_P64, 0, 0.5, 0.5, 1, 0, 1u << 30, 0, NULL), "half t");
    expect_err(sd_half_step(p, p2, 64, SD_P64, 0, 0.5, 0.5, 1, 0, 0, 1u << 7, NULL), "half flags");
    expect_err(sd_run(p, p, 64, SD_P64, 0.5, 0.5, 1, 0, 0, 5, NULL, 0, 0, NULL), "run overlap");
    expect_err(sd_run(p, p2, 64, SD_P64, 0.5, 0.5, 1, 0, 1ull << 29, 1, NULL, 0, 0, NULL), "run step0");
    expect_err(sd_run(p, p2, 64, SD_P64, 0.5, 0.5, 1, 0, 0, 5, o, 0, 0, NULL), "run obs_every");
    expect_err(sd_run(p, p2, 64, SD_P64, 0.5, NAN, 1, 0, 0, 5, NULL, 0, 0, NULL), "run NaN");
    expect_err(sd_run(p, p2, 64, SD_P64, 0.5, 0.5, 1, 0, 0, 5, NULL, 0, 1u << 9, NULL), "run flags");
    expect_err(sd_run_noalloc(p, p, 64, SD_P64, 0.5, 0.5, 1, 0, 0, 5, NULL, 0, 0, NULL), "noalloc overlap");
    expect_err(sd_run_noalloc(p, p2, 64, SD_P64, 0.5, 0.5, 1, 0, 0, 5, o, 0, 0, NULL), "noalloc obs_every");
    {
        void* sg[2] = {p, p2};
        void* tg[2] = {(char*)p2 + 64, (char*)p + 8192};
        double J[2] = {0.5, 0.5}, q[2] = {0.5, 0.5};
        uint32_t st[2] = {0, 1};
        expect_err(sd_run_many(sg, tg, 2, 64, SD_P64, J, q, 1, st, 0, 2, NULL, 0, 0, NULL), "many overlap");
        expect_err(sd_run_many(sg, tg, 0, 64, SD_P64, J, q, 1, st, 0, 2, NULL, 0, 0, NULL), "many n=0");
        expect_err(sd_run_many(sg, tg, 17, 64, SD_P64, J, q, 1, st, 0, 2, NULL, 0, 0, NULL), "many n=17");
        expect_err(sd_run_many(NULL, tg, 1, 64, SD_P64, J, q, 1, st, 0, 2, NULL, 0, 0, NULL), "many null");
    }
    expect_err(sd_observe(p, p2, 64, SD_P64, NULL, NULL), "observe null");
    expect_err(sd_corr_row(p, 64, SD_P64, 64, o, NULL), "corr rmax");
    expect_err(sd_corr_row(p, 64, SD_P64, -1, o, NULL), "corr rmax<0");
    {
        const void* lg[2] = {p, p2};
        expect_err(sd_corr_row_many(lg, 0, 64, SD_P64, 3, o, NULL), "corr many n=0");
        expect_err(sd_corr_row_many(lg, 17, 64, SD_P64, 3, o, NULL), "corr many n=17");
        expect_err(sd_corr_row_many(NULL, 2, 64, SD_P64, 3, o, NULL), "corr many null");
        expect_err(sd_corr_row_many(lg, 2, 64, SD_P64, 64, o, NULL), "corr many rmax");
    }
    expect_err(sd_corr_diag(p, 64, SD_P64, 64, o, NULL), "diag lmax");
    expect_err(sd_trajectory(p, p2, 64, SD_I8, 0.5, 0.5, 1, 0, 0, 3, NULL), "trajectory layout");
    expect_err(sd_trajectories(p, p2, -1, 64, SD_P64, 0.5, 0.5, 1, 0, 0, 3, NULL), "trajectories n");
    expect_err(sd_loglik_counts(NULL, 1, 3, 64, o, NULL), "counts null");
    expect_err(sd_loglik_counts(p, 1, 3, 40, o, NULL), "counts L");
    expect_err(sd_loglik_stats(p, 1, 0, 64, o, NULL), "stats n_lat");
    expect_err(sd_loglik_fwd(NULL, (const float*)p, (float*)p2, NULL), "fwd null");
    expect_err(sd_loglik_bwd(o, NULL, NULL, (float*)p2, NULL), "bwd null");
    expect_err(sd_replica_run(p, p2, 12, NULL, NULL, 1, 0, 0, 1, NULL), "replica null");
    {
        float t0 = 0.0f, t1 = 0.0f;
        expect_err(sd_batch_bucket_times(NULL, 0, &t0, &t1), "bucket times null plan");
    }
    {
        double J64[64], q64[64];
        for (int i = 0; i < 64; ++i) { J64[i] = 0.5; q64[i] = 0.5; }
        J64[7] = NAN;
        expect_err(sd_replica_run(p, p2, 64, J64, q64, 1, 0, 0, 1, NULL), "replica NaN");
        expect_err(sd_replica_run(p, p2, 12, J64, q64, 1, 0, 0, 1, NULL), "replica L");
    }
    {
        int64_t Tu[4];
        expect_err(sd_propp_wilson(p, p2, 4, 32, -0.5, 0.5, 1, 0, 1u << 20, 4, 64, Tu, NULL), "pw J<0");
        expect_err(sd_propp_wilson(p, p2, 4, 32, 0.5, 0.5, 1, 0, 1u << 20, 128, 64, Tu, NULL), "pw T0>Tmax");
    }
    {
        sd_batch_plan* plan = NULL;
        sd_chain_desc d[2] = {{0.5, 0.5, 64, 0}, {0.5, 0.5, 7, 1}};
        expect_err(sd_batch_plan_create(&plan, d, 0, SD_P64, 1, 10, 1, 0, NULL), "plan n=0");
        expect_err(sd_batch_plan_create(&plan, d, 2, SD_P64, 1, 10, 1, 0, NULL), "plan L=7");
        expect_err(sd_batch_plan_create(NULL, d, 1, SD_P64, 1, 10, 1, 0, NULL), "plan null");
        if (sd_batch_lattice_bytes(NULL) != 0 || sd_batch_trace_len(NULL) != 0) ++failures;
        if (sd_batch_chain_offset(NULL, 0, 0) != -1) ++failures;
        sd_batch_plan_destroy(NULL);
    }
    printf("sanitized ABI run: %d failure(s)\n", failures);
    return failures ? 1 : 0;
}
