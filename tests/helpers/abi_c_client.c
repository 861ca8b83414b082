/*
 * A plain C client of libshaken: device memory from the HIP runtime, no
 * PyTorch.  Checks, through the C ABI only:
 *   - a chain of 100 steps with (M, A, B) every 10 steps, on a lattice that
 *     takes the grid kernels (1024^2) and on one that takes the
 *     single-workgroup kernel (64^2): the last record equals sd_observe of
 *     the returned pair, and 50 + 50 steps (the second call from step 50)
 *     give the same lattices and records as 100 steps;
 *   - argument errors come back as SD_EINVAL with a message and no device work.
 * Prints one line and exits 0 on success, 1 on a failed check.
 */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "shaken.h"

#define CHECK_HIP(x)                                                         \
    do {                                                                     \
        hipError_t e_ = (x);                                                 \
        if (e_ != hipSuccess) {                                              \
            printf("abi c client: %s failed: %s\n", #x, hipGetErrorString(e_)); \
            return 1;                                                        \
        }                                                                    \
    } while (0)

#define CHECK_SD(x)                                                          \
    do {                                                                     \
        sd_status s_ = (x);                                                  \
        if (s_ != SD_OK) {                                                   \
            printf("abi c client: %s returned %d: %s\n", #x, (int)s_, sd_last_error()); \
            return 1;                                                        \
        }                                                                    \
    } while (0)

enum { kSteps = 100, kEvery = 10, kRecords = kSteps / kEvery };

static int chain_checks(int32_t L, hipStream_t st) {
    const size_t nb = sd_lattice_bytes(L, SD_P64);
    void *s1 = NULL, *t1 = NULL, *s2 = NULL, *t2 = NULL;
    int64_t *obs1 = NULL, *obs2 = NULL, *o3 = NULL;
    static uint8_t h1[1024 * 1024 / 8], h2[1024 * 1024 / 8];
    int64_t r1[kRecords * 3], r2[kRecords * 3], last[3];
    if (nb == 0 || nb > sizeof h1) {
        printf("abi c client: unexpected lattice size %zu at L=%d\n", nb, (int)L);
        return 1;
    }
    CHECK_HIP(hipMalloc(&s1, nb));
    CHECK_HIP(hipMalloc(&t1, nb));
    CHECK_HIP(hipMalloc(&s2, nb));
    CHECK_HIP(hipMalloc(&t2, nb));
    CHECK_HIP(hipMalloc((void**)&obs1, sizeof r1));
    CHECK_HIP(hipMalloc((void**)&obs2, sizeof r2));
    CHECK_HIP(hipMalloc((void**)&o3, sizeof last));
    CHECK_SD(sd_init(s1, L, SD_P64, SD_INIT_RANDOM, 0.5, 7, 3, st));
    CHECK_SD(sd_init(s2, L, SD_P64, SD_INIT_RANDOM, 0.5, 7, 3, st));
    /* one call of 100 steps */
    CHECK_SD(sd_run(s1, t1, L, SD_P64, 0.45, 0.7, 7, 3, 0, kSteps, obs1, kEvery, 0, st));
    CHECK_SD(sd_observe(s1, t1, L, SD_P64, o3, st));
    /* 50 + 50 steps, the records of each call in its own half of obs2 */
    CHECK_SD(sd_run(s2, t2, L, SD_P64, 0.45, 0.7, 7, 3, 0, kSteps / 2, obs2, kEvery, 0, st));
    CHECK_SD(sd_run(s2, t2, L, SD_P64, 0.45, 0.7, 7, 3, kSteps / 2, kSteps / 2, obs2 + 3 * (kRecords / 2), kEvery,
                    0, st));
    CHECK_HIP(hipStreamSynchronize(st));
    CHECK_HIP(hipMemcpy(r1, obs1, sizeof r1, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(r2, obs2, sizeof r2, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(last, o3, sizeof last, hipMemcpyDeviceToHost));
    if (memcmp(last, r1 + 3 * (kRecords - 1), sizeof last) != 0) {
        printf("abi c client: L=%d last record (%lld, %lld, %lld) != sd_observe (%lld, %lld, %lld)\n", (int)L,
               (long long)r1[3 * (kRecords - 1)], (long long)r1[3 * (kRecords - 1) + 1],
               (long long)r1[3 * (kRecords - 1) + 2], (long long)last[0], (long long)last[1], (long long)last[2]);
        return 1;
    }
    if (memcmp(r1, r2, sizeof r1) != 0) {
        printf("abi c client: L=%d records of 100 steps differ from 50 + 50 steps\n", (int)L);
        return 1;
    }
    CHECK_HIP(hipMemcpy(h1, s1, nb, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(h2, s2, nb, hipMemcpyDeviceToHost));
    if (memcmp(h1, h2, nb) != 0) {
        printf("abi c client: L=%d sigma after 100 steps differs from 50 + 50 steps\n", (int)L);
        return 1;
    }
    CHECK_HIP(hipMemcpy(h1, t1, nb, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(h2, t2, nb, hipMemcpyDeviceToHost));
    if (memcmp(h1, h2, nb) != 0) {
        printf("abi c client: L=%d tau after 100 steps differs from 50 + 50 steps\n", (int)L);
        return 1;
    }
    if (last[0] < -(int64_t)L * L || last[0] > (int64_t)L * L) {
        printf("abi c client: L=%d magnetisation %lld out of range\n", (int)L, (long long)last[0]);
        return 1;
    }
    hipFree(s1);
    hipFree(t1);
    hipFree(s2);
    hipFree(t2);
    hipFree(obs1);
    hipFree(obs2);
    hipFree(o3);
    return 0;
}

int main(void) {
    hipStream_t st = NULL;
    CHECK_HIP(hipStreamCreate(&st));
    /* argument errors: rejected before any device work */
    if (sd_lattice_bytes(7, SD_P64) != 0) {
        printf("abi c client: L=7 packed accepted\n");
        return 1;
    }
    if (sd_init(NULL, 64, SD_P64, SD_INIT_UP, 0.5, 1, 0, st) != SD_EINVAL || sd_last_error()[0] == '\0') {
        printf("abi c client: null lattice not rejected with a message\n");
        return 1;
    }
    if (chain_checks(1024, st) != 0 || chain_checks(64, st) != 0)
        return 1;
    CHECK_HIP(hipStreamDestroy(st));
    printf("abi c client: ok (1024^2 grid kernels and 64^2 single-workgroup kernel, resume identity, "
           "records against sd_observe, argument errors)\n");
    return 0;
}
