/* Plain-C use of the library through include/cpht.h: no Python, no torch.
 *
 * Builds a compact cuckoo table from 2^20 distinct keys, looks up those keys
 * and as many keys that were never inserted, then runs one mixed batch on a
 * compact iceberg table (find-or-put of fresh keys, each twice, and finds of
 * absent keys).  Keys are an odd-multiplier bijection of their index modulo
 * 2^w, so the expected answers are known on the host.  Prints one line and
 * exits 0 when every answer is as expected. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "cpht.h"

#define CHECK(call)                                                                 \
    do {                                                                            \
        cpht_status_t st_ = (call);                                                 \
        if (st_ != CPHT_OK) {                                                       \
            fprintf(stderr, "%s failed: %s\n", #call, cpht_status_str(st_));        \
            return 1;                                                               \
        }                                                                           \
    } while (0)

#define HIPCHECK(call)                                                              \
    do {                                                                            \
        if ((call) != hipSuccess) {                                                 \
            fprintf(stderr, "%s failed\n", #call);                                  \
            return 1;                                                               \
        }                                                                           \
    } while (0)

static uint64_t key_of(uint64_t i, uint32_t w) {
    const uint64_t mask = w == 64 ? ~0ull : ((1ull << w) - 1ull);
    return (i * 0x9E3779B97F4A7C15ull + 12345u) & mask;
}

int main(void) {
    const uint32_t w = 40;
    const uint64_t n = 1u << 20;
    uint64_t* h_keys = malloc(2 * n * sizeof(uint64_t));
    uint8_t* h_out = malloc(2 * n);
    if (!h_keys || !h_out) return 1;
    for (uint64_t i = 0; i < 2 * n; ++i) h_keys[i] = key_of(i, w); /* [0, n) inserted, [n, 2n) never */

    void* d_keys = NULL;
    uint8_t* d_out = NULL;
    uint8_t* d_ops = NULL;
    HIPCHECK(hipMalloc(&d_keys, 2 * n * sizeof(uint64_t)));
    HIPCHECK(hipMalloc((void**)&d_out, 2 * n));
    HIPCHECK(hipMalloc((void**)&d_ops, 2 * n));
    HIPCHECK(hipMemcpy(d_keys, h_keys, 2 * n * sizeof(uint64_t), hipMemcpyHostToDevice));

    /* cuckoo: 2^21 slots (load 0.5), buckets of 32 x 32-bit slots */
    cpht_config_t c;
    cpht_config_default(CPHT_CUCKOO, &c);
    c.key_bits = w;
    c.log2_slots0 = 21;
    cpht_table_t t = NULL;
    CHECK(cpht_create(&c, &t));
    CHECK(cpht_bulk_build(t, d_keys, n, d_out, NULL));
    CHECK(cpht_find(t, d_keys, 2 * n, d_out + 0, NULL)); /* stream order: after the build */
    HIPCHECK(hipMemcpy(h_out, d_out, 2 * n, hipMemcpyDeviceToHost));
    uint64_t bad = 0;
    for (uint64_t i = 0; i < 2 * n; ++i) bad += h_out[i] != (i < n ? 1 : 0);
    uint64_t occ = 0, cap = 0;
    CHECK(cpht_count(t, &occ, &cap, NULL));
    if (bad || occ != n || cap != (1u << 21)) {
        fprintf(stderr, "cuckoo: %llu wrong answers, %llu of %llu slots occupied\n", (unsigned long long)bad,
                (unsigned long long)occ, (unsigned long long)cap);
        return 1;
    }
    CHECK(cpht_destroy(t));

    /* iceberg: 2^21 + 2^18 slots of 32 bits (a 40-bit key leaves 24
     * remainder bits at 2^16 primary buckets: too many for 16-bit slots);
     * one mixed batch: keys [0, n/2) twice as find-or-put, keys [n, n + n/2)
     * as finds */
    cpht_config_default(CPHT_ICEBERG, &c);
    c.key_bits = w;
    c.log2_slots0 = 21;
    c.log2_slots1 = 18;
    c.slot_bits0 = 32;
    c.slot_bits1 = 32;
    if (cpht_config_check(&c, NULL) != CPHT_OK) return 1;
    CHECK(cpht_create(&c, &t));
    const uint64_t m = n / 2;
    uint64_t* h_mix = malloc(3 * m * sizeof(uint64_t));
    uint8_t* h_ops = malloc(3 * m);
    if (!h_mix || !h_ops) return 1;
    for (uint64_t i = 0; i < m; ++i) {
        h_mix[i] = h_keys[i];
        h_mix[m + i] = h_keys[i];
        h_mix[2 * m + i] = h_keys[n + i];
        h_ops[i] = h_ops[m + i] = CPHT_OP_INSERT;
        h_ops[2 * m + i] = CPHT_OP_FIND;
    }
    HIPCHECK(hipMemcpy(d_keys, h_mix, 3 * m * sizeof(uint64_t), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(d_ops, h_ops, 3 * m, hipMemcpyHostToDevice));
    CHECK(cpht_mixed(t, d_keys, d_ops, 3 * m, d_out, NULL));
    HIPCHECK(hipMemcpy(h_out, d_out, 3 * m, hipMemcpyDeviceToHost));
    bad = 0;
    for (uint64_t i = 0; i < m; ++i) {
        const uint8_t a = h_out[i], b = h_out[m + i];
        /* one PUT and one FOUND per key, in either order */
        bad += !((a == CPHT_PUT && b == CPHT_FOUND) || (a == CPHT_FOUND && b == CPHT_PUT));
        bad += h_out[2 * m + i] != 0;
    }
    CHECK(cpht_count(t, &occ, &cap, NULL));
    if (bad || occ != m) {
        fprintf(stderr, "iceberg: %llu wrong answers, %llu occupied\n", (unsigned long long)bad,
                (unsigned long long)occ);
        return 1;
    }
    CHECK(cpht_destroy(t));
    HIPCHECK(hipFree(d_keys));
    HIPCHECK(hipFree(d_out));
    HIPCHECK(hipFree(d_ops));
    free(h_keys);
    free(h_out);
    free(h_mix);
    free(h_ops);
    printf("c-abi ok: cuckoo %llu keys, iceberg %llu keys\n", (unsigned long long)n, (unsigned long long)m);
    return 0;
}
