/* The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer,
   with no GPU: every entry point of hj.h that works on the host (parameter
   resolution, workspace and table sizing, the cost model, batch sizing,
   status strings) over seeded random arguments, and the argument checks of
   every entry point that reaches the device.  Without a device, calls that
   get past their checks must fail with HJ_ERR_DEVICE and release what they
   created (the leak checker sees the rest).  Also compiles hj.h as C.
   Built and run by tests/test_host_sanitized.py. */
#define _POSIX_C_SOURCE 200112L
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hj.h"

static int failures = 0;
#define CHECK(c)                                                                        \
    do {                                                                                \
        if (!(c)) {                                                                     \
            fprintf(stderr, "%s:%d: check failed: %s (%s)\n", __FILE__, __LINE__, #c,   \
                    hj_last_error());                                                   \
            ++failures;                                                                 \
        }                                                                               \
    } while (0)

/* splitmix64: a seeded stream for the random arguments */
static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t rnd(void) {
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static uint64_t below(uint64_t n) { return n ? rnd() % n : 0; }

static uint64_t random_size(void) {
    switch (below(6)) {
        case 0: return 0;
        case 1: return 1 + below(100);
        case 2: return 1 + below(10000);
        case 3: return 1 + below(1u << 24);
        case 4: return (uint64_t)1 << below(32);
        default: return below((uint64_t)1 << 33);  /* beyond the 2^31 limit at times */
    }
}

static hj_params random_params(void) {
    hj_params p;
    hj_default_params(&p);
    p.algo = (uint32_t)below(4);                 /* 3: invalid */
    p.passes = (uint32_t)below(4);               /* 3: invalid */
    p.bits[0] = (uint32_t)below(16);
    p.bits[1] = (uint32_t)below(16);
    p.hash = (uint32_t)below(3);                 /* 2: invalid */
    switch (below(4)) {
        case 0: p.tile = 0; break;
        case 1: p.tile = 1024u << below(4); break;
        case 2: p.tile = 512u << below(6); break;
        default: p.tile = (uint32_t)below(20000); break;
    }
    switch (below(3)) {
        case 0: p.lds_cap = 0; break;
        case 1: p.lds_cap = 64u * (uint32_t)below(140); break;
        default: p.lds_cap = (uint32_t)below(10000); break;
    }
    p.flags = (uint32_t)below(3);                /* 2: invalid */
    return p;
}

static int same_params(const hj_params* a, const hj_params* b) { return memcmp(a, b, sizeof *a) == 0; }

static void fuzz_resolution(void) {
    int valid = 0;
    for (int it = 0; it < 40000; ++it) {
        const hj_params p = random_params();
        const uint64_t n_r = random_size(), n_s = random_size();
        hj_params q;
        const hj_status st = hj_resolve_params(&p, n_r, n_s, &q);
        const size_t ws = hj_workspace_bytes(&p, n_r, n_s);
        double t = -1.0;
        const hj_status mst = hj_model_seconds(&p, n_r, n_s, n_s, &t);
        if (st == HJ_OK) {
            ++valid;
            /* resolution is idempotent and sizes the same workspace */
            hj_params q2;
            CHECK(hj_resolve_params(&q, n_r, n_s, &q2) == HJ_OK);
            CHECK(same_params(&q, &q2));
            CHECK(ws > 0);
            CHECK(hj_workspace_bytes(&q, n_r, n_s) == ws);
            CHECK(q.algo == HJ_SHJ || q.algo == HJ_PHJ);
            CHECK(mst == HJ_OK && isfinite(t) && t > 0.0);
            const size_t tb = hj_table_bytes(&p, n_r);
            (void)tb;
        } else {
            CHECK(st == HJ_ERR_INVALID || st == HJ_ERR_UNSUPPORTED);
            CHECK(ws == 0);
            CHECK(strlen(hj_last_error()) > 0);
            CHECK(mst != HJ_OK);
        }
    }
    CHECK(valid > 1000);
}

static void argument_checks(int have_device) {
    hj_params p;
    hj_default_params(&p);
    static int32_t key[64], rid[64];
    static int32_t o_r[64], o_s[64];
    uint64_t cnt = 0;
    hj_rel R = {key, rid, 64}, S = {key, rid, 64};
    hj_out out = {o_r, o_s, 64};
    /* aligned fake workspace (host memory: only used when no device exists) */
    void* ws = NULL;
    CHECK(posix_memalign(&ws, 256, 1u << 20) == 0);
    CHECK(hj_join(NULL, &R, &S, &out, ws, 1u << 20, &cnt, NULL) == HJ_ERR_INVALID);
    CHECK(hj_join(&p, NULL, &S, &out, ws, 1u << 20, &cnt, NULL) == HJ_ERR_INVALID);
    CHECK(hj_join(&p, &R, &S, &out, ws, 1u << 20, NULL, NULL) == HJ_ERR_INVALID);
    CHECK(hj_join(&p, &R, &S, &out, (char*)ws + 8, 1u << 20, &cnt, NULL) == HJ_ERR_INVALID);
    CHECK(hj_join(&p, &R, &S, &out, ws, 16, &cnt, NULL) == HJ_ERR_WORKSPACE);
    hj_rel bad = {NULL, rid, 64};
    CHECK(hj_join(&p, &bad, &S, &out, ws, 1u << 20, &cnt, NULL) == HJ_ERR_INVALID);
    hj_out bad_out = {NULL, o_s, 64};
    CHECK(hj_join(&p, &R, &S, &bad_out, ws, 1u << 20, &cnt, NULL) == HJ_ERR_INVALID);
    CHECK(hj_build(&p, &R, ws, 16, NULL, NULL) == HJ_ERR_INVALID);
    hj_table tab;
    memset(&tab, 0, sizeof tab);
    CHECK(hj_probe(&tab, &S, &out, ws, 1u << 20, &cnt, NULL) != HJ_OK);
    CHECK(hj_probe_workspace_bytes(NULL, 10) == 0);
    uint64_t h = 0;
    CHECK(hj_join_external(&p, &R, &S, &out, ws, 1u << 10, &h, NULL) == HJ_ERR_WORKSPACE);  /* < 64 MiB */
    CHECK(hj_join_noalloc(&p, &R, &S, &out, NULL, NULL) != HJ_OK || have_device);
    hj_server* sv = NULL;
    hj_server_config cfg = {1u << 30, 0, 8, 0};
    CHECK(hj_server_create(&cfg, ws, 1u << 20, &sv) == HJ_ERR_INVALID && sv == NULL);
    cfg.slots = 2;
    cfg.flags = 1;
    CHECK(hj_server_create(&cfg, ws, 1u << 20, &sv) == HJ_ERR_INVALID && sv == NULL);
    CHECK(hj_batch_plan_create(0, NULL, NULL, 0, NULL) == HJ_ERR_INVALID);
    if (!have_device) {
        /* past the checks with no device: a device error, and nothing left behind */
        CHECK(hj_join(&p, &R, &S, &out, ws, 1u << 20, &cnt, NULL) == HJ_ERR_DEVICE ||
              hj_workspace_bytes(&p, 64, 64) > (1u << 20));
        cfg.flags = 0;
        CHECK(hj_server_create(&cfg, ws, 1u << 20, &sv) == HJ_ERR_DEVICE && sv == NULL);
        hj_job job = {R, S, out, &cnt};
        hj_batch_plan* plan = NULL;
        const hj_status bst = hj_batch_plan_create(1, &job, NULL, 0, &plan);
        CHECK((bst == HJ_OK) == (plan != NULL));
        if (plan) hj_batch_plan_destroy(plan);
    }
    free(ws);
}

static void batch_sizing(void) {
    enum { N = 300 };
    static hj_job jobs[N];
    static hj_params ps[N];
    static int32_t dummy[4];
    static uint64_t cnt;
    for (int trial = 0; trial < 50; ++trial) {
        const uint32_t n = 1 + (uint32_t)below(N);
        for (uint32_t i = 0; i < n; ++i) {
            const uint64_t nr = below(3) ? below(1u << 20) : below(9000);
            const uint64_t ns = below(1u << 20);
            hj_job j = {{dummy, dummy, nr}, {dummy, dummy, ns}, {dummy, dummy, ns}, &cnt};
            jobs[i] = j;
            hj_default_params(&ps[i]);
            ps[i].algo = HJ_AUTO;
            ps[i].flags = HJ_FLAG_ONE_PASS;
        }
        const size_t a = hj_batch_bytes(n, jobs, NULL);
        const size_t b = hj_batch_bytes(n, jobs, ps);
        CHECK(a > 0 && b > 0);
    }
}

static void status_strings(void) {
    for (int s = 0; s <= 6; ++s) CHECK(hj_status_str((hj_status)s) != NULL);
}

int hip_device_count(void);  /* api_host_devices.cpp */

int main(void) {
    const int have_device = hip_device_count() > 0;
    fuzz_resolution();
    argument_checks(have_device);
    batch_sizing();
    status_strings();
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("host API: all checks passed%s\n", have_device ? " (device-reaching calls skipped)" : "");
    return 0;
}
