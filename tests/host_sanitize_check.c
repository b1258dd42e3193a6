/*
 * Host-side memory-safety driver for libcorr -- TEST INFRASTRUCTURE ONLY.
 *
 * Linked with the library's host sources built under AddressSanitizer and
 * UndefinedBehaviorSanitizer (hipcc with -fsanitize after -Xarch_host: the
 * device code is not instrumented).  Without a GPU it walks the host paths
 * that need none: status strings, configuration validation and workspace
 * sizing over a grid of valid and invalid configurations, plan creation and
 * destruction on a workspace the plan never touches from the host, dump
 * sizes, the argument checks of every entry point, the error state a failed
 * launch leaves, and the scheduler's argument checks.  With a GPU (argument
 * "gpu") it also correlates a small integration through a plan and through
 * the serving scheduler and checks the sums against a direct host sum.
 * Exit status 0 means every call ran clean and every check held.
 */
#define _POSIX_C_SOURCE 200112L
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <hip/hip_runtime_api.h>

#include "corr.h"

static int fails = 0;
#define CHECK(c, ...)                              \
    do {                                           \
        if (!(c)) {                                \
            fprintf(stderr, "FAIL: " __VA_ARGS__); \
            fprintf(stderr, "\n");                 \
            ++fails;                               \
        }                                          \
    } while (0)

static corr_config base_config(void)
{
    corr_config c;
    memset(&c, 0, sizeof c);
    c.n_inputs = 64;
    c.n_channels = 8;
    c.sample_type = CORR_CI8;
    c.engine = CORR_X_I8;
    c.max_abs = 7;
    return c;
}

static void status_strings(void)
{
    for (int s = -20; s <= 5; ++s) {
        const char *t = corr_status_str((corr_status)s);
        CHECK(t != NULL && strlen(t) > 0, "status string %d", s);
    }
}

static void config_grid(void)
{
    static const int32_t n_inputs[] = {-1, 0, 1, 2, 63, 64, 65, 1024, 65535, 65536, 65537};
    static const int32_t n_channels[] = {-1, 0, 1, 128, 768, 65535, 65536};
    static const int32_t fft[] = {0, 128, 256, 100};
    static const int32_t engines[] = {-1, CORR_X_FP32, CORR_X_I8, CORR_X_F16, CORR_X_F8, CORR_X_FP32M, 5};
    static const int32_t samples[] = {-1, CORR_CF32, CORR_CI8, CORR_CI4, 3};
    static const int32_t max_abs[] = {-1, 0, 7, 127, 128};
    static const int32_t taps[] = {0, 1, 3, 4};
    static const int64_t ring[] = {-1, 0, 1, 1000};
    int64_t n_ok = 0, n_all = 0;
    for (size_t a = 0; a < sizeof n_inputs / sizeof *n_inputs; ++a)
        for (size_t b = 0; b < sizeof n_channels / sizeof *n_channels; ++b)
            for (size_t f = 0; f < sizeof fft / sizeof *fft; ++f)
                for (size_t e = 0; e < sizeof engines / sizeof *engines; ++e)
                    for (size_t s = 0; s < sizeof samples / sizeof *samples; ++s)
                        for (size_t m = 0; m < sizeof max_abs / sizeof *max_abs; ++m)
                            for (size_t t = 0; t < sizeof taps / sizeof *taps; ++t)
                                for (size_t r = 0; r < sizeof ring / sizeof *ring; ++r)
                                    for (int lr = 0; lr < 2; ++lr) {
                                        corr_config c;
                                        memset(&c, 0, sizeof c);
                                        c.n_inputs = n_inputs[a];
                                        c.n_channels = n_channels[b];
                                        c.fft_size = fft[f];
                                        c.engine = engines[e];
                                        c.sample_type = samples[s];
                                        c.max_abs = max_abs[m];
                                        c.requant_scale = 0.1f;
                                        c.fp64_longrun = lr;
                                        c.ring_samples = ring[r];
                                        c.volt_format = fft[f] == 128 ? CORR_VOLT_CW16 : CORR_VOLT_R8;
                                        c.pfb_taps = fft[f] == 0 ? 0 : taps[t];
                                        size_t bytes = 0;
                                        const corr_status st = corr_workspace_bytes(&c, &bytes);
                                        ++n_all;
                                        if (st == CORR_OK) {
                                            ++n_ok;
                                            CHECK(bytes > 0 && bytes % 256 == 0, "workspace size %zu", bytes);
                                        }
                                    }
    CHECK(n_ok > 0 && n_ok < n_all, "config grid: %lld valid of %lld", (long long)n_ok, (long long)n_all);
    size_t bytes = 0;
    CHECK(corr_workspace_bytes(NULL, &bytes) != CORR_OK, "NULL config");
    corr_config c = base_config();
    CHECK(corr_workspace_bytes(&c, NULL) != CORR_OK, "NULL size");
}

/* Plans on a host allocation standing in for device memory: creation with
 * fft_size 0 and no long-run sum queues no device work, and the host never
 * dereferences the workspace. */
static void plan_paths(int have_gpu)
{
    corr_config c = base_config();
    size_t bytes = 0;
    CHECK(corr_workspace_bytes(&c, &bytes) == CORR_OK, "base config");
    void *ws = NULL;
    if (posix_memalign(&ws, 256, bytes) != 0) {
        ++fails;
        return;
    }
    corr_plan *p = NULL;
    CHECK(corr_create(&c, ws, bytes, NULL, NULL) != CORR_OK, "NULL out");
    CHECK(corr_create(&c, NULL, bytes, NULL, &p) == CORR_E_WORKSPACE, "NULL workspace");
    CHECK(corr_create(&c, (char *)ws + 16, bytes - 16, NULL, &p) == CORR_E_WORKSPACE, "misaligned workspace");
    CHECK(corr_create(&c, ws, bytes - 256, NULL, &p) == CORR_E_WORKSPACE, "short workspace");
    if (!have_gpu) {
        CHECK(corr_create(&c, ws, bytes, NULL, &p) == CORR_OK && p != NULL, "create");
        if (p) {
            for (int32_t what = -1; what <= 4; ++what) {
                size_t db = 0;
                (void)corr_dump_bytes(p, what, &db);
            }
            CHECK(corr_dump_bytes(p, 0, NULL) != CORR_OK, "dump_bytes NULL");
            CHECK(corr_correlate(p, NULL, 10, 10) != CORR_OK, "correlate NULL samples");
            CHECK(corr_correlate(p, ws, -1, 10) != CORR_OK, "correlate negative count");
            CHECK(corr_correlate(p, ws, 10, 5) != CORR_OK, "correlate stride below count");
            CHECK(corr_channelise(p, ws, 1, 0, NULL) != CORR_OK, "channelise without F-stage");
            int64_t n = 0;
            int32_t exact = 0;
            (void)corr_dump(p, 16, ws, 1, &n, &exact);   /* an unknown flag bit */
            int64_t n_long = -1;
            uint64_t seq = 1;
            int32_t valid = -1;
            CHECK(corr_state(p, &n_long, &seq, &valid) == CORR_OK, "state");
            CHECK(corr_state(p, NULL, NULL, NULL) == CORR_OK, "state, NULL outs");
            CHECK(corr_restore(p, ws, 1, 10, 5, 1) != CORR_OK, "restore without a long-run sum");
            CHECK(corr_destroy(p) == CORR_OK, "destroy");
        }
    }
    CHECK(corr_destroy(NULL) == CORR_OK, "destroy NULL (documented as safe)");
    free(ws);

    corr_sched *s = NULL;
    CHECK(corr_sched_create(NULL, 1 << 20, 4, &s) != CORR_OK, "sched NULL arena");
    CHECK(corr_sched_create((void *)(uintptr_t)256, 1 << 20, 0, &s) != CORR_OK, "sched 0 streams");
    CHECK(corr_sched_create((void *)(uintptr_t)256, 1 << 20, 17, &s) != CORR_OK, "sched 17 streams");
    CHECK(corr_sched_create((void *)(uintptr_t)256, 1024, 4, &s) != CORR_OK, "sched arena below the queue");
    CHECK(corr_sched_now() >= 0.0, "clock");
}

/* Small integration on the GPU through a plan and through the scheduler,
 * against a direct host sum. */
static void gpu_paths(void)
{
    const int n_in = 40, n_ch = 3, T = 300;
    const int64_t P = (int64_t)n_in * (n_in + 1) / 2;
    int8_t *x = (int8_t *)malloc((size_t)n_ch * n_in * T * 2);
    uint32_t r = 12345u;
    for (int64_t k = 0; k < (int64_t)n_ch * n_in * T * 2; ++k) {
        r = r * 1664525u + 1013904223u;
        x[k] = (int8_t)((int)((r >> 16) % 15u) - 7);
    }
    int32_t *want = (int32_t *)calloc((size_t)(n_ch * P * 2), sizeof(int32_t));
    for (int c = 0; c < n_ch; ++c)
        for (int i = 0; i < n_in; ++i)
            for (int j = 0; j <= i; ++j) {
                int32_t re = 0, im = 0;
                for (int t = 0; t < T; ++t) {
                    const int8_t *a = x + (((int64_t)c * n_in + i) * T + t) * 2;
                    const int8_t *b = x + (((int64_t)c * n_in + j) * T + t) * 2;
                    re += a[0] * b[0] + a[1] * b[1];
                    im += a[1] * b[0] - a[0] * b[1];
                }
                const int64_t k = (c * P + (int64_t)i * (i + 1) / 2 + j) * 2;
                want[k] = re;
                want[k + 1] = im;
            }
    void *dx = NULL, *ws = NULL, *arena = NULL, *dres = NULL;
    const size_t xb = (size_t)n_ch * n_in * T * 2, rb = (size_t)n_ch * P * 2 * sizeof(int32_t);
    corr_config c = base_config();
    c.n_inputs = n_in;
    c.n_channels = n_ch;
    size_t wsb = 0;
    CHECK(corr_workspace_bytes(&c, &wsb) == CORR_OK, "gpu config");
    if (hipMalloc(&dx, xb) != hipSuccess || hipMalloc(&ws, wsb) != hipSuccess ||
        hipMalloc(&arena, (size_t)64 << 20) != hipSuccess || hipMalloc(&dres, rb) != hipSuccess) {
        ++fails;
        fprintf(stderr, "FAIL: hipMalloc\n");
        return;
    }
    CHECK(hipMemcpy(dx, x, xb, hipMemcpyHostToDevice) == hipSuccess, "copy samples");
    int32_t *got = (int32_t *)malloc(rb);
    corr_plan *p = NULL;
    CHECK(corr_create(&c, ws, wsb, NULL, &p) == CORR_OK, "create on GPU");
    if (p) {
        CHECK(corr_correlate(p, dx, T, T) == CORR_OK, "correlate");
        int64_t n = 0;
        int32_t exact = 0;
        CHECK(corr_dump(p, CORR_DUMP_INTEG, got, 0, &n, &exact) == CORR_OK, "dump");
        CHECK(n == T && exact == 1, "dump count");
        CHECK(memcmp(got, want, rb) == 0, "plan sums");
        CHECK(corr_destroy(p) == CORR_OK, "destroy on GPU");
    }
    corr_sched *s = NULL;
    CHECK(corr_sched_create(arena, (size_t)64 << 20, 2, &s) == CORR_OK, "sched create");
    if (s) {
        corr_job_desc j;
        memset(&j, 0, sizeof j);
        j.n_inputs = n_in;
        j.n_channels = n_ch;
        j.n_samples = T;
        j.max_abs = 7;
        j.d_samples = dx;
        j.row_stride = T;
        j.dst = dres;
        j.dst_is_device = 1;
        uint64_t ids[4];
        for (int k = 0; k < 4; ++k) CHECK(corr_sched_submit(s, &j, corr_sched_now(), &ids[k]) == CORR_OK, "submit");
        for (int k = 0; k < 4; ++k) {
            corr_status st;
            int64_t n = 0;
            while ((st = corr_sched_poll(s, ids[k], &n, NULL, NULL, NULL)) == CORR_E_BUSY) {
            }
            CHECK(st == CORR_OK && n == T, "job %d", k);
        }
        memset(got, 0, rb);
        CHECK(hipMemcpy(got, dres, rb, hipMemcpyDeviceToHost) == hipSuccess, "copy result");
        CHECK(memcmp(got, want, rb) == 0, "scheduler sums");
        int64_t stats[8];
        CHECK(corr_sched_stats(s, stats) == CORR_OK && stats[2] == 4, "stats");
        CHECK(corr_sched_destroy(s) == CORR_OK, "sched destroy");
    }
    (void)hipFree(dx);
    (void)hipFree(ws);
    (void)hipFree(arena);
    (void)hipFree(dres);
    free(x);
    free(want);
    free(got);
}

int main(int argc, char **argv)
{
    const int gpu = argc > 1 && strcmp(argv[1], "gpu") == 0;
    status_strings();
    config_grid();
    plan_paths(gpu);
    if (gpu) gpu_paths();
    if (fails) {
        fprintf(stderr, "%d check(s) failed\n", fails);
        fflush(stderr);
        if (gpu) _exit(1);
        return 1;
    }
    printf("host library sanitizer run clean%s\n", gpu ? " (with GPU paths)" : "");
    fflush(stdout);
    /* With the GPU runtime loaded, end without its exit-time teardown, which
     * the sanitizer runtime's device-allocation hooks do not survive (the
     * GPU test runs without leak detection). */
    if (gpu) _exit(0);
    return 0;
}
