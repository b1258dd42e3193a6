/* Host twin of the counter-based ci8 test-signal generator (same definition
 * as synth_dev.hip and the numpy reference in synth/__init__.py).  Test-signal
 * generator only: it holds none of the correlator's arithmetic. */
#include <stdint.h>

static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int8_t level(uint32_t u, const uint32_t *thr, int n_thr, int max_abs)
{
    int k = -max_abs;
    for (int m = 0; m < n_thr; ++m) k += (u >= thr[m]);
    return (int8_t)k;
}

/* out: int8 [n_ch][n_rows][n_t][2]; channel c = ch0 + ci; row r is input
 * rows[r] (or r if rows == NULL); sample t0 + t. */
void synth_ci8_host(int8_t *out, int64_t ch0, int64_t n_ch, const int32_t *rows, int64_t n_rows,
                    int64_t t0, int64_t n_t, uint64_t seed, const uint32_t *thr, int n_thr, int max_abs)
{
    const uint64_t key = mix64(seed);
    int64_t cr;
#pragma omp parallel for schedule(static)
    for (cr = 0; cr < n_ch * n_rows; ++cr) {
        const uint64_t ch = (uint64_t)(ch0 + cr / n_rows);
        const int64_t r = cr % n_rows;
        const uint64_t inp = (uint64_t)(rows ? rows[r] : r);
        const uint64_t base = (ch << 44) | (inp << 24);
        int8_t *dst = out + cr * n_t * 2;
        for (int64_t t = 0; t < n_t; ++t) {
            const uint64_t h = mix64(key + (base | (uint64_t)(t0 + t)) * 0x9E3779B97F4A7C15ull);
            dst[2 * t] = level((uint32_t)h, thr, n_thr, max_abs);
            dst[2 * t + 1] = level((uint32_t)(h >> 32), thr, n_thr, max_abs);
        }
    }
}
