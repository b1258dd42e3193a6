/*
 * Memory-safety driver for the CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Built by the test suite together with oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer (gcc -fsanitize=address,undefined, no recovery).
 * It calls every exported oracle function on small shapes, including the
 * empty and degenerate ones, with every buffer allocated to exactly the size
 * the function's contract states, so that a read or write past a buffer, an
 * uninitialised-size allocation or signed overflow in index arithmetic stops
 * the run.  A few invariants of the results are checked on the way (autos
 * real and non-negative, product count, folds adding exactly).  Exit status 0
 * means every call ran clean.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_xengine_ci8(const int8_t *x, int64_t n_ch, int64_t n_in, int64_t T, int64_t *V);
void oracle_xengine_cf64(const double *x, int64_t n_ch, int64_t n_in, int64_t T, double *V);
void oracle_xengine_pairs_ci8(const int8_t *xc, int64_t n_in, int64_t T, const int32_t *ii,
                              const int32_t *jj, int64_t n, int64_t *out);
void oracle_dft_real(const int8_t *v, int64_t N, int64_t n_in, int64_t n_blocks, int64_t n_keep, double *X);
void oracle_pfb_coeffs(int64_t P, int64_t N, double *h);
void oracle_pfb_real(const int8_t *v, const double *h, int64_t N, int64_t P, int64_t n_in, int64_t n_blocks,
                     int64_t n_keep, double *X);
void oracle_dft_complex(const int8_t *v, int64_t N, int64_t n_in, int64_t n_blocks, double *X);
void oracle_unpack_w16(const uint16_t *w, int64_t n, int8_t *out);
void oracle_unpack_b8(const uint8_t *b, int64_t n, int8_t *out);
int64_t oracle_aggregate_w16(const uint16_t *rec, int64_t n_streams, int64_t w_per, int64_t n_rec,
                             uint32_t first_counter, uint16_t *out);
void oracle_requant(const double *y, int64_t n, double s, int32_t max_abs, int8_t *q);
void oracle_f16_encode(const double *x, int64_t n, uint16_t *out);
void oracle_f16_decode(const uint16_t *h, int64_t n, double *out);
void oracle_e4m3_encode(const double *x, int64_t n, uint8_t *out);
void oracle_e4m3_decode(const uint8_t *b, int64_t n, double *out);
double oracle_e4m3_scale(const double *x, int64_t n);
void oracle_fold_i64(double *L, const int64_t *V, int64_t n);
void oracle_fold_f64(double *L, const double *V, int64_t n);
int oracle_num_threads(void);
void oracle_set_num_threads(int n);

static uint64_t rng = 0x9E3779B97F4A7C15ull;
static uint32_t next32(void)
{
    rng = rng * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(rng >> 33);
}
static int8_t small_int(int m) { return (int8_t)((int)(next32() % (uint32_t)(2 * m + 1)) - m); }

/* malloc of exactly n elements (at least one byte, so that n = 0 still gives
 * a distinct pointer that must not be touched). */
static void *alloc(size_t n, size_t size) { return malloc(n * size > 0 ? n * size : 1); }

static int fails = 0;
#define CHECK(c, ...)                                  \
    do {                                               \
        if (!(c)) {                                    \
            fprintf(stderr, "FAIL: " __VA_ARGS__);     \
            fprintf(stderr, "\n");                     \
            ++fails;                                   \
        }                                              \
    } while (0)

static int64_t tri(int64_t n) { return n * (n + 1) / 2; }

static void xengine_cases(void)
{
    static const int64_t shapes[][3] = {{1, 1, 1}, {2, 3, 5}, {1, 7, 0}, {3, 1, 17}, {2, 16, 9}, {0, 4, 4}};
    for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s) {
        const int64_t n_ch = shapes[s][0], n_in = shapes[s][1], T = shapes[s][2];
        const int64_t nx = n_ch * n_in * T * 2, nv = n_ch * tri(n_in) * 2;
        int8_t *x = alloc((size_t)nx, 1);
        double *xf = alloc((size_t)nx, sizeof(double));
        int64_t *V = alloc((size_t)nv, sizeof(int64_t));
        double *Vf = alloc((size_t)nv, sizeof(double));
        for (int64_t k = 0; k < nx; ++k) {
            x[k] = small_int(127);
            xf[k] = (double)x[k];
        }
        oracle_xengine_ci8(x, n_ch, n_in, T, V);
        oracle_xengine_cf64(xf, n_ch, n_in, T, Vf);
        for (int64_t c = 0; c < n_ch; ++c)
            for (int64_t i = 0; i < n_in; ++i) {
                const int64_t b = (c * tri(n_in) + tri(i) + i) * 2;   /* auto (i, i) */
                CHECK(V[b] >= 0 && V[b + 1] == 0, "xengine_ci8 auto (%lld,%lld)", (long long)c, (long long)i);
            }
        for (int64_t k = 0; k < nv; ++k) CHECK((double)V[k] == Vf[k], "cf64 != ci8 at %lld", (long long)k);
        if (n_ch > 0 && n_in > 0) {
            const int64_t np = tri(n_in);
            int32_t *ii = alloc((size_t)np, sizeof(int32_t));
            int32_t *jj = alloc((size_t)np, sizeof(int32_t));
            int64_t *out = alloc((size_t)np * 2, sizeof(int64_t));
            int64_t k = 0;
            for (int32_t i = 0; i < n_in; ++i)
                for (int32_t j = 0; j <= i; ++j, ++k) {
                    ii[k] = i;
                    jj[k] = j;
                }
            oracle_xengine_pairs_ci8(x, n_in, T, ii, jj, np, out);
            for (k = 0; k < 2 * np; ++k) CHECK(out[k] == V[k], "pairs != full at %lld", (long long)k);
            free(ii);
            free(jj);
            free(out);
        }
        free(x);
        free(xf);
        free(V);
        free(Vf);
    }
}

static void fstage_cases(void)
{
    static const int64_t shapes[][3] = {{8, 1, 1}, {16, 3, 2}, {256, 2, 1}, {4, 5, 0}, {32, 1, 3}};
    for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s) {
        const int64_t N = shapes[s][0], n_in = shapes[s][1], nb = shapes[s][2];
        const int64_t n_keep = N / 2;
        int8_t *v = alloc((size_t)(nb * N * n_in), 1);
        for (int64_t k = 0; k < nb * N * n_in; ++k) v[k] = small_int(127);
        double *X = alloc((size_t)(n_keep * n_in * nb * 2), sizeof(double));
        oracle_dft_real(v, N, n_in, nb, n_keep, X);
        /* complex DFT: [nb*N][n_in][2] samples -> [N][n_in][nb][2] */
        int8_t *vc = alloc((size_t)(nb * N * n_in * 2), 1);
        for (int64_t k = 0; k < nb * N * n_in * 2; ++k) vc[k] = small_int(15);
        double *Xc = alloc((size_t)(N * n_in * nb * 2), sizeof(double));
        oracle_dft_complex(vc, N, n_in, nb, Xc);
        /* filterbank, P taps: (nb + P - 1) blocks in */
        for (int64_t P = 1; P <= 4; P += 3) {
            double *h = alloc((size_t)(P * N), sizeof(double));
            oracle_pfb_coeffs(P, N, h);
            int8_t *vp = alloc((size_t)((nb + P - 1) * N * n_in), 1);
            for (int64_t k = 0; k < (nb + P - 1) * N * n_in; ++k) vp[k] = small_int(127);
            double *Xp = alloc((size_t)(n_keep * n_in * nb * 2), sizeof(double));
            oracle_pfb_real(vp, h, N, P, n_in, nb, n_keep, Xp);
            free(h);
            free(vp);
            free(Xp);
        }
        /* requantiser over the spectra */
        int8_t *q = alloc((size_t)(n_keep * n_in * nb * 2), 1);
        oracle_requant(X, n_keep * n_in * nb * 2, 0.01, 7, q);
        for (int64_t k = 0; k < n_keep * n_in * nb * 2; ++k) CHECK(q[k] >= -7 && q[k] <= 7, "requant range");
        free(v);
        free(X);
        free(vc);
        free(Xc);
        free(q);
    }
}

static void codec_cases(void)
{
    for (int64_t n = 0; n <= 33; n += 11) {
        uint16_t *w = alloc((size_t)n, sizeof(uint16_t));
        uint8_t *b = alloc((size_t)n, 1);
        int8_t *o = alloc((size_t)n * 2, 1);
        for (int64_t k = 0; k < n; ++k) {
            w[k] = (uint16_t)next32();
            b[k] = (uint8_t)next32();
        }
        oracle_unpack_w16(w, n, o);
        for (int64_t k = 0; k < 2 * n; ++k) CHECK(o[k] >= -16 && o[k] <= 15, "w16 range");
        oracle_unpack_b8(b, n, o);
        for (int64_t k = 0; k < 2 * n; ++k) CHECK(o[k] >= -8 && o[k] <= 7, "b8 range");
        double *x = alloc((size_t)n, sizeof(double));
        double *y = alloc((size_t)n, sizeof(double));
        uint16_t *h = alloc((size_t)n, sizeof(uint16_t));
        uint8_t *e = alloc((size_t)n, 1);
        for (int64_t k = 0; k < n; ++k) x[k] = ((double)next32() / 4294967296.0 - 0.5) * 1000.0;
        oracle_f16_encode(x, n, h);
        oracle_f16_decode(h, n, y);
        const double sc = oracle_e4m3_scale(x, n);
        CHECK(sc > 0.0, "e4m3 scale");
        oracle_e4m3_encode(x, n, e);
        oracle_e4m3_decode(e, n, y);
        free(w);
        free(b);
        free(o);
        free(x);
        free(y);
        free(h);
        free(e);
    }
    /* aggregation: n_streams x n_rec records of 1 + w_per words */
    static const int64_t shapes[][3] = {{1, 1, 1}, {4, 3, 5}, {2, 0, 3}, {3, 2, 0}};
    for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s) {
        const int64_t ns = shapes[s][0], w_per = shapes[s][1], nr = shapes[s][2];
        uint16_t *rec = alloc((size_t)(ns * nr * (1 + w_per)), sizeof(uint16_t));
        uint16_t *out = alloc((size_t)(nr * ns * w_per), sizeof(uint16_t));
        for (int64_t st = 0; st < ns; ++st)
            for (int64_t r = 0; r < nr; ++r) {
                uint16_t *p = rec + (st * nr + r) * (1 + w_per);
                p[0] = (uint16_t)(65534 + r);   /* counter wraps at 2^16 */
                for (int64_t k = 0; k < w_per; ++k) p[1 + k] = (uint16_t)next32();
            }
        CHECK(oracle_aggregate_w16(rec, ns, w_per, nr, 65534u, out) == 0, "aggregate counters");
        free(rec);
        free(out);
    }
}

static void fold_cases(void)
{
    const int64_t n = 7;
    double *L = alloc((size_t)n, sizeof(double));
    int64_t *Vi = alloc((size_t)n, sizeof(int64_t));
    double *Vf = alloc((size_t)n, sizeof(double));
    for (int64_t k = 0; k < n; ++k) {
        L[k] = 0.0;
        Vi[k] = (int64_t)k * 1000003 - 5;
        Vf[k] = 0.25 * (double)k;
    }
    oracle_fold_i64(L, Vi, n);
    oracle_fold_f64(L, Vf, n);
    for (int64_t k = 0; k < n; ++k) CHECK(L[k] == (double)Vi[k] + 0.25 * (double)k, "fold %lld", (long long)k);
    oracle_fold_i64(L, Vi, 0);
    oracle_fold_f64(L, Vf, 0);
    free(L);
    free(Vi);
    free(Vf);
}

int main(void)
{
    oracle_set_num_threads(oracle_num_threads());
    xengine_cases();
    fstage_cases();
    codec_cases();
    fold_cases();
    if (fails) {
        fprintf(stderr, "%d check(s) failed\n", fails);
        return 1;
    }
    printf("oracle sanitizer run clean\n");
    return 0;
}
