/*
 * CPU oracle for the FX correlator -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct C99.  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load this library; the GPU
 * library never does, and the two share no code.
 *
 * Every function follows a passage of Wayth, Greenhill & Briggs (2009),
 * "A GPU based real-time software correlation system for the Murchison
 * Widefield Array prototype" (arXiv:0906.1887):
 *
 *   oracle_xengine_ci8 / _cf64 / _pairs_ci8
 *       Sec. 2 (an FX correlator multiplies each spectrum by the complex
 *       conjugate of every other, channel by channel, and accumulates) and
 *       Sec. 2's product count N_I(N_I+1)/2 including autos; Fig. 2 (the
 *       per-channel outer product x x^H, autos on the diagonal, redundant
 *       halves).  V_ij[c] = sum_t x_i[c,t] conj(x_j[c,t]), lower triangle
 *       j <= i, packed row-major: b(i,j) = i(i+1)/2 + j.
 *       Integer samples: int64 accumulation (exact).  Float samples: FP64,
 *       built with -ffp-contract=off.
 *   oracle_dft_real
 *       Sec. 2 / Sec. 4 (real input: 2 N_C samples give N_C+1 channels incl.
 *       DC; the redundant half of the transform is ignored).  Direct DFT in
 *       FP64: X_k = sum_n x_n exp(-2 pi i ((k n) mod N) / N), k < N/2
 *       (DC kept, Nyquist dropped), unnormalised, no window.
 *   oracle_requant
 *       Requantiser of the F-stage output (not in the paper, which correlates
 *       floats): q = clip(round_half_even(s*y), -max_abs, max_abs).
 *   oracle_pfb_coeffs / oracle_pfb_real
 *       Sec. 6.1 (further work): a polyphase filterbank in place of the plain
 *       FFT, to cut the leakage of signals between channel centres.  The
 *       paper gives no design; read here as the critically sampled
 *       weighted-overlap-add form with P taps of N points: y_b[n] =
 *       sum_{p<P} h[pN + n] x[(b + p)N + n], then the same real DFT as
 *       oracle_dft_real.  Prototype filter h[m] = w[m] sinc((m - (PN-1)/2)/N),
 *       Hamming window w[m] = 0.54 - 0.46 cos(2 pi m / (PN - 1)), m < PN.
 *   oracle_unpack_w16 / oracle_unpack_b8
 *       Sec. 3: a recorded sample has 5-bit real and 5-bit imaginary parts in
 *       two's complement, stored in a 16-bit word; Sec. 5's "1-byte" mode
 *       keeps one bit less of each part in a single byte.  The bit positions
 *       are not stated; read here as re = bits 9..5, im = bits 4..0 (upper
 *       six bits ignored) and re = bits 7..4, im = bits 3..0.
 *   oracle_aggregate_w16
 *       Sec. 3: each capture stream is a run of records of one marker/counter
 *       word followed by one word per receiver input; the aggregator drops
 *       the marker words and interleaves the streams so that all inputs of
 *       one time instant are adjacent.  The marker is read here as a 16-bit
 *       record counter; records whose counter differs from the expected one
 *       in any stream are counted.
 *   oracle_dft_complex
 *       Sec. 2 / Sec. 4: complex samples, N samples give N channels.  Direct
 *       DFT in FP64, X_k = sum_n x_n exp(-2 pi i ((k n) mod N) / N) for every
 *       k < N, natural order (DC first), unnormalised, no window.
 *   oracle_f16_* / oracle_e4m3_*
 *       IEEE binary16 and OCP FP8 E4M3FN codecs with round-half-even (E4M3:
 *       bias 7, no infinities, saturating at 448), written from the formats'
 *       definitions.
 *   oracle_fold_i64 / oracle_fold_f64
 *       Fig. 1: accumulators are read after a time interval (and divided by
 *       the number of updates); the long-run sum L += V is kept in FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static int64_t tri(int64_t n) { return n * (n + 1) / 2; }

/* ---------------------------------------------------------------- X-engine */

/* x: int8 [n_ch][n_in][T][2] (re, im); V: int64 [n_ch][n_in(n_in+1)/2][2]. */
void oracle_xengine_ci8(const int8_t *x, int64_t n_ch, int64_t n_in, int64_t T, int64_t *V)
{
    const int64_t P = tri(n_in);
    int64_t c;
#pragma omp parallel for schedule(dynamic, 1)
    for (c = 0; c < n_ch; ++c) {
        const int8_t *xc = x + c * n_in * T * 2;
        int64_t *Vc = V + c * P * 2;
        for (int64_t i = 0; i < n_in; ++i) {
            const int8_t *xi = xc + i * T * 2;
            for (int64_t j = 0; j <= i; ++j) {
                const int8_t *xj = xc + j * T * 2;
                int64_t re = 0, im = 0;
                for (int64_t t = 0; t < T; ++t) {
                    const int64_t ar = xi[2 * t], ai = xi[2 * t + 1];
                    const int64_t br = xj[2 * t], bi = xj[2 * t + 1];
                    /* (ar + i ai)(br - i bi) */
                    re += ar * br + ai * bi;
                    im += ai * br - ar * bi;
                }
                const int64_t b = i * (i + 1) / 2 + j;
                Vc[2 * b] = re;
                Vc[2 * b + 1] = im;
            }
        }
    }
}

/* Same definition on FP64 complex samples [n_ch][n_in][T][2]. */
void oracle_xengine_cf64(const double *x, int64_t n_ch, int64_t n_in, int64_t T, double *V)
{
    const int64_t P = tri(n_in);
    int64_t c;
#pragma omp parallel for schedule(dynamic, 1)
    for (c = 0; c < n_ch; ++c) {
        const double *xc = x + c * n_in * T * 2;
        double *Vc = V + c * P * 2;
        for (int64_t i = 0; i < n_in; ++i) {
            const double *xi = xc + i * T * 2;
            for (int64_t j = 0; j <= i; ++j) {
                const double *xj = xc + j * T * 2;
                double re = 0.0, im = 0.0;
                for (int64_t t = 0; t < T; ++t) {
                    const double ar = xi[2 * t], ai = xi[2 * t + 1];
                    const double br = xj[2 * t], bi = xj[2 * t + 1];
                    re += ar * br + ai * bi;
                    im += ai * br - ar * bi;
                }
                const int64_t b = i * (i + 1) / 2 + j;
                Vc[2 * b] = re;
                Vc[2 * b + 1] = im;
            }
        }
    }
}

/* Selected products of one channel: xc int8 [n_in][T][2]; for k < n,
 * out[k] = V_{ii[k], jj[k]} (any i, j in range; no triangle restriction). */
void oracle_xengine_pairs_ci8(const int8_t *xc, int64_t n_in, int64_t T,
                              const int32_t *ii, const int32_t *jj, int64_t n, int64_t *out)
{
    int64_t k;
    (void)n_in;
#pragma omp parallel for schedule(static)
    for (k = 0; k < n; ++k) {
        const int8_t *xi = xc + (int64_t)ii[k] * T * 2;
        const int8_t *xj = xc + (int64_t)jj[k] * T * 2;
        int64_t re = 0, im = 0;
        for (int64_t t = 0; t < T; ++t) {
            const int64_t ar = xi[2 * t], ai = xi[2 * t + 1];
            const int64_t br = xj[2 * t], bi = xj[2 * t + 1];
            re += ar * br + ai * bi;
            im += ai * br - ar * bi;
        }
        out[2 * k] = re;
        out[2 * k + 1] = im;
    }
}

/* ------------------------------------------------------------ F-stage DFT */

/* v: int8 [n_blocks*N][n_in] (time-major, input fastest).
 * X: double [n_keep][n_in][n_blocks][2], X[k][i][b] = DFT_k of block b of
 * input i, for k < n_keep (n_keep <= N). */
void oracle_dft_real(const int8_t *v, int64_t N, int64_t n_in, int64_t n_blocks,
                     int64_t n_keep, double *X)
{
    const double two_pi = 6.283185307179586476925286766559;
    if (N <= 0) return;
    double *cs = (double *)malloc((size_t)N * sizeof(double));
    double *sn = (double *)malloc((size_t)N * sizeof(double));
    if (!cs || !sn) { free(cs); free(sn); return; }
    for (int64_t m = 0; m < N; ++m) {
        cs[m] = cos(two_pi * (double)m / (double)N);
        sn[m] = sin(two_pi * (double)m / (double)N);
    }
    int64_t i;
#pragma omp parallel for schedule(dynamic, 1)
    for (i = 0; i < n_in; ++i) {
        for (int64_t b = 0; b < n_blocks; ++b) {
            for (int64_t k = 0; k < n_keep; ++k) {
                double re = 0.0, im = 0.0;
                for (int64_t n = 0; n < N; ++n) {
                    const double xn = (double)v[(b * N + n) * n_in + i];
                    const int64_t m = (k * n) % N;
                    re += xn * cs[m];
                    im -= xn * sn[m];
                }
                double *dst = X + ((k * n_in + i) * n_blocks + b) * 2;
                dst[0] = re;
                dst[1] = im;
            }
        }
    }
    free(cs);
    free(sn);
}

/* h: double [P*N] prototype filter (see the header). */
void oracle_pfb_coeffs(int64_t P, int64_t N, double *h)
{
    const double pi = 3.14159265358979323846264338327950288;
    const int64_t L = P * N;
    for (int64_t m = 0; m < L; ++m) {
        const double w = (L > 1) ? 0.54 - 0.46 * cos(2.0 * pi * (double)m / (double)(L - 1)) : 1.0;
        const double x = ((double)m - 0.5 * (double)(L - 1)) / (double)N;
        const double sinc = (x == 0.0) ? 1.0 : sin(pi * x) / (pi * x);
        h[m] = w * sinc;
    }
}

/* v: int8 [(n_blocks + P - 1)*N][n_in] time-major; h: double [P*N].
 * X: double [n_keep][n_in][n_blocks][2], the real DFT of y_b (see the header). */
void oracle_pfb_real(const int8_t *v, const double *h, int64_t N, int64_t P, int64_t n_in, int64_t n_blocks,
                     int64_t n_keep, double *X)
{
    const double two_pi = 6.283185307179586476925286766559;
    if (N <= 0 || P <= 0) return;
    double *cs = (double *)malloc((size_t)N * sizeof(double));
    double *sn = (double *)malloc((size_t)N * sizeof(double));
    if (!cs || !sn) { free(cs); free(sn); return; }
    for (int64_t m = 0; m < N; ++m) {
        cs[m] = cos(two_pi * (double)m / (double)N);
        sn[m] = sin(two_pi * (double)m / (double)N);
    }
    int64_t i;
#pragma omp parallel for schedule(dynamic, 1)
    for (i = 0; i < n_in; ++i) {
        double *y = (double *)malloc((size_t)N * sizeof(double));
        if (!y) continue;
        for (int64_t b = 0; b < n_blocks; ++b) {
            for (int64_t n = 0; n < N; ++n) {
                double acc = 0.0;
                for (int64_t p = 0; p < P; ++p)
                    acc += h[p * N + n] * (double)v[((b + p) * N + n) * n_in + i];
                y[n] = acc;
            }
            for (int64_t k = 0; k < n_keep; ++k) {
                double re = 0.0, im = 0.0;
                for (int64_t n = 0; n < N; ++n) {
                    const int64_t m = (k * n) % N;
                    re += y[n] * cs[m];
                    im -= y[n] * sn[m];
                }
                double *dst = X + ((k * n_in + i) * n_blocks + b) * 2;
                dst[0] = re;
                dst[1] = im;
            }
        }
        free(y);
    }
    free(cs);
    free(sn);
}

/* v: int8 [n_blocks*N][n_in][2] complex (re, im), time-major, input fastest.
 * X: double [N][n_in][n_blocks][2], X[k][i][b] = DFT_k of block b of input i. */
void oracle_dft_complex(const int8_t *v, int64_t N, int64_t n_in, int64_t n_blocks, double *X)
{
    const double two_pi = 6.283185307179586476925286766559;
    if (N <= 0) return;
    double *cs = (double *)malloc((size_t)N * sizeof(double));
    double *sn = (double *)malloc((size_t)N * sizeof(double));
    if (!cs || !sn) { free(cs); free(sn); return; }
    for (int64_t m = 0; m < N; ++m) {
        cs[m] = cos(two_pi * (double)m / (double)N);
        sn[m] = sin(two_pi * (double)m / (double)N);
    }
    int64_t i;
#pragma omp parallel for schedule(dynamic, 1)
    for (i = 0; i < n_in; ++i) {
        for (int64_t b = 0; b < n_blocks; ++b) {
            for (int64_t k = 0; k < N; ++k) {
                double re = 0.0, im = 0.0;
                for (int64_t n = 0; n < N; ++n) {
                    const int8_t *x = v + ((b * N + n) * n_in + i) * 2;
                    const double xr = (double)x[0], xi = (double)x[1];
                    const int64_t m = (k * n) % N;
                    /* (xr + i xi)(cos - i sin) */
                    re += xr * cs[m] + xi * sn[m];
                    im += xi * cs[m] - xr * sn[m];
                }
                double *dst = X + ((k * n_in + i) * n_blocks + b) * 2;
                dst[0] = re;
                dst[1] = im;
            }
        }
    }
    free(cs);
    free(sn);
}

/* ---------------------------------------------------------- sample formats */

/* Two's-complement value of the low `bits` bits of u. */
static int32_t sext(uint32_t u, int bits)
{
    const uint32_t m = (1u << bits) - 1u;
    const uint32_t v = u & m;
    return (v & (1u << (bits - 1))) ? (int32_t)v - (int32_t)(1u << bits) : (int32_t)v;
}

/* w: uint16 [n]; out: int8 [n][2] (re, im). */
void oracle_unpack_w16(const uint16_t *w, int64_t n, int8_t *out)
{
    for (int64_t k = 0; k < n; ++k) {
        out[2 * k] = (int8_t)sext((uint32_t)w[k] >> 5, 5);
        out[2 * k + 1] = (int8_t)sext((uint32_t)w[k], 5);
    }
}

/* b: uint8 [n]; out: int8 [n][2] (re, im). */
void oracle_unpack_b8(const uint8_t *b, int64_t n, int8_t *out)
{
    for (int64_t k = 0; k < n; ++k) {
        out[2 * k] = (int8_t)sext((uint32_t)b[k] >> 4, 4);
        out[2 * k + 1] = (int8_t)sext((uint32_t)b[k], 4);
    }
}

/* rec: uint16 [n_streams][n_rec][1 + w_per]; out: uint16 [n_rec][n_streams * w_per],
 * out[r][s * w_per + w] = rec[s][r][1 + w].  Returns the number of records r
 * for which some stream's word 0 differs from (first_counter + r) mod 2^16. */
int64_t oracle_aggregate_w16(const uint16_t *rec, int64_t n_streams, int64_t w_per, int64_t n_rec,
                             uint32_t first_counter, uint16_t *out)
{
    int64_t bad = 0;
    for (int64_t r = 0; r < n_rec; ++r) {
        int mismatch = 0;
        const uint16_t want = (uint16_t)((first_counter + (uint64_t)r) & 0xFFFFu);
        for (int64_t s = 0; s < n_streams; ++s) {
            const uint16_t *src = rec + (s * n_rec + r) * (1 + w_per);
            if (src[0] != want) mismatch = 1;
            for (int64_t w = 0; w < w_per; ++w) out[r * n_streams * w_per + s * w_per + w] = src[1 + w];
        }
        bad += mismatch;
    }
    return bad;
}

/* ------------------------------------------------------------ requantiser */

/* q[k] = clip(round_half_even(s * y[k]), -max_abs, max_abs).  The default
 * rounding mode is round-to-nearest-even, which nearbyint() uses. */
void oracle_requant(const double *y, int64_t n, double s, int32_t max_abs, int8_t *q)
{
    for (int64_t k = 0; k < n; ++k) {
        double r = nearbyint(s * y[k]);
        if (r > (double)max_abs) r = (double)max_abs;
        if (r < -(double)max_abs) r = -(double)max_abs;
        q[k] = (int8_t)r;
    }
}

/* ----------------------------------------------------------------- codecs */

/* Round |a| to a multiple of the power-of-two quantum q, ties to even. */
static double round_to_quantum(double a, double q) { return nearbyint(a / q) * q; }

static uint16_t f16_encode1(double x)
{
    uint16_t sign = signbit(x) ? 0x8000u : 0u;
    double a = fabs(x);
    if (isnan(x)) return 0x7E00u;
    if (a == 0.0) return sign;
    int e2;
    frexp(a, &e2);              /* a = m 2^e2, m in [0.5, 1): a in [2^(e2-1), 2^e2) */
    int E = e2 - 1;
    double q = (E < -14) ? ldexp(1.0, -24) : ldexp(1.0, E - 10);
    double r = round_to_quantum(a, q);
    if (r >= 65536.0) return sign | 0x7C00u;           /* overflow to infinity */
    if (r < ldexp(1.0, -14)) {                          /* subnormal (or zero) */
        return sign | (uint16_t)(r / ldexp(1.0, -24));
    }
    frexp(r, &e2);
    E = e2 - 1;
    if (E > 15) return sign | 0x7C00u;
    uint16_t mant = (uint16_t)(r / ldexp(1.0, E - 10) - 1024.0);
    return sign | (uint16_t)((E + 15) << 10) | mant;
}

static double f16_decode1(uint16_t h)
{
    int s = (h >> 15) & 1, e = (h >> 10) & 0x1F, m = h & 0x3FF;
    double v;
    if (e == 0) v = ldexp((double)m, -24);
    else if (e == 31) v = (m == 0) ? INFINITY : NAN;
    else v = ldexp(1.0 + (double)m / 1024.0, e - 15);
    return s ? -v : v;
}

void oracle_f16_encode(const double *x, int64_t n, uint16_t *out)
{
    for (int64_t k = 0; k < n; ++k) out[k] = f16_encode1(x[k]);
}

void oracle_f16_decode(const uint16_t *h, int64_t n, double *out)
{
    for (int64_t k = 0; k < n; ++k) out[k] = f16_decode1(h[k]);
}

/* OCP FP8 E4M3FN: 1 sign, 4 exponent (bias 7), 3 mantissa bits; exponent 15
 * with mantissa 7 is NaN, there is no infinity; largest finite 448 = 1.75*2^8;
 * smallest subnormal 2^-9.  Saturating: finite values beyond 448 encode 448. */
static uint8_t e4m3_encode1(double x)
{
    uint8_t sign = signbit(x) ? 0x80u : 0u;
    double a = fabs(x);
    if (isnan(x)) return 0x7Fu;
    if (a == 0.0) return sign;
    int e2;
    frexp(a, &e2);
    int E = e2 - 1;
    double q = (E < -6) ? ldexp(1.0, -9) : ldexp(1.0, E - 3);
    double r = round_to_quantum(a, q);
    if (r > 448.0) r = 448.0;
    if (r < ldexp(1.0, -6)) return sign | (uint8_t)(r / ldexp(1.0, -9));
    frexp(r, &e2);
    E = e2 - 1;
    uint8_t mant = (uint8_t)(r / ldexp(1.0, E - 3) - 8.0);
    return sign | (uint8_t)((E + 7) << 3) | mant;
}

static double e4m3_decode1(uint8_t b)
{
    int s = (b >> 7) & 1, e = (b >> 3) & 0xF, m = b & 7;
    double v;
    if (e == 15 && m == 7) return NAN;
    if (e == 0) v = ldexp((double)m, -9);
    else v = ldexp(1.0 + (double)m / 8.0, e - 7);
    return s ? -v : v;
}

void oracle_e4m3_encode(const double *x, int64_t n, uint8_t *out)
{
    for (int64_t k = 0; k < n; ++k) out[k] = e4m3_encode1(x[k]);
}

void oracle_e4m3_decode(const uint8_t *b, int64_t n, double *out)
{
    for (int64_t k = 0; k < n; ++k) out[k] = e4m3_decode1(b[k]);
}

/* Per-channel power-of-two scale for E4M3: the largest s = 2^e with
 * s * m <= 448, where m = max |re|, |im| over the channel (s = 1 if m = 0). */
double oracle_e4m3_scale(const double *x, int64_t n)
{
    double m = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double a = fabs(x[k]);
        if (a > m) m = a;
    }
    if (m == 0.0) return 1.0;
    double s = 1.0;
    while (s * m > 448.0) s *= 0.5;
    while (2.0 * s * m <= 448.0) s *= 2.0;
    return s;
}

/* --------------------------------------------------------------- long-run */

void oracle_fold_i64(double *L, const int64_t *V, int64_t n)
{
    for (int64_t k = 0; k < n; ++k) L[k] += (double)V[k];
}

void oracle_fold_f64(double *L, const double *V, int64_t n)
{
    for (int64_t k = 0; k < n; ++k) L[k] += V[k];
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
