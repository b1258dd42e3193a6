"""Pins of the oracle's polyphase filterbank F-stage (Sec. 6.1 names a PFB as
the way to cut the FFT's spectral leakage, without a design; the reading here:
P taps of N points, y_b[n] = sum_p h[pN + n] x[(b + p)N + n], h = Hamming
window x sinc((m - (PN-1)/2)/N), then the real DFT of the plain F-stage)."""
import numpy as np

import oracle

N, P = 256, 4


def _c(X):
    return X[..., 0] + 1j * X[..., 1]


def test_coeffs_are_hamming_times_sinc():
    L = P * N
    h = oracle.pfb_coeffs(P, N)
    ref = np.hamming(L) * np.sinc((np.arange(L) - (L - 1) / 2.0) / N)
    assert np.abs(h - ref).max() < 1e-15
    assert np.abs(h - h[::-1]).max() < 1e-15
    assert abs(h[0] / np.sinc(-(L - 1) / 2.0 / N) - 0.08) < 1e-15     # Hamming end value


def test_one_tap_rectangular_is_the_plain_dft():
    rng = np.random.default_rng(41)
    v = rng.integers(-128, 128, size=(5 * N, 3), dtype=np.int8)
    X = oracle.pfb_real(v, N, 1, h=np.ones(N))
    assert np.array_equal(X, oracle.dft_real(v, N))


def test_impulse_response_closed_form():
    # x = a delta at sample (b + p) N + n0 of input 1: y_b[n0] = a h[pN + n0], others 0
    h = oracle.pfb_coeffs(P, N)
    nb, a, n0 = 3, 9, 41
    v = np.zeros(((nb + P - 1) * N, 2), np.int8)
    v[(1 + 2) * N + n0, 1] = a                     # block 3 = b + p for (b, p) = (1, 2), (2, 1), (0, 3)
    X = _c(oracle.pfb_real(v, N, P))[:, 1, :]      # [k][block]
    k = np.arange(N // 2)
    for b in range(nb):
        p = 3 - b
        want = a * h[p * N + n0] * np.exp(-2j * np.pi * k * n0 / N)
        assert np.allclose(X[:, b], want, atol=1e-10)
    assert np.abs(_c(oracle.pfb_real(v, N, P))[:, 0, :]).max() == 0.0


def test_one_block_shift_moves_the_output_by_one_block():
    rng = np.random.default_rng(42)
    v = rng.integers(-100, 100, size=((6 + P - 1) * N, 2), dtype=np.int8)
    X = oracle.pfb_real(v, N, P)
    Xs = oracle.pfb_real(v[N:], N, P)
    assert np.array_equal(X[:, :, 1:], Xs)


def test_against_numpy_rfft_of_the_weighted_sum():
    rng = np.random.default_rng(43)
    nb = 4
    v = rng.integers(-128, 128, size=((nb + P - 1) * N, 2), dtype=np.int8)
    h = oracle.pfb_coeffs(P, N).reshape(P, N)
    blocks = v.astype(np.float64).reshape(nb + P - 1, N, 2)
    y = np.stack([(h[:, :, None] * blocks[b:b + P]).sum(axis=0) for b in range(nb)])   # [b][n][i]
    ref = np.fft.rfft(y, axis=1)[:, : N // 2, :].transpose(1, 2, 0)
    X = _c(oracle.pfb_real(v, N, P))
    assert np.abs(X - ref).max() <= 1e-12 * np.abs(ref).max()


def _tone_power(bin_pos, P_taps, h=None):
    nb = 8
    t = np.arange((nb + P_taps - 1) * N)
    v = np.rint(100 * np.cos(2 * np.pi * bin_pos * t / N)).astype(np.int8)[:, None]
    X = _c(oracle.pfb_real(v, N, P_taps, h=h))[:, 0, :]
    return (np.abs(X) ** 2).mean(axis=1)


def test_less_leakage_and_scalloping_than_the_plain_dft():
    # a tone between channel centres (37.5): power 3 or more channels away,
    # relative to the peak, falls by far more than 20 dB with the PFB
    dft = _tone_power(37.5, 1, h=np.ones(N))
    pfb = _tone_power(37.5, P)
    far = np.r_[0:35, 41:128]
    leak_dft = dft[far].max() / dft.max()
    leak_pfb = pfb[far].max() / pfb.max()
    assert leak_pfb < leak_dft * 1e-2, (leak_dft, leak_pfb)
    # the two channels either side of the tone hold nearly all of the PFB's
    # output power (a sinc prototype one channel wide crosses at -6 dB at the
    # channel edge, so the pair sums flat), far more than the DFT's
    frac_dft = dft[37:39].sum() / dft.sum()
    frac_pfb = pfb[37:39].sum() / pfb.sum()
    assert frac_pfb > 0.999 and frac_dft < 0.9, (frac_dft, frac_pfb)
