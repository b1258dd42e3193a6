"""CPU checks of the F-stage parity helper (tests/fcheck.py): the a-priori
FP32 FFT error bound must hold for an independent FP32 FFT (scipy's pocketfft
in single precision) on the C2-shaped signal, and the tie-band rule must
reject a requantised code that differs outside the band."""
import math

import numpy as np
import pytest
import scipy.fft

import fcheck
import oracle
import synth

S = float(np.float32(2.0 / (16.0 * math.sqrt(128.0))))


def f32_rfft_like_gpu(v: np.ndarray) -> np.ndarray:
    """FP32 real FFT of each 256-sample block -> [128][n_in][nb][2] float32."""
    nb = v.shape[0] // 256
    x = v.astype(np.float32).reshape(nb, 256, -1)
    Z = scipy.fft.rfft(x, axis=1)[:, :128, :]                       # complex64 [nb][128][n_in]
    assert Z.dtype == np.complex64
    out = np.stack([Z.real, Z.imag], axis=-1).transpose(1, 2, 0, 3)
    return np.ascontiguousarray(out, dtype=np.float32)


def test_bound_holds_for_an_fp32_fft():
    v = synth.real_voltages(seed=2, index=0, n_blocks=24, n_inputs=16)
    X = oracle.dft_real(v, 256)
    Xg = f32_rfft_like_gpu(v)
    bound = fcheck.real_bound(v, 256)
    err = np.abs(Xg.astype(np.float64) - X).max()
    assert 0 < err <= bound
    # the bound is a worst case, but not a vacuous one for this signal
    assert bound < 1e-3 * np.sqrt(np.mean(X ** 2)) * 10
    q = oracle.requant(Xg.astype(np.float64), S, 7)          # codes from the FP32 spectra
    r = fcheck.check_spectra_requant(X, Xg, q, S, 7, bound, "scipy fp32")
    assert r["mismatch_frac"] <= 8 * S * bound


def test_tie_band_rejects_a_code_outside_it():
    v = synth.real_voltages(seed=2, index=1, n_blocks=4, n_inputs=8)
    X = oracle.dft_real(v, 256)
    Xg = f32_rfft_like_gpu(v)
    q = oracle.requant(Xg.astype(np.float64), S, 7)
    y = S * X
    far = np.abs(y - np.floor(y) - 0.5) > 0.25                    # far from any .5 boundary
    k = np.flatnonzero(far & (np.abs(y) < 5))[0]
    q.flat[k] += 1                                                 # a wrong code away from a tie
    with pytest.raises(AssertionError):
        fcheck.check_spectra_requant(X, Xg, q, S, 7, fcheck.real_bound(v, 256), "planted")


def test_complex_and_pfb_bounds_hold_for_fp32():
    rec, lv = synth.capture_records(seed=4, index=0, n_records=8 * 128, n_streams=1, w_per=8)
    lvd = oracle.unpack_w16(np.ascontiguousarray(rec[0, :, 1:]))
    X = oracle.dft_complex(lvd, 128)
    z = (lvd[..., 0].astype(np.float32) + 1j * lvd[..., 1].astype(np.float32)).astype(np.complex64)
    Z = scipy.fft.fft(z.reshape(8, 128, 8), axis=1)                # [nb][k][n_in]
    Xg = np.stack([Z.real, Z.imag], axis=-1).transpose(1, 2, 0, 3)
    assert np.abs(Xg.astype(np.float64) - X).max() <= fcheck.complex_bound(lvd, 128)

    P, N = 4, 256
    v = synth.real_voltages(seed=9, index=0, n_blocks=6 + P - 1, n_inputs=4)
    Xp = oracle.pfb_real(v, N, P)
    h = oracle.pfb_coeffs(P, N).astype(np.float32)
    x = v.astype(np.float32).reshape(6 + P - 1, N, -1)
    y = np.zeros((6, N, x.shape[2]), np.float32)
    for p in range(P):
        y += h[p * N:(p + 1) * N][None, :, None] * x[p:p + 6]
    Zp = scipy.fft.rfft(y, axis=1)[:, :128, :]
    Xpg = np.stack([Zp.real, Zp.imag], axis=-1).transpose(1, 2, 0, 3)
    assert np.abs(Xpg.astype(np.float64) - Xp).max() <= fcheck.pfb_bound(v, N, P)
