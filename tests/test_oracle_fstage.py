"""Pins of the oracle F-stage (direct real DFT) and requantiser.

Real input: 2 N_C samples give N_C + 1 channels including DC; the build keeps
k = 0 .. N_C-1 (Sec. 2 and Sec. 4).  Forward sign, unnormalised.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from conftest import read_golden

N = 256


def _to_complex(X):
    return X[..., 0] + 1j * X[..., 1]


def test_against_numpy_rfft():
    rng = np.random.default_rng(21)
    v = rng.integers(-128, 128, size=(5 * N, 3), dtype=np.int8)
    X = _to_complex(oracle.dft_real(v, N))          # [k][input][block]
    ref = np.fft.rfft(v.astype(np.float64).reshape(5, N, 3), axis=1)  # [block][k][input]
    ref = ref[:, : N // 2, :].transpose(1, 2, 0)
    scale = np.abs(ref).max()
    assert np.abs(X - ref).max() <= 1e-12 * scale


def test_channel_count():
    v = np.zeros((N, 1), np.int8)
    assert oracle.dft_real(v, N).shape == (128, 1, 1, 2)   # 256-pt real -> 128 channels (DC kept)


def test_parseval():
    rng = np.random.default_rng(22)
    v = rng.integers(-128, 128, size=(4 * N, 2), dtype=np.int8)
    Xf = _to_complex(oracle.dft_real(v, N, n_keep=N))   # full spectrum
    x = v.astype(np.float64).reshape(4, N, 2)
    for b in range(4):
        for i in range(2):
            e_t = np.sum(x[b, :, i] ** 2)
            Xk = Xf[:, i, b]
            e_f = (abs(Xk[0]) ** 2 + 2 * np.sum(np.abs(Xk[1:N // 2]) ** 2) + abs(Xk[N // 2]) ** 2) / N
            assert abs(e_t - e_f) <= 1e-9 * e_t


def test_real_input_symmetry():
    rng = np.random.default_rng(23)
    v = rng.integers(-128, 128, size=(N, 2), dtype=np.int8)
    Xf = _to_complex(oracle.dft_real(v, N, n_keep=N))
    for k in range(1, N):
        np.testing.assert_allclose(Xf[N - k], np.conj(Xf[k]), atol=1e-9)


def test_pure_tone_bin37():
    """A rounded cosine of amplitude 100 at 37 cycles per 256 samples: bin 37
    holds N*A/2 = 12800 up to the rounding error, every other bin is bounded
    by the rounding error's l1 norm (256 * 0.5)."""
    n = np.arange(N)
    v = np.rint(100 * np.cos(2 * np.pi * 37 * n / N)).astype(np.int8)[:, None]
    X = _to_complex(oracle.dft_real(v, N))[:, 0, 0]
    assert abs(X[37] - 12800) <= 128
    others = np.delete(np.abs(X), 37)
    assert others.max() <= 128
    assert np.argmax(np.abs(X)) == 37


def test_exact_tone_quarter_band():
    """cos(pi n / 2) takes values 1, 0, -1, 0 exactly: X_64 = 128 A, all else 0."""
    n = np.arange(N)
    v = (50 * np.round(np.cos(np.pi * n / 2))).astype(np.int8)[:, None]
    X = _to_complex(oracle.dft_real(v, N))[:, 0, 0]
    assert abs(X[64] - 6400) < 1e-9
    assert np.abs(np.delete(X, 64)).max() < 1e-9


def test_impulse_and_constant():
    v = np.zeros((2 * N, 1), np.int8)
    v[0, 0] = 7            # block 0: impulse at n = 0
    v[N:, 0] = -3          # block 1: constant
    X = _to_complex(oracle.dft_real(v, N))[:, 0, :]
    np.testing.assert_allclose(X[:, 0], 7.0, atol=1e-12)
    assert abs(X[0, 1] - (-3 * N)) < 1e-9
    assert np.abs(X[1:, 1]).max() < 1e-9


def test_requant_hand_table():
    rows = read_golden("requant_table.txt")
    y = np.array([float(r[0]) for r in rows])
    q = np.array([int(r[1]) for r in rows])
    assert np.array_equal(oracle.requant(y, 1.0, 7), q)


def test_requant_scale_and_clip():
    y = np.array([10.0, -10.0, 1e9, -1e9, 0.1])
    assert np.array_equal(oracle.requant(y, 0.25, 7), [2, -2, 7, -7, 0])   # 2.5 -> 2 (even)


def _gauss_quant_factor(sigma, max_abs=7):
    """E[x Q(x)]^2 / (Var x Var Q) for x ~ N(0, sigma^2) and Q = clip(round(x)):
    first-order (small rho) ratio of output to input correlation, from closed
    Gaussian integrals (int_a^b x phi_s(x) dx = s^2 (phi_s(a) - phi_s(b)))."""
    def pdf(z):
        return 0.0 if math.isinf(z) else math.exp(-0.5 * (z / sigma) ** 2) / (sigma * math.sqrt(2 * math.pi))
    p = synth.level_probabilities(sigma, max_abs)
    ks = np.arange(-max_abs, max_abs + 1)
    exq = 0.0
    for k in ks:
        lo = -math.inf if k == -max_abs else k - 0.5
        hi = math.inf if k == max_abs else k + 0.5
        exq += k * sigma ** 2 * (pdf(lo) - pdf(hi))
    varq = float(np.sum(p * ks ** 2))
    return exq ** 2 / (sigma ** 2 * varq)


def test_requant_histogram_and_coherence_pipeline():
    """Oracle F-stage on the real-voltage workload (sigma 16, 10% common noise
    power on inputs 0..7, tone at bin 37): the requantised levels follow the
    clipped rounded Gaussian at sigma_q = 2 (chi-square), and the X-engine on
    the requantised spectra recovers the injected coherence 0.1 scaled by the
    quantiser's correlation factor."""
    s = 2.0 / (16.0 * math.sqrt(128.0))
    s32 = float(np.float32(s))
    nb = 400
    v = synth.real_voltages(seed=2, index=0, n_blocks=nb)
    X = oracle.dft_real(v, N)                                    # [128][64][nb][2]
    q = oracle.requant(X, s32, 7)
    # histogram over bins other than DC and the tone
    sel = np.ones(128, bool)
    sel[[0, 37]] = False
    levels = q[sel].ravel()
    counts = np.bincount(levels.astype(np.int64) + 7, minlength=15)
    p = synth.level_probabilities(2.0, 7)
    expct = p * levels.size
    chi2 = float(np.sum((counts - expct) ** 2 / expct))
    assert chi2 < 60.0, chi2      # 14 dof; p < 1e-6 beyond 60
    # coherence of the injected common noise
    V = oracle.xengine_ci8(q)                                     # [128][2080][2]
    f = _gauss_quant_factor(2.0)
    expected = 0.1 * f
    chans = np.nonzero(sel)[0]
    rc = [oracle.coherence(V[chans], 64, i, j, real_part=True).mean() for i in range(8) for j in range(i)]
    assert abs(np.mean(rc) - expected) < 0.006, (np.mean(rc), expected)
    # uncorrelated pairs: complex mean near zero
    unc = []
    for i, j in ((20, 10), (63, 9), (40, 33), (50, 2)):
        b = oracle.baseline_index(i, j)
        vij = V[chans, b, 0] + 1j * V[chans, b, 1]
        unc.append(np.mean(vij / np.sqrt(V[chans, oracle.baseline_index(i, i), 0] * V[chans, oracle.baseline_index(j, j), 0])))
    assert abs(np.mean(unc)) < 0.006
    # the tone dominates bin 37 on every input: real-part coherence about 0.5
    r37 = np.mean([oracle.coherence(V[[37]], 64, i, j, real_part=True)[0] for i in range(20, 30) for j in range(10, 20)])
    assert 0.4 < r37 < 0.6, r37
