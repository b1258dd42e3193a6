"""Host-side checks of the seeded generators (device identity is a GPU test)."""
import numpy as np

import synth


def test_level_distribution_chi2():
    x = synth.ci8_channel(seed=1, ch=3, n_inputs=64, n_samples=4000)
    assert x.min() >= -7 and x.max() <= 7
    counts = np.bincount(x.ravel().astype(np.int64) + 7, minlength=15)
    p = synth.level_probabilities(2.0, 7)
    e = p * x.size
    chi2 = float(np.sum((counts - e) ** 2 / e))
    assert chi2 < 60.0, chi2
    assert abs(np.var(x.astype(np.float64)) - float(np.sum(p * np.arange(-7, 8) ** 2))) < 0.02


def test_deterministic_and_subset():
    a = synth.ci8_channel(5, 7, 10, 100)
    b = synth.ci8_channel(5, 7, 10, 100)
    assert np.array_equal(a, b)
    sub = synth.ci8_channel(5, 7, 10, 60, t0=40, inputs=[3, 9])
    assert np.array_equal(sub, a[[3, 9], 40:100])
    assert not np.array_equal(a, synth.ci8_channel(6, 7, 10, 100))
    assert not np.array_equal(a, synth.ci8_channel(5, 8, 10, 100))


def test_thresholds_monotone():
    t = synth.level_thresholds()
    assert t.size == 14 and np.all(np.diff(t.astype(np.int64)) > 0)


def test_real_voltages_shape_and_power():
    v = synth.real_voltages(2, 0, 50)
    assert v.shape == (50 * 256, 64) and v.dtype == np.int8
    assert abs(v[:, 10:].astype(np.float64).std() - 16.06) < 0.3
    # common noise on inputs 0..7: zero-lag correlation about 0.1
    c = np.corrcoef(v[:, :8].T.astype(np.float64))
    assert abs(c[np.triu_indices(8, 1)].mean() - 0.1) < 0.02


def test_complex_float_gains_pairs():
    pairs = synth.coherent_pairs(4, 256)
    flat = [i for p in pairs for i in p]
    assert len(pairs) == 16 and len(set(flat)) == 32
    x = synth.complex_float(4, 0, 256, 4096)
    z = x[..., 0].astype(np.float64) + 1j * x[..., 1]
    g = synth.input_gains(4, 256)
    np.testing.assert_allclose(np.mean(np.abs(z) ** 2, axis=1) / g ** 2, 1.0, atol=0.1)
    i, j = pairs[0]
    r = np.mean(z[i] * np.conj(z[j])) / (g[i] * g[j])
    assert abs(r - 0.1) < 0.05


def test_c_twin_matches_numpy():
    for args in ((5, 7, 10, 100), (0, 0, 1, 1), (123456789, 1000, 33, 257)):
        assert np.array_equal(synth.ci8_channel(*args), synth.ci8_channel_numpy(*args))
    assert np.array_equal(synth.ci8_channel(5, 7, 10, 60, t0=40, inputs=[3, 9]),
                          synth.ci8_channel_numpy(5, 7, 10, 60, t0=40, inputs=[3, 9]))
    blk = synth.ci8_block(2, 3, 4, 6, 50)
    for c in range(4):
        assert np.array_equal(blk[c], synth.ci8_channel_numpy(2, 3 + c, 6, 50))
