"""Pins of the oracle's complex front end: the recorded sample formats, the
aggregation of capture streams, and the complex DFT.

Sec. 3 describes the prototype's recorded data: 5-bit real and imaginary
parts in two's complement stored in 16-bit words, records of one
marker/counter word and 16 data words per capture PC, four PCs interleaved
into 64 inputs per time instant.  Sec. 5 adds a 1-byte mode with one bit less
per part.  Sec. 2 / Sec. 4: for complex samples, N_C samples give N_C
channels.
"""
import numpy as np

import oracle
from conftest import read_golden


def test_formats_golden():
    rows = read_golden("frontend_formats.txt")
    assert len(rows) >= 16
    for kind, word, re, im in rows:
        v = int(word, 16)
        got = oracle.unpack_w16(np.array([v], np.uint16)) if kind == "w16" else \
            oracle.unpack_b8(np.array([v], np.uint8))
        assert got.tolist() == [[int(re), int(im)]], (kind, word)


def test_w16_is_a_bijection_on_ten_bits():
    words = np.arange(1024, dtype=np.uint16)
    d = oracle.unpack_w16(words).astype(np.int64)
    assert d.min() == -16 and d.max() == 15
    # re-encode with Python's modulo (two's complement of 5 bits) and compare
    enc = ((d[:, 0] % 32) << 5) | (d[:, 1] % 32)
    assert np.array_equal(enc, words.astype(np.int64))
    # the upper six bits do not matter
    rng = np.random.default_rng(3)
    hi = rng.integers(0, 64, 1024).astype(np.uint16) << 10
    assert np.array_equal(oracle.unpack_w16(words | hi), oracle.unpack_w16(words))


def test_b8_is_a_bijection_on_eight_bits():
    b = np.arange(256, dtype=np.uint8)
    d = oracle.unpack_b8(b).astype(np.int64)
    assert d.min() == -8 and d.max() == 7
    enc = ((d[:, 0] % 16) << 4) | (d[:, 1] % 16)
    assert np.array_equal(enc, b.astype(np.int64))


def test_b8_is_w16_with_one_bit_less():
    # Sec. 5: the 1-byte mode keeps one bit less of each part; dropping the
    # low bit of each 5-bit part (floor halving) gives the 4-bit part.
    words = np.arange(1024, dtype=np.uint16)
    d5 = oracle.unpack_w16(words).astype(np.int64)
    bytes_ = ((((d5[:, 0] >> 1) % 16) << 4) | ((d5[:, 1] >> 1) % 16)).astype(np.uint8)
    d4 = oracle.unpack_b8(bytes_).astype(np.int64)
    assert np.array_equal(d4, d5 >> 1)


def test_aggregate_hand_example():
    # two streams of two records, three inputs each; counters 5, 6
    rec = np.array([[[5, 1, 2, 3], [6, 4, 5, 6]],
                    [[5, 11, 12, 13], [6, 14, 15, 16]]], dtype=np.uint16)
    out, bad = oracle.aggregate_w16(rec, first_counter=5)
    assert bad == 0
    assert out.tolist() == [[1, 2, 3, 11, 12, 13], [4, 5, 6, 14, 15, 16]]
    rec[1, 1, 0] = 7               # stream 1 skipped a record
    assert oracle.aggregate_w16(rec, first_counter=5)[1] == 1
    assert oracle.aggregate_w16(rec, first_counter=4)[1] == 2


def test_aggregate_counter_wraps_and_keeps_every_sample():
    rng = np.random.default_rng(9)
    ns, nr, wp = 4, 300, 16
    data = rng.integers(0, 1 << 16, (ns, nr, wp)).astype(np.uint16)
    cnt = ((0xFF80 + np.arange(nr)) & 0xFFFF).astype(np.uint16)
    rec = np.concatenate([np.broadcast_to(cnt[None, :, None], (ns, nr, 1)), data], axis=2)
    out, bad = oracle.aggregate_w16(rec, first_counter=0xFF80)
    assert bad == 0 and out.shape == (nr, ns * wp)
    # every sample lands once, in time order, stream-major within a time instant
    assert np.array_equal(out.reshape(nr, ns, wp).transpose(1, 0, 2), data)


def _c(X):
    return X[..., 0] + 1j * X[..., 1]


def test_dft_complex_against_numpy_fft():
    rng = np.random.default_rng(31)
    N, nb, ni = 128, 5, 3
    x = rng.integers(-16, 16, (nb * N, ni, 2)).astype(np.int8)
    X = _c(oracle.dft_complex(x, N))                                 # [k][input][block]
    z = (x[..., 0] + 1j * x[..., 1]).astype(np.complex128).reshape(nb, N, ni)
    ref = np.fft.fft(z, axis=1).transpose(1, 2, 0)
    assert X.shape == (N, ni, nb)                                     # N samples -> N channels
    assert np.abs(X - ref).max() <= 1e-12 * np.abs(ref).max()


def test_dft_complex_integer_tone_and_impulse():
    N = 128
    n = np.arange(N)
    # exp(2 pi i 32 n / 128) = i^n: integer samples, all power in channel 32
    ph = np.array([[1, 0], [0, 1], [-1, 0], [0, -1]], np.int8)[n % 4] * 10
    X = _c(oracle.dft_complex(ph[:, None, :], N))[:, 0, 0]
    assert abs(X[32] - 10 * N) < 1e-9
    assert np.abs(np.delete(X, 32)).max() < 1e-9
    # negative frequency: exp(-2 pi i 32 n / 128) lands in channel 96 (natural order)
    ph_neg = ph.copy()
    ph_neg[:, 1] = -ph_neg[:, 1]
    Xn = _c(oracle.dft_complex(ph_neg[:, None, :], N))[:, 0, 0]
    assert int(np.argmax(np.abs(Xn))) == 96
    # impulse at n0: X_k = a exp(-2 pi i k n0 / N)
    n0, a = 5, 7 - 3j
    imp = np.zeros((N, 1, 2), np.int8)
    imp[n0, 0] = [7, -3]
    Xi = _c(oracle.dft_complex(imp, N))[:, 0, 0]
    assert np.allclose(Xi, a * np.exp(-2j * np.pi * n * n0 / N), atol=1e-12)


def test_dft_complex_parseval():
    rng = np.random.default_rng(32)
    N = 128
    x = rng.integers(-16, 16, (4 * N, 2, 2)).astype(np.int8)
    X = _c(oracle.dft_complex(x, N))
    z = (x[..., 0] + 1j * x[..., 1]).reshape(4, N, 2)
    lhs = (np.abs(X) ** 2).sum(axis=0)                  # [input][block]
    rhs = N * (np.abs(z) ** 2).sum(axis=1).T
    assert np.allclose(lhs, rhs, rtol=1e-12)
