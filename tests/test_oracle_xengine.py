"""Pins of the oracle X-engine against things other than itself.

Definition: Sec. 2 (each spectrum times the complex conjugate of the other,
accumulated per baseline, N_I(N_I+1)/2 products incl. autos) and Fig. 2 (the
per-channel outer product x x^H with autos on the diagonal).
"""
import itertools

import numpy as np
import pytest

import oracle
from conftest import read_golden


def _hand():
    rows = read_golden("xengine_hand_example.txt")
    mode = None
    samples, expected = [], []
    for r in rows:
        if r[0] in ("samples", "expected"):
            mode = r[0]
            continue
        (samples if mode == "samples" else expected).append([int(v) for v in r])
    return samples, expected


def test_hand_example():
    samples, expected = _hand()
    x = np.zeros((1, 2, 2, 2), dtype=np.int8)
    for i, t, re, im in samples:
        x[0, i, t] = (re, im)
    V = oracle.xengine_ci8(x)
    for i, j, re, im in expected:
        b = oracle.baseline_index(i, j)
        assert (V[0, b, 0], V[0, b, 1]) == (re, im)


def test_product_count():
    for n in (1, 2, 3, 15, 64, 1024):
        assert oracle.n_products(n) == n * (n - 1) // 2 + n
    assert oracle.n_products(64) == 2080
    assert oracle.n_products(1024) == 524800
    x = np.ones((1, 17, 3, 2), dtype=np.int8)
    assert oracle.xengine_ci8(x).shape == (1, 17 * 18 // 2, 2)


def test_exhaustive_tiny_against_python_complex():
    """Brute force over every input with entries in {-1,0,1}^2 for N_I=2, T=2
    and N_I=3, T=1 (each combination is one channel), compared with Python's
    own complex arithmetic."""
    vals = [complex(a, b) for a in (-1, 0, 1) for b in (-1, 0, 1)]
    for n_in, T in ((2, 2), (3, 1), (1, 3)):
        combos = list(itertools.product(range(9), repeat=n_in * T))
        x = np.zeros((len(combos), n_in, T, 2), dtype=np.int8)
        for c, combo in enumerate(combos):
            for k, v in enumerate(combo):
                i, t = divmod(k, T)
                x[c, i, t] = (int(vals[v].real), int(vals[v].imag))
        V = oracle.xengine_ci8(x)
        for c in range(0, len(combos), max(1, len(combos) // 997)):
            for i in range(n_in):
                for j in range(i + 1):
                    s = 0j
                    for t in range(T):
                        xi = complex(x[c, i, t, 0], x[c, i, t, 1])
                        xj = complex(x[c, j, t, 0], x[c, j, t, 1])
                        s += xi * xj.conjugate()
                    b = oracle.baseline_index(i, j)
                    assert V[c, b, 0] == s.real and V[c, b, 1] == s.imag


def test_matches_numpy_gram():
    """numpy X X^H in FP64 (exact for these small integers)."""
    rng = np.random.default_rng(11)
    x = rng.integers(-7, 8, size=(5, 37, 129, 2), dtype=np.int8)
    V = oracle.xengine_ci8(x)
    ii, jj = np.tril_indices(37)
    b = oracle.baseline_index(ii, jj)
    for c in range(5):
        X = x[c, ..., 0].astype(np.float64) + 1j * x[c, ..., 1].astype(np.float64)
        G = X @ X.conj().T
        assert np.array_equal(V[c, b, 0], G[ii, jj].real.astype(np.int64))
        assert np.array_equal(V[c, b, 1], G[ii, jj].imag.astype(np.int64))


def test_invariants():
    rng = np.random.default_rng(12)
    n_in, T = 23, 301
    x = rng.integers(-7, 8, size=(3, n_in, T, 2), dtype=np.int8)
    V = oracle.xengine_ci8(x)
    d = oracle.baseline_index(np.arange(n_in), np.arange(n_in))
    # autos real, >= 0, imaginary part exactly 0
    assert np.all(V[:, d, 1] == 0) and np.all(V[:, d, 0] >= 0)
    # Cauchy-Schwarz |V_ij|^2 <= V_ii V_jj, exact in integers
    for c in range(3):
        for i in range(n_in):
            for j in range(i):
                b = oracle.baseline_index(i, j)
                lhs = int(V[c, b, 0]) ** 2 + int(V[c, b, 1]) ** 2
                assert lhs <= int(V[c, d[i], 0]) * int(V[c, d[j], 0])
    # Hermitian: V_ji from the pair routine is conj(V_ij)
    ii = np.array([5, 17, 22, 3], dtype=np.int32)
    jj = np.array([2, 9, 0, 3], dtype=np.int32)
    a = oracle.xengine_pairs_ci8(x[1], ii, jj)
    bb = oracle.xengine_pairs_ci8(x[1], jj, ii)
    assert np.array_equal(a[:, 0], bb[:, 0]) and np.array_equal(a[:, 1], -bb[:, 1])
    assert np.array_equal(a, V[1, oracle.baseline_index(ii, jj)])
    # additivity over a split of the time axis
    V1 = oracle.xengine_ci8(x[:, :, :100])
    V2 = oracle.xengine_ci8(x[:, :, 100:])
    assert np.array_equal(V1 + V2, V)
    # zero input gives zero
    assert not oracle.xengine_ci8(np.zeros((2, 5, 7, 2), np.int8)).any()


def test_permutation_permutes():
    rng = np.random.default_rng(13)
    n_in = 11
    x = rng.integers(-7, 8, size=(1, n_in, 50, 2), dtype=np.int8)
    perm = rng.permutation(n_in)
    M = oracle.full_matrix(oracle.xengine_ci8(x)[0], n_in)
    Mp = oracle.full_matrix(oracle.xengine_ci8(x[:, perm])[0], n_in)
    assert np.array_equal(Mp, M[np.ix_(perm, perm)])


def test_conjugation_side():
    """x_j = i x_i gives V_ij = -i V_ii (conjugate taken on the second input)."""
    rng = np.random.default_rng(14)
    xi = rng.integers(-7, 8, size=(40, 2)).astype(np.int8)
    xj = np.stack([-xi[:, 1], xi[:, 0]], axis=1)  # i * (re + i im) = -im + i re
    x = np.stack([xj, xi])[None]  # input 0 = x_j, input 1 = x_i
    V = oracle.xengine_ci8(x)[0]
    vii = V[oracle.baseline_index(1, 1)]
    vij = V[oracle.baseline_index(1, 0)]  # V_{1,0} = sum x_1 conj(x_0) = x_i conj(i x_i)
    assert vij[0] == 0 and vij[1] == -vii[0]


def test_rank_one_at_t1():
    rng = np.random.default_rng(15)
    x = rng.integers(-7, 8, size=(1, 9, 1, 2), dtype=np.int8)
    z = x[0, :, 0, 0].astype(np.float64) + 1j * x[0, :, 0, 1]
    M = oracle.full_matrix(oracle.xengine_ci8(x)[0], 9)
    assert np.array_equal(M, np.outer(z, z.conj()))
    assert np.linalg.matrix_rank(M) <= 1


def test_float_oracle_agrees():
    rng = np.random.default_rng(16)
    xi = rng.integers(-7, 8, size=(2, 13, 77, 2), dtype=np.int8)
    assert np.array_equal(oracle.xengine_cf64(xi.astype(np.float64)), oracle.xengine_ci8(xi).astype(np.float64))
    xf = rng.standard_normal((2, 13, 77, 2))
    V = oracle.xengine_cf64(xf)
    ii, jj = np.tril_indices(13)
    b = oracle.baseline_index(ii, jj)
    for c in range(2):
        X = xf[c, ..., 0] + 1j * xf[c, ..., 1]
        G = X @ X.conj().T
        np.testing.assert_allclose(V[c, b, 0] + 1j * V[c, b, 1], G[ii, jj], rtol=1e-12, atol=1e-12)
    d = oracle.baseline_index(np.arange(13), np.arange(13))
    assert np.all(V[:, d, 1] == 0.0)


def test_empty_time_axis():
    V = oracle.xengine_ci8(np.zeros((2, 4, 0, 2), np.int8))
    assert V.shape == (2, 10, 2) and not V.any()


@pytest.mark.parametrize("seed", [0, 1])
def test_longrun_fold_exact(seed):
    rng = np.random.default_rng(seed)
    dumps = [rng.integers(-(2 ** 31), 2 ** 31, size=(3, 10, 2), dtype=np.int64) for _ in range(10)]
    L = np.zeros((3, 10, 2))
    for d in dumps:
        oracle.fold(L, d)
    exact = sum(d.astype(object) for d in dumps)
    assert all(int(a) == b for a, b in zip(L.ravel(), exact.ravel()))


@pytest.mark.parametrize("seed", [0, 1])
def test_longrun_fold_f64_exact_dyadic(seed):
    """FP64 fold of float dumps (the FP32/FP16/FP8 engines' accumulators):
    dyadic values with at most 40 significant bits between 2^-20 and 2^20, so
    every partial sum of 10 is representable and the fold must equal the exact
    rational sum (Fig. 1: L += V after each read-out)."""
    from fractions import Fraction
    rng = np.random.default_rng(seed)
    dumps = [rng.integers(-(2 ** 40), 2 ** 40, size=(3, 10, 2)).astype(np.float64) * 2.0 ** -20
             for _ in range(10)]
    L = np.zeros((3, 10, 2))
    for d in dumps:
        oracle.fold(L, d)
    exact = [sum(Fraction(float(d.flat[k])) for d in dumps) for k in range(L.size)]
    assert all(Fraction(float(a)) == b for a, b in zip(L.ravel(), exact))


def test_longrun_fold_f64_rounds_each_step():
    """Each fold is one IEEE FP64 addition, rounded to nearest even: 1 + 2^-53
    is a tie that rounds back to 1, twice, although the exact sum 1 + 2^-52 is
    representable; and a fold of -L gives exactly +0."""
    L = np.array([1.0, 3.5])
    for _ in range(2):
        oracle.fold(L, np.array([2.0 ** -53, 0.0]))
    assert L[0] == 1.0
    oracle.fold(L, np.array([-1.0, -3.5]))
    assert L[0] == 0.0 and L[1] == 0.0 and not np.signbit(L[0])
    L = np.array([1.0])
    oracle.fold(L, np.array([3 * 2.0 ** -53]))                    # 1 + 1.5 ulp -> 1 + 2 ulp
    assert L[0] == 1.0 + 2.0 ** -51
