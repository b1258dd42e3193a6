"""CPU oracle for the FX correlator -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never loads it, and
it loads nothing from the GPU library: the two share no code.

The arithmetic lives in ``oracle.c`` (plain C99, int64 / FP64, built with
``-ffp-contract=off``); this module marshals numpy arrays to it.  See the
header of ``oracle.c`` for the passage of the paper each function follows.
Derived quantities that are plain arithmetic on oracle outputs (coherence,
average) are written here in numpy.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C99 + OpenMP, no FP contraction)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-std=c99", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.oracle_xengine_ci8.argtypes = [P, I64, I64, I64, P]
        lib.oracle_xengine_cf64.argtypes = [P, I64, I64, I64, P]
        lib.oracle_xengine_pairs_ci8.argtypes = [P, I64, I64, P, P, I64, P]
        lib.oracle_dft_real.argtypes = [P, I64, I64, I64, I64, P]
        lib.oracle_requant.argtypes = [P, I64, ctypes.c_double, ctypes.c_int32, P]
        lib.oracle_dft_complex.argtypes = [P, I64, I64, I64, P]
        lib.oracle_pfb_coeffs.argtypes = [I64, I64, P]
        lib.oracle_pfb_real.argtypes = [P, P, I64, I64, I64, I64, I64, P]
        lib.oracle_unpack_w16.argtypes = [P, I64, P]
        lib.oracle_unpack_b8.argtypes = [P, I64, P]
        lib.oracle_aggregate_w16.argtypes = [P, I64, I64, I64, ctypes.c_uint32, P]
        lib.oracle_aggregate_w16.restype = I64
        lib.oracle_f16_encode.argtypes = [P, I64, P]
        lib.oracle_f16_decode.argtypes = [P, I64, P]
        lib.oracle_e4m3_encode.argtypes = [P, I64, P]
        lib.oracle_e4m3_decode.argtypes = [P, I64, P]
        lib.oracle_e4m3_scale.argtypes = [P, I64]
        lib.oracle_e4m3_scale.restype = ctypes.c_double
        lib.oracle_fold_i64.argtypes = [P, P, I64]
        lib.oracle_fold_f64.argtypes = [P, P, I64]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def n_products(n_inputs: int) -> int:
    """Sec. 2: N_I(N_I-1)/2 crosses plus N_I autos."""
    return n_inputs * (n_inputs + 1) // 2


def baseline_index(i, j):
    """Packed lower-triangle index b(i, j) = i(i+1)/2 + j for j <= i."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    return i * (i + 1) // 2 + j


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    _load().oracle_set_num_threads(int(n))


# ------------------------------------------------------------------ X-engine
def xengine_ci8(x: np.ndarray) -> np.ndarray:
    """x: int8 [n_ch][n_in][T][2] -> int64 [n_ch][P][2] (exact)."""
    x = np.ascontiguousarray(x, dtype=np.int8)
    n_ch, n_in, T, two = x.shape
    assert two == 2
    V = np.zeros((n_ch, n_products(n_in), 2), dtype=np.int64)
    if V.size:
        _load().oracle_xengine_ci8(_ptr(x), n_ch, n_in, T, _ptr(V))
    return V


def xengine_cf64(x: np.ndarray) -> np.ndarray:
    """x: float [n_ch][n_in][T][2] (converted to FP64) -> FP64 [n_ch][P][2]."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n_ch, n_in, T, two = x.shape
    assert two == 2
    V = np.zeros((n_ch, n_products(n_in), 2), dtype=np.float64)
    if V.size:
        _load().oracle_xengine_cf64(_ptr(x), n_ch, n_in, T, _ptr(V))
    return V


def xengine_pairs_ci8(xc: np.ndarray, ii, jj) -> np.ndarray:
    """One channel xc int8 [n_in][T][2]; returns int64 [n][2] = V_{ii[k], jj[k]}."""
    xc = np.ascontiguousarray(xc, dtype=np.int8)
    n_in, T, _ = xc.shape
    ii = np.ascontiguousarray(ii, dtype=np.int32)
    jj = np.ascontiguousarray(jj, dtype=np.int32)
    assert ii.shape == jj.shape
    if ii.size and (ii.min() < 0 or jj.min() < 0 or ii.max() >= n_in or jj.max() >= n_in):
        raise IndexError("pair index out of range")
    out = np.zeros((ii.size, 2), dtype=np.int64)
    if ii.size:
        _load().oracle_xengine_pairs_ci8(_ptr(xc), n_in, T, _ptr(ii), _ptr(jj), ii.size, _ptr(out))
    return out


# ------------------------------------------------------------------- F-stage
def dft_real(v: np.ndarray, N: int, n_keep: int | None = None) -> np.ndarray:
    """v: int8 [n_blocks*N][n_in] time-major -> FP64 [n_keep][n_in][n_blocks][2]."""
    v = np.ascontiguousarray(v, dtype=np.int8)
    ns, n_in = v.shape
    assert ns % N == 0
    nb = ns // N
    n_keep = N // 2 if n_keep is None else n_keep
    X = np.zeros((n_keep, n_in, nb, 2), dtype=np.float64)
    if X.size:
        _load().oracle_dft_real(_ptr(v), N, n_in, nb, n_keep, _ptr(X))
    return X


def dft_complex(x: np.ndarray, N: int) -> np.ndarray:
    """x: int8 [n_blocks*N][n_in][2] complex, time-major -> FP64 [N][n_in][n_blocks][2]."""
    x = np.ascontiguousarray(x, dtype=np.int8)
    ns, n_in, two = x.shape
    assert two == 2 and ns % N == 0
    nb = ns // N
    X = np.zeros((N, n_in, nb, 2), dtype=np.float64)
    if X.size:
        _load().oracle_dft_complex(_ptr(x), N, n_in, nb, _ptr(X))
    return X


def pfb_coeffs(P: int, N: int) -> np.ndarray:
    """Prototype filter h[m], m < P*N: Hamming window times sinc((m - (PN-1)/2)/N)."""
    h = np.zeros(P * N, dtype=np.float64)
    _load().oracle_pfb_coeffs(P, N, _ptr(h))
    return h


def pfb_real(v: np.ndarray, N: int, P: int, h: np.ndarray | None = None, n_keep: int | None = None) -> np.ndarray:
    """v: int8 [(n_blocks + P - 1)*N][n_in] -> FP64 [n_keep][n_in][n_blocks][2]: the real DFT of
    y_b[n] = sum_p h[pN + n] v[(b + p)N + n] (h defaults to pfb_coeffs(P, N))."""
    v = np.ascontiguousarray(v, dtype=np.int8)
    ns, n_in = v.shape
    assert ns % N == 0 and ns // N >= P
    nb = ns // N - (P - 1)
    h = pfb_coeffs(P, N) if h is None else np.ascontiguousarray(h, dtype=np.float64)
    assert h.shape == (P * N,)
    n_keep = N // 2 if n_keep is None else n_keep
    X = np.zeros((n_keep, n_in, nb, 2), dtype=np.float64)
    if X.size:
        _load().oracle_pfb_real(_ptr(v), _ptr(h), N, P, n_in, nb, n_keep, _ptr(X))
    return X


def unpack_w16(w) -> np.ndarray:
    """uint16 words (5-bit re in bits 9..5, 5-bit im in bits 4..0) -> int8 [..., 2]."""
    w = np.ascontiguousarray(w, dtype=np.uint16)
    out = np.zeros(w.shape + (2,), dtype=np.int8)
    if w.size:
        _load().oracle_unpack_w16(_ptr(w), w.size, _ptr(out))
    return out


def unpack_b8(b) -> np.ndarray:
    """uint8 bytes (4-bit re in bits 7..4, 4-bit im in bits 3..0) -> int8 [..., 2]."""
    b = np.ascontiguousarray(b, dtype=np.uint8)
    out = np.zeros(b.shape + (2,), dtype=np.int8)
    if b.size:
        _load().oracle_unpack_b8(_ptr(b), b.size, _ptr(out))
    return out


def aggregate_w16(rec: np.ndarray, first_counter: int = 0):
    """rec: uint16 [n_streams][n_rec][1 + w_per] -> (uint16 [n_rec][n_streams * w_per], number
    of records whose marker/counter word is not first_counter + r (mod 2^16) in some stream)."""
    rec = np.ascontiguousarray(rec, dtype=np.uint16)
    ns, nr, wp1 = rec.shape
    out = np.zeros((nr, ns * (wp1 - 1)), dtype=np.uint16)
    bad = 0
    if rec.size:
        bad = int(_load().oracle_aggregate_w16(_ptr(rec), ns, wp1 - 1, nr, int(first_counter) & 0xFFFF, _ptr(out)))
    return out, bad


def requant(y: np.ndarray, s: float, max_abs: int = 7) -> np.ndarray:
    y = np.ascontiguousarray(y, dtype=np.float64)
    q = np.zeros(y.shape, dtype=np.int8)
    if y.size:
        _load().oracle_requant(_ptr(y), y.size, float(s), int(max_abs), _ptr(q))
    return q


# -------------------------------------------------------------------- codecs
def f16_encode(x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(x.shape, dtype=np.uint16)
    if x.size:
        _load().oracle_f16_encode(_ptr(x), x.size, _ptr(out))
    return out


def f16_decode(h) -> np.ndarray:
    h = np.ascontiguousarray(h, dtype=np.uint16)
    out = np.zeros(h.shape, dtype=np.float64)
    if h.size:
        _load().oracle_f16_decode(_ptr(h), h.size, _ptr(out))
    return out


def e4m3_encode(x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(x.shape, dtype=np.uint8)
    if x.size:
        _load().oracle_e4m3_encode(_ptr(x), x.size, _ptr(out))
    return out


def e4m3_decode(b) -> np.ndarray:
    b = np.ascontiguousarray(b, dtype=np.uint8)
    out = np.zeros(b.shape, dtype=np.float64)
    if b.size:
        _load().oracle_e4m3_decode(_ptr(b), b.size, _ptr(out))
    return out


def e4m3_scale(x) -> float:
    """Largest power of two s with s * max|x| <= 448 (1 if x is all zero)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    return float(_load().oracle_e4m3_scale(_ptr(x), x.size))


# ------------------------------------------------------------------ long-run
def fold(L: np.ndarray, V: np.ndarray) -> None:
    """L += V in FP64, in place (V int64 or FP64)."""
    assert L.dtype == np.float64 and L.flags.c_contiguous and L.shape == V.shape
    if V.dtype == np.int64:
        V = np.ascontiguousarray(V)
        _load().oracle_fold_i64(_ptr(L), _ptr(V), V.size)
    else:
        V = np.ascontiguousarray(V, dtype=np.float64)
        _load().oracle_fold_f64(_ptr(L), _ptr(V), V.size)


# ------------------------------------------------------------ derived checks
def coherence(V: np.ndarray, n_inputs: int, i, j, real_part: bool = False) -> np.ndarray:
    """rho_ij[c] = |V_ij| / sqrt(V_ii V_jj) per channel (or Re V_ij / ...)."""
    V = np.asarray(V, dtype=np.float64)
    b = baseline_index(max(i, j), min(i, j))
    vij = V[:, b, 0] + 1j * V[:, b, 1]
    if i < j:
        vij = np.conj(vij)
    vii = V[:, baseline_index(i, i), 0]
    vjj = V[:, baseline_index(j, j), 0]
    num = vij.real if real_part else np.abs(vij)
    return num / np.sqrt(vii * vjj)


def full_matrix(Vc: np.ndarray, n_inputs: int) -> np.ndarray:
    """Packed triangle of one channel [P][2] -> Hermitian N x N complex matrix."""
    M = np.zeros((n_inputs, n_inputs), dtype=np.complex128)
    ii, jj = np.tril_indices(n_inputs)
    b = baseline_index(ii, jj)
    v = Vc[b, 0].astype(np.float64) + 1j * Vc[b, 1].astype(np.float64)
    M[ii, jj] = v
    M[jj, ii] = np.conj(v)
    return M
