"""Shared F-stage parity check (imported by the GPU tests; not a test module).

The GPU transforms in FP32 and the oracle in FP64, so a value that lies within
the FFT's rounding error of a .5 boundary may be requantised either way.  The
check, for every spectrum value:

(i)   |X_gpu - X_oracle| is at most the a-priori rounding-error bound of an
      FP32 FFT (below), and at most 1e-5 of the channel RMS;
(ii)  a requantised code may differ from the oracle's only where the oracle's
      scaled value lies within delta = 2 s max|X_gpu - X_oracle| of a .5
      boundary, and delta itself is below 2 s times the a-priori bound;
(iii) the mismatch fraction is printed and must stay below the fraction of
      values a uniform density would put inside the a-priori tie band
      (2 x 2 s x bound), with a factor 2 of margin.

A-priori bound.  For a radix-2 FFT of length N computed in floating point with
unit roundoff u and twiddle factors accurate to mu, Higham (Accuracy and
Stability of Numerical Algorithms, 2nd ed., Thm 24.2) gives
    ||y_hat - y||_2 <= ||y||_2 * L eta / (1 - L eta),   L = log2 N,
    eta = mu + gamma_4 (sqrt(2) + mu),   gamma_k = k u / (1 - k u),
and ||y||_2 = sqrt(N) ||x||_2, so every single output is within that bound.
Here u = 2^-24 (FP32), mu = u (twiddles rounded once from FP64).  The kernels
use radix-4/16 butterflies and, on real input, transform two inputs as one
complex sequence (||z|| <= sqrt(2) max ||x||) followed by the split
(Z_k +- conj Z_{N-k}) / 2; the bound is doubled to cover both.  A polyphase
filterbank adds the error of its weighted sum of P blocks, computed in FP32
with FP32 coefficients: each input sample is off by at most
(gamma_P + u) sum_p |h_p x_p|, which the DFT carries into one output by at most
sqrt(N) times its 2-norm over the block.
"""
from __future__ import annotations

import math
import sys

import numpy as np

import oracle

U32 = 2.0 ** -24


def gamma(k: int) -> float:
    return k * U32 / (1.0 - k * U32)


def fft_bound(N: int, max_norm2: float) -> float:
    """Doubled Higham bound on one FFT output, input 2-norm max_norm2."""
    L = math.log2(N)
    eta = U32 + gamma(4) * (math.sqrt(2.0) + U32)
    return 2.0 * math.sqrt(N) * max_norm2 * L * eta / (1.0 - L * eta)


def real_bound(v: np.ndarray, N: int) -> float:
    """v: int8 [n_blocks*N][n_in] time-major; two inputs per complex FFT."""
    nb = v.shape[0] // N
    blocks = v[: nb * N].astype(np.float64).reshape(nb, N, -1)
    norm = float(np.sqrt((blocks ** 2).sum(axis=1)).max()) if blocks.size else 0.0
    return fft_bound(N, math.sqrt(2.0) * norm)


def complex_bound(levels: np.ndarray, N: int) -> float:
    """levels: int8 [n_blocks*N][n_in][2] complex, time-major; one input per FFT."""
    nb = levels.shape[0] // N
    blocks = levels[: nb * N].astype(np.float64).reshape(nb, N, levels.shape[1], 2)
    norm = float(np.sqrt((blocks ** 2).sum(axis=(1, 3))).max()) if blocks.size else 0.0
    return fft_bound(N, norm)


def pfb_bound(v: np.ndarray, N: int, P: int) -> float:
    """v: int8 [(n_blocks+P-1)*N][n_in]; spectrum b transforms
    y_b[n] = sum_p h[pN+n] v[(b+p)N+n]."""
    h = oracle.pfb_coeffs(P, N)
    nb = v.shape[0] // N - (P - 1)
    x = v[: (nb + P - 1) * N].astype(np.float64).reshape(nb + P - 1, N, -1)
    habs = np.zeros((nb, N, x.shape[2]))
    for p in range(P):
        habs += np.abs(h[p * N:(p + 1) * N])[None, :, None] * np.abs(x[p:p + nb])
    s_norm = float(np.sqrt((habs ** 2).sum(axis=1)).max()) if habs.size else 0.0
    # ||y|| <= ||sum |h x| ||; the input error is (gamma_P + u) sum |h x| per sample
    return fft_bound(N, math.sqrt(2.0) * s_norm) + math.sqrt(N) * math.sqrt(2.0) * (gamma(P) + U32) * s_norm


def check_spectra_requant(X: np.ndarray, dbg: np.ndarray, q_gpu: np.ndarray, s: float, max_abs: int,
                          bound: float, label: str = "") -> dict:
    """X: oracle FP64 spectra; dbg: GPU FP32 spectra (same shape); q_gpu: GPU
    codes.  Asserts (i)-(iii) of the module docstring; returns the figures."""
    Xg = dbg.astype(np.float64)
    rms = float(np.sqrt(np.mean(X ** 2)))
    err = float(np.abs(Xg - X).max()) if X.size else 0.0
    assert err <= 1e-5 * rms, (label, err / rms)
    assert err <= bound, (label, err, bound)
    q_or = oracle.requant(X, s, max_abs)
    y = s * X
    delta = 2.0 * s * err
    assert delta <= 2.0 * s * bound
    tie = np.abs(y - np.floor(y) - 0.5) < delta
    mism = q_or != q_gpu
    outside = int(np.sum(mism & ~tie))
    assert outside == 0, (label, outside)
    frac = float(mism.mean()) if mism.size else 0.0
    allowed = 2.0 * (2.0 * 2.0 * s * bound)
    print(f"    {label} spectra err {err:.3e} = {err / bound:.3f} of the a-priori bound {bound:.3e}; "
          f"requant mismatches {int(mism.sum())} of {mism.size} ({frac:.2e}, allowed {allowed:.2e})", flush=True)
    sys.stdout.flush()
    assert frac <= allowed, (label, frac, allowed)
    return {"err": err, "bound": bound, "mismatch_frac": frac}
