"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module holds no correlator arithmetic: it only draws the test
signals.  Everything here is a *generator*; the oracle (``oracle/``) and the
HIP library (``paper_0906_1887_amd``) both consume its outputs, neither is
imported from here.

Signals (all seeded, all reproducible):

* ``ci8``  -- complex 4-bit-range samples, re and im i.i.d. draws of
  ``clip(round(sigma*z), -7, 7)`` with ``z ~ N(0,1)`` (clip, not resample).
  Drawn by a counter-based generator so that the host (numpy, below) and
  the device (``synth_dev.hip``) produce bit-identical values for any
  (seed, channel, input, t): a SplitMix64 finaliser (Steele, Lea & Flood,
  OOPSLA 2014) hashes the counter, and each 32-bit half is mapped to a level
  by comparing it against cumulative-probability thresholds that are
  computed once here in FP64.  No libm call is involved on either side.
* ``real_voltages`` -- real 8-bit voltage streams with a common tone and
  correlated noise on a subset of inputs (numpy PCG64, host only; the GPU
  reads the uploaded array).
* ``complex_float`` -- complex Gaussian float inputs with per-input gains
  and coherent pairs (numpy PCG64, host only, uploaded).
* ``capture_records`` / ``complex_bytes`` -- the prototype's recorded
  complex samples: Gaussian noise with a correlated component on a subset of
  inputs and a complex tone, rounded and clipped to 5-bit (or 4-bit) two's
  complement and packed as 16-bit words in marker-led records (or bytes)
  (numpy PCG64, host only, uploaded).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

__all__ = [
    "GOLDEN_GAMMA",
    "level_thresholds",
    "level_probabilities",
    "mix64",
    "counter",
    "ci8",
    "ci8_channel",
    "ci8_channel_numpy",
    "ci8_block",
    "real_voltages",
    "complex_float",
    "coherent_pairs",
    "DeviceGen",
]

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Counter layout: channel in bits 44..63, input in bits 24..43, t in 0..23.
CH_BITS, IN_BITS, T_BITS = 20, 20, 24


def _phi(x: float) -> float:
    return 0.5 * math.erfc(-x / math.sqrt(2.0))


def level_thresholds(sigma: float = 2.0, max_abs: int = 7) -> np.ndarray:
    """uint32 thresholds t[m], m = 0 .. 2*max_abs-1.

    A uniform 32-bit word u maps to level ``-max_abs + #{m : u >= t[m]}``.
    t[m] = floor(2^32 * Phi((m - max_abs + 0.5) / sigma)): the boundary
    between levels k and k+1 of ``round(sigma*z)`` sits at z = (k+0.5)/sigma,
    and every tail beyond +-max_abs is folded onto the end level (clip).
    """
    n = 2 * max_abs
    t = np.empty(n, dtype=np.uint32)
    for m in range(n):
        p = _phi((m - max_abs + 0.5) / sigma)
        t[m] = min(int(math.floor(p * 4294967296.0)), 0xFFFFFFFF)
    return t


def level_probabilities(sigma: float = 2.0, max_abs: int = 7) -> np.ndarray:
    """Exact FP64 probabilities of the clipped rounded Gaussian levels."""
    k = np.arange(-max_abs, max_abs + 1)
    p = np.empty(k.size)
    for idx, kk in enumerate(k):
        lo = -math.inf if kk == -max_abs else (kk - 0.5) / sigma
        hi = math.inf if kk == max_abs else (kk + 0.5) / sigma
        p[idx] = (_phi(hi) if hi != math.inf else 1.0) - (_phi(lo) if lo != -math.inf else 0.0)
    return p


def mix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output finaliser on uint64 (wrapping arithmetic)."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x ^ (x >> np.uint64(30))
        z = z * _M1
        z = z ^ (z >> np.uint64(27))
        z = z * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def counter(ch, inp, t) -> np.ndarray:
    ch = np.asarray(ch, dtype=np.uint64)
    inp = np.asarray(inp, dtype=np.uint64)
    t = np.asarray(t, dtype=np.uint64)
    return (ch << np.uint64(IN_BITS + T_BITS)) | (inp << np.uint64(T_BITS)) | t


def _hash(seed: int, c: np.ndarray) -> np.ndarray:
    key = mix64(np.uint64(seed & 0xFFFFFFFFFFFFFFFF))
    with np.errstate(over="ignore"):
        return mix64(key + c * GOLDEN_GAMMA)


def _levels(u32: np.ndarray, thr: np.ndarray, max_abs: int) -> np.ndarray:
    # count of thresholds <= u, as int8
    lv = np.searchsorted(thr, u32, side="right").astype(np.int16) - max_abs
    return lv.astype(np.int8)


def ci8_channel_numpy(seed: int, ch: int, n_inputs: int, n_samples: int,
                      sigma: float = 2.0, max_abs: int = 7, t0: int = 0,
                      inputs=None) -> np.ndarray:
    """numpy form of ``ci8_channel`` (slow; the reference the C twin is tested against)."""
    if n_samples + t0 > (1 << T_BITS) or ch >= (1 << CH_BITS) or n_inputs > (1 << IN_BITS):
        raise ValueError("counter field overflow")
    thr = level_thresholds(sigma, max_abs)
    rows = np.arange(n_inputs) if inputs is None else np.asarray(inputs)
    t = np.arange(t0, t0 + n_samples, dtype=np.uint64)
    c = counter(ch, rows[:, None], t[None, :])
    h = _hash(seed, c)
    out = np.empty((rows.size, n_samples, 2), dtype=np.int8)
    out[..., 0] = _levels((h & np.uint64(0xFFFFFFFF)).astype(np.uint32), thr, max_abs)
    out[..., 1] = _levels((h >> np.uint64(32)).astype(np.uint32), thr, max_abs)
    return out


_host = None
HOST_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsynth_host.so")
HOST_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "synth_host.c")


def build_host() -> str:
    import subprocess
    tmp = HOST_LIB + ".tmp"
    subprocess.run(["gcc", "-std=c99", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, HOST_SRC], check=True)
    os.replace(tmp, HOST_LIB)
    return HOST_LIB


def _host_lib():
    global _host
    if _host is None:
        if not os.path.exists(HOST_LIB):
            build_host()
        L = ctypes.CDLL(HOST_LIB)
        P, I64 = ctypes.c_void_p, ctypes.c_int64
        L.synth_ci8_host.argtypes = [P, I64, I64, P, I64, I64, I64, ctypes.c_uint64, P, ctypes.c_int, ctypes.c_int]
        L.synth_ci8_host.restype = None
        _host = L
    return _host


def ci8_block(seed: int, ch0: int, n_channels: int, n_inputs: int, n_samples: int,
              sigma: float = 2.0, max_abs: int = 7, t0: int = 0, inputs=None) -> np.ndarray:
    """Channels ch0 .. ch0+n_channels-1: int8 [n_channels][rows][n_samples][2]
    (rows = all n_inputs, or the selected ``inputs``), by the C twin."""
    if n_samples + t0 > (1 << T_BITS) or ch0 + n_channels > (1 << CH_BITS) or n_inputs > (1 << IN_BITS):
        raise ValueError("counter field overflow")
    thr = level_thresholds(sigma, max_abs)
    rows = None if inputs is None else np.ascontiguousarray(inputs, dtype=np.int32)
    n_rows = n_inputs if rows is None else rows.size
    out = np.empty((n_channels, n_rows, n_samples, 2), dtype=np.int8)
    if out.size:
        _host_lib().synth_ci8_host(out.ctypes.data, ch0, n_channels,
                                   None if rows is None else rows.ctypes.data, n_rows, t0, n_samples,
                                   seed & 0xFFFFFFFFFFFFFFFF, thr.ctypes.data, thr.size, max_abs)
    return out


def ci8_channel(seed: int, ch: int, n_inputs: int, n_samples: int,
                sigma: float = 2.0, max_abs: int = 7, t0: int = 0,
                inputs=None) -> np.ndarray:
    """One channel of ``ci8``: int8 array [n_inputs][n_samples][2] (re, im).

    ``inputs`` optionally selects a subset of input indices (the row order
    of the result follows it)."""
    return ci8_block(seed, ch, 1, n_inputs, n_samples, sigma, max_abs, t0, inputs)[0]


def ci8(seed: int, n_channels: int, n_inputs: int, n_samples: int,
        sigma: float = 2.0, max_abs: int = 7) -> np.ndarray:
    """All channels: int8 [n_channels][n_inputs][n_samples][2]."""
    return ci8_block(seed, 0, n_channels, n_inputs, n_samples, sigma, max_abs)


# ---------------------------------------------------------------------------
# Real 8-bit voltages: Gaussian noise of rms ``sigma`` per input, a fraction
# ``rho`` of the noise *power* common to inputs 0..n_corr-1, and a tone of
# amplitude ``tone_amp`` at ``tone_bin`` cycles per ``fft_size`` samples with
# phase 0, common to all inputs; rounded half-to-even and clipped to int8.
# ---------------------------------------------------------------------------
def real_voltages(seed: int, index: int, n_blocks: int, n_inputs: int = 64,
                  fft_size: int = 256, sigma: float = 16.0, rho: float = 0.1,
                  n_corr: int = 8, tone_bin: int = 37, tone_amp: float = 2.0,
                  chunk_blocks: int = 2048) -> np.ndarray:
    """int8 [n_blocks*fft_size][n_inputs], time-major (input fastest).

    ``index`` selects an independent stretch of data (e.g. one integration).
    """
    rng = np.random.default_rng([seed, index])
    out = np.empty((n_blocks * fft_size, n_inputs), dtype=np.int8)
    tone = tone_amp * np.cos(2.0 * np.pi * ((tone_bin * np.arange(fft_size)) % fft_size) / fft_size)
    a = np.ones(n_inputs)
    b = np.zeros(n_inputs)
    a[:n_corr] = math.sqrt(1.0 - rho)
    b[:n_corr] = math.sqrt(rho)
    for b0 in range(0, n_blocks, chunk_blocks):
        nb = min(chunk_blocks, n_blocks - b0)
        ns = nb * fft_size
        n = rng.standard_normal((ns, n_inputs))
        c = rng.standard_normal((ns, 1))
        v = sigma * (a[None, :] * n + b[None, :] * c)
        v += np.tile(tone, nb)[:, None]
        out[b0 * fft_size:b0 * fft_size + ns] = np.clip(np.rint(v), -128, 127).astype(np.int8)
    return out


# ---------------------------------------------------------------------------
# Complex Gaussian float inputs with per-input gains and coherent pairs.
# ---------------------------------------------------------------------------
def coherent_pairs(seed: int, n_inputs: int, n_pairs: int = 16):
    """n_pairs disjoint input pairs from a seeded permutation (fewer when
    n_inputs < 2 n_pairs)."""
    n_pairs = min(n_pairs, n_inputs // 2)
    rng = np.random.default_rng([seed, 0x9A15])
    perm = rng.permutation(n_inputs)[: 2 * n_pairs]
    return [(int(perm[2 * k]), int(perm[2 * k + 1])) for k in range(n_pairs)]


def input_gains(seed: int, n_inputs: int, lo: float = 0.5, hi: float = 2.0) -> np.ndarray:
    rng = np.random.default_rng([seed, 0x6A1])
    return rng.uniform(lo, hi, size=n_inputs)


def complex_float(seed: int, ch: int, n_inputs: int, n_samples: int,
                  rho: float = 0.1, n_pairs: int = 16) -> np.ndarray:
    """One channel, float32 [n_inputs][n_samples][2]: x = g*(sqrt(1-rho) n + sqrt(rho) c)
    on each coherent pair (c common to the pair), x = g*n elsewhere; n, c ~ CN(0,1)
    (independent N(0, 1/2) real and imaginary parts)."""
    g = input_gains(seed, n_inputs).astype(np.float32)
    pairs = coherent_pairs(seed, n_inputs, n_pairs)
    rng = np.random.default_rng([seed, 1, ch])
    s = np.float32(math.sqrt(0.5))
    x = rng.standard_normal((n_inputs, n_samples, 2), dtype=np.float32)
    x *= s
    c = rng.standard_normal((len(pairs), n_samples, 2), dtype=np.float32)
    c *= s
    a = np.float32(math.sqrt(1.0 - rho))
    b = np.float32(math.sqrt(rho))
    for k, (i, j) in enumerate(pairs):
        x[i] = a * x[i] + b * c[k]
        x[j] = a * x[j] + b * c[k]
    x *= g[:, None, None]
    return x


# ---------------------------------------------------------------------------
# Device generator (HIP), bit-identical to ``ci8_channel``.
# ---------------------------------------------------------------------------
_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsynth.so")


def build() -> str:
    """Compile libsynth.so (the device generator) for gfx950 with hipcc."""
    import subprocess
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-x", "hip", os.path.join(_HERE, "synth_dev.hip"), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for synth_dev.hip:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Thr(ctypes.Structure):
    _fields_ = [("t", ctypes.c_uint32 * 16), ("n", ctypes.c_int32), ("max_abs", ctypes.c_int32)]


class _JobFill(ctypes.Structure):
    _fields_ = [("base_seed", ctypes.c_uint64), ("th", _Thr)]


class DeviceGen:
    """ctypes wrapper of ``synth_fill_ci8`` (``libsynth.so``)."""

    def __init__(self, path: str = LIB_PATH):
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
        self.lib = ctypes.CDLL(path)
        self.lib.synth_fill_ci8.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_int64, ctypes.c_uint64, ctypes.POINTER(_Thr), ctypes.c_void_p]
        self.lib.synth_fill_ci8.restype = ctypes.c_int

    def job_fill(self, base_seed: int, sigma: float = 2.0, max_abs: int = 7):
        """(function pointer, user pointer, keep-alive) for a serving-scheduler
        fill callback: job j gets the ci8 signal of seed base_seed + j."""
        thr = level_thresholds(sigma, max_abs)
        jf = _JobFill()
        jf.base_seed = base_seed
        for i, v in enumerate(thr):
            jf.th.t[i] = int(v)
        jf.th.n = thr.size
        jf.th.max_abs = max_abs
        fn = ctypes.cast(self.lib.synth_fill_job, ctypes.c_void_p).value
        return fn, ctypes.addressof(jf), jf

    def fill_ci8(self, d_ptr: int, n_channels: int, n_inputs: int, n_samples: int,
                 seed: int, sigma: float = 2.0, max_abs: int = 7, stream: int = 0,
                 ch0: int = 0, row_stride: int | None = None) -> None:
        """Write int8 [n_channels][n_inputs][row_stride samples][2] at ``d_ptr``
        (channels ch0 .. ch0+n_channels-1); ``row_stride`` defaults to n_samples."""
        thr = level_thresholds(sigma, max_abs)
        s = _Thr()
        for i, v in enumerate(thr):
            s.t[i] = int(v)
        s.n = thr.size
        s.max_abs = max_abs
        rs = n_samples if row_stride is None else row_stride
        rc = self.lib.synth_fill_ci8(ctypes.c_void_p(d_ptr), ch0, n_channels, n_inputs, n_samples, rs,
                                     seed & 0xFFFFFFFFFFFFFFFF, ctypes.byref(s), ctypes.c_void_p(stream))
        if rc != 0:
            raise RuntimeError(f"synth_fill_ci8 failed ({rc})")


# ---------------------------------------------------------------------------
# The prototype's recorded complex samples (5+5-bit words in records; 4+4-bit
# bytes).  Field layout: re in the upper field, im in the lower field, two's
# complement; words carry arbitrary bits above bit 9.
# ---------------------------------------------------------------------------
def complex_levels(seed: int, index: int, n_samples: int, n_inputs: int, bits: int = 5,
                   sigma: float = 4.0, rho: float = 0.1, n_corr: int = 8, tone_bin: int = 19,
                   tone_amp: float = 1.5, fft_size: int = 128) -> np.ndarray:
    """int8 [n_samples][n_inputs][2] (re, im) levels in [-2^(bits-1), 2^(bits-1)-1]:
    rint(sigma*(a n + b c) + tone), n, c ~ CN(0, 1) per part, c common to inputs
    0..n_corr-1 (a = sqrt(1-rho), b = sqrt(rho) there), the tone
    tone_amp*exp(2 pi i tone_bin t / fft_size) on every input."""
    rng = np.random.default_rng([seed, index, bits])
    lo, hi = -(1 << (bits - 1)), (1 << (bits - 1)) - 1
    a = np.ones(n_inputs)
    b = np.zeros(n_inputs)
    a[:n_corr] = math.sqrt(1.0 - rho)
    b[:n_corr] = math.sqrt(rho)
    n = rng.standard_normal((n_samples, n_inputs, 2)) * math.sqrt(0.5)
    c = rng.standard_normal((n_samples, 1, 2)) * math.sqrt(0.5)
    v = sigma * (a[None, :, None] * n + b[None, :, None] * c)
    ph = 2.0 * np.pi * ((tone_bin * np.arange(n_samples)) % fft_size) / fft_size
    v[..., 0] += tone_amp * np.cos(ph)[:, None]
    v[..., 1] += tone_amp * np.sin(ph)[:, None]
    return np.clip(np.rint(v), lo, hi).astype(np.int8)


def capture_records(seed: int, index: int, n_records: int, n_streams: int = 4, w_per: int = 16,
                    first_counter: int = 0, **kw):
    """(records uint16 [n_streams][n_records][1 + w_per], levels int8 [n_records][n_streams*w_per][2]).
    Word 0 of record r is (first_counter + r) mod 2^16; data words pack the 5-bit
    levels as (re & 31) << 5 | (im & 31) with random bits 15..10."""
    lv = complex_levels(seed, index, n_records, n_streams * w_per, bits=5, **kw)
    rng = np.random.default_rng([seed, index, 0xC0FFEE])
    junk = rng.integers(0, 64, size=(n_records, n_streams * w_per)).astype(np.uint16) << 10
    words = (((lv[..., 0].astype(np.int64) & 31) << 5) | (lv[..., 1].astype(np.int64) & 31)).astype(np.uint16)
    words |= junk
    rec = np.empty((n_streams, n_records, 1 + w_per), dtype=np.uint16)
    rec[:, :, 0] = ((first_counter + np.arange(n_records)) & 0xFFFF).astype(np.uint16)[None, :]
    rec[:, :, 1:] = words.reshape(n_records, n_streams, w_per).transpose(1, 0, 2)
    return rec, lv


def complex_bytes(seed: int, index: int, n_samples: int, n_inputs: int, **kw):
    """(bytes uint8 [n_samples][n_inputs], levels int8 [n_samples][n_inputs][2]): 4-bit
    levels packed as (re & 15) << 4 | (im & 15)."""
    kw.setdefault("sigma", 2.0)
    lv = complex_levels(seed, index, n_samples, n_inputs, bits=4, **kw)
    b = (((lv[..., 0].astype(np.int64) & 15) << 4) | (lv[..., 1].astype(np.int64) & 15)).astype(np.uint8)
    return b, lv


def real_tone(seed: int, n_samples: int, n_inputs: int, bin_pos: float, amp: float = 60.0,
              sigma: float = 1.0, fft_size: int = 256) -> np.ndarray:
    """int8 [n_samples][n_inputs]: rint(amp cos(2 pi bin_pos t / fft_size) + sigma n), a tone
    continuous across blocks (any bin position, also between channel centres) over
    Gaussian noise (numpy PCG64)."""
    rng = np.random.default_rng([seed, 0x70E])
    t = np.arange(n_samples, dtype=np.float64)
    v = amp * np.cos(2.0 * np.pi * bin_pos * t / fft_size)[:, None] + sigma * rng.standard_normal((n_samples, n_inputs))
    return np.clip(np.rint(v), -128, 127).astype(np.int8)
