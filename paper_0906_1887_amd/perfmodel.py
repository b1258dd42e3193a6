"""Work, traffic and roofline arithmetic of the X-engine and F-stage.

Pure arithmetic, no device code.  The memory-bound model is the one of
Sec. 6 of Wayth, Greenhill & Briggs (2009): at signal bandwidth B the
X-engine must do B N_I(N_I+1)/2 complex multiply-accumulates (CMAC) per
second and, with eps global reads per channel per product of single-precision
complex samples (8 bytes), fetch eps * 4 B N_I(N_I+1) bytes per second; a
memory throughput M therefore caps the bandwidth at M / (4 eps N_I (N_I+1)).
The eps values of the paper's five designs (pair parallel, hybrid group and
group parallel with G = 2 or 4) are in ``PAPER_EPS``.
"""
from __future__ import annotations

# Sec. 6: global reads per channel per product for each design.
PAPER_EPS = {"PP": 2.0, "HG2": 1.5, "HG4": 1.25, "GP2": 1.0, "GP4": 0.5}

# MI355X published peaks (dense).
MI355X = {
    "cus": 256,
    "clock_hz": 2.4e9,
    "hbm_Bps": 8.0e12,
    "int8_ops": 5.0e15,      # dense int8 MFMA, ops/s (1 MAC = 2 ops)
    "fp8_flops": 5.0e15,
    "fp16_flops": 2.5e15,
    "fp32_vec_flops": 157.3e12,  # published vector FP32 rate
    "fp64_vec_flops": 78.6e12,
}

REAL_MACS_PER_CMAC = 4
FLOPS_PER_CMAC = 8


def n_products(n_inputs: int) -> int:
    """Sec. 2: N_I(N_I-1)/2 cross products plus N_I autos."""
    return n_inputs * (n_inputs + 1) // 2


def realtime_cmac_rate(bandwidth_hz: float, n_inputs: int) -> float:
    """CMAC per second needed in real time: B N_I (N_I+1) / 2 (Sec. 6)."""
    return bandwidth_hz * n_inputs * (n_inputs + 1) / 2.0


def global_read_rate(eps: float, bandwidth_hz: float, n_inputs: int,
                     bytes_per_sample: float = 8.0) -> float:
    """Bytes per second fetched: eps * (bytes_per_sample/2) * B * N_I (N_I+1).

    With 8-byte complex floats this is the paper's eps * 4 B N_I (N_I+1)."""
    return eps * (bytes_per_sample / 2.0) * bandwidth_hz * n_inputs * (n_inputs + 1)


def max_signal_bandwidth(mem_Bps: float, eps: float, n_inputs: int,
                         bytes_per_sample: float = 8.0) -> float:
    """Largest signal bandwidth (Hz) a memory throughput can feed (Sec. 6)."""
    return mem_Bps / (eps * (bytes_per_sample / 2.0) * n_inputs * (n_inputs + 1))


# --------------------------------------------------------------- this build
def xengine_cmac(n_channels: int, n_inputs: int, n_samples: int) -> int:
    """Useful CMAC of one integration: channels x products x samples."""
    return n_channels * n_products(n_inputs) * n_samples


def xengine_bytes(n_channels: int, n_inputs: int, n_samples: int,
                  bytes_per_sample: int, bytes_per_product: int,
                  accumulate: bool = False) -> int:
    """Algorithmic HBM bytes of one X-engine pass: every sample read once
    plus the packed triangle written once (read too when accumulating)."""
    inp = n_channels * n_inputs * n_samples * bytes_per_sample
    out = n_channels * n_products(n_inputs) * bytes_per_product
    return inp + out * (2 if accumulate else 1)


def eps_of_one_pass(n_inputs: int) -> float:
    """Reading every sample exactly once is eps = 2/(N_I+1) in the paper's
    terms (2 N_I reads spread over N_I(N_I+1)/2 products)."""
    return 2.0 / (n_inputs + 1)


def fstage_bytes(n_inputs: int, n_blocks: int, fft_size: int, out_bytes_per_sample: int = 2,
                 n_keep: int | None = None) -> int:
    """F-stage HBM bytes: int8 voltages in, n_keep channels of requantised
    complex samples out (int8 pairs)."""
    keep = fft_size // 2 if n_keep is None else n_keep
    return n_inputs * n_blocks * fft_size + keep * n_inputs * n_blocks * out_bytes_per_sample


def int8_cmac_peak() -> float:
    """Dense int8 MFMA ceiling in CMAC/s (4 real MACs per CMAC, 2 ops per MAC)."""
    return MI355X["int8_ops"] / 2.0 / REAL_MACS_PER_CMAC


def fp32_cmac_peak() -> float:
    """Vector FP32 ceiling in CMAC/s (MI355X's published 157.3 TFLOP/s, 8 flops
    per CMAC).  gfx950 reaches more than half of it with plain v_fma_f32, so no
    separate packed / unpacked figure is kept."""
    return MI355X["fp32_vec_flops"] / FLOPS_PER_CMAC
