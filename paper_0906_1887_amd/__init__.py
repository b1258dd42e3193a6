"""FX correlator for AMD MI355X (gfx950): Python front of libcorr.

``_lib`` mirrors the C ABI of ``include/corr.h`` name for name.
``Correlator`` wraps one plan, using torch only for device memory (the
workspace, output buffers) and the current HIP stream; all correlator work
runs in libcorr's kernels.
"""
from __future__ import annotations

from . import _lib
from ._lib import (CORR_CF32, CORR_CI4, CORR_CI8, CORR_DUMP_FOLD, CORR_DUMP_INTEG, CORR_DUMP_LONGRUN,
                   CORR_DUMP_NO_RESET, CORR_X_F8, CORR_X_F16, CORR_X_FP32, CORR_X_FP32M, CORR_X_I8, CorrError,
                   corr_aggregate_w16, corr_channelise, corr_cmac_design, corr_config, corr_correlate, corr_create, corr_destroy, corr_dump,
                   corr_dump_bytes, corr_job_desc, corr_ring_read, corr_sched_create, corr_sched_destroy,
                   corr_restore, corr_sched_now, corr_sched_poll, corr_sched_stats, corr_sched_submit,
                   corr_seq_reset, corr_stage_read, corr_state, corr_status_str, corr_workspace_bytes)

__all__ = [
    "Correlator", "CorrError", "corr_config", "corr_workspace_bytes", "corr_create", "corr_destroy",
    "corr_channelise", "corr_seq_reset", "corr_correlate", "corr_dump", "corr_ring_read", "corr_stage_read",
    "corr_dump_bytes", "corr_job_desc", "corr_sched_now", "corr_sched_create", "corr_sched_submit",
    "corr_sched_poll", "corr_sched_stats", "corr_sched_destroy", "Scheduler",
    "corr_status_str", "ENGINES", "SAMPLE_TYPES", "VOLT_FORMATS", "corr_aggregate_w16", "aggregate_w16",
    "corr_cmac_design", "cmac_design", "DESIGNS", "corr_state", "corr_restore",
]

ENGINES = {"fp32": CORR_X_FP32, "i8": CORR_X_I8, "f16": CORR_X_F16, "f8": CORR_X_F8, "fp32m": CORR_X_FP32M}
SAMPLE_TYPES = {"cf32": CORR_CF32, "ci8": CORR_CI8, "ci4": CORR_CI4}
# F-stage input formats: real int8; complex 5+5-bit in 16-bit words; complex 4+4-bit bytes
VOLT_FORMATS = {"r8": 0, "cw16": 1, "cb8": 2}


def make_config(n_inputs: int, n_channels: int, engine: str = "i8", sample_type: str = "ci8",
                fft_size: int = 0, max_abs: int = 7, requant_scale: float = 0.0,
                ring_samples: int = 0, fp64_longrun: bool = False, volt_format: str = "r8",
                pfb_taps: int = 0) -> corr_config:
    c = corr_config()
    c.n_inputs = n_inputs
    c.n_channels = n_channels
    c.fft_size = fft_size
    c.sample_type = SAMPLE_TYPES[sample_type]
    c.engine = ENGINES[engine]
    c.max_abs = max_abs
    c.requant_scale = requant_scale
    c.fp64_longrun = int(bool(fp64_longrun))
    c.ring_samples = ring_samples
    c.volt_format = VOLT_FORMATS[volt_format]
    c.pfb_taps = pfb_taps
    return c


def aggregate_w16(records, first_counter: int = 0, out=None, bad=None):
    """Drop the marker words of capture-stream records and interleave the
    streams (the aggregation of Sec. 3), on the records' device and current
    stream.  records: uint16/int16 device tensor [n_streams][n_records][1 + w].
    Returns (out [n_records][n_streams * w] of the same dtype, bad: uint32 device
    tensor [1] counting records whose marker/counter word is not first_counter + r
    mod 2^16 in some stream; accumulates into a given ``bad``)."""
    import torch

    assert records.dim() == 3 and records.is_contiguous() and records.element_size() == 2
    ns, nr, wp1 = records.shape
    if out is None:
        out = torch.empty((nr, ns * (wp1 - 1)), dtype=records.dtype, device=records.device)
    if bad is None:
        bad = torch.zeros(1, dtype=torch.uint32, device=records.device)
    stream = torch.cuda.current_stream(records.device).cuda_stream
    corr_aggregate_w16(records.data_ptr(), ns, wp1 - 1, nr, first_counter, out.data_ptr(), bad.data_ptr(), stream)
    return out, bad


# The paper's CMAC designs: name -> (corr_design_t, group G)
DESIGNS = {"pp": (0, 1), "gp2": (1, 2), "gp4": (1, 4), "hg2": (2, 2), "hg4": (2, 4)}


def cmac_design(name: str, spectra, out=None, accumulate: bool = False):
    """Run one of the paper's CMAC designs on complex float32 spectra laid out
    [n_samples][n_inputs][n_channels][2] (a float32 device tensor), on the
    current stream.  Returns out [n_channels][P][2] float32."""
    import torch

    design, group = DESIGNS[name]
    assert spectra.dtype == torch.float32 and spectra.is_contiguous() and spectra.shape[-1] == 2
    T, n_in, n_ch, _ = spectra.shape
    P = n_in * (n_in + 1) // 2
    if out is None:
        out = torch.zeros((n_ch, P, 2), dtype=torch.float32, device=spectra.device)
    stream = torch.cuda.current_stream(spectra.device).cuda_stream
    corr_cmac_design(design, group, spectra.data_ptr(), T, n_in, n_ch, out.data_ptr(), accumulate, stream)
    return out


class Correlator:
    """One correlator plan on one device.

    Output of ``dump()``: a tensor [n_channels][P][2] (P = n_inputs(n_inputs+1)/2,
    packed lower triangle b(i,j) = i(i+1)/2 + j), int32 for the int8 engine,
    float32 otherwise, float64 for the long-run accumulator.
    """

    def __init__(self, n_inputs: int, n_channels: int, engine: str = "i8", sample_type: str = "ci8",
                 fft_size: int = 0, max_abs: int = 7, requant_scale: float = 0.0, ring_samples: int = 0,
                 fp64_longrun: bool = False, device: str = "cuda:0", volt_format: str = "r8",
                 pfb_taps: int = 0):
        import torch

        self._torch = torch
        self.device = torch.device(device)
        self.n_inputs = n_inputs
        self.n_channels = n_channels
        self.engine = engine
        self.cfg = make_config(n_inputs, n_channels, engine, sample_type, fft_size, max_abs,
                               requant_scale, ring_samples, fp64_longrun, volt_format, pfb_taps)
        self.volt_format = volt_format
        self.ws_bytes = corr_workspace_bytes(self.cfg)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.plan = corr_create(self.cfg, self.workspace.data_ptr(), self.ws_bytes, self.stream.cuda_stream)
        self.n_products = n_inputs * (n_inputs + 1) // 2

    # -- plan calls ---------------------------------------------------------
    def channelise(self, volt, first_seq: int, spectra_dbg=None) -> None:
        """volt: device tensor [n_blocks*fft_size][n_inputs] (time-major) of the
        plan's volt_format, plus pfb_taps - 1 blocks of history with a filterbank."""
        t = self._torch
        want = {"r8": (t.int8,), "cw16": (t.int16, t.uint16), "cb8": (t.uint8, t.int8)}[self.volt_format]
        assert volt.dtype in want and volt.is_contiguous() and volt.device == self.device
        assert volt.dim() == 2 and volt.shape[1] == self.n_inputs, (tuple(volt.shape), self.n_inputs)
        assert volt.shape[0] % self.cfg.fft_size == 0, "whole blocks only"
        # with a filterbank of P taps the input carries P - 1 blocks of history
        n_blocks = volt.shape[0] // self.cfg.fft_size - max(0, self.cfg.pfb_taps - 1)
        assert n_blocks >= 0
        dbg = 0
        if spectra_dbg is not None:
            assert spectra_dbg.dtype == t.float32 and spectra_dbg.is_contiguous()
            assert spectra_dbg.device == self.device
            assert spectra_dbg.numel() >= self.n_channels * self.n_inputs * n_blocks * 2
            dbg = spectra_dbg.data_ptr()
        corr_channelise(self.plan, volt.data_ptr(), n_blocks, first_seq, dbg)

    def correlate(self, samples=None, n_samples: int | None = None, row_stride: int = 0) -> None:
        """samples: device tensor [n_channels][n_inputs][T][2] (int8 for ci8,
        float32 for cf32) or [n_channels][n_inputs][T] (int8/uint8 bytes for
        ci4); the first n_samples (default T) of each row are correlated.
        None drains the F-stage ring."""
        if samples is None:
            corr_correlate(self.plan, 0, 0, 0)
            return
        t = self._torch
        if self.cfg.sample_type == CORR_CI4:
            assert samples.dtype in (t.int8, t.uint8), samples.dtype
            assert samples.dim() == 3, tuple(samples.shape)
        else:
            want = t.int8 if self.cfg.sample_type == CORR_CI8 else t.float32
            assert samples.dtype == want, (samples.dtype, want)
            assert samples.dim() == 4 and samples.shape[3] == 2, tuple(samples.shape)
        assert samples.device == self.device and samples.is_contiguous()
        assert (samples.shape[0], samples.shape[1]) == (self.n_channels, self.n_inputs), tuple(samples.shape)
        stride = samples.shape[2]
        if n_samples is None:
            n_samples = stride
        assert 0 <= n_samples <= stride, (n_samples, stride)
        assert row_stride in (0, stride), "a contiguous tensor's row stride is its time extent"
        corr_correlate(self.plan, samples.data_ptr(), n_samples, stride)

    def correlate_ptr(self, d_samples: int, n_samples: int, row_stride: int = 0) -> None:
        """Raw form: device pointer to [n_channels][n_inputs][row_stride] samples."""
        corr_correlate(self.plan, d_samples, n_samples, row_stride)

    def _dump_dtype(self, what: int):
        t = self._torch
        if what & CORR_DUMP_LONGRUN:
            return t.float64
        return t.int32 if self.engine == "i8" else t.float32

    def dump(self, what: int = CORR_DUMP_INTEG, out=None, device_out: bool = True):
        """Returns (tensor, n_samples, exact)."""
        t = self._torch
        dtype = self._dump_dtype(what)
        copies = bool(what & (CORR_DUMP_INTEG | CORR_DUMP_LONGRUN))
        if out is None and copies:
            dev = self.device if device_out else t.device("cpu")
            out = t.empty((self.n_channels, self.n_products, 2), dtype=dtype, device=dev)
        elif out is not None and copies:
            assert out.dtype == dtype and out.is_contiguous(), (out.dtype, dtype)
            assert out.numel() >= self.n_channels * self.n_products * 2, out.numel()
            assert out.device.type == "cpu" or out.device == self.device
        ptr = out.data_ptr() if (out is not None and copies) else 0
        is_dev = out is not None and out.device.type == "cuda"
        n, exact = corr_dump(self.plan, what, ptr, is_dev)
        return out, n, exact

    def ring_read(self):
        t = self._torch
        buf = t.empty((self.n_channels, self.n_inputs, max(1, self.cfg.ring_samples), 2), dtype=t.int8)
        n = corr_ring_read(self.plan, buf.data_ptr(), False)
        flat = buf.reshape(-1)[: self.n_channels * self.n_inputs * n * 2]
        return flat.reshape(self.n_channels, self.n_inputs, n, 2)

    def stage_read(self):
        """FP16/FP8 engines: (staged elements [n_ch][n_in][n][2] as a numpy
        uint16/uint8 array, per-channel scales) of the last staged chunk."""
        import numpy as np
        esz = 2 if self.engine == "f16" else 1
        dt = np.uint16 if esz == 2 else np.uint8
        buf = np.empty(self.n_channels * self.n_inputs * max(1, self.cfg.ring_samples) * 2, dtype=dt)
        sc = np.empty(self.n_channels, dtype=np.float32)
        n = corr_stage_read(self.plan, buf.ctypes.data, sc.ctypes.data)
        return buf[: self.n_channels * self.n_inputs * n * 2].reshape(self.n_channels, self.n_inputs, n, 2), sc

    def seq_reset(self) -> None:
        corr_seq_reset(self.plan)

    def state(self):
        """(n_long, next_seq, seq_valid): what a checkpoint keeps besides the long-run sum."""
        return corr_state(self.plan)

    def restore(self, longrun, n_long: int, next_seq: int = 0, seq_valid: bool = False) -> None:
        """Load a checkpoint: longrun is a float64 tensor [n_channels][P][2] (host or device)."""
        t = self._torch
        src = longrun.contiguous()
        assert src.dtype == t.float64 and src.numel() == self.n_channels * self.n_products * 2
        corr_restore(self.plan, src.data_ptr(), src.is_cuda, n_long, next_seq, seq_valid)

    def close(self) -> None:
        if getattr(self, "plan", 0):
            corr_destroy(self.plan)
            self.plan = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Scheduler:
    """Serving scheduler over a device arena (torch tensor) with n_streams
    concurrent jobs.  ``submit`` takes the job shape, a fill callback address
    (a C function pointer of type corr_fill_fn) with its user pointer, or
    device samples, and a result tensor (device, or pinned host); ``poll``
    returns None until the job's result has landed there."""

    def __init__(self, arena_bytes: int, n_streams: int = 4, device: str = "cuda:0"):
        import torch

        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=device)
        self.handle = corr_sched_create(self.arena.data_ptr(), arena_bytes, n_streams)

    @staticmethod
    def now() -> float:
        return corr_sched_now()

    def submit(self, n_inputs: int, n_channels: int, n_samples: int, dst, max_abs: int = 7,
               fill: int = 0, fill_user: int = 0, d_samples: int = 0, row_stride: int = 0,
               t_arrival: float | None = None) -> int:
        j = corr_job_desc()
        j.n_inputs = n_inputs
        j.n_channels = n_channels
        j.n_samples = n_samples
        j.max_abs = max_abs
        j.fill = fill or None
        j.fill_user = fill_user or None
        j.d_samples = d_samples or None
        j.row_stride = row_stride
        import torch
        P = n_inputs * (n_inputs + 1) // 2
        assert dst.dtype == torch.int32 and dst.is_contiguous(), dst.dtype
        assert dst.numel() >= n_channels * P * 2, (dst.numel(), n_channels * P * 2)
        assert dst.device.type == "cpu" or dst.device == self.arena.device
        j.dst = dst.data_ptr()
        j.dst_is_device = int(dst.device.type == "cuda")
        return corr_sched_submit(self.handle, j, corr_sched_now() if t_arrival is None else t_arrival)

    def poll(self, job_id: int):
        return corr_sched_poll(self.handle, job_id)

    def stats(self):
        return corr_sched_stats(self.handle)

    def close(self) -> None:
        if getattr(self, "handle", 0):
            corr_sched_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
