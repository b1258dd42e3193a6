"""ctypes binding of libcorr's C ABI (include/corr.h), same names, argument
marshalling only.  Every step of the correlator runs in the HIP library;
this module raises if the library is not built."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcorr.so")

CORR_OK = 0
CORR_E_INVAL = -1
CORR_E_WORKSPACE = -2
CORR_E_HIP = -3
CORR_E_STATE = -4
CORR_E_OVERFLOW = -5
CORR_E_SEQ = -6
CORR_E_BUSY = -7
CORR_E_UNSUPPORTED = -8
CORR_E_CORRUPT = -9

CORR_CF32 = 0
CORR_CI8 = 1
CORR_CI4 = 2

CORR_X_FP32 = 0
CORR_X_I8 = 1
CORR_X_F16 = 2
CORR_X_F8 = 3
CORR_X_FP32M = 4

CORR_DUMP_INTEG = 1
CORR_DUMP_LONGRUN = 2
CORR_DUMP_FOLD = 4
CORR_DUMP_NO_RESET = 8

EXPORTED = [
    "corr_workspace_bytes", "corr_create", "corr_destroy", "corr_channelise", "corr_seq_reset",
    "corr_correlate", "corr_dump", "corr_ring_read", "corr_stage_read", "corr_dump_bytes", "corr_status_str",
    "corr_sched_now", "corr_sched_create", "corr_sched_submit", "corr_sched_poll", "corr_sched_stats",
    "corr_sched_destroy", "corr_aggregate_w16", "corr_cmac_design", "corr_correlate_static",
    "corr_state", "corr_restore",
]


class corr_config(ctypes.Structure):
    _fields_ = [
        ("n_inputs", ctypes.c_int32),
        ("n_channels", ctypes.c_int32),
        ("fft_size", ctypes.c_int32),
        ("sample_type", ctypes.c_int32),
        ("engine", ctypes.c_int32),
        ("max_abs", ctypes.c_int32),
        ("requant_scale", ctypes.c_float),
        ("fp64_longrun", ctypes.c_int32),
        ("ring_samples", ctypes.c_int64),
        ("volt_format", ctypes.c_int32),
        ("pfb_taps", ctypes.c_int32),
    ]


class corr_job_desc(ctypes.Structure):
    _fields_ = [
        ("n_inputs", ctypes.c_int32),
        ("n_channels", ctypes.c_int32),
        ("n_samples", ctypes.c_int64),
        ("max_abs", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("fill", ctypes.c_void_p),
        ("fill_user", ctypes.c_void_p),
        ("d_samples", ctypes.c_void_p),
        ("row_stride", ctypes.c_int64),
        ("dst", ctypes.c_void_p),
        ("dst_is_device", ctypes.c_int32),
        ("reserved2", ctypes.c_int32),
    ]


class CorrError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {corr_status_str(status)} ({status})")


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                               "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        I32, I64 = ctypes.c_int32, ctypes.c_int64
        cfgp = ctypes.POINTER(corr_config)
        L.corr_workspace_bytes.argtypes = [cfgp, ctypes.POINTER(ctypes.c_size_t)]
        L.corr_create.argtypes = [cfgp, P, ctypes.c_size_t, P, ctypes.POINTER(P)]
        L.corr_destroy.argtypes = [P]
        L.corr_channelise.argtypes = [P, P, I64, ctypes.c_uint64, P]
        L.corr_seq_reset.argtypes = [P]
        L.corr_state.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(I32)]
        L.corr_restore.argtypes = [P, P, I32, I64, ctypes.c_uint64, I32]
        L.corr_aggregate_w16.argtypes = [P, I32, I32, I64, ctypes.c_uint32, P, P, P]
        L.corr_cmac_design.argtypes = [I32, I32, P, I64, I32, I32, P, I32, P]
        L.corr_correlate.argtypes = [P, P, I64, I64]
        L.corr_correlate_static.argtypes = [ctypes.POINTER(corr_config), P, I64, I64, P, I32, P]
        L.corr_dump.argtypes = [P, I32, P, I32, ctypes.POINTER(I64), ctypes.POINTER(I32)]
        L.corr_ring_read.argtypes = [P, P, I32, ctypes.POINTER(I64)]
        L.corr_stage_read.argtypes = [P, P, P, ctypes.POINTER(I64)]
        L.corr_dump_bytes.argtypes = [P, I32, ctypes.POINTER(ctypes.c_size_t)]
        L.corr_status_str.argtypes = [ctypes.c_int]
        L.corr_status_str.restype = ctypes.c_char_p
        L.corr_sched_now.argtypes = []
        L.corr_sched_create.argtypes = [P, ctypes.c_size_t, I32, ctypes.POINTER(P)]
        L.corr_sched_submit.argtypes = [P, ctypes.POINTER(corr_job_desc), ctypes.c_double, ctypes.POINTER(ctypes.c_uint64)]
        L.corr_sched_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(I64), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.corr_sched_stats.argtypes = [P, ctypes.POINTER(I64)]
        L.corr_sched_destroy.argtypes = [P]
        for name in EXPORTED:
            if name not in ("corr_status_str", "corr_sched_now"):
                getattr(L, name).restype = ctypes.c_int
        L.corr_sched_now.restype = ctypes.c_double
        _lib = L
    return _lib


def corr_status_str(status: int) -> str:
    return lib().corr_status_str(int(status)).decode()


def _check(status: int, where: str) -> None:
    if status != CORR_OK:
        raise CorrError(status, where)


def corr_workspace_bytes(cfg: corr_config) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().corr_workspace_bytes(ctypes.byref(cfg), ctypes.byref(n)), "corr_workspace_bytes")
    return int(n.value)


def corr_create(cfg: corr_config, d_workspace: int, ws_bytes: int, hip_stream: int) -> int:
    out = ctypes.c_void_p(0)
    _check(lib().corr_create(ctypes.byref(cfg), ctypes.c_void_p(d_workspace), ws_bytes,
                             ctypes.c_void_p(hip_stream), ctypes.byref(out)), "corr_create")
    return int(out.value)


def corr_destroy(plan: int) -> None:
    _check(lib().corr_destroy(ctypes.c_void_p(plan)), "corr_destroy")


def corr_aggregate_w16(d_records: int, n_streams: int, words_per_record: int, n_records: int,
                       first_counter: int, d_out: int, d_bad_records: int = 0, stream: int = 0) -> None:
    _check(lib().corr_aggregate_w16(ctypes.c_void_p(d_records), n_streams, words_per_record, n_records,
                                    first_counter & 0xFFFFFFFF, ctypes.c_void_p(d_out),
                                    ctypes.c_void_p(d_bad_records or None), ctypes.c_void_p(stream or None)),
           "corr_aggregate_w16")


def corr_cmac_design(design: int, group: int, d_spectra: int, n_samples: int, n_inputs: int, n_channels: int,
                     d_out: int, accumulate: bool = False, stream: int = 0) -> None:
    _check(lib().corr_cmac_design(design, group, ctypes.c_void_p(d_spectra), n_samples, n_inputs, n_channels,
                                  ctypes.c_void_p(d_out), int(bool(accumulate)), ctypes.c_void_p(stream or None)),
           "corr_cmac_design")


def corr_channelise(plan: int, d_volt: int, n_blocks: int, first_seq: int, d_spectra_dbg: int = 0) -> None:
    _check(lib().corr_channelise(ctypes.c_void_p(plan), ctypes.c_void_p(d_volt), n_blocks,
                                 first_seq & 0xFFFFFFFFFFFFFFFF, ctypes.c_void_p(d_spectra_dbg or None)),
           "corr_channelise")


def corr_seq_reset(plan: int) -> None:
    _check(lib().corr_seq_reset(ctypes.c_void_p(plan)), "corr_seq_reset")


def corr_state(plan: int):
    """(n_long, next_seq, seq_valid) of a plan: what a checkpoint keeps besides the long-run sum."""
    n = ctypes.c_int64(0)
    seq = ctypes.c_uint64(0)
    valid = ctypes.c_int32(0)
    _check(lib().corr_state(ctypes.c_void_p(plan), ctypes.byref(n), ctypes.byref(seq), ctypes.byref(valid)),
           "corr_state")
    return int(n.value), int(seq.value), bool(valid.value)


def corr_restore(plan: int, longrun: int, src_is_device: bool, n_long: int, next_seq: int, seq_valid: bool) -> None:
    _check(lib().corr_restore(ctypes.c_void_p(plan), ctypes.c_void_p(longrun), int(src_is_device),
                              ctypes.c_int64(n_long), ctypes.c_uint64(next_seq), int(seq_valid)), "corr_restore")


def corr_correlate(plan: int, d_samples: int, n_samples: int, row_stride: int = 0) -> None:
    _check(lib().corr_correlate(ctypes.c_void_p(plan), ctypes.c_void_p(d_samples or None), n_samples,
                                row_stride), "corr_correlate")


def corr_correlate_static(cfg: corr_config, d_samples: int, n_samples: int, row_stride: int, d_out: int,
                          accumulate: bool, stream: int = 0) -> None:
    _check(lib().corr_correlate_static(ctypes.byref(cfg), ctypes.c_void_p(d_samples or None), n_samples, row_stride,
                                       ctypes.c_void_p(d_out or None), int(bool(accumulate)),
                                       ctypes.c_void_p(stream or None)), "corr_correlate_static")


def corr_dump(plan: int, what: int, dst: int, dst_is_device: bool):
    n = ctypes.c_int64(0)
    exact = ctypes.c_int32(0)
    _check(lib().corr_dump(ctypes.c_void_p(plan), what, ctypes.c_void_p(dst), int(bool(dst_is_device)),
                           ctypes.byref(n), ctypes.byref(exact)), "corr_dump")
    return int(n.value), bool(exact.value)


def corr_ring_read(plan: int, dst: int, dst_is_device: bool) -> int:
    n = ctypes.c_int64(0)
    _check(lib().corr_ring_read(ctypes.c_void_p(plan), ctypes.c_void_p(dst), int(bool(dst_is_device)),
                                ctypes.byref(n)), "corr_ring_read")
    return int(n.value)


def corr_stage_read(plan: int, dst: int, scales: int = 0) -> int:
    n = ctypes.c_int64(0)
    _check(lib().corr_stage_read(ctypes.c_void_p(plan), ctypes.c_void_p(dst), ctypes.c_void_p(scales or None),
                                 ctypes.byref(n)), "corr_stage_read")
    return int(n.value)


def corr_dump_bytes(plan: int, what: int) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().corr_dump_bytes(ctypes.c_void_p(plan), what, ctypes.byref(n)), "corr_dump_bytes")
    return int(n.value)


def corr_sched_now() -> float:
    return float(lib().corr_sched_now())


def corr_sched_create(d_arena: int, arena_bytes: int, n_streams: int) -> int:
    out = ctypes.c_void_p(0)
    _check(lib().corr_sched_create(ctypes.c_void_p(d_arena), arena_bytes, n_streams, ctypes.byref(out)),
           "corr_sched_create")
    return int(out.value)


def corr_sched_submit(sched: int, job: corr_job_desc, t_arrival: float) -> int:
    jid = ctypes.c_uint64(0)
    _check(lib().corr_sched_submit(ctypes.c_void_p(sched), ctypes.byref(job), t_arrival, ctypes.byref(jid)),
           "corr_sched_submit")
    return int(jid.value)


def corr_sched_poll(sched: int, job_id: int):
    """None while the job is queued or running; else (status, n_samples,
    t_admit, t_done, t_device)."""
    n = ctypes.c_int64(0)
    ta = ctypes.c_double(0.0)
    tv = ctypes.c_double(0.0)
    td = ctypes.c_double(0.0)
    st = lib().corr_sched_poll(ctypes.c_void_p(sched), job_id, ctypes.byref(n), ctypes.byref(ta), ctypes.byref(tv),
                               ctypes.byref(td))
    if st == CORR_E_BUSY:
        return None
    if st == CORR_E_INVAL:
        raise CorrError(st, "corr_sched_poll")
    return int(st), int(n.value), float(ta.value), float(td.value), float(tv.value)


def corr_sched_stats(sched: int):
    arr = (ctypes.c_int64 * 8)()
    _check(lib().corr_sched_stats(ctypes.c_void_p(sched), arr), "corr_sched_stats")
    keys = ["submitted", "admitted", "completed", "failed", "queued", "running", "peak_arena_bytes", "arena_bytes"]
    return dict(zip(keys, [int(v) for v in arr]))


def corr_sched_destroy(sched: int) -> None:
    _check(lib().corr_sched_destroy(ctypes.c_void_p(sched)), "corr_sched_destroy")
