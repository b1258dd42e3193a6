"""Serving scheduler on the GPU through the C ABI: each job's result is the
same alone and inside a concurrent mix (bit-exact, integer data), matches the
oracle, and admission by HBM footprint queues jobs that do not fit.  Jobs
with 16-byte aligned rows run on the device job queue (a persistent grid, no
per-job plan or launch; the grid closes when the queue idles and the
scheduler launches a new one for later work); results land in device or
pinned host buffers; caller buffers with an odd row stride take the per-job
plan path."""
import sys
import time

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_0906_1887_amd import CorrError, Scheduler, _lib

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
BASE_SEED = 5000

JOBS = [(16, 64, 1000), (512, 64, 1500), (64, 256, 2000), (128, 64, 1234), (1024, 64, 1000),
        (16, 256, 3000), (64, 64, 999), (512, 256, 1200), (128, 256, 1001), (16, 64, 8000),
        (1024, 64, 2048), (64, 768, 1000)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def result_buf(n_in, n_ch, device=True):
    P = n_in * (n_in + 1) // 2
    return torch.empty((n_ch, P, 2), dtype=torch.int32, device=DEV if device else "cpu")


def wait(s, jid, timeout=60.0):
    t0 = time.time()
    while True:
        r = s.poll(jid)
        if r is not None:
            return r
        assert time.time() - t0 < timeout, f"job {jid} not done"
        time.sleep(0.0005)


def run_jobs(jobs, concurrent, arena_bytes=8 << 30, n_streams=4):
    gen = synth.DeviceGen()
    fn, user, keep = gen.job_fill(BASE_SEED)
    s = Scheduler(arena_bytes, n_streams)
    outs, ids, lat = [], [], []
    try:
        for (n_in, n_ch, T) in jobs:
            out = result_buf(n_in, n_ch)
            jid = s.submit(n_in, n_ch, T, out, fill=fn, fill_user=user)
            outs.append(out)
            ids.append(jid)
            if not concurrent:
                st, n, ta, td, tv = wait(s, jid)
                assert st == 0 and n == T
        if concurrent:
            for jid, (n_in, n_ch, T) in zip(ids, jobs):
                st, n, ta, td, tv = wait(s, jid)
                assert st == 0 and n == T
        stats = s.stats()
    finally:
        s.close()
    del keep
    return ids, [o.cpu().numpy() for o in outs], stats


def test_alone_equals_mix_and_oracle():
    say("[serving] alone")
    ids_a, alone, _ = run_jobs(JOBS, concurrent=False)
    say("[serving] mix")
    ids_m, mix, stats = run_jobs(JOBS, concurrent=True)
    assert ids_a == ids_m == list(range(1, len(JOBS) + 1))
    assert stats["completed"] == len(JOBS) and stats["failed"] == 0
    for k, (a, m) in enumerate(zip(alone, mix)):
        assert np.array_equal(a, m), f"job {k} differs alone vs mix"
    # oracle on the smaller jobs (host regeneration of seed BASE_SEED + job id)
    for k, (n_in, n_ch, T) in enumerate(JOBS):
        if n_in * n_in * n_ch * T > 3e10:
            continue
        x = synth.ci8(BASE_SEED + ids_a[k], n_ch, n_in, T)
        assert np.array_equal(mix[k].astype(np.int64), oracle.xengine_ci8(x)), k


def test_admission_queues_when_arena_is_small():
    jobs = [(128, 64, 2000)] * 6 + [(16, 64, 1000)] * 4
    from paper_0906_1887_amd import make_config
    ws = _lib.corr_workspace_bytes(make_config(128, 64, engine="i8", max_abs=7))
    foot = 64 * 128 * 2000 * 2 + ws
    arena = int(2.5 * foot) // 256 * 256          # at most two of the large jobs at once
    say(f"[serving] small arena {arena / 2**20:.1f} MiB, job footprint {foot / 2**20:.1f} MiB")
    ids, outs, stats = run_jobs(jobs, concurrent=True, arena_bytes=arena, n_streams=4)
    assert stats["completed"] == len(jobs)
    assert stats["peak_arena_bytes"] <= stats["arena_bytes"]
    first = outs[0]
    x = synth.ci8(BASE_SEED + ids[0], 64, 128, 2000)
    assert np.array_equal(first.astype(np.int64), oracle.xengine_ci8(x))
    fn, user, keep = synth.DeviceGen().job_fill(BASE_SEED)
    s = Scheduler(64 << 20, 2)
    try:
        # footprint beyond the whole arena: refused at submission, before the
        # result buffer is touched (the raw C call; the Python wrapper would
        # already refuse the one-element buffer)
        j = _lib.corr_job_desc()
        j.n_inputs, j.n_channels, j.n_samples, j.max_abs = 1024, 768, 8000, 7
        j.fill, j.fill_user = fn, user
        j.dst = result_buf(1, 1).data_ptr()
        j.dst_is_device = 1
        with pytest.raises(CorrError) as e:
            _lib.corr_sched_submit(s.handle, j, _lib.corr_sched_now())
        assert e.value.status == _lib.CORR_E_WORKSPACE
        with pytest.raises(AssertionError):               # the wrapper checks the buffer size
            s.submit(1024, 768, 8000, result_buf(1, 1), fill=fn, fill_user=user)
    finally:
        s.close()
    del keep


def test_caller_device_samples_and_host_result():
    n_in, n_ch, T = 40, 3, 333
    x = synth.ci8(77, n_ch, n_in, T)
    xt = torch.from_numpy(x).to(DEV)
    out = result_buf(n_in, n_ch, device=False).pin_memory()
    s = Scheduler(64 << 20, 2)
    try:
        jid = s.submit(n_in, n_ch, T, out, d_samples=xt.data_ptr())
        st, n, ta, td, tv = wait(s, jid)
        assert st == 0 and n == T and td >= ta
    finally:
        s.close()
    assert np.array_equal(out.numpy().astype(np.int64), oracle.xengine_ci8(x))


def test_caller_ring_with_row_stride():
    """Jobs read the first n_samples of each row of a wider ring buffer; the
    samples past n_samples (filled with other values) are never used."""
    n_in, n_ch, T, stride = 48, 5, 700, 1024
    ring = synth.ci8(91, n_ch, n_in, stride)
    x = np.ascontiguousarray(ring[:, :, :T])
    rt = torch.from_numpy(ring).to(DEV)
    out = result_buf(n_in, n_ch)
    s = Scheduler(64 << 20, 2)
    try:
        with pytest.raises(CorrError) as e:
            s.submit(n_in, n_ch, T, out, d_samples=rt.data_ptr(), row_stride=T - 1)
        assert e.value.status == _lib.CORR_E_INVAL
        jid = s.submit(n_in, n_ch, T, out, d_samples=rt.data_ptr(), row_stride=stride)
        st, n, ta, td, tv = wait(s, jid)
        assert st == 0 and n == T
    finally:
        s.close()
    assert np.array_equal(out.cpu().numpy().astype(np.int64), oracle.xengine_ci8(x))


def test_queue_host_and_device_destinations_alone_equals_mix():
    """The device job queue with results copied to pinned host memory and
    written straight to device memory, large and small jobs submitted
    together (a large job first, small ones behind it): every result equals
    the same job run alone, and the oracle; the device-complete time precedes
    the host landing."""
    jobs = [(520, 256, 1000), (16, 64, 1000), (100, 3, 77), (64, 128, 2000), (200, 7, 64), (17, 1, 1)]
    gen = synth.DeviceGen()
    fn, user, keep = gen.job_fill(BASE_SEED)
    results = {}
    for mode in ("alone", "mix"):
        s = Scheduler(4 << 30, 2)
        outs, ids = [], []
        try:
            for k, (n_in, n_ch, T) in enumerate(jobs):
                host = k % 2 == 0
                out = result_buf(n_in, n_ch, device=not host)
                if host:
                    out = out.pin_memory()
                jid = s.submit(n_in, n_ch, T, out, fill=fn, fill_user=user)
                outs.append(out)
                ids.append(jid)
                if mode == "alone":
                    st, n, ta, td, tv = wait(s, jid)
                    assert st == 0 and n == T and ta <= tv <= td
            if mode == "mix":
                for jid, (n_in, n_ch, T) in zip(ids, jobs):
                    st, n, ta, td, tv = wait(s, jid)
                    assert st == 0 and n == T and ta <= tv <= td
            stats = s.stats()
        finally:
            s.close()
        assert stats["completed"] == len(jobs) and stats["failed"] == 0
        results[mode] = (ids, [o.cpu().numpy() for o in outs])
        say(f"[serving queue] {mode} done")
    del keep
    ids_a, alone = results["alone"]
    ids_m, mix = results["mix"]
    for k, (n_in, n_ch, T) in enumerate(jobs):
        assert np.array_equal(alone[k], mix[k]), k
        x = synth.ci8(BASE_SEED + ids_m[k], n_ch, n_in, T)
        assert np.array_equal(mix[k].astype(np.int64), oracle.xengine_ci8(x)), k


def test_grid_closes_and_new_work_gets_a_new_grid():
    """Jobs separated by idle gaps longer than the grid's idle close (0.1 ms):
    each is run by a freshly launched grid; then a burst behind a small first
    job (the first grid must not stay sized for it: every grid is launched at
    full size).  Every result equals the oracle."""
    gen = synth.DeviceGen()
    fn, user, keep = gen.job_fill(BASE_SEED)
    s = Scheduler(2 << 30, 2)
    jobs = [(16, 8, 200), (130, 5, 300), (17, 3, 64)] + [(16, 4, 100)] + [(300, 16, 500)] * 3 + [(64, 32, 777)] * 4
    outs, ids = [], []
    try:
        for k, (n_in, n_ch, T) in enumerate(jobs):
            out = result_buf(n_in, n_ch)
            ids.append(s.submit(n_in, n_ch, T, out, fill=fn, fill_user=user))
            outs.append(out)
            if k < 3:
                st, n, ta, td, tv = wait(s, ids[-1])
                assert st == 0 and n == T
                time.sleep(0.005)
        for jid, (n_in, n_ch, T) in zip(ids[3:], jobs[3:]):
            st, n, ta, td, tv = wait(s, jid)
            assert st == 0 and n == T
        stats = s.stats()
    finally:
        s.close()
    del keep
    assert stats["completed"] == len(jobs) and stats["failed"] == 0
    for k, (n_in, n_ch, T) in enumerate(jobs):
        x = synth.ci8(BASE_SEED + ids[k], n_ch, n_in, T)
        assert np.array_equal(outs[k].cpu().numpy().astype(np.int64), oracle.xengine_ci8(x)), k
    say("[serving] grid close and relaunch done")


def test_odd_row_stride_takes_the_plan_path():
    """Caller rows whose stride is not a multiple of 8 samples (not 16-byte
    aligned) are correlated through a per-job plan; the result is the same."""
    n_in, n_ch, T, stride = 70, 3, 500, 1001
    ring = synth.ci8(93, n_ch, n_in, stride)
    x = np.ascontiguousarray(ring[:, :, :T])
    rt = torch.from_numpy(ring).to(DEV)
    out = result_buf(n_in, n_ch, device=False).pin_memory()
    s = Scheduler(64 << 20, 2)
    try:
        jid = s.submit(n_in, n_ch, T, out, d_samples=rt.data_ptr(), row_stride=stride)
        st, n, ta, td, tv = wait(s, jid)
        assert st == 0 and n == T
    finally:
        s.close()
    assert np.array_equal(out.numpy().astype(np.int64), oracle.xengine_ci8(x))
