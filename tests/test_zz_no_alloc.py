"""corr_correlate_static (the X-engine pass for callers that cannot allocate:
its K-split partials live in a fixed device array inside the library)
against corr_correlate on the same inputs, through the C ABI.

Two calls in a row, the second with a smaller input, per case; each result must
equal the plan path's dump and the oracle bit for bit (integer samples).  The
cases cover the K-split path (partials in the array), wide arrays with no
split, accumulation into the caller's buffer, and the refusal of a request
larger than the array."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_0906_1887_amd import CORR_DUMP_INTEG, CorrError, Correlator, _lib, make_config

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def static_pass(x, engine, accumulate=False, out=None):
    n_ch, n_in, T, _ = x.shape
    st = "ci8" if x.dtype == torch.int8 else "cf32"
    cfg = make_config(n_in, n_ch, engine=engine, sample_type=st, max_abs=7)
    dtype = torch.int32 if engine == "i8" else torch.float32
    if out is None:
        out = torch.full((n_ch, n_in * (n_in + 1) // 2, 2), -1, dtype=dtype, device=DEV)
    stream = torch.cuda.current_stream().cuda_stream
    _lib.corr_correlate_static(cfg, x.data_ptr(), T, T, out.data_ptr(), accumulate, stream)
    torch.cuda.synchronize()
    return out


def plan_pass(x, engine):
    n_ch, n_in, T, _ = x.shape
    st = "ci8" if x.dtype == torch.int8 else "cf32"
    c = Correlator(n_in, n_ch, engine=engine, sample_type=st, max_abs=7, device=DEV)
    c.correlate(x)
    out, n, exact = c.dump(CORR_DUMP_INTEG, device_out=True)
    c.close()
    assert n == T and exact
    return out


@pytest.mark.parametrize("engine", ["i8", "fp32"])
def test_static_scratch_matches_plan_two_calls(engine):
    # (large, then smaller): K-split partials in the array (64 inputs x 128
    # channels x 1000 samples: 8 splits, 17 MB), then a smaller split pass.
    for n_ch, n_in, T in ((128, 64, 1000), (3, 40, 96)):
        say(f"[static {engine}] n_ch={n_ch} n_in={n_in} T={T}")
        xh = synth.ci8(seed=n_in * 31 + T, n_channels=n_ch, n_inputs=n_in, n_samples=T)
        x = torch.from_numpy(xh).to(DEV)
        if engine == "fp32":
            x = x.float()
        got = static_pass(x, engine)
        want = plan_pass(x, engine)
        assert torch.equal(got, want), (engine, n_ch, n_in, T)
        assert np.array_equal(got.cpu().numpy().astype(np.int64), oracle.xengine_ci8(xh))


def test_static_scratch_wide_arrays_and_accumulate():
    # wide arrays without a K split (640 inputs, 72 channels; 1100 inputs, 16
    # channels), twice into the same buffer (store, then add), then a smaller
    # call that splits K (its partials overwrite the array's old contents).
    for n_ch, n_in, T in ((72, 640, 200), (16, 1100, 72)):
        say(f"[static i8] n_ch={n_ch} n_in={n_in} T={T}")
        xh = synth.ci8(seed=n_in + T, n_channels=n_ch, n_inputs=n_in, n_samples=T)
        x = torch.from_numpy(xh).to(DEV)
        want = oracle.xengine_ci8(xh)
        out = static_pass(x, "i8")
        assert torch.equal(out, plan_pass(x, "i8"))
        static_pass(x, "i8", accumulate=True, out=out)
        assert np.array_equal(out.cpu().numpy().astype(np.int64), 2 * want)
    xh = synth.ci8(seed=5, n_channels=2, n_inputs=70, n_samples=100)
    out = static_pass(torch.from_numpy(xh).to(DEV), "i8")
    assert np.array_equal(out.cpu().numpy().astype(np.int64), oracle.xengine_ci8(xh))


def test_static_scratch_ci4_samples():
    # one byte per sample (CI4): 1000 inputs on 33 channels (no split), then
    # 64 inputs on 96 channels (8 K splits, partials in the array); each
    # equals the plan path and the oracle on the decoded bytes
    from paper_0906_1887_amd import make_config
    for n_in, n_ch, T in ((1000, 33, 144), (64, 96, 992)):
        say(f"[static ci4] n_ch={n_ch} n_in={n_in} T={T}")
        x = synth.ci8(seed=n_in + 7, n_channels=n_ch, n_inputs=n_in, n_samples=T)
        re = x[..., 0].astype(np.int16) & 0xF
        im = x[..., 1].astype(np.int16) & 0xF
        b = ((re << 4) | im).astype(np.uint8)
        assert np.array_equal(oracle.unpack_b8(b), x)
        bt = torch.from_numpy(b).to(DEV)
        cfg = make_config(n_in, n_ch, engine="i8", sample_type="ci4", max_abs=7)
        out = torch.full((n_ch, n_in * (n_in + 1) // 2, 2), -1, dtype=torch.int32, device=DEV)
        _lib.corr_correlate_static(cfg, bt.data_ptr(), T, T, out.data_ptr(), False,
                                   torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        c = Correlator(n_in, n_ch, engine="i8", sample_type="ci4", max_abs=7, device=DEV)
        c.correlate(bt)
        want, n, exact = c.dump(CORR_DUMP_INTEG, device_out=True)
        c.close()
        assert n == T and exact and torch.equal(out, want)
        assert np.array_equal(out.cpu().numpy().astype(np.int64), oracle.xengine_ci8(x))


def test_static_scratch_refuses_oversized_requests():
    # 128 inputs x 900 channels x 1000 samples needs 2 K splits of 119 MB of
    # partials: more than the 64 MiB array; refused before any launch.
    cfg = make_config(128, 900, engine="i8", sample_type="ci8", max_abs=7)
    with pytest.raises(CorrError) as e:
        _lib.corr_correlate_static(cfg, 1 << 20, 1000, 1000, 1 << 20, False, 0)
    assert e.value.status == _lib.CORR_E_WORKSPACE
    cfg = make_config(64, 4, engine="f16", sample_type="cf32", max_abs=0, ring_samples=64)
    with pytest.raises(CorrError) as e:
        _lib.corr_correlate_static(cfg, 1 << 20, 10, 10, 1 << 20, False, 0)
    assert e.value.status == _lib.CORR_E_UNSUPPORTED
