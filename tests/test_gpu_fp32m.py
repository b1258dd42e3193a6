"""GPU parity of the FP32 matrix-core engine (CORR_X_FP32M:
v_mfma_f32_16x16x4_f32, FP32 accumulation, complex float32 input) through
the C ABI.

Integer-valued samples (|re|, |im| <= 7) give exact products and exact FP32
sums below 2^24, so the engine must equal the oracle's integer X-engine bit
for bit, and the plain FP32 engine too.  On Gaussian float samples the
relative Frobenius error against the FP64 oracle must stay within the 1e-5
the method asks of float inputs.  Cases: input counts around the 64-row
tiles, ragged sample counts, K-split passes (small arrays), row strides,
accumulation over calls, the full C1 configuration, and the refusal of rows
that are not 16-byte aligned."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_0906_1887_amd import CORR_DUMP_INTEG, CorrError, Correlator, _lib

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run(engine, x, T=None, stride=None, calls=None, max_abs=7):
    """x: float32 [ch][in][S][2] on the host; correlates the first T samples
    of each row (rows S samples apart), in the given (t0, t1) calls."""
    n_ch, n_in, S, _ = x.shape
    T = S if T is None else T
    buf = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    c = Correlator(n_in, n_ch, engine=engine, sample_type="cf32", max_abs=max_abs, device=DEV)
    for t0, t1 in (calls or [(0, T)]):
        c.correlate_ptr(buf.data_ptr() + 8 * t0, t1 - t0, S)
    out, n, exact = c.dump(CORR_DUMP_INTEG, device_out=True)
    c.close()
    assert n == T and exact == (max_abs > 0)
    return out


def test_integer_samples_bit_exact_on_edge_shapes():
    cases = [(1, 1, 8), (5, 3, 7), (17, 2, 65), (63, 2, 100), (64, 3, 64), (65, 2, 100), (130, 3, 300),
             (200, 1, 1), (64, 40, 1000)]
    for n_in, n_ch, T in cases:
        for pad in (0, 2):
            S = T + T % 2 + pad                    # even strides keep rows 16-byte aligned
            say(f"[fp32m] n_in={n_in} n_ch={n_ch} T={T} stride={S}")
            xi = synth.ci8(seed=n_in * 7 + T, n_channels=n_ch, n_inputs=n_in, n_samples=T)
            x = np.zeros((n_ch, n_in, S, 2), np.float32)
            x[:, :, :T] = xi
            x[:, :, T:] = 1e30                     # past the call: never read into the sums
            got = run("fp32m", x, T=T)
            assert np.array_equal(got.cpu().numpy().astype(np.int64), oracle.xengine_ci8(xi)), (n_in, n_ch, T)
            if pad == 0:
                assert torch.equal(got, run("fp32", x, T=T))


def test_accumulation_over_calls_and_alignment():
    n_in, n_ch, T = 70, 4, 600
    xi = synth.ci8(seed=17, n_channels=n_ch, n_inputs=n_in, n_samples=T)
    x = xi.astype(np.float32)
    got = run("fp32m", x, calls=[(0, 256), (256, 300), (300, T)])
    assert np.array_equal(got.cpu().numpy().astype(np.int64), oracle.xengine_ci8(xi))
    buf = torch.zeros((n_ch, n_in, 101, 2), dtype=torch.float32, device=DEV)
    c = Correlator(n_in, n_ch, engine="fp32m", sample_type="cf32", max_abs=7, device=DEV)
    with pytest.raises(CorrError) as e:
        c.correlate_ptr(buf.data_ptr(), 100, 101)            # odd stride: rows 8-byte aligned only
    assert e.value.status == _lib.CORR_E_UNSUPPORTED
    with pytest.raises(CorrError) as e:
        c.correlate_ptr(buf.data_ptr() + 8, 16, 100)          # base 8-byte aligned only
    assert e.value.status == _lib.CORR_E_UNSUPPORTED
    c.close()
    with pytest.raises(CorrError):                           # X-engine on CF32 only
        Correlator(8, 1, engine="fp32m", sample_type="ci8", max_abs=7, device=DEV)


def test_float_samples_within_1e5():
    for n_in, n_ch, T in ((64, 3, 1000), (150, 2, 334)):
        x = np.stack([synth.complex_float(11, ch, n_in, T) for ch in range(n_ch)])
        V = run("fp32m", x, max_abs=0).cpu().numpy().astype(np.float64)
        W = oracle.xengine_cf64(x)
        err = np.sqrt(np.sum((V - W) ** 2, axis=(1, 2))) / np.sqrt(np.sum(W ** 2, axis=(1, 2)))
        say(f"[fp32m float] n_in={n_in} T={T}: rel. Frobenius error max {err.max():.2e}")
        assert err.max() < 1e-5
        d = oracle.baseline_index(np.arange(n_in), np.arange(n_in))
        assert np.all(V[:, d, 1] == 0.0)


def test_c1_configuration():
    """N_I = 64, 128 channels, 1000 integer samples stored as complex float32
    (8 K splits): equal to the plain FP32 engine on every product and to the
    oracle on four channels."""
    n_in, n_ch, T = 64, 128, 1000
    xi = synth.ci8(seed=1, n_channels=n_ch, n_inputs=n_in, n_samples=T)
    x = xi.astype(np.float32)
    got = run("fp32m", x)
    assert torch.equal(got, run("fp32", x))
    sample = [0, 1, 64, 127]
    assert np.array_equal(got[sample].cpu().numpy().astype(np.int64), oracle.xengine_ci8(xi[sample]))
