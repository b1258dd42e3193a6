"""GPU parity of the int8 engine on 4-bit complex samples packed one per byte
(CORR_CI4: re in bits 7..4, im in bits 3..0, the "1-byte" mode of Sec. 5),
through the C ABI.

The bytes are packed from int8 pairs in the test; the expected visibilities
are the oracle's X-engine on the oracle's own decode of those bytes
(oracle.unpack_b8, pinned by hand-decoded goldens), which must also give the
pairs back.  Integer samples: every result bit-exact."""
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


def pack(x: np.ndarray) -> np.ndarray:
    """int8 pairs [..., 2] in [-7, 7] -> one byte per sample, re in the high nibble."""
    re = x[..., 0].astype(np.int16) & 0xF
    im = x[..., 1].astype(np.int16) & 0xF
    return ((re << 4) | im).astype(np.uint8)


def expected(b: np.ndarray, x: np.ndarray) -> np.ndarray:
    d = oracle.unpack_b8(b)
    assert np.array_equal(d, x)
    return oracle.xengine_ci8(d)


def run_ci4(b: np.ndarray, T=None, stride=None, chunks=None, max_abs=7):
    n_ch, n_in, S = b.shape
    T = S if T is None else T
    c = Correlator(n_in, n_ch, engine="i8", sample_type="ci4", max_abs=max_abs, device=DEV)
    bt = torch.from_numpy(np.ascontiguousarray(b)).to(DEV)
    if chunks is None:
        c.correlate_ptr(bt.data_ptr(), T, S)
    else:
        for t0, t1 in chunks:
            c.correlate_ptr(bt.data_ptr() + t0, t1 - t0, S)
    out, n, exact = c.dump(CORR_DUMP_INTEG, device_out=False)
    c.close()
    assert n == T and exact
    return out.numpy().astype(np.int64)


def test_ci4_edge_shapes():
    """Input counts around the 128-row tiles (diagonal and off-diagonal tiles,
    ragged panels, one input), sample counts of whole and partial 64-sample
    stages, zero samples, one to three channels."""
    for n_in in (1, 2, 17, 64, 65, 127, 128, 129, 200, 260):
        for T in (0, 16, 48, 64, 208):
            n_ch = 3 if (n_in + T) % 2 else 1
            say(f"[ci4] n_in={n_in} n_ch={n_ch} T={T}")
            x = synth.ci8(seed=n_in * 977 + T, n_channels=n_ch, n_inputs=n_in, n_samples=T)
            b = pack(x)
            assert np.array_equal(run_ci4(b), expected(b, x)), (n_in, n_ch, T)


def test_ci4_row_stride_chunks_and_alignment():
    """Rows of T samples inside a wider buffer (stride a multiple of 16),
    two aligned calls accumulated into one integration, and the refusal of
    rows that are not 16-byte aligned."""
    n_ch, n_in, S = 3, 150, 336
    x = synth.ci8(seed=71, n_channels=n_ch, n_inputs=n_in, n_samples=S)
    b = pack(x)
    T = 300
    assert np.array_equal(run_ci4(b, T=T), expected(b[:, :, :T], x[:, :, :T]))
    assert np.array_equal(run_ci4(b, chunks=[(0, 160), (160, S)]), expected(b, x))
    c = Correlator(n_in, n_ch, engine="i8", sample_type="ci4", max_abs=7, device=DEV)
    bt = torch.from_numpy(np.ascontiguousarray(b)).to(DEV)
    with pytest.raises(CorrError) as e:
        c.correlate_ptr(bt.data_ptr(), 100, 100)               # 100-byte rows
    assert e.value.status == _lib.CORR_E_UNSUPPORTED
    with pytest.raises(CorrError) as e:
        c.correlate_ptr(bt.data_ptr() + 8, 16, S)               # base not 16-byte aligned
    assert e.value.status == _lib.CORR_E_UNSUPPORTED
    c.close()
    with pytest.raises(CorrError):                              # nibbles hold at most |7|
        Correlator(8, 1, engine="i8", sample_type="ci4", max_abs=8, device=DEV)
    with pytest.raises(CorrError):                              # int8 engine only
        Correlator(8, 1, engine="fp32", sample_type="ci4", max_abs=7, device=DEV)


def test_ci4_extremes_near_the_bound():
    """Every sample at +-7 in both parts, T close to the bound: the engine sums
    256 times the visibility, so 2 * 7^2 * T * 256 <= 2^31 - 1 (T <= 85598);
    an accumulation past it is refused."""
    rng = np.random.default_rng(6)
    T = 85584
    x = (rng.integers(0, 2, size=(1, 130, T, 2)) * 14 - 7).astype(np.int8)
    x[0, 3] = 7
    b = pack(x)
    want = expected(b, x)
    assert want[0, oracle.baseline_index(3, 3), 0] == 2 * 49 * T
    assert np.array_equal(run_ci4(b), want)
    c = Correlator(130, 1, engine="i8", sample_type="ci4", max_abs=7, device=DEV)
    bt = torch.from_numpy(np.ascontiguousarray(b)).to(DEV)
    c.correlate_ptr(bt.data_ptr(), T, T)
    with pytest.raises(CorrError) as e:
        c.correlate_ptr(bt.data_ptr(), 32, T)
    assert e.value.status == _lib.CORR_E_OVERFLOW
    c.close()


def test_ci4_many_tiles():
    """1000 inputs on 33 channels: over 1000 tiles, no K split."""
    n_in, n_ch, T = 1000, 33, 144
    x = synth.ci8(seed=123, n_channels=n_ch, n_inputs=n_in, n_samples=T)
    b = pack(x)
    assert np.array_equal(run_ci4(b), expected(b, x))


def test_ci4_c3_full_array_equals_int8_pairs():
    """The C3 array (1024 inputs, 768 channels, 8000 samples from the device
    generator) packed one byte per sample: the CI4 engine's dump equals the
    int8-pair engine's dump bit for bit on all 403 M products, and two whole
    channels equal the oracle."""
    n_in, n_ch, T, seed = 1024, 768, 8000, 3
    gen = synth.DeviceGen()
    say("[C3 ci4] device generation")
    x = torch.empty((n_ch, n_in, T, 2), dtype=torch.int8, device=DEV)
    gen.fill_ci8(x.data_ptr(), n_ch, n_in, T, seed, stream=torch.cuda.current_stream().cuda_stream)
    b = ((x[..., 0] & 15) << 4) | (x[..., 1] & 15)                # int8 ops; wraps to the packed byte
    b = b.to(torch.int8).contiguous()
    say("[C3 ci4] int8 pairs")
    c = Correlator(n_in, n_ch, engine="i8", max_abs=7, device=DEV)
    c.correlate(x)
    v8, _, _ = c.dump(CORR_DUMP_INTEG)
    c.close()
    del x
    say("[C3 ci4] one byte per sample")
    c = Correlator(n_in, n_ch, engine="i8", sample_type="ci4", max_abs=7, device=DEV)
    c.correlate(b)
    v4, n, exact = c.dump(CORR_DUMP_INTEG)
    c.close()
    assert n == T and exact
    assert torch.equal(v4, v8)
    del v8
    for ch in (0, 767):
        xc = synth.ci8_channel(seed, ch, n_in, T)
        bc = b[ch].cpu().numpy().view(np.uint8)
        assert np.array_equal(oracle.unpack_b8(bc), xc)
        assert np.array_equal(v4[ch].cpu().numpy().astype(np.int64), oracle.xengine_ci8(xc[None])[0]), ch
