"""GPU parity of the X-engines against the CPU oracle, through the C ABI.

Integer-valued samples: every engine must be bit-exact (int32 accumulation
for the int8 MFMA engine, FP32 for the plain engine, both exact within the
host-checked bounds).
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_0906_1887_amd import CORR_DUMP_INTEG, CORR_DUMP_NO_RESET, Correlator

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_vis(x, engine, sample_type="ci8", chunks=None, max_abs=7):
    n_ch, n_in, T, _ = x.shape
    c = Correlator(n_in, n_ch, engine=engine, sample_type=sample_type, max_abs=max_abs, device=DEV)
    if sample_type == "ci8":
        xt = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
        esz = 2
    else:
        xt = torch.from_numpy(np.ascontiguousarray(x.astype(np.float32))).to(DEV)
        esz = 8
    if chunks is None:
        c.correlate(xt, T)
    else:
        for t0, t1 in chunks:
            c.correlate_ptr(xt.data_ptr() + t0 * esz, t1 - t0, T)
    out, n, exact = c.dump(CORR_DUMP_INTEG, device_out=False)
    c.close()
    assert n == T and exact
    return out.numpy().astype(np.int64)


EDGE_NI = [1, 2, 3, 15, 16, 17, 63, 64, 65, 127, 129, 200]
EDGE_T = [0, 1, 7, 63, 64, 65, 200]


@pytest.mark.parametrize("engine", ["i8", "fp32"])
def test_edge_shapes_ci8(engine):
    for n_in in EDGE_NI:
        for T in EDGE_T:
            n_ch = 3 if (n_in + T) % 2 else 1
            say(f"[xengine {engine} ci8] n_in={n_in} n_ch={n_ch} T={T}")
            x = synth.ci8(seed=n_in * 1000 + T, n_channels=n_ch, n_inputs=n_in, n_samples=T)
            got = gpu_vis(x, engine)
            want = oracle.xengine_ci8(x)
            assert np.array_equal(got, want), (engine, n_in, n_ch, T)


def test_wide_arrays_all_tile_kinds():
    """3 to 9 row blocks of 128 inputs (odd and even block counts, ragged last
    block) reach every kind of work item of the 128-row engine: tile pairs
    below the diagonal, a pair ending on the diagonal, and two diagonal tiles
    of different rows in one workgroup; T = 1500 on two channels also splits
    K.  int8 engine against the oracle."""
    for n_in, T in ((260, 129), (390, 70), (520, 1500), (777, 65), (1100, 200)):
        say(f"[xengine i8 ci8] n_in={n_in} n_ch=2 T={T}")
        x = synth.ci8(seed=n_in + 31 * T, n_channels=2, n_inputs=n_in, n_samples=T)
        assert np.array_equal(gpu_vis(x, "i8"), oracle.xengine_ci8(x)), (n_in, T)


def test_edge_shapes_cf32_fp32():
    for n_in in (1, 17, 64, 65, 129):
        for T in (1, 7, 64, 100):
            say(f"[xengine fp32 cf32] n_in={n_in} T={T}")
            x = synth.ci8(seed=7 + n_in + T, n_channels=2, n_inputs=n_in, n_samples=T)
            got = gpu_vis(x, "fp32", "cf32")
            assert np.array_equal(got, oracle.xengine_ci8(x)), (n_in, T)


def test_extreme_values_i8():
    """All samples at +-max_abs (largest products, both signs) and one
    all-(-7) input: still exact."""
    rng = np.random.default_rng(5)
    x = (rng.integers(0, 2, size=(2, 130, 333, 2)) * 14 - 7).astype(np.int8)
    x[1, 5] = -7
    for engine in ("i8", "fp32"):
        say(f"[xengine {engine}] extremes")
        assert np.array_equal(gpu_vis(x, engine), oracle.xengine_ci8(x))


def full_range(seed, n_ch, n_in, T):
    """Integers uniform in [-127, 127] (the whole declared int8 range), with
    inputs 0..3 pinned at the extremes (+-127 in both parts, all four sign
    patterns) so that their autos reach 2 * 127^2 * T."""
    rng = np.random.default_rng(seed)
    x = rng.integers(-127, 128, size=(n_ch, n_in, T, 2)).astype(np.int8)
    for k, (a, b) in enumerate(((127, 127), (-127, 127), (127, -127), (-127, -127))):
        if k < n_in:
            x[:, k, :, 0] = a
            x[:, k, :, 1] = b
    return x


@pytest.mark.parametrize("engine", ["i8", "fp32"])
def test_full_int8_range_near_bounds(engine):
    """max_abs = 127 (the largest declared range): the byte rotation of the
    int8 engine on large magnitudes and sums close to the exactness bounds,
    2 * 127^2 * T <= 2^31 - 1 (int32, T <= 66572) and <= 2^24 (FP32 on integer
    data, T <= 520).  16-byte aligned rows (T a multiple of 8) take the
    matrix-core kernel with its LDS-staged loads, odd T the register-staged
    int8 kernel; N_I = 130 has a diagonal and an off-diagonal 128-row tile
    with a ragged last panel, N_I = 61 the 64-row engine (both split K)."""
    shapes = ((130, 66568), (61, 66571), (130, 66571)) if engine == "i8" else ((130, 520), (61, 517), (130, 519))
    for n_in, T in shapes:
        say(f"[xengine {engine}] max_abs=127 n_in={n_in} T={T}")
        x = full_range(n_in * 7 + T, 1, n_in, T)
        want = oracle.xengine_ci8(x)
        d = oracle.baseline_index(np.arange(4), np.arange(4))
        assert want[0, d, 0].max() == 2 * 127 * 127 * T          # the bound itself is reached
        got = gpu_vis(x, engine, max_abs=127)
        assert np.array_equal(got, want), (engine, n_in, T)
    if engine == "i8":
        # many channels (>= 1024 tiles: one pass, no K split) at the full range
        say("[xengine i8] max_abs=127 n_in=150 n_ch=350 T=1000 (no K split)")
        x = full_range(3, 350, 150, 1000)
        assert np.array_equal(gpu_vis(x, "i8", max_abs=127), oracle.xengine_ci8(x))


def test_aligned_calls_accumulate_in_the_epilogue():
    """Two 16-byte aligned corr_correlate calls into one integration with no K
    split: the second pass adds its tile into the accumulator in the
    read-modify-write epilogue of the 128-row int8 matrix-core kernel.  One
    channel of N_I = 200 with 128-sample calls (too few samples to split), and
    350 channels of N_I = 150 (>= 1024 tiles), against one call and the
    oracle."""
    for n_ch, n_in, T in ((1, 200, 256), (350, 150, 1024)):
        say(f"[xengine i8] aligned chunks n_ch={n_ch} n_in={n_in} T={T}")
        x = full_range(n_in + T, n_ch, n_in, T)
        want = oracle.xengine_ci8(x)
        half = T // 2
        assert (half * 2) % 16 == 0 and (T * 2) % 16 == 0
        got = gpu_vis(x, "i8", chunks=[(0, half), (half, T)], max_abs=127)
        one = gpu_vis(x, "i8", max_abs=127)
        assert np.array_equal(one, want)
        assert np.array_equal(got, want)


def test_wide_arrays_with_many_tiles():
    """Arrays of 5 to 9 row panels of 128 inputs with 1000 or more tiles (no K
    split): 640 inputs on 72 channels, 1000 (a ragged last panel) on 33
    channels, and 1100 on 16 channels with few samples."""
    for n_in, n_ch, T in ((640, 72, 200), (1000, 33, 136), (1100, 16, 72)):
        say(f"[xengine i8] n_in={n_in} n_ch={n_ch} T={T}")
        x = synth.ci8(seed=n_in + n_ch + T, n_channels=n_ch, n_inputs=n_in, n_samples=T)
        assert np.array_equal(gpu_vis(x, "i8"), oracle.xengine_ci8(x)), (n_in, n_ch, T)


def test_chunked_calls_equal_one_call():
    """Several corr_correlate calls over consecutive time ranges (ragged,
    misaligned chunk starts, row stride > n) accumulate to the same dump."""
    x = synth.ci8(seed=11, n_channels=3, n_inputs=150, n_samples=1000)
    want = oracle.xengine_ci8(x)
    chunks = [(0, 100), (100, 333), (333, 334), (334, 1000)]
    for engine in ("i8", "fp32"):
        say(f"[xengine {engine}] chunked")
        assert np.array_equal(gpu_vis(x, engine, chunks=chunks), want)


def test_dump_reset_and_no_reset():
    x = synth.ci8(seed=12, n_channels=2, n_inputs=40, n_samples=96)
    want = oracle.xengine_ci8(x)
    c = Correlator(40, 2, engine="i8", max_abs=7, device=DEV)
    xt = torch.from_numpy(x).to(DEV)
    c.correlate(xt)
    a, n1, _ = c.dump(CORR_DUMP_INTEG | CORR_DUMP_NO_RESET, device_out=False)
    c.correlate(xt)
    b, n2, _ = c.dump(CORR_DUMP_INTEG, device_out=False)
    z, n3, _ = c.dump(CORR_DUMP_INTEG, device_out=True)
    c.correlate(xt)
    d, n4, _ = c.dump(CORR_DUMP_INTEG, device_out=False)
    c.close()
    assert (n1, n2, n3, n4) == (96, 192, 0, 96)
    assert np.array_equal(a.numpy(), want)
    assert np.array_equal(b.numpy().astype(np.int64), 2 * want)
    assert not z.cpu().numpy().any()
    assert np.array_equal(d.numpy(), want)


def test_c1_plain_fp32_full():
    """N_I=64, 128 channels, 1000 samples, complex float32 integer samples,
    FP32 engine: bit-exact against the oracle (one integration dump)."""
    say("[C1] generating")
    x = synth.ci8(seed=1, n_channels=128, n_inputs=64, n_samples=1000)
    say("[C1] gpu")
    got = gpu_vis(x, "fp32", "cf32")
    say("[C1] oracle")
    want = oracle.xengine_ci8(x)
    assert np.array_equal(got, want)
    d = oracle.baseline_index(np.arange(64), np.arange(64))
    assert np.all(got[:, d, 1] == 0)


def test_c3_full_array():
    """N_I=1024, 768 channels, 8000 samples (4-bit range, int8 pairs), from the
    device generator: int8 MFMA and plain FP32 engines agree bit for bit on
    the whole output; three whole channels and 4096 sampled products across
    all channels are checked against the oracle on host-regenerated rows."""
    n_in, n_ch, T, seed = 1024, 768, 8000, 3
    gen = synth.DeviceGen()
    say("[C3] device generation")
    x = torch.empty((n_ch, n_in, T, 2), dtype=torch.int8, device=DEV)
    gen.fill_ci8(x.data_ptr(), n_ch, n_in, T, seed, stream=torch.cuda.current_stream().cuda_stream)
    say("[C3] int8 engine")
    c = Correlator(n_in, n_ch, engine="i8", max_abs=7, device=DEV)
    c.correlate(x)
    vi8, n, exact = c.dump(CORR_DUMP_INTEG)
    assert n == T and exact
    c.close()
    del c
    say("[C3] fp32 engine")
    c = Correlator(n_in, n_ch, engine="fp32", sample_type="ci8", max_abs=7, device=DEV)
    c.correlate(x)
    vf, n, exact = c.dump(CORR_DUMP_INTEG)
    c.close()
    del c
    assert torch.equal(vi8.to(torch.float32), vf), "int8 and FP32 engines differ"
    del vf
    say("[C3] oracle channels")
    for ch in (0, 383, 767):
        xc = synth.ci8_channel(seed, ch, n_in, T)
        want = oracle.xengine_ci8(xc[None])[0]
        got = vi8[ch].cpu().numpy().astype(np.int64)
        assert np.array_equal(got, want), ch
    say("[C3] oracle sampled products")
    rng = np.random.default_rng(99)
    chans = rng.integers(0, n_ch, 64)
    for ch in chans:
        ii = rng.integers(0, n_in, 64)
        jj = (rng.random(64) * (ii + 1)).astype(np.int64)
        ii[:4] = [1023, 1023, 128, 127]
        jj[:4] = [1023, 0, 127, 127]
        rows = np.unique(np.concatenate([ii, jj]))
        xc = synth.ci8_channel(seed, int(ch), n_in, T, inputs=rows)
        pos = {r: k for k, r in enumerate(rows)}
        want = oracle.xengine_pairs_ci8(xc, [pos[i] for i in ii], [pos[j] for j in jj])
        b = torch.from_numpy(oracle.baseline_index(ii, jj)).to(DEV)
        got = vi8[int(ch)].index_select(0, b).cpu().numpy().astype(np.int64)
        assert np.array_equal(got, want), int(ch)
