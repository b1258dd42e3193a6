"""GPU parity of the F-stage (real 256-point DFT, requantiser, corner turn)
and of the full FX path with the FP64 long-run accumulator, through the C ABI.

Requantisation: the GPU transforms in FP32 and the oracle in FP64, so a
value within the FFT's rounding error of a .5 boundary may round either way.
The test (i) bounds the spectra error (by 1e-5 of the channel RMS and by the
a-priori FP32 FFT bound), (ii) allows requantised mismatches only inside that
tie band and reports their fraction (tests/fcheck.py), and (iii) requires the
X-engine to be bit-exact on the GPU's own requantised spectra.
"""
import math
import sys

import numpy as np
import pytest
import torch

import fcheck
import oracle
import synth
from paper_0906_1887_amd import (CORR_DUMP_FOLD, CORR_DUMP_INTEG, CORR_DUMP_LONGRUN, CorrError,
                                 Correlator, _lib)

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
S = float(np.float32(2.0 / (16.0 * math.sqrt(128.0))))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def fx(n_in, ring, longrun=False):
    return Correlator(n_in, 128, engine="i8", fft_size=256, max_abs=7, requant_scale=S, ring_samples=ring,
                      fp64_longrun=longrun, device=DEV)


def check_spectra_and_requant(v, dbg, q_gpu, n_in, label=""):
    X = oracle.dft_real(v, 256)                                   # [128][n_in][nb][2] FP64
    r = fcheck.check_spectra_requant(X, dbg, q_gpu, S, 7, fcheck.real_bound(v, 256), label)
    return r["mismatch_frac"]


def test_fstage_small_and_x_on_gpu_spectra():
    # 16 inputs per workgroup: 64, 48 (ragged block groups); 8: 24, 8; bytewise: 13
    for n_in, nb_list in ((64, [64]), (48, [16, 23]), (24, [40]), (13, [37, 20]), (8, [16, 1, 15])):
        say(f"[fstage] n_in={n_in} blocks={nb_list}")
        c = fx(n_in, ring=sum(nb_list) + 5)
        seq = 100
        vs, qs = [], []
        for k, nb in enumerate(nb_list):
            v = synth.real_voltages(seed=2, index=k, n_blocks=nb, n_inputs=n_in)
            dbg = torch.empty((128, n_in, nb, 2), dtype=torch.float32, device=DEV)
            c.channelise(torch.from_numpy(v).to(DEV), first_seq=seq, spectra_dbg=dbg)
            seq += nb
            vs.append((v, dbg.cpu().numpy()))
        q = c.ring_read().numpy()
        assert q.shape == (128, n_in, sum(nb_list), 2)
        t0 = 0
        for v, dbg in vs:
            nb = dbg.shape[2]
            check_spectra_and_requant(v, dbg, q[:, :, t0:t0 + nb], n_in, f"n_in={n_in}")
            t0 += nb
        c.correlate(None)
        out, n, exact = c.dump(CORR_DUMP_INTEG, device_out=False)
        assert n == sum(nb_list) and exact
        assert np.array_equal(out.numpy().astype(np.int64), oracle.xengine_ci8(q))
        c.close()


def test_fstage_wide_launches_every_block():
    """Launches of several waves of 16-input workgroups (1591 blocks: 400
    items, 3189 blocks: 800 items; both end in a ragged block group), every
    block's spectra and requantised codes checked."""
    n_in = 64
    for nb in (1591, 3189):
        say(f"[fstage] wide launch n_in={n_in} blocks={nb}")
        c = fx(n_in, ring=nb + 3)
        v = synth.real_voltages(seed=5, index=nb, n_blocks=nb, n_inputs=n_in)
        dbg = torch.empty((128, n_in, nb, 2), dtype=torch.float32, device=DEV)
        c.channelise(torch.from_numpy(v).to(DEV), first_seq=0, spectra_dbg=dbg)
        q = c.ring_read().numpy()
        check_spectra_and_requant(v, dbg.cpu().numpy(), q[:, :, :nb], n_in, f"blocks={nb}")
        c.close()


def test_sequence_and_ring_errors():
    c = fx(8, ring=40)
    v = torch.from_numpy(synth.real_voltages(seed=2, index=0, n_blocks=16, n_inputs=8)).to(DEV)
    c.channelise(v, first_seq=5)
    with pytest.raises(CorrError) as e:
        c.channelise(v, first_seq=5)          # duplicate
    assert e.value.status == _lib.CORR_E_SEQ
    with pytest.raises(CorrError) as e:
        c.channelise(v, first_seq=22)         # gap
    assert e.value.status == _lib.CORR_E_SEQ
    c.channelise(v, first_seq=21)
    with pytest.raises(CorrError) as e:
        c.channelise(v, first_seq=37)         # 48 > 40 ring samples
    assert e.value.status == _lib.CORR_E_BUSY
    c.correlate(None)
    c.channelise(v, first_seq=37)             # drained: room again
    c.seq_reset()
    c.channelise(v[: 256 * 4].contiguous(), first_seq=0)
    _, n, _ = c.dump(CORR_DUMP_INTEG, device_out=False)
    assert n == 32
    c.close()


def test_c2_full_fx_longrun():
    """64 real 8-bit streams, 256-point real FFT -> 128 channels, requantised to
    4-bit complex, 10 000 blocks per integration, 10 dumps folded in FP64.
    Checks: spectra and requantiser on the first 64 blocks, X bit-exact on the
    GPU's own requantised spectra (integrations 0 and 9), FP64 long-run equal
    to the exact sum of the 10 int32 dumps, tone in channel 37 and the
    injected coherence recovered on inputs 0..7."""
    n_in, nb, n_dump = 64, 10000, 10
    c = fx(n_in, ring=nb, longrun=True)
    dumps = []
    seq = 0
    for d in range(n_dump):
        say(f"[C2] integration {d}")
        v = synth.real_voltages(seed=2, index=d, n_blocks=nb, n_inputs=n_in)
        vt = torch.from_numpy(v).to(DEV)
        if d == 0:
            dbg = torch.empty((128, n_in, 64, 2), dtype=torch.float32, device=DEV)
            c.channelise(vt[: 64 * 256].contiguous(), first_seq=seq, spectra_dbg=dbg)
            c.channelise(vt[64 * 256:].contiguous(), first_seq=seq + 64)
        else:
            c.channelise(vt, first_seq=seq)
        seq += nb
        if d in (0, n_dump - 1):
            q = c.ring_read().numpy()
            if d == 0:
                check_spectra_and_requant(v[: 64 * 256], dbg.cpu().numpy(), q[:, :, :64], n_in, "C2")
        c.correlate(None)
        out, n, exact = c.dump(CORR_DUMP_INTEG | CORR_DUMP_FOLD, device_out=False)
        assert n == nb and exact
        V = out.numpy().astype(np.int64)
        if d in (0, n_dump - 1):
            say(f"[C2] oracle X on GPU spectra, integration {d}")
            assert np.array_equal(V, oracle.xengine_ci8(q))
        dumps.append(V)
    L, _, _ = c.dump(CORR_DUMP_LONGRUN, device_out=False)
    c.close()
    L = L.numpy()
    exact_sum = np.zeros_like(dumps[0])
    for V in dumps:
        exact_sum += V
    assert np.array_equal(L, exact_sum.astype(np.float64))
    assert np.all(np.abs(exact_sum) < 2 ** 53)
    # coherence on the long-run sum
    chans = np.array([k for k in range(128) if k not in (0, 37)])
    rc = [oracle.coherence(L[chans], n_in, i, j, real_part=True).mean() for i in range(8) for j in range(i)]
    say(f"[C2] coherence inputs 0..7: {np.mean(rc):.5f}")
    assert abs(np.mean(rc) - 0.1 * 0.97953) < 0.002
    unc = []
    for i, j in ((20, 10), (63, 9), (40, 33), (50, 2), (31, 30)):
        b = oracle.baseline_index(i, j)
        vij = L[chans, b, 0] + 1j * L[chans, b, 1]
        norm = np.sqrt(L[chans, oracle.baseline_index(i, i), 0] * L[chans, oracle.baseline_index(j, j), 0])
        unc.append(np.mean(vij / norm))
    assert abs(np.mean(unc)) < 0.001
    # the tone: channel 37 autos carry the most power of all channels
    d = oracle.baseline_index(np.arange(n_in), np.arange(n_in))
    auto_power = L[:, d, 0].mean(axis=1)
    assert int(np.argmax(auto_power[1:])) + 1 == 37
