"""Run-to-run determinism and launch-order independence on the GPU, through
the C ABI.

Every engine's result is a fixed function of its samples: the order of the
adds inside a tile, the order in which K-split partials are reduced and the
mapping of tiles to workgroups do not depend on which workgroup runs first.
So the same samples in a fresh plan must give the same bits, for the exact
engines (where any order gives the same sums) and for the floating-point ones
(where a race or an order that varied between runs would show up as changed
low bits).  An LDS or synchronisation race shows up the same way.

Cases:
* every engine twice in fresh plans, with K split (64 inputs x 128 channels x
  1000 samples: 8 splits) and without (300 inputs x 16 channels x 2000);
* the F-stage twice: the requantised ring and the FP32 spectra;
* launch mapping: the int8 engine over 32 channels of 1024 inputs against 31
  channels of the same samples, whose work items land on other XCDs and
  workgroup slots: equal on the 31.
"""
import math
import sys

import numpy as np
import pytest
import torch

import synth
from paper_0906_1887_amd import CORR_DUMP_INTEG, Correlator

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dump_once(engine, sample_type, x, max_abs, ring=0):
    n_ch, n_in, T, _ = x.shape
    c = Correlator(n_in, n_ch, engine=engine, sample_type=sample_type, max_abs=max_abs, ring_samples=ring,
                   device=DEV)
    c.correlate(x)
    out, n, _ = c.dump(CORR_DUMP_INTEG, device_out=True)
    c.close()
    assert n == T
    return out


@pytest.mark.parametrize("shape", [(64, 128, 1000), (300, 16, 2000)])
def test_every_engine_repeats_bit_for_bit(shape):
    n_in, n_ch, T = shape
    xi = torch.from_numpy(synth.ci8(seed=31, n_channels=n_ch, n_inputs=n_in, n_samples=T)).to(DEV)
    xf = torch.from_numpy(np.stack([synth.complex_float(32, ch, n_in, T) for ch in range(n_ch)])).to(DEV)
    cases = [("i8", "ci8", xi, 7, 0), ("fp32", "ci8", xi, 7, 0), ("fp32", "cf32", xf, 0, 0),
             ("fp32m", "cf32", xf, 0, 0), ("f16", "cf32", xf, 0, T), ("f16", "cf32", xf, 0, 0),
             ("f8", "cf32", xf, 0, T), ("f8", "cf32", xf, 0, 0)]
    for engine, st, x, m, ring in cases:
        say(f"[determinism] {engine} {st} ring={ring} n_in={n_in} n_ch={n_ch} T={T}")
        a = dump_once(engine, st, x, m, ring)
        b = dump_once(engine, st, x, m, ring)
        assert torch.equal(a, b), (engine, st, ring)
        assert bool(torch.isfinite(a.float()).all())


def test_fstage_repeats_bit_for_bit():
    n_in, nb = 64, 200
    s = float(np.float32(2.0 / (16.0 * math.sqrt(128.0))))
    v = torch.from_numpy(synth.real_voltages(seed=33, index=0, n_blocks=nb, n_inputs=n_in)).to(DEV)
    runs = []
    for _ in range(2):
        c = Correlator(n_in, 128, engine="i8", fft_size=256, max_abs=7, requant_scale=s, ring_samples=nb,
                       device=DEV)
        dbg = torch.empty((128, n_in, nb, 2), dtype=torch.float32, device=DEV)
        c.channelise(v, first_seq=0, spectra_dbg=dbg)
        runs.append((c.ring_read(), dbg.cpu()))
        c.close()
    assert torch.equal(runs[0][0], runs[1][0])
    assert torch.equal(runs[0][1], runs[1][1])


def test_item_mapping_does_not_change_the_sums():
    n_in, T = 1024, 64
    x = torch.from_numpy(synth.ci8(seed=34, n_channels=32, n_inputs=n_in, n_samples=T)).to(DEV)
    say("[determinism] 32 channels against 31 (another item-to-XCD mapping)")
    a = dump_once("i8", "ci8", x, 7)
    b = dump_once("i8", "ci8", x[:31].contiguous(), 7)
    assert torch.equal(a[:31], b)
