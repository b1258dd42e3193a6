"""Large shapes through the C ABI: arrays of thousands of inputs (many
lower-triangle tiles, a ragged last panel) for the exact engines, and F-stages
with hundreds of inputs, each against the oracle."""
import math
import sys

import numpy as np
import pytest
import torch

import fcheck
import oracle
import synth
from paper_0906_1887_amd import CORR_DUMP_INTEG, Correlator

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("engine", ["i8", "fp32"])
def test_thousands_of_inputs(engine):
    for n_in, T in ((2050, 33), (4100, 9)):
        say(f"[large {engine}] n_in={n_in} T={T}")
        x = synth.ci8(seed=n_in + T, n_channels=1, n_inputs=n_in, n_samples=T)
        c = Correlator(n_in, 1, engine=engine, sample_type="ci8", max_abs=7, device=DEV)
        c.correlate(torch.from_numpy(x).to(DEV))
        out, n, exact = c.dump(CORR_DUMP_INTEG, device_out=False)
        assert n == T and exact
        assert np.array_equal(out.numpy().astype(np.int64), oracle.xengine_ci8(x)), (engine, n_in)
        c.close()


def test_fstage_hundreds_of_inputs():
    s_real = float(np.float32(2.0 / (16.0 * math.sqrt(128.0))))
    n_in, nb = 512, 20
    say(f"[large fstage] real n_in={n_in} blocks={nb}")
    v = synth.real_voltages(seed=12, index=0, n_blocks=nb, n_inputs=n_in)
    c = Correlator(n_in, 128, engine="i8", fft_size=256, max_abs=7, requant_scale=s_real, ring_samples=nb,
                   device=DEV)
    dbg = torch.empty((128, n_in, nb, 2), dtype=torch.float32, device=DEV)
    c.channelise(torch.from_numpy(v).to(DEV), first_seq=0, spectra_dbg=dbg)
    q = c.ring_read().numpy()
    X = oracle.dft_real(v, 256)
    fcheck.check_spectra_requant(X, dbg.cpu().numpy(), q, s_real, 7, fcheck.real_bound(v, 256), "real n_in=512")
    c.close()

    s_cplx = float(np.float32(1.0 / 16.0))
    n_in, nb = 256, 24
    say(f"[large fstage] complex n_in={n_in} blocks={nb}")
    rec, lv = synth.capture_records(seed=13, index=0, n_records=nb * 128, n_streams=1, w_per=n_in)
    raw = torch.from_numpy(np.ascontiguousarray(rec[0, :, 1:]).view(np.int16)).to(DEV)
    c = Correlator(n_in, 128, engine="i8", fft_size=128, max_abs=7, requant_scale=s_cplx, ring_samples=nb,
                   device=DEV, volt_format="cw16")
    dbg = torch.empty((128, n_in, nb, 2), dtype=torch.float32, device=DEV)
    c.channelise(raw, first_seq=0, spectra_dbg=dbg)
    q = c.ring_read().numpy()
    # expected spectra from the oracle's decode of the words the GPU read
    lvd = oracle.unpack_w16(np.ascontiguousarray(rec[0, :, 1:]))
    assert np.array_equal(lvd, lv)
    X = oracle.dft_complex(lvd, 128)
    fcheck.check_spectra_requant(X, dbg.cpu().numpy(), q, s_cplx, 7, fcheck.complex_bound(lvd, 128),
                                 "complex n_in=256")
    c.correlate(None)
    out, n, exact = c.dump(CORR_DUMP_INTEG, device_out=False)
    assert n == nb and exact
    assert np.array_equal(out.numpy().astype(np.int64), oracle.xengine_ci8(q))
    c.close()
