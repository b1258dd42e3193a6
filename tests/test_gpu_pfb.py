"""GPU parity of the polyphase-filterbank F-stage (the remedy for the FFT's
spectral leakage suggested as further work) through the C ABI: 4 taps of 256
points, Hamming-windowed sinc prototype; consecutive corr_channelise calls
overlap by the 3 blocks of history.  Same three checks as the plain F-stage
(spectra error bound incl. the a-priori FP32 bound of the weighted sum and
FFT, tie-band requantiser with its mismatch fraction, X bit-exact on the
GPU's ring; tests/fcheck.py),
then the leakage of a tone between channel centres, against a plain-FFT plan.
"""
import math
import sys

import numpy as np
import pytest
import torch

import fcheck
import oracle
import synth
from paper_0906_1887_amd import CORR_DUMP_INTEG, CorrError, Correlator

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
S = float(np.float32(2.0 / (16.0 * math.sqrt(128.0))))
P = 4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def plan(n_in, ring, taps):
    return Correlator(n_in, 128, engine="i8", fft_size=256, max_abs=7, requant_scale=S, ring_samples=ring,
                      device=DEV, pfb_taps=taps)


def test_pfb_parity_with_history_overlap():
    for n_in, nb_list in ((64, [40, 9]), (13, [17, 20])):
        say(f"[pfb] n_in={n_in} blocks={nb_list}")
        total = sum(nb_list)
        v = synth.real_voltages(seed=9, index=n_in, n_blocks=total + P - 1, n_inputs=n_in)
        c = plan(n_in, total + 2, P)
        dbgs = []
        b0 = 0
        for nb in nb_list:
            part = torch.from_numpy(np.ascontiguousarray(v[b0 * 256:(b0 + nb + P - 1) * 256])).to(DEV)
            dbg = torch.empty((128, n_in, nb, 2), dtype=torch.float32, device=DEV)
            c.channelise(part, first_seq=b0, spectra_dbg=dbg)
            dbgs.append(dbg.cpu().numpy())
            b0 += nb
        q = c.ring_read().numpy()
        X = oracle.pfb_real(v, 256, P)                                  # [128][n_in][total][2]
        Xg = np.concatenate(dbgs, axis=2)
        fcheck.check_spectra_requant(X, Xg, q, S, 7, fcheck.pfb_bound(v, 256, P), f"pfb n_in={n_in}")
        c.correlate(None)
        out, n, exact = c.dump(CORR_DUMP_INTEG, device_out=False)
        assert n == total and exact
        assert np.array_equal(out.numpy().astype(np.int64), oracle.xengine_ci8(q))
        c.close()


def test_pfb_cuts_leakage_end_to_end():
    # a strong tone between channel centres over a weak noise floor; the GPU's
    # pre-quantisation spectra (the requantiser would round the leakage away)
    n_in, nb = 4, 300
    v = synth.real_tone(seed=10, n_samples=(nb + P - 1) * 256, n_inputs=n_in, bin_pos=37.5)
    power = {}
    for taps, vin in ((0, v[(P - 1) * 256:]), (P, v)):
        c = plan(n_in, nb, taps)
        dbg = torch.empty((128, n_in, nb, 2), dtype=torch.float32, device=DEV)
        c.channelise(torch.from_numpy(np.ascontiguousarray(vin)).to(DEV), first_seq=0, spectra_dbg=dbg)
        torch.cuda.synchronize()
        X = dbg.cpu().numpy().astype(np.float64)
        power[taps] = (X ** 2).sum(axis=3).mean(axis=(1, 2))          # per channel
        c.close()
    far = np.r_[1:33, 43:128]
    leak = {t: power[t][far].mean() / power[t].max() for t in power}
    say(f"[pfb] mean power 5+ channels from a tone at 37.5, relative to the peak: "
        f"fft {10 * np.log10(leak[0]):.1f} dB, pfb {10 * np.log10(leak[P]):.1f} dB")
    assert leak[P] < 0.05 * leak[0]


def test_pfb_unsupported_configs():
    with pytest.raises(CorrError):
        plan(8, 16, 3)
    with pytest.raises(CorrError):
        Correlator(8, 128, engine="i8", fft_size=128, max_abs=7, requant_scale=S, ring_samples=16, device=DEV,
                   volt_format="cw16", pfb_taps=4)


def test_pfb_full_c2_size_sampled_blocks():
    """The benchmark's filterbank launch: 64 inputs, 10 000 blocks (+3 of
    history) in one call.  The ring and the FP32 spectra of 40 blocks (both
    ends, workgroup boundaries, random others) meet the three checks against
    the oracle's filterbank, each block from its own 4-block window."""
    n_in, nb = 64, 10000
    v = synth.real_voltages(seed=2, index=0, n_blocks=nb + P - 1, n_inputs=n_in)
    say(f"[pfb] full size: {n_in} inputs, {nb} blocks")
    c = plan(n_in, nb, P)
    dbg = torch.empty((128, n_in, nb, 2), dtype=torch.float32, device=DEV)
    c.channelise(torch.from_numpy(v).to(DEV), first_seq=0, spectra_dbg=dbg)
    q = c.ring_read().numpy()
    c.close()
    rng = np.random.default_rng(12)
    blocks = sorted(set([0, 1, 15, 16, 17, 63, 64, 4999, 5000, 9983, 9984, 9998, 9999]
                        + rng.integers(0, nb, 27).tolist()))
    X = np.concatenate([oracle.pfb_real(v[b * 256:(b + P) * 256], 256, P) for b in blocks], axis=2)
    bound = max(fcheck.pfb_bound(v[b * 256:(b + P) * 256], 256, P) for b in blocks)
    idx = torch.tensor(blocks, device=DEV)
    Xg = dbg.index_select(2, idx).cpu().numpy()
    fcheck.check_spectra_requant(X, Xg, q[:, :, blocks], S, 7, bound, "pfb full size")
