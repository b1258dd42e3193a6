"""GPU parity of the complex front end through the C ABI: aggregation of
capture streams (Sec. 3), the complex F-stage on 5+5-bit words and on the
1-byte mode (Sec. 2, Sec. 4, Sec. 5), and one second of the prototype's data
(64 inputs, 1.28 MHz complex samples, 128 channels) through the X-engine.

As for the real F-stage, the GPU transforms in FP32 and the oracle in FP64:
the spectra error is bounded (also by the a-priori FP32 FFT bound),
requantised codes may differ only inside the tie band (their fraction is
reported), and the X-engine must be bit-exact on the GPU's own ring
(tests/fcheck.py).  The expected spectra are the oracle's DFT of the oracle's
decode of the very words or bytes the GPU read; that decode is checked
separately against the generator's levels.
"""
import sys

import numpy as np
import pytest
import torch

import fcheck
import oracle
import synth
from paper_0906_1887_amd import CORR_DUMP_INTEG, CorrError, Correlator, aggregate_w16

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
S = float(np.float32(1.0 / 16.0))     # complex 5-bit data: spectra parts ~ 2.8 * sqrt(128)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def fe(n_in, ring, fmt):
    return Correlator(n_in, 128, engine="i8", fft_size=128, max_abs=7, requant_scale=S, ring_samples=ring,
                      device=DEV, volt_format=fmt)


def check(levels, dbg, q_gpu, n_in, label=""):
    """levels: int8 [n_blocks*128][n_in][2], the oracle's decode of the words or
    bytes the GPU read; dbg: [128][n_in][nb][2]; q_gpu: [128][n_in][nb][2]."""
    X = oracle.dft_complex(levels, 128)
    fcheck.check_spectra_requant(X, dbg, q_gpu, S, 7, fcheck.complex_bound(levels, 128), label)


def decoded(raw_cpu: np.ndarray, fmt: str, lv: np.ndarray) -> np.ndarray:
    """The oracle's decode of the raw words (cw16) or bytes (cb8) handed to the
    GPU, checked against the generator's levels (a separate check: the
    expected spectra come from the decode, not from the generator)."""
    d = oracle.unpack_w16(raw_cpu.view(np.uint16)) if fmt == "cw16" else oracle.unpack_b8(raw_cpu.view(np.uint8))
    assert np.array_equal(d, lv), fmt
    return d


def test_aggregate_bit_exact_and_counters():
    # 16-word records: 16-byte loads (record count a multiple of 8; a ragged
    # last workgroup of 184 records) and dword loads (1282 records: 2 in the
    # last workgroup); then the generic kernel.
    for ns, nr, wp, c0 in ((4, 3000, 16, 65000), (4, 1282, 16, 7), (2, 512, 16, 0), (3, 77, 5, 0), (1, 1, 1, 9)):
        say(f"[aggregate] streams={ns} records={nr} words={wp}")
        rec, _ = synth.capture_records(seed=3, index=nr, n_records=nr, n_streams=ns, w_per=wp, first_counter=c0)
        want, bad = oracle.aggregate_w16(rec, c0)
        assert bad == 0
        d = torch.from_numpy(rec.view(np.int16)).to(DEV)
        out, badc = aggregate_w16(d, first_counter=c0)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(np.uint16), want)
        assert int(badc.cpu().item()) == 0
        if nr > 20:
            rec[2 % ns, 17, 0] ^= 1          # one stream skips a beat at record 17
            rec[0, nr - 1, 0] += 5           # and another record is out of order
            rec[ns - 1, nr - 1, 0] += 1      # (the same record in two streams counts once)
            want, bad = oracle.aggregate_w16(rec, c0)
            assert bad == 2
            out, badc = aggregate_w16(torch.from_numpy(rec.view(np.int16)).to(DEV), first_counter=c0)
            torch.cuda.synchronize()
            assert int(badc.cpu().item()) == 2
            assert np.array_equal(out.cpu().numpy().view(np.uint16), want)


def test_aggregate_pointer_alignment():
    """The same records at 2-, 4- and 16-byte aligned addresses (the generic
    kernel, the per-record kernel with dword loads, and with 16-byte loads),
    written to an output 16 bytes past an allocation boundary."""
    ns, nr, wp, c0 = 4, 1024, 16, 300
    rec, _ = synth.capture_records(seed=6, index=0, n_records=nr, n_streams=ns, w_per=wp, first_counter=c0)
    rec[1, 500, 0] ^= 4                       # one record out of step in one stream
    want, bad = oracle.aggregate_w16(rec, c0)
    assert bad == 1
    flat = torch.from_numpy(np.ascontiguousarray(rec).view(np.int16).reshape(-1)).to(DEV)
    for off in (1, 2, 8):                     # int16 elements: 2, 4 and 16 bytes
        say(f"[aggregate] record pointer offset {2 * off} bytes")
        big = torch.zeros(flat.numel() + off, dtype=torch.int16, device=DEV)
        big[off:] = flat
        d = big[off:].view(ns, nr, wp + 1)
        assert d.data_ptr() % 256 == 2 * off
        out_big = torch.empty(nr * ns * wp + 8, dtype=torch.int16, device=DEV)
        out = out_big[8:].view(nr, ns * wp)
        o, b = aggregate_w16(d, first_counter=c0, out=out)
        torch.cuda.synchronize()
        assert np.array_equal(o.cpu().numpy().view(np.uint16), want)
        assert int(b.cpu().item()) == 1


@pytest.mark.parametrize("fmt", ["cw16", "cb8"])
def test_complex_fstage_shapes(fmt):
    # 64 and 24: vector loads (8 inputs per workgroup); 13: bytewise loads
    for n_in, nb_list in ((64, [40]), (24, [16, 23]), (13, [9, 20])):
        say(f"[complex fstage {fmt}] n_in={n_in} blocks={nb_list}")
        c = fe(n_in, sum(nb_list) + 3, fmt)
        seq = 7
        parts = []
        for k, nb in enumerate(nb_list):
            if fmt == "cw16":
                rec, lv = synth.capture_records(seed=4, index=k, n_records=nb * 128, n_streams=1, w_per=n_in)
                raw = torch.from_numpy(np.ascontiguousarray(rec[0, :, 1:]).view(np.int16)).to(DEV)
            else:
                b, lv = synth.complex_bytes(seed=4, index=k, n_samples=nb * 128, n_inputs=n_in)
                raw = torch.from_numpy(b).to(DEV)
            dbg = torch.empty((128, n_in, nb, 2), dtype=torch.float32, device=DEV)
            c.channelise(raw, first_seq=seq, spectra_dbg=dbg)
            seq += nb
            parts.append((decoded(raw.cpu().numpy(), fmt, lv), dbg.cpu().numpy()))
        q = c.ring_read().numpy()
        t0 = 0
        for lv, dbg in parts:
            nb = dbg.shape[2]
            check(lv, dbg, q[:, :, t0:t0 + nb], n_in, f"{fmt} n_in={n_in}")
            t0 += nb
        c.correlate(None)
        out, n, exact = c.dump(CORR_DUMP_INTEG, device_out=False)
        assert n == sum(nb_list) and exact
        assert np.array_equal(out.numpy().astype(np.int64), oracle.xengine_ci8(q))
        c.close()


def test_complex_config_errors():
    with pytest.raises(CorrError):      # complex input needs fft_size == n_channels
        Correlator(8, 128, engine="i8", fft_size=256, max_abs=7, requant_scale=S, ring_samples=16,
                   device=DEV, volt_format="cw16")
    with pytest.raises(CorrError):      # this build implements the 128-point complex DFT
        Correlator(8, 64, engine="i8", fft_size=64, max_abs=7, requant_scale=S, ring_samples=16,
                   device=DEV, volt_format="cb8")


def test_prototype_one_second():
    """Four capture streams of 1.28 M records (8 antennas x 2 polarisations
    each) -> aggregation -> complex F-stage (5+5-bit words) -> int8 X-engine:
    one second of the 64-input, 1.28 MHz prototype at 128 channels."""
    ns, wp, nr = 4, 16, 1_280_000
    n_in, nb = ns * wp, nr // 128
    rec, lv = synth.capture_records(seed=6, index=0, n_records=nr, n_streams=ns, w_per=wp, first_counter=123)
    d = torch.from_numpy(rec.view(np.int16)).to(DEV)
    say("[prototype 1 s] aggregate")
    agg, bad = aggregate_w16(d, first_counter=123)
    torch.cuda.synchronize()
    assert int(bad.cpu().item()) == 0
    want, _ = oracle.aggregate_w16(rec[:, :64 * 128], 123)
    assert np.array_equal(agg[:64 * 128].cpu().numpy().view(np.uint16), want)
    del d
    say("[prototype 1 s] channelise + correlate")
    c = fe(n_in, nb, "cw16")
    dbg = torch.empty((128, n_in, 64, 2), dtype=torch.float32, device=DEV)
    c.channelise(agg[:64 * 128].contiguous(), first_seq=0, spectra_dbg=dbg)
    c.channelise(agg[64 * 128:].contiguous(), first_seq=64)
    q = c.ring_read().numpy()
    # expected spectra from the oracle's decode of the aggregated words the F-stage read
    check(decoded(want, "cw16", lv[:64 * 128]), dbg.cpu().numpy(), q[:, :, :64], n_in, "prototype")
    c.correlate(None)
    out, n, exact = c.dump(CORR_DUMP_INTEG, device_out=False)
    assert n == nb and exact
    V = out.numpy().astype(np.int64)
    say("[prototype 1 s] oracle X on the GPU's ring")
    assert np.array_equal(V, oracle.xengine_ci8(q))
    c.close()
    # the tone (channel 19) carries the most auto power; inputs 0..7 share a
    # correlated component (rho = 0.1 before quantisation)
    dg = oracle.baseline_index(np.arange(n_in), np.arange(n_in))
    auto = V[:, dg, 0].mean(axis=1)
    assert int(np.argmax(auto)) == 19
    chans = np.array([k for k in range(128) if k != 19])
    coh = [oracle.coherence(V[chans], n_in, i, j, real_part=True).mean() for i in range(8) for j in range(i)]
    unc = [oracle.coherence(V[chans], n_in, i, j, real_part=True).mean() for i, j in ((20, 10), (63, 9), (40, 33))]
    say(f"[prototype 1 s] coherence inputs 0..7: {np.mean(coh):.4f}, others: {np.mean(unc):.4f}")
    assert 0.07 < np.mean(coh) < 0.11
    assert abs(np.mean(unc)) < 0.005
