"""Checkpoint and resume of a long run on the GPU, through the C ABI.

A plan that channelises, correlates and folds integrations into its FP64
long-run sum is checkpointed after two of them (the long-run dump, the
folded sample count and the next block sequence number, corr_state); a fresh
plan restored from the checkpoint (corr_restore, from host memory and from
device memory) then takes the third integration exactly like the original:
its long-run dump equals the original's bit for bit and the exact sum of the
three int32 integration dumps, the sequence check continues (a block number
that does not follow is refused with CORR_E_SEQ) and the exactness report of
the long-run dump counts the restored samples."""
import math
import sys

import numpy as np
import pytest
import torch

import synth
from paper_0906_1887_amd import (CORR_DUMP_FOLD, CORR_DUMP_INTEG, CORR_DUMP_LONGRUN, CorrError, Correlator,
                                 _lib)

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
S = float(np.float32(2.0 / (16.0 * math.sqrt(128.0))))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def plan(n_in, nb):
    return Correlator(n_in, 128, engine="i8", fft_size=256, max_abs=7, requant_scale=S, ring_samples=nb,
                      fp64_longrun=True, device=DEV)


def integrate(c, v, seq):
    c.channelise(v, first_seq=seq)
    c.correlate(None)
    out, n, exact = c.dump(CORR_DUMP_INTEG | CORR_DUMP_FOLD, device_out=False)
    assert exact
    return out.numpy().astype(np.int64)


@pytest.mark.parametrize("src_on_device", [False, True])
def test_restored_plan_continues_the_long_run(src_on_device):
    n_in, nb = 24, 300
    vs = [torch.from_numpy(synth.real_voltages(seed=51, index=k, n_blocks=nb, n_inputs=n_in)).to(DEV)
          for k in range(3)]
    a = plan(n_in, nb)
    first = 1000
    dumps = [integrate(a, vs[0], first), integrate(a, vs[1], first + nb)]
    L2, _, exact = a.dump(CORR_DUMP_LONGRUN, device_out=src_on_device)
    assert exact
    n_long, next_seq, valid = a.state()
    assert (n_long, next_seq, valid) == (2 * nb, first + 2 * nb, True)
    say(f"[checkpoint] n_long={n_long} next_seq={next_seq} source on device: {src_on_device}")

    b = plan(n_in, nb)
    assert b.state() == (0, 0, False)
    b.restore(L2, n_long, next_seq, valid)
    assert b.state() == (n_long, next_seq, True)
    with pytest.raises(CorrError) as e:                     # the sequence check continues
        b.channelise(vs[2], first_seq=next_seq + 1)
    assert e.value.status == _lib.CORR_E_SEQ
    dumps.append(integrate(a, vs[2], next_seq))
    assert np.array_equal(integrate(b, vs[2], next_seq), dumps[-1])
    La, na, ea = a.dump(CORR_DUMP_LONGRUN, device_out=False)
    Lb, nb_, eb = b.dump(CORR_DUMP_LONGRUN, device_out=False)
    assert torch.equal(La, Lb) and ea and eb
    assert np.array_equal(Lb.numpy(), np.sum(dumps, axis=0).astype(np.float64))
    assert b.state()[0] == 3 * nb
    a.close()
    b.close()


def test_restore_refusals():
    c = Correlator(16, 2, engine="i8", max_abs=7, device=DEV)             # no long-run sum
    src = torch.zeros((2, 136, 2), dtype=torch.float64)
    with pytest.raises(CorrError) as e:
        c.restore(src, 10)
    assert e.value.status == _lib.CORR_E_INVAL
    c.close()
    c = Correlator(16, 2, engine="i8", max_abs=7, fp64_longrun=True, device=DEV)
    with pytest.raises(CorrError) as e:
        _lib.corr_restore(c.plan, 0, False, 10, 0, False)                 # NULL source
    assert e.value.status == _lib.CORR_E_INVAL
    with pytest.raises(CorrError) as e:
        c.restore(src, -1)                                                # negative count
    assert e.value.status == _lib.CORR_E_INVAL
    c.close()
