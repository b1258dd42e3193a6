"""GPU parity of the paper's three CMAC designs (Sec. 4: pair parallel, group
parallel G = 2, 4, hybrid group G = 2, 4) through the C ABI.

Integer-valued FP32 samples make every partial sum exact, so each design must
match the oracle's int64 visibilities bit for bit; Gaussian float samples are
compared with the FP64 oracle at FP32 accumulation accuracy.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_0906_1887_amd import DESIGNS, CorrError, cmac_design, corr_cmac_design

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_tic(x):
    """[ch][in][T][2] -> float32 [T][in][ch][2] on the device (the designs' layout)."""
    return torch.from_numpy(np.ascontiguousarray(x.transpose(2, 1, 0, 3)).astype(np.float32)).to(DEV)


@pytest.mark.parametrize("name", sorted(DESIGNS))
def test_design_bit_exact_integer_samples(name):
    for n_in, n_ch, T in ((64, 128, 300), (8, 200, 77), (12, 33, 5), (4, 1, 1)):
        say(f"[design {name}] n_in={n_in} n_ch={n_ch} T={T}")
        x = synth.ci8(seed=n_in * 7 + T, n_channels=n_ch, n_inputs=n_in, n_samples=T)
        want = oracle.xengine_ci8(x)
        xs = to_tic(x)
        got = cmac_design(name, xs)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy().astype(np.int64), want), (name, n_in, n_ch, T)
        cmac_design(name, xs, out=got, accumulate=True)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy().astype(np.int64), 2 * want), (name, "accumulate")


@pytest.mark.parametrize("name", sorted(DESIGNS))
def test_design_float_samples(name):
    n_in, n_ch, T = 16, 64, 2000
    x = np.stack([synth.complex_float(seed=8, ch=c, n_inputs=n_in, n_samples=T) for c in range(n_ch)])
    want = oracle.xengine_cf64(x.astype(np.float64))
    got = cmac_design(name, to_tic(x)).cpu().numpy().astype(np.float64)
    d = oracle.baseline_index(np.arange(n_in), np.arange(n_in))
    auto = want[:, d, 0]
    ii, jj = np.tril_indices(n_in)
    norm = np.sqrt(auto[:, ii] * auto[:, jj])                     # [ch][P]
    err = np.abs(got - want).max(axis=2) / norm
    say(f"[design {name}] float max error / sqrt(Vii Vjj) = {err.max():.2e}")
    assert err.max() < 1e-5


def test_design_argument_errors():
    buf = torch.zeros((2, 8, 4, 2), dtype=torch.float32, device=DEV)
    out = torch.zeros((4, 36, 2), dtype=torch.float32, device=DEV)
    for design, group, n_in in ((0, 2, 8), (1, 1, 8), (1, 3, 8), (2, 4, 6), (3, 1, 8)):
        with pytest.raises(CorrError):
            corr_cmac_design(design, group, buf.data_ptr(), 2, n_in, 4, out.data_ptr())
    with pytest.raises(CorrError):            # beyond the 128-input pair table
        corr_cmac_design(0, 1, buf.data_ptr(), 2, 130, 4, out.data_ptr())
