"""The device test-signal generator reproduces the host generator bit for bit."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def test_device_matches_host():
    gen = synth.DeviceGen()
    s = torch.cuda.current_stream().cuda_stream
    for n_ch, n_in, T, seed in ((3, 5, 37, 1), (2, 64, 1000, 3), (1, 1, 1, 0)):
        x = torch.empty((n_ch, n_in, T, 2), dtype=torch.int8, device="cuda:0")
        gen.fill_ci8(x.data_ptr(), n_ch, n_in, T, seed, stream=s)
        assert np.array_equal(x.cpu().numpy(), synth.ci8(seed, n_ch, n_in, T)), (n_ch, n_in, T)
    # channel offset and padded rows
    x = torch.zeros((2, 4, 40, 2), dtype=torch.int8, device="cuda:0")
    gen.fill_ci8(x.data_ptr(), 2, 4, 33, 9, stream=s, ch0=5, row_stride=40)
    h = x.cpu().numpy()
    for c in range(2):
        assert np.array_equal(h[c, :, :33], synth.ci8_channel(9, 5 + c, 4, 33))
    assert not h[:, :, 33:].any()
