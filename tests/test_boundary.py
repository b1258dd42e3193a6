"""Host-side checks of the C ABI (no GPU): the library loads, exports every
entry point the header declares, validates configurations and refuses
overflowing accumulations before any launch."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "corr.h")


def _declared():
    with open(HEADER) as fh:
        txt = fh.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(corr_\w+)\s*\(", txt, flags=re.M)))


def test_header_symbols_exported():
    from paper_0906_1887_amd import _lib
    L = _lib.lib()
    names = _declared()
    assert "corr_create" in names and "corr_correlate" in names and "corr_dump" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.EXPORTED)


def _cfg(**kw):
    from paper_0906_1887_amd import make_config
    return make_config(**kw)


def test_workspace_and_validation():
    from paper_0906_1887_amd import _lib
    ws = _lib.corr_workspace_bytes(_cfg(n_inputs=1024, n_channels=768, engine="i8"))
    assert ws >= 768 * 524800 * 8
    lowp = _lib.corr_workspace_bytes(_cfg(n_inputs=256, n_channels=1024, engine="f8", sample_type="cf32",
                                          max_abs=0, ring_samples=4096))
    assert lowp >= 1024 * 32896 * 8 + 1024 * 256 * 4096 * 2
    small = _lib.corr_workspace_bytes(_cfg(n_inputs=64, n_channels=128, engine="i8"))
    assert small > 128 * 2080 * 8        # includes K-split partials at small N_I
    fx = _lib.corr_workspace_bytes(_cfg(n_inputs=64, n_channels=128, engine="i8", fft_size=256,
                                        requant_scale=0.011, ring_samples=10000, fp64_longrun=True))
    assert fx >= 128 * 2080 * (8 + 16) + 128 * 64 * 10000 * 2
    bad = [
        dict(n_inputs=0, n_channels=4),
        dict(n_inputs=4, n_channels=0),
        dict(n_inputs=4, n_channels=4, engine="i8", sample_type="cf32"),
        dict(n_inputs=4, n_channels=4, engine="i8", max_abs=0),
        dict(n_inputs=4, n_channels=64, fft_size=256, requant_scale=0.1, ring_samples=10),
        dict(n_inputs=4, n_channels=128, fft_size=256, requant_scale=0.0, ring_samples=10),
        dict(n_inputs=4, n_channels=128, fft_size=256, requant_scale=0.1, ring_samples=0),
        dict(n_inputs=4, n_channels=4, engine="f16", sample_type="ci8", max_abs=0, ring_samples=64),
        dict(n_inputs=4, n_channels=4, engine="f8", sample_type="cf32", max_abs=7, ring_samples=64),
        dict(n_inputs=4, n_channels=4, engine="f8", sample_type="cf32", max_abs=0, ring_samples=-1),
    ]
    for kw in bad:
        with pytest.raises(_lib.CorrError) as e:
            _lib.corr_workspace_bytes(_cfg(**kw))
        assert e.value.status == _lib.CORR_E_INVAL, kw
    # converting FP16 / FP8 plans (ring_samples 0) hold no staging buffer
    conv = _lib.corr_workspace_bytes(_cfg(n_inputs=256, n_channels=1024, engine="f8", sample_type="cf32",
                                          max_abs=0, ring_samples=0))
    assert conv == lowp - 1024 * 256 * 4096 * 2
    for kw in (dict(n_inputs=4, n_channels=64, fft_size=128, requant_scale=0.1, ring_samples=10),):
        with pytest.raises(_lib.CorrError) as e:
            _lib.corr_workspace_bytes(_cfg(**kw))
        assert e.value.status == _lib.CORR_E_UNSUPPORTED, kw


def test_front_end_and_filterbank_validation():
    """The complex front end (volt_format) and the filterbank (pfb_taps)."""
    from paper_0906_1887_amd import _lib
    base = dict(n_inputs=64, n_channels=128, engine="i8", requant_scale=0.0625, ring_samples=100)
    plain = _lib.corr_workspace_bytes(_cfg(fft_size=256, **base))
    pfb = _lib.corr_workspace_bytes(_cfg(fft_size=256, pfb_taps=4, **base))
    assert pfb >= plain + 4 * 256 * 4                    # the coefficient table
    assert _lib.corr_workspace_bytes(_cfg(fft_size=128, volt_format="cw16", **base)) > 0
    assert _lib.corr_workspace_bytes(_cfg(fft_size=128, volt_format="cb8", **base)) > 0
    inval = [
        dict(fft_size=256, volt_format="cw16", **base),    # complex: fft_size must equal n_channels
        dict(fft_size=0, volt_format="cb8", **base),       # a format without an F-stage
        dict(fft_size=0, pfb_taps=4, **base),              # a filterbank without an F-stage
        dict(fft_size=256, pfb_taps=-1, **base),
    ]
    for kw in inval:
        with pytest.raises(_lib.CorrError) as e:
            _lib.corr_workspace_bytes(_cfg(**kw))
        assert e.value.status == _lib.CORR_E_INVAL, kw
    unsup = [
        dict(fft_size=256, pfb_taps=3, **base),            # this build's filterbank has 4 taps
        dict(fft_size=128, volt_format="cw16", pfb_taps=4, **base),   # the filterbank is real-input only
        dict(n_inputs=8, n_channels=64, engine="i8", fft_size=64, volt_format="cb8", requant_scale=0.1,
             ring_samples=10),                             # this build's complex DFT is 128 points
    ]
    for kw in unsup:
        with pytest.raises(_lib.CorrError) as e:
            _lib.corr_workspace_bytes(_cfg(**kw))
        assert e.value.status == _lib.CORR_E_UNSUPPORTED, kw
    c = _cfg(**base)
    c.volt_format = 7
    c.fft_size = 128
    with pytest.raises(_lib.CorrError) as e:
        _lib.corr_workspace_bytes(c)
    assert e.value.status == _lib.CORR_E_INVAL


def test_plan_free_entry_points_reject_bad_arguments():
    """corr_aggregate_w16 and corr_cmac_design validate on the host before any
    launch (null pointers are never dereferenced)."""
    from paper_0906_1887_amd import _lib
    for args in ((0, 1, 4, 16, 0, 0), (1, 0, 1, 16, 0, 0), (1, 4, 0, 16, 0, 0), (1, 4, 16, -1, 0, 0)):
        d_rec, ns, wp, nr, c0, d_out = args
        with pytest.raises(_lib.CorrError) as e:
            _lib.corr_aggregate_w16(d_rec, ns, wp, nr, c0, d_out)
        assert e.value.status == _lib.CORR_E_INVAL, args
    for design, group, n_in, n_ch, T in ((3, 1, 8, 4, 1), (0, 2, 8, 4, 1), (1, 3, 8, 4, 1), (2, 4, 6, 4, 1),
                                         (0, 1, 0, 4, 1), (0, 1, 8, 0, 1), (0, 1, 8, 4, -1)):
        with pytest.raises(_lib.CorrError) as e:
            _lib.corr_cmac_design(design, group, 0x1000, T, n_in, n_ch, 0x2000)
        assert e.value.status == _lib.CORR_E_INVAL, (design, group, n_in, n_ch, T)
    with pytest.raises(_lib.CorrError) as e:      # null spectra
        _lib.corr_cmac_design(0, 1, 0, 1, 8, 4, 0x2000)
    assert e.value.status == _lib.CORR_E_INVAL
    with pytest.raises(_lib.CorrError) as e:      # beyond the 128-input pair table
        _lib.corr_cmac_design(0, 1, 0x1000, 1, 130, 4, 0x2000)
    assert e.value.status == _lib.CORR_E_UNSUPPORTED


def test_create_rejects_bad_workspace():
    from paper_0906_1887_amd import _lib
    cfg = _cfg(n_inputs=16, n_channels=2, engine="i8")
    n = _lib.corr_workspace_bytes(cfg)
    for ptr, size in ((0, n), (0x1000_0000_0100 + 16, n), (0x1000_0000_0000, n - 1)):
        with pytest.raises(_lib.CorrError) as e:
            _lib.corr_create(cfg, ptr, size, 0)
        assert e.value.status == _lib.CORR_E_WORKSPACE


def _gpu_visible() -> bool:
    import torch
    return torch.cuda.device_count() > 0


@pytest.mark.skipif(_gpu_visible(), reason="uses a fake device pointer; host-only check")
def test_host_checks_before_launch():
    """A plan with neither F-stage nor long-run queues no device work at
    creation, so its host-side refusals can be exercised without a GPU (the
    workspace pointer is never dereferenced; skipped where a GPU is visible)."""
    from paper_0906_1887_amd import _lib
    fake = 0x7F00_0000_0000
    cfg = _cfg(n_inputs=16, n_channels=2, engine="i8", max_abs=7)
    plan = _lib.corr_create(cfg, fake, _lib.corr_workspace_bytes(cfg), 0)
    try:
        # 2*49*n > 2^31-1 for n >= 21_913_099 samples: refused before launch
        with pytest.raises(_lib.CorrError) as e:
            _lib.corr_correlate(plan, fake, 21_913_099, 0)
        assert e.value.status == _lib.CORR_E_OVERFLOW
        with pytest.raises(_lib.CorrError) as e:
            _lib.corr_channelise(plan, fake, 1, 0)
        assert e.value.status == _lib.CORR_E_STATE          # no F-stage in this plan
        with pytest.raises(_lib.CorrError) as e:
            _lib.corr_correlate(plan, fake, 10, 5)           # row stride < n
        assert e.value.status == _lib.CORR_E_INVAL
        with pytest.raises(_lib.CorrError) as e:
            _lib.corr_correlate(plan, fake + 1, 10, 0)       # misaligned int8 pairs
        assert e.value.status == _lib.CORR_E_INVAL
        assert _lib.corr_dump_bytes(plan, _lib.CORR_DUMP_INTEG) == 2 * 136 * 8
        assert _lib.corr_state(plan) == (0, 0, False)                 # checkpoint state of a new plan
        with pytest.raises(_lib.CorrError) as e:                       # no long-run sum to restore
            _lib.corr_restore(plan, fake, True, 10, 5, True)
        assert e.value.status == _lib.CORR_E_INVAL
    finally:
        _lib.corr_destroy(plan)
    cfg = _cfg(n_inputs=16, n_channels=2, engine="fp32", sample_type="ci8", max_abs=7)
    plan = _lib.corr_create(cfg, fake, _lib.corr_workspace_bytes(cfg), 0)
    try:
        with pytest.raises(_lib.CorrError) as e:            # FP32 exactness bound 2^24
            _lib.corr_correlate(plan, fake, 171_200, 0)
        assert e.value.status == _lib.CORR_E_OVERFLOW
    finally:
        _lib.corr_destroy(plan)


def test_status_strings():
    from paper_0906_1887_amd import _lib
    for s in range(-8, 1):
        assert _lib.corr_status_str(s) and "unknown" not in _lib.corr_status_str(s)
