"""The largest shapes the plans accept, on the GPU through the C ABI.

At N_I = 65 536 one channel has 2 147 516 416 products (17.2 GB of int32
pairs), past 2^31, so every index the engines form (packed triangle,
tile and row offsets) runs beyond 32 bits.  The samples are built so that
every product has a closed form: input i carries base sequence g(i) = (i *
2654435761 mod 2^32) mod 7 of 7 random complex integer sequences (|re|, |im|
<= 7), so V_ij = G[g(i)][g(j)] with G the 7 x 7 Gram matrix of the bases
(sum_t u_a[t] conj(u_b[t]), computed exactly on the host).  The check
gathers, on the GPU, 4 million random products, every product of the last
rows (the ragged last tile) and of the first row, and compares them with G.
Cases: the int8 engine at 65 536 inputs; the plain FP32 engine on the same
samples, equal to the int8 result on every product; the converting FP16
and FP8 engines at 65 535 inputs (their limit), exact on these integers
(FP8 scales by 64: 7 * 64 = 448); and 2^20 channels of 3 inputs."""
import sys

import numpy as np
import pytest
import torch

from paper_0906_1887_amd import CORR_DUMP_INTEG, Correlator

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
T = 64


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bases(seed=71):
    rng = np.random.default_rng(seed)
    u = rng.integers(-7, 8, size=(7, T, 2)).astype(np.int64)
    uc = u[..., 0] + 1j * u[..., 1]
    G = np.einsum("at,bt->ab", uc, np.conj(uc))          # exact: small integers in float64
    return u.astype(np.int8), np.stack([G.real, G.imag], axis=-1).astype(np.int64)


def group(i):
    return ((i.to(torch.int64) * 2654435761) % (1 << 32)) % 7


def samples(n_in, u, dtype):
    g = group(torch.arange(n_in, device=DEV))
    x = torch.from_numpy(u).to(DEV)[g]                   # [n_in][T][2]
    return x.to(dtype).unsqueeze(0).contiguous()         # one channel


def check(out, n_in, G):
    """Gathered products of the packed triangle out[0] against G."""
    v = out.reshape(-1, 2)
    gen = torch.Generator(device=DEV).manual_seed(5)
    i = torch.randint(0, n_in, (4_000_000,), device=DEV, generator=gen, dtype=torch.int64)
    j = (torch.rand(i.shape, device=DEV, generator=gen, dtype=torch.float64) * (i + 1).to(torch.float64)).to(torch.int64)
    j = torch.minimum(j, i)
    last = torch.arange(n_in - 3, n_in, device=DEV, dtype=torch.int64)
    li = last.repeat_interleave(n_in)
    lj = torch.arange(n_in, device=DEV, dtype=torch.int64).repeat(3)
    keep = lj <= li
    i = torch.cat([i, li[keep], torch.zeros(1, device=DEV, dtype=torch.int64)])
    j = torch.cat([j, lj[keep], torch.zeros(1, device=DEV, dtype=torch.int64)])
    got = v[i * (i + 1) // 2 + j].to(torch.int64)
    Gt = torch.from_numpy(G).to(DEV)
    want = Gt[group(i), group(j)]
    want[i == j, 1] = 0
    bad = (got != want).any(dim=1)
    assert int(bad.sum()) == 0, (int(bad.sum()), i[bad][:5].tolist(), j[bad][:5].tolist())


def dump(c):
    out, n, exact = c.dump(CORR_DUMP_INTEG, device_out=True)
    assert n == T
    return out, exact


def test_int8_and_fp32_at_65536_inputs():
    n_in = 65536
    u, G = bases()
    x = samples(n_in, u, torch.int8)
    say(f"[max] int8 engine, {n_in} inputs ({n_in * (n_in + 1) // 2} products)")
    c = Correlator(n_in, 1, engine="i8", max_abs=7, device=DEV)
    c.correlate(x)
    a, exact = dump(c)
    c.close()
    assert exact
    check(a, n_in, G)
    say("[max] plain FP32 engine, same samples")
    c = Correlator(n_in, 1, engine="fp32", sample_type="ci8", max_abs=7, device=DEV)
    c.correlate(x)
    b, exact = dump(c)
    c.close()
    assert exact
    av, bv = a.reshape(-1), b.reshape(-1)
    step = 1 << 28
    for k in range(0, av.numel(), step):                 # equal on every product, in chunks
        assert torch.equal(av[k:k + step].to(torch.float32), bv[k:k + step])
    del a, b, av, bv
    torch.cuda.empty_cache()


@pytest.mark.parametrize("engine", ["f16", "f8"])
def test_converting_engines_at_65535_inputs(engine):
    n_in = 65535
    u, G = bases()
    x = samples(n_in, u, torch.float32)
    say(f"[max] {engine} converting engine, {n_in} inputs")
    c = Correlator(n_in, 1, engine=engine, sample_type="cf32", max_abs=0, ring_samples=0, device=DEV)
    c.correlate(x)
    out, _ = dump(c)
    c.close()
    check(out, n_in, G)
    del out
    torch.cuda.empty_cache()


def test_a_million_channels():
    n_ch, n_in = 1 << 20, 3
    u, G = bases()
    g = group(torch.arange(n_ch * n_in, device=DEV)).reshape(n_ch, n_in)
    x = torch.from_numpy(u).to(DEV)[g].contiguous()      # [n_ch][n_in][T][2]
    say(f"[max] int8 engine, {n_ch} channels of {n_in} inputs")
    c = Correlator(n_in, n_ch, engine="i8", max_abs=7, device=DEV)
    c.correlate(x)
    out, exact = dump(c)
    c.close()
    assert exact
    Gt = torch.from_numpy(G).to(DEV)
    ii = torch.tensor([0, 1, 1, 2, 2, 2], device=DEV)
    jj = torch.tensor([0, 0, 1, 0, 1, 2], device=DEV)
    want = Gt[g[:, ii], g[:, jj]]                        # [n_ch][6][2]
    want[:, ii == jj, 1] = 0
    assert torch.equal(out.to(torch.int64), want)
