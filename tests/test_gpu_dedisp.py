"""Coherent dedispersion (section 4.3) through the C ABI against the oracle
(numpy FP64 transforms): the detected, integrated output of the GPU's FP32
transforms for block lengths whose transform takes 2 to 4 passes (every first-pass
radix and every per-spectrum size the library instantiates), channel
counts from 16 to 8192 (the per-spectrum inverse DFT at its largest), one and
two polarisations, several integrations, zero DM; and a dispersed impulse put
back into one sample."""
import numpy as np
import pytest

import oracle
import paper_0910_1517_amd as corr

pytestmark = pytest.mark.gpu

FS, NU0 = 33.333333e6, 325e6


def voltages(npol, T, C, seed):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=(npol, T, C)) + 1j * rng.normal(size=(npol, T, C))).astype(np.complex64)


def run(V, dm, n_int):
    import torch
    v = torch.from_numpy(V).cuda()
    out, _ = corr.dedisperse(v, sample_rate=FS, nu0=NU0, dm=dm, n_int=n_int)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("npol,T,C,dm,n_int", [(2, 1024, 64, 0.05, 1), (1, 64, 1024, 0.02, 16), (2, 4096, 256, 0.3, 64),
                                               (1, 16, 8192, 0.1, 4), (2, 512, 256, 0.0, 8), (1, 16384, 1024, 1.0, 1024)])
def test_dedispersion_matches_oracle(npol, T, C, dm, n_int):
    print("dedisp", npol, T, C, dm, n_int, flush=True)
    V = voltages(npol, T, C, T + C)
    got = run(V, dm, n_int)
    ref = oracle.dedisperse(V.astype(np.complex128), FS, NU0, dm, n_int)
    rms = np.sqrt(np.mean(ref ** 2))
    err = np.abs(got - ref)
    print("  max err %.3g rms err %.3g of rms" % (err.max() / rms, np.sqrt(np.mean(err ** 2)) / rms), flush=True)
    # FP32 transforms of up to 2^24 points: the error of each voltage is about
    # 1e-6 of the rms, of each intensity 2e-6 of its size
    assert np.sqrt(np.mean(err ** 2)) <= 2e-5 * rms
    assert err.max() <= 2e-4 * rms * max(1.0, ref.max() / rms)


# Every shape of transform kernel the library instantiates: the block length's
# first pass takes log2 L mod 8 = 4 (the smallest block, whose stride equals
# the tile width), 5, 6, 7, 0, 2, 3, 5, 6, 7 bits, and the per-spectrum
# transform every C from 16 (one in-register stage) to 8192 (four stages, a
# whole workgroup per spectrum).
@pytest.mark.parametrize("T,C", [(256, 16), (256, 32), (128, 128), (64, 512), (32, 2048), (16, 4096), (8, 8192),
                                 (1024, 256), (2048, 256), (8192, 256), (16384, 256), (32768, 256)])
def test_every_transform_shape_matches_oracle(T, C):
    print("dedisp shape", T, C, flush=True)
    V = voltages(2, T, C, 7 * T + C)
    dm, n_int = 0.01, 16
    got = run(V, dm, n_int)
    ref = oracle.dedisperse(V.astype(np.complex128), FS, NU0, dm, n_int)
    rms = np.sqrt(np.mean(ref ** 2))
    err = np.abs(got - ref)
    print("  max err %.3g rms err %.3g of rms" % (err.max() / rms, np.sqrt(np.mean(err ** 2)) / rms), flush=True)
    assert np.sqrt(np.mean(err ** 2)) <= 2e-5 * rms
    assert err.max() <= 2e-4 * rms * max(1.0, ref.max() / rms)


def test_dispersed_impulse_is_recovered():
    C, T, dm = 64, 1024, 0.05
    L = C * T
    t0 = L - 200
    z = np.zeros(L, np.complex128)
    z[t0] = 1.0
    f = np.arange(L) * (FS / (2.0 * L))
    ph = oracle.dispersion_phase_cycles(f, NU0, dm)
    zd = np.fft.ifft(np.fft.fft(z) * np.exp(2j * np.pi * (ph - np.floor(ph))))
    V = (np.fft.fft(zd.reshape(T, C), axis=-1) / C)[None].astype(np.complex64)
    I = run(V, dm, 1)
    assert int(np.argmax(I)) == t0
    assert I[t0] > 0.99 * I.sum()
