"""Pins of the coherent-dedispersion oracle (section 4.3: phased-array
voltages to a broadband series by inverse FFT, multiplied by the inverse of
the interstellar dispersion transfer function in the Fourier domain, then
intensities of both polarisations added and integrated) against the
cold-plasma delay law, brute-force sums and a dispersed impulse."""
import numpy as np
import pytest

import oracle

FS = 33.333333e6   # complex baseband at FS / 2
NU0 = 325e6        # sky frequency of channel 0


def channelise(z, C):
    """Channel voltages whose baseband series is z (the forward DFT per block
    of C samples, divided by C), written here."""
    T = z.shape[-1] // C
    return np.fft.fft(z.reshape(z.shape[:-1] + (T, C)), axis=-1) / C


def test_baseband_series_is_the_inverse_dft_per_spectrum():
    rng = np.random.default_rng(1)
    V = rng.normal(size=(2, 3, 8)) + 1j * rng.normal(size=(2, 3, 8))
    z = oracle.baseband_series(V)
    for p in range(2):
        for m in range(3):
            for n in range(8):
                ref = sum(V[p, m, k] * np.exp(2j * np.pi * k * n / 8) for k in range(8))
                assert abs(z[p, m * 8 + n] - ref) < 1e-12


def test_group_delay_is_the_cold_plasma_delay():
    """-d(phase)/d(nu) of the transfer function = K DM (nu^-2 - nu0^-2)."""
    dm = 50.0
    f = np.linspace(1e5, 16e6, 40)
    h = 10.0
    tau = -(oracle.dispersion_phase_cycles(f + h, NU0, dm) - oracle.dispersion_phase_cycles(f - h, NU0, dm)) / (2 * h)
    law = oracle.K_DM * dm * ((NU0 + f) ** -2 - NU0 ** -2)
    assert np.allclose(tau, law, rtol=1e-6, atol=1e-12)
    assert np.all(law < 0)  # higher frequencies arrive earlier than nu0


def dispersed_impulse(dm, L, t0):
    z = np.zeros(L, np.complex128)
    z[t0] = 1.0
    f = np.arange(L) * (FS / (2.0 * L))
    ph = oracle.dispersion_phase_cycles(f, NU0, dm)
    return np.fft.ifft(np.fft.fft(z) * np.exp(2j * np.pi * (ph - np.floor(ph))))


def test_dispersed_impulse_follows_the_delay_law_and_dedisperses_to_an_impulse():
    dm, C, T = 0.05, 64, 1024
    L = C * T
    n_d = oracle.smear_samples(FS, NU0, dm)
    assert 1000 < n_d < L // 2
    t0 = L - 200  # arrives last at nu0, earlier at higher frequencies
    zd = dispersed_impulse(dm, L, t0)
    # sub-band arrival times: the band split in 8, each sub-band's peak
    Z = np.fft.fft(zd)
    edges = np.linspace(0, L, 9).astype(int)
    for a, b in zip(edges[:-1], edges[1:]):
        zs = np.fft.ifft(np.where((np.arange(L) >= a) & (np.arange(L) < b), Z, 0))
        t_peak = int(np.argmax(np.abs(zs)))
        fc = 0.5 * (a + b) * FS / (2.0 * L)
        t_law = t0 + oracle.K_DM * dm * ((NU0 + fc) ** -2 - NU0 ** -2) * FS / 2
        assert abs(t_peak - t_law) <= 0.02 * (b - a) + 3, (a, t_peak, t_law)
    # dedispersion puts the energy back into the impulse
    V = channelise(zd[None], C)
    I = oracle.dedisperse(V, FS, NU0, dm, 1)
    assert int(np.argmax(I)) == t0
    assert I[t0] > 0.99 * I.sum()
    # without it the energy is spread over the sweep
    raw = np.abs(zd) ** 2
    assert raw.max() < 0.01 * raw.sum()


def test_zero_dm_is_detection_only_and_polarisations_add():
    rng = np.random.default_rng(2)
    V = rng.normal(size=(2, 16, 32)) + 1j * rng.normal(size=(2, 16, 32))
    I = oracle.dedisperse(V, FS, NU0, 0.0, 4)
    z = oracle.baseband_series(V)
    ref = (np.abs(z) ** 2).sum(0).reshape(-1, 4).sum(1)
    assert np.allclose(I, ref, rtol=1e-12)
    I2 = oracle.dedisperse(np.stack([V[0], V[0]]), FS, NU0, 3.0, 1)
    I1 = oracle.dedisperse(V[:1], FS, NU0, 3.0, 1)
    assert np.allclose(I2, 2 * I1, rtol=1e-12)
    assert np.allclose(oracle.dedisperse(V, FS, NU0, 3.0, 8), oracle.dedisperse(V, FS, NU0, 3.0, 1).reshape(-1, 8).sum(1))
