"""Pins of the oracle beamformer (section 2.2: incoherent array mode = detected
intensities added; coherent mode = voltages added, then detected, with the
voltage cross products the Stokes parameters need) against facts outside its
own loops: the correlator's visibilities (oracle.xengine, a separate
function), closed forms for a common signal in independent noise, the
phasing of the array, linearity and the odd-signal case."""
import numpy as np

import oracle


def rand_Y(S, T, C, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(S, T, C)) + 1j * rng.normal(size=(S, T, C))


def vis(V, i, j):
    """V_ij = sum_m Y_i conj(Y_j) from the X oracle's pair table (either order)."""
    return V[:, oracle.pair_index(i, j)] if i <= j else np.conj(V[:, oracle.pair_index(j, i)])


def test_coherent_power_is_the_weighted_sum_over_all_baselines():
    """Summed over time, |V_pol|^2 = sum over (i, j) of that polarisation of
    c_i conj(c_j) V_ij -- the phased beam is the correlator's visibilities,
    weighted and summed -- and V_0 conj(V_1) the same over the cross-polar
    block."""
    S, T, C = 7, 24, 5
    Y = rand_Y(S, T, C, 1)
    rng = np.random.default_rng(11)
    c = rng.normal(size=S) + 1j * rng.normal(size=S)
    _, coh = oracle.beamform(Y, c=[c], mode=oracle.BEAM_FULLPOL, tint=T)
    V = oracle.xengine(Y)
    pols = [[s for s in range(S) if s % 2 == p] for p in (0, 1)]
    wsum = lambda I, J: sum(c[i] * np.conj(c[j]) * vis(V, i, j) for i in I for j in J)
    for p in (0, 1):
        blk = wsum(pols[p], pols[p])
        assert np.allclose(coh[0, p, 0], blk.real, rtol=1e-12) and np.allclose(blk.imag, 0, atol=1e-9)
    cross = wsum(pols[0], pols[1])
    assert np.allclose(coh[0, 2, 0], cross.real, rtol=1e-12)
    assert np.allclose(coh[0, 3, 0], cross.imag, rtol=1e-12)


def test_incoherent_is_the_weighted_sum_of_autocorrelations():
    S, T, C = 6, 16, 4
    Y = rand_Y(S, T, C, 2)
    w = np.array([1.0, 0.5, 0.0, 2.0, 3.0, 0.25])  # w = 0 leaves a signal out
    inc, coh = oracle.beamform(Y, w=w, tint=T)
    assert coh is None
    V = oracle.xengine(Y)
    for p in (0, 1):
        ref = sum(w[s] * vis(V, s, s).real for s in range(p, S, 2))
        assert np.allclose(inc[p, 0], ref, rtol=1e-12)


def test_single_antenna_beam_gives_its_self_and_cross_polar_products():
    """A coherent beam of one antenna (both polarisations, unit weight) is that
    antenna's RR*, LL* and RL* -- the X oracle's pairs (2a, 2a), (2a+1, 2a+1),
    (2a, 2a+1)."""
    S, T, C, a = 8, 12, 3, 2
    Y = rand_Y(S, T, C, 3)
    c = np.zeros(S, complex)
    c[2 * a] = c[2 * a + 1] = 1.0
    _, coh = oracle.beamform(Y, c=[c], mode=oracle.BEAM_FULLPOL, tint=T)
    V = oracle.xengine(Y)
    assert np.allclose(coh[0, 0, 0], vis(V, 2 * a, 2 * a).real)
    assert np.allclose(coh[0, 1, 0], vis(V, 2 * a + 1, 2 * a + 1).real)
    assert np.allclose(coh[0, 2, 0] + 1j * coh[0, 3, 0], vis(V, 2 * a, 2 * a + 1))


def test_common_signal_coherent_and_incoherent_gains():
    """Y_s = z + n_s, z common to all antennas: per polarisation with A
    antennas, E|V|^2 = A^2 E|z|^2 + A E|n|^2 (voltages add coherently), while
    E[I] = A (E|z|^2 + E|n|^2) (intensities add)."""
    A, T, C = 6, 4000, 8
    S = 2 * A
    rng = np.random.default_rng(4)
    pz, pn = 0.5, 2.0  # E|z|^2, E|n|^2
    z = np.sqrt(pz / 2) * (rng.normal(size=(2, T, C)) + 1j * rng.normal(size=(2, T, C)))
    n = np.sqrt(pn / 2) * (rng.normal(size=(S, T, C)) + 1j * rng.normal(size=(S, T, C)))
    Y = z[np.arange(S) % 2] + n
    inc, coh = oracle.beamform(Y, w=np.ones(S), c=[np.ones(S)], mode=oracle.BEAM_INTENSITY)
    for p in (0, 1):
        ec, ei = coh[0, p].mean(), inc[p].mean()
        assert abs(ec / (A * A * pz + A * pn) - 1) < 0.03, ec
        assert abs(ei / (A * (pz + pn)) - 1) < 0.02, ei


def test_phasing_the_array_recovers_the_coherent_gain():
    """Antenna-based phases theta_a on the common signal: unit weights lose the
    coherent gain, weights exp(-i theta_a) restore it (the calibration of
    antenna phases before the voltages are added)."""
    A, T, C = 8, 3000, 4
    S = 2 * A
    rng = np.random.default_rng(5)
    theta = rng.uniform(0, 2 * np.pi, A)
    z = (rng.normal(size=(T, C)) + 1j * rng.normal(size=(T, C))) / np.sqrt(2)
    n = 0.1 * (rng.normal(size=(S, T, C)) + 1j * rng.normal(size=(S, T, C)))
    Y = np.exp(1j * theta[np.arange(S) // 2])[:, None, None] * z[None] + n
    c_cal = np.exp(-1j * theta[np.arange(S) // 2])
    _, coh = oracle.beamform(Y, c=[np.ones(S), c_cal], mode=oracle.BEAM_INTENSITY)
    raw, cal = coh[0, 0].mean(), coh[1, 0].mean()
    pn = 0.02  # E|n|^2 of each signal
    assert abs(cal / (A * A + A * pn) - 1) < 0.05, cal
    assert raw < 0.5 * cal
    assert abs(raw / (abs(np.exp(1j * theta).sum()) ** 2 + A * pn) - 1) < 0.1, raw


def test_voltage_beams_are_linear_and_sum_over_time():
    S, T, C = 5, 8, 3
    Y1, Y2 = rand_Y(S, T, C, 6), rand_Y(S, T, C, 7)
    c = np.exp(1j * np.arange(S)) * np.linspace(0.5, 2, S)
    _, v1 = oracle.beamform(Y1, c=[c], mode=oracle.BEAM_VOLTAGE)
    _, v2 = oracle.beamform(Y2, c=[c], mode=oracle.BEAM_VOLTAGE)
    _, v12 = oracle.beamform(Y1 + 2.0 * Y2, c=[c, 3j * c], mode=oracle.BEAM_VOLTAGE)
    assert np.allclose(v12[0], v1[0] + 2.0 * v2[0]) and np.allclose(v12[1], 3j * (v1[0] + 2.0 * v2[0]))
    # odd S: the last signal (antenna 2, polarisation 0) only enters V_0
    assert np.allclose(oracle.beamform(Y1[-1:] * 0 + Y1, c=[np.eye(S)[S - 1]], mode=oracle.BEAM_VOLTAGE)[1][0, 1], 0)
    # tint sums consecutive spectra
    inc1, coh1 = oracle.beamform(Y1, w=np.ones(S), c=[c], mode=oracle.BEAM_FULLPOL, tint=1)
    inc4, coh4 = oracle.beamform(Y1, w=np.ones(S), c=[c], mode=oracle.BEAM_FULLPOL, tint=4)
    assert np.allclose(inc4, inc1.reshape(2, T // 4, 4, C).sum(axis=2))
    assert np.allclose(coh4, coh1.reshape(1, 4, T // 4, 4, C).sum(axis=3))
