"""Pins of the delay-model geometry (section 2.1, Eq. 1-2): the oracle's
exact-arithmetic version against closed forms and a second method, planted
mistakes that must fail, and the library's host helper corr_geom_from_model
(host code, no GPU) against the oracle."""
import math

import numpy as np
import pytest

import oracle
import paper_0910_1517_amd as corr
import synth

FS = 66.666666e6
NU_LO = 1.4e9


def test_whole_sample_delays_have_no_fraction():
    # tau = k / fs (up to the FP64 rounding of tau, ~1e-16 relative): D = k and f is that
    # rounding, below 1e-11 samples, whatever k, up to the paper's 128 us (8533 samples at
    # 66.7 MS/s) and past it; a rounding below k is carried, never left as f = 1 - 1e-12
    ks = np.array([0, 1, 5, 16, 8533, 16383, 65535])
    g = oracle.geom_from_model(ks / FS, np.zeros(ks.size), FS, NU_LO)
    assert np.array_equal(g.D, ks) and np.all(g.f < 1e-11)


def test_fraction_is_the_remainder_of_tau_fs():
    rng = np.random.default_rng(1)
    tau = rng.uniform(0, 128e-6, 200)
    g = oracle.geom_from_model(tau, np.zeros(200), FS, NU_LO)
    # D + f = tau fs to float32 rounding of f (2^-24), with f in [0, 1)
    assert np.all((g.f >= 0) & (g.f < 1))
    assert np.max(np.abs(g.D + g.f - tau * FS)) < 2 ** -24 + 1e-9
    half = oracle.geom_from_model((np.arange(5) + 0.5) / FS, np.zeros(5), FS, NU_LO)
    assert np.array_equal(half.D, np.arange(5)) and np.max(np.abs(half.f - 0.5)) < 1e-6


def test_fringe_phase_reduced_for_large_lo_times_delay():
    # 1.4 GHz x 128 us = 179200 cycles exactly: psi0 ~ 0 (mod 1); a quarter-cycle offset gives
    # 0.25.  The float64 tau carries ~1e-20 s of rounding, i.e. ~1e-11 cycles.
    g = oracle.geom_from_model([128e-6, 128e-6 + 0.25 / NU_LO, 128e-6 - 0.125 / NU_LO], [0, 0, 0], FS, NU_LO)
    wrap = lambda c, v: abs((c - v + 0.5) % 1.0 - 0.5)
    assert wrap(g.psi0[0], 0.0) < 1e-9
    assert wrap(g.psi0[1], 0.25) < 1e-9
    assert wrap(g.psi0[2], 0.875) < 1e-9
    assert np.all((g.psi0 >= 0) & (g.psi0 < 1))


def test_fringe_phase_agrees_with_fp64_product_and_rate():
    # a second method: frac of the plain FP64 product, good to ~ulp(179200) ~ 3e-11 cycles
    rng = np.random.default_rng(2)
    tau = rng.uniform(0, 128e-6, 100)
    tdot = rng.uniform(-4e-9, 4e-9, 100)
    t0 = 12.5
    g = oracle.geom_from_model(tau, tdot, FS, NU_LO, t0=t0)
    tz = tau - tdot * t0  # the delay at t = 0, also the evaluation time of D and f here
    naive = np.mod(NU_LO * tz + NU_LO * tdot * tz, 1.0)
    d = np.abs((g.psi0 - naive + 0.5) % 1.0 - 0.5)
    assert d.max() < 1e-9
    assert np.array_equal(g.rate, NU_LO * tdot)  # one FP64 product: exact as rounded
    assert np.all(np.abs(g.rate) <= 5.7)


def test_model_epoch_and_evaluation_time():
    # the same delay line written about two epochs gives the same geometry
    tau, tdot = np.array([3.3e-6, 40e-6]), np.array([2e-9, -3e-9])
    t0 = 7.0
    a = oracle.geom_from_model(tau, tdot, FS, NU_LO, t0=t0, t_delay=1.0)
    b = oracle.geom_from_model(tau - tdot * t0, tdot, FS, NU_LO, t0=0.0, t_delay=1.0)
    assert np.array_equal(a.D, b.D) and np.max(np.abs(a.f - b.f)) < 1e-6
    assert np.max(np.abs((a.psi0 - b.psi0 + 0.5) % 1 - 0.5)) < 1e-9
    # the integer and fractional delay follow the rate to the evaluation time
    c = oracle.geom_from_model(tau, tdot, FS, NU_LO, t0=t0, t_delay=t0 + 1.0)
    assert np.max(np.abs((c.D + c.f) - (tau + tdot) * FS)) < 1e-5


def _planted(tau0, taudot, fs, nu_lo, t0=0.0, t_delay=0.0, which=""):
    """The oracle's definition with one planted mistake (test-only)."""
    tau0, taudot = np.asarray(tau0, float), np.asarray(taudot, float)
    sgn = 1.0 if which != "t0_sign" else -1.0
    x = (tau0 + taudot * (t_delay - t0)) * fs
    D = np.floor(x) if which != "round" else np.rint(x)
    f = x - D
    c = nu_lo * (tau0 - sgn * taudot * t0) + nu_lo * taudot * x / fs
    if which == "delay_time":
        c = nu_lo * (tau0 + taudot * (t_delay - t0))
    if which == "no_arrival":
        c = nu_lo * (tau0 - taudot * t0)
    psi0 = c - np.floor(c) if which != "no_mod" else c
    return D, f, psi0


@pytest.mark.parametrize("which", ["t0_sign", "round", "no_mod", "delay_time", "no_arrival"])
def test_planted_mistakes_fail_the_pins(which):
    rng = np.random.default_rng(3)
    tau = rng.uniform(0, 128e-6, 50)
    tdot = rng.uniform(-4e-9, 4e-9, 50)
    g = oracle.geom_from_model(tau, tdot, FS, NU_LO, t0=10.0, t_delay=3.0)
    D, f, psi0 = _planted(tau, tdot, FS, NU_LO, t0=10.0, t_delay=3.0, which=which)
    ok = (np.array_equal(D, g.D) and np.all((f >= 0) & (f < 1)) and np.max(np.abs(f - g.f)) < 1e-6
          and np.all((psi0 >= 0) & (psi0 < 1)) and np.max(np.abs((psi0 - g.psi0 + 0.5) % 1 - 0.5)) < 1e-6)
    assert not ok


def _model_case(sideband, seed=41):
    """Four antennas at up to the paper's 128 us of delay and +-5 Hz of fringe rate."""
    rng = np.random.default_rng(seed)
    tau0 = np.repeat(np.array([8533.7, 16200.25, 0.4, 4097.9]) / FS, 2)
    rate = np.repeat(np.array([5.0, -5.0, 3.0, -4.5]), 2)
    return tau0, rate / NU_LO


@pytest.mark.parametrize("sideband", [1, -1])
def test_zero_phase_from_the_delay_model_at_large_delays(sideband):
    # The forward model: each antenna's samples carry its common signal delayed by
    # tau = D + f samples and the fringe phase nu_lo tau(t) at the sample's own (arrival)
    # time t.  Corrected by the oracle F-engine with the geometry of the delay model,
    # every same-polarisation baseline has zero phase within the broadband bound of
    # test_zero_phase_after_correction_broadband -- and not without the arrival term,
    # which is r tau ~ 4 mrad here.
    S, N, T = 8, 512, 512
    tau0, tdot = _model_case(sideband)
    t_delay = T * N / 2 / FS
    g = oracle.geom_from_model(tau0, tdot, FS, NU_LO, t_delay=t_delay)
    # phase and rate of the forward model at the row's own sample times (t = n / fs)
    fwd = synth.Geom(g.D, g.f, np.mod(NU_LO * tau0, 1.0), NU_LO * tdot)
    x = synth.voltages(S, N * T + 16400, fwd, FS, seed=42, rho=1.0, sigma_t=12.0, noise=False, sideband=sideband)
    ks = np.arange(8, N // 2 - 8)
    leak = 1 / (math.pi ** 2 * ks) + 1 / (math.pi ** 2 * (N // 2 - ks))
    pairs = [(i, j) for i in range(S) for j in range(i + 1, S) if (i - j) % 2 == 0]

    def phases(geom):
        V = oracle.xengine(oracle.fengine(x, N, T, geom, FS, sideband=sideband))
        return {(i, j): np.angle(V[ks, oracle.pair_index(i, j)]) for i, j in pairs}

    good = phases(g)
    for i, j in pairs:
        eps = 2 * abs(g.f[i] - g.f[j]) / N + 2 * (1 / 12) / 144
        sd = math.sqrt(eps / (2 * T))
        assert np.all(np.abs(good[i, j]) < 6 * sd + leak), (i, j)
        assert abs(np.mean(good[i, j])) < 6 * sd / math.sqrt(len(ks)) + np.mean(leak), (i, j)
    # negative control: the fringe phase taken at the aligned time stamp only
    bad_psi0 = np.mod(NU_LO * tau0, 1.0)
    bad = phases(oracle.Geometry(g.D, g.f, bad_psi0, g.rate))
    worst = max(abs(np.mean(bad[i, j])) - (6 * math.sqrt((2 * abs(g.f[i] - g.f[j]) / N + 2 / 12 / 144) / (2 * T))
                                           / math.sqrt(len(ks)) + np.mean(leak)) for i, j in pairs)
    assert worst > 0


# --------------------------------------------- the library's host helper (no GPU)
def test_library_helper_matches_the_oracle():
    rng = np.random.default_rng(4)
    S = 64
    tau = np.repeat(rng.uniform(0, 128e-6, S // 2), 2)
    tdot = np.repeat(rng.uniform(-3.5e-9, 3.5e-9, S // 2), 2)
    tau[:4] = np.array([0, 8533, 16383, 4097]) / FS  # whole samples, D mod 4 = 0, 1, 3, 1
    for t0, td in ((0.0, 0.0), (12.5, 0.7), (-3.0, 100.25)):
        # 4 samples of margin keep the delay positive after 103 s at 3.5 ns/s
        tl = tau + 4 / FS
        g = corr.geom_from_model(tl, tdot, t0=t0, t_delay=td, sample_rate=FS, nu_lo=NU_LO, max_delay=20000)
        o = oracle.geom_from_model(tl, tdot, FS, NU_LO, t0=t0, t_delay=td)
        tot_lib = g["D"] + g["frac"].astype(np.float64)
        assert np.max(np.abs(tot_lib - (o.D + o.f))) <= 2 ** -24
        assert np.all((g["frac"] >= 0) & (g["frac"] < 1))
        assert np.max(np.abs((g["psi0"] - o.psi0 + 0.5) % 1 - 0.5)) < 1e-15
        assert np.all((g["psi0"] >= 0) & (g["psi0"] < 1))
        assert np.array_equal(g["rate"], o.rate)
    g = corr.geom_from_model(tau[:4], np.zeros(4), sample_rate=FS, nu_lo=NU_LO, max_delay=20000)
    assert list(g["D"]) == [0, 8533, 16383, 4097] and np.all(g["frac"] < 1e-11)


def test_library_helper_rejects_bad_models():
    with pytest.raises(corr.CorrError) as e:
        corr.geom_from_model([200e-6], [0.0], sample_rate=FS, nu_lo=NU_LO, max_delay=8192)
    assert e.value.status == -1 and "signal 0" in str(e.value)
    with pytest.raises(corr.CorrError):
        corr.geom_from_model([-1e-6], [0.0], sample_rate=FS, nu_lo=NU_LO, max_delay=8192)
    with pytest.raises(corr.CorrError):
        corr.geom_from_model([1e-6], [math.nan], sample_rate=FS, nu_lo=NU_LO, max_delay=8192)
    with pytest.raises(corr.CorrError):
        corr.geom_from_model([1e-6], [0.0], sample_rate=FS, nu_lo=-1.0, max_delay=8192)
    with pytest.raises(corr.CorrError):
        corr.geom_from_model([1e-6], [0.0], sample_rate=0.0, nu_lo=NU_LO, max_delay=8192)
