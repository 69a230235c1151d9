"""Pins of the oracle F-engine in table mode (the 1440-step sin/cos look-up
table of section 2.3.2, 0.25 degree steps) against the directly evaluated
phase of Eq. 2: exact agreement where the phase is zero or a whole table step,
and the phase error bounded by half a step, 2 sin(pi / 2880) of |Y|,
otherwise."""
import math

import numpy as np

import oracle
import synth

FS = 66.666666e6


def setup(S=4, N=512, T=24, seed=3):
    geo = synth.make_geometry(S // 2, seed=seed)
    x = synth.voltages(S, N * T + 32, geo, FS, seed=seed + 1)
    return x, oracle.Geometry(geo.D, geo.f, geo.psi0, geo.rate), N, T


def test_zero_phase_is_exact():
    x, g, N, T = setup()
    z = np.zeros_like(g.f)
    g0 = oracle.Geometry(g.D, z, z, z)
    assert np.array_equal(oracle.fengine_lut(x, N, T, g0, FS), oracle.fengine(x, N, T, g0, FS))


def test_phase_error_is_at_most_half_a_step():
    x, g, N, T = setup()
    for nu_bb, sb in ((0.0, 1), (150e6, -1)):
        Yl = oracle.fengine_lut(x, N, T, g, FS, nu_bb=nu_bb, sideband=sb, spectrum0=1000)
        Yd = oracle.fengine(x, N, T, g, FS, nu_bb=nu_bb, sideband=sb, spectrum0=1000)
        mag = np.abs(Yd)
        ok = mag > 1e-9 * mag.max()
        err = np.abs(Yl - Yd)[ok] / mag[ok]
        bound = 2 * math.sin(math.pi / 2880)  # half of a 0.25 degree step
        assert err.max() <= bound * (1 + 1e-9)
        assert err.max() > 0.6 * bound          # the table is really used
        # the phase errors are spread over the half-step interval
        assert 0.3 * bound < np.sqrt(np.mean(err ** 2)) * math.sqrt(3) < 1.1 * bound


def test_phase_on_a_table_step_is_exact():
    x, g, N, T = setup()
    z = np.zeros_like(g.f)
    steps = np.array([0, 1, 359, 719, 1439])[: g.f.size]
    psi = steps.astype(np.float64) / 1440.0
    gs = oracle.Geometry(g.D, z, psi, z)
    Yl = oracle.fengine_lut(x, N, T, gs, FS)
    Yd = oracle.fengine(x, N, T, gs, FS)
    assert np.max(np.abs(Yl - Yd)) <= 1e-12 * np.max(np.abs(Yd))
