"""GPU parity at the paper's delay range (section 2.1: up to 128 us of total
delay, 8533 samples at 66.7 MS/s; the overlap of section 2.3.2 that keeps
delayed reads inside the slice), and the F-engine driven end to end by the
delay model of Eq. 1-2 through corr_geom_from_model."""
import math

import numpy as np
import pytest

import oracle
import paper_0910_1517_amd as corr
import synth
from gpu_util import FS, geom_dev, run_fengine, run_x_integrate, upload_streams

pytestmark = pytest.mark.gpu

NU_LO = 1.4e9
MAXD = 16384


def _spectra(spec, prec, S, C, T):
    Yg = corr.unpack_spectra(spec, prec, S, C, T)
    if prec == corr.FP32:
        return Yg[..., 0].astype(np.float64) + 1j * Yg[..., 1]
    return Yg.astype(np.int64)


@pytest.mark.parametrize("spectrum0", [0, 7, 123457])
def test_fengine_at_large_integer_delays(spectrum0):
    # integer delays up to 16383 samples, D mod 4 = 1, 3, 2, 0 (every byte offset of the
    # aligned dword reads), fractional delays, fringe phases and rates
    import torch
    S, N, T = 8, 1024, 64
    C = N // 2
    g = synth.rng(91, spectrum0)
    D = np.repeat(np.array([8533, 16383, 10002, 12]), 2)
    geo = synth.Geom(D, np.repeat(g.random(4).astype(np.float32).astype(np.float64), 2),
                     np.repeat(g.random(4), 2), np.repeat(g.uniform(-5, 5, 4), 2))
    x = synth.voltages(S, N * T + MAXD, geo, FS, seed=92 + spectrum0, tone_bin=37, tone_N=N)
    x_dev, rs = upload_streams(x, N, T, MAXD)
    og = oracle.Geometry(geo.D, geo.f, geo.psi0, geo.rate)
    Y = oracle.fengine(x, N, T, og, FS, spectrum0=spectrum0)
    # FP32 spectra, relative to each spectrum's RMS (the bound of the all-lengths test)
    plan = corr.Plan(S, N, T, precision=corr.FP32, max_delay=MAXD)
    Yg = _spectra(run_fengine(plan, x_dev, rs, geom_dev(geo), spectrum0=spectrum0), corr.FP32, S, C, T)
    plan.check_device_errors()
    rms = np.sqrt(np.mean(np.abs(Y) ** 2, axis=-1, keepdims=True))
    err = np.abs(Yg - Y) / rms
    print("large delays, spectrum0 %d: FP32 max %.3g rms %.3g" % (spectrum0, err.max(), np.sqrt(np.mean(err ** 2))))
    assert err.max() < 2e-5 and np.sqrt(np.mean(err ** 2)) < 2e-6
    # int8 codes with the oracle's held scales: the quantiser pin
    oscale = oracle.int8_scale(oracle.sigma(Y)).astype(np.float32)
    plan8 = corr.Plan(S, N, T, precision=corr.INT8, max_delay=MAXD, scale_mode=corr.SCALE_HOLD)
    sc = torch.from_numpy(oscale.ravel()).cuda()
    qg = _spectra(run_fengine(plan8, x_dev, rs, geom_dev(geo), sc, spectrum0=spectrum0), corr.INT8, S, C, T)
    plan8.check_device_errors()
    qo = oracle.quantize_int8(Y, oscale.astype(np.float64)).astype(np.int64)
    u = np.stack([Y.real, Y.imag], -1) / oscale.astype(np.float64)[:, None, :, None]
    frac = np.abs(np.abs(u - np.floor(u)) - 0.5)
    bad = qg != qo
    print("large delays, spectrum0 %d: int8 mismatches %d of %d" % (spectrum0, bad.sum(), bad.size))
    assert np.abs(qg - qo).max() <= 1 and np.all(frac[bad] < 1e-3) and bad.mean() <= 1e-4


@pytest.mark.parametrize("sideband", [1, -1])
def test_fx_driven_by_the_delay_model(sideband):
    # Antennas at up to 16200 samples of delay and +-5 Hz of fringe rate.  The library's
    # geometry helper turns the delay model into corr_geom_t; the forward model carries the
    # fringe phase at each sample's own arrival time.  The FP32 F + X + integrate chain
    # matches the FP64 oracle driven by the oracle's geometry (e_max <= 1e-5), and every
    # same-polarisation baseline has zero phase within the broadband bound.
    S, N, T = 8, 512, 512
    tau0 = np.repeat(np.array([8533.7, 16200.25, 0.4, 4097.9]) / FS, 2)
    tdot = np.repeat(np.array([5.0, -5.0, 3.0, -4.5]), 2) / NU_LO
    t_delay = T * N / 2 / FS
    gl = corr.geom_from_model(tau0, tdot, t_delay=t_delay, sample_rate=FS, nu_lo=NU_LO, max_delay=MAXD)
    go = oracle.geom_from_model(tau0, tdot, FS, NU_LO, t_delay=t_delay)
    assert np.array_equal(gl["D"], go.D) and np.max(np.abs(gl["frac"] - go.f)) <= 2 ** -24
    fwd = synth.Geom(go.D, go.f, np.mod(NU_LO * tau0, 1.0), NU_LO * tdot)
    x = synth.voltages(S, N * T + MAXD, fwd, FS, seed=43, rho=1.0, sigma_t=12.0, noise=False, sideband=sideband)
    plan = corr.Plan(S, N, T, precision=corr.FP32, max_delay=MAXD, sideband=sideband)
    x_dev, rs = upload_streams(x, N, T, MAXD)
    spec = run_fengine(plan, x_dev, rs, corr.geom_to_device(gl))
    _, V, _ = run_x_integrate(plan, spec)
    plan.check_device_errors()
    V64 = oracle.xengine(oracle.fengine(x, N, T, go, FS, sideband=sideband))
    e_max, e_fro = oracle.normalized_error(V, V64, S)
    print("delay model, sideband %+d: e_max %.3g e_fro %.3g" % (sideband, e_max, e_fro))
    assert e_max <= 1e-5
    ks = np.arange(8, N // 2 - 8)
    leak = 1 / (math.pi ** 2 * ks) + 1 / (math.pi ** 2 * (N // 2 - ks))
    for i in range(S):
        for j in range(i + 1, S):
            if (i - j) % 2:
                continue
            ph = np.angle(V[ks, oracle.pair_index(i, j)])
            sd = math.sqrt((2 * abs(go.f[i] - go.f[j]) / N + 2 * (1 / 12) / 144) / (2 * T))
            assert np.all(np.abs(ph) < 6 * sd + leak), (i, j)
            assert abs(np.mean(ph)) < 6 * sd / math.sqrt(len(ks)) + np.mean(leak), (i, j)
