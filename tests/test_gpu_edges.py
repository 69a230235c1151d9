"""Degenerate and extreme inputs through the C ABI: silent streams (sigma = 0),
full-scale constant streams (all power at DC, clipping-sized spectra), and a
late start time (large spectrum0: the fringe phase must still be reduced
exactly), each against the CPU oracle."""
import numpy as np
import pytest

import oracle
import paper_0910_1517_amd as corr
import synth
from gpu_util import FS, geom_dev, run_fengine, run_x_integrate, upload_streams

pytestmark = pytest.mark.gpu


def ogeom(g):
    return oracle.Geometry(g.D, g.f, g.psi0, g.rate)


@pytest.mark.parametrize("prec", [corr.INT8, corr.FP8_E4M3, corr.FP32])
def test_silent_input(prec):
    """All-zero samples: sigma = 0 gives scale 1 (never 0 or NaN), every
    spectrum is zero (the 8-bit codes are the +0 code), and every accumulator
    and visibility is exactly zero."""
    import torch
    S, N, T = 8, 512, 64
    geo = synth.make_geometry(S // 2, seed=3)
    x = np.zeros((S, N * T + 16), dtype=np.int8)
    plan = corr.Plan(S, N, T, precision=prec,
                     scale_mode=corr.SCALE_HOLD if prec == corr.FP32 else corr.SCALE_COMPUTE)
    x_dev, rs = upload_streams(x, N, T, 16)
    scale = torch.full((S * plan.C,), -1.0, dtype=torch.float32, device="cuda")
    spec = run_fengine(plan, x_dev, rs, geom_dev(geo), None if prec == corr.FP32 else scale)
    acc, state, vis = run_x_integrate(plan, spec, None if prec == corr.FP32 else scale)
    if prec == corr.FP32:  # float spectra: +-0 are both zero
        assert (spec.view(torch.float32) == 0).all().item()
    else:                  # int8 and e4m3 codes: zero is the +0 code
        assert not spec.any().item()
    assert not np.any(acc) and not np.any(state) and not np.any(vis)
    if prec != corr.FP32:
        assert torch.all(scale == 1.0).item()


def test_full_scale_constant_input():
    """Every sample +127 (or -127 on odd signals): all power is in the DC bin,
    the other channels are exactly zero, and the int8 path equals the oracle's
    own int8 path (its scales, RNE codes, int64 products) channel by channel."""
    import torch
    S, N, T = 4, 512, 64
    geo = synth.make_geometry(S // 2, seed=4)
    x = np.full((S, N * T + 16), 127, dtype=np.int8)
    x[1::2] = -127
    Y = oracle.fengine(x, N, T, ogeom(geo), FS)
    oscale = oracle.int8_scale(oracle.sigma(Y))
    q = oracle.quantize_int8(Y, oscale.astype(np.float64))
    vq = oracle.scale_visibilities(oracle.xengine_int(q), oscale.astype(np.float64))
    plan = corr.Plan(S, N, T, precision=corr.INT8)
    x_dev, rs = upload_streams(x, N, T, 16)
    scale_dev = torch.from_numpy(oscale.astype(np.float32).ravel()).cuda()
    spec = run_fengine(plan, x_dev, rs, geom_dev(geo), scale_dev)
    _, state, _ = run_x_integrate(plan, spec, scale_dev)
    Vq = vq[..., 0] + 1j * vq[..., 1]
    assert np.abs(Vq[1:]).max() == 0 and np.abs(state[1:]).max() == 0  # only DC carries power
    assert np.abs(state[0] - Vq[0]).max() <= 1e-6 * np.abs(Vq[0]).max()
    # FP32: DC against the FP64 oracle
    plan32 = corr.Plan(S, N, T, precision=corr.FP32)
    spec32 = run_fengine(plan32, x_dev, rs, geom_dev(geo))
    _, state32, _ = run_x_integrate(plan32, spec32)
    V64 = oracle.xengine(Y)
    assert np.abs(state32 - V64).max() <= 1e-5 * np.abs(V64).max()


def test_late_start_spectrum0():
    """A start 10^9 spectra in (about 8.5 hours at 33 MHz with N = 512): the
    fringe phase (psi0 + r t, r up to 5 Hz) is tens of thousands of cycles and
    must be reduced in FP64 before the FP32 sincos."""
    S, N, T = 8, 512, 256
    s0 = 10 ** 9
    geo = synth.make_geometry(S // 2, seed=5)
    x = synth.voltages(S, N * T + 64, geo, FS, seed=6, tone_bin=37, tone_N=N)
    plan = corr.Plan(S, N, T, precision=corr.FP32)
    x_dev, rs = upload_streams(x, N, T, 16)
    spec = run_fengine(plan, x_dev, rs, geom_dev(geo), spectrum0=s0)
    _, state, _ = run_x_integrate(plan, spec)
    V64 = oracle.xengine(oracle.fengine(x, N, T, ogeom(geo), FS, spectrum0=s0))
    e_max, _ = oracle.normalized_error(state, V64, S)
    assert e_max <= 1e-5, e_max
